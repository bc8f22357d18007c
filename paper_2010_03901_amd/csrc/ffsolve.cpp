// Fourier Forwarding solver of the wave equation (Sec. 4.2), host set-up and
// orchestration.  A large step [T_j, T_j + dT] combines (eq. ff_soln)
//  * U_FC: the 2D-FC extensions of u and u_t at T_j (boundary samples from the
//    Dirichlet data), their spectra advanced in closed form (eq. wave_2d_ff),
//    valid where the disc of radius c (t - T_j) lies in Omega, and
//  * U_B: on the boundary region, explicit second-order Taylor steps of size
//    dt (CFL 0.125) with second derivatives from the 1D-FC of Sec. 2.3 (both
//    blends) along grid lines, the Dirichlet condition imposed at the grid
//    points next to Gamma by cubic interpolation along the grid line from the
//    value at the line's crossing with Gamma, and values farther inside taken
//    from U_FC at the current time (an inverse FFT of the propagated spectrum).
// Set-up (boundary-sized work) runs here; every per-step operation runs in the
// kernels of kernels_ffsolve.hip and the library's FFT / propagation kernels.
//
// Definitions (the paper defers the details of U_B to a later paper):
//  boundary region  IN points within Chebyshev grid distance n_c + 2 of a
//                   non-IN grid point; dT = n_c h / c, dt = dT / ceil(8 n_c)
//  boundary points  boundary-region points next to a non-IN point along x or
//                   y; interpolated along that line (the longer IN run when
//                   both qualify, x on ties) from the 4 nearest of: the
//                   stepped points of the run and the two crossings bounding it
//  stepped points   the other boundary-region points; u^{n+1} = u + dt v +
//                   dt^2/2 a, v^{n+1} = v + dt (a + a^{n+1}) / 2, a = c^2 Lap u
//  segments         per IN run with stepped points: runs of fewer than 2 d
//                   points take the second derivative of the Lagrange
//                   interpolant through the run and its crossings (a crossing
//                   within h/2 of the run's end point is left out); longer
//                   runs take, per contiguous stepped sub-run, the 1D-FC second
//                   derivative over the sub-run extended by d points each way
//                   (clipped to the run, widened to 2 d points), as a dense
//                   matrix D2_n = first n rows of T_P E_n (E_n: continuation
//                   to P = n + C points, T_P: the spectral second derivative of
//                   period P h), formed in long double.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "ffsolve_int.h"
#include "internal.h"

using namespace fc2d;

struct fc2d_ff {
    const fc2d_plan* pl = nullptr;
    double c = 1.0, dT = 0.0, dt = 0.0;
    int n_c = 6, K = 0, M_b = 4;
    // host
    std::vector<int8_t> region;      // [nx][ny]: FFR_*
    std::vector<double> cross_xy;    // [ncross][2]
    int64_t n_stepped = 0, n_bnd = 0, n_ub = 0;
    int nseg = 0, max_seg = 0;
    // device
    int8_t* d_region = nullptr;
    int32_t* d_sidx = nullptr;       // [ns] flat index of each stepped point
    int32_t* d_sgrid = nullptr;      // [npts] stepped index or -1
    FfBnd* d_bnd = nullptr;          // [nbnd]
    FfSeg* d_seg = nullptr;          // [nseg]
    double* d_mats = nullptr;        // derivative matrices (c^2 and 1/h^2 included)
    double* d_work = nullptr;        // one allocation: spectra, U_FC grids, accelerations
    double *spec_u = nullptr, *spec_ut = nullptr, *prop_u = nullptr, *prop_ut = nullptr;
    double *ufc = nullptr, *utfc = nullptr, *acc = nullptr, *accd = nullptr;
};

namespace {

struct Run {
    int a, b;
};

// inclusive runs of true entries of a line
void line_runs(const std::vector<uint8_t>& m, std::vector<Run>& out) {
    out.clear();
    const int n = (int)m.size();
    for (int q = 0; q < n;) {
        if (!m[q]) { ++q; continue; }
        int e = q;
        while (e + 1 < n && m[e + 1]) ++e;
        out.push_back({q, e});
        q = e + 1;
    }
}

// Lagrange basis values L_k(x) of the nodes (long double)
void lagrange_basis(const std::vector<long double>& xs, long double x, std::vector<long double>& w) {
    const size_t n = xs.size();
    w.assign(n, 1.0L);
    for (size_t k = 0; k < n; ++k)
        for (size_t j = 0; j < n; ++j)
            if (j != k) w[k] *= (x - xs[j]) / (xs[k] - xs[j]);
}

// second derivatives L_k''(x)
void lagrange_d2(const std::vector<long double>& xs, long double x, std::vector<long double>& w) {
    const size_t n = xs.size();
    w.assign(n, 0.0L);
    for (size_t k = 0; k < n; ++k) {
        long double den = 1.0L;
        for (size_t j = 0; j < n; ++j)
            if (j != k) den *= xs[k] - xs[j];
        long double num = 0.0L;   // d2/dx2 of prod_{j != k} (x - x_j): sum over ordered pairs a != b of the rest
        for (size_t a = 0; a < n; ++a) {
            if (a == k) continue;
            for (size_t b = 0; b < n; ++b) {
                if (b == k || b == a) continue;
                long double pr = 1.0L;
                for (size_t j = 0; j < n; ++j)
                    if (j != k && j != a && j != b) pr *= x - xs[j];
                num += pr;
            }
        }
        w[k] = num / den;
    }
}

// D2_n (n x n, row-major) for the 1D-FC second derivative, scaled by s
void fc_d2_matrix(const fc2d_plan* pl, int n, double h, long double s, std::vector<double>& out) {
    const int d = pl->d, C = pl->C, P = n + C;
    const long double PI = 3.141592653589793238462643383279502884L;
    // circulant kernel of the spectral second derivative of period P h
    std::vector<long double> t(P, 0.0L);
    for (int j = 0; j < P; ++j) {
        long double acc = 0.0L;
        for (int m = 1; 2 * m < P; ++m) {
            const long double k = 2.0L * PI * m / ((long double)P * h);
            acc -= 2.0L * k * k * cosl(2.0L * PI * (long double)((int64_t)m * j % P) / P);
        }
        if (P % 2 == 0) {
            const long double k = PI / (long double)h;
            acc -= k * k * ((j % 2) ? -1.0L : 1.0L);
        }
        t[j] = acc / P;
    }
    // A Q^T (C x d): the blend-to-zero continuation of d matching values
    std::vector<long double> AQ((size_t)C * d, 0.0L);
    for (int l = 0; l < C; ++l)
        for (int j = 0; j < d; ++j) {
            long double acc = 0.0L;
            for (int i = 0; i < d; ++i) acc += (long double)pl->A[(size_t)l * d + i] * (long double)pl->Q[(size_t)j * d + i];
            AQ[(size_t)l * d + j] = acc;
        }
    // continuation rows: value at position n - 1 + l (l = 1..C) = sum_j AQ[l-1][j] f[n-d+j] (rightward blend)
    //                                                          + sum_j AQ[C-l][j] f[d-1-j] (leftward blend)
    std::vector<long double> D((size_t)n * n, 0.0L);
    auto tk = [&](int a) { return t[((a % P) + P) % P]; };
    for (int i = 0; i < n; ++i) {
        for (int q = 0; q < n; ++q) D[(size_t)i * n + q] = tk(i - q);
        for (int l = 1; l <= C; ++l) {
            const long double tv = tk(i - (n - 1 + l));
            for (int j = 0; j < d; ++j) {
                D[(size_t)i * n + (n - d + j)] += tv * AQ[(size_t)(l - 1) * d + j];
                D[(size_t)i * n + (d - 1 - j)] += tv * AQ[(size_t)(C - l) * d + j];
            }
        }
    }
    out.resize((size_t)n * n);
    for (size_t k = 0; k < out.size(); ++k) out[k] = (double)(s * D[k]);
}

template <class T>
int upload(T** dst, const std::vector<T>& src) {
    *dst = nullptr;
    if (src.empty()) return FC2D_OK;
    if (hipMalloc((void**)dst, src.size() * sizeof(T)) != hipSuccess) {
        set_error("hipMalloc failed (Fourier Forwarding set-up)");
        return FC2D_E_NOMEM;
    }
    if (hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("hipMemcpy failed (Fourier Forwarding set-up)");
        return FC2D_E_HIP;
    }
    return FC2D_OK;
}

void ff_free(fc2d_ff* f) {
    if (!f) return;
    void* ptrs[] = {f->d_region, f->d_sidx, f->d_sgrid, f->d_bnd, f->d_seg, f->d_mats, f->d_work};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete f;
}

int ff_build(fc2d_ff* f) {
    const fc2d_plan* pl = f->pl;
    const fc2d_grid& g = pl->grid;
    const int nx = g.nx, ny = g.ny, d = pl->d;
    const double h = g.h;
    const int nB = f->n_c + 2;
    const int n_o = d;
    const size_t npts = (size_t)nx * ny;
    std::vector<uint8_t> in(npts), near0(npts), ub(npts);
    if (int st = plan_host_lists(pl)) return st;
    for (size_t k = 0; k < npts; ++k) in[k] = pl->cls[k] == 1;
    // Chebyshev dilation of the non-IN set by nB (outside the grid counts as non-IN), separably
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            bool o = false;
            for (int di = -nB; di <= nB && !o; ++di) {
                const int ii = i + di;
                o = ii < 0 || ii >= nx || !in[(size_t)ii * ny + j];
            }
            near0[(size_t)i * ny + j] = o;
        }
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            bool o = false;
            for (int dj = -nB; dj <= nB && !o; ++dj) {
                const int jj = j + dj;
                o = jj < 0 || jj >= ny || near0[(size_t)i * ny + jj];
            }
            ub[(size_t)i * ny + j] = in[(size_t)i * ny + j] && o;
        }
    // runs along both directions: ax = 0 is the line y = y_line (position i), ax = 1 the line x = x_line (position j)
    std::vector<std::vector<Run>> runs[2];
    runs[0].resize(ny);
    runs[1].resize(nx);
    {
        std::vector<uint8_t> m;
        for (int j = 0; j < ny; ++j) {
            m.assign(nx, 0);
            for (int i = 0; i < nx; ++i) m[i] = in[(size_t)i * ny + j];
            line_runs(m, runs[0][j]);
        }
        for (int i = 0; i < nx; ++i) {
            m.assign(in.begin() + (size_t)i * ny, in.begin() + (size_t)(i + 1) * ny);
            line_runs(m, runs[1][i]);
        }
    }
    auto flat = [&](int ax, int line, int q) -> int64_t { return ax == 0 ? (int64_t)q * ny + line : (int64_t)line * ny + q; };
    // crossings bounding every run, in order (ax, line, run, lower end then upper end)
    std::map<std::tuple<int, int, int>, int> cross_id;   // (ax, line, outside position) -> crossing index
    std::vector<double> cpos;                             // crossing position along its line, in units of h
    f->cross_xy.clear();
    for (int ax = 0; ax < 2; ++ax)
        for (int line = 0; line < (int)runs[ax].size(); ++line)
            for (const Run& r : runs[ax][line])
                for (int side = 0; side < 2; ++side) {
                    const int end = side ? r.b : r.a, outn = side ? r.b + 1 : r.a - 1;
                    const bool vertical = ax == 1;   // x fixed, bisect along y
                    const double a_line = vertical ? g.x0 + line * h : g.y0 + line * h;
                    const double base = vertical ? g.y0 : g.x0;
                    double pos;
                    int st = gridline_crossing(pl, vertical, a_line, base + end * h, base + outn * h, &pos);
                    if (st) return st;
                    cross_id[{ax, line, outn}] = (int)cpos.size();
                    cpos.push_back((pos - base) / h);
                    if (vertical) { f->cross_xy.push_back(a_line); f->cross_xy.push_back(pos); }
                    else { f->cross_xy.push_back(pos); f->cross_xy.push_back(a_line); }
                }
    auto run_of = [&](int ax, int line, int q) -> const Run* {
        for (const Run& r : runs[ax][line])
            if (r.a <= q && q <= r.b) return &r;
        return nullptr;
    };
    // regions and boundary points
    f->region.assign(npts, FFR_OUT);
    std::vector<int8_t> bdir(npts, -1);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            const size_t k = (size_t)i * ny + j;
            if (!in[k]) continue;
            if (!ub[k]) { f->region[k] = FFR_INT; continue; }
            int best_len = -1, best_ax = -1;
            for (int ax = 0; ax < 2; ++ax) {
                const int line = ax == 0 ? j : i, q = ax == 0 ? i : j;
                const Run* r = run_of(ax, line, q);
                if (q == r->a || q == r->b) {
                    const int len = r->b - r->a + 1;
                    if (len > best_len) { best_len = len; best_ax = ax; }   // x first: ties keep x
                }
            }
            f->region[k] = best_ax >= 0 ? FFR_BND : FFR_STEP;
            bdir[k] = (int8_t)best_ax;
        }
    // stepped points
    std::vector<int32_t> sidx, sgrid(npts, -1);
    for (size_t k = 0; k < npts; ++k)
        if (f->region[k] == FFR_STEP) { sgrid[k] = (int32_t)sidx.size(); sidx.push_back((int32_t)k); }
    // boundary-point stencils
    std::vector<FfBnd> bnd;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            const size_t k = (size_t)i * ny + j;
            if (f->region[k] != FFR_BND) continue;
            const int ax = bdir[k], line = ax == 0 ? j : i, p = ax == 0 ? i : j;
            const Run* r = run_of(ax, line, p);
            struct Cand { long double pos; int32_t ref; };
            std::vector<Cand> cand;
            for (int q = r->a; q <= r->b; ++q)
                if (f->region[flat(ax, line, q)] == FFR_STEP) cand.push_back({(long double)q, (int32_t)flat(ax, line, q)});
            const int ca = cross_id.at({ax, line, r->a - 1}), cb = cross_id.at({ax, line, r->b + 1});
            cand.push_back({(long double)cpos[ca], -(1 + ca)});
            cand.push_back({(long double)cpos[cb], -(1 + cb)});
            std::stable_sort(cand.begin(), cand.end(), [&](const Cand& x, const Cand& y) {
                const long double dx = fabsl(x.pos - p), dy = fabsl(y.pos - p);
                return dx != dy ? dx < dy : x.pos < y.pos;
            });
            const int m = std::min<int>(f->M_b, (int)cand.size());
            FfBnd b{};
            b.target = (int32_t)k;
            b.nref = m;
            std::vector<long double> xs(m), w;
            for (int q = 0; q < m; ++q) { xs[q] = cand[q].pos; b.ref[q] = cand[q].ref; }
            lagrange_basis(xs, (long double)p, w);
            for (int q = 0; q < m; ++q) b.w[q] = (double)w[q];
            bnd.push_back(b);
        }
    // derivative segments
    std::vector<FfSeg> segs;
    std::vector<double> mats;
    std::map<int, int64_t> fc_mat;   // length -> offset of D2_n
    const long double scale = (long double)f->c * (long double)f->c;
    for (int ax = 0; ax < 2; ++ax)
        for (int line = 0; line < (int)runs[ax].size(); ++line)
            for (const Run& r : runs[ax][line]) {
                bool any = false;
                for (int q = r.a; q <= r.b && !any; ++q) any = f->region[flat(ax, line, q)] == FFR_STEP;
                if (!any) continue;
                FfSeg sg{};
                sg.base = (int32_t)(ax == 0 ? line : (int64_t)line * ny);
                sg.stride = ax == 0 ? ny : 1;
                const int n_run = r.b - r.a + 1;
                if (n_run < 2 * d) {
                    // Lagrange through the run and the crossings bounding it
                    const int ca = cross_id.at({ax, line, r.a - 1}), cb = cross_id.at({ax, line, r.b + 1});
                    const bool use_a = r.a - cpos[ca] >= 0.5, use_b = cpos[cb] - r.b >= 0.5;
                    std::vector<long double> xs;
                    if (use_a) xs.push_back(cpos[ca]);
                    for (int q = r.a; q <= r.b; ++q) xs.push_back(q);
                    if (use_b) xs.push_back(cpos[cb]);
                    sg.lo = r.a;
                    sg.n = n_run;
                    sg.r0 = r.a;
                    sg.r1 = r.b;
                    sg.ld = n_run + 2;        // values, then the two crossing columns
                    sg.ca = use_a ? ca : -1;
                    sg.cb = use_b ? cb : -1;
                    sg.mat = (int64_t)mats.size();
                    std::vector<long double> w;
                    for (int p = r.a; p <= r.b; ++p) {
                        std::vector<double> row(sg.ld, 0.0);
                        lagrange_d2(xs, (long double)p, w);
                        size_t o = 0;
                        if (use_a) row[n_run] = (double)(scale * w[o++] / ((long double)h * h));
                        for (int q = 0; q < n_run; ++q) row[q] = (double)(scale * w[o++] / ((long double)h * h));
                        if (use_b) row[n_run + 1] = (double)(scale * w[o++] / ((long double)h * h));
                        mats.insert(mats.end(), row.begin(), row.end());
                    }
                    sg.row0 = r.a;
                    segs.push_back(sg);
                    f->max_seg = std::max(f->max_seg, sg.n);
                    continue;
                }
                for (int q = r.a; q <= r.b;) {
                    if (f->region[flat(ax, line, q)] != FFR_STEP) { ++q; continue; }
                    int s1 = q;
                    while (s1 + 1 <= r.b && f->region[flat(ax, line, s1 + 1)] == FFR_STEP) ++s1;
                    int lo = std::max(r.a, q - n_o), hi = std::min(r.b, s1 + n_o);
                    while (hi - lo + 1 < 2 * d) {
                        if (lo > r.a) --lo;
                        if (hi - lo + 1 < 2 * d && hi < r.b) ++hi;
                    }
                    const int n = hi - lo + 1;
                    auto it = fc_mat.find(n);
                    if (it == fc_mat.end()) {
                        std::vector<double> D;
                        fc_d2_matrix(pl, n, h, scale, D);
                        it = fc_mat.emplace(n, (int64_t)mats.size()).first;
                        mats.insert(mats.end(), D.begin(), D.end());
                    }
                    sg.lo = lo;
                    sg.n = n;
                    sg.r0 = q;
                    sg.r1 = s1;
                    sg.ld = n;
                    sg.ca = sg.cb = -1;
                    sg.mat = it->second;
                    sg.row0 = lo;
                    segs.push_back(sg);
                    f->max_seg = std::max(f->max_seg, n);
                    q = s1 + 1;
                }
            }
    if (f->max_seg > kFfMaxSeg) {
        set_error("Fourier Forwarding: a derivative segment longer than " + std::to_string(kFfMaxSeg) + " points");
        return FC2D_E_GEOMETRY;
    }
    f->n_stepped = (int64_t)sidx.size();
    f->n_bnd = (int64_t)bnd.size();
    f->n_ub = f->n_stepped + f->n_bnd;
    f->nseg = (int)segs.size();
    int st;
    if ((st = upload(&f->d_region, f->region))) return st;
    if ((st = upload(&f->d_sidx, sidx))) return st;
    if ((st = upload(&f->d_sgrid, sgrid))) return st;
    if ((st = upload(&f->d_bnd, bnd))) return st;
    if ((st = upload(&f->d_seg, segs))) return st;
    if ((st = upload(&f->d_mats, mats))) return st;
    // work: four half spectra, two grids, accelerations a [ns] and per direction [2][ns]
    const size_t nsp = (size_t)nx * (ny / 2 + 1) * 2;
    const size_t ns = std::max<size_t>(sidx.size(), 1);
    const size_t tot = 4 * nsp + 2 * npts + 3 * ns;
    if (hipMalloc((void**)&f->d_work, tot * sizeof(double)) != hipSuccess) {
        set_error("hipMalloc failed (Fourier Forwarding work space)");
        return FC2D_E_NOMEM;
    }
    double* w = f->d_work;
    f->spec_u = w; w += nsp;
    f->spec_ut = w; w += nsp;
    f->prop_u = w; w += nsp;
    f->prop_ut = w; w += nsp;
    f->ufc = w; w += npts;
    f->utfc = w; w += npts;
    f->acc = w; w += ns;
    f->accd = w;
    return FC2D_OK;
}

}  // namespace

extern "C" {

int fc2d_ff_create(const fc2d_plan* pl, double c, int n_c, int closure_nodes, hipStream_t s, fc2d_ff** out) {
    if (closure_nodes == 0) closure_nodes = 4;
    if (!pl || !out || !(c > 0) || n_c < 1 || n_c > 64 || closure_nodes < 2 || closure_nodes > 4) {
        set_error("fc2d_ff_create: invalid arguments");
        return FC2D_E_ARG;
    }
    *out = nullptr;
    const fc2d_grid& g = pl->grid;
    if (g.nx < 16 || g.nx > 4096 || (g.nx & (g.nx - 1)) || g.ny < 16 || g.ny > 8192 || (g.ny & (g.ny - 1)) ||
        pl->interior_only) {
        set_error("fc2d_ff_create: the plan needs a power-of-two grid and boundary data");
        return FC2D_E_ARG;
    }
    fc2d_ff* f = new (std::nothrow) fc2d_ff();
    if (!f) { set_error("out of host memory"); return FC2D_E_NOMEM; }
    f->pl = pl;
    f->c = c;
    f->n_c = n_c;
    f->M_b = closure_nodes;
    f->dT = n_c * g.h / c;
    f->K = 8 * n_c;                 // CFL 0.125: dt = dT / (n_c / 0.125)
    f->dt = f->dT / f->K;
    int st;
    try {
        st = ff_build(f);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        st = FC2D_E_NOMEM;
    }
    if (st) { ff_free(f); return st; }
    (void)s;
    *out = f;
    return FC2D_OK;
}

int fc2d_ff_destroy(fc2d_ff* f) {
    ff_free(f);
    return FC2D_OK;
}

int fc2d_ff_get_info(const fc2d_ff* f, fc2d_ff_info* info) {
    if (!f || !info) { set_error("NULL argument"); return FC2D_E_ARG; }
    info->c = f->c;
    info->dT = f->dT;
    info->dt = f->dt;
    info->K = f->K;
    info->n_c = f->n_c;
    info->M_b = f->M_b;
    info->n_cross = (int64_t)f->cross_xy.size() / 2;
    info->n_stepped = f->n_stepped;
    info->n_bnd = f->n_bnd;
    info->n_segments = f->nseg;
    info->max_segment = f->max_seg;
    return FC2D_OK;
}

int fc2d_ff_crossings(const fc2d_ff* f, int64_t* n, double* xy) {
    if (!f || !n) { set_error("NULL argument"); return FC2D_E_ARG; }
    *n = (int64_t)f->cross_xy.size() / 2;
    if (xy) memcpy(xy, f->cross_xy.data(), f->cross_xy.size() * sizeof(double));
    return FC2D_OK;
}

int fc2d_ff_regions(const fc2d_ff* f, int8_t* region) {
    if (!f) { set_error("NULL argument"); return FC2D_E_ARG; }
    if (region) memcpy(region, f->region.data(), f->region.size());
    return FC2D_OK;
}

int fc2d_ff_advance(fc2d_ff* f, double* u, double* ut, const double* fb_u, const double* fb_ut, const double* bc_u,
                    const double* bc_ut, int nsmall, hipStream_t s) {
    if (!f || !u || !ut || !fb_u || !fb_ut || !bc_u || !bc_ut || nsmall < 1 || nsmall > f->K) {
        set_error("fc2d_ff_advance: NULL argument or nsmall outside 1..K");
        return FC2D_E_ARG;
    }
    const fc2d_plan* pl = f->pl;
    const fc2d_grid* g = &pl->grid;
    const int64_t ncross = (int64_t)f->cross_xy.size() / 2;
    int st;
    // U_FC at T_j: spectra of the 2D-FC extensions (STRIP values written into u / ut themselves)
    if ((st = fc2d_extend_fft(pl, u, fb_u, u, f->spec_u, 1, s))) return st;
    if ((st = fc2d_extend_fft(pl, ut, fb_ut, ut, f->spec_ut, 1, s))) return st;
    const FfDev dv{f->d_region, f->d_sidx, f->d_sgrid, f->d_bnd, f->d_seg, f->d_mats, f->n_stepped, f->n_bnd,
                   f->nseg, (int64_t)g->nx * g->ny};
    // acceleration at T_j from u itself (every IN value is valid then)
    if ((st = ffs_accel(dv, u, u, bc_u, f->accd, s))) return st;
    if ((st = ffs_sum_acc(dv, f->accd, f->acc, s))) return st;
    for (int k = 1; k <= nsmall; ++k) {
        const double tau = k * f->dt;
        if ((st = ffs_position(dv, u, ut, f->acc, f->dt, s))) return st;
        // U_FC(t) on the grid: the propagated spectrum, inverse transformed
        if ((st = prop_c2r(g, f->c, tau, f->spec_u, f->spec_ut, f->prop_u, f->ufc, 1, s))) return st;
        if ((st = ffs_boundary(dv, u, bc_u + (int64_t)k * ncross, s))) return st;
        if ((st = ffs_accel(dv, u, f->ufc, bc_u + (int64_t)k * ncross, f->accd, s))) return st;
        if ((st = ffs_velocity(dv, ut, f->acc, f->accd, f->dt, s))) return st;
        if ((st = ffs_boundary(dv, ut, bc_ut + (int64_t)k * ncross, s))) return st;
    }
    // the combination of eq. ff_soln at T_j + nsmall dt
    const double tau = nsmall * f->dt;
    if ((st = ff_apply(g, f->c, tau, f->spec_u, f->spec_ut, f->prop_u, f->prop_ut, 1, s))) return st;
    if ((st = fft2_c2r(g, f->prop_u, f->ufc, 1, s))) return st;
    if ((st = fft2_c2r(g, f->prop_ut, f->utfc, 1, s))) return st;
    return ffs_combine(dv, f->ufc, f->utfc, u, ut, s);
}

}  // extern "C"
