// Host side of the Geometrical Setup (Sec. 3.5 steps 1-4) and the C ABI.
//
// Boundary-sized work (boundary grid, admissibility, the FC-Gram tables, the
// placement and selection of the matching stencils' red stars and nodes) runs
// here and in matching_host.cpp on the host in C++; grid-sized and strip-sized
// work (classification of H, foot of the normal, the lists built from the
// classes, the red stars' grid-line scans and crossings with Gamma) runs in the
// device kernels of kernels_plan.hip.
//
// Classification (reading of Sec. 3.3-3.4, the same rule the checking code
// follows): IN / FAR by the parity of crossings of each grid column with a
// 16 B-vertex polygon of Gamma; every point whose nearest boundary sample is
// within C k1 + ds/2 (outside) or h + ds/2 (inside), ds the largest sample
// spacing, is reclassified by the signed normal distance eta of its foot:
// IN (eta <= 0), STRIP (0 < eta <= C k1) or FAR; a point with
// eta <= 1e-13 (1 + |x| + |y|) lies on Gamma to rounding and is IN.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "poisson_int.h"

namespace fc2d {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// kernel tracer: an event after every launch; a kernel's time is measured from
// the previous event on the same stream (a marker, name == nullptr, is recorded
// after each cross-stream wait so waiting is not counted)
struct TraceRec {
    const char* name;
    hipEvent_t ev;
    hipStream_t stream;
};
static std::mutex g_trace_mu;
static bool g_trace_on = false;
static std::vector<TraceRec> g_trace;

void trace_point(const char* name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    if (!g_trace_on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, s) != hipSuccess) {
        (void)hipEventDestroy(e);
        return;
    }
    g_trace.push_back({name, e, s});
}

static int hip_fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return FC2D_E_HIP;
}

#define HIPCHK(call)                                          \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #call);    \
    } while (0)

template <typename T>
static int dev_upload(T** dst, const T* src, size_t n) {
    *dst = nullptr;
    if (n == 0) return FC2D_OK;
    hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
    if (e != hipSuccess) {
        set_error("hipMalloc failed");
        return FC2D_E_NOMEM;
    }
    e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy H2D");
    return FC2D_OK;
}

// a plan-creation temporary from the library's stream-ordered pool, filled
// from host memory on stream s (the source must stay alive until s is
// synchronised; every caller here synchronises before it returns)
template <typename T>
static int ws_upload(T** dst, const T* src, size_t n, hipStream_t s) {
    *dst = nullptr;
    if (n == 0) return FC2D_OK;
    void* p = nullptr;
    int st = ws_alloc(n * sizeof(T), s, &p);
    if (st) return st;
    *dst = (T*)p;
    hipError_t e = hipMemcpyAsync(p, src, n * sizeof(T), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync H2D");
    return FC2D_OK;
}

// ----------------------------------------------------------------------------
// FC-Gram table cache
// ----------------------------------------------------------------------------
struct TableKey {
    int d, C, Z, n_os, n_r, mf;
    bool operator==(const TableKey& o) const {
        return d == o.d && C == o.C && Z == o.Z && n_os == o.n_os && n_r == o.n_r && mf == o.mf;
    }
};
struct TableEntry {
    TableKey k;
    std::vector<double> Q, A, Ar;
};
static std::mutex g_tab_mu;
static std::vector<TableEntry> g_tabs;

static int get_tables(const TableKey& k, std::vector<double>& Q, std::vector<double>& A,
                      std::vector<double>& Ar) {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    for (auto& e : g_tabs)
        if (e.k == k) {
            Q = e.Q; A = e.A; Ar = e.Ar;
            return FC2D_OK;
        }
    TableEntry e;
    e.k = k;
    e.Q.resize(k.d * k.d);
    e.A.resize(k.C * k.d);
    e.Ar.resize(k.C * k.n_r * k.d);
    if (gram_tables(k.d, k.C, k.Z, k.n_os, k.n_r, k.mf, e.Q.data(), e.A.data(), e.Ar.data()) != 0) {
        set_error("FC-Gram table construction failed for these parameters");
        return FC2D_E_TABLE;
    }
    g_tabs.push_back(e);
    Q = e.Q; A = e.A; Ar = e.Ar;
    return FC2D_OK;
}

// ----------------------------------------------------------------------------
// host foot solve dispatch
// ----------------------------------------------------------------------------
static int foot_host(int M, const CurveC& cv, const BndView& bd, double X, double Y, int p, int maxit,
                     double* th, double* eta, int* it) {
    switch (M) {
        case 4: return foot_solve<4>(cv, bd, X, Y, p, maxit, th, eta, it);
        case 5: return foot_solve<5>(cv, bd, X, Y, p, maxit, th, eta, it);
        case 6: return foot_solve<6>(cv, bd, X, Y, p, maxit, th, eta, it);
        case 7: return foot_solve<7>(cv, bd, X, Y, p, maxit, th, eta, it);
        case 8: return foot_solve<8>(cv, bd, X, Y, p, maxit, th, eta, it);
        case 9: return foot_solve<9>(cv, bd, X, Y, p, maxit, th, eta, it);
        case 10: return foot_solve<10>(cv, bd, X, Y, p, maxit, th, eta, it);
        case 11: return foot_solve<11>(cv, bd, X, Y, p, maxit, th, eta, it);
        case 12: return foot_solve<12>(cv, bd, X, Y, p, maxit, th, eta, it);
        case 13: return foot_solve<13>(cv, bd, X, Y, p, maxit, th, eta, it);
        case 15: return foot_solve<15>(cv, bd, X, Y, p, maxit, th, eta, it);
    }
    return FOOT_NO_BRACKET;
}

// nearest boundary sample by discrete descent from p
static int nearest_sample(const fc2d_plan* pl, double X, double Y, int p) {
    auto d2 = [&](int q) {
        const int r = imod(q, pl->B);
        const double dx = pl->bx[r] - X, dy = pl->by[r] - Y;
        return dx * dx + dy * dy;
    };
    double best = d2(p);
    for (int dir = -1; dir <= 1; dir += 2) {
        for (;;) {
            const double v = d2(p + dir);
            if (v < best) {
                best = v;
                p += dir;
            } else {
                break;
            }
        }
    }
    return imod(p, pl->B);
}

// ----------------------------------------------------------------------------
// matching stencils (Sec. 3.2)
// ----------------------------------------------------------------------------

// Red stars and their nodes (Sec. 3.2, Fig. 3).  The host places each normal's
// 2M candidate stars (matching_host.cpp); the device scans their grid lines for
// the IN runs next to them and bisects the lines' crossings with Gamma
// (k_star_scan); the host then picks the stars and nodes and forms the weights.
static int build_matching(fc2d_plan* pl, int maxit, const BndView& dbd, hipStream_t stream,
                          HostVec<int32_t>& mref, HostVec<double>& mwv, HostVec<double>& mwn) {
    const fc2d_grid& g = pl->grid;
    MatchGeom mg;
    mg.x0 = g.x0; mg.y0 = g.y0; mg.h = g.h; mg.nx = g.nx; mg.ny = g.ny;
    mg.M = pl->M; mg.d = pl->d; mg.B = pl->B; mg.interior_only = pl->interior_only; mg.k1 = pl->k1;
    mg.bx = pl->bx.data(); mg.by = pl->by.data(); mg.bnx = pl->bnx.data(); mg.bny = pl->bny.data();
    HostVec<StarQ> q;
    HostVec<long double> delta, bstar;
    place_stars(mg, q, delta, bstar);
    const size_t nst = q.size();
    // device: IN runs along the candidates' lines and the squares bounding them
    HostVec<StarR> res(nst);
    {
        StarArgs sa;
        sa.curve = pl->curve;
        sa.bx = dbd.x; sa.by = dbd.y; sa.bnx = dbd.nx; sa.bny = dbd.ny;
        sa.B = pl->B; sa.M = pl->M; sa.maxit = maxit; sa.io = pl->interior_only ? 1 : 0;
        sa.k2 = pl->k2; sa.x0 = g.x0; sa.y0 = g.y0; sa.h = g.h;
        sa.nx = g.nx; sa.ny = g.ny;
        StarQ* d_q = nullptr;
        StarR* d_r = nullptr;
        int st = ws_upload(&d_q, q.data(), nst, stream);
        hipError_t e = hipSuccess;
        if (!st) st = ws_alloc(nst * sizeof(StarR), stream, (void**)&d_r);
        if (!st) st = launch_star_scan(sa, pl->d_cls, d_q, d_r, (int)nst, stream);
        if (!st && ((e = hipMemcpyAsync(res.data(), d_r, nst * sizeof(StarR), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
                    (e = hipStreamSynchronize(stream)) != hipSuccess))
            st = hip_fail(e, "red-star scan");
        if (d_q) (void)ws_free(d_q, stream);
        if (d_r) (void)ws_free(d_r, stream);
        if (st) return st;
    }
    for (size_t k = 0; k < nst; ++k)
        if ((res[k].side[0] | res[k].side[1]) & 2) {
            set_error("foot of the normal failed while locating grid-line crossings with the boundary");
            return FC2D_E_NEWTON;
        }
    const int bad = select_matching(mg, q.data(), res.data(), delta.data(), bstar.data(), mref, mwv, mwn, pl->squares);
    if (bad < 0) {
        char buf[160];
        snprintf(buf, sizeof buf, "matching stencil: too few usable red stars at normal %d", -bad - 1);
        set_error(buf);
        return FC2D_E_GEOMETRY;
    }
    return FC2D_OK;
}

// ----------------------------------------------------------------------------
// plan creation
// ----------------------------------------------------------------------------
static void free_plan(fc2d_plan* pl) {
    if (!pl) return;
    void* ptrs[] = {pl->d_Q, pl->d_Ar, pl->d_mref, pl->d_mlab, pl->d_mwv, pl->d_mwn, pl->d_sidx,
                    pl->d_sth, pl->d_seta, pl->d_run_ptr, pl->d_run, pl->d_cls2, pl->d_bxy,
                    pl->d_cls, pl->d_rm_idx, pl->d_rm_seed, pl->d_rm_th, pl->d_rm_eta};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete pl;
}

static int create_plan(const fc2d_curve* curve, const fc2d_grid* grid, int d, int C,
                       const fc2d_opts* opts_in, hipStream_t stream, fc2d_plan** out) {
    if (!curve || !grid || !out) { set_error("NULL argument"); return FC2D_E_ARG; }
    *out = nullptr;
    fc2d_opts o;
    fc2d_opts_default(grid, &o);
    if (opts_in) {
        if (opts_in->B > 0) o.B = opts_in->B;
        if (opts_in->k1 > 0) o.k1 = opts_in->k1;
        if (opts_in->M > 0) o.M = opts_in->M;
        if (opts_in->n_r > 0) o.n_r = opts_in->n_r;
        if (opts_in->Z > 0) o.Z = opts_in->Z;
        if (opts_in->n_os > 0) o.n_os = opts_in->n_os;
        if (opts_in->mf > 0) o.mf = opts_in->mf;
        if (opts_in->newton_maxit > 0) o.newton_maxit = opts_in->newton_maxit;
        o.seed = opts_in->seed;
        if (opts_in->mlp_tol != 0.0) o.mlp_tol = opts_in->mlp_tol < 0.0 ? -1.0 : opts_in->mlp_tol;
        o.mlp_weights = opts_in->mlp_weights;
        o.interior_only = opts_in->interior_only != 0;
    }
    if (o.seed < FC2D_SEED_PROXIMITY || o.seed > FC2D_SEED_MLP ||
        (o.seed != FC2D_SEED_PROXIMITY && curve->kind != FC2D_CURVE_POLAR) ||
        (o.seed == FC2D_SEED_MLP && !o.mlp_weights)) {
        set_error("invalid seed option (POLAR and MLP need a polar curve, MLP needs weights)");
        return FC2D_E_ARG;
    }
    if (o.M <= 0) o.M = d + 3;
    const bool m_ok = (o.M >= 4 && o.M <= 8) || o.M == 13 || o.M == 15;   // compiled stencil sizes
    if (d < 2 || d > 12 || C < 2 || !m_ok || o.M < d - 1 || grid->h <= 0 || grid->nx < 8 ||
        grid->ny < 8 || (int64_t)grid->nx * grid->ny >= (int64_t)1 << 31 || o.B < 16 ||
        curve->nmodes < 0 || curve->nmodes > kMaxModes || !curve->a ||
        (curve->kind == FC2D_CURVE_CARTESIAN && !curve->b) ||
        (curve->kind != FC2D_CURVE_POLAR && curve->kind != FC2D_CURVE_CARTESIAN)) {
        set_error("invalid plan arguments (supported: 2 <= d <= 12, M in 4..8, 13, 15, M >= d - 1, B >= 16)");
        return FC2D_E_ARG;
    }
    fc2d_plan* pl = new (std::nothrow) fc2d_plan();
    if (!pl) { set_error("out of host memory"); return FC2D_E_NOMEM; }
    auto t_last = std::chrono::steady_clock::now();
    auto lap = [&](int phase) {   // host wall clock of the phase that ends here
        const auto t = std::chrono::steady_clock::now();
        pl->t_ms[phase] += std::chrono::duration<double, std::milli>(t - t_last).count();
        t_last = t;
    };
    pl->grid = *grid;
    pl->d = d; pl->C = C; pl->M = o.M; pl->n_r = o.n_r; pl->Cr = C * o.n_r; pl->B = o.B;
    pl->k1 = o.k1;
    pl->k2 = 2.0 * M_PI / o.B;
    pl->seed = o.seed;
    pl->interior_only = o.interior_only != 0;
    memset(&pl->curve, 0, sizeof pl->curve);
    pl->curve.kind = curve->kind;
    pl->curve.nmodes = curve->nmodes;
    for (int i = 0; i < 1 + 2 * curve->nmodes; ++i) {
        pl->curve.a[i] = curve->a[i];
        if (curve->kind == FC2D_CURVE_CARTESIAN) pl->curve.b[i] = curve->b[i];
    }
    int st = get_tables(TableKey{d, C, o.Z, o.n_os, o.n_r, o.mf}, pl->Q, pl->A, pl->Ar);
    if (st) { free_plan(pl); return st; }

    // step 1: boundary discretisation and normals (eq. bdry_grid)
    const int B = pl->B;
    pl->bx.resize(B); pl->by.resize(B); pl->bnx.resize(B); pl->bny.resize(B);
    std::vector<double> spd(B);   // |q'(theta_p)|
    double spmax = 0.0;
#pragma omp parallel for reduction(max : spmax)
    for (int p = 0; p < B; ++p) {
        double v[6];
        curve_eval(pl->curve, p * pl->k2, v);
        const double sp = sqrt(v[2] * v[2] + v[3] * v[3]);
        pl->bx[p] = v[0]; pl->by[p] = v[1];
        pl->bnx[p] = v[3] / sp; pl->bny[p] = -v[2] / sp;
        spd[p] = sp;
        spmax = std::max(spmax, sp);
    }
    // admissibility: exterior reach and the box.  The 16 B curve samples are
    // also the vertices of the polygon whose column crossings the proximity
    // seed's parity test uses (kept when that seed is chosen).
    double reach_ext = INFINITY;
    const int nv = 16 * B;
    const bool keep_poly = o.seed == FC2D_SEED_PROXIMITY;
    std::vector<double> px(keep_poly ? nv : 0), py(keep_poly ? nv : 0);
    {
        const int ns = nv;
        double kmin = 0.0;   // most negative curvature
#pragma omp parallel for reduction(min : kmin)
        for (int k = 0; k < ns; ++k) {
            double v[6];
            curve_eval(pl->curve, k * (2.0 * M_PI / ns), v);
            if (keep_poly) { px[k] = v[0]; py[k] = v[1]; }
            const double s2 = v[2] * v[2] + v[3] * v[3];
            const double kap = (v[2] * v[5] - v[3] * v[4]) / (s2 * sqrt(s2));
            kmin = std::min(kmin, kap);
        }
        reach_ext = kmin < 0 ? 1.0 / -kmin : INFINITY;
        if (C * pl->k1 > 0.9 * reach_ext) {
            char buf[160];
            snprintf(buf, sizeof buf, "C k1 = %.4g exceeds 0.9 x exterior reach %.4g", C * pl->k1, reach_ext);
            set_error(buf);
            free_plan(pl);
            return FC2D_E_GEOMETRY;
        }
        const double xlo = grid->x0, xhi = grid->x0 + (grid->nx - 1) * grid->h;
        const double ylo = grid->y0, yhi = grid->y0 + (grid->ny - 1) * grid->h;
        for (int p = 0; p < B; ++p) {
            const double ox = pl->bx[p] + pl->bnx[p] * (C * pl->k1);
            const double oy = pl->by[p] + pl->bny[p] * (C * pl->k1);
            const double xs[2] = {pl->bx[p], ox}, ys[2] = {pl->by[p], oy};
            for (int k = 0; k < 2; ++k)
                if (xs[k] < xlo || xs[k] > xhi || ys[k] < ylo || ys[k] > yhi) {
                    set_error("Omega u V+ is not inside the box");
                    free_plan(pl);
                    return FC2D_E_GEOMETRY;
                }
        }
    }
    // column crossings of the 16 B-vertex polygon (parity test of the proximity seed)
    std::vector<int32_t> col_ptr(grid->nx + 1, 0);
    std::vector<double> col_y;
    if (keep_poly) {
        // (column, y) of every crossing, gathered per thread, then sorted:
        // each column's crossings in increasing y whatever the thread count
        std::vector<std::pair<int32_t, double>> xing;
#pragma omp parallel
        {
            std::vector<std::pair<int32_t, double>> loc;
#pragma omp for schedule(static) nowait
            for (int k = 0; k < nv; ++k) {
                const int k1 = (k + 1) % nv;
                const double ax = px[k], ay = py[k], bx = px[k1], by = py[k1];
                const double xmin = std::min(ax, bx), xmax = std::max(ax, bx);
                const long i0 = (long)ceil((xmin - grid->x0) / grid->h);
                const long i1 = (long)ceil((xmax - grid->x0) / grid->h);
                for (long i = i0; i < i1; ++i) {
                    if (i < 0 || i >= grid->nx) continue;
                    const double xc = grid->x0 + i * grid->h;
                    const double s = (xc - ax) / (bx - ax);
                    loc.emplace_back((int32_t)i, ay + s * (by - ay));
                }
            }
#pragma omp critical
            xing.insert(xing.end(), loc.begin(), loc.end());
        }
        std::sort(xing.begin(), xing.end());
        col_y.resize(xing.size());
        for (size_t m = 0; m < xing.size(); ++m) {
            ++col_ptr[xing[m].first + 1];
            col_y[m] = xing[m].second;
        }
        for (int i = 0; i < grid->nx; ++i) col_ptr[i + 1] += col_ptr[i];
    }
    lap(FC2D_PHASE_GEOMETRY);
    // steps 3-4 on the device: classification and foot of the normal
    const int64_t npts = (int64_t)grid->nx * grid->ny;
    const double ds = pl->k2 * spmax;
    ClassifyArgs ca;
    ca.curve = pl->curve;
    ca.x0 = grid->x0; ca.y0 = grid->y0; ca.h = grid->h; ca.nx = grid->nx; ca.ny = grid->ny;
    ca.B = B; ca.M = pl->M; ca.k2 = pl->k2;
    ca.r_out = C * pl->k1 + 0.5 * ds + 1e-12;
    ca.r_in = 0.5 * ds + grid->h;
    ca.width = C * pl->k1;
    ca.maxit = o.newton_maxit;
    double *d_bx = nullptr, *d_by = nullptr, *d_bnx = nullptr, *d_bny = nullptr, *d_coly = nullptr;
    int32_t* d_colptr = nullptr;
    int8_t* d_cls = nullptr;
    StripRec* d_rec = nullptr;
    HostVec<int32_t> mref;
    HostVec<double> mwv, mwn;
    uint64_t* d_near = nullptr;
    int32_t* d_cand = nullptr;
    float* d_w = nullptr;
    int* d_cnt = nullptr;
    // capacity for STRIP records: twice the area of a band of width r_out
    // along the boundary, plus a margin of a few grid rows
    double perim = 0.0, rmin = INFINITY, rmax = 0.0, slope = 0.0;
    for (int p = 0; p < B; ++p) perim += spd[p] * pl->k2;
    if (pl->curve.kind == FC2D_CURVE_POLAR) {
#pragma omp parallel for reduction(min : rmin) reduction(max : rmax, slope)
        for (int p = 0; p < B; ++p) {
            double r, r1, r2;
            series3(pl->curve.a, pl->curve.nmodes, p * pl->k2, &r, &r1, &r2);
            rmin = std::min(rmin, r);
            rmax = std::max(rmax, r);
            slope = std::max(slope, fabs(r1) / r);
        }
    }
    const double hh = grid->h;
    int64_t cap = std::min<int64_t>(
        npts, (int64_t)(2.0 * perim * ca.r_out / (hh * hh) + 4.0 * perim / hh) + 4096);
    // polar seeds: candidates have rho - r(phi) in [band_lo, band_hi].  To first
    // order rho - r(phi) = eta sqrt(1 + (r'/r)^2); the band takes 1.25 times
    // that for the outer search radius plus two grid steps, and inside only
    // points within rounding distance of Gamma (the rest are IN).
    SeedArgs sa;
    memset(&sa, 0, sizeof sa);
    int64_t cap_cand = 0;
    if (o.seed != FC2D_SEED_PROXIMITY) {
        if (!(rmin > 0.0)) {
            set_error("polar seeds need r(t) > 0");
            free_plan(pl);
            return FC2D_E_ARG;
        }
        sa.curve = pl->curve;
        sa.x0 = grid->x0; sa.y0 = grid->y0; sa.h = grid->h; sa.nx = grid->nx; sa.ny = grid->ny;
        sa.B = B; sa.maxit = o.newton_maxit; sa.k2 = pl->k2;
        sa.band_hi = 1.25 * ca.r_out * sqrt(1.0 + slope * slope) + 2.0 * hh;
        sa.band_lo = -1e-12 * (1.0 + rmax);
        sa.width = ca.width;
        const double dmax = std::min(sa.band_hi, 0.99 * reach_ext);
        sa.dist2_max = dmax * dmax;
        sa.mlp_tol = o.mlp_tol;
        cap_cand = std::min<int64_t>(
            npts, (int64_t)(2.0 * perim * (sa.band_hi - sa.band_lo) / (hh * hh) + 4.0 * perim / hh) + 4096);
    }
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // temporaries of the plan's creation come from the library's stream-ordered
    // pool and go back to it on the plan's stream
    auto cleanup = [&]() {
        void* ps[] = {d_bx, d_by, d_bnx, d_bny, d_coly, d_colptr, d_rec, d_near, d_cand, d_w, d_cnt};
        for (void* q : ps)
            if (q) (void)ws_free(q, stream);
    };
    st = FC2D_OK;
    do {
        if (hipMalloc((void**)&pl->d_cls, npts) != hipSuccess) {
            set_error("hipMalloc failed (classes)");
            st = FC2D_E_NOMEM;
            break;
        }
        if ((st = ws_alloc(cap * sizeof(StripRec), stream, (void**)&d_rec)) ||
            (st = ws_alloc(8 * sizeof(int), stream, (void**)&d_cnt)))
            break;
        d_cls = pl->d_cls;
        hipError_t e;
        // boundary samples on the device: proximity seeds and the red-star scan
        if ((st = ws_upload(&d_bx, pl->bx.data(), B, stream))) break;
        if ((st = ws_upload(&d_by, pl->by.data(), B, stream))) break;
        if ((st = ws_upload(&d_bnx, pl->bnx.data(), B, stream))) break;
        if ((st = ws_upload(&d_bny, pl->bny.data(), B, stream))) break;
        if (o.seed == FC2D_SEED_PROXIMITY) {
            if ((st = ws_upload(&d_colptr, col_ptr.data(), col_ptr.size(), stream))) break;
            if (!col_y.empty() && (st = ws_upload(&d_coly, col_y.data(), col_y.size(), stream))) break;
            if ((st = ws_alloc(npts * sizeof(uint64_t), stream, (void**)&d_near))) break;
            ca.bx = d_bx; ca.by = d_by; ca.bnx = d_bnx; ca.bny = d_bny;
            ca.col_ptr = d_colptr; ca.col_y = d_coly;
            trace_point("plan_host", stream);   // kernel times below exclude the host set-up
            if ((st = launch_classify(ca, d_cls, d_rec, cap, d_near, d_cnt, stream))) break;
        } else {
            if ((st = ws_alloc(cap_cand * sizeof(int32_t), stream, (void**)&d_cand))) break;
            if (o.seed == FC2D_SEED_MLP && (st = ws_upload(&d_w, o.mlp_weights, FC2D_MLP_NW, stream))) break;
            trace_point("plan_host", stream);
            if ((st = launch_radial_band(sa, d_cls, d_cand, cap_cand, d_cnt, stream))) break;
            if ((e = hipMemcpyAsync(cnt, d_cnt, 8 * sizeof(int), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
                (e = hipStreamSynchronize(stream)) != hipSuccess) {
                st = hip_fail(e, "radial band");
                break;
            }
            if (cnt[3] > cap_cand) { set_error("candidate capacity exceeded"); st = FC2D_E_GEOMETRY; break; }
            trace_point("plan_host", stream);
            st = o.seed == FC2D_SEED_MLP
                     ? launch_seed_mlp(sa, d_w, d_cand, cnt[3], d_cls, d_rec, cap, d_cnt, stream)
                     : launch_seed_polar(sa, d_cand, cnt[3], d_cls, d_rec, cap, d_cnt, stream);
            if (st) break;
        }
        if ((e = hipMemcpyAsync(cnt, d_cnt, 8 * sizeof(int), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess) {
            st = hip_fail(e, "classification kernels");
            break;
        }
        if (cnt[1] > 0) {
            char buf[128];
            snprintf(buf, sizeof buf, "foot of the normal failed at %d grid points", cnt[1]);
            set_error(buf);
            st = FC2D_E_NEWTON;
            break;
        }
        if (cnt[0] > cap) { set_error("STRIP capacity exceeded"); st = FC2D_E_GEOMETRY; break; }
        lap(FC2D_PHASE_CLASSIFY);
        // runs, pair classes and the STRIP lists, built on the device
        if ((st = plan_device_lists(pl, d_rec, cnt[0], stream))) break;
        pl->newton_max_iters = cnt[2];
        pl->n_solved = cnt[3];
        pl->n_fallback = cnt[4];
        pl->newton_iters = cnt[5];
        lap(FC2D_PHASE_LISTS);
        // matching stencils
        const BndView dbd{d_bx, d_by, d_bnx, d_bny, B, pl->k2};
        st = build_matching(pl, o.newton_maxit, dbd, stream, mref, mwv, mwn);
        if (st) break;
        lap(FC2D_PHASE_MATCHING);
    } while (0);
    cleanup();
    if (st) { free_plan(pl); return st; }
    // uploads
    do {
        if ((st = dev_upload(&pl->d_Q, pl->Q.data(), pl->Q.size()))) break;
        if ((st = dev_upload(&pl->d_Ar, pl->Ar.data(), pl->Ar.size()))) break;
        {
            // device layout of the matching stencils: each normal's M*M entries in
            // address order, dealt to the 4 lanes of a group (entry 4u + sq to lane
            // sq), and the weights interleaved over the 4 lanes
            const int M = pl->M, d = pl->d, B = pl->B;
            const int nq = pl->interior_only ? d : d - 1;   // matching values along the normal
            const int MM = M * M, NU = (MM + 15) / 16 * 4, RQ = (nq + 3) / 4;
            const int64_t npts = (int64_t)grid->nx * grid->ny;
            const int RS = (M + 3) / 4;   // stars per lane
            // filled per normal (padding first) inside the parallel loop
            HostVec<int32_t> dref((size_t)B * 4 * NU);
            HostVec<uint8_t> dlab((size_t)B * 4 * NU);
            HostVec<double> dwv((size_t)B * RS * M * 4 * 2), dwn((size_t)B * RQ * M * 4 * 2);
#pragma omp parallel for
            for (int p = 0; p < B; ++p) {
                std::fill_n(&dref[(size_t)p * 4 * NU], 4 * NU, 0);
                std::fill_n(&dlab[(size_t)p * 4 * NU], 4 * NU, (uint8_t)255);
                std::fill_n(&dwv[(size_t)p * RS * M * 4 * 2], RS * M * 4 * 2, 0.0);
                std::fill_n(&dwn[(size_t)p * RQ * M * 4 * 2], RQ * M * 4 * 2, 0.0);
                int ord[kMaxStencil * kMaxStencil];
                const int32_t* r0 = &mref[(size_t)p * MM];
                auto key = [&](int e) { return r0[e] >= 0 ? (int64_t)r0[e] : npts + (int64_t)(-r0[e] - 1); };
                int nuse = 0;   // entries of unused stencils stay padding (label 255)
                for (int e = 0; e < MM; ++e)
                    if (r0[e] != kUnusedRef) ord[nuse++] = e;
                std::stable_sort(ord, ord + nuse, [&](int a, int b) { return key(a) < key(b); });
                for (int i = 0; i < nuse; ++i) {
                    const size_t o = ((size_t)p * 4 + i % 4) * NU + i / 4;
                    dref[o] = r0[ord[i]];
                    dlab[o] = (uint8_t)ord[i];
                }
                for (int r = 0; r < RS; ++r)
                    for (int k = 0; k < M; ++k)
                        for (int sq = 0; sq < 4; ++sq) {
                            const int sv = 4 * r + sq;
                            if (sv >= M) continue;
                            const size_t on = (((size_t)p * RS + r) * M + k) * 4 + sq;
                            const size_t oo = ((size_t)p * M + sv) * M + k;
                            dwv[2 * on] = mwv[2 * oo];
                            dwv[2 * on + 1] = mwv[2 * oo + 1];
                        }
                for (int r = 0; r < RQ; ++r)
                    for (int sv = 0; sv < M; ++sv)
                        for (int sq = 0; sq < 4; ++sq) {
                            const int q = 4 * r + sq;
                            if (q >= nq) continue;
                            const size_t on = (((size_t)p * RQ + r) * M + sv) * 4 + sq;
                            const size_t oo = ((size_t)p * nq + q) * M + sv;
                            dwn[2 * on] = mwn[2 * oo];
                            dwn[2 * on + 1] = mwn[2 * oo + 1];
                        }
            }
            if ((st = dev_upload(&pl->d_mref, dref.data(), dref.size()))) break;
            if ((st = dev_upload(&pl->d_mlab, dlab.data(), dlab.size()))) break;
            if ((st = dev_upload(&pl->d_mwv, dwv.data(), dwv.size()))) break;
            if ((st = dev_upload(&pl->d_mwn, dwn.data(), dwn.size()))) break;
        }
        {
            std::vector<double> bxy(2 * (size_t)B + pl->squares.size());
            for (int p = 0; p < B; ++p) { bxy[2 * p] = pl->bx[p]; bxy[2 * p + 1] = pl->by[p]; }
            std::copy(pl->squares.begin(), pl->squares.end(), bxy.begin() + 2 * B);
            if ((st = dev_upload(&pl->d_bxy, bxy.data(), bxy.size()))) break;
        }
        if (pl->d_cls2) {
            // set-up on this device for the extension calls that allocate nothing
            // (fc2d_extend_fft_noalloc): the FFT tables and the fixed scratch's address
            if ((st = fft_prepare(grid->nx, grid->ny))) { set_error("FFT table set-up failed"); break; }
            double* scr = nullptr;
            size_t scr_bytes = 0;
            if ((st = static_scratch(&scr, &scr_bytes))) break;
        }
    } while (0);
    if (st) { free_plan(pl); return st; }
    lap(FC2D_PHASE_LAYOUT);
    *out = pl;
    return FC2D_OK;
}



// Crossing of the grid-line segment {a = a_line, b between b_in (inside) and
// b_out (outside)} with Gamma: bisection on the sign of eta (64 halvings, one
// foot solve each).  vertical: the line x = a_line (b runs along y).
int gridline_crossing(const fc2d_plan* pl, bool vertical, double a_line, double b_in, double b_out, double* out) {
    const BndView bd{pl->bx.data(), pl->by.data(), pl->bnx.data(), pl->bny.data(), pl->B, pl->k2};
    int seed = 0;
    {
        const double X = vertical ? a_line : b_in, Y = vertical ? b_in : a_line;
        double best = INFINITY;
        for (int p = 0; p < pl->B; ++p) {
            const double dx = pl->bx[p] - X, dy = pl->by[p] - Y, d2 = dx * dx + dy * dy;
            if (d2 < best) { best = d2; seed = p; }
        }
    }
    double lo = b_in, hi = b_out;
    for (int it = 0; it < 64; ++it) {
        const double mid = 0.5 * (lo + hi);
        const double X = vertical ? a_line : mid;
        const double Y = vertical ? mid : a_line;
        seed = nearest_sample(pl, X, Y, seed);
        double th, eta;
        int its;
        if (foot_host(pl->M, pl->curve, bd, X, Y, seed, 60, &th, &eta, &its) != FOOT_OK) {
            set_error("foot of the normal failed while locating a grid-line crossing with the boundary");
            return FC2D_E_NEWTON;
        }
        if (eta <= 0) lo = mid;
        else hi = mid;
    }
    *out = 0.5 * (lo + hi);
    return FC2D_OK;
}

// Host copies of the classes and the row-major STRIP list, downloaded from the
// plan's device arrays on first use (synchronous; the plan's device data is
// complete once fc2d_plan_create has returned).
int plan_host_lists(const fc2d_plan* pl) {
    std::lock_guard<std::mutex> lk(pl->host_mu);
    if (pl->host_ready) return FC2D_OK;
    const size_t npts = (size_t)pl->grid.nx * pl->grid.ny, S = (size_t)pl->n_strip;
    pl->cls.resize(npts);
    pl->strip_idx.resize(S); pl->strip_seed.resize(S); pl->strip_theta.resize(S); pl->strip_eta.resize(S);
    hipError_t e;
    if ((e = hipMemcpy(pl->cls.data(), pl->d_cls, npts, hipMemcpyDeviceToHost)) != hipSuccess ||
        (S && ((e = hipMemcpy(pl->strip_idx.data(), pl->d_rm_idx, S * sizeof(int32_t), hipMemcpyDeviceToHost)) != hipSuccess ||
               (e = hipMemcpy(pl->strip_seed.data(), pl->d_rm_seed, S * sizeof(int32_t), hipMemcpyDeviceToHost)) != hipSuccess ||
               (e = hipMemcpy(pl->strip_theta.data(), pl->d_rm_th, S * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess ||
               (e = hipMemcpy(pl->strip_eta.data(), pl->d_rm_eta, S * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)))
        return hip_fail(e, "plan lists download");
    pl->host_ready = true;
    return FC2D_OK;
}

}  // namespace fc2d

using namespace fc2d;

extern "C" {

void fc2d_opts_default(const fc2d_grid* grid, fc2d_opts* o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->n_r = 6; o->Z = 12; o->n_os = 20; o->mf = 20; o->newton_maxit = 60;
    o->seed = FC2D_SEED_PROXIMITY; o->mlp_tol = 1e-13; o->mlp_weights = nullptr;
    o->M = 0;
    o->k1 = grid ? grid->h : 0.0;
    int B = 256;
    if (grid && grid->h > 0) {
        const double t = 2.0 * M_PI / grid->h;
        B = 1 << (int)lround(log2(t));
    }
    o->B = B;
}

int fc2d_plan_create(const fc2d_curve* curve, const fc2d_grid* grid, int d, int C, const fc2d_opts* opts,
                     hipStream_t stream, fc2d_plan** out) {
    try {
        return create_plan(curve, grid, d, C, opts, stream, out);
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return FC2D_E_NOMEM;
    }
}

int fc2d_plan_destroy(fc2d_plan* plan) {
    free_plan(plan);
    return FC2D_OK;
}

int fc2d_plan_get_info(const fc2d_plan* pl, fc2d_plan_info* info) {
    if (!pl || !info) { set_error("NULL argument"); return FC2D_E_ARG; }
    info->d = pl->d; info->C = pl->C; info->M = pl->M; info->n_r = pl->n_r; info->Cr = pl->Cr; info->B = pl->B;
    info->k1 = pl->k1; info->k2 = pl->k2;
    info->n_bdry = pl->B + (int64_t)pl->squares.size() / 2;
    info->n_strip = pl->n_strip;
    info->n_in = pl->n_in; info->n_far = pl->n_far;
    info->newton_max_iters = pl->newton_max_iters;
    info->seed = pl->seed;
    info->n_solved = pl->n_solved;
    info->n_fallback = pl->n_fallback;
    info->newton_iters = pl->newton_iters;
    for (int k = 0; k < FC2D_PLAN_PHASES; ++k) info->t_ms[k] = pl->t_ms[k];
    return FC2D_OK;
}

int fc2d_boundary_points(const fc2d_plan* pl, int64_t* n, double* xy) {
    if (!pl || !n) { set_error("NULL argument"); return FC2D_E_ARG; }
    const int64_t ns = (int64_t)pl->squares.size() / 2;
    *n = pl->B + ns;
    if (xy) {
        for (int p = 0; p < pl->B; ++p) { xy[2 * p] = pl->bx[p]; xy[2 * p + 1] = pl->by[p]; }
        memcpy(xy + 2 * pl->B, pl->squares.data(), pl->squares.size() * sizeof(double));
    }
    return FC2D_OK;
}

int fc2d_plan_classes(const fc2d_plan* pl, int8_t* classes) {
    if (!pl) { set_error("NULL argument"); return FC2D_E_ARG; }
    if (int st = plan_host_lists(pl)) return st;
    if (classes) memcpy(classes, pl->cls.data(), pl->cls.size());
    return FC2D_OK;
}

int fc2d_plan_strip(const fc2d_plan* pl, int64_t* index, double* theta, double* eta, int32_t* seed) {
    if (!pl) { set_error("NULL argument"); return FC2D_E_ARG; }
    if (int st = plan_host_lists(pl)) return st;
    const size_t S = pl->strip_idx.size();
    for (size_t k = 0; k < S; ++k) {
        if (index) index[k] = pl->strip_idx[k];
        if (theta) theta[k] = pl->strip_theta[k];
        if (eta) eta[k] = pl->strip_eta[k];
        if (seed) seed[k] = pl->strip_seed[k];
    }
    return FC2D_OK;
}

static int check_fields(const fc2d_plan* pl, int nf) {
    if (!pl || nf < 0) { set_error("invalid plan or field count"); return FC2D_E_ARG; }
    return FC2D_OK;
}

int fc2d_matching(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, double* fD, int nf,
                  hipStream_t s) {
    int st = check_fields(pl, nf);
    if (st) return st;
    if (nf == 0) return FC2D_OK;
    if (!f_grid || (!f_bdry && !pl->interior_only) || !fD) { set_error("NULL argument"); return FC2D_E_ARG; }
    WorkSpace ws;
    if ((st = ws.alloc(gram_bytes(pl, nf), s))) return st;
    const int64_t nb = pl->B + (int64_t)pl->squares.size() / 2;
    return launch_match(pl, f_grid, f_bdry, nb, (double*)ws.p, fD, nf, s);
}

int fc2d_blend(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, double* F, int nf,
               hipStream_t s) {
    int st = check_fields(pl, nf);
    if (st) return st;
    if (nf == 0) return FC2D_OK;
    if (!f_grid || (!f_bdry && !pl->interior_only) || !F) { set_error("NULL argument"); return FC2D_E_ARG; }
    WorkSpace ws;
    if ((st = ws.alloc(gram_bytes(pl, nf), s))) return st;
    double* c = (double*)ws.p;
    const int64_t nb = pl->B + (int64_t)pl->squares.size() / 2;
    if ((st = launch_match(pl, f_grid, f_bdry, nb, c, nullptr, nf, s))) return st;
    return launch_blend(pl, c, F, nf, s);
}

int fc2d_extend(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, double* out, int nf,
                hipStream_t s) {
    int st = check_fields(pl, nf);
    if (st) return st;
    if (nf == 0) return FC2D_OK;
    if (!f_grid || (!f_bdry && !pl->interior_only) || !out) { set_error("NULL argument"); return FC2D_E_ARG; }
    WorkSpace ws;
    if ((st = ws.alloc(gram_bytes(pl, nf), s))) return st;
    double* c = (double*)ws.p;
    const int64_t nb = pl->B + (int64_t)pl->squares.size() / 2;
    if ((st = launch_match(pl, f_grid, f_bdry, nb, c, nullptr, nf, s))) return st;
    if ((st = launch_mask(pl, f_grid, out, nf, s))) return st;
    return launch_strip(pl, c, f_bdry, nb, out, nf, s);
}

static int extend_fft_check(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, const double* work,
                            const void* spec, int nf) {
    int st = check_fields(pl, nf);
    if (st) return st;
    if (nf == 0) return FC2D_OK;
    const fc2d_grid* g = &pl->grid;
    if (!f_grid || (!f_bdry && !pl->interior_only) || !work || !spec) { set_error("NULL argument"); return FC2D_E_ARG; }
    if (g->nx < 16 || g->nx > 4096 || (g->nx & (g->nx - 1)) || g->ny < 16 || g->ny > 8192 || (g->ny & (g->ny - 1)) ||
        !pl->d_cls2) {
        set_error("fc2d_extend_fft: the plan's grid must have power-of-two sizes (nx <= 4096, ny <= 8192)");
        return FC2D_E_ARG;
    }
    return FC2D_OK;
}

// matching -> strip -> masked row pass -> column pass, Gram records in c,
// half-spectrum rows at pitch ld (complex elements; 0 -> ny/2 + 1)
static int extend_fft_run(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, double* work, void* spec,
                          int nf, double* c, hipStream_t s, int ld = 0) {
    int st;
    const int64_t nb = pl->B + (int64_t)pl->squares.size() / 2;
    if ((st = launch_match(pl, f_grid, f_bdry, nb, c, nullptr, nf, s))) return st;
    if ((st = launch_strip(pl, c, f_bdry, nb, work, nf, s))) return st;
    return fft2_r2c(&pl->grid, f_grid, (double*)spec, nf, s, work, pl->d_cls2, ld);
}

int fc2d_extend_fft(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, double* work, void* spec,
                    int nf, hipStream_t s) {
    int st = extend_fft_check(pl, f_grid, f_bdry, work, spec, nf);
    if (st || nf == 0) return st;
    WorkSpace ws;
    if ((st = ws.alloc(gram_bytes(pl, nf), s))) return st;
    return extend_fft_run(pl, f_grid, f_bdry, work, spec, nf, (double*)ws.p, s);
}

int fc2d_extend_fft_ld(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, double* work, void* spec,
                       int spec_ld, int nf, hipStream_t s) {
    int st = extend_fft_check(pl, f_grid, f_bdry, work, spec, nf);
    if (st || nf == 0) return st;
    if (spec_ld < pl->grid.ny / 2 + 1) {
        set_error("fc2d_extend_fft_ld: spec_ld must be at least ny/2 + 1");
        return FC2D_E_ARG;
    }
    WorkSpace ws;
    if ((st = ws.alloc(gram_bytes(pl, nf), s))) return st;
    return extend_fft_run(pl, f_grid, f_bdry, work, spec, nf, (double*)ws.p, s, spec_ld);
}

int fc2d_extend_fft_noalloc(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, double* work,
                            void* spec, int nf, hipStream_t s) {
    int st = extend_fft_check(pl, f_grid, f_bdry, work, spec, nf);
    if (st || nf == 0) return st;
    double* c = nullptr;
    size_t cap = 0;
    if ((st = static_scratch(&c, &cap))) return st;
    if (gram_bytes(pl, nf) > cap) {
        set_error("fc2d_extend_fft_noalloc: nf B (d + 2 rounded down to even) doubles exceed the fixed scratch of " +
                  std::to_string(cap) + " bytes");
        return FC2D_E_ARG;
    }
    if (!fft_ready(pl->grid.nx, pl->grid.ny)) {
        set_error("fc2d_extend_fft_noalloc: no FFT tables on this device (create a plan on it first)");
        return FC2D_E_ARG;
    }
    return extend_fft_run(pl, f_grid, f_bdry, work, spec, nf, c, s);
}

int fc2d_boundary_values(const fc2d_plan* pl, const double* u, double* f_bdry, int nf, hipStream_t s) {
    int st = check_fields(pl, nf);
    if (st) return st;
    if (nf == 0) return FC2D_OK;
    if (!u || !f_bdry) { set_error("NULL argument"); return FC2D_E_ARG; }
    return launch_bvals(pl, u, f_bdry, nf, s);
}

static bool pow2_ok(int n, int nmax) { return n >= 16 && n <= nmax && (n & (n - 1)) == 0; }

int fc2d_fft_ld(const fc2d_grid* g, void* in, void* out, int dir, int spec_ld, int nf, hipStream_t s) {
    if (!g || !pow2_ok(g->nx, 4096) || !pow2_ok(g->ny, 8192) || nf < 0) {
        set_error("fc2d_fft: nx must be a power of two in [16, 4096] and ny one in [16, 8192]");
        return FC2D_E_ARG;
    }
    if (spec_ld < g->ny / 2 + 1) {
        set_error("fc2d_fft: spec_ld must be at least ny/2 + 1");
        return FC2D_E_ARG;
    }
    if (nf == 0) return FC2D_OK;
    if (!in || !out || in == out) { set_error("fc2d_fft: NULL or aliased buffers"); return FC2D_E_ARG; }
    if (dir == FC2D_FORWARD) return fft2_r2c(g, (const double*)in, (double*)out, nf, s, nullptr, nullptr, spec_ld);
    if (dir == FC2D_INVERSE) return fft2_c2r(g, (double*)in, (double*)out, nf, s, spec_ld);
    set_error("fc2d_fft: dir must be FC2D_FORWARD or FC2D_INVERSE");
    return FC2D_E_ARG;
}

int fc2d_fft(const fc2d_grid* g, void* in, void* out, int dir, int nf, hipStream_t s) {
    return fc2d_fft_ld(g, in, out, dir, g ? g->ny / 2 + 1 : 0, nf, s);
}

int fc2d_spectral_apply(const fc2d_grid* g, int op, const void* in, void* out, int nf, hipStream_t s) {
    if (!g || g->nx < 2 || g->ny < 2 || g->h <= 0 || nf < 0 ||
        (op != FC2D_LAPLACE_INV && op != FC2D_DX && op != FC2D_DY)) {
        set_error("fc2d_spectral_apply: invalid arguments");
        return FC2D_E_ARG;
    }
    if (nf == 0) return FC2D_OK;
    if (!in || !out) { set_error("NULL argument"); return FC2D_E_ARG; }
    return spectral_apply(g, op, (const double*)in, (double*)out, nf, s);
}

int ff_propagate(const fc2d_grid* g, double c, double t, const void* u0h, const void* u1h, void* uh, void* uth,
                 int nf, hipStream_t s) {
    if (!g || g->nx < 2 || g->ny < 2 || g->h <= 0 || nf < 0) {
        set_error("ff_propagate: invalid arguments");
        return FC2D_E_ARG;
    }
    if (nf == 0) return FC2D_OK;
    if (!u0h || !u1h || !uh || !uth) { set_error("NULL argument"); return FC2D_E_ARG; }
    return ff_apply(g, c, t, (const double*)u0h, (const double*)u1h, (double*)uh, (double*)uth, nf, s);
}

const char* fc2d_strerror(int status) {
    switch (status) {
        case FC2D_OK: return "ok";
        case FC2D_E_ARG: return "invalid argument";
        case FC2D_E_TABLE: return "FC-Gram table unavailable";
        case FC2D_E_GEOMETRY: return "inadmissible geometry";
        case FC2D_E_NEWTON: return "foot-of-normal solve failed";
        case FC2D_E_HIP: return "HIP runtime error";
        case FC2D_E_NOMEM: return "out of memory";
    }
    return "unknown status";
}

const char* fc2d_last_error(void) { return g_last_error.c_str(); }

int fc2d_tune_set(int knob, int n, int value) {
    int st = FC2D_E_ARG;
    if (knob == FC2D_TUNE_COL_TILE) st = col_tile_set(n, value);
    else if (knob == FC2D_TUNE_COL_ELEMS) st = col_elems_set(n, value);
    else if (knob == FC2D_TUNE_STRIP_FIELDS) st = strip_fpt_set(value);
    else if (knob == FC2D_TUNE_STRIP_WINDOW) st = strip_wcap_set(value);
    else if (knob == FC2D_TUNE_FF_SHAPE) st = colff_set(n, value);
    if (st) set_error("fc2d_tune_set: unsupported knob or value");
    return st;
}

int fc2d_tune_get(int knob, int n, int* value) {
    if (!value) { set_error("NULL argument"); return FC2D_E_ARG; }
    if (knob == FC2D_TUNE_COL_TILE) *value = col_tile_get(n);
    else if (knob == FC2D_TUNE_COL_ELEMS) *value = col_elems_get(n);
    else if (knob == FC2D_TUNE_STRIP_FIELDS) *value = strip_fpt_get();
    else if (knob == FC2D_TUNE_STRIP_WINDOW) *value = strip_wcap_get();
    else if (knob == FC2D_TUNE_FF_SHAPE) *value = colff_get(n);
    else { set_error("fc2d_tune_get: unknown knob"); return FC2D_E_ARG; }
    return FC2D_OK;
}

int fc2d_trace_begin(hipStream_t stream) {
    {
        std::lock_guard<std::mutex> lk(g_trace_mu);
        for (auto& t : g_trace) (void)hipEventDestroy(t.ev);
        g_trace.clear();
        g_trace_on = true;
    }
    trace_point("begin", stream);
    return FC2D_OK;
}

int fc2d_trace_end(int* n, const char** names, float* ms, int cap) {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    g_trace_on = false;
    int k = 0;
    int st = FC2D_OK;
    for (const TraceRec& r : g_trace) {
        hipError_t e = hipEventSynchronize(r.ev);
        if (e != hipSuccess) { st = hip_fail(e, "fc2d_trace_end"); break; }
    }
    for (size_t i = 1; i < g_trace.size() && st == FC2D_OK; ++i) {
        if (!g_trace[i].name) continue;   // marker
        size_t j = i;
        while (j > 0 && g_trace[j - 1].stream != g_trace[i].stream) --j;
        const size_t prev = j > 0 ? j - 1 : 0;
        if (k < cap) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, g_trace[prev].ev, g_trace[i].ev) != hipSuccess) t = -1.0f;
            if (names) names[k] = g_trace[i].name;
            if (ms) ms[k] = t;
        }
        ++k;
    }
    for (auto& t : g_trace) (void)hipEventDestroy(t.ev);
    g_trace.clear();
    if (n) *n = std::min(k, cap);
    return st;
}

int fc2d_version(void) { return FC2D_VERSION; }

}  // extern "C"
