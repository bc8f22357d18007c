// Full 2D-FC Poisson solve (Sec. 4.1), host orchestration: every numerical
// step runs in the library's kernels (extension + FFT, spectral inversion,
// mean term, boundary interpolation, Nystrom matrix, GMRES vector operations,
// density refinement, double-layer evaluation); the host only sequences the
// launches and runs GMRES's small Hessenberg least-squares problem.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <mutex>
#include <vector>

#include "internal.h"
#include "poisson_int.h"

using namespace fc2d;

namespace {

constexpr int kRefine = 1 << (kPoisLevels - 1);   // finest density refinement of the near-boundary sums
constexpr int kRestart = 80;     // GMRES restart length
constexpr int kMaxRestarts = 20;
constexpr double kGmresTol = 1e-14;

// (x, y, x', y', x'', y'') at t_j = 2 pi j / n
void node_data(const CurveC& cv, int n, std::vector<double>& qd) {
    qd.resize(6 * (size_t)n);
    for (int j = 0; j < n; ++j) curve_eval(cv, 2.0 * M_PI * (double)j / (double)n, &qd[6 * (size_t)j]);
}

// all device buffers of a solve in one per-call work space (256-byte aligned
// pieces), taken on the solve's stream and returned on it when the solve ends
struct PoisArena {
    std::vector<std::pair<void**, size_t>> req;
    WorkSpace ws;
    template <class T>
    void add(T** p, size_t n) {
        req.push_back({(void**)p, (std::max<size_t>(n, 1) * sizeof(T) + 255) & ~(size_t)255});
    }
    int commit(hipStream_t s) {
        size_t tot = 0;
        for (auto& r : req) tot += r.second;
        int st = ws.alloc(tot, s);
        if (st) return st;
        size_t off = 0;
        for (auto& r : req) {
            *r.first = (char*)ws.p + off;
            off += r.second;
        }
        return FC2D_OK;
    }
};

}  // namespace

namespace {

int hip_err(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return FC2D_E_HIP;
}

// Pinned host memory and two events for the GMRES Hessenberg columns, one set
// per calling thread, grown on demand and kept for the thread's life (never
// freed: a pinned allocation and its release cost more than a solve's
// iterations, and releasing it at thread exit could outlive the runtime);
// the events belong to the device current at creation.
struct PinnedCols {
    double* p;
    size_t cap;
    int dev;
    hipEvent_t ev[2];
};
thread_local PinnedCols t_pin = {nullptr, 0, -1, {nullptr, nullptr}};

int pinned_get(size_t doubles) {
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_err(e, "gmres");
    if (t_pin.dev != dev) {
        for (hipEvent_t& v : t_pin.ev) {
            if (v) (void)hipEventDestroy(v);
            v = nullptr;
        }
        t_pin.dev = -1;
        if ((e = hipEventCreateWithFlags(&t_pin.ev[0], hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&t_pin.ev[1], hipEventDisableTiming)) != hipSuccess)
            return hip_err(e, "gmres");
        t_pin.dev = dev;
    }
    if (t_pin.cap < doubles) {
        if (t_pin.p) (void)hipHostFree(t_pin.p);
        t_pin.p = nullptr;
        t_pin.cap = 0;
        if ((e = hipHostMalloc((void**)&t_pin.p, doubles * sizeof(double), hipHostMallocDefault)) != hipSuccess)
            return hip_err(e, "gmres");
        t_pin.cap = doubles;
    }
    return FC2D_OK;
}

// Restarted GMRES with classical Gram-Schmidt applied twice, for nfc systems
// A x_f = b_f at once (A column-major n x n on the device, read once per
// iteration for all of them; b and x hold the fields n apart; x starts at
// zero).  The next basis vector is normalised on the device, so Arnoldi step
// j + 1 is queued before the host takes step j's Hessenberg column (one copy
// into a pinned double buffer and one wait per step for all fields): the
// device never waits for the host's Givens rotations.  A step queued past a
// field's convergence is discarded (its basis columns take zero weights; a
// zero norm gives a zero vector).  V: nfc (m + 1) n, w: nfc n, hd: nfc
// (3 (m + 2) + m) device doubles; iters: iterations summed over fields.
int gmres(const double* A, const double* b, double* x, int n, int nfc, double* V, double* w, double* hd,
          double* part, hipStream_t s, int* iters) {
    const int m = std::min(n, kRestart);
    const int64_t VS = (int64_t)(m + 1) * n;                 // basis stride per field
    const int64_t HS = 3 * (int64_t)(m + 2) + m;             // h1 [m + 1], h2 [m + 1], norm, y [m]
    const int64_t o2 = m + 1, on = 2 * (m + 1), oy = 2 * (m + 1) + 1;
    std::vector<double> H((size_t)nfc * (m + 1) * m), cs((size_t)nfc * m), sn((size_t)nfc * m),
        g((size_t)nfc * (m + 1)), hh((size_t)nfc * HS), bnorm(nfc), beta(nfc), scal(nfc);
    std::vector<int> k(nfc, 0);
    std::vector<char> done(nfc, 0), act(nfc, 0), conv(nfc, 0);
    int st;
    hipError_t e;
    *iters = 0;
    if ((e = hipMemsetAsync(x, 0, (size_t)nfc * n * sizeof(double), s)) != hipSuccess) return hip_err(e, "gmres");
    // pinned double buffer for the Hessenberg columns and one event per slot
    // (kept by the calling thread across solves)
    if ((st = pinned_get(2 * hh.size()))) return st;
    PinnedCols& pin = t_pin;
    // Arnoldi step j: w = A V_j orthogonalised twice against V_0..V_j, its
    // column to pinned slot j & 1, V_{j+1} = w / |w|
    auto step = [&](int j) -> int {
        int r;
        if ((r = pois_matvec(A, V + (size_t)j * n, VS, n, nfc, part, w, s)) ||
            (r = pois_dots(V, VS, j + 1, w, n, n, nfc, hd, HS, s)) ||
            (r = pois_sub(V, VS, j + 1, hd, HS, n, nfc, w, n, s)) ||
            (r = pois_dots(V, VS, j + 1, w, n, n, nfc, hd + o2, HS, s)) ||
            (r = pois_sub(V, VS, j + 1, hd + o2, HS, n, nfc, w, n, s)) ||
            (r = pois_dots(w, n, 1, w, n, n, nfc, hd + on, HS, s)))
            return r;
        double* slot = pin.p + (size_t)(j & 1) * hh.size();
        if ((e = hipMemcpyAsync(slot, hd, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipEventRecord(pin.ev[j & 1], s)) != hipSuccess)
            return hip_err(e, "gmres");
        return pois_normalize(w, n, n, nfc, hd + on, HS, V + (size_t)(j + 1) * n, VS, s);
    };
    auto fetch = [&]() -> int {
        if ((e = hipMemcpyAsync(hh.data(), hd, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_err(e, "gmres");
        return FC2D_OK;
    };
    if ((st = pois_dots(b, n, 1, b, n, n, nfc, hd + on, HS, s)) || (st = fetch())) return st;
    bool all = true;
    for (int f = 0; f < nfc; ++f) {
        bnorm[f] = beta[f] = sqrt(hh[f * HS + on]);
        done[f] = bnorm[f] == 0.0;
        scal[f] = done[f] ? 0.0 : 1.0 / beta[f];
        all = all && done[f];
    }
    if (all) return FC2D_OK;
    if ((st = pois_scale(scal.data(), b, n, n, nfc, V, VS, s))) return st;   // V_f,0 = b_f / |b_f|
    for (int rs = 0; rs < kMaxRestarts; ++rs) {
        for (int f = 0; f < nfc; ++f) {
            std::fill(g.begin() + (size_t)f * (m + 1), g.begin() + (size_t)(f + 1) * (m + 1), 0.0);
            g[(size_t)f * (m + 1)] = beta[f];
            k[f] = 0;
            act[f] = !done[f];
            conv[f] = 0;
        }
        int kmax = 0;
        if ((st = step(0))) return st;
        for (int j = 0; j < m; ++j) {
            if (j + 1 < m && (st = step(j + 1))) return st;   // queued ahead of the host's work on column j
            if ((e = hipEventSynchronize(pin.ev[j & 1])) != hipSuccess) return hip_err(e, "gmres");
            const double* col = pin.p + (size_t)(j & 1) * hh.size();
            bool any = false;
            for (int f = 0; f < nfc; ++f) {
                if (!act[f]) continue;
                double* Hf = &H[(size_t)f * (m + 1) * m];
                double* csf = &cs[(size_t)f * m];
                double* snf = &sn[(size_t)f * m];
                double* gf = &g[(size_t)f * (m + 1)];
                const double* hf = &col[(size_t)f * HS];
                const double hn = sqrt(hf[on]);
                for (int i = 0; i <= j; ++i) Hf[(size_t)i * m + j] = hf[i] + hf[o2 + i];
                Hf[(size_t)(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {   // previous rotations
                    const double a = Hf[(size_t)i * m + j], c = Hf[(size_t)(i + 1) * m + j];
                    Hf[(size_t)i * m + j] = csf[i] * a + snf[i] * c;
                    Hf[(size_t)(i + 1) * m + j] = -snf[i] * a + csf[i] * c;
                }
                const double a = Hf[(size_t)j * m + j], c = Hf[(size_t)(j + 1) * m + j];
                const double r = hypot(a, c);
                csf[j] = r > 0 ? a / r : 1.0;
                snf[j] = r > 0 ? c / r : 0.0;
                Hf[(size_t)j * m + j] = r;
                Hf[(size_t)(j + 1) * m + j] = 0.0;
                gf[j + 1] = -snf[j] * gf[j];
                gf[j] = csf[j] * gf[j];
                k[f] = j + 1;
                ++*iters;
                if (fabs(gf[j + 1]) <= kGmresTol * bnorm[f] || hn == 0.0) {
                    act[f] = 0;   // converged (or an exact breakdown): this cycle ends for f
                    conv[f] = 1;
                } else {
                    any = true;
                }
            }
            kmax = j + 1;
            if (!any) break;
        }
        // y_f = H_f(0:k, 0:k)^-1 g_f, x_f += V_f y_f (as x_f -= sum (-y_f,i) V_f,i; zeros past k_f)
        std::fill(hh.begin(), hh.end(), 0.0);
        for (int f = 0; f < nfc; ++f) {
            const double* Hf = &H[(size_t)f * (m + 1) * m];
            const double* gf = &g[(size_t)f * (m + 1)];
            double* yf = &hh[(size_t)f * HS + oy];
            for (int i = k[f] - 1; i >= 0; --i) {
                double t = gf[i];
                for (int l = i + 1; l < k[f]; ++l) t -= Hf[(size_t)i * m + l] * yf[l];
                yf[i] = t / Hf[(size_t)i * m + i];
            }
            for (int i = 0; i < k[f]; ++i) yf[i] = -yf[i];
        }
        if ((e = hipMemcpyAsync(hd, hh.data(), hh.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_err(e, "gmres");
        if ((st = pois_sub(V, VS, kmax, hd + oy, HS, n, nfc, x, n, s))) return st;
        all = true;
        for (int f = 0; f < nfc; ++f) {
            done[f] = done[f] || conv[f];
            all = all && done[f];
        }
        if (all) return FC2D_OK;
        // restart the open fields from their true residuals r_f = b_f - A x_f
        if ((st = pois_matvec(A, x, n, n, nfc, part, w, s)) ||
            (st = pois_axpbz(1.0, b, -1.0, w, nfc * n, w, s)) ||
            (st = pois_dots(w, n, 1, w, n, n, nfc, hd + on, HS, s)) || (st = fetch()))
            return st;
        all = true;
        for (int f = 0; f < nfc; ++f) {
            if (!done[f]) {
                beta[f] = sqrt(hh[f * HS + on]);
                done[f] = beta[f] <= kGmresTol * bnorm[f];
            }
            scal[f] = done[f] ? 0.0 : 1.0 / beta[f];
            all = all && done[f];
        }
        if (all) return FC2D_OK;
        if ((st = pois_scale(scal.data(), w, n, n, nfc, V, VS, s))) return st;
    }
    set_error("GMRES did not converge");
    return FC2D_E_NEWTON;
}

bool pow2(int n) { return n >= 8 && (n & (n - 1)) == 0; }

}  // namespace

extern "C" {

int fc2d_poisson_nodes(const fc2d_plan* pl, int nb, double* xy) {
    if (!pl || nb < 8 || !xy) { set_error("invalid Poisson node arguments"); return FC2D_E_ARG; }
    std::vector<double> qd;
    node_data(pl->curve, nb, qd);
    for (int j = 0; j < nb; ++j) {
        xy[2 * j] = qd[6 * (size_t)j];
        xy[2 * j + 1] = qd[6 * (size_t)j + 1];
    }
    return FC2D_OK;
}

int fc2d_poisson_solve(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, const double* g_nodes,
                       int nb, double* u, int nf, hipStream_t s, int* gmres_iters) {
    if (!pl || !f_grid || (!f_bdry && !pl->interior_only) || !g_nodes || !u || nb < 8 || nb > 16384 || nf < 1) {
        set_error("invalid Poisson solve arguments");
        return FC2D_E_ARG;
    }
    const fc2d_grid& g = pl->grid;
    if (!pow2(g.nx) || !pow2(g.ny)) {
        set_error("Poisson solve: power-of-two grids only");
        return FC2D_E_ARG;
    }
    const int M = pl->M;
    const int64_t npts = (int64_t)g.nx * g.ny;
    const int64_t nbdry = pl->B + (int64_t)pl->squares.size() / 2;
    const int nbf = nb * kRefine;
    const int m = std::min(nb, kRestart);
    // largest node spacing of the nb nodes (host); node data, classes and the
    // rest on the device
    std::vector<double> qc;
    node_data(pl->curve, nb, qc);
    double dsmax = 0.0;
    for (int j = 0; j < nb; ++j) dsmax = std::max(dsmax, hypot(qc[6 * (size_t)j + 2], qc[6 * (size_t)j + 3]));
    dsmax *= 2.0 * M_PI / nb;
    // grid points within h of Gamma (the only ones that can be near points): at most the tube
    // area 2 (h + h / sqrt 2) P + pi (h + h / sqrt 2)^2 over h^2, P the perimeter
    double perim = 0.0;
    for (int j = 0; j < nb; ++j) perim += hypot(qc[6 * (size_t)j + 2], qc[6 * (size_t)j + 3]);
    perim *= 2.0 * M_PI / nb;
    // largest curvature at the nodes (twice, for safety) -> how far an arc of length <= dsmax
    // leaves its chord: kappa dsmax^2 / 8
    double kmax = 0.0;
    for (int j = 0; j < nb; ++j) {
        const double* q = &qc[6 * (size_t)j];
        const double sp = hypot(q[2], q[3]);
        kmax = std::max(kmax, fabs(q[2] * q[5] - q[3] * q[4]) / (sp * sp * sp));
    }
    const double sag = 2.0 * kmax * dsmax * dsmax / 8.0;
    const int capn = (int)std::min<double>((double)std::max<int64_t>(pl->n_in, 1), ceil(4.0 * perim / g.h) + 64.0);
    const int64_t nall = (int64_t)nb * (2 * kRefine - 1);   // nodes of all levels
    const int64_t cap = std::max<int64_t>(pl->n_in, 1);
    // band entries of a level whose nodes are split over blocks (2^15 nodes or more): such a
    // point lies closer to Gamma than D = 7 dsmax / 2^(L - 1) + 2 sag (its distance bound plus
    // the polygon's deviation both ways), so its h-square lies in the tube of radius
    // D + h / sqrt 2 about Gamma, whose area is at most 2 r P + pi r^2
    int lc = 1;
    while (lc < kPoisLevels - 1 && ((int64_t)nb << lc) < (1 << 15)) ++lc;
    const double rb = (7.0 * dsmax / (double)(1 << (lc - 1))) * (1.0 + 1e-5) + 2.0 * sag + g.h * M_SQRT1_2;
    const int capb = (int)std::min<double>((double)cap, ceil((2.0 * rb * perim * 1.01 + M_PI * rb * rb) / (g.h * g.h)) + 64.0);
    const int64_t scap = (int64_t)capn * (M - 1);
    const int nfm = std::min(nf, kPoisChunk);   // fields per chunk at most
    double *spec, *work, *up, *mean, *d_qc, *d_geo, *rec, *ghom, *rhs, *A, *phi, *phif, *wtab, *part, *V, *w, *hd;
    double *bx, *by, *bnx, *bny;
    int8_t* cls;
    int32_t *cand, *bl;
    int* cnt;
    PoisArena db;
    db.add(&spec, (size_t)g.nx * (g.ny / 2 + 1) * 2);
    db.add(&work, (size_t)npts);
    db.add(&up, (size_t)npts * nfm);
    db.add(&mean, 1);
    db.add(&d_qc, 6 * (size_t)nb);
    db.add(&d_geo, 4 * (size_t)nall);
    db.add(&rec, (2 + 2 * (size_t)nfm) * nall);
    double *seg, *sinv;
    db.add(&seg, 4 * (size_t)nb);
    db.add(&sinv, nb);
    db.add(&ghom, (size_t)nb * nfm);
    db.add(&rhs, (size_t)nb * nfm);
    db.add(&A, (size_t)nb * nb);
    db.add(&phi, (size_t)nb * nfm);
    db.add(&phif, (size_t)nbf * nfm);
    db.add(&wtab, (size_t)nbf);   // (kRefine - 1) nb weights
    db.add(&part, (size_t)pois_matvec_splits(nb) * nb * nfm);
    db.add(&V, (size_t)(m + 1) * nb * nfm);
    db.add(&w, (size_t)nb * nfm);
    db.add(&hd, (3 * (size_t)(m + 2) + m) * nfm);
    db.add(&cls, (size_t)npts);
    db.add(&cand, (size_t)cap);
    db.add(&cnt, kPoisCounters);
    int32_t *nidx, *sl;
    int8_t* slev;
    double *nw, *nv0, *samp, *sval, *bpart;
    db.add(&nidx, capn);
    db.add(&nw, (size_t)capn * M);
    db.add(&nv0, (size_t)capn * nfm);
    db.add(&samp, (size_t)scap * 2);
    db.add(&sval, (size_t)16 * scap * nfm);
    db.add(&sl, (size_t)scap * kPoisLevels);
    db.add(&slev, (size_t)scap);
    db.add(&bl, (size_t)cap * kPoisLevels);
    db.add(&bpart, (size_t)16 * capb * nfm);
    db.add(&bx, pl->B);
    db.add(&by, pl->B);
    db.add(&bnx, pl->B);
    db.add(&bny, pl->B);
    if (int st0 = db.commit(s)) return st0;
    hipError_t e;
    if ((e = hipMemcpyAsync(bx, pl->bx.data(), pl->B * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(by, pl->by.data(), pl->B * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(bnx, pl->bnx.data(), pl->B * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(bny, pl->bny.data(), pl->B * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_err(e, "Poisson solve upload");
    trace_point("pois_setup", s);
    int st;
    if ((st = pois_nodes(pl->curve, nb, d_qc, d_geo, seg, sinv, s))) return st;
    if ((st = pois_classes(pl->d_run_ptr, pl->d_run, g.nx, g.ny, cls, s))) return st;
    const BndView bd{bx, by, bnx, bny, pl->B, pl->k2};
    if ((st = pois_nystrom(d_qc, nb, A, s))) return st;
    int iters_total = 0;
    // chunks of 4, 2 or 1 fields: the particular solution, boundary data and
    // density of each field, then the double-layer sums of the chunk together
    for (int f0 = 0; f0 < nf;) {
        const int nfc = nf - f0 >= 4 ? 4 : (nf - f0 >= 2 ? 2 : 1);
        for (int c = 0; c < nfc; ++c) {
            const int f = f0 + c;
            double* upc = up + (int64_t)c * npts;
            double* ghc = ghom + (int64_t)c * nb;
            // particular solution: extension + R2C, -1/|k|^2, C2R, mean term
            if ((st = fc2d_extend_fft(pl, f_grid + (int64_t)f * npts, f_bdry ? f_bdry + (int64_t)f * nbdry : f_bdry,
                                      work, spec, 1, s)))
                return st;
            if ((st = pois_mean(&g, spec, mean, s))) return st;
            if ((st = spectral_apply(&g, FC2D_LAPLACE_INV, spec, spec, 1, s))) return st;
            if ((st = fft2_c2r(&g, spec, upc, 1, s))) return st;
            if ((st = pois_add_quad(&g, mean, upc, s))) return st;
            // boundary data of the harmonic part and its density
            if ((st = pois_ghom(M, &g, upc, d_qc, nb, g_nodes + (int64_t)f * nb, ghc, s))) return st;
            if ((st = pois_axpbz(-2.0, ghc, 0.0, ghc, nb, rhs + (int64_t)c * nb, s))) return st;
        }
        int it = 0;
        if ((st = gmres(A, rhs, phi, nb, nfc, V, w, hd, part, s, &it))) return st;
        iters_total += it;
        if ((st = pois_records(phi, nb, nfc, d_geo, wtab, phif, rec, s))) return st;
        // v on the grid, then the points next to Gamma
        double* uc = u + (int64_t)f0 * npts;
        if ((e = hipMemsetAsync(cnt, 0, kPoisCounters * sizeof(int), s)) != hipSuccess)
            return hip_err(e, "Poisson solve");
        const PoisDl dl{&g,    nfc,   M,   nb,  60,   cls,  up,   rec,  ghom, dsmax, seg, sinv, sag,
                        pl->curve, bd, cap, bl, cand, capb, bpart, capn, nidx, nw, nv0, samp, sl, slev,
                        sval, cnt,  uc};
        if ((st = pois_dl_eval(dl, s))) return st;
        int hc[kPoisCounters] = {};
        if ((e = hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_err(e, "Poisson solve");
        if (hc[1] > 0) {
            set_error("Poisson solve: foot of the normal failed next to the boundary");
            return FC2D_E_NEWTON;
        }
        if (hc[3 + kPoisLevels] > 0) {
            set_error("Poisson solve: more points next to the boundary than the bound allows");
            return FC2D_E_HIP;
        }
        f0 += nfc;
    }
    if (gmres_iters) *gmres_iters = iters_total;
    return FC2D_OK;
}

}  // extern "C"
