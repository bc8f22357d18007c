// Batches: many fields on several domains and grid sizes advanced together by
// Fourier Forwarding (Sec. 4.2), one step being
//   boundary values <- tensor interpolation of the full-box fields (u, u_t)
//   Gram records     <- matching values + blend            (Sec. 3.2)
//   STRIP values     <- interpolation onto H n V+         (Sec. 3.4)
//   spectra          <- extension fused into the forward 2D FFT (Sec. 3.5)
//   spectra          <- modal propagation by dt            (eq. wave_2d_ff)
//   (u, u_t)         <- inverse 2D FFT on the whole box
// The plan-specific stages run as single persistent launches over every
// (plan, field set) of the batch; the FFT passes run once per grid size with
// the fields of all domains of that size contiguous.  A step can be captured
// in a HIP graph and replayed.  An optional autotuner times, on the batch's
// own buffers, the column-pass tile widths, the separate against the fused
// spectral step and the fused kernel's shapes, row-major against transposed
// spectra, and the strip kernel's fields per thread, and keeps the fastest.
#include <string.h>

#include <algorithm>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace fc2d;

namespace fc2d {
struct Group {
    fc2d_grid grid;
    int nf_total = 0;
    std::vector<int> members;     // plan indices
    double* state = nullptr;      // [2][nf_total][nx][ny]: u then u_t
    double* spec = nullptr;       // [2][nf_total][nx][ny/2+1] complex128
    bool fused_ff = false;        // column passes and propagation in one launch (k_cols_ff)
    bool trans = false;           // spectra stored transposed, rows in groups of 8 (implies fused_ff)
};
}  // namespace fc2d

struct fc2d_batch {
    std::vector<const fc2d_plan*> plans;
    std::vector<int> nf, group_of, field_off;
    std::vector<Group> groups;
    std::vector<double*> bufs;    // boundary values and Gram records (freed at destroy)
    std::vector<PlanDev> pd;
    PlanDev* d_pd = nullptr;
    int64_t tot_match = 0, tot_strip = 0, tot_bv = 0;
    int M = 0, D = 0, Cr = 0, strip_fpt = 4, grid_blocks = 2048;
    int strip_wmax = 1;   // widest strip-kernel block window over the plans (normals)
    bool trans_fixed = false;   // layout of the spectra fixed by the caller (FC2D_BATCH_TRANSPOSED)
    const double* d_Ar = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;        // capture / replay stream (the caller's may be the null stream)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    double graph_c = 0.0, graph_dt = 0.0;
    int launches_per_step = 0;
};

static void batch_free(fc2d_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (Group& g : b->groups) {
        if (g.state) (void)hipFree(g.state);
        if (g.spec) (void)hipFree(g.spec);
    }
    for (double* p : b->bufs)
        if (p) (void)hipFree(p);
    if (b->d_pd) (void)hipFree(b->d_pd);
    delete b;
}

// column transforms and propagation of one grid-size group (rows already transformed)
static int spectral_step(Group& g, double c, double dt, hipStream_t s) {
    const int64_t nsp = (int64_t)g.grid.nx * (g.grid.ny / 2 + 1) * 2;
    double* su = g.spec;
    double* sut = g.spec + (int64_t)g.nf_total * nsp;
    if (g.trans || g.fused_ff) return cols_ff(&g.grid, c, dt, su, sut, g.nf_total, s, g.trans);
    int st;
    if ((st = fft_cols(&g.grid, g.spec, 2 * g.nf_total, false, s))) return st;
    if ((st = ff_apply(&g.grid, c, dt, su, sut, su, sut, g.nf_total, s))) return st;
    return fft_cols(&g.grid, g.spec, 2 * g.nf_total, true, s);
}

// the spectral part of a step for one grid-size group: forward row passes
// with the extension (per member plan), column passes + propagation, inverse
// row passes; *launches counts the kernels
static int group_fft_step(fc2d_batch* b, Group& g, double c, double dt, hipStream_t s, int* launches) {
    int st;
    const int64_t npts = (int64_t)g.grid.nx * g.grid.ny;
    const int64_t nsp = (int64_t)g.grid.nx * (g.grid.ny / 2 + 1) * 2;   // doubles per spectrum
    int n = 0;
    for (int k : g.members) {
        const fc2d_plan* pl = b->plans[k];
        for (int half = 0; half < 2; ++half) {
            const int64_t f0 = (int64_t)half * g.nf_total + b->field_off[k];
            double* u = g.state + f0 * npts;
            st = g.trans ? fft_rows_fwd_t(&g.grid, u, g.spec + f0 * nsp, b->nf[k], s, u, pl->d_cls2)
                         : fft_rows_fwd(&g.grid, u, g.spec + f0 * nsp, b->nf[k], s, u, pl->d_cls2);
            if (st) return st;
            ++n;
        }
    }
    if ((st = spectral_step(g, c, dt, s))) return st;
    st = g.trans ? fft_rows_inv_t(&g.grid, g.spec, g.state, 2 * g.nf_total, s)
                 : fft_rows_inv(&g.grid, g.spec, g.state, 2 * g.nf_total, s);
    if (st) return st;
    n += (g.trans || g.fused_ff) ? 2 : 4;
    *launches = n;
    return FC2D_OK;
}

// enqueue one Fourier-Forwarding step of the whole batch on s
static int batch_step(fc2d_batch* b, double c, double dt, hipStream_t s) {
    int st;
    const int np = (int)b->pd.size();
    int n = 0;
    if ((st = launch_multi(2, b->M, b->d_pd, np, b->tot_bv, 0, b->d_Ar, b->D, b->Cr, 1, b->grid_blocks, s))) return st;
    if ((st = launch_multi(0, b->M, b->d_pd, np, b->tot_match, 0, b->d_Ar, b->D, b->Cr, 1, b->grid_blocks, s))) return st;
    if ((st = launch_multi(1, b->M, b->d_pd, np, b->tot_strip, b->strip_fpt, b->d_Ar, b->D, b->Cr, b->strip_wmax, b->grid_blocks,
                           s)))
        return st;
    n += 3;
    for (Group& g : b->groups) {
        int ng = 0;
        if ((st = group_fft_step(b, g, c, dt, s, &ng))) return st;
        n += ng;
    }
    b->launches_per_step = n;
    return FC2D_OK;
}

// the fastest of reps timed calls after one warm-up call (the minimum is the
// least disturbed by other work on the device)
static float time_ms(hipStream_t s, const std::function<int()>& fn, int reps) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0f;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1.0f; }
    (void)fn();   // warm-up
    float best = -1.0f;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, s);
        (void)fn();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = -1.0f;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms >= 0.0f && (best < 0.0f || ms < best)) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

// Trial steps propagate by a generic nonzero time so that the propagation's
// transcendental work is timed as in a real step (the batch's state is reset
// to zero after tuning).
constexpr double kTuneC = 1.0, kTuneT = 0.0123;

static int autotune(fc2d_batch* b, hipStream_t s) {
    // column-pass shape (elements per thread, columns per block) per grid size
    for (Group& g : b->groups) {
        int best_E = col_elems_get(g.grid.nx), best_T = col_tile_get(g.grid.nx);
        float best = 1e30f;
        const int ecand[] = {2, 4, 8, 16};
        const int tcand[] = {1, 2, 4, 8, 16};
        for (int E : ecand)
            for (int T : tcand) {
                if (col_cfg_set(g.grid.nx, E, T) != FC2D_OK) continue;
                const float ms =
                    time_ms(s, [&]() { return fft_cols(&g.grid, g.spec, 2 * g.nf_total, false, s); }, 3);
                if (ms >= 0 && ms < best) { best = ms; best_E = E; best_T = T; }
            }
        col_cfg_set(g.grid.nx, best_E, best_T);
        // separate column passes + propagation, or the fused kernel, on spectra
        // of the (filled) state: one untimed group step first
        float t_sep = -1.0f, t_fused = -1.0f;
        {
            int nl0 = 0;
            (void)group_fft_step(b, g, kTuneC, kTuneT, s, &nl0);
        }
        g.fused_ff = false;
        t_sep = time_ms(s, [&]() { return spectral_step(g, kTuneC, kTuneT, s); }, 3);
        g.fused_ff = true;
        int best_v = colff_get(g.grid.nx);
        for (int v = 0; v < colff_variants(g.grid.nx); ++v) {
            colff_set(g.grid.nx, v);
            const float ms = time_ms(s, [&]() { return spectral_step(g, kTuneC, kTuneT, s); }, 3);
            if (ms >= 0 && (t_fused < 0 || ms < t_fused)) { t_fused = ms; best_v = v; }
        }
        colff_set(g.grid.nx, best_v);
        g.fused_ff = t_fused >= 0 && (t_sep < 0 || t_fused < t_sep);
        // row-major spectra (as chosen above) against transposed spectra, unless
        // the layout was fixed: the fused kernel's shape on transposed spectra
        // by its own launch (the row passes around it would only add noise),
        // then the two layouts, each with its best shape, over the group's whole
        // step (the row passes differ between them)
        if (!b->trans_fixed && g.grid.ny <= 4096 && g.grid.nx % 8 == 0) {
            int nl = 0;
            g.trans = true;
            (void)group_fft_step(b, g, kTuneC, kTuneT, s, &nl);   // transposed spectra of the state
            float t_sp = -1.0f;
            int best_tv = colff_get(g.grid.nx);
            for (int v = 0; v < colff_variants(g.grid.nx); ++v) {
                colff_set(g.grid.nx, v);
                const float ms = time_ms(s, [&]() { return spectral_step(g, kTuneC, kTuneT, s); }, 3);
                if (ms >= 0 && (t_sp < 0 || ms < t_sp)) { t_sp = ms; best_tv = v; }
            }
            g.trans = false;
            colff_set(g.grid.nx, best_v);
            const float t_rm = time_ms(s, [&]() { return group_fft_step(b, g, kTuneC, kTuneT, s, &nl); }, 3);
            g.trans = true;
            colff_set(g.grid.nx, best_tv);
            const float t_tr = time_ms(s, [&]() { return group_fft_step(b, g, kTuneC, kTuneT, s, &nl); }, 3);
            g.trans = t_tr >= 0 && (t_rm < 0 || t_tr < t_rm);
            colff_set(g.grid.nx, g.trans ? best_tv : best_v);
        } else if (g.trans) {
            int best_tv = colff_get(g.grid.nx), nl = 0;
            float t_tr = -1.0f;
            for (int v = 0; v < colff_variants(g.grid.nx); ++v) {
                colff_set(g.grid.nx, v);
                const float ms = time_ms(s, [&]() { return spectral_step(g, kTuneC, kTuneT, s); }, 3);
                if (ms >= 0 && (t_tr < 0 || ms < t_tr)) { t_tr = ms; best_tv = v; }
            }
            (void)nl;
            colff_set(g.grid.nx, best_tv);
        }
    }
    // strip kernel: fields per thread
    int best_f = b->strip_fpt;
    float best = 1e30f;
    const int fcand[] = {1, 2, 4, 8, 16};
    for (int fpt : fcand) {
        int64_t tot = 0;
        for (PlanDev& P : b->pd) {
            P.off_strip = tot;
            tot += ((P.S + 511) / 512) * ((P.nf + fpt - 1) / fpt);
        }
        if (hipMemcpy(b->d_pd, b->pd.data(), b->pd.size() * sizeof(PlanDev), hipMemcpyHostToDevice) != hipSuccess)
            return FC2D_E_HIP;
        const float ms = time_ms(s, [&]() {
            return launch_multi(1, b->M, b->d_pd, (int)b->pd.size(), tot, fpt, b->d_Ar, b->D, b->Cr, b->strip_wmax,
                                b->grid_blocks, s);
        }, 3);
        if (ms >= 0 && ms < best) { best = ms; best_f = fpt; }
    }
    b->strip_fpt = best_f;
    int64_t tot = 0;
    for (PlanDev& P : b->pd) {
        P.off_strip = tot;
        tot += ((P.S + 511) / 512) * ((P.nf + best_f - 1) / best_f);
    }
    b->tot_strip = tot;
    if (hipMemcpy(b->d_pd, b->pd.data(), b->pd.size() * sizeof(PlanDev), hipMemcpyHostToDevice) != hipSuccess)
        return FC2D_E_HIP;
    return FC2D_OK;
}

extern "C" {

int fc2d_batch_create(const fc2d_plan* const* plans, const int* nf, int nplans, unsigned flags, hipStream_t s,
                      fc2d_batch** out) {
    if (!plans || !nf || nplans <= 0 || !out) { set_error("invalid batch arguments"); return FC2D_E_ARG; }
    *out = nullptr;
    fc2d_batch* b = new (std::nothrow) fc2d_batch();
    if (!b) { set_error("out of host memory"); return FC2D_E_NOMEM; }
    b->M = plans[0]->M;
    b->D = plans[0]->d;
    b->Cr = plans[0]->Cr;
    b->d_Ar = plans[0]->d_Ar;
    for (int k = 0; k < nplans; ++k) {
        const fc2d_plan* pl = plans[k];
        if (!pl || nf[k] <= 0 || pl->M != b->M || pl->d != b->D || pl->Cr != b->Cr || pl->Ar != plans[0]->Ar ||
            !pl->d_cls2) {
            set_error("batch plans must share d, C, n_r, M and tables, have power-of-two grids and nf > 0");
            batch_free(b);
            return FC2D_E_ARG;
        }
        b->plans.push_back(pl);
        b->nf.push_back(nf[k]);
        int gi = -1;
        for (size_t g = 0; g < b->groups.size(); ++g)
            if (b->groups[g].grid.nx == pl->grid.nx && b->groups[g].grid.ny == pl->grid.ny &&
                b->groups[g].grid.h == pl->grid.h)
                gi = (int)g;   // same transform sizes and wavenumbers
        if (gi < 0) {
            Group g;
            g.grid = pl->grid;
            b->groups.push_back(g);
            gi = (int)b->groups.size() - 1;
        }
        b->group_of.push_back(gi);
        b->field_off.push_back(b->groups[gi].nf_total);
        b->groups[gi].nf_total += nf[k];
        b->groups[gi].members.push_back(k);
    }
    int st = FC2D_OK;
    for (Group& g : b->groups) {
        const size_t npts = (size_t)g.grid.nx * g.grid.ny;
        const size_t nsp = (size_t)g.grid.nx * (g.grid.ny / 2 + 1) * 2;
        if (hipMalloc((void**)&g.state, 2 * g.nf_total * npts * sizeof(double)) != hipSuccess ||
            hipMalloc((void**)&g.spec, 2 * g.nf_total * nsp * sizeof(double)) != hipSuccess) {
            set_error("hipMalloc failed (batch state)");
            batch_free(b);
            return FC2D_E_NOMEM;
        }
        if (hipMemset(g.state, 0, 2 * g.nf_total * npts * sizeof(double)) != hipSuccess ||
            hipMemset(g.spec, 0, 2 * g.nf_total * nsp * sizeof(double)) != hipSuccess ||
            fft_prepare(g.grid.nx, g.grid.ny) != FC2D_OK) {
            set_error("batch initialisation failed");
            batch_free(b);
            return FC2D_E_HIP;
        }
    }
    // descriptors: entry 2k = u of plan k, 2k+1 = u_t of plan k
    int64_t om = 0, ob = 0;
    for (int k = 0; k < nplans; ++k) {
        const fc2d_plan* pl = b->plans[k];
        const Group& g = b->groups[b->group_of[k]];
        const int64_t npts = (int64_t)g.grid.nx * g.grid.ny;
        const int64_t nb = pl->B + (int64_t)pl->squares.size() / 2;
        const int DP = (pl->d + 2) & ~1;
        for (int half = 0; half < 2; ++half) {
            PlanDev P;
            memset(&P, 0, sizeof P);
            P.mref = pl->d_mref; P.mlab = pl->d_mlab; P.mwv = pl->d_mwv; P.mwn = pl->d_mwn; P.Q = pl->d_Q;
            P.sidx = pl->d_sidx; P.sth = pl->d_sth; P.seta = pl->d_seta; P.bxy = pl->d_bxy;
            P.B = pl->B; P.D = pl->d; P.nf = b->nf[k]; P.nx = g.grid.nx; P.ny = g.grid.ny;
            P.io = pl->interior_only ? 1 : 0;
            P.npts = npts; P.nbdry = nb; P.S = pl->n_strip;
            P.k2 = pl->k2; P.lev_scale = pl->n_r / pl->k1; P.x0 = g.grid.x0; P.y0 = g.grid.y0; P.h = g.grid.h;
            P.u = g.state + ((int64_t)half * g.nf_total + b->field_off[k]) * npts;
            double *fb = nullptr, *cb = nullptr;
            if (hipMalloc((void**)&fb, (size_t)P.nf * nb * sizeof(double)) != hipSuccess ||
                hipMalloc((void**)&cb, (size_t)P.nf * pl->B * DP * sizeof(double)) != hipSuccess) {
                if (fb) (void)hipFree(fb);
                set_error("hipMalloc failed (batch work)");
                batch_free(b);
                return FC2D_E_NOMEM;
            }
            b->bufs.push_back(fb);
            b->bufs.push_back(cb);
            P.fb = fb;
            P.c = cb;
            P.off_match = om;
            om += (int64_t)((((P.B + 3) / 4) + 7) & ~7) * ((P.nf + 3) / 4);   // k_match_multi: 4 normals x 4 fields
            P.off_bv = ob;
            ob += (int64_t)P.nf * nb;
            b->pd.push_back(P);
        }
    }
    b->tot_match = om;
    b->tot_bv = ob;
    for (int k = 0; k < nplans; ++k) b->strip_wmax = std::max(b->strip_wmax, plans[k]->strip_wmax);
    int64_t ot = 0;
    for (PlanDev& P : b->pd) {
        P.off_strip = ot;
        ot += ((P.S + 511) / 512) * ((P.nf + b->strip_fpt - 1) / b->strip_fpt);
    }
    b->tot_strip = ot;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b->grid_blocks = std::max(8, (cus * 8 / 8) * 8);
    if (hipMalloc((void**)&b->d_pd, b->pd.size() * sizeof(PlanDev)) != hipSuccess ||
        hipMemcpy(b->d_pd, b->pd.data(), b->pd.size() * sizeof(PlanDev), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("batch descriptor upload failed");
        batch_free(b);
        return FC2D_E_HIP;
    }
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        set_error("batch stream/event creation failed");
        batch_free(b);
        return FC2D_E_HIP;
    }
    if (flags & FC2D_BATCH_FUSED_FF)
        for (Group& g : b->groups) g.fused_ff = true;
    if (flags & FC2D_BATCH_TRANSPOSED) {
        b->trans_fixed = true;
        for (Group& g : b->groups) g.trans = g.grid.ny <= 4096 && g.grid.nx % 8 == 0;
    }
    if (flags & FC2D_BATCH_AUTOTUNE) {
        // trial steps on a nonzero state (every byte 0x3f: each value about
        // 4.8e-4): the FP64 kernels run measurably faster on zeros than on data
        for (Group& g : b->groups) {
            const int64_t npts = (int64_t)g.grid.nx * g.grid.ny;
            if (hipMemsetAsync(g.state, 0x3f, 2 * g.nf_total * npts * sizeof(double), s) != hipSuccess) {
                set_error("batch state fill failed");
                batch_free(b);
                return FC2D_E_HIP;
            }
        }
        st = autotune(b, s);
    }
    if (st) { batch_free(b); return st; }
    // the timed trial steps ran on the batch's own buffers: back to zero
    for (Group& g : b->groups) {
        const int64_t npts = (int64_t)g.grid.nx * g.grid.ny;
        const int64_t nsp = (int64_t)g.grid.nx * (g.grid.ny / 2 + 1) * 2;
        if (hipMemsetAsync(g.state, 0, 2 * g.nf_total * npts * sizeof(double), s) != hipSuccess ||
            hipMemsetAsync(g.spec, 0, 2 * g.nf_total * nsp * sizeof(double), s) != hipSuccess) {
            set_error("batch state reset failed");
            batch_free(b);
            return FC2D_E_HIP;
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess) { set_error("batch set-up failed"); batch_free(b); return FC2D_E_HIP; }
    *out = b;
    return FC2D_OK;
}

int fc2d_batch_state(fc2d_batch* b, int k, double** u, double** ut) {
    if (!b || k < 0 || k >= (int)b->plans.size()) { set_error("invalid batch or plan index"); return FC2D_E_ARG; }
    const Group& g = b->groups[b->group_of[k]];
    const int64_t npts = (int64_t)g.grid.nx * g.grid.ny;
    if (u) *u = g.state + (int64_t)b->field_off[k] * npts;
    if (ut) *ut = g.state + ((int64_t)g.nf_total + b->field_off[k]) * npts;
    return FC2D_OK;
}

int fc2d_batch_info(const fc2d_batch* b, int64_t* points_per_step, int* launches_per_step, int* strip_fields) {
    if (!b) { set_error("NULL batch"); return FC2D_E_ARG; }
    int64_t pts = 0;
    for (const Group& g : b->groups) pts += 2 * (int64_t)g.nf_total * g.grid.nx * g.grid.ny;
    if (points_per_step) *points_per_step = pts;
    if (launches_per_step) *launches_per_step = b->launches_per_step;
    if (strip_fields) *strip_fields = b->strip_fpt;
    return FC2D_OK;
}

int fc2d_batch_run_ff(fc2d_batch* b, double c, double dt, int steps, int use_graph, hipStream_t s) {
    if (!b || steps < 0) { set_error("invalid batch arguments"); return FC2D_E_ARG; }
    int st;
    if (!use_graph) {
        for (int i = 0; i < steps; ++i)
            if ((st = batch_step(b, c, dt, s))) return st;
        return FC2D_OK;
    }
    // capture and replay on the batch's own stream, ordered after and before `s`
    hipStream_t cs = b->cap;
    hipError_t e = hipEventRecord(b->ev_in, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, b->ev_in, 0);
    if (e != hipSuccess) { set_error(std::string("batch stream ordering: ") + hipGetErrorString(e)); return FC2D_E_HIP; }
    if (!b->exec || b->graph_c != c || b->graph_dt != dt) {
        if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) { set_error(std::string("hipStreamBeginCapture: ") + hipGetErrorString(e)); return FC2D_E_HIP; }
        st = batch_step(b, c, dt, cs);
        e = hipStreamEndCapture(cs, &b->graph);
        if (st) return st;
        if (e != hipSuccess) { set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e)); return FC2D_E_HIP; }
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e)); return FC2D_E_HIP; }
        b->graph_c = c;
        b->graph_dt = dt;
    }
    for (int i = 0; i < steps; ++i) {
        e = hipGraphLaunch(b->exec, cs);
        if (e != hipSuccess) { set_error(std::string("hipGraphLaunch: ") + hipGetErrorString(e)); return FC2D_E_HIP; }
    }
    e = hipEventRecord(b->ev_out, cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->ev_out, 0);
    if (e != hipSuccess) { set_error(std::string("batch stream ordering: ") + hipGetErrorString(e)); return FC2D_E_HIP; }
    return FC2D_OK;
}

int fc2d_batch_destroy(fc2d_batch* b) {
    batch_free(b);
    return FC2D_OK;
}

}  // extern "C"
