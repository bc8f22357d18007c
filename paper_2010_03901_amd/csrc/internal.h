// Internal declarations shared by the host plan code (g++) and the HIP
// kernel translation units (hipcc).  Not part of the public ABI.
#pragma once

#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/fc2d.h"
#include "geom.h"
#include "matching.h"

namespace fc2d {

// FC-Gram tables (fcgram_quad.cpp): Q [d][d], A [C][d], Ar [n_r C][d], row-major.
int gram_tables(int d, int C, int Z, int n_os, int n_r, int mf, double* Q, double* A, double* Ar);

void set_error(const std::string& msg);

// Kernel tracer: when a trace is open (fc2d_trace_begin), records a HIP event
// on `s` after each launch so fc2d_trace_end can report per-kernel times.
void trace_point(const char* name, hipStream_t s);

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Per-call device work space, stream-ordered (workspace.cpp): taken from a
// library-owned pool on stream s and returned on s, so calls on different
// streams never share it.
int ws_alloc(size_t bytes, hipStream_t s, void** p);
int ws_free(void* p, hipStream_t s);
// Holder that returns its memory on the stream when the call ends; work
// already queued on that stream still sees it (the release is stream-ordered).
struct WorkSpace {
    void* p = nullptr;
    hipStream_t s = nullptr;
    int alloc(size_t bytes, hipStream_t st) {
        s = st;
        return ws_alloc(bytes, st, &p);
    }
    WorkSpace() = default;
    WorkSpace(const WorkSpace&) = delete;
    WorkSpace& operator=(const WorkSpace&) = delete;
    ~WorkSpace() {
        if (p) (void)ws_free(p, s);
    }
};

}  // namespace fc2d

// The plan: host copies needed by the host-side queries plus device arrays
// used by the extension kernels.
struct fc2d_plan {
    fc2d_grid grid;
    int d, C, M, n_r, Cr, B;
    double k1, k2;
    fc2d::CurveC curve;
    // host
    std::vector<double> Q, A, Ar;                // tables
    std::vector<double> bx, by, bnx, bny;        // boundary samples and normals
    std::vector<double> squares;                 // 2 per square (x, y)
    // host copies of the classes and the row-major STRIP list, downloaded from
    // the device copies on first use (plan_host_lists)
    mutable std::mutex host_mu;
    mutable bool host_ready = false;
    mutable std::vector<int8_t> cls;                     // nx * ny
    mutable std::vector<int32_t> strip_idx, strip_seed;  // row-major STRIP list
    mutable std::vector<double> strip_theta, strip_eta;
    int64_t n_strip = 0;
    int newton_max_iters = 0;
    int strip_wmax = 0;   // widest stencil window (normals) of a block of 512 theta-sorted STRIP points
    int64_t n_in = 0, n_far = 0;
    int seed = 0;
    bool interior_only = false;   // Remark 3.1 II: no boundary samples, d matching values interpolated
    int64_t n_solved = 0, n_fallback = 0, newton_iters = 0;
    double t_ms[FC2D_PLAN_PHASES] = {};   // host wall clock per set-up phase (fc2d_plan_info.t_ms)
    // device
    double* d_Q = nullptr;          // [d][d]
    double* d_Ar = nullptr;         // [Cr][d]
    // matching stencils, per normal (NU = 4 ceil(M*M / 16), RQ = ceil((d-1) / 4)):
    int32_t* d_mref = nullptr;      // [B][4][NU] stencil entries in address order (entry 4u + sq at [sq][u]):
                                    //   grid flat index (>= 0) or -(1 + square)
    uint8_t* d_mlab = nullptr;      // [B][4][NU] star s, node k of each entry as s M + k (255: padding)
    double* d_mwv = nullptr;        // [B][RS][M][4][2] (RS = ceil(M / 4)) weights along the grid line of star 4r + sq, node k at
                                    //   [r][k][sq] (double-double; zero for stars >= M)
    double* d_mwn = nullptr;        // [B][RQ][M][4][2] weights along the normal of matching value 4r + sq,
                                    //   star s at [r][s][sq] (double-double; zero for values >= d-1)
    int32_t* d_sidx = nullptr;      // [S] STRIP flat index
    double* d_sth = nullptr;        // [S] theta^Q
    double* d_seta = nullptr;       // [S] eta_Q
    int32_t* d_run_ptr = nullptr;   // [nx + 1] row runs
    int32_t* d_run = nullptr;       // [nruns][3] (start, end, class)
    double* d_bxy = nullptr;        // [n_bdry][2] boundary points (feet, then squares)
    uint8_t* d_cls2 = nullptr;      // [nx][ny/2] pair classes (2 bits per point) in row-pass thread order
    int8_t* d_cls = nullptr;        // [nx][ny] classes (0 FAR, 1 IN, 2 STRIP)
    int32_t* d_rm_idx = nullptr;    // [S] row-major STRIP list: flat index, seed normal
    int32_t* d_rm_seed = nullptr;
    double* d_rm_th = nullptr;      // [S] theta^Q, eta_Q in row-major order
    double* d_rm_eta = nullptr;
    int nruns = 0;
};

namespace fc2d {

// ---- plan kernels (kernels_plan.hip) ----
struct ClassifyArgs {
    CurveC curve;
    double x0, y0, h;
    int nx, ny;
    const double *bx, *by, *bnx, *bny;
    int B, M;
    double k2, r_out, r_in, width;   // width = C k1
    const int32_t* col_ptr;          // [nx + 1]
    const double* col_y;             // crossings of column x_i with the polygon, sorted
    int maxit;
};
struct StripRec {
    int32_t idx;
    int32_t seed;
    int32_t iters;
    int32_t pad;
    double theta;
    double eta;
};
// Runs nearest-sample scatter + classification; fills cls (device, nx*ny),
// strip records (device, capacity cap) and counters[0] = count, counters[1] =
// foot failures, counters[2] = max iterations.
int launch_classify(const ClassifyArgs& a, int8_t* d_cls, StripRec* d_rec, int64_t cap,
                    uint64_t* d_near, int* d_counters, hipStream_t s);

// Seeds from the polar angle (FC2D_SEED_POLAR, FC2D_SEED_MLP).
struct SeedArgs {
    CurveC curve;                 // polar
    double x0, y0, h;
    int nx, ny;
    int B, maxit;
    double k2;
    double band_lo, band_hi;      // candidates: band_lo <= rho - r(phi) <= band_hi
    double width;                 // C k1
    double dist2_max;             // MLP roots farther than this (squared) from Q are rejected
    double mlp_tol;               // residual threshold after the two MLP-seeded steps
};
// counters: [0] STRIP records, [1] failed solves, [2] most Newton steps of a
// STRIP point, [3] candidates, [4] fallbacks, [5] Newton steps summed.
int launch_radial_band(const SeedArgs& a, int8_t* d_cls, int32_t* d_cand, int64_t cap, int* d_counters,
                       hipStream_t s);
int launch_seed_polar(const SeedArgs& a, const int32_t* d_cand, int64_t ncand, int8_t* d_cls, StripRec* d_rec,
                      int64_t cap, int* d_counters, hipStream_t s);
int launch_seed_mlp(const SeedArgs& a, const float* d_w, const int32_t* d_cand, int64_t ncand, int8_t* d_cls,
                    StripRec* d_rec, int64_t cap, int* d_counters, hipStream_t s);

// Lists of the plan built on the device from the classes and the STRIP records:
// per-row runs of equal class (d_run_ptr, d_run), the row pass's pair classes
// (d_cls2, when pair_E > 0), the row-major STRIP list (d_rm_*) and the STRIP
// list in order of theta (d_sidx, d_sth, d_seta) with the widest strip-kernel
// block window (strip_wmax), plus n_in / n_far.  The classification work space
// (d_cls, rec with S records) must be complete on stream s.
int plan_device_lists(fc2d_plan* pl, const StripRec* d_rec, int64_t S, hipStream_t s);
// host copies of the classes and the row-major STRIP list (downloaded once)
int plan_host_lists(const fc2d_plan* pl);

struct StarArgs {
    CurveC curve;
    const double *bx, *by, *bnx, *bny;
    int B, M, maxit, io;
    double k2, x0, y0, h;
    int nx, ny;
};
int launch_star_scan(const StarArgs& a, const int8_t* d_cls, const StarQ* d_q, StarR* d_r, int n, hipStream_t s);

// ---- batches: one descriptor per (plan, field set) for the persistent kernels ----
struct PlanDev {
    const int32_t* mref;
    const uint8_t* mlab;
    const double* mwv;
    const double* mwn;
    const double* Q;
    const int32_t* sidx;
    const double* sth;
    const double* seta;
    const double* bxy;
    int B, D, nf, nx, ny, io;   // io: plan built from interior data only
    int64_t npts, nbdry, S;
    double k2, lev_scale, x0, y0, h;
    double* u;    // [nf][nx][ny] fields: IN values read, STRIP values written
    double* fb;   // [nf][nbdry] boundary values
    double* c;    // [nf][B][DP] Gram records
    int64_t off_match, off_strip, off_bv;   // first work item of this entry
};
// which: 0 match, 1 strip, 2 boundary values
// LDS bytes of the strip kernels for a widest block window wmax (normals), and
// the stage shape they use: at most lcap normals, fstage fields per stage
size_t strip_lds(int wmax, int d, int Cr, int fpt, int* lcap, int* fstage);
int launch_multi(int which, int M, const PlanDev* d_pd, int np, int64_t total, int fpt, const double* Ar, int D,
                 int Cr, int wmax, int grid_blocks, hipStream_t s);
int launch_bvals(const fc2d_plan* pl, const double* u, double* fb, int nf, hipStream_t s);

// crossing of a grid-line segment with Gamma (plan.cpp; bisection on eta)
int gridline_crossing(const fc2d_plan* pl, bool vertical, double a_line, double b_in, double b_out, double* out);

// ---- extension kernels (kernels_extend.hip) ----
int launch_match(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, int64_t nbdry,
                 double* c_out, double* fD_out, int nf, hipStream_t s);
int launch_blend(const fc2d_plan* pl, const double* c, double* F, int nf, hipStream_t s);
int launch_strip(const fc2d_plan* pl, const double* c, const double* f_bdry, int64_t nbdry,
                 double* out, int nf, hipStream_t s);
int launch_mask(const fc2d_plan* pl, const double* f_grid, double* out, int nf, hipStream_t s);
// Gram records [nf][B][DP] (c_0..c_{d-1}, boundary value, zero pad; DP = (d+2)&~1)
// written by launch_match and read by launch_strip
inline size_t gram_bytes(const fc2d_plan* pl, int nf) {
    return (size_t)nf * (size_t)pl->B * (size_t)((pl->d + 2) & ~1) * sizeof(double);
}
// The library's fixed scratch array for callers that cannot allocate
// (kernels_extend.hip): its device address on the current device (looked up
// once per device) and its size in bytes.
int static_scratch(double** p, size_t* bytes);

// ---- FFT and spectral kernels (kernels_fft.hip) ----
// strip / cls2 non-null: the rows are assembled on the fly from `in` (IN),
// `strip` (STRIP) and zeros (FAR) using the per-pair class bytes cls2.
// ld: row pitch of the half spectrum in complex elements (0 -> ny/2 + 1, the numpy layout)
int fft2_r2c(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s,
             const double* strip = nullptr, const uint8_t* cls2 = nullptr, int ld = 0);
int fft2_c2r(const fc2d_grid* g, double* in, double* out, int nf, hipStream_t s, int ld = 0);
// single passes (batches) and twiddle set-up outside stream capture
int fft_prepare(int nx, int ny);
// true when the twiddle tables of lengths nx and ny exist on the current device
// (then the FFT launches allocate nothing)
bool fft_ready(int nx, int ny);
int fft_rows_fwd(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s, const double* strip,
                 const uint8_t* cls2, int ld = 0);
int fft_cols(const fc2d_grid* g, double* data, int nf, bool inv, hipStream_t s, int ld = 0);
int fft_rows_inv(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s, int ld = 0);
// the same row passes with the half spectrum transposed, [field][bin][row] (ny <= 4096)
int fft_rows_fwd_t(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s, const double* strip,
                   const uint8_t* cls2);
int fft_rows_inv_t(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s);
int spectral_apply(const fc2d_grid* g, int op, const double* in, double* out, int nf, hipStream_t s);
int ff_apply(const fc2d_grid* g, double c, double t, const double* u0, const double* u1, double* uh,
             double* uth, int nf, hipStream_t s);
// column pass + propagation by t + inverse column pass in one launch, in place
// on row-transformed spectra su, sut ([nf][nx][ny/2+1] each)
// trans: spectra stored transposed ([field][column][row]), as fft_rows_fwd_t writes them
// U_FC(t) on the grid: out = inverse FFT of cos(w t) u0 + sin(w t) / w u1 (half
// spectra [nf][nx][ny/2+1]); spec receives the column-transformed spectrum
int prop_c2r(const fc2d_grid* g, double c, double t, const double* u0, const double* u1, double* spec, double* out,
             int nf, hipStream_t s);
int cols_ff(const fc2d_grid* g, double c, double t, double* su, double* sut, int nf, hipStream_t s,
            bool trans = false);
int colff_variants(int nx);   // compiled launch shapes of cols_ff for length nx
int colff_get(int nx);
int colff_set(int nx, int v);

// masked row pass: elements per thread and the thread-order class layout
int row_elems(int L);
void row_class_layout(int L, const uint8_t* pairs, uint8_t* out);

// tuning knobs (autotuner)
int col_tile_get(int nx);
int col_tile_set(int nx, int T);
int col_elems_get(int nx);
int col_elems_set(int nx, int E);
int col_cfg_set(int nx, int E, int T);
int strip_fpt_get();
int strip_fpt_set(int v);
int strip_wcap_get();
int strip_wcap_set(int v);

}  // namespace fc2d
