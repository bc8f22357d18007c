/*
 * fc2d.h -- C ABI of the MI355X (gfx950) two-dimensional Fourier Continuation
 * library (libfc2d.so).
 *
 * Method: O. P. Bruno and J. Paul, "Two-dimensional Fourier Continuation and
 * applications", arXiv 2010.03901.  Section numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 *  - Status: 0 (FC2D_OK) on success, a negative FC2D_E_* code on failure;
 *    fc2d_last_error() returns a message for the calling thread's last failure.
 *  - Grid arrays are row-major [field][i][j] <-> (x_i, y_j) = (x0 + i h, y0 + j h)
 *    with j (the y index) fastest, float64 (eq. cart_grid).  The box is periodic
 *    with period N h; the right edge is excluded.
 *  - Half spectra are [field][i][j'] with j' = 0..N_y/2, interleaved complex128
 *    (re, im), the real-to-complex convention along y then a complex transform
 *    along x (the layout of numpy.fft.rfft2).
 *  - Device pointers are hipMalloc'ed (or torch) memory on the current device;
 *    host pointers are ordinary memory.  The library never frees caller memory.
 *  - Calls taking a stream enqueue work asynchronously on it (NULL = the null
 *    stream); enqueue-time errors are returned, kernel faults surface at the
 *    next synchronisation.
 *  - A plan is read-only after creation.  Calls that need device work space
 *    (the Gram records of the matching step, the buffers of a Poisson solve)
 *    take it per call from a library-owned memory pool, ordered on the call's
 *    stream, and return it on that stream; so calls sharing one plan may run
 *    concurrently on different streams (and from different host threads).
 *    Plan creation takes its temporaries from the same pool.  The pool (one
 *    per device) keeps what it has held until the process ends, so later
 *    calls reach no device allocator (at 4096^2 a plan's creation leaves about
 *    0.3 GB in it).
 *    The exceptions are named where they occur: a batch (fc2d_batch_*) is
 *    advanced by one stream at a time, the tuning knobs are process-wide, and
 *    fc2d_extend_fft_noalloc shares one fixed scratch per device.
 */
#ifndef FC2D_H
#define FC2D_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FC2D_VERSION 100

enum {
    FC2D_OK = 0,
    FC2D_E_ARG = -1,          /* invalid argument (NULL, size, unsupported combination) */
    FC2D_E_TABLE = -2,        /* FC-Gram table could not be built for the parameters */
    FC2D_E_GEOMETRY = -3,     /* domain/grid inadmissible (reach, box, matching stencils) */
    FC2D_E_NEWTON = -4,       /* foot-of-normal solve did not converge */
    FC2D_E_HIP = -5,          /* a HIP runtime call failed */
    FC2D_E_NOMEM = -6         /* device or host allocation failed */
};

enum { FC2D_CURVE_POLAR = 1, FC2D_CURVE_CARTESIAN = 2 };
enum { FC2D_FORWARD = -1, FC2D_INVERSE = 1 };
enum { FC2D_LAPLACE_INV = 1, FC2D_DX = 2, FC2D_DY = 3 };
enum {
    FC2D_TUNE_COL_TILE = 1,
    FC2D_TUNE_STRIP_FIELDS = 2,
    FC2D_TUNE_COL_ELEMS = 3,
    FC2D_TUNE_STRIP_WINDOW = 4,
    FC2D_TUNE_FF_SHAPE = 5
};

/* How the foot-of-normal solve of each grid point near Gamma is started
 * (fc2d_opts.seed):
 *  PROXIMITY  every boundary sample marks the grid points within C k1 of it
 *             (the proximity map of Sec. 3.3, reduced to the nearest sample),
 *             the seed is T(tau) over the normals of S_{theta_p} (Sec. 3.4);
 *             any curve; points away from Gamma are classified by the
 *             crossing parity of their grid column.
 *  POLAR      polar curves only: points with rho - r(phi) in a band around
 *             Gamma (phi = atan2(y, x)) are solved from the seed phi; the
 *             others are IN (rho < r(phi)) or FAR.
 *  MLP        as POLAR, but the seed comes from the learned network
 *             (fc2d_opts.mlp_weights) followed by two plain Newton steps;
 *             the root is kept when the residual |g / g'| after them is at
 *             most mlp_tol, g' > 0 and it lies within the exterior reach,
 *             otherwise the point falls back to the bracketed solve of POLAR.
 * All three give the same classes and STRIP list, and feet equal to rounding. */
enum { FC2D_SEED_PROXIMITY = 0, FC2D_SEED_POLAR = 1, FC2D_SEED_MLP = 2 };

/* The learned seed network: 8 inputs, three hidden layers of 64 tanh units, 2
 * linear outputs, float32 weights stored flat layer by layer, each layer as W
 * (row-major [fan_in][fan_out]) followed by its bias. */
#define FC2D_MLP_NIN 8
#define FC2D_MLP_HIDDEN 64
#define FC2D_MLP_NW 9026

/* Boundary Gamma as a smooth 2 pi-periodic counter-clockwise curve q(theta)
 * (eq. param).  Series s(t) = s0 + sum_{m=1..nmodes} (s_{2m-1} cos mt + s_{2m} sin mt),
 * arrays of 1 + 2 nmodes doubles:
 *   POLAR      q = r(t) (cos t, sin t) with r = series a; b unused;
 *   CARTESIAN  x(t) = series a, y(t) = series b.
 * The outward normal is n = (y', -x') / |q'| (Sec. 3.1).  Host memory; copied. */
typedef struct {
    int kind;
    int nmodes;
    const double* a;
    const double* b;
} fc2d_curve;

/* Cartesian grid H of eq. cart_grid: x_i = x0 + i h (0 <= i < nx), y_j = y0 + j h. */
typedef struct {
    double x0, y0, h;
    int nx, ny;
} fc2d_grid;

/* Plan options; fc2d_opts_default() fills the paper's choices (Remark 3.3):
 * n_r = 6, Z = 12, n_os = 20, M = d + 3, k1 = h, B = nearest power of two to
 * 2 pi / h, trigonometric band limit mf = 20. */
typedef struct {
    int B;             /* boundary points, k2 = 2 pi / B (eq. bdry_grid) */
    double k1;         /* normal step (eq. vnbj_m, eq. vnbj_p); 0 -> h */
    int M;             /* interpolation nodes (degree M - 1); 0 -> d + 3; compiled sizes
                          4..8, 13 and 15 (d = 10, 12 with M = d + 3, Remark 3.5); M >= d - 1 */
    int n_r;           /* refinement factor, C_r = n_r C (Remark 2.2) */
    int Z;             /* zero-matching points (eq. min_prob) */
    int n_os;          /* oversampling factor (eq. q_over) */
    int mf;            /* band limit of the trigonometric fit (eq. auxi_trig_poly) */
    int newton_maxit;  /* cap on foot-of-normal iterations (failure testing); 0 -> 60 */
    int seed;          /* FC2D_SEED_*; 0 -> PROXIMITY */
    double mlp_tol;    /* MLP seed: residual threshold; 0 -> 1e-13; < 0 -> every point falls back */
    const float* mlp_weights;   /* MLP seed: FC2D_MLP_NW floats, host memory (copied) */
    int interior_only; /* 1: extension from interior data only (Remark 3.1 II): the matching
                          stencils use IN grid points only and the matching value on Gamma is
                          interpolated along the normal like the others; the extension calls
                          then read no boundary samples (f_bdry may be NULL).  0: the paper's
                          default, boundary samples at the feet and squares. */
} fc2d_opts;

typedef struct fc2d_plan fc2d_plan;

/* Phases of plan creation timed in fc2d_plan_info.t_ms (host wall clock; device
 * work inside a phase is waited for by that phase). */
enum {
    FC2D_PHASE_GEOMETRY = 0,   /* boundary grid, admissibility, crossing polygon */
    FC2D_PHASE_CLASSIFY = 1,   /* classification and foot kernels, until their results are on the host */
    FC2D_PHASE_LISTS = 2,      /* STRIP list order, class counts */
    FC2D_PHASE_MATCHING = 3,   /* matching stencils, squares and weights */
    FC2D_PHASE_LAYOUT = 4,     /* device layouts (stencils, row runs, pair classes) and uploads */
    FC2D_PLAN_PHASES = 5
};

typedef struct {
    int d, C, M, n_r, Cr, B;
    double k1, k2;
    int64_t n_bdry;     /* B feet + squares: length of f_bdry */
    int64_t n_strip;    /* grid points with 0 < eta <= C k1 */
    int64_t n_in, n_far;
    int newton_max_iters;   /* most Newton steps taken by a STRIP point */
    int seed;               /* FC2D_SEED_* the plan was built with */
    int64_t n_solved;       /* grid points whose foot was solved (candidates near Gamma) */
    int64_t n_fallback;     /* MLP seed: points that took the bracketed fallback */
    int64_t newton_iters;   /* Newton steps summed over the solved points */
    double t_ms[FC2D_PLAN_PHASES];   /* host wall clock of plan creation by phase, ms: FC2D_PHASE_* */
} fc2d_plan_info;

void fc2d_opts_default(const fc2d_grid* grid, fc2d_opts* opts);

/* Geometrical Setup (Sec. 3.5 steps 1-4): boundary grid and normals,
 * admissibility (C k1 <= 0.9 exterior reach; Omega u V+ inside the box),
 * classification of H into IN / STRIP / FAR with the foot of the normal
 * (theta^Q, eta_Q) of every STRIP point (Sec. 3.3, 3.4), the matching stencils
 * of Sec. 3.2 and the FC-Gram tables of Sec. 2.2 / Remark 2.2.  Runs kernels on
 * `stream` and synchronises it.  *out owns its device memory; immutable after
 * creation; release with fc2d_plan_destroy.  Errors: FC2D_E_ARG, FC2D_E_TABLE,
 * FC2D_E_GEOMETRY, FC2D_E_NEWTON, FC2D_E_HIP, FC2D_E_NOMEM. */
int fc2d_plan_create(const fc2d_curve* curve, const fc2d_grid* grid, int d, int C,
                     const fc2d_opts* opts, hipStream_t stream, fc2d_plan** out);
int fc2d_plan_destroy(fc2d_plan* plan);
int fc2d_plan_get_info(const fc2d_plan* plan, fc2d_plan_info* info);

/* Boundary points whose values f_bdry must hold (host memory): the B feet
 * q(theta_p) first, then the crossings of the matching-stencil grid lines with
 * Gamma (the "squares" of Fig. 3).  *n receives the count; xy (2 n doubles,
 * x then y per point) may be NULL to query n. */
int fc2d_boundary_points(const fc2d_plan* plan, int64_t* n, double* xy);

/* Plan contents for checking (host memory).  classes: nx*ny int8 with
 * 0 = FAR, 1 = IN, 2 = STRIP.  strip arrays: n_strip entries in row-major order
 * of the flat grid index; theta in [0, 2 pi), eta in (0, C k1]; seed = the
 * proximity-map normal index used to start the foot solve.  Any pointer may be NULL. */
int fc2d_plan_classes(const fc2d_plan* plan, int8_t* classes);
int fc2d_plan_strip(const fc2d_plan* plan, int64_t* index, double* theta, double* eta, int32_t* seed);

/* Matching values f_{D_p} (Sec. 3.2): fD [nf][B][d] device float64, from
 * f_grid [nf][nx][ny] (device; only IN entries read) and f_bdry [nf][n_bdry]
 * (device).  Sums are carried in double-double and rounded once.  With a plan
 * built from interior data only (fc2d_opts.interior_only; Remark 3.1 II)
 * f_bdry is not read and may be NULL, here and in fc2d_blend, fc2d_extend,
 * fc2d_extend_fft and fc2d_poisson_solve. */
int fc2d_matching(const fc2d_plan* plan, const double* f_grid, const double* f_bdry,
                  double* fD, int nf, hipStream_t stream);

/* Blending to zero on V+_{B,C_r} (eq. b_to_z, Remark 2.2): F [nf][C_r+1][B]
 * device float64 with F[0][p] = f_{D_p}[d-1] (f_bdry[p], or its interpolated value from
 * interior data only) and F[l][p] = (A_r Q^T f_{D_p})_{l-1}.
 * A materialised check of the blend; fc2d_extend never forms F. */
int fc2d_blend(const fc2d_plan* plan, const double* f_grid, const double* f_bdry,
               double* F, int nf, hipStream_t stream);

/* 2D-FC extension f^c on H (Sec. 3.5 steps 5-6): out [nf][nx][ny] device with
 * IN points = f (bitwise), STRIP points = interpolated continuation, FAR = 0.
 * out may alias f_grid (in place: then only STRIP and FAR entries are written). */
int fc2d_extend(const fc2d_plan* plan, const double* f_grid, const double* f_bdry,
                double* out, int nf, hipStream_t stream);

/* Boundary values for a later Fourier-Forwarding step (the paper takes them
 * from its near-boundary solver; here they are read off the full-box field):
 * f_bdry [nf][n_bdry] (device) = degree-(M-1) tensor-product Lagrange
 * interpolation of u [nf][nx][ny] (device) on the centred M x M node block
 * around each boundary point of fc2d_boundary_points (indices periodic). */
int fc2d_boundary_values(const fc2d_plan* plan, const double* u, double* f_bdry, int nf, hipStream_t stream);

/* Extension fused with the forward 2D FFT (Sec. 3.5 steps 5-7): spec [nf][nx][ny/2+1]
 * complex128 = the unnormalised forward transform of the grid fc2d_extend would
 * produce, without materialising it: the STRIP values are written into `work`
 * ([nf][nx][ny] float64, only STRIP entries are touched; it may alias f_grid)
 * and the row transform assembles IN / STRIP / FAR values while loading.
 * The plan's grid must have power-of-two sizes (nx <= 4096, ny <= 8192). */
int fc2d_extend_fft(const fc2d_plan* plan, const double* f_grid, const double* f_bdry, double* work,
                    void* spec, int nf, hipStream_t stream);

/* fc2d_extend_fft with the half spectrum's rows spec_ld >= ny/2 + 1 complex
 * elements apart: spec [nf][nx][spec_ld], columns ny/2 + 1 .. spec_ld - 1 of
 * each row neither read nor written.  spec_ld = ny/2 + 1 is the layout of
 * fc2d_extend_fft; a multiple of 8 starts every row on a 128-byte boundary,
 * so the column pass reads and writes whole cache lines (the numpy layout's
 * 16 (ny/2 + 1)-byte rows start 16 bytes further into a line each row). */
int fc2d_extend_fft_ld(const fc2d_plan* plan, const double* f_grid, const double* f_bdry, double* work,
                       void* spec, int spec_ld, int nf, hipStream_t stream);

/* fc2d_extend_fft for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * same arguments, kernels and results (bitwise), but the Gram records live in
 * the library's fixed scratch, a 16 MiB device array per device held until the
 * process ends, and no allocation routine is called.  Requires
 * nf * B * ((d + 2) & ~1) * 8 <= 16 MiB (FC2D_E_ARG otherwise; e.g. 170 fields
 * at B = 2048, d = 5) and a plan created on the current device (its FFT tables
 * and the scratch's address are set up there; FC2D_E_ARG otherwise).  Every
 * call on one device shares the scratch: calls that overlap on one device
 * (different streams or threads, or graphs replayed concurrently)
 * race and give wrong results; order them on one stream. */
int fc2d_extend_fft_noalloc(const fc2d_plan* plan, const double* f_grid, const double* f_bdry, double* work,
                            void* spec, int nf, hipStream_t stream);

/* 2D FFT (Sec. 3.5 step 7); nx a power of two in [16, 4096], ny a power of
 * two in [16, 8192] (Remark 3.2: the grid is padded to FFT-friendly sizes).
 * FC2D_FORWARD: in = real [nf][nx][ny] (not modified), out = half spectrum,
 * unnormalised.
 * FC2D_INVERSE: in = half spectrum, overwritten: the inverse column pass runs
 * in place on it before the row pass writes the reals (keeping it would take a
 * second spectrum-sized buffer per call), out = real, scaled by 1/(nx ny).
 * in and out must not overlap; `in` is therefore not const. */
int fc2d_fft(const fc2d_grid* grid, void* in, void* out, int dir, int nf, hipStream_t stream);
/* fc2d_fft with the half spectrum's rows spec_ld >= ny/2 + 1 complex elements
 * apart (as fc2d_extend_fft_ld). */
int fc2d_fft_ld(const fc2d_grid* grid, void* in, void* out, int dir, int spec_ld, int nf, hipStream_t stream);

/* Full Poisson solve (Sec. 4.1; eq. def_poisson): Delta u = f in Omega, u = g on
 * Gamma, as u = u_p + v (eq. total_soln).  u_p is the 2D-FC particular solution
 * (eq. poisson_ps: the extension's spectrum over -|k|^2, plus f_00 (x^2 + y^2)/4
 * with f_00 the extension's mean -- the printed formula's minus sign on this
 * term is read as a plus, so that Delta u_p = f); v is harmonic with
 * v = g - u_p on Gamma (eq. def_laplace, eq. laplace_bc), a double-layer
 * potential whose density solves the second-kind Nystrom system of the
 * trapezoidal rule on nb nodes q(2 pi j / nb), by GMRES; u_p on Gamma comes from
 * degree-(M-1) tensor interpolation (the plan's M).  v is summed at the IN grid
 * points (density refined up to 128x near Gamma); points within h/2 of Gamma use the
 * foot value and M - 1 values along the inward normal at h/2, h, ...
 * interpolated in the distance with degree M - 1.  Fields are solved in chunks
 * of up to four that share the GMRES passes over the Nystrom matrix and the
 * geometry work of the double-layer sums (results per field as when alone, to
 * rounding).
 * fc2d_poisson_nodes writes the nodes, host xy [2 nb], where the caller samples
 * g.  fc2d_poisson_solve: device f_grid [nf][nx][ny] (IN entries read),
 * f_bdry [nf][n_bdry] (the plan's boundary points), g_nodes [nf][nb]; writes
 * u [nf][nx][ny] (IN points; every other point 0).  Power-of-two grids, 8 <= nb
 * <= 16384.  Takes its device work space per call on `stream` (from the
 * library's pool, so solves on one plan may overlap on different streams);
 * synchronises `stream` (GMRES reads its scalars on the host), returns the GMRES iterations summed over the fields in *gmres_iters
 * (may be NULL).  FC2D_E_NEWTON when GMRES or a foot solve fails;
 * FC2D_E_NOMEM when the work buffers (about 3 + min(nf, 4) grids of nx ny
 * doubles plus 8 nb^2 bytes) do not fit. */
int fc2d_poisson_nodes(const fc2d_plan* plan, int nb, double* xy);
int fc2d_poisson_solve(const fc2d_plan* plan, const double* f_grid, const double* f_bdry, const double* g_nodes,
                       int nb, double* u, int nf, hipStream_t stream, int* gmres_iters);

/* Spectral operators on half spectra (in place allowed): FC2D_LAPLACE_INV
 * multiplies by -1/|k|^2 with the (0,0) mode set to 0 (eq. poisson_ps_coeffs);
 * FC2D_DX / FC2D_DY multiply by i k_x / i k_y with the Nyquist mode zeroed;
 * k = (2 pi l / (nx h), 2 pi m / (ny h)), l in (-nx/2, nx/2]. */
int fc2d_spectral_apply(const fc2d_grid* grid, int op, const void* in, void* out, int nf,
                        hipStream_t stream);

/* Fourier Forwarding modal propagation (eq. wave_2d_ff_modal, eq. wave_2d_ff):
 * uh = cos(w t) u0h + sin(w t)/w u1h and uth = -w sin(w t) u0h + cos(w t) u1h with
 * w = 2 pi c |(l/(nx h), m/(ny h))|; the (0,0) mode gets u0h + t u1h and u1h.
 * Half spectra, device; outputs may alias inputs. */
int ff_propagate(const fc2d_grid* grid, double c, double t, const void* u0h, const void* u1h,
                 void* uh, void* uth, int nf, hipStream_t stream);

/* ---- Fourier Forwarding solver of the wave equation (Sec. 4.2) ----
 * u_tt = c^2 (u_xx + u_yy) in Omega (eq. wave_2d) with Dirichlet data
 * u = b(x, y, t) on Gamma.  fc2d_ff_advance takes the solution from T_j to
 * T_j + nsmall dt (nsmall <= K, K dt = dT = n_c h / c) as eq. ff_soln
 * combines it:
 *  - U_FC (eq. aux_sol): the 2D-FC extensions of u and u_t at T_j (boundary
 *    samples fb_u, fb_ut = b, b_t at T_j on the plan's fc2d_boundary_points),
 *    their spectra advanced in closed form (eq. wave_2d_ff); it is taken at
 *    the interior points, which lie at least c dT from Gamma;
 *  - U_B: on the boundary region (IN points within Chebyshev grid distance
 *    n_c + 2 of a non-IN point) explicit second-order Taylor steps of
 *    dt = dT / (8 n_c) (CFL 0.125): u += dt v + dt^2/2 a, v += dt (a + a')/2
 *    with a = c^2 (u_xx + u_yy) from the 1D-FC of Sec. 2.3 (both blends)
 *    along grid lines (runs shorter than 2 d: the Lagrange interpolant through
 *    the run and its crossings with Gamma); the grid points next to Gamma
 *    (along x or y) take the cubic interpolant along their grid line through
 *    the Dirichlet value at the line's crossing with Gamma and the nearest
 *    stepped points; values needed beyond the region come from U_FC at the
 *    current time.  The paper defers the details of U_B; these are the
 *    library's readings.
 * The solver owns its work buffers (4 half spectra and 2 grids per field) and
 * is advanced by one stream at a time.  One field per call. */
typedef struct fc2d_ff fc2d_ff;
typedef struct {
    double c, dT, dt;        /* wave speed, large step, small step */
    int K, n_c, M_b;         /* small steps per large step, region width, closure nodes */
    int64_t n_cross;         /* crossings of grid lines with Gamma: Dirichlet data per small step */
    int64_t n_stepped, n_bnd;   /* stepped and interpolated (boundary) points of U_B */
    int n_segments, max_segment;
} fc2d_ff_info;
/* Solver on the plan's grid (power of two, boundary data; the plan must
 * outlive it).  c > 0, 1 <= n_c <= 64 (the paper's examples: 6);
 * closure_nodes 2..4 (0 -> 4): nodes of the interpolation closure at the grid
 * points next to Gamma.  Host set-up
 * (crossings by bisection on eta, closure and derivative matrices in long
 * double) plus device uploads; FC2D_E_GEOMETRY if a derivative segment would
 * exceed 2048 points. */
int fc2d_ff_create(const fc2d_plan* plan, double c, int n_c, int closure_nodes, hipStream_t stream, fc2d_ff** out);
int fc2d_ff_destroy(fc2d_ff* ff);
int fc2d_ff_get_info(const fc2d_ff* ff, fc2d_ff_info* info);
/* The crossings (host xy [2 n]) where the caller supplies b and b_t at every
 * small step; xy may be NULL to query n. */
int fc2d_ff_crossings(const fc2d_ff* ff, int64_t* n, double* xy);
/* Per grid point (host [nx][ny]): 0 outside Omega, 1 interior (U_FC),
 * 2 stepped, 3 boundary point of U_B. */
int fc2d_ff_regions(const fc2d_ff* ff, int8_t* region);
/* Advance one field by nsmall small steps (1 <= nsmall <= K) from T_j.  u, ut
 * [nx][ny] device: the solution and its time derivative at T_j at the IN
 * points on entry, at T_j + nsmall dt on return (0 outside Omega).  fb_u,
 * fb_ut [n_bdry]: b and b_t at T_j on the plan's boundary points.  bc_u,
 * bc_ut [nsmall + 1][n_cross]: b and b_t at the crossings at T_j + k dt,
 * k = 0..nsmall.  Asynchronous on `stream`. */
int fc2d_ff_advance(fc2d_ff* ff, double* u, double* ut, const double* fb_u, const double* fb_ut,
                    const double* bc_u, const double* bc_ut, int nsmall, hipStream_t stream);

/* Launch-shape knobs, process-wide (set by the autotuner; results do not
 * depend on them beyond rounding).  For the column FFT pass of length n = nx:
 * FC2D_TUNE_COL_TILE = columns per block T, FC2D_TUNE_COL_ELEMS = elements per
 * thread E; compiled (E, T): n <= 64 (2; 4/8/16), 128 (2; 4/8), 256 (4; 4/8),
 * 512 (4 or 8; 4/8), 1024 (8 or 16; 2/4/8), 2048 (16; 1/2/4 and 8; 1/2),
 * 4096 (16; 1/2 and 8; 1).  A setting that would form an uncompiled pair is
 * refused with FC2D_E_ARG.  FC2D_TUNE_STRIP_FIELDS: fields per thread of the
 * strip interpolation (0 = automatic, n ignored).  FC2D_TUNE_STRIP_WINDOW: at
 * most this many normals of Gram records are staged in LDS per block of 512
 * STRIP points (0 = no cap beyond the LDS budget; n ignored); blocks whose
 * stencils span more normals read the records from device memory instead.
 * FC2D_TUNE_FF_SHAPE: index of the compiled shape of the fused column-pass +
 * propagation kernel for length n (batches; n = 256, 512: 0..2, n = 1024:
 * 0..5, n = 2048: 0..5, n = 4096: 0..1, other lengths: 0; index 3 of 1024, the
 * last two of 2048 and the last of 4096 take one column of both spectra per
 * block, propagated in registers).  Not thread-safe against
 * concurrent launches. */
int fc2d_tune_set(int knob, int n, int value);
int fc2d_tune_get(int knob, int n, int* value);

/* Kernel tracing (a profiling aid, not needed for results).  fc2d_trace_begin
 * opens a trace and records a HIP event on `stream`; until fc2d_trace_end every
 * kernel the library launches records one more event after it on its own
 * stream.  fc2d_trace_end synchronises, closes the trace and returns, in
 * launch order, up to `cap` entries of kernel name (static strings owned by
 * the library) and milliseconds since the previous event -- the kernel's
 * duration when the traced calls share one stream.  *n receives the number
 * of entries written.  Either output array may be NULL. */
int fc2d_trace_begin(hipStream_t stream);
int fc2d_trace_end(int* n, const char** names, float* ms, int cap);

/* Batches (Fourier Forwarding of many fields on several domains and grid
 * sizes, Sec. 4.2).  A batch holds, for plan k, nf[k] field pairs (u, u_t) on
 * the plan's full box and advances them together; one step is
 *   f_bdry <- fc2d_boundary_values(u), (u_t likewise)
 *   spectra <- fc2d_extend_fft of u and u_t
 *   spectra <- ff_propagate by dt
 *   (u, u_t) <- inverse FFT (whole box).
 * The plan-specific stages run as single persistent launches over all plans;
 * the FFT passes run once per (nx, ny, h) with those fields contiguous.  The
 * plans must share d, C, n_r, M and have power-of-two grids, and must outlive
 * the batch.  flags: FC2D_BATCH_FUSED_FF runs the forward column pass, the
 * propagation and the inverse column pass of each grid size as one kernel
 * (instead of three); FC2D_BATCH_AUTOTUNE times the column-pass shapes, the
 * fused against the separate spectral step per grid size, row-major against
 * transposed spectra, and the strip kernel's fields per thread on the batch's
 * buffers and keeps the fastest (launch shapes are process-wide, see
 * fc2d_tune_set); FC2D_BATCH_TRANSPOSED keeps each grid size's spectra
 * transposed (bin-major within groups of 8 rows, so a bin's 8 rows fill one
 * 128-byte line: the column passes read whole lines, the row passes a group's
 * bins as one contiguous range, 4 rows at a time; grids with ny <= 4096 and nx
 * a multiple of 8) and implies the fused spectral step for those sizes.  The
 * spectra are internal: results do not depend on the layout beyond rounding.
 * State starts at zero. */
typedef struct fc2d_batch fc2d_batch;
enum { FC2D_BATCH_AUTOTUNE = 1, FC2D_BATCH_FUSED_FF = 2, FC2D_BATCH_TRANSPOSED = 4 };
int fc2d_batch_create(const fc2d_plan* const* plans, const int* nf, int nplans, unsigned flags,
                      hipStream_t stream, fc2d_batch** out);
/* Device pointers to plan k's state: u and u_t, each [nf[k]][nx][ny]. */
int fc2d_batch_state(fc2d_batch* batch, int k, double** u, double** ut);
/* Grid points extended per step (u and u_t of every field), launches per
 * step, and the strip kernel's fields per thread. */
int fc2d_batch_info(const fc2d_batch* batch, int64_t* points_per_step, int* launches_per_step,
                    int* strip_fields);
/* Advance by `steps` steps of dt (wave speed c) on `stream`.  use_graph: the
 * step is captured once in a HIP graph (re-captured when c or dt change) and
 * replayed. */
int fc2d_batch_run_ff(fc2d_batch* batch, double c, double dt, int steps, int use_graph, hipStream_t stream);
int fc2d_batch_destroy(fc2d_batch* batch);

/* ---- Learned foot-of-normal seed: training data, training, inference ----
 * Not part of the paper's method; see FC2D_SEED_MLP.  For a point Q =
 * rho (cos phi, sin phi) near the polar curve r(t) and strip width w = C k1 the
 * network's inputs are (R_k = r^(k)(phi)):
 *   f0 = (rho - R_0)/w, f1 = R_0 - 1, f2 = R_1/R_0, f3..f6 = R_k/(R_0 S_k) for
 *   k = 2..5 with S = (2, 10, 60, 400), f7 = f0 f2 / (1 + f2^2);
 * its outputs are 100 (delta/w - f7/R_0, eta/w - f0/sqrt(1 + f2^2)), delta =
 * theta^Q - phi, i.e. what one Newton step from phi leaves out, and the seed is
 * theta^(0) = phi + w (f7/R_0 + out_0/100). */

/* Training pairs from the method's own foot solves.  curves: device
 * [ncurves][1 + 2 nmodes] polar coefficients (nmodes <= 16, r > 0); sample k
 * is the point q(theta[k]) + eta[k] n(theta[k]) of curve cidx[k] (device
 * arrays of n), whose foot is solved from the seed phi by the bracketed Newton.
 * Outputs (device): X [n][8] float, Y [n][2] float (features and targets for
 * width w), foot [n][2] float64 (theta^Q in [0, 2 pi), eta_Q; may be NULL),
 * iters [n] (Newton steps; -1 where the solve failed or cidx[k] is not in
 * [0, ncurves), whose other outputs are then left untouched; may be NULL). */
int fc2d_mlp_make_data(const double* curves, int ncurves, int nmodes, const int32_t* cidx,
                       const double* theta, const double* eta, int64_t n, double width,
                       float* X, float* Y, double* foot, int32_t* iters, hipStream_t stream);

/* Network outputs out [n][2] for inputs X [n][8] (device float). */
int fc2d_mlp_forward(const float* weights, const float* X, int64_t n, float* out, hipStream_t stream);

/* Loss 0.5 mean |net(X) - Y|^2 over the n samples and its gradient with
 * respect to the weights (device float: grad [FC2D_MLP_NW], loss [1]; either
 * may be NULL).  Partial sums per 64 samples are added in a fixed order, so
 * results are reproducible.  Synchronises the stream (releases work space). */
int fc2d_mlp_loss_grad(const float* weights, const float* X, const float* Y, int64_t n,
                       float* grad, float* loss, hipStream_t stream);

/* `steps` Adam steps (beta 0.9 / 0.999, eps 1e-8) on minibatches of `batch`
 * samples of (X, Y) (n samples, device).  Step s uses Adam step number
 * t = t0 + s + 1 and learning rate lr_min + (lr0 - lr_min)(1 + cos(pi t / t_total))/2
 * (t capped at t_total); its samples are positions t-1 batch ... of an endless
 * sequence that visits every sample once per pass, in an order that changes
 * from pass to pass.  weights, adam_m, adam_v: device float [FC2D_MLP_NW],
 * updated in place (moments start at zero).  loss_hist (device float [steps],
 * may be NULL) receives each step's minibatch loss.  Synchronises the stream. */
int fc2d_mlp_train(float* weights, float* adam_m, float* adam_v, const float* X, const float* Y, int64_t n,
                   int batch, int steps, int64_t t0, float lr0, float lr_min, int64_t t_total,
                   float* loss_hist, hipStream_t stream);

const char* fc2d_strerror(int status);
const char* fc2d_last_error(void);
int fc2d_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FC2D_H */
