// Device part of the Geometrical Setup (Sec. 3.5 steps 3-4): classification of
// the Cartesian grid H and the foot of the normal of every point near Gamma.
//
//  k_near_scatter: proximity of Sec. 3.3 reduced to its normal index -- every
//    boundary sample q_p scatters (distance^2, p) into the grid points within
//    r_out of it with a 64-bit atomicMin, so each point near Gamma learns its
//    nearest sample p (ties to the smaller p).
//  k_classify: one thread per grid point.  Parity of the crossings of its grid
//    column with the boundary polygon gives IN / FAR; points near Gamma (outside
//    within r_out, inside within r_in of their nearest sample) solve for the
//    foot (theta^Q, eta_Q) from the seed p and are reclassified by eta:
//    IN (eta <= 0), STRIP (0 < eta <= C k1), FAR.  STRIP points append a record.
//  k_radial_band / k_seed_polar (polar curves): rho - r(phi) decides IN / FAR
//    away from Gamma and selects the candidates near it, which are compacted
//    into a list and solved from the seed phi = atan2(y, x), one thread each.
//  k_row_stats / k_row_write / k_strip_map / k_strip_gather / k_strip_wmax: the
//    plan's lists from the classes and the STRIP records -- per-row runs of
//    equal class, the row pass's pair classes, the STRIP list in row-major order
//    and in order of theta.
//  k_star_scan: red-star candidates of the matching stencils (Sec. 3.2): the
//    runs of IN points along each candidate's grid line and the crossings of
//    the line with Gamma that bound them (where eta changes sign).
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include "internal.h"
#include "seed_dev.h"

namespace fc2d {

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_near_scatter(ClassifyArgs a, uint64_t* near) {
    const int p = blockIdx.x;
    const double qx = a.bx[p], qy = a.by[p];
    const double r2 = a.r_out * a.r_out;
    int i0 = (int)floor((qx - a.r_out - a.x0) / a.h);
    int i1 = (int)ceil((qx + a.r_out - a.x0) / a.h);
    int j0 = (int)floor((qy - a.r_out - a.y0) / a.h);
    int j1 = (int)ceil((qy + a.r_out - a.y0) / a.h);
    i0 = max(i0, 0);
    j0 = max(j0, 0);
    i1 = min(i1, a.nx - 1);
    j1 = min(j1, a.ny - 1);
    if (i1 < i0 || j1 < j0) return;
    const int wj = j1 - j0 + 1;
    const int n = (i1 - i0 + 1) * wj;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const int i = i0 + k / wj;
        const int j = j0 + k % wj;
        const double dx = (a.x0 + i * a.h) - qx;
        const double dy = (a.y0 + j * a.h) - qy;
        const double d2 = dx * dx + dy * dy;
        if (d2 <= r2) {
            const uint64_t key = ((uint64_t)__float_as_uint((float)d2) << 32) | (uint32_t)p;
            atomicMin((unsigned long long*)&near[(int64_t)i * a.ny + j], (unsigned long long)key);
        }
    }
}

template <int M>
__global__ __launch_bounds__(256) void k_classify(ClassifyArgs a, const uint64_t* near, int8_t* cls,
                                                  StripRec* rec, int64_t cap, int* counters) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)a.nx * a.ny) return;
    const int i = (int)(idx / a.ny);
    const int j = (int)(idx - (int64_t)i * a.ny);
    const double X = a.x0 + i * a.h;
    const double Y = a.y0 + j * a.h;
    // crossing parity along the column x = x_i (crossings strictly below y_j)
    int below = 0;
    for (int k = a.col_ptr[i]; k < a.col_ptr[i + 1]; ++k) below += (a.col_y[k] < Y) ? 1 : 0;
    const bool inside = (below & 1) != 0;
    int8_t c = inside ? 1 : 0;
    const uint64_t key = near[idx];
    if (key != ~0ull) {
        const float d2 = __uint_as_float((uint32_t)(key >> 32));
        const int p = (int)(key & 0xffffffffu);
        const bool band = inside ? ((double)d2 <= a.r_in * a.r_in) : true;
        if (band) {
            BndView bd{a.bx, a.by, a.bnx, a.bny, a.B, a.k2};
            double th = 0.0, eta = 0.0;
            int it = 0;
            const int stt = foot_solve<M>(a.curve, bd, X, Y, p, a.maxit, &th, &eta, &it);
            atomicAdd(&counters[3], 1);
            store_solved(idx, X, Y, stt, th, eta, it, p, a.width, cls, rec, cap, counters);
            return;
        }
    }
    cls[idx] = c;
}

// r(phi) of a polar curve at the point (X, Y) = rho (cos phi, sin phi), with
// cos m phi, sin m phi by the angle-addition recurrence from X / rho, Y / rho
__device__ inline double polar_radius_at(const CurveC& cv, double X, double Y, double rho) {
    const double c1 = X / rho, s1 = Y / rho;
    double cm = 1.0, sm = 0.0, r = cv.a[0];
    for (int m = 1; m <= cv.nmodes; ++m) {
        const double cn = cm * c1 - sm * s1;
        sm = sm * c1 + cm * s1;
        cm = cn;
        r += cv.a[2 * m - 1] * cm + cv.a[2 * m] * sm;
    }
    return r;
}

__global__ __launch_bounds__(256) void k_radial_band(SeedArgs a, int8_t* cls, int32_t* cand, int64_t cap,
                                                     int* counters) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)a.nx * a.ny) return;
    const int i = (int)(idx / a.ny);
    const int j = (int)(idx - (int64_t)i * a.ny);
    const double X = a.x0 + i * a.h;
    const double Y = a.y0 + j * a.h;
    const double rho = sqrt(X * X + Y * Y);
    int8_t c;
    if (rho == 0.0) {
        c = 1;   // the origin is inside a polar domain
    } else {
        const double dr = rho - polar_radius_at(a.curve, X, Y, rho);
        if (dr >= a.band_lo && dr <= a.band_hi) {
            const int slot = atomicAdd(&counters[3], 1);
            if (slot < cap) cand[slot] = (int32_t)idx;
            c = 3;   // pending: written by the seed kernel
        } else {
            c = dr < 0 ? 1 : 0;
        }
    }
    cls[idx] = c;
}

__global__ __launch_bounds__(256) void k_seed_polar(SeedArgs a, const int32_t* __restrict__ cand, int64_t ncand,
                                                    int8_t* cls, StripRec* rec, int64_t cap, int* counters) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncand) return;
    const int64_t idx = cand[k];
    const int i = (int)(idx / a.ny);
    const int j = (int)(idx - (int64_t)i * a.ny);
    const double X = a.x0 + i * a.h;
    const double Y = a.y0 + j * a.h;
    double th = 0.0, eta = 0.0;
    int it = 0;
    const int st = foot_from_seed(a.curve, X, Y, atan2(Y, X), 2.0 * a.k2, a.maxit, &th, &eta, &it);
    store_solved(idx, X, Y, st, th, eta, it, nearest_sample(th, a.k2, a.B), a.width, cls, rec, cap, counters);
}

__global__ void k_zero_int(int* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

int launch_classify(const ClassifyArgs& a, int8_t* d_cls, StripRec* d_rec, int64_t cap, uint64_t* d_near,
                    int* d_counters, hipStream_t s) {
    const int64_t npts = (int64_t)a.nx * a.ny;
    k_zero_int<<<1, 64, 0, s>>>(d_counters, 8);
    k_fill_u64<<<(unsigned)((npts + 255) / 256), 256, 0, s>>>(d_near, npts, ~0ull);
    k_near_scatter<<<a.B, 256, 0, s>>>(a, d_near);
    const unsigned nb = (unsigned)((npts + 255) / 256);
    switch (a.M) {
        case 4: k_classify<4><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 5: k_classify<5><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 6: k_classify<6><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 7: k_classify<7><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 8: k_classify<8><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 13: k_classify<13><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 15: k_classify<15><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("classification launch: ") + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    trace_point("k_classify", s);
    return FC2D_OK;
}

static int launch_status(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    return FC2D_OK;
}

int launch_radial_band(const SeedArgs& a, int8_t* d_cls, int32_t* d_cand, int64_t cap, int* d_counters,
                       hipStream_t s) {
    const int64_t npts = (int64_t)a.nx * a.ny;
    k_zero_int<<<1, 64, 0, s>>>(d_counters, 8);
    k_radial_band<<<(unsigned)((npts + 255) / 256), 256, 0, s>>>(a, d_cls, d_cand, cap, d_counters);
    if (int st = launch_status("radial band launch")) return st;
    trace_point("k_radial_band", s);
    return FC2D_OK;
}

int launch_seed_polar(const SeedArgs& a, const int32_t* d_cand, int64_t ncand, int8_t* d_cls, StripRec* d_rec,
                      int64_t cap, int* d_counters, hipStream_t s) {
    if (ncand <= 0) return FC2D_OK;
    k_seed_polar<<<(unsigned)((ncand + 255) / 256), 256, 0, s>>>(a, d_cand, ncand, d_cls, d_rec, cap, d_counters);
    if (int st = launch_status("polar seed launch")) return st;
    trace_point("k_seed_polar", s);
    return FC2D_OK;
}

// ---------------------------------------------------------------------------
// plan lists
// ---------------------------------------------------------------------------
constexpr int kRowThreads = 256;

// exclusive prefix sum of v over the block (kRowThreads threads); *total gets the sum
__device__ inline int block_excl_scan(int v, int* sh, int* total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kRowThreads; off <<= 1) {
        const int add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const int incl = sh[t];
    *total = sh[kRowThreads - 1];
    __syncthreads();
    return incl - v;
}

// per row i: runs of equal class, STRIP, IN and FAR counts -> stats[i][4]
__global__ __launch_bounds__(kRowThreads) void k_row_stats(const int8_t* __restrict__ cls, int ny, int32_t* stats) {
    __shared__ int sh[kRowThreads];
    const int8_t* row = cls + (int64_t)blockIdx.x * ny;
    const int chunk = (ny + kRowThreads - 1) / kRowThreads;
    const int j0 = threadIdx.x * chunk, j1 = min(ny, j0 + chunk);
    int cnt[4] = {0, 0, 0, 0};
    for (int j = j0; j < j1; ++j) {
        const int c = row[j];
        cnt[0] += (j == 0 || c != row[j - 1]) ? 1 : 0;
        cnt[1] += c == 2;
        cnt[2] += c == 1;
        cnt[3] += c == 0;
    }
    for (int k = 0; k < 4; ++k) {
        int tot;
        (void)block_excl_scan(cnt[k], sh, &tot);
        if (threadIdx.x == 0) stats[4 * blockIdx.x + k] = tot;
    }
}

__global__ void k_strip_map(const StripRec* __restrict__ rec, int64_t S, int32_t* map) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < S) map[rec[k].idx] = (int32_t)k;
}

// per row i: the runs (start, end, class) from run_ptr[i], the row-major STRIP
// list from strip_off[i], and (E > 0) the row's pair classes in the masked row
// pass's thread order: output o = t E + k holds pair t + (k / R) P + (k % R) (L / R)
// with L = ny / 2 pairs, P = L / E threads, R the first-stage radix
__global__ __launch_bounds__(kRowThreads) void k_row_write(const int8_t* __restrict__ cls, int ny,
                                                           const int32_t* __restrict__ run_ptr, int32_t* runs,
                                                           const int32_t* __restrict__ strip_off,
                                                           const int32_t* __restrict__ map,
                                                           const StripRec* __restrict__ rec, int32_t* rm_idx,
                                                           int32_t* rm_seed, double* rm_th, double* rm_eta,
                                                           uint8_t* cls2, int E, int R) {
    __shared__ int sh[kRowThreads];
    const int i = blockIdx.x;
    const int8_t* row = cls + (int64_t)i * ny;
    const int chunk = (ny + kRowThreads - 1) / kRowThreads;
    const int j0 = threadIdx.x * chunk, j1 = min(ny, j0 + chunk);
    int nr = 0, ns = 0;
    for (int j = j0; j < j1; ++j) {
        const int c = row[j];
        nr += (j == 0 || c != row[j - 1]) ? 1 : 0;
        ns += c == 2;
    }
    int tot;
    int r = run_ptr[i] + block_excl_scan(nr, sh, &tot);
    int q = strip_off[i] + block_excl_scan(ns, sh, &tot);
    for (int j = j0; j < j1; ++j) {
        const int c = row[j];
        if (j == 0 || c != row[j - 1]) {
            runs[3 * r] = j;
            runs[3 * r + 2] = c;
            if (j > 0) runs[3 * (r - 1) + 1] = j;   // end of the previous run
            ++r;
        }
        if (c == 2) {
            const int32_t idx = (int32_t)((int64_t)i * ny + j);
            const StripRec sr = rec[map[idx]];
            rm_idx[q] = idx;
            rm_seed[q] = sr.seed;
            rm_th[q] = sr.theta;
            rm_eta[q] = sr.eta;
            ++q;
        }
    }
    if (threadIdx.x == 0) runs[3 * (run_ptr[i + 1] - 1) + 1] = ny;
    if (E > 0) {
        const int L = ny / 2, P = L / E;
        uint8_t* out = cls2 + (int64_t)i * L;
        for (int o = threadIdx.x; o < L; o += kRowThreads) {
            const int t = o / E, k = o - t * E;
            const int n = t + (k / R) * P + (k % R) * (L / R);
            out[o] = (uint8_t)(row[2 * n] | (row[2 * n + 1] << 2));
        }
    }
}

__global__ void k_iota(int32_t* v, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) v[k] = (int32_t)k;
}

__global__ void k_strip_gather(const int32_t* __restrict__ pos, const int32_t* __restrict__ rm_idx,
                               const double* __restrict__ rm_eta, int32_t* sidx, double* seta, int64_t S) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S) return;
    const int32_t p = pos[k];
    sidx[k] = rm_idx[p];
    seta[k] = rm_eta[p];
}

// widest window of normals p0(first) - kl ... p0(last) - kl + M under a block of
// 512 theta-ordered STRIP points (p0 as the strip kernel forms it)
__global__ void k_strip_wmax(const double* __restrict__ th, int64_t S, double k2, int M, int* wmax) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k0 = b * 512;
    if (k0 >= S) return;
    const int64_t k1 = min(S, k0 + 512) - 1;
    auto p0 = [&](double t) { return (M % 2 == 0) ? (int)floor(t / k2) : (int)rint(t / k2); };
    atomicMax(wmax, p0(th[k1]) - p0(th[k0]) + M + 1);
}

int plan_device_lists(fc2d_plan* pl, const StripRec* d_rec, int64_t S, hipStream_t s) {
    const fc2d_grid& g = pl->grid;
    const int nx = g.nx, ny = g.ny;
    const int64_t npts = (int64_t)nx * ny;
    int32_t *d_stats = nullptr, *d_off = nullptr, *d_map = nullptr, *d_pos = nullptr, *d_pos2 = nullptr;
    int* d_wmax = nullptr;
    void* d_tmp = nullptr;
    int st = FC2D_OK;
    auto fail = [&](hipError_t e, const char* what) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FC2D_E_NOMEM : FC2D_E_HIP;
    };
    do {
        hipError_t e;
        // temporaries come from the library's stream-ordered pool (no device
        // allocator call once the pool holds enough); the plan's arrays are its own
        if ((st = ws_alloc((size_t)nx * 4 * sizeof(int32_t), s, (void**)&d_stats))) break;
        k_row_stats<<<nx, kRowThreads, 0, s>>>(pl->d_cls, ny, d_stats);
        if ((st = launch_status("row statistics launch"))) break;
        std::vector<int32_t> stats((size_t)nx * 4);
        if ((e = hipMemcpyAsync(stats.data(), d_stats, stats.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess) {
            st = fail(e, "row statistics");
            break;
        }
        // offsets: run_ptr [nx + 1], then the row-major STRIP offsets [nx + 1]
        std::vector<int32_t> off(2 * ((size_t)nx + 1), 0);
        int64_t nruns = 0, nstrip = 0, nin = 0, nfar = 0;
        for (int i = 0; i < nx; ++i) {
            off[i] = (int32_t)nruns;
            off[nx + 1 + i] = (int32_t)nstrip;
            nruns += stats[4 * i];
            nstrip += stats[4 * i + 1];
            nin += stats[4 * i + 2];
            nfar += stats[4 * i + 3];
        }
        off[nx] = (int32_t)nruns;
        off[2 * nx + 1] = (int32_t)nstrip;
        if (nstrip != S) {
            set_error("plan lists: STRIP records do not match the classes");
            st = FC2D_E_HIP;
            break;
        }
        pl->nruns = (int)nruns;
        pl->n_in = nin;
        pl->n_far = nfar;
        pl->n_strip = S;
        const int Lh = ny / 2;
        const int E = (ny % 2 == 0) ? row_elems(Lh) : 0;
        int R = 16;
        if (E > 0)
            while (R > E || Lh % R != 0) R >>= 1;
        const size_t Sa = (size_t)std::max<int64_t>(S, 1);
        if ((st = ws_alloc(off.size() * sizeof(int32_t), s, (void**)&d_off)) ||
            (st = ws_alloc((size_t)npts * sizeof(int32_t), s, (void**)&d_map)) ||
            (st = ws_alloc(Sa * sizeof(int32_t), s, (void**)&d_pos)) ||
            (st = ws_alloc(Sa * sizeof(int32_t), s, (void**)&d_pos2)) ||
            (st = ws_alloc(sizeof(int), s, (void**)&d_wmax)))
            break;
        if ((e = hipMalloc((void**)&pl->d_run_ptr, ((size_t)nx + 1) * sizeof(int32_t))) != hipSuccess ||
            (e = hipMalloc((void**)&pl->d_run, (size_t)nruns * 3 * sizeof(int32_t))) != hipSuccess ||
            (e = hipMalloc((void**)&pl->d_rm_idx, Sa * sizeof(int32_t))) != hipSuccess ||
            (e = hipMalloc((void**)&pl->d_rm_seed, Sa * sizeof(int32_t))) != hipSuccess ||
            (e = hipMalloc((void**)&pl->d_rm_th, Sa * sizeof(double))) != hipSuccess ||
            (e = hipMalloc((void**)&pl->d_rm_eta, Sa * sizeof(double))) != hipSuccess ||
            (e = hipMalloc((void**)&pl->d_sidx, Sa * sizeof(int32_t))) != hipSuccess ||
            (e = hipMalloc((void**)&pl->d_sth, Sa * sizeof(double))) != hipSuccess ||
            (e = hipMalloc((void**)&pl->d_seta, Sa * sizeof(double))) != hipSuccess ||
            (E > 0 && (e = hipMalloc((void**)&pl->d_cls2, (size_t)nx * Lh)) != hipSuccess)) {
            st = fail(e, "plan lists");
            break;
        }
        if ((e = hipMemcpyAsync(d_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, s)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(pl->d_run_ptr, d_off, ((size_t)nx + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                s)) != hipSuccess) {
            st = fail(e, "plan lists");
            break;
        }
        if (S > 0) {
            k_strip_map<<<(unsigned)((S + 255) / 256), 256, 0, s>>>(d_rec, S, d_map);
            if ((st = launch_status("STRIP map launch"))) break;
        }
        k_row_write<<<nx, kRowThreads, 0, s>>>(pl->d_cls, ny, d_off, pl->d_run, d_off + nx + 1, d_map, d_rec,
                                               pl->d_rm_idx, pl->d_rm_seed, pl->d_rm_th, pl->d_rm_eta, pl->d_cls2,
                                               E, R);
        if ((st = launch_status("row lists launch"))) break;
        int wmax = 0;
        if (S > 0) {
            // theta order, stable: equal theta keep their row-major order
            k_iota<<<(unsigned)((S + 255) / 256), 256, 0, s>>>(d_pos, S);
            if ((st = launch_status("STRIP order launch"))) break;
            size_t tmp_bytes = 0;
            if ((e = rocprim::radix_sort_pairs(nullptr, tmp_bytes, pl->d_rm_th, pl->d_sth, d_pos, d_pos2,
                                               (unsigned)S, 0, 64, s)) != hipSuccess) {
                st = fail(e, "STRIP sort by theta");
                break;
            }
            if ((st = ws_alloc(tmp_bytes, s, &d_tmp))) break;
            if ((e = rocprim::radix_sort_pairs(d_tmp, tmp_bytes, pl->d_rm_th, pl->d_sth, d_pos, d_pos2,
                                               (unsigned)S, 0, 64, s)) != hipSuccess) {
                st = fail(e, "STRIP sort by theta");
                break;
            }
            k_strip_gather<<<(unsigned)((S + 255) / 256), 256, 0, s>>>(d_pos2, pl->d_rm_idx, pl->d_rm_eta,
                                                                       pl->d_sidx, pl->d_seta, S);
            if ((st = launch_status("STRIP gather launch"))) break;
            k_zero_int<<<1, 64, 0, s>>>(d_wmax, 1);
            const int64_t nblk = (S + 511) / 512;
            k_strip_wmax<<<(unsigned)((nblk + 255) / 256), 256, 0, s>>>(pl->d_sth, S, pl->k2, pl->M, d_wmax);
            if ((st = launch_status("strip window launch"))) break;
            if ((e = hipMemcpyAsync(&wmax, d_wmax, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) {
                st = fail(e, "strip window");
                break;
            }
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) { st = fail(e, "plan lists"); break; }
        pl->strip_wmax = wmax;
        trace_point("plan_lists", s);
    } while (0);
    void* tmp[] = {d_stats, d_off, d_map, d_pos, d_pos2, d_wmax, d_tmp};
    for (void* q : tmp)
        if (q) (void)ws_free(q, s);
    return st;
}

// ---------------------------------------------------------------------------
// red stars of the matching stencils
// ---------------------------------------------------------------------------
// nearest boundary sample to (X, Y) by discrete descent from p
__device__ inline int nearest_descent(const StarArgs& a, double X, double Y, int p) {
    auto d2 = [&](int q) {
        const int r = imod(q, a.B);
        const double dx = a.bx[r] - X, dy = a.by[r] - Y;
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
    return imod(p, a.B);
}

// crossing of {line = a_line, b between b_in (eta <= 0) and b_out} with Gamma,
// where eta changes sign: false position with the Illinois modification (a
// retained end's value is halved, so both ends move) while it shrinks the
// bracket, then bisection until the bracket no longer changes (its fixed point:
// adjacent doubles or one value).  false when a foot solve fails
template <int M>
__device__ bool crossing(const StarArgs& a, const BndView& bd, bool vertical, double a_line, double b_in, double b_out,
                         int seed, double* out) {
    // the first foot is seeded from the nearest boundary sample (T(tau), as in the
    // classification); later ones by Newton from the previous foot parameter,
    // the points moving along the line by at most a few grid steps
    double th = 0.0;
    bool have_th = false;
    auto eta_at = [&](double b, double* e) {
        const double X = vertical ? a_line : b;
        const double Y = vertical ? b : a_line;
        int its;
        if (have_th && foot_from_seed(a.curve, X, Y, th, 2.0 * a.k2, a.maxit, &th, e, &its) == FOOT_OK) return true;
        seed = nearest_descent(a, X, Y, seed);
        have_th = foot_solve<M>(a.curve, bd, X, Y, seed, a.maxit, &th, e, &its) == FOOT_OK;
        return have_th;
    };
    // lo: the end with eta <= 0, hi: eta > 0 (either may be the larger coordinate)
    double lo = b_in, hi = b_out, flo, fhi;
    if (!eta_at(lo, &flo) || !eta_at(hi, &fhi)) return false;
    if (flo <= 0 && fhi > 0) {
        int kept = 0;   // -1: lo moved last (hi kept), 1: hi moved last
        for (int it = 0; it < 40; ++it) {
            const double x = (lo * fhi - hi * flo) / (fhi - flo);
            if (!((x - lo) * (x - hi) < 0.0)) break;   // not strictly inside the bracket
            double fx;
            if (!eta_at(x, &fx)) return false;
            if (fx <= 0) {
                lo = x;
                flo = fx;
                if (kept == -1) fhi *= 0.5;
                kept = -1;
            } else {
                hi = x;
                fhi = fx;
                if (kept == 1) flo *= 0.5;
                kept = 1;
            }
            if (fabs(hi - lo) <= 8.0 * 0x1p-52 * fmax(fabs(lo), fabs(hi))) break;
        }
        // false position nears the root from one side (the end that moved last):
        // step away from that end by 4, 32, 256 ... ulps until eta changes sign,
        // so the bisection below starts from a bracket a few ulps wide
        if (kept != 0) {
            const bool near_lo = kept == -1;
            const double sgn = hi > lo ? 1.0 : -1.0;   // direction from lo towards hi
            double d = 4.0 * 0x1p-52 * fmax(fabs(lo), fabs(hi));
            for (int it = 0; it < 24 && fabs(hi - lo) > d; ++it) {
                const double x = near_lo ? lo + sgn * d : hi - sgn * d;
                double fx;
                if (!eta_at(x, &fx)) return false;
                if (fx <= 0) lo = x;
                else hi = x;
                if (near_lo == (fx > 0)) break;   // the sign changes within d of that end
                d *= 8.0;
            }
        }
    }
    for (int it = 0; it < 64; ++it) {
        const double mid = 0.5 * (lo + hi);
        double eta;
        if (!eta_at(mid, &eta)) return false;
        const double lo0 = lo, hi0 = hi;
        if (eta <= 0) lo = mid;
        else hi = mid;
        if (lo == lo0 && hi == hi0) break;   // fixed point: later halvings change nothing
    }
    *out = 0.5 * (lo + hi);
    return true;
}

// two lanes per candidate: lane 2c scans below the star and locates the
// square there, lane 2c + 1 above it
template <int M>
__global__ __launch_bounds__(64) void k_star_scan(StarArgs a, const int8_t* __restrict__ cls,
                                                  const StarQ* __restrict__ q, StarR* out, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * n) return;
    const int c = k >> 1, up = k & 1;
    const StarQ sq = q[c];
    StarR* r = out + c;
    int cnt = 0, flag = 0;
    double sqv = 0.0;
    if (!sq.skip) {
        const bool vert = sq.vertical != 0;
        const int nline = vert ? a.nx : a.ny, nb = vert ? a.ny : a.nx;
        auto in_at = [&](int j) -> bool {
            if (j < 0 || j >= nb || sq.line < 0 || sq.line >= nline) return false;
            return (vert ? cls[(int64_t)sq.line * a.ny + j] : cls[(int64_t)j * a.ny + sq.line]) == 1;
        };
        // below: jb, jb - 1, ... down to jb - M; above: jb + 1, ... up to jb + 1 + M
        const int dir = up ? 1 : -1, j0 = up ? sq.jb + 1 : sq.jb;
        int j = j0;
        while (cnt <= M && in_at(j)) {
            ++cnt;
            j += dir;
        }
        if (!a.io && cnt <= M) {   // the run ends within reach: its crossing with Gamma
            const BndView bd{a.bx, a.by, a.bnx, a.bny, a.B, a.k2};
            const double b0 = vert ? a.y0 : a.x0;
            const double b_in = cnt == 0 ? sq.bstar : b0 + (j - dir) * a.h;
            flag = crossing<M>(a, bd, vert, sq.a_line, b_in, b0 + j * a.h, sq.p, &sqv) ? 1 : 2;
        }
    }
    if (up) r->nhi = cnt;
    else r->nlo = cnt;
    r->side[up] = flag;
    r->sq[up] = sqv;
}

int launch_star_scan(const StarArgs& a, const int8_t* d_cls, const StarQ* d_q, StarR* d_r, int n, hipStream_t s) {
    if (n <= 0) return FC2D_OK;
    const unsigned nb = (unsigned)((2 * (int64_t)n + 63) / 64);
    switch (a.M) {
        case 4: k_star_scan<4><<<nb, 64, 0, s>>>(a, d_cls, d_q, d_r, n); break;
        case 5: k_star_scan<5><<<nb, 64, 0, s>>>(a, d_cls, d_q, d_r, n); break;
        case 6: k_star_scan<6><<<nb, 64, 0, s>>>(a, d_cls, d_q, d_r, n); break;
        case 7: k_star_scan<7><<<nb, 64, 0, s>>>(a, d_cls, d_q, d_r, n); break;
        case 8: k_star_scan<8><<<nb, 64, 0, s>>>(a, d_cls, d_q, d_r, n); break;
        case 13: k_star_scan<13><<<nb, 64, 0, s>>>(a, d_cls, d_q, d_r, n); break;
        case 15: k_star_scan<15><<<nb, 64, 0, s>>>(a, d_cls, d_q, d_r, n); break;
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
    if (int st = launch_status("red-star scan launch")) return st;
    trace_point("plan_star_scan", s);
    return FC2D_OK;
}

}  // namespace fc2d
