// Internal interface of the full Poisson solve (Sec. 4.1): launchers of
// kernels_poisson.hip, used by poisson.cpp.  Not part of the C ABI.
#pragma once

#include "internal.h"

namespace fc2d {

// Fields are handled in chunks of nfc = 1, 2 or 4 (kPoisChunk at most) that
// share the GMRES passes over the Nystrom matrix and the geometry work of the
// double-layer sums.
constexpr int kPoisChunk = 4;

// ---- full Poisson solve (kernels_poisson.hip); qd: (x, y, x', y', x'', y'') per node
int pois_mean(const fc2d_grid* g, const double* spec, double* mean, hipStream_t s);
int pois_add_quad(const fc2d_grid* g, const double* mean, double* up, hipStream_t s);
int pois_ghom(int M, const fc2d_grid* g, const double* up, const double* qd, int nb, const double* gv,
              double* ghom, hipStream_t s);
// node data on the device: qc (x, y, x', y', x'', y'') at the nb nodes, geo
// (x, y, x', y') at the nodes of every level (t = 2 pi q / (2^(kPoisLevels-1) nb),
// q the node's finest-level index, so shared nodes agree bit for bit)
// and the chords of the nb-node polygon: seg (x, y, dx, dy) per node, sinv 1 / |chord|^2
int pois_nodes(const CurveC& cv, int nb, double* qc, double* geo, double* seg, double* sinv, hipStream_t s);
// per-point classes (nx * ny bytes) from the plan's row runs
int pois_classes(const int32_t* run_ptr, const int32_t* run, int nx, int ny, int8_t* cls, hipStream_t s);
int pois_nystrom(const double* qd, int nb, double* A, hipStream_t s);
// GMRES building blocks for nfc fields at once (nfc = 1, 2 or 4; the field
// index runs over the given strides).
// y_f = A x_f, A column-major n x n read once; y holds the fields n apart;
// part: scratch of pois_matvec_splits(n) nfc n doubles
int pois_matvec_splits(int n);
int pois_matvec(const double* A, const double* x, int64_t xs, int n, int nfc, double* part, double* y,
                hipStream_t s);
// out_f[b] = <V_f,b, w_f>, b < nv (V_f,b at V + f vs + b n)
int pois_dots(const double* V, int64_t vs, int nv, const double* w, int64_t ws, int n, int nfc, double* out,
              int64_t os, hipStream_t s);
// w_f -= sum_b c_f[b] V_f,b
int pois_sub(const double* V, int64_t vs, int nv, const double* c, int64_t cs, int n, int nfc, double* w,
             int64_t ws, hipStream_t s);
// y_f = a[f] x_f (a: nfc host values)
int pois_scale(const double* a, const double* x, int64_t xs, int n, int nfc, double* y, int64_t ys,
               hipStream_t s);
// y_f = x_f / sqrt(hn[f hs]) (zeros where that is not positive), hn on the device
int pois_normalize(const double* x, int64_t xs, int n, int nfc, const double* hn, int64_t hs, double* y, int64_t ys,
                   hipStream_t s);
int pois_axpbz(double a, const double* x, double b, const double* z, int n, double* y, hipStream_t s);
// Levels of the double-layer sums: level L (0 <= L < kPoisLevels) holds 2^L nb
// equispaced nodes at offset nb (2^L - 1) of the concatenated node arrays.
constexpr int kPoisLevels = 8;
// phi (nfc rows of nb) -> phif (nfc rows of 2^(kPoisLevels - 1) nb, the finest
// level, by the Dirichlet kernel) -> node records of every level: (x, y) and
// per field (phi y', phi x'), 2 + 2 nfc doubles each; geo: (x, y, x', y') per
// node; wtab: scratch of (2^(kPoisLevels - 1) - 1) nb doubles
int pois_records(const double* phi, int nb, int nfc, const double* geo, double* wtab, double* phif, double* rec,
                 hipStream_t s);
// v at the IN points of one chunk of nfc fields: u = u_p + v there, 0
// elsewhere (up and u hold the fields nx ny apart).  Every point first sums
// the nb nodes; points within 7 node spacings of Gamma sum the level their
// distance needs; points within h/2 of Gamma take v from the near-boundary
// interpolation, whose samples sum the levels their distances need.
struct PoisDl {
    const fc2d_grid* g;
    int nfc, M, nb, maxit;
    const int8_t* cls;                 // [nx ny] point classes
    const double* up;                  // [nfc][nx ny] particular solution
    const double* rec;                 // node records of every level (pois_records)
    const double* ghom;                // [nfc][nb] boundary data of the harmonic part
    double dsmax;                      // largest spacing of the nb nodes
    const double* seg;                 // nb-node polygon chords and their inverse squared lengths
    const double* sinv;
    double sag;                        // bound on how far an arc between two nodes leaves its chord
    CurveC cv;
    BndView bd;                        // plan boundary samples (foot seeds)
    int64_t cap;                       // >= IN points
    int32_t* bl;                       // [kPoisLevels][cap] band lists
    int32_t* cand;                     // [cap] candidates
    int capb;                          // band entries per level whose nodes are split over blocks
    double* bpart;                     // [16][capb][nfc] chunk sums of those levels
    int capn;                          // near points at most
    int32_t* nidx;                     // [capn]
    double* nw;                        // [capn M]
    double* nv0;                       // [capn nfc]
    double* samp;                      // [capn (M - 1)] point pairs
    int32_t* sl;                       // [kPoisLevels][capn (M - 1)] sample lists
    int8_t* slev;                      // [capn (M - 1)] sample levels
    double* sval;                      // [16][capn (M - 1)][nfc] chunk sums of the samples
    int* cnt;                          // kPoisCounters counters, zero on entry
    double* u;                         // [nfc][nx ny]
};
// counters: [0] candidates, [1] failed feet, [2 + L] band entries of level L,
// [2 + kPoisLevels] near points, [3 + kPoisLevels] entries beyond capn or
// capb, [4 + kPoisLevels + L] samples of level L
constexpr int kPoisCounters = 4 + 2 * kPoisLevels;
int pois_dl_eval(const PoisDl& a, hipStream_t s);

}  // namespace fc2d
