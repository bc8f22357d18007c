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
int pois_axpbz(double a, const double* x, double b, const double* z, int n, double* y, hipStream_t s);
// Levels of the double-layer sums: level L (0 <= L < kPoisLevels) holds 2^L nb
// equispaced nodes at offset nb (2^L - 1) of the concatenated node arrays.
constexpr int kPoisLevels = 6;
// phi (nfc rows of nb) -> phif (nfc rows of 2^(kPoisLevels - 1) nb, the finest
// level, by the Dirichlet kernel) -> node records of every level: (x, y) and
// per field (phi y', phi x'), 2 + 2 nfc doubles each; geo: (x, y, x', y') per
// node; wtab: scratch of (2^(kPoisLevels - 1) - 1) nb doubles
int pois_records(const double* phi, int nb, int nfc, const double* geo, double* wtab, double* phif, double* rec,
                 hipStream_t s);
// v at the IN points of nfc fields (u = u_p + v, 0 elsewhere; up and u hold
// the fields nx ny apart); points next to Gamma listed in cand.  bl:
// kPoisLevels lists of cap entries (cap >= IN points), bcnt their counts (zero
// on entry), both scratch; sag: bound on how far an arc between two nodes
// leaves its chord
int pois_dl_grid(const fc2d_grid* g, int nfc, const int8_t* cls, const double* up, const double* rec, int nb,
                 double dsmax, const double* seg, const double* sinv, double sag, double* u, int32_t* bl,
                 int64_t cap, int* bcnt, int32_t* cand, int* ncand, hipStream_t s);
// the listed points within h/2 of Gamma, nfc fields (ghom: nfc rows of nb).
// Scratch for up to capn such points: nidx [capn], nw [capn M], nv0 [capn nfc],
// samp [capn (M - 1)] point pairs, sval [capn (M - 1) nfc]; ncnt[0] counts them
// and ncnt[1] those beyond capn (both zero on entry).
int pois_dl_near(int M, int nfc, const int32_t* cand, const int* ncand, int64_t cap, const CurveC& cv,
                 const BndView& bd, int maxit, const fc2d_grid* g, const double* up, const double* ghom, int nb,
                 const double* rec, int capn, int32_t* nidx, double* nw, double* nv0, double* samp, double* sval,
                 int* ncnt, double* u, int* nfail, hipStream_t s);

}  // namespace fc2d
