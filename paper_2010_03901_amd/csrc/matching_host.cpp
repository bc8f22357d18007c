// Host part of the matching stencils (Sec. 3.2, Fig. 3); see matching.h.
//
// Readings of the paper (the same rules the checking code follows):
//  * candidate red stars are the crossings at depth >= 0 of the inward normal
//    with grid lines x = x_i (|n_x| >= |n_y|) or y = y_j, in order of depth; with
//    boundary data a candidate closer to Gamma than 1/20 of the star spacing is
//    skipped (the point on Gamma is itself a node along the normal);
//  * a star's nodes are the IN points of the run of IN points holding it (at
//    most M + 1 grid steps away) and the crossings of its line with Gamma
//    bounding the run (squares); a square closer than h/2 to one of those IN
//    nodes is dropped;
//  * the red stars are the first candidates with at least M nodes (M - 1 of them
//    with boundary data, whose M-th node along the normal is the point on Gamma
//    at depth 0; M from interior data only), each with its M nearest nodes
//    (ties: grid node before square, then the lower one);
//  * weights are formed in x87 extended precision and stored as double-double.
#include <math.h>

#include <algorithm>

#include "matching.h"

namespace fc2d {

// red stars closer to Gamma than this fraction of the star spacing (h / |n| along
// the normal) are skipped
constexpr double kStarMinDepth = 0.05;

void place_stars(const MatchGeom& g, HostVec<StarQ>& q, HostVec<long double>& delta, HostVec<long double>& bstar) {
    const int M = g.M, B = g.B, ns = 2 * M;
    const double h = g.h;
    const size_t nst = (size_t)B * ns;
    q.resize(nst);
    delta.resize(nst);
    bstar.resize(nst);
#pragma omp parallel for
    for (int p = 0; p < B; ++p) {
        const double nx = g.bnx[p], ny = g.bny[p];
        const bool vertical = fabs(nx) >= fabs(ny);
        double na, nb, qa, qb, a0, b0;
        if (vertical) {
            na = nx; nb = ny; qa = g.bx[p]; qb = g.by[p]; a0 = g.x0; b0 = g.y0;
        } else {
            na = ny; nb = nx; qa = g.by[p]; qb = g.bx[p]; a0 = g.y0; b0 = g.x0;
        }
        const double u = (qa - a0) / h;
        int i_first, step;
        if (na > 0) { i_first = (int)floor(u); step = -1; }
        else { i_first = (int)ceil(u); step = 1; }
        for (int c = 0; c < ns; ++c) {
            const size_t k = (size_t)p * ns + c;
            StarQ& r = q[k];
            r.p = p;
            r.vertical = vertical ? 1 : 0;
            r.line = i_first + step * c;
            r.a_line = a0 + r.line * h;
            delta[k] = ((long double)qa - (long double)r.a_line) / (long double)na;
            bstar[k] = (long double)qb - delta[k] * (long double)nb;
            r.bstar = (double)bstar[k];
            r.jb = (int)floor((r.bstar - b0) / h);
            r.skip = (!g.interior_only && delta[k] < (long double)kStarMinDepth * h / fabs(na)) ? 1 : 0;
            r.pad = 0;
        }
    }
}

int select_matching(const MatchGeom& g, const StarQ* q, const StarR* res, const long double* delta,
                    const long double* bstar, HostVec<int32_t>& mref, HostVec<double>& mwv, HostVec<double>& mwn,
                    std::vector<double>& squares) {
    const int M = g.M, d = g.d, B = g.B, ns = 2 * M;
    const bool io = g.interior_only;
    const int nq = io ? d : d - 1;       // matching values interpolated along the normal
    const int nstar = io ? M : M - 1;    // red stars per normal
    const double h = g.h;
    // every entry of a normal whose stars all qualify is written below
    mref.clear(); mref.resize((size_t)B * M * M);
    mwv.clear(); mwv.resize((size_t)B * M * M * 2);
    mwn.clear(); mwn.resize((size_t)B * nq * M * 2);
    HostVec<double> sqxy((size_t)B * nstar * 2 * 2);   // at most two squares per star
    std::vector<int> nsq(B, 0);
    int bad = B;   // first normal with too few usable red stars
#pragma omp parallel for reduction(min : bad)
    for (int p = 0; p < B; ++p) {
        struct Node { bool sq; int j; double b; };
        Node lo[kMaxStencil + 2], hi[kMaxStencil + 2], chosen[kMaxStencil];
        long double deltas[kMaxStencil];
        int used = 0;
        for (int c = 0; c < ns && used < nstar; ++c) {
            const size_t k = (size_t)p * ns + c;
            const StarQ& r = q[k];
            const StarR& rr = res[k];
            if (r.skip) continue;
            const double b0 = r.vertical ? g.y0 : g.x0;
            bool has[2] = {(rr.side[0] & 1) != 0, (rr.side[1] & 1) != 0};
            for (int side = 0; side < 2; ++side) {
                if (!has[side]) continue;
                bool near_node = false;
                for (int t = 0; t < rr.nlo; ++t) near_node = near_node || fabs(rr.sq[side] - (b0 + (r.jb - t) * h)) < 0.5 * h;
                for (int t = 0; t < rr.nhi; ++t) near_node = near_node || fabs(rr.sq[side] - (b0 + (r.jb + 1 + t) * h)) < 0.5 * h;
                if (near_node) has[side] = false;
            }
            const int ncand = rr.nlo + rr.nhi + has[0] + has[1];
            if (ncand < M) continue;
            int nlo = 0, nhi = 0;
            for (int t = 0; t < rr.nlo && nlo < kMaxStencil + 1; ++t) lo[nlo++] = {false, r.jb - t, b0 + (r.jb - t) * h};
            if (has[0]) lo[nlo++] = {true, -1, rr.sq[0]};
            for (int t = 0; t < rr.nhi && nhi < kMaxStencil + 1; ++t) hi[nhi++] = {false, r.jb + 1 + t, b0 + (r.jb + 1 + t) * h};
            if (has[1]) hi[nhi++] = {true, -1, rr.sq[1]};
            int nch = 0, a = 0, b = 0;
            const double bs = r.bstar;
            while (nch < M) {
                if (a < nlo && b < nhi) {
                    const double dl = bs - lo[a].b, du = hi[b].b - bs;
                    if (dl < du || (dl == du && !(lo[a].sq && !hi[b].sq))) chosen[nch++] = lo[a++];
                    else chosen[nch++] = hi[b++];
                } else if (a < nlo) {
                    chosen[nch++] = lo[a++];
                } else {
                    chosen[nch++] = hi[b++];
                }
            }
            for (int t = 0; t < M; ++t) {
                // Lagrange weight of node t: one quotient of the two products
                long double num = 1.0L, den = 1.0L;
                for (int m = 0; m < M; ++m)
                    if (m != t) {
                        num *= bstar[k] - (long double)chosen[m].b;
                        den *= (long double)chosen[t].b - (long double)chosen[m].b;
                    }
                const long double w = num / den;
                const size_t o = (((size_t)p * M + used) * M + t);
                const double whi = (double)w;
                mwv[2 * o] = whi;
                mwv[2 * o + 1] = (double)(w - (long double)whi);
                if (!chosen[t].sq) {
                    mref[o] = r.vertical ? (int32_t)((size_t)r.line * g.ny + chosen[t].j)
                                         : (int32_t)((size_t)chosen[t].j * g.ny + r.line);
                } else {
                    const int ls = nsq[p]++;
                    mref[o] = -(1 + ls);   // square number within the normal, made global below
                    double* xy = &sqxy[((size_t)p * nstar * 2 + ls) * 2];
                    if (r.vertical) { xy[0] = r.a_line; xy[1] = chosen[t].b; }
                    else { xy[0] = chosen[t].b; xy[1] = r.a_line; }
                }
            }
            deltas[used] = delta[k];
            ++used;
        }
        if (used < nstar) {
            bad = std::min(bad, p);
            continue;
        }
        if (nstar < M) {   // the point on Gamma: no stencil (entries marked unused), depth 0
            for (int t = 0; t < M; ++t) {
                const size_t o = ((size_t)p * M + M - 1) * M + t;
                mref[o] = kUnusedRef;
                mwv[2 * o] = mwv[2 * o + 1] = 0.0;
            }
            deltas[M - 1] = 0.0L;
        }
        for (int qq = 0; qq < nq; ++qq) {
            const long double x = (long double)(d - 1 - qq) * (long double)g.k1;
            for (int sv = 0; sv < M; ++sv) {
                long double num = 1.0L, den = 1.0L;
                for (int m = 0; m < M; ++m)
                    if (m != sv) {
                        num *= x - deltas[m];
                        den *= deltas[sv] - deltas[m];
                    }
                const long double w = num / den;
                const size_t o = ((size_t)p * nq + qq) * M + sv;
                const double whi = (double)w;
                mwn[2 * o] = whi;
                mwn[2 * o + 1] = (double)(w - (long double)whi);
            }
        }
    }
    if (bad < B) return -(bad + 1);
    // squares in the order normal, star, node
    std::vector<int> sq0(B + 1, 0);
    for (int p = 0; p < B; ++p) sq0[p + 1] = sq0[p] + nsq[p];
    squares.resize(2 * (size_t)sq0[B]);
    for (int p = 0; p < B; ++p) {
        std::copy(&sqxy[(size_t)p * nstar * 2 * 2], &sqxy[(size_t)p * nstar * 2 * 2] + 2 * nsq[p],
                  squares.begin() + 2 * (size_t)sq0[p]);
        for (int e = 0; e < M * M; ++e) {
            int32_t& r = mref[(size_t)p * M * M + e];
            if (r < 0 && r != kUnusedRef) r -= sq0[p];
        }
    }
    return 0;
}

}  // namespace fc2d
