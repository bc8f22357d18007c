// Host part of the matching stencils (Sec. 3.2, Fig. 3): placement of the red
// stars along each normal and, from the device's scan of their grid lines, the
// choice of stars and nodes and the interpolation weights.  No HIP dependency:
// the unit builds with a plain host compiler (and its sanitizers).
#pragma once

#include <stdint.h>

#include <memory>
#include <new>
#include <utility>
#include <vector>

namespace fc2d {

// Host arrays of the plan that their builders write in full, in parallel:
// resize() leaves the elements default-initialised (no serial zero fill), so
// the first touch of their pages happens in the parallel loops that fill them.
template <class T>
struct NoInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <class U>
    NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
    template <class U, class... A>
    void construct(U* p, A&&... a) {
        if constexpr (sizeof...(A) == 0) ::new ((void*)p) U;
        else ::new ((void*)p) U(std::forward<A>(a)...);
    }
};
template <class T>
using HostVec = std::vector<T, NoInitAlloc<T>>;

// Red-star candidates of the matching stencils: one per (normal, candidate line).
// The device scans the star's grid line for the runs of IN points next to it
// and locates the line's crossings with Gamma bounding them.
struct StarQ {
    int32_t p;          // normal
    int32_t vertical;   // 1: the line x = x_line (runs along y); 0: y = y_line
    int32_t line;       // grid line index
    int32_t jb;         // grid index along the line just below the star
    double a_line;      // the line's coordinate
    double bstar;       // the star's coordinate along the line
    int32_t skip;       // 1: too close to Gamma, not used
    int32_t pad;
};
struct StarR {
    int32_t nlo, nhi;   // IN points jb, jb-1, ... (nlo of them) and jb+1, ... (nhi)
    int32_t side[2];    // below [0] and above [1]: 1 the run ends at Gamma within M steps (square
                        // sq[s]); 2 a foot solve failed
    double sq[2];       // crossing coordinate along the line
};

constexpr int32_t kUnusedRef = INT32_MIN;   // stencil entry of the point-on-Gamma slot (not gathered)
constexpr int kMaxStencil = 15;             // largest compiled M

struct MatchGeom {
    double x0, y0, h;
    int nx, ny;
    int M, d, B;
    bool interior_only;   // Remark 3.1 II: no boundary samples
    double k1;
    const double *bx, *by, *bnx, *bny;   // boundary samples and outward normals [B]
};

// 2M candidate stars per normal (crossings of the inward normal with the grid
// lines x = x_i when |n_x| >= |n_y|, else y = y_j, by depth), with their depth
// and position along the line in extended precision.
void place_stars(const MatchGeom& g, HostVec<StarQ>& q, HostVec<long double>& delta, HostVec<long double>& bstar);

// From the scan results: per normal the red stars (the first candidates with at
// least M nodes), their M nearest nodes (grid points or squares), the weights
// along the grid lines and along the normal (double-double, formed in x87
// extended precision).  mref [B][M][M]: grid flat index or -(1 + square);
// squares: 2 per square in the order normal, star, node.  Returns 0, or the
// first normal with too few usable stars + 1 (as a negative number: -(p + 1)).
int select_matching(const MatchGeom& g, const StarQ* q, const StarR* res, const long double* delta,
                    const long double* bstar, HostVec<int32_t>& mref, HostVec<double>& mwv, HostVec<double>& mwn,
                    std::vector<double>& squares);

}  // namespace fc2d
