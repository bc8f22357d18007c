// Host-only check of the library's host C++ (matching_host.cpp, fcgram_quad.cpp),
// built with AddressSanitizer and UndefinedBehaviorSanitizer on the CPU by
// tests/test_host_sanitizers.py.  No GPU: the device's part of the matching
// stencils (scan of the red stars' grid lines for IN runs and their crossings
// with Gamma) is replaced here by its closed form on the unit disc, with the
// classes of the disc (IN: x^2 + y^2 <= 1).
#include <math.h>
#include <stdio.h>

#include <vector>

#include "../paper_2010_03901_amd/csrc/matching.h"

namespace fc2d {
int gram_tables(int d, int C, int Z, int n_os, int n_r, int mf, double* Q, double* A, double* Ar);
}
using namespace fc2d;

static int fails = 0;
#define CHECK(c, ...)                       \
    do {                                    \
        if (!(c)) {                         \
            fprintf(stderr, __VA_ARGS__);   \
            fputc('\n', stderr);            \
            ++fails;                        \
        }                                   \
    } while (0)

static void check_tables(int d) {
    const int C = 27, Z = 12, n_os = 20, n_r = 6, mf = 20;
    std::vector<double> Q(d * d), A(C * d), Ar(C * n_r * d);
    CHECK(gram_tables(d, C, Z, n_os, n_r, mf, Q.data(), A.data(), Ar.data()) == 0, "gram_tables d=%d failed", d);
    double e = 0.0;   // Q Q^T = I (Q square orthogonal)
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += Q[i * d + k] * Q[j * d + k];
            e = fmax(e, fabs(s - (i == j)));
        }
    CHECK(e < 1e-13, "tables d=%d: |Q Q^T - I| = %g", d, e);
    for (double v : Ar) CHECK(isfinite(v), "tables d=%d: non-finite A_r", d);
    // bad arguments are refused
    CHECK(gram_tables(1, C, Z, n_os, n_r, mf, Q.data(), A.data(), Ar.data()) != 0, "d=1 accepted");
}

// the scan of one red star's grid line on the unit disc: IN runs next to the
// star and the crossings of the line with the circle that bound them
static StarR scan_disc(const MatchGeom& g, const StarQ& s) {
    StarR r = {0, 0, {0, 0}, {0.0, 0.0}};
    if (s.skip) return r;
    const bool vert = s.vertical != 0;
    const int nline = vert ? g.nx : g.ny, nb = vert ? g.ny : g.nx;
    const double a0 = vert ? g.x0 : g.y0, b0 = vert ? g.y0 : g.x0;
    auto in_at = [&](int j) {
        if (j < 0 || j >= nb || s.line < 0 || s.line >= nline) return false;
        const double a = a0 + s.line * g.h, b = b0 + j * g.h;
        return a * a + b * b <= 1.0;
    };
    const int M = g.M;
    int j = s.jb;
    while (j >= s.jb - M && in_at(j)) { ++r.nlo; --j; }
    const bool lo_stop = j >= s.jb - M;
    j = s.jb + 1;
    while (j <= s.jb + 1 + M && in_at(j)) { ++r.nhi; ++j; }
    const bool hi_stop = j <= s.jb + 1 + M;
    if (!g.interior_only) {
        const double half = sqrt(fmax(0.0, 1.0 - s.a_line * s.a_line));
        if (lo_stop) { r.sq[0] = -half; r.side[0] = 1; }
        if (hi_stop) { r.sq[1] = half; r.side[1] = 1; }
    }
    return r;
}

// FNV-1a over the bytes of an array: a digest of the stencils, compared
// between runs with different thread counts
static uint64_t g_digest = 1469598103934665603ULL;
template <class V>
static void digest(const V& v) {
    const unsigned char* b = (const unsigned char*)v.data();
    for (size_t i = 0; i < v.size() * sizeof(v[0]); ++i) g_digest = (g_digest ^ b[i]) * 1099511628211ULL;
}

static void check_matching(bool interior_only) {
    const int n = 128, B = 256;
    std::vector<double> bx(B), by(B), bnx(B), bny(B);
    for (int p = 0; p < B; ++p) {
        const double t = 2.0 * M_PI * p / B;
        bx[p] = cos(t); by[p] = sin(t); bnx[p] = cos(t); bny[p] = sin(t);
    }
    MatchGeom g;
    g.x0 = -1.5; g.y0 = -1.5; g.h = 3.0 / n; g.nx = n; g.ny = n;
    g.M = 8; g.d = 5; g.B = B; g.interior_only = interior_only; g.k1 = 0.2 / 27;
    g.bx = bx.data(); g.by = by.data(); g.bnx = bnx.data(); g.bny = bny.data();
    HostVec<StarQ> q;
    HostVec<long double> delta, bstar;
    place_stars(g, q, delta, bstar);
    CHECK(q.size() == (size_t)B * 2 * g.M, "place_stars: %zu candidates", q.size());
    std::vector<StarR> res(q.size());
    for (size_t k = 0; k < q.size(); ++k) res[k] = scan_disc(g, q[k]);
    HostVec<int32_t> mref;
    HostVec<double> mwv, mwn;
    std::vector<double> squares;
    const int st = select_matching(g, q.data(), res.data(), delta.data(), bstar.data(), mref, mwv, mwn, squares);
    CHECK(st == 0, "select_matching: %d", st);
    if (st) return;
    digest(mref);
    digest(mwv);
    digest(mwn);
    digest(squares);
    const int M = g.M, nq = interior_only ? g.d : g.d - 1, nstar = interior_only ? M : M - 1;
    const int nsq = (int)squares.size() / 2;
    CHECK(!interior_only || nsq == 0, "interior-only stencils use %d squares", nsq);
    for (int p = 0; p < B; ++p) {
        for (int s = 0; s < nstar; ++s) {
            double wsum = 0.0;
            for (int t = 0; t < M; ++t) {
                const size_t o = ((size_t)p * M + s) * M + t;
                const int32_t r = mref[o];
                CHECK((r >= 0 && r < n * n) || (r < 0 && -r - 1 < nsq), "normal %d: stencil entry %d", p, r);
                if (r >= 0) {
                    const double x = g.x0 + (r / n) * g.h, y = g.y0 + (r % n) * g.h;
                    CHECK(x * x + y * y <= 1.0, "normal %d: node (%g, %g) not IN", p, x, y);
                }
                wsum += mwv[2 * o] + mwv[2 * o + 1];
            }
            CHECK(fabs(wsum - 1.0) < 1e-12, "normal %d star %d: weights sum to %.17g", p, s, wsum);
        }
        for (int qq = 0; qq < nq; ++qq) {
            double wsum = 0.0;
            for (int s = 0; s < M; ++s) wsum += mwn[2 * (((size_t)p * nq + qq) * M + s)];
            CHECK(fabs(wsum - 1.0) < 1e-9, "normal %d value %d: normal weights sum to %.17g", p, qq, wsum);
        }
    }
    for (int k = 0; k < nsq; ++k) {
        const double x = squares[2 * k], y = squares[2 * k + 1];
        CHECK(fabs(x * x + y * y - 1.0) < 1e-14, "square %d off the circle", k);
    }
}

int main() {
    for (int d : {4, 5, 10, 12}) check_tables(d);
    check_matching(false);
    check_matching(true);
    if (fails) {
        fprintf(stderr, "%d failures\n", fails);
        return 1;
    }
    printf("stencil digest %016llx\n", (unsigned long long)g_digest);
    printf("HOST_CHECK_OK\n");
    return 0;
}
