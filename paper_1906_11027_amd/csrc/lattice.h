// lattice.h -- compile-time lattice and force-stencil tables for the gfx950
// kernels.
//
// LB velocity sets (Sec. 3 of Peng, Ayala, Ayala & Wang): D2Q9 (Table 1) and
// the nearest-neighbour D3Q19 cube lattice, both with cs^2 = 1/3.  Velocity
// order is the library's storage order and is part of the state layout.
//
// Force stencils E_{2n} (Sec. 2, Eq. (1)): normalised weights w_hat(|e|^2)
// with sum w_hat e_x^2 = 1 and isotropic moment tensors through rank 2n.
// The kernels sum over +-e pairs, so only one vector of each pair is kept
// (first non-zero component positive); the pair list is enumerated at
// compile time from the shell radii below.
#pragma once

namespace sclbm {

// ---------------------------------------------------------------- D2Q9 ----
// rest, E, N, W, S, NE, NW, SW, SE
struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr double cs2 = 1.0 / 3;
};

// --------------------------------------------------------------- D3Q19 ----
// rest, 6 axis neighbours (+x -x +y -y +z -z), 12 edge neighbours
struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr double w[19] = {1.0 / 3,
                                     1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr double cs2 = 1.0 / 3;
};

// --------------------------------------------------- D2Q13, D2Q25 ----
// The larger 2D sets of Sec. 3, Table 1 (weights by |c|^2): D2Q13 with
// cs^2 = 2/5 (6th-order isotropic), D2Q25 with cs^2 = 4/7 (8th-order).
// Order: rest, then shells by |c|^2, each shell in (cx, cy) lexicographic order.
struct D2Q13 {
    static constexpr int Q = 13;
    static constexpr int D = 2;
    static constexpr int cx[13] = {0, -1, 0, 0, 1, -1, -1, 1, 1, -2, 0, 0, 2};
    static constexpr int cy[13] = {0, 0, -1, 1, 0, -1, 1, -1, 1, 0, -2, 2, 0};
    static constexpr int cz[13] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[13] = {2.0 / 5,
                                     8.0 / 75, 8.0 / 75, 8.0 / 75, 8.0 / 75,
                                     1.0 / 25, 1.0 / 25, 1.0 / 25, 1.0 / 25,
                                     1.0 / 300, 1.0 / 300, 1.0 / 300, 1.0 / 300};
    static constexpr double cs2 = 2.0 / 5;
};
struct D2Q25 {
    static constexpr int Q = 25;
    static constexpr int D = 2;
    static constexpr int cx[25] = {0, -1, 0, 0, 1, -1, -1, 1, 1, -2, 0, 0, 2,
                                   -2, -2, -1, -1, 1, 1, 2, 2, -2, -2, 2, 2};
    static constexpr int cy[25] = {0, 0, -1, 1, 0, -1, 1, -1, 1, 0, -2, 2, 0,
                                   -1, 1, -2, 2, -2, 2, -1, 1, -2, 2, -2, 2};
    static constexpr int cz[25] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0,
                                   0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[25] = {72.0 / 245,
                                     16.0 / 147, 16.0 / 147, 16.0 / 147, 16.0 / 147,
                                     16.0 / 315, 16.0 / 315, 16.0 / 315, 16.0 / 315,
                                     1.0 / 105, 1.0 / 105, 1.0 / 105, 1.0 / 105,
                                     8.0 / 2205, 8.0 / 2205, 8.0 / 2205, 8.0 / 2205,
                                     8.0 / 2205, 8.0 / 2205, 8.0 / 2205, 8.0 / 2205,
                                     1.0 / 8820, 1.0 / 8820, 1.0 / 8820, 1.0 / 8820};
    static constexpr double cs2 = 4.0 / 7;
};

// ------------------------------------------------------- force stencils ----
template <int D, int ORDER> struct Shells;

template <> struct Shells<2, 4> {
    static constexpr int n = 2;
    static constexpr int s[2] = {1, 2};
    static constexpr double w[2] = {1.0 / 3, 1.0 / 12};
};
template <> struct Shells<2, 6> {
    static constexpr int n = 3;
    static constexpr int s[3] = {1, 2, 4};
    static constexpr double w[3] = {4.0 / 15, 1.0 / 10, 1.0 / 120};
};
template <> struct Shells<2, 8> {
    static constexpr int n = 5;
    static constexpr int s[5] = {1, 2, 4, 5, 8};
    static constexpr double w[5] = {4.0 / 21, 4.0 / 45, 1.0 / 60, 2.0 / 315, 1.0 / 5040};
};
template <> struct Shells<2, 10> {
    static constexpr int n = 7;
    static constexpr int s[7] = {1, 2, 4, 5, 8, 9, 10};
    static constexpr double w[7] = {262.0 / 1785, 93.0 / 1190, 7.0 / 340, 6.0 / 595,
                                    9.0 / 9520, 2.0 / 5355, 1.0 / 7140};
};
template <> struct Shells<3, 4> {
    static constexpr int n = 2;
    static constexpr int s[2] = {1, 2};
    static constexpr double w[2] = {1.0 / 6, 1.0 / 12};
};
template <> struct Shells<3, 6> {
    static constexpr int n = 4;
    static constexpr int s[4] = {1, 2, 3, 4};
    static constexpr double w[4] = {2.0 / 15, 1.0 / 15, 1.0 / 60, 1.0 / 120};
};
template <> struct Shells<3, 8> {
    static constexpr int n = 7;
    static constexpr int s[7] = {1, 2, 3, 4, 5, 6, 8};
    static constexpr double w[7] = {4.0 / 45, 1.0 / 21, 2.0 / 105, 5.0 / 504,
                                    1.0 / 315, 1.0 / 630, 1.0 / 5040};
};

struct PairList {
    int n;          // number of +-e pairs
    int r;          // largest |e_i| (psi halo width)
    int e[48][3];   // one vector per pair
    double w[48];   // w_hat of the pair's shell
    int s[48];      // shell index of the pair (pairs are listed shell by shell)

    // true if pair p is the last of its shell: the kernels sum e (psi+ - psi-)
    // over a shell and multiply by its weight once
    constexpr bool shell_end(int p) const { return p + 1 >= n || s[p + 1] != s[p]; }
};

template <int D, int ORDER>
constexpr PairList make_pairs()
{
    PairList p{};
    p.n = 0;
    p.r = 0;
    using S = Shells<D, ORDER>;
    for (int k = 0; k < S::n; ++k) {
        const int s2 = S::s[k];
        const int m = 3;
        for (int a = -m; a <= m; ++a)
            for (int b = -m; b <= m; ++b)
                for (int c = (D == 3 ? -m : 0); c <= (D == 3 ? m : 0); ++c) {
                    if (a * a + b * b + c * c != s2) continue;
                    // keep the member of the pair whose first non-zero component is positive
                    const int first = a != 0 ? a : (b != 0 ? b : c);
                    if (first <= 0) continue;
                    p.e[p.n][0] = a;
                    p.e[p.n][1] = b;
                    p.e[p.n][2] = c;
                    p.w[p.n] = S::w[k];
                    p.s[p.n] = k;
                    ++p.n;
                    const int ma = a < 0 ? -a : a, mb = b < 0 ? -b : b, mc = c < 0 ? -c : c;
                    const int mx = ma > mb ? (ma > mc ? ma : mc) : (mb > mc ? mb : mc);
                    if (mx > p.r) p.r = mx;
                }
    }
    return p;
}

template <int D, int ORDER>
struct Stencil {
    static constexpr PairList P = make_pairs<D, ORDER>();
    static constexpr int NP = P.n;
    static constexpr int R = P.r;
};

}  // namespace sclbm
