// Per-node building blocks of the fused step for gfx950:
//   gather   pull streaming in coordinate space (Eq. (3), left-hand side)
//            with periodic axes and halfway trajectory bounce-back;
//   collide  moments, metric Hermite equilibrium through H3 (Eq. (6)),
//            stress-corrected forcing through H3 and BGK (Eq. (3),
//            right-hand side), evaluated on (c, -c) pairs.
//
// Populations are carried as offsets g_q = f_q - w_q.  Because the weights
// sum to one and have vanishing odd moments, rho' - 1 = sum g, rho' u = sum c g
// and sum c c f = sum c c g + cs2 delta, so the offsets lose no information
// and keep FP32/FP16 rounding small.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "lattice.hpp"

namespace mlbm {

template <int I, int N, class F>
__host__ __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// a x + b y + c z for compile-time a, b, c in {-1, 0, 1}; starting from -0.0
// lets the compiler drop the zero terms exactly.
template <int A, int B, int Cc, class T>
__host__ __device__ __forceinline__ T sdot(T x, T y, T z)
{
    T s = T(-0.0);
    if constexpr (A == 1) s += x; else if constexpr (A == -1) s -= x;
    if constexpr (B == 1) s += y; else if constexpr (B == -1) s -= y;
    if constexpr (Cc == 1) s += z; else if constexpr (Cc == -1) s -= z;
    return s;
}

// ------------------------------------------------------------------------
// Geometry of one cross-section node, with compile-time sparsity
// ------------------------------------------------------------------------

template <int PAT> struct Mask {
    // Delta^ij nonzero?
    static constexpr bool D(int i, int j) { return PAT == PAT_GEN ? true : i == j; }
    // Gamma^i_jk nonzero (j <= k)?
    static constexpr bool G(int i, int j, int k)
    {
        if (PAT == PAT_GEN) return true;
        if (PAT == PAT_CYL) return (i == 0 && j == 1 && k == 1) || (i == 1 && j == 0 && k == 1);
        return (i == 0 && j == 1 && k == 1) || (i == 0 && j == 2 && k == 2) ||
               (i == 1 && j == 0 && k == 1) || (i == 1 && j == 1 && k == 2) ||
               (i == 2 && j == 0 && k == 2) || (i == 2 && j == 1 && k == 1);
    }
    static constexpr bool F(int i) { return PAT == PAT_GEN ? true : i == 1; }
};

// Geometry index of node (x1, x2, x3) and the stride of a geometry field.
__host__ __device__ __forceinline__ int geo_index(const InstDesc &d, int x1, int x2, int x3)
{
    return (x1 * d.n2g + (d.n2g > 1 ? x2 : 0)) * d.n3g + (d.n3g > 1 ? x3 : 0);
}
__host__ __device__ __forceinline__ int geo_stride(const InstDesc &d) { return d.n1 * d.n2g * d.n3g; }

constexpr int d_field(int i, int j)
{
    int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? (b == 0 ? G_D11 : b == 1 ? G_D12 : G_D13) : a == 1 ? (b == 1 ? G_D22 : G_D23) : G_D33;
}
constexpr int g_field(int i, int j, int k)
{
    int a = j < k ? j : k, b = j < k ? k : j;
    int off = a == 0 ? b : a == 1 ? 2 + b : 5;   // (11,12,13,22,23,33) -> 0..5
    return G_1_11 + 6 * i + off;
}

template <int PAT, class C>
struct NodeGeo {
    C D[3][3];        // Delta^ij (zero entries never read)
    C Gm[3][3][3];    // Gamma^i_jk (symmetric in jk)
    C Fe[3];          // external force (lattice units)

    // field f at cross-section index idx: from the FP64 precompute, or for
    // FP32 arithmetic from its FP32 copy (the same values rounded once, so
    // the results are identical and the geometry traffic halves)
    __device__ __forceinline__ C field(const double *__restrict__ geo, const float *__restrict__ geof, int f, int idx,
                                       int stride) const
    {
        const uint32_t e = (uint32_t)(f * stride) + (uint32_t)idx;
        if constexpr (std::is_same<C, float>::value)
            return gload<float>(geof, 4ull * e);
        else
            return (C)gload<double>(geo, 8ull * e);
    }

    // On the double-curved slab (metric frozen at theta = 0) half of the
    // fields depend on r alone: Delta^11, Delta^33, Gamma^1_33, Gamma^2_12
    // and Gamma^3_13 take the same value at every node of an x1 row. They
    // are read at the row's first node (ridx, the same address for every
    // lane: one request per wavefront), the others at the node's own (idx).
    static constexpr bool row_only(int f)
    {
        return PAT == PAT_ELL &&
               (f == G_D11 || f == G_D33 || f == G_1_33 || f == G_2_12 || f == G_3_13);
    }

    __device__ __forceinline__ void load(const double *__restrict__ geo, const float *__restrict__ geof, int idx,
                                         int stride, C force, int ridx = -1)
    {
        if (ridx < 0) ridx = idx;
        static_for<0, 3>([&](auto I) {
            static_for<0, 3>([&](auto J) {
                if constexpr (Mask<PAT>::D(I, J)) {
                    constexpr int f = d_field(I, J);
                    D[I][J] = field(geo, geof, f, row_only(f) ? ridx : idx, stride);
                }
                static_for<0, 3>([&](auto K) {
                    if constexpr (Mask<PAT>::G(I, J < K ? J : K, J < K ? K : J)) {
                        constexpr int f = g_field(I, J, K);
                        Gm[I][J][K] = field(geo, geof, f, row_only(f) ? ridx : idx, stride);
                    }
                });
            });
            if constexpr (Mask<PAT>::F(I))
                Fe[I] = force * field(geo, geof, G_F1 + I, idx, stride);
        });
    }
};

// ------------------------------------------------------------------------
// Collision
// ------------------------------------------------------------------------

// In-place BGK update of one node's populations (Sec. II). g[q] holds the
// offset f - w, or with SCALED the scaled offset (f - w) / w, before and
// after the update. rho_out and u_out receive rho' and the lattice velocity
// u = sum c f / rho' used by the collision (no half-force shift).  R is the
// register type of the populations, C the arithmetic type (R may be
// narrower: every value is widened to C before it is used). SCALED moves
// the weights into the moment constants, so the update itself has none.
template <int PAT, class C, class R, bool SCALED = false>
__host__ __device__ __forceinline__ void collide(R (&g)[Q], const NodeGeo<PAT, C> &G, C omega, C kappa,
                                                 C &rho_out, C (&u_out)[3])
{
    // f - w = ws(q) * (register value): ws is the weight for scaled
    // registers, else 1
    constexpr auto ws = [](int q) constexpr { return SCALED ? C(wq(q)) : C(1); };
    constexpr C cs2 = (C)CS2;
    constexpr C ics2 = (C)(1.0 / CS2);
    constexpr C ics4 = (C)(1.0 / (CS2 * CS2));
    constexpr C ics6 = (C)(1.0 / (CS2 * CS2 * CS2));

    // --- moments of the offsets
    C m0 = ws(0) * (C)g[0];
    C j[3] = {C(-0.0), C(-0.0), C(-0.0)};
    C p[3][3];
    static_for<0, 3>([&](auto I) { static_for<0, 3>([&](auto J) { p[I][J] = C(-0.0); }); });
    static_for<0, NPAIR>([&](auto P) {
        constexpr int d = PAIR[P][0], k = PAIR[P][1], qp = PAIR[P][2], qm = PAIR[P][3];
        const C gp = (C)g[qp], gm = (C)g[qm];
        const C s = gp + gm;
        const C df = gp - gm;
        constexpr C wp = ws(qp);     // opposite populations share a weight
        m0 += wp * s;
        static_for<0, 3>([&](auto I) {
            constexpr int ci = DIR[d][I] * k;
            if constexpr (ci != 0) j[I] += (C(ci) * wp) * df;
            static_for<I, 3>([&](auto J) {
                constexpr int cij = DIR[d][I] * DIR[d][J] * k * k;
                if constexpr (cij != 0) p[I][J] += (C(cij) * wp) * s;
            });
        });
    });
    const C rho = C(1) + m0;
    const C irho = C(1) / rho;
    C u[3];
    static_for<0, 3>([&](auto I) { u[I] = j[I] * irho; });
    const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

    // --- per-node quantities
    C trD = C(-0.0);
    static_for<0, 3>([&](auto I) { if constexpr (Mask<PAT>::D(I, I)) trD += G.D[I][I]; });
    // Delta u
    C Du[3];
    static_for<0, 3>([&](auto I) {
        Du[I] = C(-0.0);
        static_for<0, 3>([&](auto J) { if constexpr (Mask<PAT>::D(I, J)) Du[I] += G.D[I < J ? I : J][I < J ? J : I] * u[J]; });
    });
    // a2 = a2_eq + kappa (Pi - Pi_eq), a2_eq = rho (cs2 Delta + u u),
    // Pi - Pi_eq = sum c c g - cs2 m0 delta - a2_eq
    C a2[3][3];
    static_for<0, 3>([&](auto I) {
        static_for<I, 3>([&](auto J) {
            C Dij = C(0);
            if constexpr (Mask<PAT>::D(I, J)) Dij = G.D[I][J];
            const C A = rho * (cs2 * Dij + u[I] * u[J]);
            C pn = p[I][J] - A;
            if constexpr (I == J) pn -= cs2 * m0;
            a2[I][J] = A + kappa * pn;
            a2[J][I] = a2[I][J];
        });
    });
    const C tra2 = a2[0][0] + a2[1][1] + a2[2][2];
    C uFe = C(-0.0);
    static_for<0, 3>([&](auto I) { if constexpr (Mask<PAT>::F(I)) uFe += u[I] * G.Fe[I]; });

    const C om = omega;
    const C omw = C(1) - omega;
    const C wr = omega * rho;
    // c-independent part of the even coefficient (also the rest population)
    const C baseE = om * m0 + wr * (C(-0.5) * trD - C(0.5) * ics2 * uu) - rho * ics2 * uFe;
    const C P0 = wr * (ics2 - C(0.5) * ics4 * uu - C(0.5) * ics2 * trD);
    const C P1 = wr * (ics6 / C(6));
    const C P2 = wr * (C(0.5) * ics4);
    const C Q0 = rho * ics2 - C(0.5) * ics4 * tra2;
    const C half_ics6 = C(0.5) * ics6;
    const C rics4 = rho * ics4;
    const C rics2 = rho * ics2;
    const C wics2 = wr * ics2;

    // FP32 arithmetic tracks the mass and momentum the rounded update actually
    // moves (sums of the small per-population changes, exact differences of
    // nearby floats) so that they can be set to their exact values below.
    constexpr bool CONSERVE = sizeof(C) == 4;
    C dm = C(-0.0), dj[3] = {C(-0.0), C(-0.0), C(-0.0)};
    {
        constexpr C w0 = SCALED ? C(1) : C(W_REST);
        const R n0 = (R)(omw * (C)g[0] + w0 * baseE);
        if constexpr (CONSERVE) dm += ws(0) * ((C)n0 - (C)g[0]);
        g[0] = n0;
    }

    // --- 13 unit directions, each used by one or two (k = 1, 3) pairs
    static_for<0, NDIR>([&](auto Dd) {
        constexpr int h1 = DIR[Dd][0], h2 = DIR[Dd][1], h3 = DIR[Dd][2];
        const C cu = sdot<h1, h2, h3>(u[0], u[1], u[2]);
        const C cDu = sdot<h1, h2, h3>(Du[0], Du[1], Du[2]);
        // chat Delta chat
        C cDc = C(-0.0);
        static_for<0, 3>([&](auto I) {
            static_for<0, 3>([&](auto J) {
                constexpr int hh = DIR[Dd][I] * DIR[Dd][J];
                if constexpr (hh != 0 && Mask<PAT>::D(I, J)) {
                    if constexpr (hh > 0) cDc += G.D[I < J ? I : J][I < J ? J : I];
                    else cDc -= G.D[I < J ? I : J][I < J ? J : I];
                }
            });
        });
        // Gamma(chat, chat)
        C Gv[3];
        static_for<0, 3>([&](auto I) {
            Gv[I] = C(-0.0);
            static_for<0, 3>([&](auto J) {
                static_for<0, 3>([&](auto K) {
                    constexpr int hh = DIR[Dd][J] * DIR[Dd][K];
                    constexpr int a = J < K ? J : K, b = J < K ? K : J;
                    if constexpr (hh != 0 && Mask<PAT>::G(I, a, b)) {
                        if constexpr (hh > 0) Gv[I] += G.Gm[I][J][K];
                        else Gv[I] -= G.Gm[I][J][K];
                    }
                });
            });
        });
        // a2 chat
        C a2c[3];
        static_for<0, 3>([&](auto I) { a2c[I] = sdot<h1, h2, h3>(a2[I][0], a2[I][1], a2[I][2]); });
        const C ca2c = sdot<h1, h2, h3>(a2c[0], a2c[1], a2c[2]);
        const C Gc = sdot<h1, h2, h3>(Gv[0], Gv[1], Gv[2]);
        const C uG = u[0] * Gv[0] + u[1] * Gv[1] + u[2] * Gv[2];
        const C a2cG = a2c[0] * Gv[0] + a2c[1] * Gv[1] + a2c[2] * Gv[2];
        C Fec = C(-0.0), a2cFe = C(-0.0);
        static_for<0, 3>([&](auto I) {
            if constexpr (Mask<PAT>::F(I)) {
                if constexpr (DIR[Dd][I] == 1) Fec += G.Fe[I];
                else if constexpr (DIR[Dd][I] == -1) Fec -= G.Fe[I];
                a2cFe += a2c[I] * G.Fe[I];
            }
        });

        static_for<0, NPAIR>([&](auto P) {
            if constexpr (PAIR[P][0] == Dd) {
                constexpr int k = PAIR[P][1], qp = PAIR[P][2], qm = PAIR[P][3];
                constexpr C kk = C(k * k), k3 = C(k * k * k), kf = C(k);
                const C cuk = kf * cu;
                const C cuk2 = cuk * cuk;
                const C Fc = kf * Fec - k3 * Gc;                // F . c
                const C cDck = kk * cDc;
                // even part: equilibrium (E - 1) and forcing E_F
                const C Ev = baseE + wr * (C(0.5) * ics2 * cDck) + P2 * cuk2
                           + rics4 * cuk * Fc + rics2 * kk * uG;
                // odd part: equilibrium O and forcing O_F
                const C Oeq = cuk * (P0 + P1 * cuk2 + P2 * cDck) - wics2 * kf * cDu;
                const C ca2F = kf * (a2cFe - kk * a2cG);        // c . a2 . F
                const C OF = Fc * (Q0 + half_ics6 * kk * ca2c) - ics4 * ca2F;
                const C Od = Oeq + OF;
                constexpr C w = SCALED ? C(1) : C(wq(qp));
                const C te = w * Ev, to = w * Od;
                const R np = (R)(omw * (C)g[qp] + (te + to));
                const R nm = (R)(omw * (C)g[qm] + (te - to));
                if constexpr (CONSERVE) {
                    constexpr C wp = ws(qp);
                    const C dp = (C)np - (C)g[qp], dq = (C)nm - (C)g[qm];
                    dm += wp * (dp + dq);
                    const C dd = dp - dq;
                    static_for<0, 3>([&](auto I) {
                        constexpr int ci = DIR[Dd][I] * k;
                        if constexpr (ci != 0) dj[I] += (C(ci) * wp) * dd;
                    });
                }
                g[qp] = np;
                g[qm] = nm;
            }
        });
    });
    // In exact arithmetic the update changes the mass by sum F = -2 rho' u^i
    // Gamma^k_ki and the momentum by S^m = rho' F_ext^m - Gamma^m_jk M^jk -
    // 2 Gamma^k_kj M^mj, M = rho' cs2 delta + a2 (moments of the forcing
    // term).  Float weights and constants miss these by a relative ~1e-7 with
    // the same sign at every node, which acts as a spurious body force in
    // slowly damped flows; the defect goes into the rest population (mass)
    // and the +-e_i pairs (momentum).
    if constexpr (CONSERVE) {
        C tr[3];   // Gamma^k_ki
        static_for<0, 3>([&](auto I) {
            tr[I] = C(-0.0);
            static_for<0, 3>([&](auto K) {
                constexpr int a = K < I ? K : I, b = K < I ? I : K;
                if constexpr (Mask<PAT>::G(K, a, b)) tr[I] += G.Gm[K][K][I];
            });
        });
        const C dm_exp = C(-2) * rho * (u[0] * tr[0] + u[1] * tr[1] + u[2] * tr[2]);
        g[0] = (R)((C)g[0] + (dm_exp - dm) * (C(1) / ws(0)));
        static_for<0, 3>([&](auto I) {
            C s = C(-0.0);
            if constexpr (Mask<PAT>::F(I)) s += rho * G.Fe[I];
            static_for<0, 3>([&](auto J) {
                const C MIJ = (I == J) ? a2[I][J] + rho * cs2 : a2[I][J];
                static_for<0, 3>([&](auto K) {
                    constexpr int a = J < K ? J : K, b = J < K ? K : J;
                    if constexpr (Mask<PAT>::G(I, a, b)) {
                        const C MJK = (J == K) ? a2[J][K] + rho * cs2 : a2[J][K];
                        s -= G.Gm[I][J][K] * MJK;
                    }
                });
                s -= C(2) * tr[J] * MIJ;
            });
            const C h = (C(0.5) / ws(1 + 2 * I)) * (s - dj[I]);   // +-e_I share a weight
            g[1 + 2 * I] = (R)((C)g[1 + 2 * I] + h);
            g[2 + 2 * I] = (R)((C)g[2 + 2 * I] - h);
        });
    }
    rho_out = rho;
    u_out[0] = u[0]; u_out[1] = u[1]; u_out[2] = u[2];
}

// Moments only (for the observables): rho' and u from offsets.
template <class C>
__device__ __forceinline__ void moments_only(const C (&g)[Q], C &rho_out, C (&u_out)[3])
{
    C m0 = g[0];
    C j[3] = {C(-0.0), C(-0.0), C(-0.0)};
    static_for<0, NPAIR>([&](auto P) {
        constexpr int d = PAIR[P][0], k = PAIR[P][1], qp = PAIR[P][2], qm = PAIR[P][3];
        m0 += g[qp] + g[qm];
        const C df = g[qp] - g[qm];
        static_for<0, 3>([&](auto I) {
            constexpr int ci = DIR[d][I] * k;
            if constexpr (ci != 0) j[I] += C(ci) * df;
        });
    });
    rho_out = C(1) + m0;
    const C ir = C(1) / rho_out;
    static_for<0, 3>([&](auto I) { u_out[I] = j[I] * ir; });
}

// Equilibrium (Dirichlet) wall node of Sec. III: the streamed populations
// only give the density rho'; the node is set to f_eq(rho', u = 0), i.e.
// f/w - 1 = (rho' - 1) + rho' (c Delta c - cs2 tr Delta) / (2 cs2), and does
// not collide. Register conventions as in collide().
template <int PAT, class C, class R, bool SCALED = false>
__host__ __device__ __forceinline__ void wall_equilibrium(R (&g)[Q], const NodeGeo<PAT, C> &G, C &rho_out)
{
    constexpr auto ws = [](int q) constexpr { return SCALED ? C(wq(q)) : C(1); };
    C m0 = ws(0) * (C)g[0];
    static_for<1, Q>([&](auto q) { m0 += ws(q) * (C)g[q]; });
    const C rho = C(1) + m0;
    C trD = C(-0.0);
    static_for<0, 3>([&](auto I) { if constexpr (Mask<PAT>::D(I, I)) trD += G.D[I][I]; });
    const C half_ics2 = (C)(0.5 / CS2);
    static_for<0, Q>([&](auto q) {
        C cDc = C(-0.0);
        static_for<0, 3>([&](auto I) {
            static_for<0, 3>([&](auto J) {
                constexpr int cc = CV[q][I] * CV[q][J];
                if constexpr (cc != 0 && Mask<PAT>::D(I, J))
                    cDc += C(cc) * G.D[I < J ? I : J][I < J ? J : I];
            });
        });
        const C h = m0 + rho * (half_ics2 * cDc - C(0.5) * trD);   // f / w - 1
        if constexpr (SCALED) g[q] = (R)h;
        else g[q] = (R)(C(wq(q)) * h);
    });
    rho_out = rho;
}

// ------------------------------------------------------------------------
// Streaming
// ------------------------------------------------------------------------

// Periodic wrap of a coordinate shifted by at most 3 cells, v in [-3, n + 2]
// (every pull, including the folded ones: a wall-reflected source lies at
// most 3 cells along each axis from the node). One correction each way is
// exact for n >= 3; axes of 1 or 2 nodes take two more.
__host__ __device__ __forceinline__ int wrap_axis(int v, int n)
{
    v += v < 0 ? n : 0;
    v -= v >= n ? n : 0;
    if (n < 3) {
        v += v < 0 ? n : 0;
        v += v < 0 ? n : 0;
        v -= v >= n ? n : 0;
        v -= v >= n ? n : 0;
    }
    return v;
}

// Axis 2 (theta) is periodic, or open at both ends (walls bit 16, the inlet
// and outlet of Sec. IV): a pull from beyond an end slab reads that end slab
// (zero gradient along theta of the populations entering the domain).
__host__ __device__ __forceinline__ int axis2(int v, int n2, bool open2)
{
    return open2 ? (v < 0 ? 0 : (v > n2 - 1 ? n2 - 1 : v)) : wrap_axis(v, n2);
}

constexpr int cslot(int c) { return c == -3 ? 0 : c == -1 ? 1 : c == 0 ? 2 : c == 1 ? 3 : 4; }
constexpr int CVALS[5] = {-3, -1, 0, 1, 3};

// Per-lane byte offsets of the pull sources inside an x1 row: o2[s] for the
// theta shift -CVALS[s] (always periodic), o3[s] for the x3 shift.
// Storage order of an instance's populations: x1 rows outermost, then the
// 41 population planes of that row (Pp = n2*n3p values each, x3 fastest
// with the padded pitch n3p). Element (q, x1, col) with the storage column
// col = x2*n3p + x3 sits at (x1*Q + q)*Pp + col, so the 41 read and the 41
// write streams of a tile each lie within one block of 41*Pp values; with
// planes N values apart the same streams cost about 15 % more HBM time.
__host__ __device__ __forceinline__ uint64_t pop_elem(int q, int x1, int col, int Pp)
{
    return ((uint64_t)x1 * Q + (uint64_t)q) * (uint64_t)Pp + (uint64_t)col;
}

// Storage column of node n (x1 row, in-row node index x2*n3 + x3).
__host__ __device__ __forceinline__ int storage_col(const InstDesc &d, int in_row)
{
    const int x2 = in_row / d.n3;
    return x2 * d.n3p + (in_row - x2 * d.n3);
}

// Random seeds of the stochastic rounding of node n's 41 populations in the
// step that reads step counter c: two hashed words of (instance salt, n,
// c); population q takes one of them rotated by its own amount (one
// funnel shift), so the top bits the conversion consumes differ between
// populations. Every bit of a good hash is uniform, so each rounding stays
// unbiased; seeds of different populations overlap, which only correlates
// their rounding. Results stay bitwise reproducible.
struct RoundBits {
    uint32_t a, b;
    __device__ __forceinline__ RoundBits(uint32_t salt, uint32_t n, uint32_t c)
    {
        const uint32_t key = salt + n * 0x9E3779B9u + c * 0x85EBCA77u;
        a = mix32(key);
        b = mix32(key ^ 0x68E31DA4u);
    }
    template <int q> __device__ __forceinline__ uint32_t get() const
    {
        constexpr uint32_t rot = (uint32_t)((q * 7) & 31);
        const uint32_t w = (q & 1) ? b : a;
        return rot == 0 ? w : ((w << rot) | (w >> (32u - rot)));
    }
};

// Reference offsets of the 16-bit storage formats as a gather sees them.
// The instance's table holds r [n1][41]; a view answers, for the source row
// `row` = x1 - t of a pull and a population q, r.
// RefScalar: for rows uniform across the wavefront (the step kernel's
// gathers and store), read through the scalar cache; reads only.
// RefRow: per-lane rows (auxiliary kernels).
struct RefScalar {
    static constexpr bool UNIFORM = true;
    const float *ref;
    __device__ __forceinline__ float get_r(int, int row, int q) const
    {
        return ((const MLBM_CONST float *)ref)[__builtin_amdgcn_readfirstlane(row) * Q + q];
    }
};
struct RefRow {
    static constexpr bool UNIFORM = false;
    const float *ref;
    __device__ __forceinline__ float get_r(int, int row, int q) const { return ref[row * Q + q]; }
};

// Decode of a pulled value; with the scalar reference view r is uniform
// across the wavefront.
template <int ST, class R>
__device__ __forceinline__ typename Codec<ST>::C decode_wave(typename Codec<ST>::T v, typename Codec<ST>::C r)
{
    if constexpr (ST == ST_F16 && R::UNIFORM) return Codec<ST>::decode_uniform(v, r);
    else return Codec<ST>::decode(v, r);
}

// Decode of a pulled value whose r was chosen per lane.
template <int ST>
__device__ __forceinline__ typename Codec<ST>::C decode_lane(typename Codec<ST>::T v, typename Codec<ST>::C r)
{
    if constexpr (ST == ST_F16) return Codec<ST>::decode_lane(v, r);
    else return Codec<ST>::decode(v, r);
}

struct LaneOffsets {
    uint32_t o2[5], o3[5];
    __device__ __forceinline__ void init(int x2, int x3, int n2, int n3, int n3p, bool per3, bool open2, uint32_t S)
    {
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            o2[s] = (uint32_t)(axis2(x2 - CVALS[s], n2, open2) * n3p) * S;
            o3[s] = (uint32_t)(per3 ? wrap_axis(x3 - CVALS[s], n3) : x3 - CVALS[s]) * S;
        }
    }
};

// Pull from x - c inside the domain (no wall within reach): the row x1 - c1
// is uniform across the wavefront, only the in-row byte offset is per lane.
template <int ST, bool EQW = false, class R>
__device__ __forceinline__ void gather_fast(const void *src, const InstDesc &d, int x1, const LaneOffsets &L,
                                            const R &ref, typename Codec<ST>::G (&g)[Q])
{
    using T = typename Codec<ST>::T;
    using C = typename Codec<ST>::C;
    constexpr uint64_t S = sizeof(T);
    const bool per1 = !(d.walls & 1);
    const uint64_t PS = (uint64_t)d.Pp * S;
    int rows[5];      // source row x1 - CVALS[s]
    uint64_t rb[5];   // byte offset of plane 0 of that row
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        int r1 = x1 - CVALS[k];
        if (per1) r1 = wrap_axis(r1, d.n1);
        // equilibrium walls: the region beyond a wall node is at rest in the
        // wall node's state, so a pull from beyond it reads the wall node
        if (EQW && d.eqwall) r1 = r1 < 0 ? 0 : (r1 > d.n1 - 1 ? d.n1 - 1 : r1);
        rows[k] = r1;
        rb[k] = (uint64_t)r1 * (uint64_t)Q * PS;
    }
    static_for<0, Q>([&](auto q) {
        constexpr int c1 = CV[q][0], c2 = CV[q][1], c3 = CV[q][2];
        const void *rowp = (const char *)src + rb[cslot(c1)] + (uint64_t)q * PS;
        const C r = Codec<ST>::REF ? (C)ref.get_r(c1, rows[cslot(c1)], q) : C(0);
        g[q] = decode_wave<ST, R>(gload<T>(rowp, L.o2[cslot(c2)] + L.o3[cslot(c3)]), r);
    });
}

// gather_fast for a wavefront of an instance with x3 walls none of whose
// lanes is within reach of them: x3 - c3 needs no wrap, so the in-row offset
// is (x3 - c3) S + the x2 offset, and the constant -c3 S goes into the
// wavefront-uniform row address. Five per-lane offsets (one per x2 shift)
// serve all 41 loads, with no per-population address arithmetic.
template <int ST, bool EQW = false, bool OPEN2 = true, class R>
__device__ __forceinline__ void gather_fast_walled3(const void *src, const InstDesc &d, int x1, int x2, int x3,
                                                    const R &ref, typename Codec<ST>::G (&g)[Q])
{
    using T = typename Codec<ST>::T;
    using C = typename Codec<ST>::C;
    constexpr uint64_t S = sizeof(T);
    const bool per1 = !(d.walls & 1);
    const uint64_t PS = (uint64_t)d.Pp * S;
    int rows[5];      // source row x1 - CVALS[s]
    uint64_t rb[5];   // byte offset of plane 0 of that row
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        int r1 = x1 - CVALS[k];
        if (per1) r1 = wrap_axis(r1, d.n1);
        if (EQW && d.eqwall) r1 = r1 < 0 ? 0 : (r1 > d.n1 - 1 ? d.n1 - 1 : r1);
        rows[k] = r1;
        rb[k] = (uint64_t)r1 * (uint64_t)Q * PS;
    }
    uint32_t o[5];    // in-row byte offset of (x2 - CVALS[s], x3)
    const bool open2 = OPEN2 && (d.walls & 16);
#pragma unroll
    for (int s = 0; s < 5; ++s) o[s] = (uint32_t)(axis2(x2 - CVALS[s], d.n2, open2) * d.n3p + x3) * (uint32_t)S;
    static_for<0, Q>([&](auto q) {
        constexpr int c1 = CV[q][0], c2 = CV[q][1], c3 = CV[q][2];
        const char *rowp = (const char *)src + rb[cslot(c1)] + (uint64_t)q * PS - (int64_t)c3 * (int64_t)S;
        const C r = Codec<ST>::REF ? (C)ref.get_r(c1, rows[cslot(c1)], q) : C(0);
        g[q] = decode_wave<ST, R>(gload<T>(rowp, o[cslot(c2)]), r);
    });
}

// Pull for a wavefront whose x1 row is out of reach of x1 walls while some
// of its lanes are within reach of an x3 wall (x3 walled, n3 >= 5). Only the
// x3 wall can then be met, and at most once: a population with c3 != 0 whose
// backward path from x meets the wall behind it (dist = x3 or n3 - 1 - x3
// nodes; a crossing when 2 dist + 1 < 2m, m = max |c_a|) comes from the
// opposite population at x - (c/m) sb with sb = 2 dist + 1 - m, the
// single-reflection case of fold_source below. Every other population is
// the plain pull. Candidates are formed from per-wave row offsets and
// per-lane in-row offsets and chosen per lane by selects, so the path has
// no branches; byte offsets fit in 32 bits (buffers are below 4 GiB).
template <int ST, bool OPEN2 = true, class R>
__device__ __forceinline__ void gather_x3wall(const void *src, const InstDesc &d, int x1, int x2, int x3,
                                              const LaneOffsets &L, const R &ref, typename Codec<ST>::G (&g)[Q])
{
    using T = typename Codec<ST>::T;
    using C = typename Codec<ST>::C;
    constexpr uint32_t S = sizeof(T);
    const bool per1 = !(d.walls & 1);
    const uint32_t PS = (uint32_t)d.Pp * S;
    int rows[7];      // source row x1 - t, t = -3..3
    uint32_t rb[7];   // byte offset of plane 0 of that row
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        int r1 = x1 - (k - 3);
        if (per1) r1 = wrap_axis(r1, d.n1);
        rows[k] = r1;
        rb[k] = (uint32_t)r1 * (uint32_t)Q * PS;
    }
    const uint32_t n3S = (uint32_t)d.n3p * S;
    // in-row x2 offsets of x2 - t for t = -3..3
    const bool open2 = OPEN2 && (d.walls & 16);
    const uint32_t o2t[7] = {L.o2[0], (uint32_t)axis2(x2 + 2, d.n2, open2) * n3S, L.o2[1], L.o2[2], L.o2[3],
                             (uint32_t)axis2(x2 - 2, d.n2, open2) * n3S, L.o2[4]};
    const uint32_t x3S = (uint32_t)x3 * S;
    const int dlo = x3, dhi = d.n3 - 1 - x3;
    static_for<0, Q>([&](auto q) {
        constexpr int c1 = CV[q][0], c2 = CV[q][1], c3 = CV[q][2];
        constexpr int a1 = c1 < 0 ? -c1 : c1, a2 = c2 < 0 ? -c2 : c2, a3 = c3 < 0 ? -c3 : c3;
        constexpr int m = a1 > a2 ? (a1 > a3 ? a1 : a3) : (a2 > a3 ? a2 : a3);
        constexpr bool REF = Codec<ST>::REF;
        uint32_t off = rb[3 + c1] + (uint32_t)q * PS + L.o2[cslot(c2)] + L.o3[cslot(c3)];
        C r = REF ? (C)ref.get_r(c1, rows[3 + c1], q) : C(0);
        if constexpr (c3 != 0) {
            constexpr int qo = opposite(q);
            constexpr int h1 = c1 / m, h2 = c2 / m, h3 = c3 / m;
            const int dist = c3 > 0 ? dlo : dhi;
            const uint32_t base = (uint32_t)qo * PS;
            if constexpr (m == 1) {
                const uint32_t o0 = rb[3] + base + L.o2[2] + x3S;            // sb = 0: the node itself
                off = dist == 0 ? o0 : off;
                if constexpr (REF) {
                    const C r0 = (C)ref.get_r(0, rows[3], qo);   // read unconditionally, then select
                    r = dist == 0 ? r0 : r;
                }
            } else {
                const uint32_t oa = rb[3 - 2 * h1] + base + o2t[3 - 2 * h2] + (uint32_t)((int)x3S + 2 * h3 * (int)S);
                const uint32_t ob = rb[3] + base + L.o2[2] + x3S;
                const uint32_t oc = rb[3 + 2 * h1] + base + o2t[3 + 2 * h2] + (uint32_t)((int)x3S - 2 * h3 * (int)S);
                off = dist == 0 ? oa : (dist == 1 ? ob : (dist == 2 ? oc : off));
                if constexpr (REF) {
                    const C ra = (C)ref.get_r(-2 * h1, rows[3 - 2 * h1], qo);
                    const C rbv = (C)ref.get_r(0, rows[3], qo);
                    const C rc = (C)ref.get_r(2 * h1, rows[3 + 2 * h1], qo);
                    r = dist == 0 ? ra : (dist == 1 ? rbv : (dist == 2 ? rc : r));
                }
            }
        }
        if constexpr (c3 != 0) g[q] = decode_lane<ST>(gload<T>(src, (uint64_t)off), r);   // r chosen per lane
        else g[q] = decode_wave<ST, R>(gload<T>(src, (uint64_t)off), r);
    });
}

// Pull for a wavefront in a row within reach of an x1 wall while none of its
// lanes is within reach of an x3 wall. x1 is uniform across the wavefront,
// so whether a population meets the x1 wall behind it (back = 2 x1 + 1 or
// 2 n1 - 1 - 2 x1 half-cells, a crossing when back < 2m) and its step count
// sb = back - m are scalars: the source row and plane are uniform and only
// the in-row offset of x - (c/m) sb varies per lane. One x1 crossing at
// most (a single walled axis of >= 4 nodes), as in fold_source below.
template <int ST, bool OPEN2 = true, class R>
__device__ __forceinline__ void gather_x1wall(const void *src, const InstDesc &d, int x1, int x2, int x3,
                                              const LaneOffsets &L, const R &ref, typename Codec<ST>::G (&g)[Q])
{
    using T = typename Codec<ST>::T;
    using C = typename Codec<ST>::C;
    constexpr uint32_t S = sizeof(T);
    const bool per3 = !(d.walls & 4);
    const uint32_t PS = (uint32_t)d.Pp * S;
    const uint32_t n3S = (uint32_t)d.n3p * S;
    // in-row offsets of x - t along x2 and x3 for t = -2, 0, 2 (index 0, 1, 2)
    const bool open2 = OPEN2 && (d.walls & 16);
    const uint32_t o2s[3] = {(uint32_t)axis2(x2 + 2, d.n2, open2) * n3S, L.o2[2],
                             (uint32_t)axis2(x2 - 2, d.n2, open2) * n3S};
    const uint32_t o3s[3] = {(uint32_t)(per3 ? wrap_axis(x3 + 2, d.n3) : x3 + 2) * S, L.o3[2],
                             (uint32_t)(per3 ? wrap_axis(x3 - 2, d.n3) : x3 - 2) * S};
    const int lo = 2 * x1 + 1, hi = 2 * d.n1 - 1 - 2 * x1;
    static_for<0, Q>([&](auto q) {
        constexpr int c1 = CV[q][0], c2 = CV[q][1], c3 = CV[q][2];
        constexpr int a1 = c1 < 0 ? -c1 : c1, a2 = c2 < 0 ? -c2 : c2, a3 = c3 < 0 ? -c3 : c3;
        constexpr int m = a1 > a2 ? (a1 > a3 ? a1 : a3) : (a2 > a3 ? a2 : a3);
        uint32_t rowoff, inrow;
        int srow = x1, splane = q;                      // uniform source row and plane
        if constexpr (c1 == 0) {
            rowoff = ((uint32_t)x1 * (uint32_t)Q + (uint32_t)q) * PS;
            inrow = L.o2[cslot(c2)] + L.o3[cslot(c3)];
        } else {
            constexpr int qo = opposite(q);
            constexpr int h1 = c1 / m, h2 = c2 / m, h3 = c3 / m;
            const int back = c1 > 0 ? lo : hi;
            if (back >= 2 * m) {                        // no crossing: the plain pull
                srow = x1 - c1;
                rowoff = ((uint32_t)srow * (uint32_t)Q + (uint32_t)q) * PS;
                inrow = L.o2[cslot(c2)] + L.o3[cslot(c3)];
            } else {                                    // reflected: plane qo at x - (c/m) sb
                const int sb = back - m;                // -2, 0 or 2 (m = 3), 0 (m = 1)
                srow = x1 - h1 * sb;
                splane = qo;
                rowoff = ((uint32_t)srow * (uint32_t)Q + (uint32_t)qo) * PS;
                const int k = sb == 0 ? 1 : (sb > 0 ? 2 : 0);   // index of t = sb
                const int k2 = h2 == 0 ? 1 : (h2 > 0 ? k : 2 - k), k3 = h3 == 0 ? 1 : (h3 > 0 ? k : 2 - k);
                inrow = (k2 == 0 ? o2s[0] : (k2 == 1 ? o2s[1] : o2s[2])) + (k3 == 0 ? o3s[0] : (k3 == 1 ? o3s[1] : o3s[2]));
            }
        }
        const C r = Codec<ST>::REF ? (C)ref.get_r(x1 - srow, srow, splane) : C(0);
        g[q] = Codec<ST>::decode(gload<T>(src, (uint64_t)(rowoff + inrow)), r);
    });
}

// Source of a pull when a wall may be within reach.  Ticks of 1/(2m) step
// (m = max |c_a|) put the walls at odd and the nodes at even tick counts.
// The backward trajectory from x along -c runs inside [-front, back]; it is
// unfolded to y = front + 2m and folded back into [0, L], L = back + front:
// crossings n_c = floor(y / L), every crossing reverses the velocity.
// Returns the source storage column x2*n3p + x3 within the source row
// (written to row).
template <int C1, int C2, int C3, bool OPEN2 = true>
__host__ __device__ __forceinline__ int fold_source(const InstDesc &d, int x1, int x2, int x3, bool &flip,
                                                    int &row)
{
    constexpr int a1 = C1 < 0 ? -C1 : C1, a2 = C2 < 0 ? -C2 : C2, a3 = C3 < 0 ? -C3 : C3;
    constexpr int m = a1 > a2 ? (a1 > a3 ? a1 : a3) : (a2 > a3 ? a2 : a3);
    flip = false;
    if constexpr (m == 0) {
        row = x1;
        return x2 * d.n3p + x3;
    } else {
        constexpr int h1 = C1 / m, h2 = C2 / m, h3 = C3 / m;
        if (d.eqwall) {   // wall nodes on axis 1 (clamped pull), x3 periodic
            int s1 = x1 - C1;
            s1 = s1 < 0 ? 0 : (s1 > d.n1 - 1 ? d.n1 - 1 : s1);
            row = s1;
            return axis2(x2 - C2, d.n2, OPEN2 && (d.walls & 16)) * d.n3p + wrap_axis(x3 - C3, d.n3);
        }
        int back = 1 << 28, front = 1 << 28;
        if constexpr (C1 != 0) {
            if (d.walls & 1) {
                const int lo = 2 * x1 + 1, hi = 2 * d.n1 - 1 - 2 * x1;
                back = C1 > 0 ? lo : hi;
                front = C1 > 0 ? hi : lo;
            }
        }
        if constexpr (C3 != 0) {
            if (d.walls & 4) {
                const int lo = 2 * x3 + 1, hi = 2 * d.n3 - 1 - 2 * x3;
                const int b3 = C3 > 0 ? lo : hi, f3 = C3 > 0 ? hi : lo;
                back = b3 < back ? b3 : back;
                front = f3 < front ? f3 : front;
            }
        }
        int sb = m;   // unit steps back along chat
        if (back < 2 * m) {
            const int L = back + front;
            const int y = front + 2 * m;
            int nc = 0;
#pragma unroll
            for (int it = 0; it < 4; ++it) nc += (y > (nc + 1) * L) ? 1 : 0;
            const int yf = (nc & 1) ? (nc + 1) * L - y : y - nc * L;
            sb = (yf - front) / 2;
            flip = nc & 1;
        }
        int s1 = x1 - h1 * sb, s2 = x2 - h2 * sb, s3 = x3 - h3 * sb;
        if (!(d.walls & 1)) s1 = wrap_axis(s1, d.n1);
        s2 = axis2(s2, d.n2, OPEN2 && (d.walls & 16));
        if (!(d.walls & 4)) s3 = wrap_axis(s3, d.n3);
        row = s1;
        return s2 * d.n3p + s3;
    }
}

// General pull (any lane position, walls on any axis).
template <int ST, bool OPEN2 = true, class R>
__device__ __forceinline__ void gather_general(const void *src, const InstDesc &d, int x1, int x2, int x3,
                                               const R &ref, typename Codec<ST>::G (&g)[Q])
{
    using T = typename Codec<ST>::T;
    using C = typename Codec<ST>::C;
    constexpr uint32_t S = sizeof(T);
    static_for<0, Q>([&](auto q) {
        constexpr int qo = opposite(q);
        bool flip;
        int row;
        const int col = fold_source<CV[q][0], CV[q][1], CV[q][2], OPEN2>(d, x1, x2, x3, flip, row);
        const uint32_t qs = flip ? (uint32_t)qo : (uint32_t)q;
        const uint32_t e = ((uint32_t)row * (uint32_t)Q + qs) * (uint32_t)d.Pp + (uint32_t)col;
        C r = C(0);
        if constexpr (Codec<ST>::REF) r = (C)RefRow{d.ref}.get_r(0, row, (int)qs);   // per-lane row
        g[q] = Codec<ST>::decode(gload<T>(src, (uint64_t)(e * S)), r);
    });
}

}  // namespace mlbm
