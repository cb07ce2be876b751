// Fused collide-and-stream step for gfx950 (Sec. II, Eq. (3)).
//
// One workgroup processes one tile: `blockDim.x` consecutive columns of the
// (x2, x3) plane of one x1 row of one instance.  Because x1 is uniform per
// wavefront, the choice between the plain pull and the bounce-back pull,
// the source row x1 - c1 and the geometry of x3-independent cases are
// scalar; only the in-row offset of a pull is per lane, so the 41 loads of a
// node are coalesced runs along x3. Wavefronts next to an x3 wall take a
// branch-free variant that resolves the single x3 reflection per lane, rows
// next to an x1 wall one whose reflections are uniform per wavefront;
// wavefronts at a corner of both take the general fold.  The launch is persistent: workgroups
// stride over the flat tile queue of all active instances (grouped by XCD
// for the 16-bit formats), and the number of queued tiles is read from device memory so that a
// captured graph stays valid when instances retire.
//
// With equilibrium walls (Sec. III) the first and last x1 rows are wall
// nodes: pulls from beyond them read the wall row, and a wall row is set to
// the equilibrium at zero velocity instead of colliding. That branch is
// compiled only into the EQW variant: merged into the plain kernel it costs
// some 30 registers per lane and one wave per SIMD of occupancy.
//
// The CHECK variant (every K-th step) also writes the lattice velocity the
// collision used to the snapshot buffer and reduces, per tile, the squared
// change against the previous snapshot, the squared velocity and an
// instability flag (wavefront shuffles, then LDS, fixed order: results are
// bitwise reproducible).
#pragma once

#include "core.hpp"
#include "kernels.hpp"

namespace mlbm {

template <int PAT, int ST, bool CHECK, bool EQW>
__global__ void __launch_bounds__(512) step_kernel(StepArgs a)
{
    using T = typename Codec<ST>::T;
    using C = typename Codec<ST>::C;
    // open theta ends are served by the general-pattern kernels only (a batch
    // with an open instance runs them); the others compile the periodic wrap
    constexpr bool OPEN2 = PAT == PAT_GEN;
    __shared__ double red[8][3];

    const int ntiles = load_uniform(a.ntiles);
    // Workgroups go to the 8 XCDs round-robin (v mod 8), and each XCD has
    // its own L2. Neighbouring tiles of a row share the cache lines that
    // their x3 pulls straddle; with xcd_group each XCD takes one contiguous
    // eighth of the queue instead of every eighth tile, so that a straddled
    // line is fetched once, not by two XCDs. Without it the queue is dealt
    // to the XCDs in runs of G = 2^group_log2 consecutive tiles (G = 1:
    // every eighth tile): the tiles of one run, neighbours in a row, share
    // the straddled lines and the cross-section geometry in one L2 while
    // all XCDs still stream through neighbouring memory; the last
    // ntiles mod 8G tiles keep their order. (Both maps are bijections of
    // [0, ntiles); with a persistent grid that is a multiple of 8 the
    // grouping holds on every pass.)
    const int per = ntiles >> 3, rem = ntiles & 7;
    const int lg = a.group_log2, full = ntiles & ~((8 << lg) - 1);
    for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
        const int xcd = v & 7, s = v >> 3;
        const int t = a.xcd_group ? xcd * per + min(xcd, rem) + s
                                  : (v < full ? ((((s >> lg) << 3) + xcd) << lg) | (s & ((1 << lg) - 1)) : v);
        const Tile tl = load_uniform(a.tiles + t);
        const InstDesc d = load_uniform(a.insts + tl.inst);
        const int x1 = tl.x1;
        // storage column col = x2 * n3p + x3s. Lanes on the x3 padding
        // (x3s >= n3) repeat the row's last node and store the copy into the
        // padding, so that every 64-byte segment of a row is written whole
        // (a partly written segment costs the memory a read-modify-write:
        // 19 % of the step time at n3 = 113); nothing ever reads the copies.
        const int lane = tl.chunk * (int)blockDim.x + (int)threadIdx.x;
        const bool valid = lane < d.Pp;              // the lane owns a storage column
        const int col = valid ? lane : 0;
        const int x2 = (int)(((uint64_t)col * d.n3_magic) >> 40);
        const int x3s = col - x2 * d.n3p;
        const int x3 = x3s < d.n3 ? x3s : d.n3 - 1;
        const bool real = valid && x3s < d.n3;       // ... that holds a node
        // selects, not an indexed read: a run-time index into the local copy
        // of the descriptor would move the whole copy to scratch memory
        const void *src = a.parity ? d.f[1] : d.f[0];
        void *dst = a.parity ? d.f[0] : d.f[1];
        constexpr uint32_t S = sizeof(T);
        const RefScalar R{d.ref};
        uint32_t ctr = 0;                      // step counter of the stochastic rounding
        if constexpr (Codec<ST>::REF) {
            ctr = gload<uint32_t>(d.ctr, 4ull * (uint32_t)a.parity);
            // the instance's first tile advances the counter for the next step
            // (nothing reads that entry during this step)
            if (x1 == 0 && tl.chunk == 0 && threadIdx.x == 0)
                gstore<uint32_t>(d.ctr, 4ull * (uint32_t)(a.parity ^ 1), ctr + 1u);
        }

        // bounce-back rows within reach of an x1 wall; equilibrium walls pull
        // through clamped rows in the fast gather instead
        const bool wall1_row = (d.walls & 1) && !d.eqwall && (x1 < 3 || x1 > d.n1 - 4);
        const bool eq_row = EQW && d.eqwall && (x1 == 0 || x1 == d.n1 - 1);   // a wall-node row
        const bool near3 = valid && (d.walls & 4) && (x3 < 3 || x3 > d.n3 - 4);
        const bool any3 = __ballot(near3) != 0;

        double dsq = 0.0, usq = 0.0, badf = 0.0;
        if (valid) {
            typename Codec<ST>::G g[Q];
            if (!wall1_row && !any3 && (d.walls & 4)) {
                gather_fast_walled3<ST, EQW, OPEN2>(src, d, x1, x2, x3, R, g);
            } else if (!wall1_row && !any3) {
                LaneOffsets L;
                L.init(x2, x3, d.n2, d.n3, d.n3p, true, OPEN2 && (d.walls & 16), S);
                gather_fast<ST, EQW>(src, d, x1, L, R, g);
            } else if (!wall1_row && d.n3 >= 5) {
                LaneOffsets L;
                L.init(x2, x3, d.n2, d.n3, d.n3p, false, OPEN2 && (d.walls & 16), S);
                gather_x3wall<ST, OPEN2>(src, d, x1, x2, x3, L, R, g);
            } else if (!any3) {
                LaneOffsets L;
                L.init(x2, x3, d.n2, d.n3, d.n3p, !(d.walls & 4), OPEN2 && (d.walls & 16), S);
                gather_x1wall<ST, OPEN2>(src, d, x1, x2, x3, L, R, g);
            } else {
                gather_general<ST, OPEN2>(src, d, x1, x2, x3, R, g);
            }
            // per cross-section geometry; only the general pattern may depend on theta
            const int gidx = PAT == PAT_GEN ? geo_index(d, x1, x2, x3) : x1 * d.n3g + (d.n3g > 1 ? x3 : 0);
            const int gstride = PAT == PAT_GEN ? geo_stride(d) : d.n1 * d.n3g;
            NodeGeo<PAT, C> geo;
            geo.load(d.geo, d.geof, gidx, gstride, (C)d.force, PAT == PAT_GEN ? gidx : x1 * d.n3g);
            C rho, u[3];
            if (eq_row) {
                wall_equilibrium<PAT, C, typename Codec<ST>::G, Codec<ST>::SCALED>(g, geo, rho);
                u[0] = u[1] = u[2] = C(0);
            } else {
                collide<PAT, C, typename Codec<ST>::G, Codec<ST>::SCALED>(g, geo, (C)d.omega, (C)d.kappa, rho, u);
            }
            const size_t n = (size_t)x1 * d.P + (size_t)x2 * d.n3 + x3;   // node index
            void *drow = (char *)dst + pop_elem(0, x1, 0, d.Pp) * S;
            const uint32_t loff = (uint32_t)col * S;
            if constexpr (Codec<ST>::REF) {
                const RoundBits rb(d.salt, (uint32_t)n, ctr);
                static_for<0, Q>([&](auto q) {
                    void *plane = (char *)drow + (uint64_t)q * (uint64_t)d.Pp * S;
                    gstore_nt<T>(plane, loff,
                                 Codec<ST>::encode_sr(g[q], (C)R.get_r(0, x1, q), rb.template get<q>()));
                });
            } else {
                static_for<0, Q>([&](auto q) {
                    void *plane = (char *)drow + (uint64_t)q * (uint64_t)d.Pp * S;
                    gstore_nt<T>(plane, loff, Codec<ST>::encode(g[q], C(0)));
                });
            }
            if (CHECK && real) {
                double *us = d.usnap;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double v = (double)u[i];
                    const uint64_t off = 8ull * ((uint64_t)i * d.N + n);
                    const double dv = v - gload<double>(us, off);
                    dsq += dv * dv;
                    usq += v * v;
                    if (!(fabs(v) <= 1.0)) badf = 1.0;
                    gstore<double>(us, off, v);
                }
                if (!(rho > C(0))) badf = 1.0;
            }
        }
        if constexpr (CHECK) {
            for (int off = 32; off > 0; off >>= 1) {
                dsq += __shfl_xor(dsq, off, 64);
                usq += __shfl_xor(usq, off, 64);
                badf += __shfl_xor(badf, off, 64);
            }
            const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
            if (lane == 0) { red[wave][0] = dsq; red[wave][1] = usq; red[wave][2] = badf; }
            __syncthreads();
            if (threadIdx.x == 0) {
                double s0 = 0.0, s1 = 0.0, s2 = 0.0;
                const int nw = (blockDim.x + 63) >> 6;
                for (int w = 0; w < nw; ++w) { s0 += red[w][0]; s1 += red[w][1]; s2 += red[w][2]; }
                a.partials[3 * tl.part + 0] = s0;
                a.partials[3 * tl.part + 1] = s1;
                a.partials[3 * tl.part + 2] = s2;
            }
            __syncthreads();
        }
    }
}

}  // namespace mlbm
