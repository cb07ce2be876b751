// Host-visible launchers of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace mlbm {

struct StepArgs {
    const InstDesc *insts;   // device array of instance descriptors
    const Tile *tiles;       // device tile queue
    const int *ntiles;       // device: number of queued tiles
    double *partials;        // [tiles][3] check sums
    int parity;              // read f[parity], write f[parity ^ 1]
    int xcd_group = 0;       // 1: each XCD takes a contiguous eighth of the tile queue
    int group_log2 = 0;      // else: runs of 2^group_log2 consecutive tiles per XCD, interleaved
};

hipError_t launch_step(const StepArgs &a, int pat, int st, bool check, bool eqw, int grid, int block, hipStream_t s);
// the two compiled variants (eqw: with the equilibrium-wall rows)
hipError_t launch_step_plain(const StepArgs &a, int pat, int st, bool check, int grid, int block, hipStream_t s);
hipError_t launch_step_eq(const StepArgs &a, int pat, int st, bool check, int grid, int block, hipStream_t s);

// geometry of one instance (FP64, on the device)
struct GeoParams {
    int kind, n1, n2, n3, n2g, n3g;
    int eqwall;    // node placement of equilibrium walls (wall nodes at r_i, r_o)
    double r_inner, width, b, dt, s[3];
};
hipError_t launch_geometry(double *geo, const GeoParams &p, hipStream_t s);

// f* = f_eq(rho' = 1/sqrt(g), u) for one instance; init_u (device, physical
// [3][N]) may be null
hipError_t launch_geo_to_f32(const double *geo, float *geof, long count, hipStream_t s);
hipError_t launch_ref(const InstDesc *d_desc, const InstDesc &h_desc, const double *init_u, float *ref,
                      hipStream_t s);
hipError_t launch_init(const InstDesc *d_desc, const InstDesc &h_desc, int st, const double *init_u,
                       int parity, hipStream_t s);
// 16-bit storage: re-take the row means r from the current state (buffer
// `parity`) and re-encode the stored values against them, in place
hipError_t launch_reref(const InstDesc *d_desc, const InstDesc &h_desc, int st, int parity, float *ref,
                        hipStream_t s);

// residual / flag reduction over the partial sums of each instance's tiles
hipError_t launch_reduce(const double *partials, const int *part_begin, const int *part_count,
                         WindowState *ws, int ninst, hipStream_t s);

// moments of the streamed state: rho = rho' sqrt(g), u = s_i U^i (physical)
hipError_t launch_moments(const InstDesc *d_desc, const InstDesc &h_desc, int st, int parity,
                          double *rho, double *u, hipStream_t s);

// observables: partial sums [blocks][3] of (v numerator, omega numerator, area)
// over the nodes of the theta slabs x2lo <= x2 < x2hi
hipError_t launch_vortex(const InstDesc &h_desc, int kind, double b, double h1, double h3, int x2lo, int x2hi,
                         const double *u, double *partials, int *nblocks, hipStream_t s);
// out[0..2] = sums of the partial triples over blocks 0..nb-1, in block order
hipError_t launch_sum_partials(const double *partials, int nb, double *out, hipStream_t s);

// decode (storage -> absolute FP64 f) and encode
hipError_t launch_decode(const InstDesc &h_desc, int st, int parity, double *f, hipStream_t s);
hipError_t launch_encode(const InstDesc &h_desc, int st, int parity, const double *f, hipStream_t s);

// one update of a list of nodes from the current state (no write-back)
hipError_t launch_step_nodes(const InstDesc *d_desc, const InstDesc &h_desc, int pat, int st, int parity,
                             const int64_t *nodes, int64_t count, double *out, hipStream_t s);

}  // namespace mlbm
