// Device-side data layout shared by the kernels and the host runtime.
//
// HBM layout of one instance:
//   populations  two buffers (pull: read one, write the other), each
//                [n1][41][n2][n3p] of the storage type (the 41 planes of an
//                x1 row together), x3 fastest, with the x3 pitch n3p = n3
//                rounded up to 16 values so that every x2 row of every plane
//                starts on a 64-byte boundary (odd n3 cost a third of the
//                step kernel's throughput); the padding is never read.  Stored
//                values are offsets from the lattice weights: g = f - w_q
//                for FP64/FP32, d = f / w_q - 1 - r for FP16/BF16 (r: the
//                row's reference offset of the population).
//   geometry     FP64, structure of arrays [NGEO][n1][n2g][n3g] (n3g = 1
//                when nothing depends on x3, e.g. the cylinder; n2g = n2 only
//                for the full ellipsoid, whose metric depends on theta):
//                Delta^ij = g^ij - delta^ij, Christoffels, unit force,
//                sqrt(g) and coordinates.  Read through L2.
//   usnap        FP64 [3][N], lattice velocity at the previous check.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlbm {

enum GeoField {
    G_D11, G_D12, G_D13, G_D22, G_D23, G_D33,               // Delta^ij (upper)
    G_1_11, G_1_12, G_1_13, G_1_22, G_1_23, G_1_33,         // Gamma^1_jk (lattice)
    G_2_11, G_2_12, G_2_13, G_2_22, G_2_23, G_2_33,         // Gamma^2_jk
    G_3_11, G_3_12, G_3_13, G_3_22, G_3_23, G_3_33,         // Gamma^3_jk
    G_F1, G_F2, G_F3,                                       // force per unit K (lattice)
    G_SQRTG,                                                // sqrt(det g) (lattice)
    G_X1, G_X3,                                             // physical x1, x3 of the node
    NGEO
};

// Geometry sparsity the step kernel is compiled for.
enum Pattern {
    PAT_CYL = 0,   // diagonal metric, Gamma^1_22 and Gamma^2_12 only (flat, cylinder)
    PAT_ELL = 1,   // diagonal metric, the six Christoffels of the ellipsoid
    PAT_GEN = 2,   // full metric and all 18 Christoffels
};

enum Storage { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3, ST_F32D = 4 };

struct InstDesc {
    void *f[2];            // population buffers
    const double *geo;     // [NGEO][n1*n3g]
    const float *geof;     // the same geometry rounded to FP32 (read by FP32 arithmetic)
    double *usnap;         // [3][N]
    const float *ref;      // FP16/BF16 storage: per-row reference r [n1][41]; else null
    uint32_t *ctr;         // FP16/BF16 storage: step counter [2] (read [parity], next in [parity ^ 1])
    uint32_t salt;         // per-instance key of the stochastic rounding
    int n1, n2, n3, walls;
    int eqwall;            // 1: the x1 walls are equilibrium walls (wall-node rows 0 and n1 - 1)
    int P, N;              // n2*n3, n1*n2*n3 (node count; node n = (x1*n2 + x2)*n3 + x3)
    int n3p, Pp;           // storage pitch of x3 (n3 rounded up to 16) and of a plane (n2*n3p)
    int n3g;               // 1 or n3
    int n2g;               // 1, or n2 when the metric depends on theta (full ellipsoid)
    int tpr;               // tiles per x1 row (over the Pp storage columns)
    uint64_t n3_magic;     // ceil(2^40 / n3p): col / n3p = (col * magic) >> 40 for storage columns
    double omega;          // 1 / tau
    double kappa;          // 1 - 1/(2 tau) (improved forcing) or 0 (old)
    double force;          // covariant body force K
    double s[3];           // scale factors Dx^i / Dt
};

// One tile: a run of `block` columns of one x1 row of one instance.
struct Tile {
    int inst, x1, chunk, part;   // part: index of its partial sums
};

struct WindowState {           // per instance, device resident
    double residual;           // last residual (-1 before two checks)
    int checks;                // checks done
    int bad;                   // sticky instability flag
};

// --- global-memory access ------------------------------------------------
// Pointers that live inside descriptors are generic to the compiler, which
// then emits flat loads.  Casting them to the global address space lets it
// use global loads with a scalar base and a 32-bit per-lane byte offset.
#define MLBM_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ T gload(const void *base, uint64_t byte_off)
{
    return *(const MLBM_GLOBAL T *)((const MLBM_GLOBAL char *)base + byte_off);
}

template <class T>
__device__ __forceinline__ void gstore(void *base, uint64_t byte_off, T v)
{
    *(MLBM_GLOBAL T *)((MLBM_GLOBAL char *)base + byte_off) = v;
}

// Tables that no kernel writes while it runs (instance descriptors, the
// tile queue, the 16-bit reference rows). Read through the constant address
// space with a wavefront-uniform address they become scalar loads into
// SGPRs. Read as plain global memory behind the kernel's own stores, the
// compiler cannot prove them unchanged between loop iterations: it reloads
// each field with a vector load and a wait where it is used, and carries the
// arithmetic on it in VGPRs.
#define MLBM_CONST __attribute__((address_space(4)))

template <class T>
__device__ __forceinline__ T load_uniform(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized records only");
    uint32_t w[sizeof(T) / 4];
    const MLBM_CONST uint32_t *s = (const MLBM_CONST uint32_t *)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = s[i];
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}

// Store that is not expected to be read again soon (streamed output).
template <typename T>
__device__ __forceinline__ void gstore_nt(void *base, uint64_t byte_off, T v)
{
    __builtin_nontemporal_store(v, (MLBM_GLOBAL T *)((MLBM_GLOBAL char *)base + byte_off));
}

// --- storage codecs ------------------------------------------------------

__device__ __forceinline__ float bf16_bits_to_float(uint16_t h)
{
    return __uint_as_float(((uint32_t)h) << 16);
}

// round to nearest even; NaN stays NaN (a select, not a branch)
__device__ __forceinline__ uint16_t float_to_bf16_bits(float x)
{
    const uint32_t u = __float_as_uint(x);
    const uint32_t rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const uint32_t quiet = (u >> 16) | 0x40u;
    return (uint16_t)(((u & 0x7fffffffu) > 0x7f800000u) ? quiet : rounded);
}

__device__ __forceinline__ float f16_bits_to_float(uint16_t h) { return __half2float(__ushort_as_half(h)); }
__device__ __forceinline__ uint16_t float_to_f16_bits(float x) { return __half_as_ushort(__float2half_rn(x)); }

// Stochastic rounding with the CDNA4 conversions v_cvt_sr_f16_f32 and
// v_cvt_sr_bf16_f32: the magnitude of x is rounded up with probability
// equal to the dropped fraction, taken from the top bits of `seed` (13 of
// them for binary16, 16 for bfloat16; a seed whose random bits sit in the
// low half always truncates -- measured on the part). Each rounding is
// unbiased, so increments below the storage resolution (the per-step body
// force, for one) are kept on average instead of being lost.
// The builtins write one half of a register pair whose other half they
// keep, which costs a register copy per conversion; only the low half is
// stored here, so the instruction is issued directly with a fresh result
// register (an arithmetic instruction: no memory access, no wait needed).
__device__ __forceinline__ uint16_t float_to_f16_bits_sr(float x, uint32_t seed)
{
    uint32_t v;
    asm("v_cvt_sr_f16_f32 %0, %1, %2" : "=v"(v) : "v"(x), "v"(seed));
    return (uint16_t)v;
}
__device__ __forceinline__ uint16_t float_to_bf16_bits_sr(float x, uint32_t seed)
{
    uint32_t v;
    asm("v_cvt_sr_bf16_f32 %0, %1, %2" : "=v"(v) : "v"(x), "v"(seed));
    return (uint16_t)v;
}

// 32-bit integer hash (xorshift-multiply, two rounds): the published
// "lowbias32" constants of C. Wellons' hash-prospector search.
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// T: stored type; C: compute type; G: register type of the 41 populations.
// In registers a population is the offset g = f - w (w = its weight) for the
// wide formats, and the scaled offset h = f / w - 1 for the 16-bit formats
// (SCALED). Those store d = h - r, where r is the reference offset of the
// population in the row the value is stored in (REF): decode(v, r) gives the
// register value, encode(x, r) the stored one; the wide formats ignore r.
// to_f64 / from_f64 convert between stored values and FP64 offsets g.
template <int ST> struct Codec;

template <> struct Codec<ST_F64> {
    using T = double;
    using C = double;
    using G = double;
    static constexpr bool REF = false;
    static constexpr bool SCALED = false;
    __device__ static __forceinline__ C decode(T v, C) { return v; }
    __device__ static __forceinline__ T encode(G g, C) { return g; }
    __device__ static __forceinline__ T encode_sr(G g, C, uint32_t) { return g; }
    __device__ static __forceinline__ double to_f64(T v, double, double) { return v; }
    __device__ static __forceinline__ T from_f64(double g, double, double) { return g; }
};

template <> struct Codec<ST_F32> {
    using T = float;
    using C = float;
    using G = float;
    static constexpr bool REF = false;
    static constexpr bool SCALED = false;
    __device__ static __forceinline__ C decode(T v, C) { return v; }
    __device__ static __forceinline__ T encode(G g, C) { return g; }
    __device__ static __forceinline__ T encode_sr(G g, C, uint32_t) { return g; }
    __device__ static __forceinline__ double to_f64(T v, double, double) { return (double)v; }
    __device__ static __forceinline__ T from_f64(double g, double, double) { return (float)g; }
};

template <> struct Codec<ST_F32D> {   // FP32 storage, FP64 collision, FP32 registers
    using T = float;
    using C = double;
    using G = float;
    static constexpr bool REF = false;
    static constexpr bool SCALED = false;
    __device__ static __forceinline__ G decode(T v, C) { return v; }
    __device__ static __forceinline__ T encode(G g, C) { return g; }
    __device__ static __forceinline__ T encode_sr(G g, C, uint32_t) { return g; }
    __device__ static __forceinline__ double to_f64(T v, double, double) { return (double)v; }
    __device__ static __forceinline__ T from_f64(double g, double, double) { return (float)g; }
};

template <> struct Codec<ST_F16> {
    using T = uint16_t;    // IEEE binary16 bits of d = f / w - 1 - r
    using C = float;
    using G = float;
    static constexpr bool REF = true;
    static constexpr bool SCALED = true;
    __device__ static __forceinline__ C decode(T v, C r) { return f16_bits_to_float(v) + r; }
    // decode with a wavefront-uniform r (a scalar register): one mixed-precision
    // FMA, d * 1 + r with d read as binary16, instead of a conversion and an add
    // (the same single rounding of d + r, so the same result)
    __device__ static __forceinline__ C decode_uniform(T v, C r)
    {
        float x;
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(x) : "v"((uint32_t)v), "s"(r));
        return x;
    }
    // the same with r chosen per lane (a vector register)
    __device__ static __forceinline__ C decode_lane(T v, C r)
    {
        float x;
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(x) : "v"((uint32_t)v), "v"(r));
        return x;
    }
    __device__ static __forceinline__ T encode(G h, C r) { return float_to_f16_bits(h - r); }
    __device__ static __forceinline__ T encode_sr(G h, C r, uint32_t rnd) { return float_to_f16_bits_sr(h - r, rnd); }
    __device__ static __forceinline__ double to_f64(T v, double w, double r)
    {
        return w * ((double)f16_bits_to_float(v) + r);
    }
    __device__ static __forceinline__ T from_f64(double g, double w, double r)
    {
        return float_to_f16_bits((float)(g / w - r));
    }
};

template <> struct Codec<ST_BF16> {
    using T = uint16_t;    // bfloat16 bits of d = f / w - 1 - r
    using C = float;
    using G = float;
    static constexpr bool REF = true;
    static constexpr bool SCALED = true;
    __device__ static __forceinline__ C decode(T v, C r) { return bf16_bits_to_float(v) + r; }
    __device__ static __forceinline__ T encode(G h, C r) { return float_to_bf16_bits(h - r); }
    __device__ static __forceinline__ T encode_sr(G h, C r, uint32_t rnd) { return float_to_bf16_bits_sr(h - r, rnd); }
    __device__ static __forceinline__ double to_f64(T v, double w, double r)
    {
        return w * ((double)bf16_bits_to_float(v) + r);
    }
    __device__ static __forceinline__ T from_f64(double g, double w, double r)
    {
        return float_to_bf16_bits((float)(g / w - r));
    }
};

inline size_t storage_bytes(int st) { return st == ST_F64 ? 8 : (st == ST_F32 || st == ST_F32D) ? 4 : 2; }

}  // namespace mlbm
