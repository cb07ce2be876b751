// Learned warm start: a small fully connected network, trained and run on
// the GPU by the kernels below.
//
// Network: 5 inputs -> H -> ... -> H -> 3 outputs (`depth` hidden layers,
// SiLU s(z) = z / (1 + exp(-z)), linear output), FP32.  Parameters are laid
// out per layer as W [n_out][n_in] row-major followed by b [n_out].
//
// Inputs of a cross-section node of a case: (De / 100, R1/d / 20,
// ln(R2/R1) / ln 4, 2 (r - r_i)/d - 1, arc position / (2 d)) where the arc
// position is phi r_i (ellipsoid) or z - L/2 (cylinder, flat).  Outputs:
// the physical velocity components (u^r, sqrt(g_thth) u^th, sqrt(g_33) u^3)
// divided by the nominal mean speed of the case.
//
// Training: minibatches drawn by a counter-based hash, forward pass that
// keeps the hidden activations, per-sample backpropagation, weight
// gradients summed over samples in fixed order (chunk partial sums, then a
// second pass), Adam.  Every reduction has a fixed order, so training is
// bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mlbm.h"

namespace {

constexpr int NIN = 5, NOUT = 3, MAXDEPTH = 6, CHUNK = 64;

thread_local std::string g_net_err;

mlbm_status nfail(mlbm_status s, const std::string &m)
{
    g_net_err = m;
    return s;
}

#define NET_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return nfail(e_ == hipErrorOutOfMemory ? MLBM_E_OOM : MLBM_E_HIP,                           \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                            \
    } while (0)

// Device memory owned by one call: freed on every return path, once the
// stream is done with it.
struct CallBuf {
    hipStream_t s;
    void *p = nullptr;
    explicit CallBuf(hipStream_t st) : s(st) {}
    ~CallBuf()
    {
        if (p) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(p);
        }
    }
    CallBuf(const CallBuf &) = delete;
    CallBuf &operator=(const CallBuf &) = delete;
};

struct Shape {
    int H, depth;
    long np;
    long off[MAXDEPTH + 2];
    __host__ __device__ int nin(int l) const { return l == 0 ? NIN : H; }
    __host__ __device__ int nout(int l) const { return l == depth ? NOUT : H; }
};

Shape make_shape(int H, int depth)
{
    Shape s{};
    s.H = H;
    s.depth = depth;
    long o = 0;
    for (int l = 0; l <= depth; ++l) {
        s.off[l] = o;
        o += (long)s.nout(l) * s.nin(l) + s.nout(l);
    }
    s.off[depth + 1] = o;
    s.np = o;
    return s;
}

uint64_t mix64_host(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z)
{
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Forward pass, one thread per sample, parameters staged in LDS (every lane
// reads the same weight: broadcast, no bank conflicts).  If `hid` is given
// the hidden pre-activations are kept for backpropagation ([n][depth][H]).
// The launch bound (the CHUNK-thread blocks it always runs with) lets the
// compiler keep a sample's activations in registers: without it the default
// 1024-thread bound caps a lane at 128 VGPRs and the arrays spill to scratch.
template <int H>
__global__ __launch_bounds__(CHUNK) void forward_kernel(const float *p, Shape sh, const float *X, int64_t M, uint64_t seed, int64_t n,
                               float *Y, float *hid, int64_t *sel)
{
    extern __shared__ float sp[];
    for (long k = threadIdx.x; k < sh.np; k += blockDim.x) sp[k] = p[k];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t src = seed ? (int64_t)(mix64(seed ^ (uint64_t)s) % (uint64_t)M) : s;
    if (sel) sel[s] = src;
    float a[H], z[H];
#pragma unroll
    for (int i = 0; i < NIN; ++i) a[i] = X[src * NIN + i];
    for (int l = 0; l <= sh.depth; ++l) {
        const int ni = sh.nin(l), no = sh.nout(l);
        const float *W = sp + sh.off[l], *b = W + no * ni;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            if (j < no) {
                float acc = b[j];
                if (ni == NIN) {
#pragma unroll
                    for (int i = 0; i < NIN; ++i) acc += W[j * NIN + i] * a[i];
                } else {
#pragma unroll
                    for (int i = 0; i < H; ++i) acc += W[j * H + i] * a[i];
                }
                z[j] = acc;
            }
        }
        if (l == sh.depth) {
#pragma unroll
            for (int j = 0; j < NOUT; ++j) Y[s * NOUT + j] = z[j];
        } else {
#pragma unroll
            for (int j = 0; j < H; ++j) {
                if (hid) hid[(s * sh.depth + l) * H + j] = z[j];
                a[j] = silu(z[j]);
            }
        }
    }
}

// Backpropagation of L = 1/(3n) sum (y - t)^2: per-sample deltas of every
// layer's pre-activations, dl [n][depth + 1][H] (the output layer uses the
// first 3 entries of its slot), and per-chunk loss partial sums.
template <int H>
__global__ __launch_bounds__(CHUNK) void backward_kernel(const float *p, Shape sh, const float *T, const int64_t *sel, int64_t n,
                                const float *Y, const float *hid, float *dl, double *lossp)
{
    extern __shared__ float sp[];
    __shared__ double red[CHUNK / 64];
    for (long k = threadIdx.x; k < sh.np; k += blockDim.x) sp[k] = p[k];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double le = 0.0;
    if (s < n) {
        const int64_t src = sel[s];
        float d[H], dn[H];
        const float inv = 2.0f / (3.0f * (float)n);
#pragma unroll
        for (int j = 0; j < NOUT; ++j) {
            const float e = Y[s * NOUT + j] - T[src * NOUT + j];
            le += (double)e * (double)e;
            d[j] = inv * e;
            dl[(s * (sh.depth + 1) + sh.depth) * H + j] = d[j];
        }
        for (int l = sh.depth; l >= 1; --l) {
            const int ni = sh.nin(l), no = sh.nout(l);
            const float *W = sp + sh.off[l];
#pragma unroll
            for (int i = 0; i < H; ++i) {
                float acc = 0.0f;
                if (no == NOUT) {
#pragma unroll
                    for (int j = 0; j < NOUT; ++j) acc += W[j * ni + i] * d[j];
                } else {
#pragma unroll
                    for (int j = 0; j < H; ++j) acc += W[j * ni + i] * d[j];
                }
                dn[i] = acc * dsilu(hid[(s * sh.depth + (l - 1)) * H + i]);
            }
#pragma unroll
            for (int i = 0; i < H; ++i) {
                d[i] = dn[i];
                dl[(s * (sh.depth + 1) + (l - 1)) * H + i] = dn[i];
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) le += __shfl_xor(le, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = le;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        lossp[blockIdx.x] = t;
    }
}

// Weight and bias gradients: thread k owns parameter k, block row c sums
// the samples of chunk c (fixed order) into part[c][k].
__global__ void wgrad_kernel(Shape sh, const float *X, const int64_t *sel, int64_t n, const float *hid,
                             const float *dl, float *part)
{
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= sh.np) return;
    int l = 0;
    while (l < sh.depth && k >= sh.off[l + 1]) ++l;
    const int ni = sh.nin(l), no = sh.nout(l), H = sh.H;
    const long r = k - sh.off[l];
    const bool bias = r >= (long)no * ni;
    const int j = bias ? (int)(r - (long)no * ni) : (int)(r / ni);
    const int i = bias ? 0 : (int)(r % ni);
    const int64_t s0 = (int64_t)blockIdx.y * CHUNK, s1 = s0 + CHUNK < n ? s0 + CHUNK : n;
    float acc = 0.0f;
    for (int64_t s = s0; s < s1; ++s) {
        const float dj = dl[(s * (sh.depth + 1) + l) * H + j];
        float ai = 1.0f;
        if (!bias) ai = l == 0 ? X[sel[s] * NIN + i] : silu(hid[(s * sh.depth + (l - 1)) * H + i]);
        acc += dj * ai;
    }
    part[(long)blockIdx.y * sh.np + k] = acc;
}

__global__ void sum_parts_kernel(const float *part, int nparts, long np, float *g)
{
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    double acc = 0.0;
    for (int c = 0; c < nparts; ++c) acc += (double)part[(long)c * np + k];
    g[k] = (float)acc;
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, long np, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// ---- features, targets and predictions of a case ------------------------

struct CaseGeo {
    int kind, n1, n2, n3, eqwall;
    double r_inner, width, b, s2, s3;
    double f0, f1, f2;   // De/100, R1/d/20, ln(R2/R1)/ln 4
};

__device__ void node_geo(const CaseGeo &c, int x1, int x3, double &sq2, double &sq3, double &arc)
{
    // node placement of the solver: cell centred, or wall nodes at both ends
    const double dt = c.width / (c.eqwall ? c.n1 - 1 : c.n1);
    const double o1 = c.eqwall ? 0.0 : 0.5;
    const double r = c.kind == MLBM_FLAT ? (x1 + o1) * dt : c.r_inner + (x1 + o1) * dt;
    sq2 = 1.0; sq3 = 1.0;
    if (c.kind == MLBM_ELLIPSOID || c.kind == MLBM_ELLIPSOID_FULL) {
        const double ph = (x3 + 0.5 - 0.5 * c.n3) * dt * c.s3;
        sq2 = r * c.b * cos(ph);
        sq3 = r;
        arc = ph * c.r_inner;
    } else {
        if (c.kind == MLBM_CYLINDER) sq2 = r;
        arc = (x3 + 0.5 - 0.5 * c.n3) * dt;
    }
}

__global__ void features_kernel(CaseGeo c, float *X)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= c.n1 * c.n3) return;
    const int x1 = p / c.n3, x3 = p - x1 * c.n3;
    double sq2, sq3, arc;
    node_geo(c, x1, x3, sq2, sq3, arc);
    X[p * NIN + 0] = (float)c.f0;
    X[p * NIN + 1] = (float)c.f1;
    X[p * NIN + 2] = (float)c.f2;
    X[p * NIN + 3] = (float)(2.0 * (x1 + 0.5) / c.n1 - 1.0);
    X[p * NIN + 4] = (float)(arc / (2.0 * c.width));
}

// The cross-section components of a steady field are 1e-3 to 1e-1 of the
// streamwise speed; they are scaled up by SEC in the targets so that the
// squared-error loss weighs the secondary flow comparably to the streamwise
// profile, and scaled back in the prediction.
constexpr double SEC = 10.0;

// targets from a velocity field u [3][N] (theta slab 0): physical components
// over U, the cross-section ones times SEC
__global__ void targets_kernel(CaseGeo c, const double *u, double invU, float *T)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= c.n1 * c.n3) return;
    const int x1 = p / c.n3, x3 = p - x1 * c.n3;
    double sq2, sq3, arc;
    node_geo(c, x1, x3, sq2, sq3, arc);
    const long N = (long)c.n1 * c.n2 * c.n3;
    const long n = ((long)x1 * c.n2) * c.n3 + x3;
    T[p * NOUT + 0] = (float)(u[n] * invU * SEC);
    T[p * NOUT + 1] = (float)(u[N + n] * sq2 * invU);
    T[p * NOUT + 2] = (float)(u[2 * N + n] * sq3 * invU * SEC);
}

// prediction -> physical contravariant velocity on every theta slab
__global__ void predict_map_kernel(CaseGeo c, const float *Y, double U, double *u)
{
    const long N = (long)c.n1 * c.n2 * c.n3;
    const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x1 = (int)(n / ((long)c.n2 * c.n3)), x3 = (int)(n % c.n3);
    const int p = x1 * c.n3 + x3;
    double sq2, sq3, arc;
    node_geo(c, x1, x3, sq2, sq3, arc);
    u[n] = U * Y[p * NOUT + 0] / SEC;
    u[N + n] = U * Y[p * NOUT + 1] / sq2;
    u[2 * N + n] = U * Y[p * NOUT + 2] / (sq3 * SEC);
}

CaseGeo case_geo(const mlbm_desc &d, double De, double R1_d, double R2_d)
{
    CaseGeo c{};
    c.kind = d.kind; c.n1 = d.n1; c.n2 = d.n2; c.n3 = d.n3;
    c.eqwall = (d.walls & MLBM_WALL_EQUILIBRIUM) ? 1 : 0;
    c.r_inner = d.r_inner; c.width = d.width; c.b = d.b;
    const bool ell = d.kind == MLBM_ELLIPSOID || d.kind == MLBM_ELLIPSOID_FULL;
    c.s2 = ell ? 1.0 / (d.b * d.r_inner) : 1.0;
    c.s3 = ell ? 1.0 / d.r_inner : 1.0;
    c.f0 = De / 100.0;
    c.f1 = R1_d / 20.0;
    c.f2 = (R1_d > 0.0 && R2_d > 0.0) ? std::log(R2_d / R1_d) / std::log(4.0) : 0.0;
    return c;
}

}  // namespace

struct mlbm_net_s {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Shape sh{};
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    long t = 0;
    float *X = nullptr, *T = nullptr;
    int64_t M = 0, cap = 0;
    // per-batch scratch
    int64_t bcap = 0;
    float *Y = nullptr, *hid = nullptr, *dl = nullptr, *part = nullptr;
    int64_t *sel = nullptr;
    double *lossp = nullptr;
};

namespace {

template <class F>
hipError_t dispatch_H(int H, F &&f)
{
    if (H == 32) return f(std::integral_constant<int, 32>{});
    if (H == 64) return f(std::integral_constant<int, 64>{});
    return hipErrorInvalidValue;
}

mlbm_status ensure_batch(mlbm_net_s *N, int64_t n)
{
    if (n <= N->bcap) return MLBM_OK;
    (void)hipStreamSynchronize(N->stream);
    (void)hipFree(N->Y); (void)hipFree(N->hid); (void)hipFree(N->dl); (void)hipFree(N->part); (void)hipFree(N->sel); (void)hipFree(N->lossp);
    N->Y = N->hid = N->dl = N->part = nullptr;   // nothing dangles if an allocation below fails
    N->sel = nullptr;
    N->lossp = nullptr;
    N->bcap = 0;
    const int H = N->sh.H, D = N->sh.depth;
    const int64_t nch = (n + CHUNK - 1) / CHUNK;
    NET_TRY(hipMalloc(&N->Y, sizeof(float) * NOUT * n));
    NET_TRY(hipMalloc(&N->hid, sizeof(float) * (size_t)n * D * H));
    NET_TRY(hipMalloc(&N->dl, sizeof(float) * (size_t)n * (D + 1) * H));
    NET_TRY(hipMalloc(&N->part, sizeof(float) * (size_t)nch * N->sh.np));
    NET_TRY(hipMalloc(&N->sel, sizeof(int64_t) * n));
    NET_TRY(hipMalloc(&N->lossp, sizeof(double) * nch));
    N->bcap = n;
    return MLBM_OK;
}

// gradient of the minibatch (X, T, M) drawn with `seed` (0: the first n rows)
mlbm_status run_gradient(mlbm_net_s *N, const float *X, const float *T, int64_t M, int64_t n, uint64_t seed,
                         double *loss)
{
    mlbm_status st = ensure_batch(N, n);
    if (st != MLBM_OK) return st;
    const Shape sh = N->sh;
    const int64_t nch = (n + CHUNK - 1) / CHUNK;
    const size_t lds = sizeof(float) * sh.np;
    NET_TRY(dispatch_H(sh.H, [&](auto Hc) {
        constexpr int H = decltype(Hc)::value;
        hipLaunchKernelGGL(forward_kernel<H>, dim3((unsigned)nch), dim3(CHUNK), lds, N->stream, N->p, sh, X, M, seed, n,
                           N->Y, N->hid, N->sel);
        hipLaunchKernelGGL(backward_kernel<H>, dim3((unsigned)nch), dim3(CHUNK), lds, N->stream, N->p, sh, T, N->sel, n,
                           N->Y, N->hid, N->dl, N->lossp);
        return hipGetLastError();
    }));
    hipLaunchKernelGGL(wgrad_kernel, dim3((unsigned)((sh.np + 255) / 256), (unsigned)nch), dim3(256), 0, N->stream, sh,
                       X, N->sel, n, N->hid, N->dl, N->part);
    NET_TRY(hipGetLastError());
    hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((sh.np + 255) / 256)), dim3(256), 0, N->stream, N->part,
                       (int)nch, sh.np, N->g);
    NET_TRY(hipGetLastError());
    if (loss) {
        std::vector<double> lp(nch);
        NET_TRY(hipMemcpyAsync(lp.data(), N->lossp, sizeof(double) * nch, hipMemcpyDeviceToHost, N->stream));
        NET_TRY(hipStreamSynchronize(N->stream));
        double s = 0.0;
        for (double x : lp) s += x;
        *loss = s / (3.0 * (double)n);
    }
    return MLBM_OK;
}

}  // namespace

extern "C" {

const char *mlbm_net_last_error(void) { return g_net_err.c_str(); }

int64_t mlbm_net_num_params(int hidden, int depth)
{
    if ((hidden != 32 && hidden != 64) || depth < 1 || depth > MAXDEPTH) return -1;
    const long np = make_shape(hidden, depth).np;
    return np * (long)sizeof(float) <= 65536 ? np : -1;   // parameters are staged in 64 KiB of LDS
}

mlbm_status mlbm_net_create(int hidden, int depth, const double *init_params, void *hip_stream, mlbm_net *out)
{
    if (!out || !init_params) return nfail(MLBM_E_ARG, "null argument");
    if (mlbm_net_num_params(hidden, depth) < 0)
        return nfail(MLBM_E_ARG, "hidden must be 32 or 64, depth in 1..6, parameters within 64 KiB");
    mlbm_net_s *N = new mlbm_net_s();
    N->sh = make_shape(hidden, depth);
    if (hip_stream) N->stream = (hipStream_t)hip_stream;
    else if (hipStreamCreate(&N->stream) != hipSuccess) { delete N; return nfail(MLBM_E_HIP, "hipStreamCreate"); }
    else N->own_stream = true;
    const long np = N->sh.np;
    std::vector<float> h(np);
    for (long k = 0; k < np; ++k) h[k] = (float)init_params[k];
    if (hipMalloc(&N->p, sizeof(float) * np) != hipSuccess || hipMalloc(&N->m, sizeof(float) * np) != hipSuccess ||
        hipMalloc(&N->v, sizeof(float) * np) != hipSuccess || hipMalloc(&N->g, sizeof(float) * np) != hipSuccess ||
        hipMemcpy(N->p, h.data(), sizeof(float) * np, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(N->m, 0, sizeof(float) * np) != hipSuccess || hipMemset(N->v, 0, sizeof(float) * np) != hipSuccess) {
        mlbm_net_destroy(N);
        return nfail(MLBM_E_OOM, "network allocation failed");
    }
    *out = N;
    return MLBM_OK;
}

void mlbm_net_destroy(mlbm_net N)
{
    if (!N) return;
    if (N->stream) (void)hipStreamSynchronize(N->stream);
    (void)hipFree(N->p); (void)hipFree(N->m); (void)hipFree(N->v); (void)hipFree(N->g);
    (void)hipFree(N->X); (void)hipFree(N->T);
    (void)hipFree(N->Y); (void)hipFree(N->hid); (void)hipFree(N->dl); (void)hipFree(N->part); (void)hipFree(N->sel); (void)hipFree(N->lossp);
    if (N->own_stream) (void)hipStreamDestroy(N->stream);
    delete N;
}

mlbm_status mlbm_net_params(mlbm_net N, double *params, int get)
{
    if (!N || !params) return nfail(MLBM_E_ARG, "null argument");
    const long np = N->sh.np;
    std::vector<float> h(np);
    if (get) {
        NET_TRY(hipMemcpyAsync(h.data(), N->p, sizeof(float) * np, hipMemcpyDeviceToHost, N->stream));
        NET_TRY(hipStreamSynchronize(N->stream));
        for (long k = 0; k < np; ++k) params[k] = h[k];
    } else {
        for (long k = 0; k < np; ++k) h[k] = (float)params[k];
        NET_TRY(hipMemcpyAsync(N->p, h.data(), sizeof(float) * np, hipMemcpyHostToDevice, N->stream));
        NET_TRY(hipStreamSynchronize(N->stream));
    }
    return MLBM_OK;
}

mlbm_status mlbm_net_forward(mlbm_net N, const float *x, int64_t n, float *y)
{
    if (!N || !x || !y || n <= 0) return nfail(MLBM_E_ARG, "null argument or n <= 0");
    mlbm_status st = ensure_batch(N, n);
    if (st != MLBM_OK) return st;
    CallBuf bx(N->stream);
    NET_TRY(hipMalloc(&bx.p, sizeof(float) * NIN * n));
    float *dx = (float *)bx.p;
    NET_TRY(hipMemcpyAsync(dx, x, sizeof(float) * NIN * n, hipMemcpyHostToDevice, N->stream));
    const Shape sh = N->sh;
    const int64_t nch = (n + CHUNK - 1) / CHUNK;
    hipError_t e = dispatch_H(sh.H, [&](auto Hc) {
        constexpr int H = decltype(Hc)::value;
        hipLaunchKernelGGL(forward_kernel<H>, dim3((unsigned)nch), dim3(CHUNK), sizeof(float) * sh.np, N->stream, N->p,
                           sh, dx, n, (uint64_t)0, n, N->Y, (float *)nullptr, (int64_t *)nullptr);
        return hipGetLastError();
    });
    if (e == hipSuccess) e = hipMemcpyAsync(y, N->Y, sizeof(float) * NOUT * n, hipMemcpyDeviceToHost, N->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(N->stream);
    NET_TRY(e);
    return MLBM_OK;
}

mlbm_status mlbm_net_gradient(mlbm_net N, const float *x, const float *t, int64_t n, double *loss, double *grad)
{
    if (!N || !x || !t || n <= 0) return nfail(MLBM_E_ARG, "null argument or n <= 0");
    CallBuf bx(N->stream), bt(N->stream);
    NET_TRY(hipMalloc(&bx.p, sizeof(float) * NIN * n));
    NET_TRY(hipMalloc(&bt.p, sizeof(float) * NOUT * n));
    float *dx = (float *)bx.p, *dt = (float *)bt.p;
    NET_TRY(hipMemcpyAsync(dx, x, sizeof(float) * NIN * n, hipMemcpyHostToDevice, N->stream));
    NET_TRY(hipMemcpyAsync(dt, t, sizeof(float) * NOUT * n, hipMemcpyHostToDevice, N->stream));
    mlbm_status st = run_gradient(N, dx, dt, n, n, 0, loss);
    if (st == MLBM_OK && grad) {
        std::vector<float> h(N->sh.np);
        hipError_t e = hipMemcpyAsync(h.data(), N->g, sizeof(float) * N->sh.np, hipMemcpyDeviceToHost, N->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(N->stream);
        if (e != hipSuccess) st = nfail(MLBM_E_HIP, hipGetErrorString(e));
        for (long k = 0; k < N->sh.np; ++k) grad[k] = h[k];
    }
    return st;
}

mlbm_status mlbm_net_dataset_clear(mlbm_net N)
{
    if (!N) return nfail(MLBM_E_ARG, "null network");
    N->M = 0;
    return MLBM_OK;
}

int64_t mlbm_net_dataset_size(mlbm_net N) { return N ? N->M : -1; }

mlbm_status mlbm_net_dataset_add(mlbm_net N, const mlbm_desc *d, double De, double R1_d, double R2_d, double U_nom,
                                 const double *u, int on_device)
{
    if (!N || !d || !u || !(U_nom > 0.0)) return nfail(MLBM_E_ARG, "null argument or U_nom <= 0");
    const int64_t P = (int64_t)d->n1 * d->n3;
    const int64_t N3 = (int64_t)d->n1 * d->n2 * d->n3;
    if (N->M + P > N->cap) {
        const int64_t cap = std::max<int64_t>(2 * N->cap, N->M + P);
        CallBuf bX(N->stream), bT(N->stream);
        NET_TRY(hipMalloc(&bX.p, sizeof(float) * NIN * cap));
        NET_TRY(hipMalloc(&bT.p, sizeof(float) * NOUT * cap));
        if (N->M) {
            NET_TRY(hipMemcpyAsync(bX.p, N->X, sizeof(float) * NIN * N->M, hipMemcpyDeviceToDevice, N->stream));
            NET_TRY(hipMemcpyAsync(bT.p, N->T, sizeof(float) * NOUT * N->M, hipMemcpyDeviceToDevice, N->stream));
        }
        NET_TRY(hipStreamSynchronize(N->stream));
        (void)hipFree(N->X);
        (void)hipFree(N->T);
        N->X = (float *)bX.p;              // the set takes the new buffers over
        N->T = (float *)bT.p;
        bX.p = bT.p = nullptr;
        N->cap = cap;
    }
    const double *du = u;
    CallBuf btmp(N->stream);
    if (!on_device) {
        NET_TRY(hipMalloc(&btmp.p, sizeof(double) * 3 * N3));
        NET_TRY(hipMemcpyAsync(btmp.p, u, sizeof(double) * 3 * N3, hipMemcpyHostToDevice, N->stream));
        du = (const double *)btmp.p;
    }
    const CaseGeo c = case_geo(*d, De, R1_d, R2_d);
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, N->stream, c, N->X + NIN * N->M);
    hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, N->stream, c, du, 1.0 / U_nom,
                       N->T + NOUT * N->M);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(N->stream);
    NET_TRY(e);
    N->M += P;
    return MLBM_OK;
}

mlbm_status mlbm_net_train(mlbm_net N, int64_t steps, int64_t batch, double lr, uint64_t seed, double *last_loss)
{
    if (!N || steps < 0 || batch <= 0 || N->M <= 0) return nfail(MLBM_E_ARG, "empty dataset or bad arguments");
    const long np = N->sh.np;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    double loss = 0.0;
    for (int64_t it = 0; it < steps; ++it) {
        const uint64_t s = mix64_host(seed * 0x100000001B3ull + (uint64_t)(N->t + 1)) | 1ull;
        mlbm_status st = run_gradient(N, N->X, N->T, N->M, batch, s, (it == steps - 1) ? &loss : nullptr);
        if (st != MLBM_OK) return st;
        N->t += 1;
        const float c1 = (float)(1.0 - std::pow(b1, (double)N->t)), c2 = (float)(1.0 - std::pow(b2, (double)N->t));
        hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, N->stream, N->p, N->g, N->m,
                           N->v, np, (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
        NET_TRY(hipGetLastError());
    }
    NET_TRY(hipStreamSynchronize(N->stream));
    if (last_loss) *last_loss = loss;
    return MLBM_OK;
}

mlbm_status mlbm_net_adam_step(mlbm_net N, double lr)
{
    if (!N) return nfail(MLBM_E_ARG, "null network");
    const long np = N->sh.np;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    N->t += 1;
    const float c1 = (float)(1.0 - std::pow(b1, (double)N->t)), c2 = (float)(1.0 - std::pow(b2, (double)N->t));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, N->stream, N->p, N->g, N->m, N->v,
                       np, (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
    NET_TRY(hipGetLastError());
    NET_TRY(hipStreamSynchronize(N->stream));
    return MLBM_OK;
}

mlbm_status mlbm_net_dataset_loss(mlbm_net N, double *loss)
{
    if (!N || !loss || N->M <= 0) return nfail(MLBM_E_ARG, "empty dataset");
    return run_gradient(N, N->X, N->T, N->M, N->M, 0, loss);
}

static const char NET_MAGIC[8] = {'M', 'L', 'B', 'M', 'N', 'E', 'T', '1'};

mlbm_status mlbm_warmstart_save(mlbm_net N, const char *path)
{
    if (!N || !path) return nfail(MLBM_E_ARG, "null argument");
    const int64_t np = N->sh.np;
    std::vector<double> p(np);
    mlbm_status st = mlbm_net_params(N, p.data(), 1);
    if (st != MLBM_OK) return st;
    FILE *fp = fopen(path, "wb");
    if (!fp) return nfail(MLBM_E_IO, std::string("cannot open ") + path);
    const int32_t hd[2] = {N->sh.H, N->sh.depth};
    bool ok = fwrite(NET_MAGIC, 1, 8, fp) == 8 && fwrite(hd, sizeof(hd), 1, fp) == 1 && fwrite(&np, sizeof(np), 1, fp) == 1 &&
              fwrite(p.data(), sizeof(double), (size_t)np, fp) == (size_t)np;
    ok = (fclose(fp) == 0) && ok;
    return ok ? MLBM_OK : nfail(MLBM_E_IO, std::string("write failed: ") + path);
}

mlbm_status mlbm_warmstart_load(const char *path, void *hip_stream, mlbm_net *out)
{
    if (!path || !out) return nfail(MLBM_E_ARG, "null argument");
    FILE *fp = fopen(path, "rb");
    if (!fp) return nfail(MLBM_E_IO, std::string("cannot open ") + path);
    char mg[8];
    int32_t hd[2] = {0, 0};
    int64_t np = 0;
    bool ok = fread(mg, 1, 8, fp) == 8 && !memcmp(mg, NET_MAGIC, 8) && fread(hd, sizeof(hd), 1, fp) == 1 &&
              fread(&np, sizeof(np), 1, fp) == 1;
    if (!ok || mlbm_net_num_params(hd[0], hd[1]) != np) {
        fclose(fp);
        return nfail(MLBM_E_IO, "not a warm-start network file, or a shape this library does not support");
    }
    std::vector<double> p((size_t)np);
    ok = fread(p.data(), sizeof(double), (size_t)np, fp) == (size_t)np;
    fclose(fp);
    if (!ok) return nfail(MLBM_E_IO, "network file truncated");
    return mlbm_net_create(hd[0], hd[1], p.data(), hip_stream, out);
}

mlbm_status mlbm_warmstart_predict(mlbm_net N, const mlbm_desc *d, double De, double R1_d, double R2_d, double U_nom,
                                   double *u_out, int on_device)
{
    if (!N || !d || !u_out) return nfail(MLBM_E_ARG, "null argument");
    const int64_t P = (int64_t)d->n1 * d->n3;
    const int64_t N3 = (int64_t)d->n1 * d->n2 * d->n3;
    mlbm_status st = ensure_batch(N, P);
    if (st != MLBM_OK) return st;
    CallBuf bX(N->stream), bu(N->stream);
    NET_TRY(hipMalloc(&bX.p, sizeof(float) * NIN * P));
    if (!on_device) NET_TRY(hipMalloc(&bu.p, sizeof(double) * 3 * N3));
    float *X = (float *)bX.p;
    double *du = (double *)bu.p;
    const CaseGeo c = case_geo(*d, De, R1_d, R2_d);
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, N->stream, c, X);
    const Shape sh = N->sh;
    const int64_t nch = (P + CHUNK - 1) / CHUNK;
    hipError_t e = dispatch_H(sh.H, [&](auto Hc) {
        constexpr int H = decltype(Hc)::value;
        hipLaunchKernelGGL(forward_kernel<H>, dim3((unsigned)nch), dim3(CHUNK), sizeof(float) * sh.np, N->stream, N->p,
                           sh, X, P, (uint64_t)0, P, N->Y, (float *)nullptr, (int64_t *)nullptr);
        return hipGetLastError();
    });
    double *target = on_device ? u_out : du;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(predict_map_kernel, dim3((unsigned)((N3 + 255) / 256)), dim3(256), 0, N->stream, c, N->Y,
                           U_nom, target);
        e = hipGetLastError();
    }
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(u_out, du, sizeof(double) * 3 * N3, hipMemcpyDeviceToHost, N->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(N->stream);
    NET_TRY(e);
    return MLBM_OK;
}

}  // extern "C"
