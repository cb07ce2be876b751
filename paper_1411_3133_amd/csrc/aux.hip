// Auxiliary device kernels: geometry precompute (FP64), initial state,
// window reductions, moments, observables, storage codecs and a sampled
// one-step update.
#include "core.hpp"
#include "kernels.hpp"

namespace mlbm {

// ------------------------------------------------------------------------
// Geometry (Sec. III cylinder, Sec. IV ellipsoid at theta = 0), FP64.
// Physical metric g_ij (diagonal for every supported kind at theta = 0),
// printed Christoffel symbols, lattice scaling with s_i = Dx^i / Dt:
//   lattice g^ij = g^ij / (s_i s_j), Gamma_lat^i_jk = Dt Gamma^i_jk s_j s_k / s_i,
//   unit force F^i = Dt g^{i theta} / s_i (times the covariant K at run time).
// ------------------------------------------------------------------------

__global__ void geometry_kernel(double *geo, GeoParams p)
{
    const int NX = p.n1 * p.n2g * p.n3g;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= NX) return;
    const int x1 = idx / (p.n2g * p.n3g), rem = idx - x1 * p.n2g * p.n3g;
    const int x2 = rem / p.n3g, x3 = rem - x2 * p.n3g;
    const double dt = p.dt;
    // nodes cell centred between halfway walls, or on r_i + x1 Dr whose first
    // and last are the wall nodes of equilibrium walls (Sec. III)
    const double o1 = p.eqwall ? 0.0 : 0.5;
    double X1, X3;
    double g11 = 1.0, g22 = 1.0, g33 = 1.0, g12 = 0.0, g13 = 0.0, g23 = 0.0;
    double G[3][3][3] = {};
    if (p.kind == 0) {                        // flat
        X1 = (x1 + o1) * dt * p.s[0];
        X3 = (x3 + 0.5) * dt * p.s[2];
    } else if (p.kind == 1) {                 // cylinder (r, theta, z)
        const double r = p.r_inner + (x1 + o1) * dt * p.s[0];
        X1 = r;
        X3 = (x3 + 0.5) * dt * p.s[2];
        g22 = r * r;
        G[0][1][1] = -r;                      // Gamma^r_{theta theta}
        G[1][0][1] = G[1][1][0] = 1.0 / r;    // Gamma^theta_{r theta}
    } else {                                  // ellipsoid (r, theta, phi), a = c = 1
        const double r = p.r_inner + (x1 + o1) * dt * p.s[0];
        const double ph = (x3 + 0.5 - 0.5 * p.n3) * dt * p.s[2];
        const double cp = cos(ph), sp = sin(ph), b2 = p.b * p.b;
        X1 = r;
        X3 = ph;
        if (p.kind == 3) {                    // the metric at the node's theta (sector centred on 0)
            const double th = (x2 + 0.5 - 0.5 * p.n2) * dt * p.s[1];
            const double ct = cos(th), st = sin(th);
            g11 = sp * sp + cp * cp * (ct * ct + b2 * st * st);
            g22 = r * r * cp * cp * (st * st + b2 * ct * ct);
            g33 = r * r * (cp * cp + sp * sp * (ct * ct + b2 * st * st));
            g12 = r * (b2 - 1.0) * cp * cp * ct * st;
            g13 = r * (1.0 - b2) * st * st * cp * sp;
            g23 = r * r * (1.0 - b2) * cp * sp * ct * st;
        } else {                              // frozen at theta = 0
            g22 = r * r * b2 * cp * cp;
            g33 = r * r;
        }
        G[0][1][1] = -r * cp * cp;                    // Gamma^r_{theta theta}
        G[0][2][2] = -r;                              // Gamma^r_{phi phi}
        G[1][0][1] = G[1][1][0] = 1.0 / r;            // Gamma^theta_{r theta}
        G[2][0][2] = G[2][2][0] = 1.0 / r;            // Gamma^phi_{r phi}
        G[1][1][2] = G[1][2][1] = -sp / cp;           // Gamma^theta_{theta phi}
        G[2][1][1] = sp * cp;                         // Gamma^phi_{theta theta}
    }
    const double *s = p.s;
    // inverse metric: reciprocals where it is diagonal, cofactors where it is
    // not (the full ellipsoid off theta = 0)
    double gi[3][3] = {{1.0 / g11, 0.0, 0.0}, {0.0, 1.0 / g22, 0.0}, {0.0, 0.0, 1.0 / g33}};
    double det = g11 * g22 * g33;
    if (g12 != 0.0 || g13 != 0.0 || g23 != 0.0) {
        const double c11 = g22 * g33 - g23 * g23, c12 = g13 * g23 - g12 * g33, c13 = g12 * g23 - g13 * g22;
        const double c22 = g11 * g33 - g13 * g13, c23 = g12 * g13 - g11 * g23, c33 = g11 * g22 - g12 * g12;
        det = g11 * c11 + g12 * c12 + g13 * c13;
        const double inv[3][3] = {{c11 / det, c12 / det, c13 / det}, {c12 / det, c22 / det, c23 / det},
                                  {c13 / det, c23 / det, c33 / det}};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) gi[i][j] = inv[i][j];
    }
    double *o = geo + idx;
    auto put = [&](int field, double v) { o[(size_t)field * NX] = v; };
    put(G_D11, gi[0][0] / (s[0] * s[0]) - 1.0);
    put(G_D22, gi[1][1] / (s[1] * s[1]) - 1.0);
    put(G_D33, gi[2][2] / (s[2] * s[2]) - 1.0);
    put(G_D12, gi[0][1] / (s[0] * s[1]));
    put(G_D13, gi[0][2] / (s[0] * s[2]));
    put(G_D23, gi[1][2] / (s[1] * s[2]));
    for (int i = 0; i < 3; ++i) {
        const int jk[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
        for (int e = 0; e < 6; ++e) {
            const int j = jk[e][0], k = jk[e][1];
            put(G_1_11 + 6 * i + e, dt * G[i][j][k] * s[j] * s[k] / s[i]);
        }
    }
    // covariant theta force K: contravariant g^{i theta} K (lattice units, per unit K)
    put(G_F1, dt * gi[0][1] / s[0]);
    put(G_F2, dt * gi[1][1] / s[1]);
    put(G_F3, dt * gi[2][1] / s[2]);
    put(G_SQRTG, sqrt(det) * s[0] * s[1] * s[2]);
    put(G_X1, X1);
    put(G_X3, X3);
}

__global__ void geo_to_f32_kernel(const double *geo, float *geof, long count)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) geof[i] = (float)geo[i];
}

hipError_t launch_geo_to_f32(const double *geo, float *geof, long count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(geo_to_f32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, geo, geof, count);
    return hipGetLastError();
}

hipError_t launch_geometry(double *geo, const GeoParams &p, hipStream_t s)
{
    const int NX = p.n1 * p.n2g * p.n3g;
    hipLaunchKernelGGL(geometry_kernel, dim3((NX + 255) / 256), dim3(256), 0, s, geo, p);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Initial state f* = f_eq(rho', U) with rho' = 1/sqrt(g) (rho = 1), in FP64
// ------------------------------------------------------------------------

// FP64 offsets g = f_eq - w of node n (x1 row, column col) for the initial
// state: rho' = 1/sqrt(g), contravariant velocity init_u / s (or rest).
__device__ void init_offsets(const InstDesc &d, int n, const double *init_u, double (&g)[Q])
{
    const int x1 = n / d.P, col = n - x1 * d.P, x2 = col / d.n3, x3 = col - x2 * d.n3;
    const int NX = geo_stride(d);
    const int gi = geo_index(d, x1, x2, x3);
    const double *geo = d.geo;
    double D[3][3];
    D[0][0] = geo[G_D11 * NX + gi]; D[1][1] = geo[G_D22 * NX + gi]; D[2][2] = geo[G_D33 * NX + gi];
    D[0][1] = D[1][0] = geo[G_D12 * NX + gi];
    D[0][2] = D[2][0] = geo[G_D13 * NX + gi];
    D[1][2] = D[2][1] = geo[G_D23 * NX + gi];
    const double rho = 1.0 / geo[G_SQRTG * NX + gi];
    double U[3] = {0.0, 0.0, 0.0};
    const bool wall = d.eqwall && (x1 == 0 || x1 == d.n1 - 1);   // at rest (Dirichlet)
    if (init_u && !wall)
        for (int i = 0; i < 3; ++i) U[i] = init_u[(size_t)i * d.N + n] / d.s[i];
    const double cs2 = CS2;
    const double uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
    const double trD = D[0][0] + D[1][1] + D[2][2];
    double DU[3];
    for (int i = 0; i < 3; ++i) DU[i] = D[i][0] * U[0] + D[i][1] * U[1] + D[i][2] * U[2];
    for (int q = 0; q < Q; ++q) {
        const double c0 = CV[q][0], c1 = CV[q][1], c2 = CV[q][2];
        const double cu = c0 * U[0] + c1 * U[1] + c2 * U[2];
        const double cDu = c0 * DU[0] + c1 * DU[1] + c2 * DU[2];
        double cDc = 0.0;
        const double c[3] = {c0, c1, c2};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) cDc += c[i] * D[i][j] * c[j];
        const double Em1 = (cDc - cs2 * trD) / (2.0 * cs2) + (cu * cu - cs2 * uu) / (2.0 * cs2 * cs2);
        const double Od = cu / cs2 + (cu * cu * cu - 3.0 * cs2 * uu * cu) / (6.0 * cs2 * cs2 * cs2)
                        + (cDc * cu - cs2 * trD * cu - 2.0 * cs2 * cDu) / (2.0 * cs2 * cs2);
        g[q] = wq(q) * ((rho - 1.0) + rho * (Em1 + Od));
    }
}

// Reference offsets of the 16-bit storage formats: per x1 row and
// population, the row mean r of d = f/w - 1 of the initial state (table
// [n1][41]). Values are stored as d - r, which keeps the stored magnitudes
// (and so the rounding error) small wherever the flow stays near its row
// mean. One workgroup per row, fixed summation order.
__global__ void ref_kernel(const InstDesc *dd, const double *init_u, float *ref)
{
    const InstDesc &d = *dd;
    const int x1 = blockIdx.x;
    __shared__ double part[256];
    double acc[Q];
    for (int q = 0; q < Q; ++q) acc[q] = 0.0;
    for (int col = threadIdx.x; col < d.P; col += blockDim.x) {
        double g[Q];
        init_offsets(d, x1 * d.P + col, init_u, g);
        for (int q = 0; q < Q; ++q) acc[q] += g[q] / wq(q);
    }
    for (int q = 0; q < Q; ++q) {
        part[threadIdx.x] = acc[q];
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) ref[x1 * Q + q] = (float)(part[0] / d.P);
        __syncthreads();
    }
}

template <int ST>
__global__ void init_kernel(const InstDesc *dd, const double *init_u, int parity)
{
    const InstDesc &d = *dd;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= d.N) return;
    const int x1 = n / d.P, col = storage_col(d, n - x1 * d.P);
    double g[Q];
    init_offsets(d, n, init_u, g);
    using T = typename Codec<ST>::T;
    T *dst = (T *)d.f[parity];
    for (int q = 0; q < Q; ++q) {
        const double r = Codec<ST>::REF ? (double)d.ref[x1 * Q + q] : 0.0;
        dst[pop_elem(q, x1, col, d.Pp)] = Codec<ST>::from_f64(g[q], wq(q), r);
    }
}

hipError_t launch_ref(const InstDesc *d_desc, const InstDesc &h, const double *init_u, float *ref, hipStream_t s)
{
    hipLaunchKernelGGL(ref_kernel, dim3(h.n1), dim3(256), 0, s, d_desc, init_u, ref);
    return hipGetLastError();
}

// Re-referencing of the 16-bit formats: the row means r of f/w - 1 are taken
// again from the current state and every stored value of the row is
// re-encoded against them. Against the initial means the stored magnitudes
// |d - r| grow as the flow develops and its density drifts (a drift of the
// mean density shifts every f/w - 1 alike), and the rounding noise grows
// with them. One workgroup per (x1 row, population): a fixed-order block
// reduction of the decoded values, then the re-encode in place (each value
// is read and written by the same thread) with stochastic rounding keyed
// apart from the steps' own.
template <int ST>
__global__ void reref_kernel(const InstDesc *dd, int parity, float *ref)
{
    using T = typename Codec<ST>::T;
    const InstDesc &d = *dd;
    const int x1 = blockIdx.x, q = blockIdx.y;
    __shared__ double part[256];
    T *plane = (T *)d.f[parity] + ((size_t)x1 * Q + q) * d.Pp;
    const float r_old = ref[x1 * Q + q];
    double acc = 0.0;
    for (int col = threadIdx.x; col < d.P; col += blockDim.x)
        acc += (double)Codec<ST>::decode(plane[storage_col(d, col)], r_old);
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    const float r_new = (float)(part[0] / d.P);
    const uint32_t key = mix32(d.salt ^ 0x2545F491u) + d.ctr[parity] * 0x85EBCA77u + (uint32_t)q * 0xC2B2AE3Du;
    for (int col = threadIdx.x; col < d.P; col += blockDim.x) {
        const uint32_t bits = mix32(key + (uint32_t)(x1 * d.P + col) * 0x9E3779B9u);
        T &v = plane[storage_col(d, col)];
        v = Codec<ST>::encode_sr(Codec<ST>::decode(v, r_old), r_new, bits);
    }
    if (threadIdx.x == 0) ref[x1 * Q + q] = r_new;   // this workgroup is its only reader
}

hipError_t launch_reref(const InstDesc *d_desc, const InstDesc &h, int st, int parity, float *ref, hipStream_t s)
{
    const dim3 grid(h.n1, Q), block(256);
    if (st == ST_F16)
        hipLaunchKernelGGL(reref_kernel<ST_F16>, grid, block, 0, s, d_desc, parity, ref);
    else if (st == ST_BF16)
        hipLaunchKernelGGL(reref_kernel<ST_BF16>, grid, block, 0, s, d_desc, parity, ref);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_init(const InstDesc *d_desc, const InstDesc &h, int st, const double *init_u, int parity,
                       hipStream_t s)
{
    const dim3 grid((h.N + 255) / 256), block(256);
    switch (st) {
    case ST_F64: hipLaunchKernelGGL(init_kernel<ST_F64>, grid, block, 0, s, d_desc, init_u, parity); break;
    case ST_F32: hipLaunchKernelGGL(init_kernel<ST_F32>, grid, block, 0, s, d_desc, init_u, parity); break;
    case ST_F16: hipLaunchKernelGGL(init_kernel<ST_F16>, grid, block, 0, s, d_desc, init_u, parity); break;
    case ST_F32D: hipLaunchKernelGGL(init_kernel<ST_F32D>, grid, block, 0, s, d_desc, init_u, parity); break;
    default: hipLaunchKernelGGL(init_kernel<ST_BF16>, grid, block, 0, s, d_desc, init_u, parity); break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Window reduction: one workgroup per instance, fixed summation order
// ------------------------------------------------------------------------

__global__ void __launch_bounds__(256) reduce_kernel(const double *partials, const int *pb, const int *pc,
                                                     WindowState *ws, int ninst)
{
    const int i = blockIdx.x;                 // one workgroup per instance
    if (i >= ninst || pb[i] < 0) return;      // uniform across the workgroup
    __shared__ double sa[256], sb[256], sc[256];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = t; k < pc[i]; k += blockDim.x) {
        const double *p = partials + 3 * (size_t)(pb[i] + k);
        a += p[0]; b += p[1]; c += p[2];
    }
    sa[t] = a; sb[t] = b; sc[t] = c;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {   // fixed order: bitwise reproducible
        if (t < h) { sa[t] += sa[t + h]; sb[t] += sb[t + h]; sc[t] += sc[t + h]; }
        __syncthreads();
    }
    if (t == 0) {
        WindowState w = ws[i];
        w.checks += 1;
        w.residual = w.checks >= 2 ? sqrt(sa[0]) / sqrt(sb[0]) : -1.0;
        if (sc[0] > 0.0) w.bad = 1;
        ws[i] = w;
    }
}

hipError_t launch_reduce(const double *partials, const int *pb, const int *pc, WindowState *ws, int ninst,
                         hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(ninst), dim3(256), 0, s, partials, pb, pc, ws, ninst);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Moments of the streamed state (FP64)
// ------------------------------------------------------------------------

template <int ST>
__device__ __forceinline__ void pull_f64(const InstDesc &d, int parity, int x1, int x2, int x3, double (&g)[Q])
{
    using T = typename Codec<ST>::T;
    const T *src = (const T *)d.f[parity];
    static_for<0, Q>([&](auto q) {
        constexpr int qo = opposite(q);
        bool flip;
        int row;
        const int col = fold_source<CV[q][0], CV[q][1], CV[q][2]>(d, x1, x2, x3, flip, row);
        const int qs = flip ? qo : (int)q;
        const double r = Codec<ST>::REF ? (double)d.ref[row * Q + qs] : 0.0;
        g[q] = Codec<ST>::to_f64(gload<T>(src, sizeof(T) * pop_elem(qs, row, col, d.Pp)), wq(q), r);
    });
}

template <int ST>
__global__ void moments_kernel(const InstDesc *dd, int parity, double *rho, double *u)
{
    const InstDesc &d = *dd;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= d.N) return;
    const int x1 = n / d.P, col = n - x1 * d.P, x2 = col / d.n3, x3 = col - x2 * d.n3;
    double g[Q];
    pull_f64<ST>(d, parity, x1, x2, x3, g);
    double r, U[3];
    moments_only<double>(g, r, U);
    if (d.eqwall && (x1 == 0 || x1 == d.n1 - 1)) U[0] = U[1] = U[2] = 0.0;   // Dirichlet value
    const int NX = geo_stride(d);
    const int gi = geo_index(d, x1, x2, x3);
    if (rho) rho[n] = r * d.geo[G_SQRTG * NX + gi];
    if (u)
        for (int i = 0; i < 3; ++i) u[(size_t)i * d.N + n] = d.s[i] * U[i];
}

hipError_t launch_moments(const InstDesc *d_desc, const InstDesc &h, int st, int parity, double *rho, double *u,
                          hipStream_t s)
{
    const dim3 grid((h.N + 255) / 256), block(256);
    switch (st) {
    case ST_F64: hipLaunchKernelGGL(moments_kernel<ST_F64>, grid, block, 0, s, d_desc, parity, rho, u); break;
    case ST_F32: hipLaunchKernelGGL(moments_kernel<ST_F32>, grid, block, 0, s, d_desc, parity, rho, u); break;
    case ST_F16: hipLaunchKernelGGL(moments_kernel<ST_F16>, grid, block, 0, s, d_desc, parity, rho, u); break;
    case ST_F32D: hipLaunchKernelGGL(moments_kernel<ST_F32D>, grid, block, 0, s, d_desc, parity, rho, u); break;
    default: hipLaunchKernelGGL(moments_kernel<ST_BF16>, grid, block, 0, s, d_desc, parity, rho, u); break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Observables (Sec. III, Sec. IV): per-block partial sums of
//   <v_theta> numerator, <omega> numerator and the area S.
// Derivatives: second-order central differences, periodic wrap; next to a
// wall the one-sided second-order formula through u = 0 at the halfway wall.
// ------------------------------------------------------------------------

// walled: 0 periodic, 1 halfway walls, 2 wall nodes (equilibrium walls: the
// one-sided second-order formula at the wall node itself)
__device__ __forceinline__ double ddx_axis(const double *f, int stride, int x, int n, int walled, double h)
{
    if (walled == 2) {
        if (x == 0) return (-3.0 * f[0] + 4.0 * f[stride] - f[2 * stride]) / (2.0 * h);
        if (x == n - 1) return (3.0 * f[0] - 4.0 * f[-stride] + f[-2 * stride]) / (2.0 * h);
        return (f[stride] - f[-stride]) / (2.0 * h);
    }
    if (walled) {
        if (n == 1) return 0.0;
        if (x == 0) return (f[0] + f[stride] / 3.0) / h;
        if (x == n - 1) return -(f[0] + f[-stride] / 3.0) / h;
        return (f[stride] - f[-stride]) / (2.0 * h);
    }
    const int xp = x + 1 == n ? 0 : x + 1, xm = x == 0 ? n - 1 : x - 1;
    return (f[(xp - x) * stride] - f[(xm - x) * stride]) / (2.0 * h);
}

__global__ void vortex_kernel(InstDesc d, int kind, double b, double h1, double h3, int x2lo, int x2hi,
                              const double *u, double *partials)
{
    __shared__ double red[4][3];
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int x1 = n / d.P, col = n - x1 * d.P, x2 = col / d.n3, x3 = col - x2 * d.n3;
    double vs = 0.0, os = 0.0, as = 0.0;
    // nodes of the theta slabs [x2lo, x2hi) contribute; the rest add zeros
    if (n < d.N && x2 >= x2lo && x2 < x2hi) {
        const int NX = geo_stride(d);
        const int gi = geo_index(d, x1, x2, x3);
        const double r = d.geo[G_X1 * NX + gi], ph = d.geo[G_X3 * NX + gi];
        const double *ur = u + n, *uz = u + 2 * (size_t)d.N + n;
        const double d3ur = ddx_axis(ur, 1, x3, d.n3, (d.walls & 4) ? 1 : 0, h3);
        const double d1uz = ddx_axis(uz, d.P, x1, d.n1, d.eqwall ? 2 : ((d.walls & 1) ? 1 : 0), h1);
        // trapezoidal weight over r with wall nodes at r_i and r_o
        const double tw = (d.eqwall && (x1 == 0 || x1 == d.n1 - 1)) ? 0.5 : 1.0;
        const double vort = fabs(d3ur - d1uz);
        const double uth = u[(size_t)d.N + n];
        double wv = 1.0, wo = 1.0, ws = 1.0;
        if (kind == 1) { wv = r; wo = r; }
        else if (kind >= 2) { const double cp = cos(ph); wv = r * r * b * cp; wo = r * b * cp; ws = r; }
        vs = tw * uth * wv * h1 * h3;
        os = tw * vort * wo * h1 * h3;
        as = tw * ws * h1 * h3;
    }
    for (int off = 32; off > 0; off >>= 1) {
        vs += __shfl_xor(vs, off, 64);
        os += __shfl_xor(os, off, 64);
        as += __shfl_xor(as, off, 64);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) { red[wave][0] = vs; red[wave][1] = os; red[wave][2] = as; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0, e = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a += red[w][0]; c += red[w][1]; e += red[w][2]; }
        partials[3 * blockIdx.x + 0] = a;
        partials[3 * blockIdx.x + 1] = c;
        partials[3 * blockIdx.x + 2] = e;
    }
}

hipError_t launch_vortex(const InstDesc &h, int kind, double b, double h1, double h3, int x2lo, int x2hi,
                         const double *u, double *partials, int *nblocks, hipStream_t s)
{
    const int nb = (h.N + 255) / 256;
    *nblocks = nb;
    hipLaunchKernelGGL(vortex_kernel, dim3(nb), dim3(256), 0, s, h, kind, b, h1, h3, x2lo, x2hi, u, partials);
    return hipGetLastError();
}

// Sum of the per-block triples in block order by one lane: the same sequence
// of FP64 additions as a host loop over the partials, hence the same bits.
__global__ void sum_partials_kernel(const double *partials, int nb, double *out)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double a = 0.0, c = 0.0, e = 0.0;
    for (int k = 0; k < nb; ++k) { a += partials[3 * k]; c += partials[3 * k + 1]; e += partials[3 * k + 2]; }
    out[0] = a;
    out[1] = c;
    out[2] = e;
}

hipError_t launch_sum_partials(const double *partials, int nb, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, partials, nb, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Codecs: stored offsets (row-major storage order, pop_elem) <-> absolute
// FP64 populations in the external layout [41][N]
// ------------------------------------------------------------------------

template <int ST>
__global__ void decode_kernel(InstDesc d, int parity, double *f)
{
    using T = typename Codec<ST>::T;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)Q * d.N) return;
    const int q = (int)(i / d.N);
    const int n = (int)(i - (size_t)q * d.N), x1 = n / d.P, col = storage_col(d, n - x1 * d.P);
    const double w = wq(q);
    const double r = Codec<ST>::REF ? (double)d.ref[x1 * Q + q] : 0.0;
    f[i] = Codec<ST>::to_f64(((const T *)d.f[parity])[pop_elem(q, x1, col, d.Pp)], w, r) + w;
}

template <int ST>
__global__ void encode_kernel(InstDesc d, int parity, const double *f)
{
    using T = typename Codec<ST>::T;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)Q * d.N) return;
    const int q = (int)(i / d.N);
    const int n = (int)(i - (size_t)q * d.N), x1 = n / d.P, col = storage_col(d, n - x1 * d.P);
    const double w = wq(q);
    const double r = Codec<ST>::REF ? (double)d.ref[x1 * Q + q] : 0.0;
    ((T *)d.f[parity])[pop_elem(q, x1, col, d.Pp)] = Codec<ST>::from_f64(f[i] - w, w, r);
}

hipError_t launch_decode(const InstDesc &h, int st, int parity, double *f, hipStream_t s)
{
    const size_t tot = (size_t)Q * h.N;
    const dim3 grid((unsigned)((tot + 255) / 256)), block(256);
    switch (st) {
    case ST_F64: hipLaunchKernelGGL(decode_kernel<ST_F64>, grid, block, 0, s, h, parity, f); break;
    case ST_F32: hipLaunchKernelGGL(decode_kernel<ST_F32>, grid, block, 0, s, h, parity, f); break;
    case ST_F16: hipLaunchKernelGGL(decode_kernel<ST_F16>, grid, block, 0, s, h, parity, f); break;
    case ST_F32D: hipLaunchKernelGGL(decode_kernel<ST_F32D>, grid, block, 0, s, h, parity, f); break;
    default: hipLaunchKernelGGL(decode_kernel<ST_BF16>, grid, block, 0, s, h, parity, f); break;
    }
    return hipGetLastError();
}

hipError_t launch_encode(const InstDesc &h, int st, int parity, const double *f, hipStream_t s)
{
    const size_t tot = (size_t)Q * h.N;
    const dim3 grid((unsigned)((tot + 255) / 256)), block(256);
    switch (st) {
    case ST_F64: hipLaunchKernelGGL(encode_kernel<ST_F64>, grid, block, 0, s, h, parity, f); break;
    case ST_F32: hipLaunchKernelGGL(encode_kernel<ST_F32>, grid, block, 0, s, h, parity, f); break;
    case ST_F16: hipLaunchKernelGGL(encode_kernel<ST_F16>, grid, block, 0, s, h, parity, f); break;
    case ST_F32D: hipLaunchKernelGGL(encode_kernel<ST_F32D>, grid, block, 0, s, h, parity, f); break;
    default: hipLaunchKernelGGL(encode_kernel<ST_BF16>, grid, block, 0, s, h, parity, f); break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// One update of listed nodes from the current state (same gather and
// collision as the step kernel, in the step kernel's compute precision)
// ------------------------------------------------------------------------

template <int PAT, int ST>
__global__ void step_nodes_kernel(const InstDesc *dd, int parity, const int64_t *nodes, int64_t count, double *out)
{
    using T = typename Codec<ST>::T;
    using C = typename Codec<ST>::C;
    const InstDesc &d = *dd;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int n = (int)nodes[k];
    if (n < 0 || n >= d.N) return;
    const int x1 = n / d.P, col = n - x1 * d.P, x2 = col / d.n3, x3 = col - x2 * d.n3;
    typename Codec<ST>::G g[Q];
    gather_general<ST>(d.f[parity], d, x1, x2, x3, RefRow{d.ref}, g);
    NodeGeo<PAT, C> geo;
    geo.load(d.geo, d.geof, geo_index(d, x1, x2, x3), geo_stride(d), (C)d.force);
    C rho, u[3];
    if (d.eqwall && (x1 == 0 || x1 == d.n1 - 1))
        wall_equilibrium<PAT, C, typename Codec<ST>::G, Codec<ST>::SCALED>(g, geo, rho);
    else
        collide<PAT, C, typename Codec<ST>::G, Codec<ST>::SCALED>(g, geo, (C)d.omega, (C)d.kappa, rho, u);
    static_for<0, Q>([&](auto q) {
        // round through the storage format, as the step kernel stores it
        const float r = Codec<ST>::REF ? d.ref[x1 * Q + q] : 0.0f;
        // the rounding the step kernel applies in the step that reads the
        // current counter (stochastic for the 16-bit formats)
        T tmp;
        if constexpr (Codec<ST>::REF)
            tmp = Codec<ST>::encode_sr(g[q], (C)r,
                                       RoundBits(d.salt, (uint32_t)n, d.ctr[parity]).template get<q>());
        else
            tmp = Codec<ST>::encode(g[q], (C)r);
        out[k * Q + q] = Codec<ST>::to_f64(tmp, wq(q), (double)r) + wq(q);
    });
}

template <int PAT>
static void launch_sn_pat(const InstDesc *dd, int st, int parity, const int64_t *nodes, int64_t count, double *out,
                          hipStream_t s)
{
    const dim3 grid((unsigned)((count + 63) / 64)), block(64);
    switch (st) {
    case ST_F64: hipLaunchKernelGGL((step_nodes_kernel<PAT, ST_F64>), grid, block, 0, s, dd, parity, nodes, count, out); break;
    case ST_F32: hipLaunchKernelGGL((step_nodes_kernel<PAT, ST_F32>), grid, block, 0, s, dd, parity, nodes, count, out); break;
    case ST_F16: hipLaunchKernelGGL((step_nodes_kernel<PAT, ST_F16>), grid, block, 0, s, dd, parity, nodes, count, out); break;
    case ST_F32D: hipLaunchKernelGGL((step_nodes_kernel<PAT, ST_F32D>), grid, block, 0, s, dd, parity, nodes, count, out); break;
    default: hipLaunchKernelGGL((step_nodes_kernel<PAT, ST_BF16>), grid, block, 0, s, dd, parity, nodes, count, out); break;
    }
}

hipError_t launch_step_nodes(const InstDesc *d_desc, const InstDesc &h, int pat, int st, int parity,
                             const int64_t *nodes, int64_t count, double *out, hipStream_t s)
{
    (void)h;
    if (count <= 0) return hipSuccess;
    switch (pat) {
    case PAT_CYL: launch_sn_pat<PAT_CYL>(d_desc, st, parity, nodes, count, out, s); break;
    case PAT_ELL: launch_sn_pat<PAT_ELL>(d_desc, st, parity, nodes, count, out, s); break;
    default: launch_sn_pat<PAT_GEN>(d_desc, st, parity, nodes, count, out, s); break;
    }
    return hipGetLastError();
}

}  // namespace mlbm
