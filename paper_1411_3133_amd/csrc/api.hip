// Host runtime behind the C ABI of include/mlbm.h.
//
// Every simulation lives in a batch: a single-instance handle owns a batch of
// one.  A batch holds the device descriptors of its instances, the flat tile
// queue of the active ones, the per-tile partial sums of the stationarity
// check and the per-instance window state.  Steps are issued as K-step
// windows captured in a hipGraph (K - 1 plain steps, one checking step and
// the reduction), so one host call replays K launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mlbm.h"

#include <rocprofiler-sdk-roctx/roctx.h>
#include "common.hpp"
#include "core.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

using namespace mlbm;

namespace {

thread_local std::string g_err;

mlbm_status fail(mlbm_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(e_ == hipErrorOutOfMemory ? MLBM_E_OOM : MLBM_E_HIP,                   \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                    \
    } while (0)

struct Instance {
    mlbm_desc desc{};          // init_u not retained
    InstDesc hd{};             // host copy of the device descriptor
    double dt = 0.0;
    int geo_key = -1;
    int64_t t = 0;             // completed steps
    bool active = true;
    int status = -1;           // 0 converged, 1 max steps, 2 unstable
};

struct GeoEntry {
    double *ptr = nullptr;
    float *fptr = nullptr;     // the same values rounded to FP32
    int kind, n1, n2, n3, eq;
    double r_inner, width, b, dtheta;
};

}  // namespace

// Scratch of the allocation-free entry point (mlbm_vortex_intensity_noalloc):
// a fixed device array that every GPU the library runs on holds until the
// process ends. Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol); it uses the device address
// that hipGetSymbolAddress returns for the current device, looked up once
// per device at initialisation.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(1) << 21;   // 16 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// velocity [3][N], block triples [3][ceil(N / 256)] and three sums
size_t noalloc_vortex_doubles(size_t N) { return 3 * N + 3 * ((N + 255) / 256) + 3; }

// Device address of `scratch` on device `dev`, looked up on first use with
// that device current (the library's init call does it for its device).
mlbm_status noalloc_scratch(int dev, double **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(MLBM_E_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) HIP_TRY(hipSetDevice(cur));
        HIP_TRY(e);
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return MLBM_OK;
}

}  // namespace

struct Batch {
    hipStream_t stream = nullptr;
    int dev = 0;               // device the batch was created on
    bool own_stream = false;
    std::vector<Instance> inst;
    std::vector<GeoEntry> geos;
    int st = ST_F64, pat = PAT_CYL, K = 100;
    bool eqw = false;          // some instance has equilibrium walls (kernel variant)
    int block = 256, grid = 0;
    bool use_graph = true;
    int num_cu = 256;

    InstDesc *d_insts = nullptr;
    Tile *d_tiles = nullptr;
    int *d_ntiles = nullptr;
    int ntiles = 0, tiles_cap = 0;
    double *d_partials = nullptr;
    int *d_pb = nullptr, *d_pc = nullptr;
    WindowState *d_ws = nullptr;

    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_src = nullptr;
    bool graph_valid = false;
    bool keep_retired = false; // retired instances stay out of later steps

    double *d_scratch = nullptr;
    size_t scratch_bytes = 0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int64_t timed_steps = 0;

    int64_t t = 0;             // steps of the batch clock (active instances)
};

struct mlbm_sim_s {
    Batch *b;
    int idx;
    bool owner;
};

struct mlbm_batch_s {
    Batch *b;
};

namespace {

int pattern_for_kind(int kind)
{
    return kind == MLBM_ELLIPSOID_FULL ? PAT_GEN : kind == MLBM_ELLIPSOID ? PAT_ELL : PAT_CYL;
}

bool ellipsoidal(int kind) { return kind == MLBM_ELLIPSOID || kind == MLBM_ELLIPSOID_FULL; }

// Storage pitch of x3: n3 rounded up to 16 values, so that every x2 row of
// every population plane starts on a 64-byte boundary (measured on the
// batched ellipsoid sweep: an instance with n3 = 113 stepped at 44 % of the
// HBM peak, at n3 = 112 at 64 %).
int x3_pitch(int n3) { return (n3 + 15) / 16 * 16; }

size_t storage_values(const InstDesc &h) { return (size_t)Q * h.n1 * h.Pp; }

mlbm_status validate(const mlbm_desc &d)
{
    if (d.kind < 0 || d.kind > 3)
        return fail(MLBM_E_ARG, "kind must be MLBM_FLAT, MLBM_CYLINDER, MLBM_ELLIPSOID or MLBM_ELLIPSOID_FULL");
    if (!(d.dtheta >= 0.0) || !std::isfinite(d.dtheta)) return fail(MLBM_E_ARG, "dtheta must be >= 0");
    if (d.n1 < 1 || d.n2 < 1 || d.n3 < 1) return fail(MLBM_E_ARG, "n1, n2, n3 must be >= 1");
    if ((d.walls & ~(MLBM_WALL_AXIS1 | MLBM_WALL_AXIS3 | MLBM_WALL_EQUILIBRIUM | MLBM_OPEN_AXIS2)) != 0)
        return fail(MLBM_E_ARG, "walls: unknown bits");
    if ((d.walls & MLBM_OPEN_AXIS2) && d.n2 < 4) return fail(MLBM_E_ARG, "an open axis 2 needs >= 4 nodes (n2)");
    if ((d.walls & MLBM_WALL_EQUILIBRIUM) && (d.walls & (MLBM_WALL_AXIS1 | MLBM_WALL_AXIS3)) != MLBM_WALL_AXIS1)
        return fail(MLBM_E_ARG, "equilibrium walls need walls on axis 1 and a periodic axis 3");
    if ((d.walls & MLBM_WALL_AXIS1) && d.n1 < 4) return fail(MLBM_E_ARG, "an axis with walls needs >= 4 nodes (n1)");
    if ((d.walls & MLBM_WALL_AXIS3) && d.n3 < 4) return fail(MLBM_E_ARG, "an axis with walls needs >= 4 nodes (n3)");
    const double Np = (double)d.n1 * d.n2 * x3_pitch(d.n3);
    if (Np * Q * (double)storage_bytes(d.precision < 0 || d.precision > 4 ? 0 : d.precision) >= 4294967296.0)
        return fail(MLBM_E_ARG, "one population buffer must stay below 4 GiB (41 n1 n2 n3p bytes-per-value, "
                                "n3p = n3 rounded up to 16)");
    if ((double)d.n2 * x3_pitch(d.n3) >= (double)(1 << 20))
        return fail(MLBM_E_ARG, "n2 * n3 (n3 rounded up to 16) must be < 2^20");
    if (d.forcing_mode != MLBM_FORCING_IMPROVED && d.forcing_mode != MLBM_FORCING_OLD)
        return fail(MLBM_E_ARG, "forcing_mode must be MLBM_FORCING_IMPROVED or MLBM_FORCING_OLD");
    if (d.precision < 0 || d.precision > 4) return fail(MLBM_E_ARG, "precision out of range");
    if (d.check_every != 0 && (d.check_every < 2 || (d.check_every & 1)))
        return fail(MLBM_E_ARG, "check_every must be even and >= 2 (or 0 for 100)");
    if (!(d.tau > 0.5)) return fail(MLBM_E_ARG, "tau must be > 0.5");
    if (!(d.width > 0.0)) return fail(MLBM_E_ARG, "width must be > 0");
    if (!std::isfinite(d.force)) return fail(MLBM_E_ARG, "force must be finite");
    if (!(d.target_De >= 0.0) || !std::isfinite(d.target_De)) return fail(MLBM_E_ARG, "target_De must be >= 0");
    if (d.target_De > 0.0 && d.force != 0.0) return fail(MLBM_E_ARG, "give either force or target_De, not both");
    if (!(d.perturb_amp >= 0.0) || !std::isfinite(d.perturb_amp)) return fail(MLBM_E_ARG, "perturb_amp must be >= 0");
    if (d.perturb_amp > 0.0 && d.init_u) return fail(MLBM_E_ARG, "perturb_amp builds the start: init_u must be NULL");
    if (d.init_u_xsec != 0 && d.init_u_xsec != 1) return fail(MLBM_E_ARG, "init_u_xsec must be 0 or 1");
    if (d.reserved != 0) return fail(MLBM_E_ARG, "reserved must be 0");
    if (d.kind != MLBM_FLAT && !(d.r_inner > 0.0)) return fail(MLBM_E_ARG, "r_inner must be > 0");
    if (ellipsoidal(d.kind)) {
        if (!(d.b > 0.0)) return fail(MLBM_E_ARG, "b must be > 0");
        const double dphi = d.width / d.n1 / d.r_inner;
        if (!(0.5 * d.n3 * dphi < 1.5)) return fail(MLBM_E_ARG, "phi sector must stay inside |phi| < 1.5");
    }
    return MLBM_OK;
}

bool eq_walls(const mlbm_desc &d) { return (d.walls & MLBM_WALL_EQUILIBRIUM) != 0; }

void scales(const mlbm_desc &d, double &dt, double s[3])
{
    // N_r fluid nodes between halfway walls, or n1 - 1 spacings between the
    // wall nodes of equilibrium walls
    dt = d.width / (eq_walls(d) ? d.n1 - 1 : d.n1);
    s[0] = s[1] = s[2] = 1.0;
    if (ellipsoidal(d.kind)) {   // rescaled spacings of Sec. IV B
        s[1] = 1.0 / (d.b * d.r_inner);
        s[2] = 1.0 / d.r_inner;
        if (d.kind == MLBM_ELLIPSOID_FULL && d.dtheta > 0.0) s[1] = d.dtheta / dt;
    }
}

// ---- case set-up: body force from a Dean number, closed-form start ---------

double lattice_dt(const mlbm_desc &d) { return d.width / (eq_walls(d) ? d.n1 - 1 : d.n1); }
double nu_phys(const mlbm_desc &d) { return (d.tau - 0.5) * CS2 * lattice_dt(d); }

// (A, B, C) of v(r) = A r ln r + B r + C / r with v(r_i) = v(r_o) = 0: the
// azimuthal balance nu (d/dr)((1/r) d(r v)/dr) = -K / r of a constant
// covariant force K (Sec. III), A = -K / (2 nu).
void curved_coeffs(double ri, double ro, double K, double nu, double &A, double &B, double &C)
{
    A = -K / (2.0 * nu);
    const double b0 = -A * ri * std::log(ri), b1 = -A * ro * std::log(ro);
    const double det = ri / ro - ro / ri;          // | ri 1/ri ; ro 1/ro |
    B = (b0 / ro - b1 / ri) / det;
    C = (ri * b1 - ro * b0) / det;
}

double curved_v(double r, double ri, double ro, double K, double nu)
{
    double A, B, C;
    curved_coeffs(ri, ro, K, nu, A, B, C);
    return A * r * std::log(r) + B * r + C / r;
}

// (1/d) int_{r_i}^{r_o} v dr
double curved_mean(double ri, double ro, double K, double nu)
{
    double A, B, C;
    curved_coeffs(ri, ro, K, nu, A, B, C);
    auto prim = [&](double r) { return A * (0.5 * r * r * std::log(r) - 0.25 * r * r) + 0.5 * B * r * r + C * std::log(r); };
    return (prim(ro) - prim(ri)) / (ro - ri);
}

double stream_radius(const mlbm_desc &d) { return d.kind == MLBM_CYLINDER ? d.r_inner : d.r_inner * d.b * d.b; }
// (every ellipsoidal kind: the streamwise radius at theta = 0)

// Mean streamwise speed implied by De (Eq. (8)): De nu / d (flat: the
// Reynolds number), over sqrt(d / R) for curved channels.
double nominal_velocity(const mlbm_desc &d, double De)
{
    const double v = De * nu_phys(d) / d.width;
    return d.kind == MLBM_FLAT ? v : v / std::sqrt(d.width / stream_radius(d));
}

// Covariant force giving De for the laminar closed-form flow; the ellipsoid
// uses the channel of its streamwise radius R = r_i b^2 with the physical
// force matched at the inner wall (K / b).
double nominal_force(const mlbm_desc &d, double De)
{
    const double nu = nu_phys(d), w = d.width;
    if (d.kind == MLBM_FLAT) return 12.0 * nu * nominal_velocity(d, De) / (w * w);
    const double R = stream_radius(d);
    const double K = nominal_velocity(d, De) / curved_mean(R, R + w, 1.0, nu);
    return d.kind == MLBM_CYLINDER ? K : K / d.b;
}

uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Closed-form start: laminar streamwise profile plus the seeded
// perturbation, physical contravariant [3][n1][n2][n3].
std::vector<double> closed_form_start(const mlbm_desc &d, double force)
{
    const int n1 = d.n1, n2 = d.n2, n3 = d.n3;
    const size_t N = (size_t)n1 * n2 * n3;
    const double dt = lattice_dt(d), nu = nu_phys(d), w = d.width;
    const double o1 = eq_walls(d) ? 0.0 : 0.5;
    const double Unom = d.target_De > 0.0 ? nominal_velocity(d, d.target_De) : 1.0;
    const uint64_t key = d.seed * 0x100000001B3ull;
    std::vector<double> u(3 * N, 0.0);
    for (int x1 = 0; x1 < n1; ++x1) {
        const double y = (x1 + o1) * dt;
        const double r = d.kind == MLBM_FLAT ? y : d.r_inner + y;
        for (int x3 = 0; x3 < n3; ++x3) {
            const double ph = (x3 + 0.5 - 0.5 * n3) * dt / d.r_inner;
            double lam = 0.0, sc1 = 1.0, sc2 = 1.0;
            if (d.kind == MLBM_FLAT) {
                lam = force / (2.0 * nu) * y * (w - y);
            } else if (d.kind == MLBM_CYLINDER) {
                lam = curved_v(r, d.r_inner, d.r_inner + w, force, nu) / r;
                sc1 = 1.0 / r;
            } else {
                const double R = stream_radius(d), cp = std::cos(ph);
                lam = curved_v(R + y, R, R + w, force * d.b, nu) / (r * d.b * cp);
                sc1 = 1.0 / (r * d.b * cp);
                sc2 = 1.0 / r;
            }
            double xi[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < 3; ++c) {
                const uint64_t i = ((uint64_t)c * n1 + x1) * n3 + x3;
                xi[c] = (double)(splitmix64(i ^ key) >> 11) * 0x1p-52 - 1.0;
            }
            const double amp = d.perturb_amp * Unom;
            for (int x2 = 0; x2 < n2; ++x2) {
                const size_t n = ((size_t)x1 * n2 + x2) * n3 + x3;
                u[n] = amp * xi[0];
                u[N + n] = lam + amp * xi[1] * sc1;
                u[2 * N + n] = amp * xi[2] * sc2;
            }
        }
    }
    return u;
}

mlbm_status ensure_scratch(Batch *B, size_t bytes)
{
    if (B->scratch_bytes >= bytes) return MLBM_OK;
    if (B->d_scratch) HIP_TRY(hipFree(B->d_scratch));
    B->d_scratch = nullptr;
    B->scratch_bytes = 0;
    HIP_TRY(hipMalloc(&B->d_scratch, bytes));
    B->scratch_bytes = bytes;
    return MLBM_OK;
}

void destroy_graph(Batch *B)
{
    if (B->graph) (void)hipGraphExecDestroy(B->graph);
    if (B->graph_src) (void)hipGraphDestroy(B->graph_src);
    B->graph = nullptr;
    B->graph_src = nullptr;
    B->graph_valid = false;
}

// Tile queue of the active instances for the current block size.
// Key of an instance's stochastic rounding: a hash of its description, so
// that an instance rounds the same way alone and in any batch.
uint32_t desc_salt(const mlbm_desc &d)
{
    uint32_t h = 0x3133u;
    auto add = [&h](uint64_t v) {
        h = mix32(h ^ (uint32_t)v);
        h = mix32(h ^ (uint32_t)(v >> 32));
    };
    add((uint64_t)d.kind); add((uint64_t)d.n1); add((uint64_t)d.n2); add((uint64_t)d.n3);
    add((uint64_t)d.walls); add((uint64_t)d.forcing_mode);
    const double vals[5] = {d.tau, d.force, d.b, d.r_inner, d.width};
    for (double x : vals) {
        uint64_t u;
        memcpy(&u, &x, sizeof(u));
        add(u);
    }
    if (d.dtheta != 0.0) {   // only the full ellipsoid sets it; other salts stay as they were
        uint64_t u;
        memcpy(&u, &d.dtheta, sizeof(u));
        add(u);
    }
    return h;
}

// The 16-bit storage formats keep a per-row reference table.
bool uses_ref(int st) { return st == ST_F16 || st == ST_BF16; }

mlbm_status build_tiles(Batch *B)
{
    std::vector<Tile> tiles;
    std::vector<int> pb(B->inst.size(), -1), pc(B->inst.size(), 0);
    for (size_t i = 0; i < B->inst.size(); ++i) {
        Instance &I = B->inst[i];
        I.hd.tpr = (I.hd.Pp + B->block - 1) / B->block;
        if (!I.active) continue;
        pb[i] = (int)tiles.size();
        for (int x1 = 0; x1 < I.hd.n1; ++x1)
            for (int c = 0; c < I.hd.tpr; ++c) tiles.push_back(Tile{(int)i, x1, c, (int)tiles.size()});
        pc[i] = (int)tiles.size() - pb[i];
    }
    const int ntiles = (int)tiles.size();
    // The captured window and the device lists are replaced together: wait
    // for every launch that reads the old ones, drop the window, and launch
    // nothing (ntiles = 0) unless the new lists are all in place.
    HIP_TRY(hipStreamSynchronize(B->stream));
    destroy_graph(B);
    B->ntiles = 0;
    if (ntiles > B->tiles_cap) {
        if (B->d_tiles) HIP_TRY(hipFree(B->d_tiles));
        if (B->d_partials) HIP_TRY(hipFree(B->d_partials));
        B->d_tiles = nullptr;
        B->d_partials = nullptr;
        B->tiles_cap = 0;
        const int cap = std::max<int>(1, ntiles);
        HIP_TRY(hipMalloc(&B->d_tiles, sizeof(Tile) * cap));
        HIP_TRY(hipMalloc(&B->d_partials, sizeof(double) * 3 * cap));
        B->tiles_cap = cap;
    }
    std::vector<InstDesc> hds;
    for (auto &I : B->inst) hds.push_back(I.hd);
    HIP_TRY(hipMemcpyAsync(B->d_insts, hds.data(), sizeof(InstDesc) * hds.size(), hipMemcpyHostToDevice, B->stream));
    if (!tiles.empty())
        HIP_TRY(hipMemcpyAsync(B->d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipMemcpyAsync(B->d_ntiles, &ntiles, sizeof(int), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipMemcpyAsync(B->d_pb, pb.data(), sizeof(int) * pb.size(), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipMemcpyAsync(B->d_pc, pc.data(), sizeof(int) * pc.size(), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));   // host vectors go out of scope
    B->ntiles = ntiles;
    return MLBM_OK;
}

int launch_grid(const Batch *B) { return B->grid > 0 ? std::min(B->grid, std::max(1, B->ntiles)) : std::max(1, B->ntiles); }

mlbm_status enqueue_step(Batch *B, bool check)
{
    if (B->ntiles == 0) return MLBM_OK;
    StepArgs a{B->d_insts, B->d_tiles, B->d_ntiles, B->d_partials, (int)(B->t & 1)};
    HIP_TRY(launch_step(a, B->pat, B->st, check, B->eqw, launch_grid(B), B->block, B->stream));
    if (check) HIP_TRY(launch_reduce(B->d_partials, B->d_pb, B->d_pc, B->d_ws, (int)B->inst.size(), B->stream));
    B->t += 1;
    for (auto &I : B->inst)
        if (I.active) I.t += 1;
    return MLBM_OK;
}

mlbm_status capture_window(Batch *B)
{
    // a window starts at an even step, K is even
    destroy_graph(B);
    const int64_t t0 = B->t;
    std::vector<int64_t> it0;
    for (auto &I : B->inst) it0.push_back(I.t);
    HIP_TRY(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
    mlbm_status st = MLBM_OK;
    for (int k = 0; k < B->K && st == MLBM_OK; ++k) st = enqueue_step(B, k == B->K - 1);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B->stream, &g);
    B->t = t0;
    for (size_t i = 0; i < B->inst.size(); ++i) B->inst[i].t = it0[i];
    if (st != MLBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    HIP_TRY(e);
    B->graph_src = g;
    HIP_TRY(hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0));
    B->graph_valid = true;
    return MLBM_OK;
}

// 16-bit storage: every REREF_WINDOWS windows of its own clock an instance
// re-takes its reference row means from the current state, right before it
// steps on (so the step counts at which it happens do not depend on how the
// steps are grouped into calls, batches or graphs).
constexpr int64_t REREF_WINDOWS = 10;

int parity_of(const Instance &I) { return (int)(I.t & 1); }

// true when an active instance reaches a re-reference step strictly inside
// the next m steps (a graph window must not straddle one)
bool reref_within(const Batch *B, int64_t m)
{
    if (!uses_ref(B->st)) return false;
    const int64_t every = REREF_WINDOWS * B->K;
    for (const auto &I : B->inst) {
        if (!I.active) continue;
        const int64_t to = (every - I.t % every) % every;
        if (to > 0 && to < m) return true;
    }
    return false;
}

mlbm_status reref_due(Batch *B)
{
    if (!uses_ref(B->st)) return MLBM_OK;
    const int64_t every = REREF_WINDOWS * B->K;
    for (size_t i = 0; i < B->inst.size(); ++i) {
        Instance &I = B->inst[i];
        if (!I.active || I.t == 0 || I.t % every != 0) continue;
        HIP_TRY(launch_reref(B->d_insts + i, I.hd, B->st, parity_of(I), const_cast<float *>(I.hd.ref), B->stream));
    }
    return MLBM_OK;
}

mlbm_status advance(Batch *B, int64_t n)
{
    while (n > 0) {
        mlbm_status rs = reref_due(B);
        if (rs != MLBM_OK) return rs;
        const int64_t into = B->t % B->K;
        if (into == 0 && n >= B->K && B->use_graph && B->ntiles > 0 && !reref_within(B, B->K)) {
            if (!B->graph_valid) {
                mlbm_status s = capture_window(B);
                if (s != MLBM_OK) return s;
            }
            // one host range per K-step window (rocprofv3 --marker-trace)
            roctxRangePushA("mlbm K-step window");
            const hipError_t e = hipGraphLaunch(B->graph, B->stream);
            roctxRangePop();
            HIP_TRY(e);
            B->t += B->K;
            for (auto &I : B->inst)
                if (I.active) I.t += B->K;
            n -= B->K;
        } else {
            mlbm_status s = enqueue_step(B, (B->t + 1) % B->K == 0);
            if (s != MLBM_OK) return s;
            n -= 1;
        }
    }
    return MLBM_OK;
}

// Every instance stops on a window boundary, so every step count is a
// multiple of the even K and all instances share the buffer parity of the
// batch clock: they can all be stepped again together.
mlbm_status reactivate(Batch *B, bool capped_only)
{
    bool changed = false;
    int64_t tmax = 0;
    for (auto &I : B->inst) {
        // capped_only: bring back the instances that stopped at the call's
        // step cap; converged, unstable and caller-retired ones stay out
        if (!I.active && (!capped_only || I.status == 1)) {
            I.active = true;
            changed = true;
        }
        tmax = std::max(tmax, I.t);
    }
    B->t = tmax;
    return changed ? build_tiles(B) : MLBM_OK;
}

mlbm_status reactivate_all(Batch *B) { return reactivate(B, false); }

mlbm_status read_ws(Batch *B, std::vector<WindowState> &ws)
{
    ws.resize(B->inst.size());
    HIP_TRY(hipMemcpyAsync(ws.data(), B->d_ws, sizeof(WindowState) * ws.size(), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    return MLBM_OK;
}

GeoEntry *find_or_make_geo(Batch *B, const mlbm_desc &d, int &key, mlbm_status &st)
{
    for (size_t k = 0; k < B->geos.size(); ++k) {
        GeoEntry &g = B->geos[k];
        if (g.kind == d.kind && g.n1 == d.n1 && g.n3 == d.n3 && g.r_inner == d.r_inner && g.width == d.width &&
            g.b == d.b && g.eq == (int)eq_walls(d) &&
            (d.kind != MLBM_ELLIPSOID_FULL || (g.n2 == d.n2 && g.dtheta == d.dtheta))) {
            key = (int)k;
            st = MLBM_OK;
            return &g;
        }
    }
    GeoEntry g{};
    g.kind = d.kind; g.n1 = d.n1; g.n2 = d.n2; g.n3 = d.n3; g.r_inner = d.r_inner; g.width = d.width; g.b = d.b;
    g.eq = (int)eq_walls(d);
    g.dtheta = d.dtheta;
    const int n3g = ellipsoidal(d.kind) ? d.n3 : 1;
    const int n2g = d.kind == MLBM_ELLIPSOID_FULL ? d.n2 : 1;
    hipError_t e = hipMalloc(&g.ptr, sizeof(double) * NGEO * d.n1 * n2g * n3g);
    if (e != hipSuccess) {
        st = fail(MLBM_E_OOM, "geometry allocation failed");
        return nullptr;
    }
    GeoParams p{};
    p.kind = d.kind; p.n1 = d.n1; p.n2 = d.n2; p.n3 = d.n3; p.n2g = n2g; p.n3g = n3g;
    p.eqwall = (int)eq_walls(d);
    p.r_inner = d.r_inner; p.width = d.width; p.b = d.b;
    scales(d, p.dt, p.s);
    e = launch_geometry(g.ptr, p, B->stream);
    const long count = (long)NGEO * d.n1 * n2g * n3g;
    if (e == hipSuccess) e = hipMalloc(&g.fptr, sizeof(float) * count);
    if (e == hipSuccess) e = launch_geo_to_f32(g.ptr, g.fptr, count, B->stream);
    if (e != hipSuccess) {
        (void)hipFree(g.ptr);
        if (g.fptr) (void)hipFree(g.fptr);
        st = fail(MLBM_E_HIP, std::string("geometry kernel: ") + hipGetErrorString(e));
        return nullptr;
    }
    B->geos.push_back(g);
    key = (int)B->geos.size() - 1;
    st = MLBM_OK;
    return &B->geos.back();
}

void free_batch(Batch *B)
{
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    destroy_graph(B);
    for (auto &I : B->inst) {
        if (I.hd.f[0]) (void)hipFree(I.hd.f[0]);
        if (I.hd.f[1]) (void)hipFree(I.hd.f[1]);
        if (I.hd.usnap) (void)hipFree(I.hd.usnap);
        if (I.hd.ref) (void)hipFree(const_cast<float *>(I.hd.ref));
        if (I.hd.ctr) (void)hipFree(I.hd.ctr);
    }
    for (auto &g : B->geos) {
        if (g.ptr) (void)hipFree(g.ptr);
        if (g.fptr) (void)hipFree(g.fptr);
    }
    if (B->d_insts) (void)hipFree(B->d_insts);
    if (B->d_tiles) (void)hipFree(B->d_tiles);
    if (B->d_ntiles) (void)hipFree(B->d_ntiles);
    if (B->d_partials) (void)hipFree(B->d_partials);
    if (B->d_pb) (void)hipFree(B->d_pb);
    if (B->d_pc) (void)hipFree(B->d_pc);
    if (B->d_ws) (void)hipFree(B->d_ws);
    if (B->d_scratch) (void)hipFree(B->d_scratch);
    if (B->ev0) (void)hipEventDestroy(B->ev0);
    if (B->ev1) (void)hipEventDestroy(B->ev1);
    if (B->own_stream && B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
}

mlbm_status create_batch(const mlbm_desc *ds, int n, void *stream, Batch **out)
{
    if (!ds || n < 1 || !out) return fail(MLBM_E_ARG, "null description or n < 1");
    const int K = ds[0].check_every ? ds[0].check_every : 100;
    int pat = PAT_CYL;
    bool eqw = false;
    for (int i = 0; i < n; ++i) {
        mlbm_status s = validate(ds[i]);
        if (s != MLBM_OK) return fail(s, "instance " + std::to_string(i) + ": " + g_err);
        if (ds[i].precision != ds[0].precision) return fail(MLBM_E_ARG, "every instance of a batch needs the same precision");
        if ((ds[i].check_every ? ds[i].check_every : 100) != K) return fail(MLBM_E_ARG, "every instance needs the same check_every");
        pat = std::max(pat, pattern_for_kind(ds[i].kind));
        if (ds[i].walls & MLBM_OPEN_AXIS2) pat = PAT_GEN;   // open theta ends: general-pattern kernels
        eqw |= eq_walls(ds[i]);
    }
    if (const char *e = getenv("MLBM_PATTERN")) {   // compile-time sparsity override (tests of the general kernel)
        if (!strcmp(e, "general")) pat = PAT_GEN;
    }
    Batch *B = new Batch();
    B->st = ds[0].precision;
    B->K = K;
    B->pat = pat;
    B->eqw = eqw;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&B->num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        delete B;
        return fail(MLBM_E_HIP, "no HIP device");
    }
    B->dev = dev;
    {
        double *p = nullptr;   // set-up of the allocation-free entry point for this device
        mlbm_status ss = noalloc_scratch(dev, &p);
        if (ss != MLBM_OK) {
            delete B;
            return ss;
        }
    }
    if (stream) {
        B->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreate(&B->stream) != hipSuccess) {
            delete B;
            return fail(MLBM_E_HIP, "hipStreamCreate failed");
        }
        B->own_stream = true;
    }
    auto bail = [&](mlbm_status s) {
        free_batch(B);
        return s;
    };
    if (hipEventCreate(&B->ev0) != hipSuccess || hipEventCreate(&B->ev1) != hipSuccess)
        return bail(fail(MLBM_E_HIP, "hipEventCreate failed"));
    if (hipMalloc(&B->d_insts, sizeof(InstDesc) * n) != hipSuccess || hipMalloc(&B->d_ntiles, sizeof(int)) != hipSuccess ||
        hipMalloc(&B->d_pb, sizeof(int) * n) != hipSuccess || hipMalloc(&B->d_pc, sizeof(int) * n) != hipSuccess ||
        hipMalloc(&B->d_ws, sizeof(WindowState) * n) != hipSuccess)
        return bail(fail(MLBM_E_OOM, "descriptor allocation failed"));
    std::vector<WindowState> ws0(n, WindowState{-1.0, 0, 0});
    if (hipMemcpy(B->d_ws, ws0.data(), sizeof(WindowState) * n, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(MLBM_E_HIP, "window state upload failed"));
    const size_t sbytes = storage_bytes(B->st);
    B->inst.resize(n);
    for (int i = 0; i < n; ++i) {
        const mlbm_desc &d = ds[i];
        Instance &I = B->inst[i];
        I.desc = d;
        I.desc.init_u = nullptr;
        if (!I.desc.check_every) I.desc.check_every = K;
        mlbm_status gs;
        GeoEntry *g = find_or_make_geo(B, d, I.geo_key, gs);
        if (!g) return bail(gs);
        InstDesc &h = I.hd;
        h.geo = g->ptr;
        h.geof = g->fptr;
        h.n1 = d.n1; h.n2 = d.n2; h.n3 = d.n3; h.walls = d.walls;
        h.eqwall = (int)eq_walls(d);
        h.P = d.n2 * d.n3;
        h.N = d.n1 * h.P;
        h.n3p = x3_pitch(d.n3);
        h.Pp = d.n2 * h.n3p;
        h.n3g = ellipsoidal(d.kind) ? d.n3 : 1;
        h.n2g = d.kind == MLBM_ELLIPSOID_FULL ? d.n2 : 1;
        h.n3_magic = ((1ull << 40) + (uint64_t)h.n3p - 1) / (uint64_t)h.n3p;
        h.omega = 1.0 / d.tau;
        h.kappa = d.forcing_mode == MLBM_FORCING_IMPROVED ? 1.0 - 1.0 / (2.0 * d.tau) : 0.0;
        // the retained description carries the resolved force and no start
        // recipe (a checkpoint restores the state itself)
        if (d.target_De > 0.0) I.desc.force = nominal_force(d, d.target_De);
        I.desc.target_De = 0.0;
        I.desc.perturb_amp = 0.0;
        I.desc.init_u_xsec = 0;
        h.force = I.desc.force;
        scales(d, I.dt, h.s);
        const size_t fb = sbytes * storage_values(h);
        if (hipMalloc(&h.f[0], fb) != hipSuccess || hipMalloc(&h.f[1], fb) != hipSuccess ||
            hipMalloc(&h.usnap, sizeof(double) * 3 * (size_t)h.N) != hipSuccess)
            return bail(fail(MLBM_E_OOM, "population allocation failed (instance " + std::to_string(i) + ")"));
        if (hipMemsetAsync(h.usnap, 0, sizeof(double) * 3 * (size_t)h.N, B->stream) != hipSuccess ||
            hipMemsetAsync(h.f[0], 0, fb, B->stream) != hipSuccess ||   // the x3 padding stays zero
            hipMemsetAsync(h.f[1], 0, fb, B->stream) != hipSuccess)
            return bail(fail(MLBM_E_HIP, "hipMemsetAsync failed"));
        h.ref = nullptr;
        h.ctr = nullptr;
        h.salt = desc_salt(I.desc);
        if (uses_ref(B->st)) {
            float *ref = nullptr;
            if (hipMalloc(&ref, sizeof(float) * Q * (size_t)h.n1) != hipSuccess)
                return bail(fail(MLBM_E_OOM, "reference table allocation failed"));
            h.ref = ref;
            if (hipMalloc(&h.ctr, 2 * sizeof(uint32_t)) != hipSuccess)
                return bail(fail(MLBM_E_OOM, "step counter allocation failed"));
            if (hipMemsetAsync(h.ctr, 0, 2 * sizeof(uint32_t), B->stream) != hipSuccess)
                return bail(fail(MLBM_E_HIP, "hipMemsetAsync failed"));
        }
    }
    mlbm_status s = build_tiles(B);
    if (s != MLBM_OK) return bail(s);
    for (int i = 0; i < n; ++i) {
        Instance &I = B->inst[i];
        double *du = nullptr;
        std::vector<double> field;     // host start field [3][N], when built here
        const double *src = ds[i].init_u;
        if (ds[i].perturb_amp > 0.0) {
            field = closed_form_start(ds[i], I.desc.force);
            src = field.data();
        } else if (src && ds[i].init_u_xsec) {   // the cross section repeated in every theta slab
            const int n1 = I.hd.n1, n2 = I.hd.n2, n3 = I.hd.n3;
            field.resize(3 * (size_t)I.hd.N);
            for (int c = 0; c < 3; ++c)
                for (int x1 = 0; x1 < n1; ++x1)
                    for (int x2 = 0; x2 < n2; ++x2)
                        for (int x3 = 0; x3 < n3; ++x3)
                            field[(size_t)c * I.hd.N + ((size_t)x1 * n2 + x2) * n3 + x3] =
                                src[((size_t)c * n1 + x1) * n3 + x3];
            src = field.data();
        }
        if (src) {
            const size_t bytes = sizeof(double) * 3 * (size_t)I.hd.N;
            if (hipMalloc(&du, bytes) != hipSuccess) return bail(fail(MLBM_E_OOM, "init_u staging failed"));
            if (hipMemcpyAsync(du, src, bytes, hipMemcpyHostToDevice, B->stream) != hipSuccess) {
                (void)hipFree(du);
                return bail(fail(MLBM_E_HIP, "init_u upload failed"));
            }
        }
        hipError_t e = hipSuccess;
        if (I.hd.ref) e = launch_ref(B->d_insts + i, I.hd, du, const_cast<float *>(I.hd.ref), B->stream);
        if (e == hipSuccess) e = launch_init(B->d_insts + i, I.hd, B->st, du, 0, B->stream);
        (void)hipStreamSynchronize(B->stream);
        if (du) (void)hipFree(du);
        if (e != hipSuccess) return bail(fail(MLBM_E_HIP, std::string("init kernel: ") + hipGetErrorString(e)));
    }
    if (hipStreamSynchronize(B->stream) != hipSuccess) return bail(fail(MLBM_E_HIP, "initialisation failed"));
    *out = B;
    return MLBM_OK;
}

Instance *inst_of(mlbm_handle h) { return (h && h->b) ? &h->b->inst[h->idx] : nullptr; }

// <v_theta>, <omega> and the measured Dean number (Sec. III Eq. (8), Sec. IV)
// from the sums over the cross sections of the v numerator, the omega
// numerator and the area.
void observables_from_sums(const Instance &I, double vs, double os, double as, double *omega_mean, double *v_mean,
                           double *De)
{
    const mlbm_desc &d = I.desc;
    const double vm = vs / as, om = os / as;
    double de = 0.0;
    if (d.kind != MLBM_FLAT) {
        const double nu = (d.tau - 0.5) * CS2 * I.dt;
        const double R = d.kind == MLBM_CYLINDER ? d.r_inner : d.r_inner * d.b * d.b;
        de = vm * d.width / nu * std::sqrt(d.width / R);
    }
    if (omega_mean) *omega_mean = om;
    if (v_mean) *v_mean = vm;
    if (De) *De = de;
}

template <int I, int N, class F>
void static_for_host(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for_host<I + 1, N>(f);
    }
}

}  // namespace

// =========================================================================
// C ABI
// =========================================================================

extern "C" {

const char *mlbm_last_error(void) { return g_err.c_str(); }

int mlbm_lattice(int32_t *c, double *w, double *cs2)
{
    for (int q = 0; q < Q; ++q) {
        if (c)
            for (int a = 0; a < 3; ++a) c[3 * q + a] = CV[q][a];
        if (w) w[q] = wq(q);
    }
    if (cs2) *cs2 = CS2;
    return Q;
}

mlbm_status mlbm_batch_create(const mlbm_desc *ds, int n, void *hip_stream, mlbm_batch *out)
{
    if (!out) return fail(MLBM_E_ARG, "out is null");
    Batch *B = nullptr;
    mlbm_status s = create_batch(ds, n, hip_stream, &B);
    if (s != MLBM_OK) return s;
    *out = new mlbm_batch_s{B};
    return MLBM_OK;
}

mlbm_status mlbm_init_geometry(const mlbm_desc *d, void *hip_stream, mlbm_handle *out)
{
    if (!d || !out) return fail(MLBM_E_ARG, "null argument");
    Batch *B = nullptr;
    mlbm_status s = create_batch(d, 1, hip_stream, &B);
    if (s != MLBM_OK) return s;
    *out = new mlbm_sim_s{B, 0, true};
    return MLBM_OK;
}

void mlbm_destroy(mlbm_handle h)
{
    if (!h) return;
    if (h->owner) free_batch(h->b);   // a view frees only itself, never its batch
    delete h;
}

void mlbm_batch_destroy(mlbm_batch b)
{
    if (!b) return;
    free_batch(b->b);
    delete b;
}

int mlbm_batch_size(mlbm_batch b) { return b && b->b ? (int)b->b->inst.size() : 0; }

mlbm_status mlbm_batch_get(mlbm_batch b, int i, mlbm_handle *view)
{
    if (!b || !view || i < 0 || i >= (int)b->b->inst.size()) return fail(MLBM_E_ARG, "index out of range");
    *view = new mlbm_sim_s{b->b, i, false};
    return MLBM_OK;
}

mlbm_status mlbm_step(mlbm_handle h, int64_t n)
{
    if (!h) return fail(MLBM_E_ARG, "null handle");
    if (!h->owner) return fail(MLBM_E_STATE, "mlbm_step on a batch view; use mlbm_batch_step");
    if (n < 0) return fail(MLBM_E_ARG, "n < 0");
    return advance(h->b, n);
}

mlbm_status mlbm_batch_step(mlbm_batch b, int64_t n)
{
    if (!b) return fail(MLBM_E_ARG, "null batch");
    if (n < 0) return fail(MLBM_E_ARG, "n < 0");
    Batch *B = b->b;
    HIP_TRY(hipEventRecord(B->ev0, B->stream));
    mlbm_status s = advance(B, n);
    HIP_TRY(hipEventRecord(B->ev1, B->stream));
    B->timed_steps = n;
    return s;
}

double mlbm_batch_last_step_ms(mlbm_batch b)
{
    if (!b || b->b->timed_steps <= 0) return -1.0;
    Batch *B = b->b;
    if (hipEventSynchronize(B->ev1) != hipSuccess) return -1.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, B->ev0, B->ev1) != hipSuccess) return -1.0;
    return (double)ms / (double)B->timed_steps;
}

mlbm_status mlbm_pull_map(const mlbm_desc *d, int64_t *src_node, int32_t *src_q)
{
    if (!d || !src_node || !src_q) return fail(MLBM_E_ARG, "null argument");
    mlbm_status s = validate(*d);
    if (s != MLBM_OK) return s;
    InstDesc h{};
    h.n1 = d->n1; h.n2 = d->n2; h.n3 = d->n3; h.walls = d->walls;
    h.eqwall = (int)eq_walls(*d);
    h.P = d->n2 * d->n3;
    h.N = d->n1 * h.P;
    h.n3p = d->n3;              // the host map is in node indices: no padding
    h.Pp = h.P;
    for (int x1 = 0; x1 < d->n1; ++x1)
        for (int x2 = 0; x2 < d->n2; ++x2)
            for (int x3 = 0; x3 < d->n3; ++x3) {
                const int64_t n = ((int64_t)x1 * d->n2 + x2) * d->n3 + x3;
                static_for_host<0, Q>([&](auto q) {
                    bool flip = false;
                    int row = 0;
                    const int col = fold_source<CV[q][0], CV[q][1], CV[q][2]>(h, x1, x2, x3, flip, row);
                    src_node[n * Q + q] = (int64_t)row * h.P + col;
                    src_q[n * Q + q] = flip ? opposite(q) : (int)q;
                });
            }
    return MLBM_OK;
}

int64_t mlbm_time(mlbm_handle h)
{
    Instance *I = inst_of(h);
    return I ? I->t : -1;
}

mlbm_status mlbm_residual(mlbm_handle h, double *r, int *bad)
{
    Instance *I = inst_of(h);
    if (!I) return fail(MLBM_E_ARG, "null handle");
    std::vector<WindowState> ws;
    mlbm_status s = read_ws(h->b, ws);
    if (s != MLBM_OK) return s;
    if (r) *r = ws[h->idx].residual;
    if (bad) *bad = ws[h->idx].bad;
    return MLBM_OK;
}

mlbm_status mlbm_batch_run_until(mlbm_batch b, double tol, int64_t max_steps, int64_t *steps, double *residual,
                                 int32_t *status)
{
    if (!b) return fail(MLBM_E_ARG, "null batch");
    Batch *B = b->b;
    std::vector<int64_t> start(B->inst.size());
    for (size_t i = 0; i < B->inst.size(); ++i) {
        start[i] = B->inst[i].t;
        if (B->inst[i].active) B->inst[i].status = -1;
        else if (B->inst[i].status < 0) B->inst[i].status = 3;   // retired by the caller
    }
    std::vector<WindowState> ws;
    bool any_unstable = false;
    // align to a window boundary
    if (B->t % B->K) {
        mlbm_status s = advance(B, B->K - B->t % B->K);
        if (s != MLBM_OK) return s;
    }
    for (;;) {
        bool any = false;
        for (auto &I : B->inst) any |= I.active;
        if (!any) break;
        mlbm_status s = advance(B, B->K);
        if (s != MLBM_OK) return s;
        s = read_ws(B, ws);
        if (s != MLBM_OK) return s;
        bool changed = false;
        for (size_t i = 0; i < B->inst.size(); ++i) {
            Instance &I = B->inst[i];
            if (!I.active) continue;
            int st = -1;
            if (ws[i].bad) st = 2;
            else if (ws[i].residual >= 0.0 && ws[i].residual <= tol) st = 0;
            else if (I.t - start[i] >= max_steps) st = 1;
            if (st >= 0) {
                I.active = false;
                I.status = st;
                changed = true;
                any_unstable |= st == 2;
            }
        }
        if (changed) {
            s = build_tiles(B);
            if (s != MLBM_OK) return s;
        }
    }
    for (size_t i = 0; i < B->inst.size(); ++i) {
        if (steps) steps[i] = B->inst[i].t - start[i];
        if (residual) residual[i] = ws.empty() ? -1.0 : ws[i].residual;
        if (status) status[i] = B->inst[i].status;
    }
    mlbm_status s = reactivate(B, B->keep_retired);
    if (s != MLBM_OK) return s;
    return any_unstable ? fail(MLBM_E_UNSTABLE, "an instance became unstable") : MLBM_OK;
}

mlbm_status mlbm_batch_keep_retired(mlbm_batch b, int on)
{
    if (!b) return fail(MLBM_E_ARG, "null batch");
    b->b->keep_retired = on != 0;
    return on ? MLBM_OK : reactivate_all(b->b);
}

mlbm_status mlbm_batch_retire(mlbm_batch b, int i)
{
    if (!b || i < 0 || i >= (int)b->b->inst.size()) return fail(MLBM_E_ARG, "null batch or index out of range");
    Batch *B = b->b;
    if (B->t % B->K) return fail(MLBM_E_STATE, "instances retire between windows only (step count a multiple of check_every)");
    if (!B->keep_retired) return fail(MLBM_E_STATE, "retiring needs mlbm_batch_keep_retired(b, 1)");
    Instance &I = B->inst[i];
    if (!I.active) return MLBM_OK;
    I.active = false;
    I.status = 3;
    return build_tiles(B);
}

mlbm_status mlbm_run_until(mlbm_handle h, double tol, int64_t max_steps, int64_t *steps_taken)
{
    if (!h) return fail(MLBM_E_ARG, "null handle");
    if (!h->owner) return fail(MLBM_E_STATE, "mlbm_run_until on a batch view; use mlbm_batch_run_until");
    mlbm_batch_s tmp{h->b};
    int64_t st = 0;
    int32_t status = 0;
    double r = 0.0;
    mlbm_status s = mlbm_batch_run_until(&tmp, tol, max_steps, &st, &r, &status);
    if (steps_taken) *steps_taken = st;
    return s;
}

mlbm_status mlbm_get_populations(mlbm_handle h, double *f)
{
    Instance *I = inst_of(h);
    if (!I || !f) return fail(MLBM_E_ARG, "null argument");
    Batch *B = h->b;
    const size_t bytes = sizeof(double) * Q * (size_t)I->hd.N;
    mlbm_status s = ensure_scratch(B, bytes);
    if (s != MLBM_OK) return s;
    HIP_TRY(launch_decode(I->hd, B->st, parity_of(*I), B->d_scratch, B->stream));
    HIP_TRY(hipMemcpyAsync(f, B->d_scratch, bytes, hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    return MLBM_OK;
}

mlbm_status mlbm_set_populations(mlbm_handle h, const double *f)
{
    Instance *I = inst_of(h);
    if (!I || !f) return fail(MLBM_E_ARG, "null argument");
    Batch *B = h->b;
    const size_t bytes = sizeof(double) * Q * (size_t)I->hd.N;
    mlbm_status s = ensure_scratch(B, bytes);
    if (s != MLBM_OK) return s;
    HIP_TRY(hipMemcpyAsync(B->d_scratch, f, bytes, hipMemcpyHostToDevice, B->stream));
    HIP_TRY(launch_encode(I->hd, B->st, parity_of(*I), B->d_scratch, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    return MLBM_OK;
}

mlbm_status mlbm_populations_device(mlbm_handle h, double *f, int get)
{
    Instance *I = inst_of(h);
    if (!I || !f) return fail(MLBM_E_ARG, "null argument");
    Batch *B = h->b;
    if (get) HIP_TRY(launch_decode(I->hd, B->st, parity_of(*I), f, B->stream));
    else HIP_TRY(launch_encode(I->hd, B->st, parity_of(*I), f, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    return MLBM_OK;
}

mlbm_status mlbm_moments(mlbm_handle h, double *rho, double *u, int on_device)
{
    Instance *I = inst_of(h);
    if (!I) return fail(MLBM_E_ARG, "null handle");
    Batch *B = h->b;
    const size_t N = (size_t)I->hd.N;
    double *drho = rho, *du = u;
    if (!on_device) {
        mlbm_status s = ensure_scratch(B, sizeof(double) * 4 * N);
        if (s != MLBM_OK) return s;
        drho = rho ? B->d_scratch : nullptr;
        du = u ? B->d_scratch + N : nullptr;
    }
    HIP_TRY(launch_moments(B->d_insts + h->idx, I->hd, B->st, parity_of(*I), drho, du, B->stream));
    if (!on_device) {
        if (rho) HIP_TRY(hipMemcpyAsync(rho, drho, sizeof(double) * N, hipMemcpyDeviceToHost, B->stream));
        if (u) HIP_TRY(hipMemcpyAsync(u, du, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, B->stream));
    }
    HIP_TRY(hipStreamSynchronize(B->stream));
    return MLBM_OK;
}

// Observables over the theta slabs [x2lo, x2hi): moments into the batch
// scratch, per-block partial sums on the device, the block sums in block
// order on the host.
static mlbm_status vortex_over_slabs(mlbm_handle h, int x2lo, int x2hi, double *omega_mean, double *v_mean,
                                     double *De)
{
    Instance *I = inst_of(h);
    Batch *B = h->b;
    const size_t N = (size_t)I->hd.N;
    const int nb = (int)((N + 255) / 256);
    mlbm_status s = ensure_scratch(B, sizeof(double) * (3 * N + 3 * (size_t)nb));
    if (s != MLBM_OK) return s;
    double *du = B->d_scratch, *dpart = B->d_scratch + 3 * N;
    HIP_TRY(launch_moments(B->d_insts + h->idx, I->hd, B->st, parity_of(*I), nullptr, du, B->stream));
    int nblocks = 0;
    const mlbm_desc &d = I->desc;
    HIP_TRY(launch_vortex(I->hd, d.kind, d.b, I->dt * I->hd.s[0], I->dt * I->hd.s[2], x2lo, x2hi, du, dpart,
                          &nblocks, B->stream));
    std::vector<double> part(3 * (size_t)nblocks);
    HIP_TRY(hipMemcpyAsync(part.data(), dpart, sizeof(double) * part.size(), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    double vs = 0.0, os = 0.0, as = 0.0;
    for (int k = 0; k < nblocks; ++k) { vs += part[3 * k]; os += part[3 * k + 1]; as += part[3 * k + 2]; }
    observables_from_sums(*I, vs, os, as, omega_mean, v_mean, De);
    return MLBM_OK;
}

mlbm_status mlbm_vortex_intensity(mlbm_handle h, double *omega_mean, double *v_mean, double *De)
{
    Instance *I = inst_of(h);
    if (!I) return fail(MLBM_E_ARG, "null handle");
    return vortex_over_slabs(h, 0, I->desc.n2, omega_mean, v_mean, De);
}

mlbm_status mlbm_vortex_intensity_slabs(mlbm_handle h, int x2_begin, int x2_end, double *omega_mean,
                                        double *v_mean, double *De)
{
    Instance *I = inst_of(h);
    if (!I) return fail(MLBM_E_ARG, "null handle");
    if (x2_begin < 0 || x2_end > I->desc.n2 || x2_begin >= x2_end)
        return fail(MLBM_E_ARG, "mlbm_vortex_intensity_slabs: slab range [" + std::to_string(x2_begin) + ", " +
                                    std::to_string(x2_end) + ") is empty or outside [0, " +
                                    std::to_string(I->desc.n2) + ")");
    return vortex_over_slabs(h, x2_begin, x2_end, omega_mean, v_mean, De);
}

mlbm_status mlbm_vortex_intensity_noalloc(mlbm_handle h, double *omega_mean, double *v_mean, double *De)
{
    Instance *I = inst_of(h);
    if (!I) return fail(MLBM_E_ARG, "null handle");
    Batch *B = h->b;
    const size_t N = (size_t)I->hd.N;
    const size_t nb = (N + 255) / 256;
    const size_t need = noalloc_vortex_doubles(N);
    if (need > NOALLOC_SCRATCH_DOUBLES)
        return fail(MLBM_E_ARG, "mlbm_vortex_intensity_noalloc: " + std::to_string(N) + " nodes need " +
                                    std::to_string(need * sizeof(double)) + " bytes of scratch, above the " +
                                    std::to_string(NOALLOC_SCRATCH_DOUBLES * sizeof(double)) + "-byte maximum");
    double *ptr = nullptr;
    mlbm_status s = noalloc_scratch(B->dev, &ptr);
    if (s != MLBM_OK) return s;
    // velocity field [3][N], then the per-block triples, then the three sums;
    // every element read is written earlier in the same call
    double *du = ptr, *dpart = ptr + 3 * N, *dsum = dpart + 3 * nb;
    HIP_TRY(launch_moments(B->d_insts + h->idx, I->hd, B->st, parity_of(*I), nullptr, du, B->stream));
    int nblocks = 0;
    const mlbm_desc &d = I->desc;
    HIP_TRY(launch_vortex(I->hd, d.kind, d.b, I->dt * I->hd.s[0], I->dt * I->hd.s[2], 0, d.n2, du, dpart,
                          &nblocks, B->stream));
    HIP_TRY(launch_sum_partials(dpart, nblocks, dsum, B->stream));
    double sums[3] = {0.0, 0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(sums, dsum, sizeof(sums), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    observables_from_sums(*I, sums[0], sums[1], sums[2], omega_mean, v_mean, De);
    return MLBM_OK;
}

mlbm_status mlbm_step_nodes(mlbm_handle h, const int64_t *nodes, int64_t count, double *out)
{
    Instance *I = inst_of(h);
    if (!I || (count > 0 && (!nodes || !out))) return fail(MLBM_E_ARG, "null argument");
    if (count <= 0) return MLBM_OK;
    for (int64_t k = 0; k < count; ++k)
        if (nodes[k] < 0 || nodes[k] >= I->hd.N) return fail(MLBM_E_ARG, "node index out of range");
    Batch *B = h->b;
    const size_t bytes_nodes = sizeof(int64_t) * (size_t)count, bytes_out = sizeof(double) * Q * (size_t)count;
    mlbm_status s = ensure_scratch(B, bytes_out + bytes_nodes + 64);
    if (s != MLBM_OK) return s;
    double *dout = B->d_scratch;
    int64_t *dn = (int64_t *)(B->d_scratch + Q * (size_t)count);
    HIP_TRY(hipMemcpyAsync(dn, nodes, bytes_nodes, hipMemcpyHostToDevice, B->stream));
    HIP_TRY(launch_step_nodes(B->d_insts + h->idx, I->hd, B->pat, B->st, parity_of(*I), dn, count, dout, B->stream));
    HIP_TRY(hipMemcpyAsync(out, dout, bytes_out, hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    return MLBM_OK;
}

mlbm_status mlbm_batch_set_launch(mlbm_batch b, int block, int grid)
{
    if (!b) return fail(MLBM_E_ARG, "null batch");
    if (block != 64 && block != 128 && block != 256 && block != 512) return fail(MLBM_E_ARG, "block must be 64, 128, 256 or 512");
    if (grid < 0) return fail(MLBM_E_ARG, "grid < 0");
    Batch *B = b->b;
    B->block = block;
    B->grid = grid;
    return build_tiles(B);
}

mlbm_status mlbm_batch_use_graph(mlbm_batch b, int on)
{
    if (!b) return fail(MLBM_E_ARG, "null batch");
    b->b->use_graph = on != 0;
    return MLBM_OK;
}

mlbm_status mlbm_batch_autotune(mlbm_batch b, int steps, int *best_block, int *best_grid)
{
    if (!b || steps < 2) return fail(MLBM_E_ARG, "null batch or steps < 2");
    Batch *B = b->b;
    if (steps & 1) ++steps;
    // back up the current populations of the active instances
    std::vector<void *> backup(B->inst.size(), nullptr);
    std::vector<uint32_t> ctr_backup(2 * B->inst.size(), 0);   // stochastic-rounding step counters
    const size_t sb = storage_bytes(B->st);
    for (size_t i = 0; i < B->inst.size(); ++i) {
        Instance &I = B->inst[i];
        if (!I.active) continue;
        const size_t bytes = sb * storage_values(I.hd);
        hipError_t e = hipMalloc(&backup[i], bytes);
        if (e == hipSuccess)
            e = hipMemcpyAsync(backup[i], I.hd.f[parity_of(I)], bytes, hipMemcpyDeviceToDevice, B->stream);
        if (e == hipSuccess && I.hd.ctr)
            e = hipMemcpyAsync(ctr_backup.data() + 2 * i, I.hd.ctr, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                               B->stream);
        if (e != hipSuccess) {                      // nothing stepped yet: drop the backups taken so far
            (void)hipStreamSynchronize(B->stream);
            for (void *p : backup)
                if (p) (void)hipFree(p);
            return fail(e == hipErrorOutOfMemory ? MLBM_E_OOM : MLBM_E_HIP,
                        std::string("autotune backup: ") + hipGetErrorString(e));
        }
    }
    const int blocks[4] = {64, 128, 256, 512};
    const int grids[4] = {0, 2 * B->num_cu, 4 * B->num_cu, 8 * B->num_cu};
    const int old_block = B->block, old_grid = B->grid;
    float best = 1e30f;
    int bb = old_block, bg = old_grid;
    const int64_t t_keep = B->t;
    mlbm_status st = MLBM_OK;
    // bring clocks and caches to a steady state before comparing shapes
    {
        B->block = 256;
        B->grid = 0;
        if ((st = build_tiles(B)) == MLBM_OK) {
            StepArgs a{B->d_insts, B->d_tiles, B->d_ntiles, B->d_partials, 0};
            for (int k = 0; k < 4 * steps; ++k) {
                a.parity = (int)((t_keep + k) & 1);
                if (launch_step(a, B->pat, B->st, false, B->eqw, launch_grid(B), B->block, B->stream) != hipSuccess) st = MLBM_E_HIP;
            }
        }
    }
    for (int ib = 0; ib < 4 && st == MLBM_OK; ++ib) {
        for (int ig = 0; ig < 4 && st == MLBM_OK; ++ig) {
            B->block = blocks[ib];
            B->grid = grids[ig];
            if ((st = build_tiles(B)) != MLBM_OK) break;
            if (grids[ig] > 0 && grids[ig] >= B->ntiles) continue;
            StepArgs a{B->d_insts, B->d_tiles, B->d_ntiles, B->d_partials, 0};
            for (int k = 0; k < 2; ++k) {
                a.parity = (int)((t_keep + k) & 1);
                if (launch_step(a, B->pat, B->st, false, B->eqw, launch_grid(B), B->block, B->stream) != hipSuccess) st = MLBM_E_HIP;
            }
            float cand = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                if (hipEventRecord(B->ev0, B->stream) != hipSuccess) st = MLBM_E_HIP;
                for (int k = 0; k < steps; ++k) {
                    a.parity = (int)((t_keep + k) & 1);
                    if (launch_step(a, B->pat, B->st, false, B->eqw, launch_grid(B), B->block, B->stream) != hipSuccess) st = MLBM_E_HIP;
                }
                float ms = 0.0f;
                if (hipEventRecord(B->ev1, B->stream) != hipSuccess || hipEventSynchronize(B->ev1) != hipSuccess ||
                    hipEventElapsedTime(&ms, B->ev0, B->ev1) != hipSuccess)
                    st = MLBM_E_HIP;
                cand = std::min(cand, ms);
            }
            if (cand < best) { best = cand; bb = blocks[ib]; bg = grids[ig]; }
        }
    }
    for (size_t i = 0; i < B->inst.size(); ++i) {
        if (!backup[i]) continue;
        Instance &I = B->inst[i];
        const size_t bytes = sb * storage_values(I.hd);
        if (hipMemcpyAsync(I.hd.f[parity_of(I)], backup[i], bytes, hipMemcpyDeviceToDevice, B->stream) != hipSuccess)
            st = MLBM_E_HIP;
        if (I.hd.ctr && hipMemcpyAsync(I.hd.ctr, ctr_backup.data() + 2 * i, 2 * sizeof(uint32_t), hipMemcpyHostToDevice,
                                       B->stream) != hipSuccess)
            st = MLBM_E_HIP;
    }
    if (hipStreamSynchronize(B->stream) != hipSuccess) st = MLBM_E_HIP;
    for (void *p : backup)
        if (p) (void)hipFree(p);
    if (st != MLBM_OK) {
        B->block = old_block;
        B->grid = old_grid;
        (void)build_tiles(B);
        return fail(st, "autotune launch, timing or state restore failed");
    }
    B->block = bb;
    B->grid = bg;
    if (best_block) *best_block = bb;
    if (best_grid) *best_grid = bg;
    return build_tiles(B);
}

// ---------------- checkpoints ---------------------------------------------

static const char CK_MAGIC[8] = {'M', 'L', 'B', 'M', 'C', 'K', '0', '6'};

mlbm_status mlbm_save(mlbm_handle h, const char *path)
{
    Instance *I = inst_of(h);
    if (!I || !path) return fail(MLBM_E_ARG, "null argument");
    Batch *B = h->b;
    const size_t N = (size_t)I->hd.N, sb = storage_bytes(B->st);
    std::vector<char> pops(sb * storage_values(I->hd));   // storage layout, padding included
    std::vector<double> us(3 * N);
    std::vector<float> ref(I->hd.ref ? (size_t)Q * I->hd.n1 : 0);
    std::vector<WindowState> ws;
    mlbm_status s = read_ws(B, ws);
    if (s != MLBM_OK) return s;
    HIP_TRY(hipMemcpyAsync(pops.data(), I->hd.f[parity_of(*I)], pops.size(), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipMemcpyAsync(us.data(), I->hd.usnap, sizeof(double) * us.size(), hipMemcpyDeviceToHost, B->stream));
    uint32_t ctr = 0;
    if (!ref.empty()) {
        HIP_TRY(hipMemcpyAsync(ref.data(), I->hd.ref, sizeof(float) * ref.size(), hipMemcpyDeviceToHost, B->stream));
        HIP_TRY(hipMemcpyAsync(&ctr, I->hd.ctr + parity_of(*I), sizeof(uint32_t), hipMemcpyDeviceToHost, B->stream));
    }
    HIP_TRY(hipStreamSynchronize(B->stream));
    FILE *fp = fopen(path, "wb");
    if (!fp) return fail(MLBM_E_IO, std::string("cannot open ") + path);
    mlbm_desc d = I->desc;
    d.init_u = nullptr;
    const int64_t t = I->t;
    bool ok = fwrite(CK_MAGIC, 1, 8, fp) == 8 && fwrite(&d, sizeof(d), 1, fp) == 1 && fwrite(&t, sizeof(t), 1, fp) == 1 &&
              fwrite(&ws[h->idx], sizeof(WindowState), 1, fp) == 1 && fwrite(pops.data(), 1, pops.size(), fp) == pops.size() &&
              fwrite(us.data(), sizeof(double), us.size(), fp) == us.size() &&
              fwrite(ref.data(), sizeof(float), ref.size(), fp) == ref.size() &&
              (ref.empty() || fwrite(&ctr, sizeof(ctr), 1, fp) == 1);
    ok = (fclose(fp) == 0) && ok;
    return ok ? MLBM_OK : fail(MLBM_E_IO, std::string("write failed: ") + path);
}

mlbm_status mlbm_load(const char *path, void *hip_stream, mlbm_handle *out)
{
    if (!path || !out) return fail(MLBM_E_ARG, "null argument");
    FILE *fp = fopen(path, "rb");
    if (!fp) return fail(MLBM_E_IO, std::string("cannot open ") + path);
    char mg[8];
    mlbm_desc d{};
    int64_t t = 0;
    WindowState w{};
    bool ok = fread(mg, 1, 8, fp) == 8 && !memcmp(mg, CK_MAGIC, 8) && fread(&d, sizeof(d), 1, fp) == 1 &&
              fread(&t, sizeof(t), 1, fp) == 1 && fread(&w, sizeof(w), 1, fp) == 1;
    if (!ok) {
        fclose(fp);
        return fail(MLBM_E_IO, "not an mlbm checkpoint");
    }
    d.init_u = nullptr;
    if (validate(d) != MLBM_OK) {
        fclose(fp);
        return fail(MLBM_E_IO, "checkpoint description invalid: " + g_err);
    }
    const size_t N = (size_t)d.n1 * d.n2 * d.n3, sb = storage_bytes(d.precision);
    std::vector<char> pops(sb * (size_t)Q * d.n1 * d.n2 * x3_pitch(d.n3));
    std::vector<double> us(3 * N);
    std::vector<float> ref(uses_ref(d.precision) ? (size_t)Q * d.n1 : 0);
    uint32_t ctr = 0;
    ok = fread(pops.data(), 1, pops.size(), fp) == pops.size() && fread(us.data(), sizeof(double), us.size(), fp) == us.size() &&
         fread(ref.data(), sizeof(float), ref.size(), fp) == ref.size() &&
         (ref.empty() || fread(&ctr, sizeof(ctr), 1, fp) == 1);
    fclose(fp);
    if (!ok) return fail(MLBM_E_IO, "checkpoint truncated");
    mlbm_handle h = nullptr;
    mlbm_status s = mlbm_init_geometry(&d, hip_stream, &h);
    if (s != MLBM_OK) return s;
    Batch *B = h->b;
    Instance &I = B->inst[0];
    I.t = t;
    B->t = t;
    hipError_t e = hipMemcpyAsync(I.hd.f[parity_of(I)], pops.data(), pops.size(), hipMemcpyHostToDevice, B->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(I.hd.usnap, us.data(), sizeof(double) * us.size(), hipMemcpyHostToDevice, B->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B->d_ws, &w, sizeof(w), hipMemcpyHostToDevice, B->stream);
    if (e == hipSuccess && !ref.empty())
        e = hipMemcpyAsync(const_cast<float *>(I.hd.ref), ref.data(), sizeof(float) * ref.size(), hipMemcpyHostToDevice,
                           B->stream);
    if (e == hipSuccess && !ref.empty())
        e = hipMemcpyAsync(I.hd.ctr + parity_of(I), &ctr, sizeof(uint32_t), hipMemcpyHostToDevice, B->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) {
        mlbm_destroy(h);
        return fail(MLBM_E_HIP, std::string("checkpoint upload: ") + hipGetErrorString(e));
    }
    *out = h;
    return MLBM_OK;
}

}  // extern "C"
