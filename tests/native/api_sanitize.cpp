// The library's host runtime (descriptor validation, batches, tile queues,
// retirement, graphs, checkpoints, the warm-start network) driven through
// the C ABI, with its host code built with AddressSanitizer and
// UndefinedBehaviorSanitizer (paper_1411_3133_amd/build.py, target
// api_sanitize; device code is built as usual). Run on a GPU by
// tests/test_gpu_sanitize.py; exits 0 when every call behaves as its
// declaration says, and the sanitizers abort on any invalid host access.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/mlbm.h"

static int failures = 0;
#define EXPECT(cond)                                                                              \
    do {                                                                                          \
        if (!(cond)) {                                                                            \
            std::fprintf(stderr, "FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond, mlbm_last_error()); \
            ++failures;                                                                           \
        }                                                                                         \
    } while (0)

static mlbm_desc cylinder(int n1, int n2, int n3, int precision, double De, uint64_t seed)
{
    mlbm_desc d{};
    d.kind = MLBM_CYLINDER;
    d.n1 = n1; d.n2 = n2; d.n3 = n3;
    d.walls = MLBM_WALL_AXIS1;
    d.precision = precision;
    d.check_every = 100;
    d.r_inner = 1.0; d.width = 1.0 / 9.0; d.b = 1.0; d.tau = 0.8;
    d.target_De = De; d.perturb_amp = 1e-4; d.seed = seed;
    return d;
}

int main(int argc, char **argv)
{
    std::setvbuf(stdout, nullptr, _IONBF, 0);
    const std::string dir = argc > 1 ? argv[1] : "/tmp";
    // invalid descriptions are refused, not read past
    {
        mlbm_desc d = cylinder(16, 4, 32, MLBM_F64, 20.0, 1);
        d.n1 = 0;
        mlbm_handle h = nullptr;
        EXPECT(mlbm_init_geometry(&d, nullptr, &h) == MLBM_E_ARG && h == nullptr);
        d = cylinder(16, 4, 32, MLBM_F64, 20.0, 1);
        d.tau = 0.5;
        EXPECT(mlbm_init_geometry(&d, nullptr, &h) == MLBM_E_ARG);
        EXPECT(mlbm_batch_create(nullptr, 1, nullptr, nullptr) == MLBM_E_ARG);
    }
    // a single instance: steps, observables, populations, checkpoint
    {
        mlbm_desc d = cylinder(16, 4, 32, MLBM_F32, 20.0, 5);
        mlbm_handle h = nullptr;
        EXPECT(mlbm_init_geometry(&d, nullptr, &h) == MLBM_OK);
        EXPECT(mlbm_step(h, 250) == MLBM_OK && mlbm_time(h) == 250);
        const int64_t N = 16 * 4 * 32;
        std::vector<double> rho(N), u(3 * N), f(41 * N);
        EXPECT(mlbm_moments(h, rho.data(), u.data(), 0) == MLBM_OK && std::isfinite(u[N + 5]));
        double om = 0, v = 0, De = 0, om2 = 0, v2 = 0, De2 = 0;
        EXPECT(mlbm_vortex_intensity(h, &om, &v, &De) == MLBM_OK && De > 0);
        EXPECT(mlbm_vortex_intensity_noalloc(h, &om2, &v2, &De2) == MLBM_OK && De2 == De && om2 == om);
        EXPECT(mlbm_vortex_intensity_slabs(h, 0, 4, &om2, &v2, &De2) == MLBM_OK && De2 == De && om2 == om);
        EXPECT(mlbm_vortex_intensity_slabs(h, 1, 2, &om2, nullptr, &De2) == MLBM_OK && std::isfinite(De2));
        EXPECT(mlbm_vortex_intensity_slabs(h, 2, 2, &om2, &v2, &De2) == MLBM_E_ARG);
        EXPECT(mlbm_vortex_intensity_slabs(h, 0, 5, &om2, &v2, &De2) == MLBM_E_ARG);
        EXPECT(mlbm_get_populations(h, f.data()) == MLBM_OK);
        EXPECT(mlbm_set_populations(h, f.data()) == MLBM_OK);
        const std::string ck = dir + "/api_sanitize.ckpt";
        EXPECT(mlbm_save(h, ck.c_str()) == MLBM_OK);
        mlbm_handle g = nullptr;
        EXPECT(mlbm_load(ck.c_str(), nullptr, &g) == MLBM_OK && mlbm_time(g) == 250);
        EXPECT(mlbm_step(h, 100) == MLBM_OK && mlbm_step(g, 100) == MLBM_OK);
        std::vector<double> fa(41 * N), fb(41 * N);
        EXPECT(mlbm_get_populations(h, fa.data()) == MLBM_OK && mlbm_get_populations(g, fb.data()) == MLBM_OK);
        EXPECT(fa == fb);
        EXPECT(mlbm_load((dir + "/no_such_file").c_str(), nullptr, &g) != MLBM_OK);
        int64_t nodes[3] = {0, 17, N - 1};
        std::vector<double> out(3 * 41);
        EXPECT(mlbm_step_nodes(h, nodes, 3, out.data()) == MLBM_OK);
        nodes[1] = N;   // out of range: refused
        EXPECT(mlbm_step_nodes(h, nodes, 3, out.data()) == MLBM_E_ARG);
        mlbm_destroy(g);
        mlbm_destroy(h);
    }
    // a batch of uneven instances: run_until with retirement across calls,
    // views, the caller's retire, a persistent grid, eager and graph windows
    {
        std::vector<mlbm_desc> ds = {cylinder(16, 4, 32, MLBM_F32, 10.0, 1), cylinder(12, 4, 20, MLBM_F32, 20.0, 2),
                                     cylinder(20, 2, 40, MLBM_F32, 30.0, 3)};
        mlbm_batch b = nullptr;
        EXPECT(mlbm_batch_create(ds.data(), (int)ds.size(), nullptr, &b) == MLBM_OK && mlbm_batch_size(b) == 3);
        EXPECT(mlbm_batch_keep_retired(b, 1) == MLBM_OK);
        int64_t steps[3]; double res[3]; int32_t st[3];
        EXPECT(mlbm_batch_run_until(b, 1e-6, 2000, steps, res, st) == MLBM_OK);
        EXPECT(mlbm_batch_retire(b, 2) == MLBM_OK);
        EXPECT(mlbm_batch_retire(b, 3) == MLBM_E_ARG);
        EXPECT(mlbm_batch_run_until(b, 1e-6, 2000, steps, res, st) == MLBM_OK && st[2] == 3);
        EXPECT(mlbm_batch_set_launch(b, 128, 512) == MLBM_OK);
        EXPECT(mlbm_batch_use_graph(b, 0) == MLBM_OK && mlbm_batch_step(b, 300) == MLBM_OK);
        EXPECT(mlbm_batch_use_graph(b, 1) == MLBM_OK && mlbm_batch_step(b, 300) == MLBM_OK);
        EXPECT(mlbm_batch_keep_retired(b, 0) == MLBM_OK && mlbm_batch_step(b, 200) == MLBM_OK);
        mlbm_handle view = nullptr;
        EXPECT(mlbm_batch_get(b, 1, &view) == MLBM_OK);
        std::vector<double> rho(12 * 4 * 20), u(3 * 12 * 4 * 20);
        EXPECT(mlbm_moments(view, rho.data(), u.data(), 0) == MLBM_OK);
        EXPECT(mlbm_step(view, 1) == MLBM_E_STATE);
        mlbm_handle none = nullptr;
        EXPECT(mlbm_batch_get(b, 7, &none) == MLBM_E_ARG && none == nullptr);
        mlbm_batch_destroy(b);
        mlbm_destroy(view);   // a view outliving its batch frees only itself
    }
    // the warm-start network: create, data, train, save, load, predict
    {
        EXPECT(mlbm_net_num_params(16, 2) == -1);   // hidden width 32 or 64 only
        const int H = 32, depth = 2;
        const int64_t np = mlbm_net_num_params(H, depth);
        EXPECT(np > 0);
        if (np <= 0) return 1;
        std::vector<double> p((size_t)np, 0.01);
        mlbm_net net = nullptr;
        EXPECT(mlbm_net_create(H, depth, p.data(), nullptr, &net) == MLBM_OK);
        mlbm_desc d = cylinder(12, 4, 20, MLBM_F64, 20.0, 9);
        const int64_t N = 12 * 4 * 20;
        std::vector<double> u(3 * N, 0.0);
        for (int64_t i = 0; i < N; ++i) u[N + i] = 1.0;
        EXPECT(mlbm_net_dataset_add(net, &d, 20.0, 9.0, 0.0, 1.0, u.data(), 0) == MLBM_OK);
        double loss = 0;
        EXPECT(mlbm_net_train(net, 20, 64, 1e-3, 1, &loss) == MLBM_OK && std::isfinite(loss));
        const std::string wf = dir + "/api_sanitize.net";
        EXPECT(mlbm_warmstart_save(net, wf.c_str()) == MLBM_OK);
        mlbm_net net2 = nullptr;
        EXPECT(mlbm_warmstart_load(wf.c_str(), nullptr, &net2) == MLBM_OK);
        std::vector<double> a(3 * N), c(3 * N);
        EXPECT(mlbm_warmstart_predict(net, &d, 20.0, 9.0, 0.0, 1.0, a.data(), 0) == MLBM_OK);
        EXPECT(mlbm_warmstart_predict(net2, &d, 20.0, 9.0, 0.0, 1.0, c.data(), 0) == MLBM_OK);
        EXPECT(a == c);
        mlbm_net_destroy(net2);
        mlbm_net_destroy(net);
    }
    std::printf("api_sanitize: %d failure(s)\n", failures);
    return failures ? 1 : 0;
}
