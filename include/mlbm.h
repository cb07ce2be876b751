/*
 * mlbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann library for
 * generalized metrics (Debus, Mendoza & Herrmann, "Dean Instability in
 * Double-Curved Channels", arXiv:1411.3133).
 *
 * One time step is the update of Sec. II, Eq. (3): pull streaming in
 * coordinate space with bounce-back walls and periodic axes, moments
 * (Sec. II, rho' = sum f, rho' u = sum c f), the metric Hermite equilibrium
 * through third order (Eq. (6) and the lattice f^eq that follows it), the
 * stress-corrected forcing with F_lambda^i = -Gamma^i_jk c^j c^k + F_ext^i
 * (the discrete forcing term after Eq. (7)), and BGK relaxation.
 *
 * Conventions used by every call:
 *  - Status codes are returned; no C++ exception crosses this boundary.
 *    mlbm_last_error() returns a thread-local message for the last failure.
 *  - The library owns every device allocation behind a handle.  Host
 *    pointers passed in are read (or written) during the call only and stay
 *    owned by the caller.
 *  - Node order is [x1][x2][x3] with x3 fastest: x1 = r (or x), x2 = theta
 *    (streamwise), x3 = z (cylinder) or phi (ellipsoid).  N = n1 n2 n3.
 *  - Velocity index lambda follows Table I: rest, (+-1,0,0), (0,+-1,0),
 *    (0,0,+-1), (+-1,+-1,0), (+-1,0,+-1), (0,+-1,+-1), (+-1,+-1,+-1),
 *    (+-3,0,0), (0,+-3,0), (0,0,+-3), (+-3,+-3,+-3); inside a group the
 *    signs run with "+" first and the last component fastest.
 *  - Velocities crossing the boundary are physical contravariant components
 *    u^i = dx^i/dt, laid out [3][N].  Densities are rho = rho' sqrt(g) (Sec. II).
 *  - A handle is bound to one HIP stream and is not thread safe.
 */
#ifndef MLBM_H
#define MLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MLBM_OK = 0,
    MLBM_E_ARG = 1,       /* invalid argument                                   */
    MLBM_E_HIP = 2,       /* a HIP runtime call failed                          */
    MLBM_E_OOM = 3,       /* device allocation failed                           */
    MLBM_E_UNSTABLE = 4,  /* a stationarity check found NaN, rho' <= 0 or |u| > 1 */
    MLBM_E_STATE = 5,     /* call not valid in the current state                */
    MLBM_E_IO = 6         /* checkpoint file could not be read or written       */
} mlbm_status;

typedef enum {
    MLBM_FLAT = 0,        /* Cartesian, g = delta, Gamma = 0                       */
    MLBM_CYLINDER = 1,    /* (r, theta, z), Sec. III                               */
    MLBM_ELLIPSOID = 2,   /* (r, theta, phi) with a = c = 1, Sec. IV, at theta = 0  */
    MLBM_ELLIPSOID_FULL = 3 /* the same coordinates with the metric of Sec. IV at
                           every node's theta (non-diagonal off theta = 0), on a
                           theta sector centred on 0, periodic in theta      */
} mlbm_kind;

typedef enum {
    MLBM_F64 = 0,         /* populations stored and collided in FP64              */
    MLBM_F32 = 1,         /* stored and collided in FP32                          */
    MLBM_F16 = 2,         /* stored as FP16 offsets, collided in FP32 (below)      */
    MLBM_BF16 = 3,        /* stored as BF16 offsets, collided in FP32 (below)      */
    MLBM_F32_C64 = 4      /* stored in FP32, collided in FP64                     */
} mlbm_precision;
/* 16-bit storage: population q at a node of x1 row i is stored as
 * f/w_q - 1 - r[i][q], r being the row mean of f/w_q - 1, taken from the
 * initial state at creation and again from the current state every 10
 * windows of check_every steps of the instance (right before it steps on
 * from such a step count; kept in checkpoints). Stores round
 * stochastically, seeded from (instance, node, step, q), so increments
 * below the storage resolution are kept on average; results are still
 * bitwise reproducible run to run, and do not depend on how the steps are
 * grouped into calls, batches or graphs. mlbm_set_populations and the
 * initial state round to nearest. */

enum { MLBM_WALL_AXIS1 = 1, MLBM_WALL_AXIS3 = 4, MLBM_WALL_EQUILIBRIUM = 8, MLBM_OPEN_AXIS2 = 16 };
enum { MLBM_FORCING_IMPROVED = 0, MLBM_FORCING_OLD = 1 };

/* Problem description, following the paper's statement of the problem
 * (Sec. III and Sec. IV): coordinate system and curvature, grid, tau,
 * driving force, walls, initial velocity.
 *  kind          mlbm_kind.
 *  n1, n2, n3    nodes along r, theta, z/phi; each >= 1, an axis with walls
 *                needs >= 4 nodes.
 *  walls         bit mask of MLBM_WALL_AXIS1 / MLBM_WALL_AXIS3 /
 *                MLBM_WALL_EQUILIBRIUM / MLBM_OPEN_AXIS2; axes without walls
 *                (and axis 2 unless open) are periodic.  Walls are halfway
 *                bounce-back walls, half a spacing outside the first and
 *                last node (Dt = Dr = d / n1).  With MLBM_WALL_EQUILIBRIUM
 *                (needs MLBM_WALL_AXIS1 and a periodic axis 3) the axis-1
 *                walls are instead the Dirichlet walls of Sec. III: the
 *                first and last x1 rows are wall nodes at r_i and r_o
 *                (Dt = Dr = d / (n1 - 1)), set every step to f_eq(rho',
 *                u = 0) with rho' the density streamed into them; they do
 *                not collide, a pull from beyond a wall node reads the wall
 *                node, and their velocity is reported as 0.  With
 *                MLBM_OPEN_AXIS2 (n2 >= 4) axis 2 is open at both ends, the
 *                inlet and outlet of Sec. IV: a pull from beyond an end slab
 *                reads that end slab (the populations entering the domain
 *                take the values they have at the end node); without it
 *                axis 2 is periodic.
 *  forcing_mode  MLBM_FORCING_IMPROVED (a2 = a2_eq - sigma) or MLBM_FORCING_OLD.
 *  precision     mlbm_precision.
 *  check_every   K, steps per stationarity window (even, >= 2); 0 means 100.
 *  r_inner       inner radius r_i (ignored for MLBM_FLAT).
 *  width         channel width d = r_o - r_i; Dt = Dr = d / n1 (bounce-back)
 *                or d / (n1 - 1) (equilibrium walls).
 *  b             ellipsoid semi-axis b (streamwise curvature radius r_i b^2).
 *  tau           BGK relaxation parameter, > 0.5.
 *  force         covariant streamwise body force K (physical units); the
 *                contravariant force is g^{i theta} K.
 *  init_u        NULL for rest, else the initial physical contravariant
 *                velocity (host, copied): 3 N doubles [3][N], or with
 *                init_u_xsec = 1 3 n1 n3 doubles [3][n1][n3] used in every
 *                theta slab.
 *  target_De     > 0: the body force is derived from this Dean number (Sec.
 *                III, Eq. (8)) through the closed-form laminar profile of a
 *                constant covariant force, v = A r ln r + B r + C / r with
 *                A = -K / (2 nu), nu = (tau - 1/2) cs2 Dt, on the channel of
 *                streamwise radius R (cylinder r_i, ellipsoid r_i b^2, whose
 *                force is then divided by b); flat: plane Poiseuille at
 *                Reynolds number De.  `force` must be 0.  0: use `force`.
 *  perturb_amp   > 0: start from that closed-form laminar profile (the mean
 *                speed U_nom of target_De, or 1 without it) plus
 *                perturb_amp U_nom xi of physical speed per cross-section
 *                node and component, xi in [-1, 1) from SplitMix64 (Steele,
 *                Lea & Flood 2014) keyed by `seed` (xi_i = (z_i >> 11)
 *                2^-52 - 1, z_i = splitmix64(i ^ (seed * 0x100000001B3)),
 *                i = (component n1 + x1) n3 + x3); init_u must be NULL.
 *  seed          key of the start perturbation.
 *  init_u_xsec   layout of init_u, see above.
 *  dtheta        MLBM_ELLIPSOID_FULL: theta spacing of the sector, nodes at
 *                theta = (x2 + 1/2 - n2/2) dtheta; 0 means the spacing of
 *                Sec. IV B, Dr / (b r_i).  Ignored by the other kinds. */
typedef struct {
    int32_t kind;
    int32_t n1, n2, n3;
    int32_t walls;
    int32_t forcing_mode;
    int32_t precision;
    int32_t check_every;
    double r_inner;
    double width;
    double b;
    double tau;
    double force;
    const double *init_u;
    double target_De;
    double perturb_amp;
    uint64_t seed;
    int32_t init_u_xsec;
    int32_t reserved;        /* 0 */
    double dtheta;
} mlbm_desc;

typedef struct mlbm_sim_s *mlbm_handle;
typedef struct mlbm_batch_s *mlbm_batch;

/* Create a single-instance simulation: validates `d`, computes the FP64
 * lattice geometry (metric, inverse, sqrt(g), Christoffels, unit force) on
 * the device, allocates populations and sets f* = f_eq(rho' = 1/sqrt(g), u)
 * (rho = 1 at t = 0, Sec. IV A).  `hip_stream` is a hipStream_t or NULL for
 * a stream the handle creates.  Errors: E_ARG, E_OOM, E_HIP. */
mlbm_status mlbm_init_geometry(const mlbm_desc *d, void *hip_stream, mlbm_handle *out);

/* Enqueue n time steps of Eq. (3) on the handle's stream and return without
 * waiting.  Every K-th step (counted from t = 0) also records the lattice
 * velocity and reduces the stationarity residual and the instability flag.
 * Errors: E_ARG (n < 0), E_HIP. */
mlbm_status mlbm_step(mlbm_handle h, int64_t n);

/* Moments of the current state as seen by the next collision: rho = rho'
 * sqrt(g) (N doubles) and physical contravariant u (3 N doubles, [3][N]).
 * Either pointer may be NULL.  on_device = 0: host buffers; 1: device
 * buffers.  Waits for the stream. */
mlbm_status mlbm_moments(mlbm_handle h, double *rho, double *u, int on_device);

/* Observables of Sec. III and Sec. IV from the current moments:
 * mean absolute streamwise vorticity <omega^theta> (Sec. III / Sec. IV
 * formulas, derivatives by second-order differences, one-sided next to
 * walls), mean streamwise velocity <v_theta> and the measured Dean number
 * De = <v_theta> d / nu sqrt(d / R) (Eq. (8)).  Averaged over theta slabs.
 * Waits for the stream. */
mlbm_status mlbm_vortex_intensity(mlbm_handle h, double *omega_mean, double *v_mean, double *De);

/* The same observables restricted to the theta slabs x2_begin <= x2 <
 * x2_end: every sum above runs over the nodes of those slabs only (the area
 * too), so a one-slab range gives the cross-section averages of Sec. IV at
 * that theta.  On the full ellipsoid the slab x2 sits at theta = (x2 + 1/2
 * - n2/2) dtheta, so theta = 0 lies between slabs n2/2 - 1 and n2/2 (pass
 * [n2/2 - 1, n2/2 + 1) for the pair around it).  [0, n2) gives
 * mlbm_vortex_intensity's values bit for bit.  Output pointers may be NULL.
 * Waits for the stream.  Errors: E_ARG (null handle; an empty range or one
 * outside [0, n2)), E_HIP. */
mlbm_status mlbm_vortex_intensity_slabs(mlbm_handle h, int x2_begin, int x2_end, double *omega_mean,
                                        double *v_mean, double *De);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same observables as
 * mlbm_vortex_intensity, bit for bit, computed with no device or host
 * allocation on success.  Its working memory is a fixed 16 MiB device array
 * inside the library, which each GPU the library runs on holds until the
 * process ends; it fits instances of up to 3 N + 3 ceil(N / 256) + 3 <= 2^21
 * doubles, i.e. N <= 696,000 nodes or so.  Larger instances get E_ARG and
 * nothing is launched.  The array is shared by every call on the same GPU,
 * so calls that overlap on one GPU (two host threads, or two streams) race
 * and must be serialised by the caller.  Output pointers may be NULL.  Waits
 * for the handle's stream.  Errors: E_ARG, E_HIP. */
mlbm_status mlbm_vortex_intensity_noalloc(mlbm_handle h, double *omega_mean, double *v_mean, double *De);

/* Residual of the last completed window: ||U_w - U_{w-1}|| / ||U_w|| over all
 * nodes and components (lattice units); -1 before two windows completed.
 * *bad receives the sticky instability flag.  Waits for the stream. */
mlbm_status mlbm_residual(mlbm_handle h, double *r, int *bad);

/* Advance whole windows until the residual is <= tol or max_steps are done.
 * Returns E_UNSTABLE when the flag trips. */
mlbm_status mlbm_run_until(mlbm_handle h, double tol, int64_t max_steps, int64_t *steps_taken);

/* Decoded populations f (absolute, FP64) of the current state, [41][N], host. */
mlbm_status mlbm_get_populations(mlbm_handle h, double *f);
/* Overwrite the current state (encoded into the storage precision). */
mlbm_status mlbm_set_populations(mlbm_handle h, const double *f);

/* The same two operations on a caller-owned device buffer f [41][N] (FP64,
 * absolute populations; e.g. a torch tensor's data pointer): get = 1
 * decodes the current state into it, get = 0 encodes it into the current
 * state.  Runs on the handle's stream and waits for it.  Errors: E_ARG,
 * E_HIP. */
mlbm_status mlbm_populations_device(mlbm_handle h, double *f, int get);

/* One step of the nodes listed, from the current state, without advancing:
 * out[k][41] = f* at node nodes[k] (host arrays), rounded through the
 * storage format as the step would store it.  With 16-bit storage at a
 * re-referencing step count it uses the current reference, not the one the
 * next step will re-take (the two differ by the storage rounding).  Waits
 * for the stream. */
mlbm_status mlbm_step_nodes(mlbm_handle h, const int64_t *nodes, int64_t count, double *out);

/* Pull map of the streaming step with walls, evaluated on the host with the
 * same fold the kernels use: for node n and velocity q the population is
 * read from node src_node[n*41 + q], velocity src_q[n*41 + q].  Caller-owned
 * host arrays of 41 N entries.  Needs no GPU.  Errors: E_ARG. */
mlbm_status mlbm_pull_map(const mlbm_desc *d, int64_t *src_node, int32_t *src_q);

/* Number of completed steps. */
int64_t mlbm_time(mlbm_handle h);

/* Checkpoint: raw storage-precision populations, step counter, the
 * description and, for 16-bit storage, the reference table and the rounding
 * step counter; resume is bitwise identical.  Errors: E_IO. */
mlbm_status mlbm_save(mlbm_handle h, const char *path);
mlbm_status mlbm_load(const char *path, void *hip_stream, mlbm_handle *out);

/* Free the handle and its device memory (NULL is ignored); for a batch
 * view, only the view handle. */
void mlbm_destroy(mlbm_handle h);

/* Thread-local text of the last error. */
const char *mlbm_last_error(void);

/* The library's D3Q41 table (Table I): c[41][3], w[41], c_s^2.  Returns 41. */
int mlbm_lattice(int32_t *c, double *w, double *cs2);

/* ---------------- batched persistent engine ---------------------------- */

/* Many instances advanced by one launch per step over a flat tile queue.
 * Every description must share `precision` and `check_every`; kinds,
 * sizes, tau, force and walls may differ.  Errors: E_ARG, E_OOM, E_HIP. */
mlbm_status mlbm_batch_create(const mlbm_desc *ds, int n, void *hip_stream, mlbm_batch *out);

/* Enqueue n steps of every active instance (asynchronous). */
mlbm_status mlbm_batch_step(mlbm_batch b, int64_t n);

/* Advance whole windows; an instance retires when its residual is <= tol,
 * when it becomes unstable or after max_steps.  steps[i] receives the steps
 * instance i took, residual[i] its last residual, status[i] 0 converged,
 * 1 hit max_steps, 2 unstable, 3 retired by the caller (each array may be
 * NULL). */
mlbm_status mlbm_batch_run_until(mlbm_batch b, double tol, int64_t max_steps, int64_t *steps,
                                 double *residual, int32_t *status);

/* Retirement across calls.  By default mlbm_batch_run_until brings every
 * instance back when it returns.  With mlbm_batch_keep_retired(b, 1) the
 * instances it retired as converged or unstable stay out of later
 * mlbm_batch_step / mlbm_batch_run_until calls, keeping their state and
 * step count (those that only reached the call's max_steps come back), and
 * mlbm_batch_retire(b, i) retires instance i at once (its status then reads
 * 3); mlbm_batch_keep_retired(b, 0) brings every instance back.  Retiring needs the batch on a window boundary (a step
 * count that is a multiple of check_every; E_STATE otherwise). */
mlbm_status mlbm_batch_keep_retired(mlbm_batch b, int on);
mlbm_status mlbm_batch_retire(mlbm_batch b, int i);

/* Non-owning view of instance i, usable until the batch is destroyed; every
 * single-instance query above (moments, vortex_intensity, residual,
 * get/set_populations, step_nodes, time) accepts it.  mlbm_step on a view
 * returns E_STATE.  mlbm_destroy on a view frees the view handle only (the
 * batch stays), before or after the batch is destroyed. */
mlbm_status mlbm_batch_get(mlbm_batch b, int i, mlbm_handle *view);

/* Launch shape: workgroup size (64, 128, 256, 512) and persistent grid
 * (0 = one workgroup per tile).  mlbm_batch_autotune times the candidate
 * shapes on the batch itself (hipEvents, `steps` steps each, state restored
 * afterwards) and keeps the fastest; best_block/best_grid may be NULL. */
mlbm_status mlbm_batch_set_launch(mlbm_batch b, int block, int grid);
mlbm_status mlbm_batch_autotune(mlbm_batch b, int steps, int *best_block, int *best_grid);

/* Capture K-step windows in a hipGraph (1, default) or launch eagerly (0). */
mlbm_status mlbm_batch_use_graph(mlbm_batch b, int on);

/* Mean device time per step of the step kernel measured with hipEvents on
 * the batch stream over the last mlbm_batch_step call (ms), -1 if none. */
double mlbm_batch_last_step_ms(mlbm_batch b);

int mlbm_batch_size(mlbm_batch b);
void mlbm_batch_destroy(mlbm_batch b);

/* ---------------- learned warm start ------------------------------------ */

/* A fully connected network 5 -> H -> ... -> H -> 3 (`depth` hidden layers,
 * SiLU, linear output, FP32) that maps (De, R1/d, R2/d, r, arc position) of a
 * cross-section node to its steady physical velocity over the nominal mean
 * speed; its prediction initialises a run instead of the laminar profile.
 * Parameters: per layer W [n_out][n_in] row-major, then b [n_out]. */
typedef struct mlbm_net_s *mlbm_net;

/* Number of parameters, or -1 if the shape is not supported (H in {32, 64},
 * 1 <= depth <= 6, parameters within 64 KiB). */
int64_t mlbm_net_num_params(int hidden, int depth);

/* Create a network from caller-owned initial parameters (host, copied). */
mlbm_status mlbm_net_create(int hidden, int depth, const double *init_params, void *hip_stream, mlbm_net *out);
void mlbm_net_destroy(mlbm_net n);
const char *mlbm_net_last_error(void);

/* Copy the parameters out (get = 1) or in (get = 0), host array. */
mlbm_status mlbm_net_params(mlbm_net n, double *params, int get);

/* Forward pass of n samples: x [n][5] -> y [n][3], host arrays. */
mlbm_status mlbm_net_forward(mlbm_net net, const float *x, int64_t n, float *y);

/* Mean squared error 1/(3n) sum (y - t)^2 of n samples (host arrays) and its
 * gradient with respect to the parameters (host, may be NULL); the gradient
 * stays on the device for mlbm_net_adam_step. */
mlbm_status mlbm_net_gradient(mlbm_net net, const float *x, const float *t, int64_t n, double *loss, double *grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the last gradient. */
mlbm_status mlbm_net_adam_step(mlbm_net net, double lr);

/* Append the cross-section nodes (theta slab 0) of a case to the device
 * training set: inputs from the description and (De, R1/d, R2/d), targets
 * from its velocity field u [3][N] (physical contravariant, e.g. from
 * mlbm_moments; host or device per on_device): the physical components
 * over U_nom, the two cross-section ones (x1, x3) multiplied by 10 so that
 * the loss weighs the secondary flow like the streamwise profile. */
mlbm_status mlbm_net_dataset_add(mlbm_net net, const mlbm_desc *d, double De, double R1_d, double R2_d,
                                 double U_nom, const double *u, int on_device);
mlbm_status mlbm_net_dataset_clear(mlbm_net net);
int64_t mlbm_net_dataset_size(mlbm_net net);

/* `steps` Adam steps on minibatches of `batch` samples drawn from the training
 * set by a counter-based hash of `seed`; *last_loss: loss of the last batch. */
mlbm_status mlbm_net_train(mlbm_net net, int64_t steps, int64_t batch, double lr, uint64_t seed, double *last_loss);

/* Loss over the whole training set. */
mlbm_status mlbm_net_dataset_loss(mlbm_net net, double *loss);

/* Parameters of a trained network to a file (its shape, then the
 * parameters in the order above as doubles), and a network created from
 * such a file on `hip_stream` (NULL: a stream of its own).  The Adam
 * moments are not kept.  Errors: E_ARG, E_IO (missing, truncated or of an
 * unsupported shape), E_OOM, E_HIP. */
mlbm_status mlbm_warmstart_save(mlbm_net net, const char *path);
mlbm_status mlbm_warmstart_load(const char *path, void *hip_stream, mlbm_net *out);

/* Predicted velocity field of a case, physical contravariant [3][N] (every
 * theta slab), ready to pass as mlbm_desc.init_u; host or device buffer. */
mlbm_status mlbm_warmstart_predict(mlbm_net net, const mlbm_desc *d, double De, double R1_d, double R2_d,
                                   double U_nom, double *u_out, int on_device);

#ifdef __cplusplus
}
#endif

#endif /* MLBM_H */
