/*
 * lbmp.h — C ABI of the MI355X moment-propagation library (liblbmp.so).
 *
 * Lattice-Boltzmann moment propagation with adsorption and desorption at
 * solid-liquid interfaces, after Levesque, Duvail, Pagonabarraga, Frenkel and
 * Rotenberg, "Accounting for adsorption and desorption in Lattice Boltzmann
 * simulations" (arXiv:1303.2470). All compute runs in hand-written HIP
 * kernels for gfx950; the host side only validates, carves workspaces and
 * launches.
 *
 * Conventions
 *  - Lattice units: dx = dt = 1. D3Q19 lattice (Sec. I).
 *  - A lattice is nx*ny*nz nodes; node index n = x + nx*(y + ny*z).
 *  - Every call returns an lbmp_status; nothing throws across the ABI.
 *    On a non-OK return lbmp_last_error() gives a message (thread-local).
 *  - Device memory is never allocated by the library: the caller passes
 *    device workspaces (any device pointer, 256-byte aligned) sized by the
 *    *_workspace_bytes queries, and a hipStream_t (as void*, NULL = default
 *    stream). A persistent workspace must outlive the handle built in it.
 *  - Host arrays are borrowed for the duration of a call only.
 *  - Calls on one handle are not thread-safe; different handles are.
 */
#ifndef LBMP_H
#define LBMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBMP_OK = 0,
    LBMP_EINVAL = -1,   /* invalid argument (shape, rates, parameters)           */
    LBMP_EDEVICE = -2,  /* HIP runtime error                                      */
    LBMP_ENOMEM = -3,   /* workspace too small                                    */
    LBMP_ENOTCONV = -4, /* flow solve hit max_steps before tol (flow still valid) */
    LBMP_EPROB = -5,    /* a stay probability is negative (sum p_i + p_a > 1)     */
    LBMP_ESTATE = -6,   /* call not allowed in the handle's state                 */
    LBMP_ENUMERIC = -7  /* non-finite value seen by the device watchdog           */
} lbmp_status;

typedef enum { LBMP_FP32 = 32, LBMP_FP64 = 64 } lbmp_precision;

/* Message for the last non-OK status returned on this thread. */
const char* lbmp_last_error(void);
/* Library version string. */
const char* lbmp_version(void);

/* ------------------------------------------------------------------ geometry
 * Solid/fluid nodes of a regular lattice (Sec. I). solid: host array of
 * nx*ny*nz bytes, 1 = solid. periodic[d] = 0 requires both boundary planes
 * normal to axis d to be solid. iface_nbhd selects the interfacial-node rule
 * (Sec. II, Eq. 11 node classes): a fluid node is interfacial when one of its
 * 18 D3Q19 neighbours (iface_nbhd = 18 or 0) or one of its 6 face neighbours
 * (iface_nbhd = 6) is solid. */
typedef struct {
    int nx, ny, nz;
    int periodic[3];
    const uint8_t* solid;
    int iface_nbhd;
} lbmp_geometry;

typedef struct lbmp_flow lbmp_flow; /* geometry + steady fluid velocity, on device */
typedef struct lbmp_mp lbmp_mp;     /* batched moment-propagation state, on device */

/* ------------------------------------------------------------------ fluid
 * Steady flow by the lattice-Boltzmann equation (Sec. I, Eq. 6): D3Q19 BGK with
 * relaxation time tau, body force density rho*force (Guo forcing), half-way
 * bounce-back on solid nodes, started at rest with rho = 1, in FP64. Every
 * check_every steps (0 = 100) the one-step change max|u(t)-u(t-1)|/max|u(t)|
 * is compared with tol. The node classes (solid / fluid / interfacial) and
 * the interfacial-node list are built here too.
 *
 * lb_flow_workspace_bytes: *persistent = bytes the flow keeps (geometry
 * classes, velocity); *scratch = bytes needed only during lb_flow_solve
 * (the populations). Returns LBMP_EINVAL on a bad geometry.
 * lb_flow_solve: *out receives a new handle living in dev_ws. Returns
 * LBMP_ENOTCONV (handle still created, flagged) when max_steps is reached
 * first; LBMP_EINVAL for tau <= 1/2, no fluid node, a non-periodic face that is
 * not solid, non-finite force; LBMP_ENOMEM for short workspaces. */
lbmp_status lb_flow_workspace_bytes(const lbmp_geometry* g, size_t* persistent, size_t* scratch);
lbmp_status lb_flow_solve(const lbmp_geometry* g, double tau, const double force[3], double tol,
                          int64_t max_steps, int check_every,
                          void* dev_ws, size_t ws_bytes, void* dev_scratch, size_t scratch_bytes,
                          void* hip_stream, lbmp_flow** out, int64_t* steps_done, double* residual);
/* The same solve without a scratch workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation). The populations, velocity history and
 * residual partials live in a file-scope device array of
 * LBMP_STATIC_SCRATCH_BYTES (128 MiB), which each GPU the library runs on
 * holds until the process ends; no hipMalloc, hipFree or allocating routine
 * is called. The caller still passes the persistent workspace dev_ws (the
 * returned handle lives there, as with lb_flow_solve). Arguments, results and
 * errors are those of lb_flow_solve, plus LBMP_ENOMEM for a lattice of more
 * than lb_flow_static_max_nodes() nodes (checked before any device work).
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (two host threads, or two streams) race and must be serialised by
 * the caller. */
#define LBMP_STATIC_SCRATCH_BYTES (128u << 20)
lbmp_status lb_flow_solve_static(const lbmp_geometry* g, double tau, const double force[3], double tol,
                                 int64_t max_steps, int check_every, void* dev_ws, size_t ws_bytes,
                                 void* hip_stream, lbmp_flow** out, int64_t* steps_done, double* residual);
/* Largest lattice (nx*ny*nz) lb_flow_solve_static accepts. */
int64_t lb_flow_static_max_nodes(void);
/* A flow handle from a given velocity field (host, FP64, [3][N] SoA, x then y
 * then z component; values on solid nodes are ignored). Uses dev_ws like
 * lb_flow_solve (persistent part only). */
lbmp_status lb_flow_from_velocity(const lbmp_geometry* g, const double* u_host, void* dev_ws,
                                  size_t ws_bytes, void* hip_stream, lbmp_flow** out);
/* Copies the velocity ([3][N], FP64, zero on solid nodes) to the host. */
lbmp_status lb_flow_velocity(const lbmp_flow* f, double* u_host);
/* Node classes (N bytes: 0 solid, 1 fluid, 2 interfacial) and counts. */
lbmp_status lb_flow_classes(const lbmp_flow* f, int8_t* cls_host, int64_t* n_fluid,
                            int64_t* n_iface);
void lb_flow_free(lbmp_flow* f);

/* ------------------------------------------------------------------ tracers
 * Species set for one geometry. The tracer's bulk diffusion is set by exactly
 * one of D_b (Sec. II: D_b = lambda c_s^2 dt / 4, so lambda = 12 D_b) or Delta,
 * the stay probability of a tracer on a bulk node at rest (Delta = 1 - lambda/3);
 * the other must be NaN. k_a[s], k_d[s]: adsorption (length/time) and
 * desorption (1/time) rates (Eq. 2), giving p_a = k_a dt/dx and p_d = k_d dt
 * (Sec. II, after Eq. 9). Requires k_a >= 0, 0 < k_d <= 1, 0 < lambda. */
typedef struct {
    double D_b, Delta;
    int n_species;
    const double* k_a;
    const double* k_d;
} lbmp_species;

/* Workspace for mp_init over n_geom flows, species[g] for flow g. */
lbmp_status mp_workspace_bytes(const lbmp_flow* const* flows, const lbmp_species* species,
                               int n_geom, int precision, int64_t max_steps_recorded,
                               size_t* bytes);
/*
 * Sets up the moment propagation for every (geometry, species) pair and
 * records t = 0 (Secs. II-III):
 *  - link probabilities p_i(r) = w_i (lambda/2 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2)
 *    (Eq. 8 with the local equilibrium distribution, Q = 1), zero for links
 *    into solid nodes; stay probability 1 - sum p_i - p_a [r interfacial];
 *  - initial Boltzmann weights (Eq. 11 without excess chemical potential);
 *  - the first-moment quantities P_g(r, 1), the velocity-weighted first hop;
 *  - Z_g(0) and the mean velocity V_g.
 * precision: LBMP_FP32 (propagation in FP32, every sum in FP64) or LBMP_FP64.
 * max_steps_recorded bounds the number of steps mp_step_n may run in total.
 * Returns LBMP_EPROB if some stay probability is negative, LBMP_EINVAL for bad
 * rates or parameters, LBMP_ENOMEM for a short workspace.
 */
lbmp_status mp_init(const lbmp_flow* const* flows, const lbmp_species* species, int n_geom,
                    int precision, int64_t max_steps_recorded, void* dev_ws, size_t ws_bytes,
                    void* hip_stream, lbmp_mp** out);
/*
 * Advances every (geometry, species) pair by n_steps steps of Eqs. 7, 9 and 10
 * (one simultaneous Markov step: adsorption takes p_a of the pre-step mobile
 * quantity, desorbed quantity re-enters at its node), recording the VACF of
 * Eq. 12 and the conserved totals at every step. Asynchronous on the stream.
 * LBMP_ESTATE if the total would exceed max_steps_recorded.
 */
lbmp_status mp_step_n(lbmp_mp* h, int64_t n_steps);
/* Device watchdog of the step: after every step the total probability
 * (mobile + adsorbed) of every species must stay within LBMP_MASS_DRIFT_MAX
 * of 1 and be finite; otherwise mp_vacf and mp_uptake return LBMP_ENUMERIC
 * naming the first step where it did not. The environment variable
 * LBMP_MASS_DRIFT_MAX, read by mp_init, overrides the threshold. */
#define LBMP_MASS_DRIFT_MAX 1e-6
/*
 * Synchronises the stream and returns, for geometry `geom`, times
 * t = t0 .. t0+count-1 (t <= steps done; t = 0 is the start):
 *  Z[(s*3+g)*count + k]  VACF Z_g(t) of species s (Eq. 12, g = x, y, z);
 *  D[(s*3+g)*count + k]  D_g(t) = (Z_g(0) - V_g^2)/2 + sum_{m=1..t}(Z_g(m) - V_g^2),
 *                        the discrete Eq. 3 about the mean drift (Eq. 4 as t grows);
 *  mass[s*2 + {0,1}]     total mobile and adsorbed probability at the last t;
 *  vbar[s*3 + g]         mean velocity V_g.
 * Any output pointer may be NULL. LBMP_ENUMERIC if a recorded value is not
 * finite or the watchdog (LBMP_MASS_DRIFT_MAX) fired.
 */
lbmp_status mp_vacf(lbmp_mp* h, int geom, int64_t t0, int64_t count, double* Z, double* D,
                    double* mass, double* vbar);
/* Steps done so far (0 right after mp_init). */
lbmp_status mp_steps_done(const lbmp_mp* h, int64_t* t);

/*
 * mp_init for charged tracers (Sec. II: the Q term of Eq. 8 and the excess
 * chemical potential of Eq. 11, whose mean-field electrostatic part is q psi).
 * beta_mu_ex[g]: host array of N doubles, the dimensionless excess chemical
 * potential beta mu^ex(r) of the tracers of geometry g at every node (e.g. the
 * valence times the reduced electrostatic potential), x fastest like the
 * geometry; values on solid nodes are ignored; NULL for a neutral geometry.
 * Every species of a geometry shares it (a flow may appear several times with
 * different species sets and potentials). With it:
 *  - p_i(r) = w_i (lambda Q_i(r)/2 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2),
 *    Q_i(r) = exp(-(beta mu^ex(r + c_i) - beta mu^ex(r)) / 2), the symmetric
 *    factor under which the Eq. 11 weights satisfy detailed balance at rest;
 *  - Eq. 11 weights exp(-beta mu^ex(r)) / Z on fluid nodes, times
 *    (1 + k_a / k_d) on interfacial nodes.
 * Otherwise as mp_init (same workspace size); LBMP_EINVAL also for a
 * non-finite beta_mu_ex at a fluid node, LBMP_EPROB when a Q factor makes a
 * stay probability negative.
 */
lbmp_status mp_init_charged(const lbmp_flow* const* flows, const lbmp_species* species,
                            const double* const* beta_mu_ex, int n_geom, int precision,
                            int64_t max_steps_recorded, void* dev_ws, size_t ws_bytes, void* hip_stream,
                            lbmp_mp** out);
/*
 * Out-of-equilibrium uptake (the outlook of the paper's conclusion: the
 * density as the propagated quantity of Eqs. 7, 9 and 10, irreversible
 * adsorption k_d = 0 allowed). Arguments as for mp_init, except that k_d may
 * be 0; every species starts at tau = 0 from the density 1/N_F on every fluid
 * node with nothing adsorbed. mp_step_n advances it; the handle records the
 * total mobile and adsorbed density of every species at every step and no
 * VACF (mp_vacf returns LBMP_ESTATE). Densities are stored as they are (no
 * reference weights), in FP32 with stochastic rounding or in FP64.
 */
lbmp_status mp_uptake_init(const lbmp_flow* const* flows, const lbmp_species* species, int n_geom,
                           int precision, int64_t max_steps_recorded, void* dev_ws, size_t ws_bytes,
                           void* hip_stream, lbmp_mp** out);
/*
 * Synchronises the stream and returns, for geometry `geom` and
 * tau = t0 .. t0+count-1 (tau < steps done: the totals of a state are
 * recorded by the step that reads it):
 *  mobile[s*count + k], adsorbed[s*count + k]  total mobile and adsorbed
 *  density of species s at tau = t0 + k.
 * Either pointer may be NULL. LBMP_ESTATE for a handle made by mp_init,
 * LBMP_EINVAL for times not recorded, LBMP_ENUMERIC for a non-finite total.
 */
lbmp_status mp_uptake(lbmp_mp* h, int geom, int64_t t0, int64_t count, double* mobile, double* adsorbed);

typedef struct {
    int64_t n_nodes, n_fluid, n_iface;
    double lambda;
    double min_p;          /* smallest link probability (can be < 0 at high cell Peclet) */
    double max_cell_peclet; /* max |u| / D_b over fluid nodes */
    double min_stay;       /* smallest stay probability over species */
    double mean_velocity[3];
    int tile_k;            /* variants 0, 1: z-planes per thread; 2: z-segment per block;
                              3, 5: block height in 64 x 4 tiles; 4, 6, 7: planes per block
                              (2; 4 for variant 6 when pinned); 8: 2 */
    int species_per_block; /* species per block chosen by the tile tuner */
    int kernel_variant;    /* 0: direct neighbour loads, 1: fields staged through LDS,
                              2: z-march with an LDS plane ring, 3: LDS-DMA copies (FP32),
                              4: LDS-DMA copies on blocks of 2 planes (FP32), 5 and 6:
                              variants 3 (64 x 8) and 4 with whole periodic rows, for
                              lattices 64 nodes wide (FP32; every geometry nx = 64), 7:
                              variant 4 with its fluid nodes packed onto the first
                              threads of a block (FP32; porous media), 8: gathered
                              chunks of up to 512 fluid nodes consecutive in a
                              tile-ordered compact storage, their halo copied
                              by per-node lists (FP32; porous media). The
                              tuner times them in mp_init; the environment variable
                              LBMP_TILE = "variant,tile_k,species_per_block" pins one
                              (mp_init returns LBMP_EINVAL for a choice the lattice or
                              the precision does not allow). */
} lbmp_stats;
/* Set-up statistics of geometry `geom`. */
lbmp_status mp_stats(const lbmp_mp* h, int geom, lbmp_stats* st);
/*
 * Copies the current state of one (geometry, species) to the host, in FP64:
 * X[q*N + n] the mobile quantity q (0 density, 1..3 first moments x, y, z),
 * Xads[q*N + n] the adsorbed quantity (zero off interfacial nodes).
 */
lbmp_status mp_state(lbmp_mp* h, int geom, int species, double* X, double* Xads);
/*
 * Runs n_steps steps exactly like mp_step_n, without graph replay, with HIP
 * events around every launch of the propagation kernel on the handle's
 * stream; synchronises and returns the summed propagation-kernel time and the
 * wall time of the whole sequence, in milliseconds. For measurement.
 */
lbmp_status mp_profile_steps(lbmp_mp* h, int64_t n_steps, double* ms_step_kernel, double* ms_total);
/*
 * Checkpoint and resume. A checkpoint is a host byte buffer holding the state
 * after the last step: the stored fields of every (geometry, species) in the
 * handle's storage precision (fluid nodes in lattice order, adsorbed values in
 * interface-list order, so it does not depend on the step kernel the tuner
 * chose), the recorded per-step sums and the watchdog's state, behind a
 * header with a fingerprint of the set-up (shapes, node counts, rates, Eq. 11
 * references, mean velocities, Z(0)).
 * mp_checkpoint_bytes: the size a checkpoint of h takes now.
 * mp_save: synchronises the stream and writes the checkpoint into host_buf
 *   (caller-owned, at least mp_checkpoint_bytes); LBMP_EINVAL if it is NULL or
 *   too small.
 * mp_load: restores a checkpoint into h, which must have been created for the
 *   same workload (same flows, species, precision and mode; LBMP_EINVAL
 *   otherwise, or for a buffer that is not a whole checkpoint) with
 *   max_steps_recorded at least the checkpoint's step (LBMP_ESTATE). Steps run
 *   after it give, with the same step kernel, the same bits as steps run
 *   without interruption.
 */
lbmp_status mp_checkpoint_bytes(const lbmp_mp* h, size_t* bytes);
lbmp_status mp_save(lbmp_mp* h, void* host_buf, size_t bytes);
lbmp_status mp_load(lbmp_mp* h, const void* host_buf, size_t bytes);
/* Synchronises the handle's stream and releases the handle. */
void mp_free(lbmp_mp* h);

/* ------------------------------------------------------------------ surrogate
 * A learned shortcut for the paper's first stated use (Sec. IV: predicting
 * D(t) for species of known k_a, k_d in a given medium, and the converse
 * extraction of k_a, k_d from D(t)): a network mapping the six features
 * (porosity, specific surface N_I/N, Peclet number, log10 k_a, log10 k_d,
 * log10 t) to log10(D_x(t)/D_b), trained on runs of the method above and
 * judged against it. Layers 6 -> 256 -> 256 -> 256 -> 1 with SiLU; BF16
 * matrix-core products with FP32 accumulation, FP32 master weights, Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8), loss mean((f(x) - y)^2) on z-scored
 * inputs and target. All compute on the device; device pointers below are
 * FP32 arrays: x [n][6], y [n], idx [B] (int32 row indices).
 */
typedef struct lbmp_sg lbmp_sg;
/* Number of trainable parameters (133,633). */
lbmp_status sg_param_count(int64_t* n);
/* Workspace for a network trained with batches up to batch_max (a multiple of 32). */
lbmp_status sg_workspace_bytes(int batch_max, size_t* bytes);
/* New network; weights and biases U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a
 * splitmix64 stream seeded with `seed`; identity normalisation. */
lbmp_status sg_create(int batch_max, uint64_t seed, void* dev_ws, size_t ws_bytes, void* hip_stream,
                      lbmp_sg** out);
/* Host parameter vector (FP32), layer by layer: W [out][in] row-major then b [out]. */
lbmp_status sg_set_params(lbmp_sg* h, const float* params);
lbmp_status sg_get_params(lbmp_sg* h, float* params);
/* Input z-scoring (x - mean)/std per feature, target (y - y_mean)/y_std. */
lbmp_status sg_set_normalization(lbmp_sg* h, const float* x_mean, const float* x_std, float y_mean,
                                 float y_std);
/* One Adam step on rows idx_dev[0..B-1] of (x_dev, y_dev) (idx_dev NULL: the
 * first B rows); B a multiple of 32 up to batch_max. Asynchronous unless
 * loss_host is given (then the batch loss, in normalised units, is returned). */
lbmp_status sg_train_step(lbmp_sg* h, const float* x_dev, const float* y_dev, const int32_t* idx_dev,
                          int B, float lr, float* loss_host);
/* Loss and parameter gradients (host, packed like the parameters) on the
 * first B rows, without updating. Synchronous. */
lbmp_status sg_gradients(lbmp_sg* h, const float* x_dev, const float* y_dev, int B, float* grads_host,
                         float* loss_host);
/* Predictions y_dev[i] = network(x_dev[i]) in target units, i < n. Asynchronous. */
lbmp_status sg_predict(lbmp_sg* h, const float* x_dev, int64_t n, float* y_dev);
/* Waits for the handle's stream. */
lbmp_status sg_sync(lbmp_sg* h);
void sg_free(lbmp_sg* h);

#ifdef __cplusplus
}
#endif
#endif /* LBMP_H */
