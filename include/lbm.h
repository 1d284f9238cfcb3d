/*
 * lbm.h -- C ABI of the MI355X lattice Boltzmann collide-and-stream library.
 *
 * The library advances a lattice Boltzmann fluid on one AMD Instinct MI355X
 * (gfx950).  It implements the accelerated-lattice hot path of Latt &
 * Coreixas, "Multi-GPU Acceleration of PALABOS Fluid Solver using C++
 * Standard Parallelism" (arXiv 2506.09242):
 *   - structure-of-arrays populations (Sec. 2.3, "Structure-of-array memory
 *     layout"), updated by a fused collision + streaming kernel that is
 *     thread-safe in place (the AA pattern, which Sec. 2.3 names as the
 *     single-array alternative to the two-population scheme);
 *   - per-node integer tags selecting the collision model (Sec. 2.3,
 *     "Collision-model polymorphism without virtual function calls") and a
 *     kernel specialised on the subset of models actually present
 *     (Sec. 2.3, "GPU kernel size reduction");
 *   - BGK and TRT collisions, the Smagorinsky subgrid closure, regularized
 *     BGK, standard and moving-wall half-way bounce-back (Sec. 3
 *     introduction; Sec. 3.2, 3.3), regularized velocity / pressure open
 *     boundaries on the x planes (Sec. 3.3);
 *   - populations stored with the constant offset w_i rho0 removed
 *     (Sec. 3 introduction, after Skordos), in FP64, FP32 or FP16 storage;
 *   - fused FP64 domain reductions of mass, momentum and kinetic energy
 *     (Sec. 2.2 "Reductions"; kinetic energy of Eq. (5));
 *   - a learned eddy-viscosity closure (7->32->32->1 MLP, BF16 matrix cores)
 *     fused into the collision, with its training kernels.
 *
 * Conventions common to every entry point
 *   - Every call returns lbm_status: 0 on success, a negative code on error.
 *     The text of the last error of the calling thread is lbm_last_error().
 *   - Lattice cells are indexed n = (z*ny + y)*nx + x (x fastest).  Every
 *     axis is periodic; walls are explicit non-fluid tags and open
 *     boundaries explicit boundary tags on the x planes.
 *   - Velocities use the canonical order documented at lbm_velocity().
 *   - Pointers named *_host are host memory, borrowed for the duration of the
 *     call only.  Pointers named *_dev are device memory on the lattice's
 *     GPU, borrowed for the call (the call is stream-ordered on the lattice's
 *     stream unless stated otherwise).
 *   - Calls on one lattice handle are not thread-safe.  Kernel launches are
 *     asynchronous on the handle's HIP stream unless the entry point says it
 *     synchronizes.
 *   - After any HIP runtime error the handle becomes failed: every later call
 *     on it returns LBM_ESTATE (lbm_destroy still releases it).
 *   - "The state at time t" means the pre-collision (post-streaming)
 *     populations after t steps, whatever the in-place layout parity.  Every
 *     read, reduction and checkpoint presents that natural state.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,       /* invalid argument (message says which)            */
    LBM_ENOMEM = -2,       /* device or host allocation failed                  */
    LBM_EHIP = -3,         /* HIP runtime error (handle becomes failed)         */
    LBM_EUNSTABLE = -4,    /* a reduction found non-finite density or velocity  */
    LBM_EUNSUPPORTED = -5, /* combination not built                             */
    LBM_ESTATE = -6        /* handle failed earlier, or call out of order       */
} lbm_status;

/* Velocity sets: D3Q19 (all runs of the paper, Sec. 3) and D3Q27. */
typedef enum { LBM_D3Q19 = 19, LBM_D3Q27 = 27 } lbm_q;

/* Population storage precision.  All three store h_i = f_i - w_i rho0.
 * F64: FP64 storage and arithmetic.  F32: FP32 storage and arithmetic.
 * F16S: FP16 storage (round to nearest even), FP32 arithmetic.
 * Initial equilibria and domain reductions are FP64 in every case. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2 } lbm_prec;

/* Node tags (one byte per node).  Fluid tags select the collision model;
 * non-fluid tags carry no populations and act as half-way bounce-back walls.
 * Any other value is rejected by lbm_create. */
enum {
    LBM_TAG_SOLID = 0,     /* resting wall / empty node                         */
    LBM_TAG_BGK = 1,       /* BGK, second-order equilibrium                     */
    LBM_TAG_TRT = 2,       /* two-relaxation-time, magic parameter trt_lambda   */
    LBM_TAG_BGK_SMAG = 3,  /* BGK + Smagorinsky eddy viscosity (implicit tau)  */
    LBM_TAG_BGK_MLP = 4,   /* BGK + learned eddy viscosity, Smagorinsky fallback */
    LBM_TAG_REG = 5,       /* regularized BGK: the non-equilibrium part is replaced
                              by its second-order Hermite projection before
                              relaxing (the regularized family of the paper's
                              robust RR model, Sec. 3.1-3.2)                  */
    LBM_TAG_VEL_IN = 6,    /* regularized velocity boundary on the x = 0 plane:
                              imposes bc_velocity (Sec. 3.3 open boundaries)  */
    LBM_TAG_PRES_OUT = 7,  /* regularized pressure boundary on the x = nx-1 plane:
                              imposes bc_density[1], zero tangential velocity */
    LBM_TAG_PRES_IN = 8,   /* regularized pressure boundary on the x = 0 plane:
                              imposes bc_density[0], zero tangential velocity */
    LBM_TAG_VEL_OUT = 9,   /* regularized velocity boundary on the x = nx-1 plane:
                              imposes bc_velocity                             */
    LBM_TAG_RR = 10,       /* recursive regularized: third-order Hermite
                              equilibrium, deviatoric second-order and
                              recursive third-order non-equilibrium, bulk
                              relaxation 1 (the paper's robust RR model,
                              Sec. 3.1-3.2)                                   */
    LBM_TAG_WALL0 = 16     /* 16..31: moving wall, velocity wall_velocity[tag-16] */
};
/* Open boundaries (tags 6..9; the regularized conditions of Latt et al. 2008
 * the paper uses for the Berea runs, Sec. 3.3, with pressure or velocity
 * imposed at either end).  The lattice stays periodic in x; on the x = 0
 * plane the populations with c_x = +1 (on x = nx-1 those with c_x = -1) are
 * rebuilt each step from the imposed velocity (density from mass and
 * x-momentum balance over the known populations) or the imposed density
 * (x velocity likewise, y and z velocity zero), each as equilibrium plus its
 * opposite population's non-equilibrium part; the node is then regularized
 * (second-order Hermite projection) and relaxed with tau.  The body force is
 * not applied on these nodes.  Reads and reductions report their stored
 * populations, whose entering ones are those streamed across the periodic x
 * wrap. */

typedef struct {
    int32_t nx, ny, nz;    /* lattice size, each >= 1, nx*ny*nz < 2^31          */
    int32_t q;             /* lbm_q                                              */
    int32_t prec;          /* lbm_prec                                           */
    int32_t flags;         /* 0, or LBM_FLAG_* bits below                        */
    double rho0;           /* reference density (offset and wall density), > 0  */
    double tau;            /* relaxation time, tau = 3 nu + 1/2, must be > 1/2  */
    double trt_lambda;     /* TRT magic parameter (3/16 for exact walls), > 0   */
    double smag_cs;        /* Smagorinsky constant, >= 0                         */
    double force[3];       /* uniform body-force density (Guo), |F| < 0.3       */
    double wall_velocity[16][3]; /* velocity of wall tags 16..31, |u| < 0.3     */
    double bc_velocity[3]; /* velocity of velocity-boundary nodes (6, 9), |u| < 0.3 */
    double bc_density[2];  /* density of pressure-boundary nodes (> 0): [0] on
                              x = 0 (tag 8), [1] on x = nx-1 (tag 7)          */
} lbm_config;

/* lbm_config.flags: collision switched off on every fluid node (the
 * post-collision populations equal the pre-collision ones), so a step is pure
 * streaming with the same bounce-back and moving-wall terms.  For checking
 * the streaming maps and for timing the memory access pattern of the step
 * without its arithmetic; not a physical model. */
#define LBM_FLAG_FREE_STREAM 1

/* Storage order of the nodes (tags, neighbour masks and the 4096-node blocks
 * of the population array; the Structure-of-Array layout of Sec. 2.3 is kept
 * inside each block).  Row layout: the natural order (z ny + y) nx + x.
 * Brick layout: 16^3-node blocks of 4^3-node bricks, each brick x fastest, so
 * that the 64-byte storage sectors a step reads and writes are 4 x 4 x 1 (FP32)
 * patches rather than 16-node row segments: in a porous medium (Sec. 3.3)
 * far fewer of them are mostly solid.  Default: the brick layout for tagged
 * lattices with fewer than half of their nodes fluid and every side a multiple
 * of 16, else the row layout (the variant name ends in "/bricks" for the
 * brick layout).  LBM_FLAG_LAYOUT_BRICKS requests the brick layout (EINVAL
 * unless every side is a multiple of 16); LBM_FLAG_LAYOUT_ROWS the row layout.
 * Results do not depend on the layout (populations bitwise; reductions up to
 * summation order); it is invisible through the API. */
#define LBM_FLAG_LAYOUT_BRICKS 2
#define LBM_FLAG_LAYOUT_ROWS 4

/* FP64 domain reductions of the natural state at time `step`, over fluid nodes. */
typedef struct {
    int64_t step;              /* time t of the sampled state                     */
    int64_t n_fluid;           /* number of fluid nodes                           */
    int64_t n_nonfinite;       /* nodes whose rho or u is not finite (skipped)    */
    double mass;               /* n_fluid*rho0 + mass_delta                       */
    double mass_delta;         /* sum (rho - rho0)                                */
    double momentum[3];        /* sum rho u = sum (sum_i c_i f_i + F/2)           */
    double velocity_sum[3];    /* sum u (permeability: mean over all nodes)       */
    double kinetic_energy;     /* (1/n_fluid) sum |u|^2/2   (Eq. 5)               */
    double kinetic_energy_rho; /* sum rho |u|^2 / 2                               */
} lbm_moments;

typedef struct lbm_lattice lbm_lattice;

/* ---------------------------------------------------------------- lattice */

/* Bytes of device memory one lattice's population array needs for cfg:
 * Q populations of every node in the storage precision, nodes rounded up to
 * whole blocks of 4096 (the array is blocked by node index: each block of
 * 4096 consecutive nodes stores its Q slots one after another).  The
 * in-place AA scheme needs one array (Sec. 2.3 notes it halves the
 * two-population footprint).  Returns 0 if cfg is invalid. */
size_t lbm_population_bytes(const lbm_config *cfg);

/* Create a lattice on the current HIP device (Sec. 2.1: one large block per
 * GPU).  tags_host: nx*ny*nz bytes, x fastest; validated (known values, at
 * least one fluid node).  The tag histogram selects the smallest compiled
 * kernel variant covering the models present (Sec. 2.3, kernel-size
 * reduction).  hip_stream: hipStream_t to launch on, NULL = null stream.
 * The library allocates and owns the population array.  Populations are
 * undefined until lbm_init_equilibrium or lbm_write_populations.  Besides
 * the populations the handle owns nx*ny*nz bytes of tags, 4*nx*ny*nz bytes
 * of per-node neighbour masks when the lattice has non-fluid nodes or more
 * than one fluid model, and a few per-tile words.  The slots of non-fluid
 * nodes hold unspecified values: a step may overwrite them.
 * Errors: EINVAL (config or tags), ENOMEM, EHIP. */
lbm_status lbm_create(const lbm_config *cfg, const uint8_t *tags_host, void *hip_stream,
                      lbm_lattice **out);

/* As lbm_create, but the population array is caller-owned device memory
 * (e.g. a torch tensor) of at least lbm_population_bytes(cfg) bytes, 256-byte
 * aligned.  It must outlive the handle. */
lbm_status lbm_create_on_buffer(const lbm_config *cfg, const uint8_t *tags_host, void *pops_dev,
                                size_t pops_bytes, void *hip_stream, lbm_lattice **out);

/* Release device memory the handle owns.  Safe on NULL and failed handles. */
void lbm_destroy(lbm_lattice *lat);

/* Override the launch geometry: 256-thread blocks updating tiles of tx x ty
 * nodes of one z-plane, one node per thread (tx in {32,64,128,256},
 * tx*ty == 256).  Populations are bitwise independent of the choice (the FP64
 * reductions sum per-tile partials, so their rounding follows the tile
 * shape); this exists for tuning and for that test.  The shape also decides whether a lattice
 * whose nx is a power of two in [64, 4096] uses row-form addressing (tx >= 64;
 * FP16 storage, or a tagged lattice with at least half of its nodes fluid; the
 * variant name then ends in "/rows").  By default an FP16 lattice of one fluid
 * model without walls whose nx is a power of two in [128, 4096] runs its even
 * steps with two nodes per thread (variant "/pairs"; the same node update, so
 * the populations agree with the one-node kernels up to where the compiler
 * fuses a multiply-add differently, one FP16 rounding at most); an explicit
 * shape selects the one-node kernels for every step.  EINVAL for other shapes. */
lbm_status lbm_set_launch(lbm_lattice *lat, int tx, int ty);  /* EUNSUPPORTED on brick-layout lattices */

/* ---------------------------------------------------------- initial state */

/* Set every fluid node to the second-order equilibrium of (rho, u), computed
 * in FP64 and stored as h_i = f_i^eq - w_i rho0 rounded to the storage type
 * (Sec. 3 intro: offset stripping).  rho_host: nx*ny*nz doubles or NULL
 * (rho0 everywhere).  u_host: 3 planes of nx*ny*nz doubles (ux, uy, uz) or
 * NULL (rest).  Resets the time counter to 0.  Synchronizes. */
lbm_status lbm_init_equilibrium(lbm_lattice *lat, const double *rho_host, const double *u_host);

/* ------------------------------------------------------------ time steps */

/* Advance n_steps >= 0 fused collide-and-stream steps (Sec. 2.3 push-pull
 * node update; the paper's collideAndStream()).  Asynchronous. */
lbm_status lbm_step(lbm_lattice *lat, int64_t n_steps);

/* Advance n_steps and sample the domain reductions of the states at times
 * t0 + k*every for k = 0 .. n_steps/every (t0 = time at entry).  Samples
 * before the last step are fused into the step kernels (no extra traffic,
 * Sec. 2.2 "Reductions"); a sample at t0 + n_steps uses a reduction pass.
 * series: n_series >= n_steps/every + 1 entries (host).  Synchronizes.
 * Returns EUNSTABLE if any sample saw non-finite values (series still filled). */
lbm_status lbm_step_reduce(lbm_lattice *lat, int64_t n_steps, int64_t every, lbm_moments *series,
                           int64_t n_series);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * steps, reductions and results as lbm_step_reduce (bitwise, same kernels),
 * with the reduction scratch -- per-tile partials, the finalize stage and the
 * sample series -- in one fixed array per GPU that the library holds until the
 * process ends (NRED = 10 doubles per tile, per finalize block and per sample:
 * about 48 MB).  Makes no hipMalloc, hipFree or other allocating call; the
 * first call on a device resolves that array's address there.  Limits:
 * n_steps/every + 1 <= LBM_NOALLOC_MAX_SAMPLES samples and at most
 * LBM_NOALLOC_MAX_TILES tiles of 256 nodes in the lattice's current tiling
 * (any lattice up to about 1.5e8 nodes, e.g. 512^3); EINVAL beyond either,
 * with the numbers in lbm_last_error().  Every call on one GPU shares that
 * GPU's array (nothing in it needs clearing: each call writes what it
 * reads), so calls that overlap in time on one GPU -- from two threads, or on
 * two streams -- race and must be serialised by the caller.  Synchronizes. */
#define LBM_NOALLOC_MAX_TILES 589824
#define LBM_NOALLOC_MAX_SAMPLES 4096
lbm_status lbm_step_reduce_noalloc(lbm_lattice *lat, int64_t n_steps, int64_t every, lbm_moments *series,
                                   int64_t n_series);

/* Reductions of the current state (a standalone pass): the domain sums of
 * Sec. 2.2 ("Reductions", the transform_reduce of every node's moments) with
 * the kinetic energy of Eq. (5); fields as in lbm_moments, FP64 per node,
 * summed in a fixed order (run-to-run deterministic for a fixed launch
 * shape).  out: host, one lbm_moments.  Synchronizes.  EINVAL for a null
 * out; EUNSTABLE if non-finite values were found (out still filled). */
lbm_status lbm_reduce(lbm_lattice *lat, lbm_moments *out);

/* Volume-averaged enstrophy of the natural state (Eq. 5, second part):
 * (1/N) sum over nodes of |w|^2 / 2, w = curl u, each derivative by the
 * eighth-order centred difference (coefficients 4/5, -1/5, 4/105, -1/280 at
 * distances 1..4) on the periodic lattice, u from lbm_read_fields' definition.
 * Needs an all-fluid lattice with every axis >= 9 nodes (EUNSUPPORTED
 * otherwise; the stencil is undefined across walls).  Uses a temporary device
 * buffer of 4 doubles per node.  Synchronizes. */
lbm_status lbm_enstrophy(lbm_lattice *lat, double *out);

/* Wait for all work queued on the handle's stream. */
lbm_status lbm_synchronize(lbm_lattice *lat);

/* Current time t (steps since init or since the last write). */
int64_t lbm_time(const lbm_lattice *lat);

/* ------------------------------------------------------------- readback */

/* Readback and checkpoint calls.  They play the part of the paper's bridge
 * between the GPU container and the host (Sec. 2.1: data copied between the
 * two containers at run time, on a per-need basis, for pre- and
 * post-processing; Sec. 2.3, Fig. 4: hybrid execution) and of its
 * serialized checkpoints (Sec. 2.3).  Each one gathers or scatters on the
 * device in chunks of whole z-planes (at most ~256 MB of FP64 staging) and
 * copies through host memory the caller owns. */

/* Density and velocity of the natural state at the current time, FP64:
 * rho_host nx*ny*nz, u_host 3*nx*ny*nz (planes ux, uy, uz), each nullable.
 * u = (sum c_i f_i + F/2)/rho.  Non-fluid nodes read 0.  Synchronizes.
 * ENOMEM if the host staging copy cannot be allocated. */
lbm_status lbm_read_fields(lbm_lattice *lat, double *rho_host, double *u_host);

/* All populations f_i (offset added back, FP64, canonical order, natural
 * state): f_host has q*nx*ny*nz doubles, plane i at i*nx*ny*nz.  Non-fluid
 * nodes read 0.  Synchronizes. */
lbm_status lbm_read_populations(lbm_lattice *lat, double *f_host);

/* Populations of n selected nodes: cells_host[n] node indices, f_host[n*q]
 * (node-major).  For spot checks of large lattices.  Synchronizes. */
lbm_status lbm_read_cells(lbm_lattice *lat, const int64_t *cells_host, int64_t n, double *f_host);

/* Overwrite the state with f_host (layout as lbm_read_populations; fluid
 * nodes only) and set the time counter to t.  Checkpoint restore.
 * Synchronizes. */
lbm_status lbm_write_populations(lbm_lattice *lat, const double *f_host, int64_t t);

/* Checkpoint: the stored populations h_i = f_i - w_i rho0 of the natural
 * state, widened exactly to FP64 (layout as lbm_read_populations; non-fluid
 * nodes read 0).  Writing back what was read with lbm_write_state restores
 * the lattice bit for bit in every storage precision (an unshifted round trip
 * through lbm_read_populations is exact only for FP32/FP16 storage).
 * Synchronizes. */
lbm_status lbm_read_state(lbm_lattice *lat, double *h_host);

/* Restore a state read by lbm_read_state and set the time counter to t.
 * Values are rounded to the storage precision (exact for values that came
 * from the same precision).  Synchronizes. */
lbm_status lbm_write_state(lbm_lattice *lat, const double *h_host, int64_t t);

/* --------------------------------------------------------- learned closure */

/* Number of floats in a packed closure parameter vector. */
#define LBM_MLP_NPARAMS 1359

/* Upload the closure network used by LBM_TAG_BGK_MLP nodes.  params_host:
 * LBM_MLP_NPARAMS floats, packed W1[32][7], b1[32], W2[32][32], b2[32],
 * W3[32], b3, mean[7], std[7].  Weights are rounded to BF16 on upload; biases
 * and normalisation stay FP32.  Inputs: the non-equilibrium momentum flux
 * Pi_xx, Pi_yy, Pi_zz, Pi_xy, Pi_xz, Pi_yz and rho, z-scored in FP32
 * ((x - mean) times the FP32 reciprocal of std).  Output:
 * nu_t = nu0 * softplus(W3 h2 + b3), nu0 = (tau - 1/2)/3; tau_eff =
 * 3 (nu0 + nu_t) + 1/2.  Non-finite nu_t or nu_t > 10 nu0 falls back to the
 * Smagorinsky tau_eff.  Until called, MLP nodes use the Smagorinsky value. */
lbm_status lbm_set_mlp(lbm_lattice *lat, const float *params_host, size_t n);

/* Run the fused closure network alone on n feature rows: feat_dev n*7 FP32
 * (raw, un-normalised), nut_dev n FP32 out (nu_t, before the fallback rule).
 * Same device code as the fused collision.  Stream: hip_stream.  Asynchronous. */
lbm_status lbm_mlp_infer(const float *params_host, double nu0, const float *feat_dev, int64_t n,
                         float *nut_dev, void *hip_stream);

/* Box-filter a fine lattice by factor^3 blocks (fine sizes divisible by
 * factor) and write per coarse node the 7 closure features (FP32, raw) to
 * feat_dev[ncoarse*7] and the eddy-viscosity target divided by nu_c to
 * target_dev[ncoarse], where nu_c = nu_fine / factor (convective scaling:
 * dx and dt both grow by factor).  Favre-filtered velocity U = <rho u>/<rho>,
 * SGS stress T_ij = <rho u_i u_j>/<rho> - U_i U_j, coarse strain S by
 * second-order central differences (periodic), target
 * nu_t = max(0, -dev(T):S / (2 S:S + 1e-30)), features
 * Pi = -(2/3) <rho> tau_e S with tau_e = 3 (nu_c + nu_t) + 1/2, and <rho>.
 * Coarse node order is (Z*ny/f + Y)*nx/f + X.  Synchronizes. */
lbm_status lbm_filter_snapshot(lbm_lattice *fine, int factor, float *feat_dev, float *target_dev);

/* Mean-squared-error gradient of the closure network over n samples:
 * loss = (1/n) sum (softplus(net(x)) - y)^2 with x z-scored by the packed
 * mean/std, FP32 arithmetic throughout.  params_dev/grad_dev: LBM_MLP_NPARAMS
 * floats (grad of mean/std entries is 0).  loss_dev: 1 float.  Asynchronous. */
lbm_status lbm_mlp_grad(const float *params_dev, const float *feat_dev, const float *target_dev,
                        int64_t n, float *grad_dev, float *loss_dev, void *hip_stream);

/* Train the closure network with Adam (beta1 0.9, beta2 0.999, eps 1e-8):
 * for each epoch, visit the samples in the order perm_dev[epoch*n + k]
 * (the caller's seeded shuffle), in mini-batches of `batch`, one Adam step
 * per batch.  params_dev is updated in place (FP32 master weights);
 * loss_log_dev[epochs] receives each epoch's mean batch loss.  Asynchronous. */
lbm_status lbm_mlp_train(float *params_dev, const float *feat_dev, const float *target_dev, int64_t n,
                         const int64_t *perm_dev, int batch, int epochs, double lr,
                         float *loss_log_dev, void *hip_stream);

/* ------------------------------------------------ slab faces (Sec. 2.2, 2.3) */

/* Populations of one node that cross a z face of a slab: 5 (D3Q19) or 9
 * (D3Q27), the directions with c_z = +1 (face 0) or c_z = -1 (face 1) in
 * canonical order.  Returns 0 for a bad q. */
int lbm_face_populations(int q);

/* Pack (unpack) the slots that cross a z face: the paper packs the data
 * exchanged between blocks on the device before the GPU-to-GPU transfer and
 * unpacks it there after (Sec. 2.2 "Prefix Sums"; Sec. 2.3 "GPU-GPU
 * communication using pinned memory and MPI").
 *   face 0: the z = 0 plane, slots of the directions with c_z = +1;
 *   face 1: the z = nz-1 plane, slots of the directions with c_z = -1.
 * buf_dev: device memory of lbm_face_populations(q)*nx*ny elements of the
 * storage type (8, 4 or 2 bytes: the stored bits are copied unchanged),
 * element [j][y][x] = the raw slot of the j-th such direction of node
 * (x, y) of the plane; the caller owns it.  Asynchronous on the lattice's
 * stream.  EINVAL for a bad face or null buffer.
 *
 * Slab decomposition with the in-place AA scheme.  Slabs S_0 .. S_{m-1}
 * stacked along z (each its own lattice of nz_j planes, same nx, ny, every
 * fluid node one model: lbm_create of an all-fluid single-model tag array;
 * masks across slab faces are not built) advance the stacked lattice,
 * periodic in z, exactly: even steps (lbm_time even) need nothing; around
 * each odd step,
 *   before: S_j.face0 <- S_{j+1}.face0 and S_j.face1 <- S_{j-1}.face1,
 *   after : S_{j+1}.face0 <- S_j.face0 and S_{j-1}.face1 <- S_j.face1
 * (indices mod m; pack all, then unpack all).  Each slab's own periodic
 * wrap then lands every crossing access on the neighbour's values. */
lbm_status lbm_face_pack(lbm_lattice *lat, int face, void *buf_dev);
lbm_status lbm_face_unpack(lbm_lattice *lat, int face, const void *buf_dev);

/* -------------------------------------------------------------- utilities */

/* Memory-bandwidth probe (a measured HBM ceiling, not part of the method):
 * kind 0 copies src_dev to dst_dev, kind 1 reads src_dev (one word per
 * 1024 vectors is written to dst_dev only if the sum of what was read equals
 * a fixed constant, which keeps the loads live), kind 2 fills dst_dev; each
 * lane moves lane_bytes (4, 8 or 16) per access, four accesses per lane.
 * dst_dev and src_dev: device buffers of `bytes` bytes (src_dev unused by
 * kind 2), bytes a positive multiple of 4096 * lane_bytes.  Asynchronous on
 * hip_stream.  EINVAL otherwise. */
lbm_status lbm_probe_bandwidth(int kind, void *dst_dev, const void *src_dev, size_t bytes, int lane_bytes,
                               void *hip_stream);


/* Velocity i of the canonical order of lattice q (the lattice descriptor of
 * Sec. 2.1: number of populations and lattice connectivity): returns the opposite index
 * and fills c[3] and the weight w; -1 for a bad (q, i).  Order: rest;
 * +x,+y,+z; (1,1,0),(1,-1,0),(1,0,1),(1,0,-1),(0,1,1),(0,1,-1); for D3Q27
 * (1,1,1),(1,1,-1),(1,-1,1),(1,-1,-1); then the negatives in the same order
 * (opposite of i is i + (q-1)/2 for 1 <= i <= (q-1)/2). */
int lbm_velocity(int q, int i, int c[3], double *w);

/* Text of the calling thread's last error ("" if none). */
const char *lbm_last_error(void);

/* Name of the kernel variant the handle selected: "D3Q<q>/<precision>/<model
 * set>/<uniform|tagged>", plus "/rows" when the step uses row-form addressing
 * (a wave's population rows start at wave-uniform addresses), "/pairs" when
 * FP16 even steps update two nodes per thread (odd steps in row form), or
 * "/bricks" for the brick storage layout.  Owned by the
 * handle; valid until the next lbm_set_launch or lbm_destroy. */
const char *lbm_variant_name(const lbm_lattice *lat);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
