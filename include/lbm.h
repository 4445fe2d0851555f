/*
 * lbm.h - C ABI of the MI355X chemical-potential lattice Boltzmann library.
 *
 * Method: Wen, Zhou, He, Zhang, Fang, "Chemical-potential-based lattice
 * Boltzmann method for nonideal fluids" (arXiv:1611.00907).  One time step
 * takes the moments of the D2Q9 distributions (Eq 13 state), the chemical
 * potential mu = psi'(rho) - kappa lap(rho) (Eq 8, bulk terms Eqs 18, 21, 24,
 * 27), the nonideal force F = -rho grad(mu) + c_s^2 grad(rho) (Eq 12 with the
 * ideal-gas tensor of Eq 5), the BGK collision of Eq 13 with the equilibrium
 * of Eq 14 evaluated at u + tau F / rho (forcing paragraph after Eq 14), and
 * streaming with bounce-back at solid rows whose density follows Eq 28 and
 * whose chemical potential is the surface value (Sec. IV) or, for a neutral
 * wall, that of the neighbouring fluid node (Sec. V).
 *
 * Conventions shared by every entry point
 *  - Every call returns lbm_status; nothing is thrown across the ABI.  A NULL
 *    context or required pointer gives LBM_EINVAL.
 *  - Fields are row-major [ny][nx] arrays of double, x fastest, host memory
 *    owned by the caller; solid rows are included.
 *  - Distributions are [9][ny][nx] doubles, direction order
 *    0 (0,0), 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1), 5 (1,1), 6 (-1,1),
 *    7 (-1,-1), 8 (1,-1); they are the post-streaming values f_i(x, t) of
 *    Eq 13, and zero on solid rows.
 *  - Device memory: the caller may pass a workspace of at least
 *    lbm_workspace_bytes() bytes (it keeps ownership and must keep it alive
 *    until lbm_destroy); NULL makes the library allocate and free its own.
 *  - A context belongs to one HIP stream (the one given at init; NULL = the
 *    null stream) and is not thread-safe.  lbm_step is asynchronous except at
 *    monitor points; the getters synchronise the stream.
 *  - x is always periodic.  y is periodic when both bc_bottom and bc_top are
 *    LBM_BC_PERIODIC; otherwise rows 0 and ny-1 are both solid.
 */
#ifndef CPLBM_LBM_H
#define CPLBM_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* bad argument or parameter                               */
    LBM_EDOMAIN = -2,   /* an initial density outside the EOS domain, or non-finite */
    LBM_EDIVERGED = -3, /* monitor found NaN/Inf, rho <= 0 or rho beyond the EOS pole */
    LBM_EHIP = -4,      /* a HIP runtime call failed                               */
    LBM_ENOMEM = -5,    /* workspace too small or device allocation failed         */
    LBM_ESTATE = -6     /* call not valid in the current state                    */
} lbm_status;

/* Equations of state of Sec. III. */
typedef enum {
    LBM_EOS_VDW = 0, /* Eqs 16-18                                  */
    LBM_EOS_CS = 1,  /* Carnahan-Starling, Eqs 25-27                */
    LBM_EOS_PR = 2,  /* Peng-Robinson, Eqs 22-24, Soave-type alpha  */
    LBM_EOS_RKS = 3, /* Redlich-Kwong-Soave, Eqs 19-21              */
    LBM_EOS_RK = 4   /* Redlich-Kwong, alpha = 1/sqrt(T)            */
} lbm_eos;

/* Storage of the distributions; arithmetic is FP64 for LBM_F64, else FP32. */
typedef enum {
    LBM_F64 = 0,
    LBM_F32 = 1,
    LBM_F16DEV = 2,  /* f_i - w_i rho_ref stored as IEEE half, round to nearest even */
    LBM_BF16DEV = 3  /* f_i - w_i rho_ref stored as bfloat16, round to nearest even  */
} lbm_prec;

typedef enum {
    LBM_BC_PERIODIC = 0,
    LBM_BC_CPWALL = 1,  /* solid row: Eq 28 density, surface chemical potential mu_w (Sec. IV) */
    LBM_BC_NEUTRAL = 2  /* solid row: Eq 28 density, mu of the neighbouring fluid node (Sec. V) */
} lbm_bc;

typedef struct {
    int32_t nx, ny;         /* lattice nodes including solid rows; nx >= 1, ny >= 1 (>= 3 walled); */
                            /* ny * round_up(nx, 64) * bytes per stored value < 2^32 (one plane)  */
    int32_t bc_bottom;      /* lbm_bc of row 0                                                   */
    int32_t bc_top;         /* lbm_bc of row ny-1                                                */
    int32_t eos;            /* lbm_eos                                                           */
    int32_t prec;           /* lbm_prec                                                          */
    double a, b, R;         /* EOS constants (Sec. III: a attraction, b volume, R gas constant)  */
    double omega;           /* acentric factor (PR, RKS)                                         */
    double Tr;              /* reduced temperature T / Tc; Tc is solved by the library           */
    double tau;             /* relaxation time of Eq 13, > 1/2                                   */
    double kappa;           /* gradient coefficient of Eq 1, >= 0                                */
    double rho_ref;         /* deviation base of the FP16/BF16 storage (ignored otherwise)       */
    int32_t monitor_every;  /* evaluate mass / residual / divergence every m steps; 0 = never    */
    int32_t scheme;         /* LBM_FORCE_* | LBM_COLLIDE_*; 0 = the paper's method (Eq 12, BGK) */
    double trt_lambda;      /* LBM_COLLIDE_TRT: (tau - 1/2)(tau_minus - 1/2); 0 = 1/4             */
    double mrt_s_e;         /* LBM_COLLIDE_MRT: rate of the energy moment e; 0 = 1                */
    double mrt_s_eps;       /* rate of the energy-square moment epsilon; 0 = 1                   */
    double mrt_s_q;         /* rate of the heat-flux moments; 0 = 8 (2 - 1/tau) / (8 - 1/tau)   */
} lbm_params;

/* Variants of the step that Sec. II names beside the paper's method, selected by
 * lbm_params.scheme (force | collision).  The force: the chemical-potential form
 * F = -rho grad(mu) + c_s^2 grad(rho) of Eq 12 (the paper's), or the divergence of
 * the full pressure tensor, F = -div P + c_s^2 grad(rho) with P from Eq 9 (the
 * form Eq 12 replaces; periodic lattices only, since P carries no surface
 * chemical potential).  The collision: BGK (Eq 13), two relaxation times (the
 * even part of f relaxes at 1/tau, the odd part at 1/tau_minus), or multiple
 * relaxation times on the D2Q9 moments of Lallemand and Luo (rho, e, epsilon,
 * j_x, q_x, j_y, q_y, p_xx, p_xy; the stress moments and j relax at 1/tau).  The
 * force enters every collision through the equilibrium velocity as in the
 * forcing paragraph after Eq 14, each relaxing part shifted by F / (rho s) with
 * its own rate s, so the momentum gains exactly F per step and equal rates give
 * BGK.  Schemes other than 0 need FP64 or FP32 storage, run the 64 x 16 tile
 * shape only, and are not offered for batches (LBM_EINVAL otherwise). */
enum {
    LBM_FORCE_CP = 0,        /* Eq 12, the paper's method                    */
    LBM_FORCE_PTENSOR = 1,   /* Eq 5 with the pressure tensor of Eq 9         */
    LBM_COLLIDE_BGK = 0,
    LBM_COLLIDE_TRT = 16,
    LBM_COLLIDE_MRT = 32
};

/* Bytes of device workspace that lbm_init needs for these parameters (0 if invalid). */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Sets up a lattice: T = Tr * Tc, alpha(T), and f_i = f_i^eq(rho0, u0) of Eq 14.
 * rho0 is required; ux0, uy0 may be NULL (fluid at rest).  Values on solid rows
 * are ignored.  Errors: LBM_EINVAL (parameters), LBM_EDOMAIN (a fluid rho0 that
 * is not finite, <= 0, or at or beyond 1/b (4/b for CS)), LBM_ENOMEM, LBM_EHIP.
 * Wall chemical potentials start at 0. */
lbm_status lbm_init(const lbm_params* p, const double* rho0, const double* ux0,
                    const double* uy0, void* dev_workspace, size_t workspace_bytes,
                    void* hip_stream, lbm_ctx** out);

/* Advances n >= 0 time steps (Eqs 8, 12, 13, 14, 28).  With monitor_every = m > 0
 * the monitors are evaluated on each step whose count is a multiple of m; a
 * non-finite density, rho <= 0 or rho beyond the EOS pole returns LBM_EDIVERGED
 * and the steps that follow it are not run. */
lbm_status lbm_step(lbm_ctx* c, int64_t n);

/* lbm_step bracketed by HIP events recorded on the context's stream (after a
 * stream synchronisation): *ms is the elapsed device time of the n steps,
 * monitors included.  Synchronises. */
lbm_status lbm_step_timed(lbm_ctx* c, int64_t n, double* ms);

/* Launch shapes of the fused step, as a shape code:
 *   8, 16, 32         tiles of 64 columns and that many rows, one per workgroup
 *                     (the default is 16);
 *   12816, 12832, 25608, 25616
 *                     wider tiles, 100 * columns + rows (128 x 16, 128 x 32,
 *                     256 x 8, 256 x 16), 512 threads each;
 *   1000016, 1000032  64 x 16 and 64 x 32 tiles whose ring loads are issued
 *                     together with the tile's own loads (one memory round trip
 *                     instead of two, more registers per thread);
 *   -1 .. -8          column marching: a workgroup owns a strip of at most 252
 *                     columns and marches up a segment of rows, keeping the
 *                     neighbouring rows' densities and chemical potentials on
 *                     chip; -k splits the rows into as many segments as fill k
 *                     workgroups per compute unit.  Offered when one
 *                     distribution buffer (nine planes) stays below 2 GiB.
 * Every shape computes the same step.
 *
 * Shape tuner: times trial_steps fused steps for each shape offered on this
 * lattice without changing the state (every trial maps the current state to the
 * spare buffer), keeps the fastest for this context and returns its code with its
 * time per step in ms.  Synchronises. */
lbm_status lbm_tune(lbm_ctx* c, int32_t trial_steps, int32_t* tile_y, double* best_ms);

/* Sets the shape code directly; LBM_EINVAL for a code not offered on this lattice. */
lbm_status lbm_set_tile(lbm_ctx* c, int32_t tile_y);

/* Output fields of the current state into host arrays [ny][nx]: density (Eq 28
 * values on solid rows), physical velocity v = u + F / (2 rho) (forcing
 * paragraph after Eq 14; 0 on solid rows), and chemical potential (Eq 8; the
 * wall value on solid rows).  Any pointer may be NULL.  Synchronises. */
lbm_status lbm_get_fields(lbm_ctx* c, double* rho, double* vx, double* vy, double* mu);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lbm_get_fields without any
 * allocation.  The fields go through a staging array that the library holds in
 * static device memory (64 MiB on every device it runs on, for the life of the
 * process) instead of a buffer allocated and freed per call; outputs, layout and
 * NULL handling are those of lbm_get_fields, and the values are identical.
 * LBM_EINVAL (with lbm_last_error naming the limit) if nx * ny exceeds
 * LBM_NOALLOC_MAX_NODES.  All calls on one device share the one array: calls that
 * overlap in time on the same device (several host threads, or several streams)
 * race and must be serialised by the caller.  Synchronises. */
#define LBM_NOALLOC_MAX_NODES 2097152
lbm_status lbm_get_fields_noalloc(lbm_ctx* c, double* rho, double* vx, double* vy, double* mu);

/* Surface chemical potential of a CP wall (Sec. IV): wall 0 = bottom, 1 = top;
 * count 1 sets every column, count nx sets one value per column.  Takes effect
 * from the next step.  LBM_EINVAL if the wall is not LBM_BC_CPWALL. */
lbm_status lbm_set_wall_mu(lbm_ctx* c, int32_t wall, const double* mu_w, int32_t count);

/* Last monitor values: total fluid mass, max |rho(t) - rho(t-1)| over fluid nodes,
 * the step they were taken at (-1 if never), and the divergence flags
 * (bit 0 non-finite, bit 1 rho <= 0, bit 2 rho beyond the EOS pole).  Any pointer
 * may be NULL. */
lbm_status lbm_get_monitors(lbm_ctx* c, double* mass, double* residual, int64_t* step,
                            int32_t* flags);

/* Evaluates the monitors now, on the current state and the step before it (runs
 * two steps' worth of work: it advances the lattice by one step). */
lbm_status lbm_monitor_step(lbm_ctx* c);

/* Checkpoint: the distributions f_i(x, t) [9][ny][nx] and the step count. */
lbm_status lbm_get_state(lbm_ctx* c, double* f, int64_t* step);
lbm_status lbm_set_state(lbm_ctx* c, const double* f, int64_t step);

/* Temperature actually used: T = Tr * Tc and alpha(T). */
lbm_status lbm_get_temperature(lbm_ctx* c, double* T, double* alpha);

void lbm_destroy(lbm_ctx* c);
const char* lbm_strerror(lbm_status s);

/* Text of the last HIP failure behind an LBM_EHIP in this thread ("" if none):
 * the failing call and the HIP error name.  Owned by the library. */
const char* lbm_last_error(void);

/* ---- three dimensions: D3Q19 ------------------------------------------- */

/* The same method (Eqs 8, 12, 13, 14) on the D3Q19 velocity set, w = 1/3 (rest),
 * 1/18 (axis), 1/36 (edge), c_s^2 = 1/3, with the isotropic stencils of those
 * weights (lap = 6 sum_i w_i (phi_i - phi_0), grad = 3 sum_i w_i e_i phi_i), on a
 * box periodic in x, y and z.  Sec. II notes that the chemical-potential force
 * avoids storing the pressure tensor, which in 3-D has six components.
 * Direction order (the layout of lbm3d_get_state): 0 rest; 1 +x, 2 -x, 3 +y,
 * 4 -y, 5 +z, 6 -z; 7 (+x+y), 8 (-x-y), 9 (+x-y), 10 (-x+y), 11 (+x+z),
 * 12 (-x-z), 13 (+x-z), 14 (-x+z), 15 (+y+z), 16 (-y-z), 17 (+y-z), 18 (-y+z).
 * Fields are [nz][ny][nx] doubles, x fastest. */
typedef struct lbm3d lbm3d;

/* p gives nx, ny, the EOS, Tr, tau, kappa and the storage (LBM_F64 or LBM_F32);
 * both boundaries must be LBM_BC_PERIODIC and scheme 0; nz >= 1; nx ny nz < 2^31,
 * and one z slice of one direction (ny x nx rounded up to 64, times the storage
 * size) below 4 GiB.
 * The fluid starts at rest, f = f_eq(rho0, 0).  The library allocates the device
 * memory (two 19-plane buffers and one density plane, the latter used by
 * lbm3d_get_fields) and its own stream.
 * Errors: LBM_EINVAL, LBM_EDOMAIN (rho0 outside the EOS domain), LBM_ENOMEM, LBM_EHIP. */
lbm_status lbm3d_init(const lbm_params* p, int32_t nz, const double* rho0, lbm3d** out);
/* n steps; each is one launch that pulls every node once and fuses the density,
 * the chemical potential of Eq 8, the force of Eq 12, the collision and the
 * streaming.  Asynchronous. */
lbm_status lbm3d_step(lbm3d* c, int64_t n);
/* lbm3d_step between HIP events on the box's stream; *ms is the device time. */
lbm_status lbm3d_step_timed(lbm3d* c, int64_t n, double* ms);
/* Density, physical velocity v = u + F / (2 rho) and chemical potential (any
 * pointer may be NULL).  Synchronises. */
lbm_status lbm3d_get_fields(lbm3d* c, double* rho, double* vx, double* vy, double* vz, double* mu);
/* Post-streaming distributions f_i(x, t), [19][nz][ny][nx], and the step count. */
lbm_status lbm3d_get_state(lbm3d* c, double* f, int64_t* step);
void lbm3d_destroy(lbm3d* c);

/* ---- many lattices in one launch ---------------------------------------- */

/* A batch of independent lattices (sizes, EOS, temperature, tau, kappa, walls may
 * differ; the storage precision must be the same) advanced together: each step is
 * one persistent launch over the (case, tile) list of the active cases, and runs
 * of steps are replayed as captured HIP graphs. */
typedef struct lbm_batch lbm_batch;

/* Device bytes for a batch (0 if any case is invalid or precisions differ). */
size_t lbm_batch_workspace_bytes(const lbm_params* cases, int32_t n);

/* rho0[i] is the host [ny][nx] initial density of case i (fluid at rest);
 * mu_w_bottom (may be NULL = 0) gives each case's uniform surface chemical
 * potential of a CP bottom wall.  Workspace and stream conventions as lbm_init.
 * Errors as lbm_init, for the first failing case. */
lbm_status lbm_batch_init(const lbm_params* cases, int32_t n, const double* const* rho0,
                          const double* mu_w_bottom, void* dev_workspace, size_t workspace_bytes,
                          void* hip_stream, lbm_batch** out);

/* n steps of every active case (no convergence checks). */
lbm_status lbm_batch_step(lbm_batch* b, int64_t n);

/* lbm_batch_step bracketed by HIP events on the batch's stream; *ms = device time. */
lbm_status lbm_batch_step_timed(lbm_batch* b, int64_t n, double* ms);

/* Runs until every case has converged or diverged, or max_steps have passed.  Every
 * check_every steps each active case's residual max|rho(t) - rho(t - window)| / window
 * (FP64 over its fluid nodes) is compared with tol: below tol the case converges and
 * stops; a non-finite or out-of-domain density marks it diverged and stops it.  The
 * other cases continue.  1 <= window <= check_every. */
lbm_status lbm_batch_run(lbm_batch* b, int64_t max_steps, int32_t check_every, int32_t window,
                         double tol, int64_t* steps_run);

/* Stops the listed cases for good (the caller's own criterion, e.g. a contact angle
 * that has settled): they keep their state and step count and are masked out of
 * every later step, as converged cases are.  Cases already stopped, converged or
 * diverged are left as they are.  LBM_EINVAL for an index outside [0, n). */
lbm_status lbm_batch_stop(lbm_batch* b, const int32_t* cases, int32_t count);

/* Per-case arrays of n entries (any may be NULL): state 0 active, 1 converged,
 * 2 diverged, 3 stopped by lbm_batch_stop; steps taken; last residual; last mass;
 * last divergence flags. */
lbm_status lbm_batch_status(lbm_batch* b, int32_t* state, int64_t* steps, double* residual,
                            double* mass, int32_t* flags);

/* Output fields / distributions of case i, as lbm_get_fields / lbm_get_state. */
lbm_status lbm_batch_get_fields(lbm_batch* b, int32_t i, double* rho, double* vx, double* vy,
                                double* mu);
lbm_status lbm_batch_get_state(lbm_batch* b, int32_t i, double* f);

/* Tunes the tile shape (as lbm_batch_set_schedule) and the grid of the batched launch on the active cases
 * without changing their state; keeps and returns the fastest.  The grid is k
 * workgroups per compute unit, each walking a contiguous run of the (case, tile)
 * list (*blocks_per_cu = k), or one workgroup per list entry (*blocks_per_cu = -1,
 * resized whenever the list of active cases changes). */
lbm_status lbm_batch_tune(lbm_batch* b, int32_t trial_steps, int32_t* tile_y,
                          int32_t* blocks_per_cu, double* best_ms);

/* Sets the tile shape (64-wide tiles of height 8, 16 or 32, the wide shape codes
 * 12816 and 25608: 128 x 16 and 256 x 8 tiles, or 1: a shape per size class, 64 x 32
 * tiles for cases narrower than 256 columns and 256 x 8 for the others, in the same
 * launch) and the grid of the batched launch directly:
 * blocks_per_cu = k > 0 workgroups per compute unit, 0 as many as fit, -1 one
 * workgroup per (case, tile) entry (the schedule of a new batch, with tile height
 * 16).  LBM_EINVAL for other values.  Every schedule computes the same step. */
lbm_status lbm_batch_set_schedule(lbm_batch* b, int32_t tile_y, int32_t blocks_per_cu);

/* Fluid nodes of all cases (active_only != 0: of the active ones); -1 for NULL. */
int64_t lbm_batch_fluid_nodes(lbm_batch* b, int32_t active_only);

void lbm_batch_destroy(lbm_batch* b);

/* ---- learned warm start: convolutional surrogate ------------------------ */

/* An encoder-decoder of 3x3 convolutions (4 levels of 32, 64, 96, 128 channels,
 * two ReLU convolutions per level, 2x2 average pooling down, nearest-neighbour
 * upsampling and skip concatenation up, one final 3x3 convolution to one
 * channel) mapping 4 input channels (solid mask, initial density, T/Tc, wall
 * chemical potential; the caller chooses their scaling) to one output channel
 * (the equilibrium density, same scaling).  Weights and activations are BF16,
 * products accumulate in FP32 on the matrix cores; the master weights, their
 * gradients and the Adam moments are FP32.  Not part of the paper's method: a
 * warm start for it (the lattice Boltzmann solver still relaxes the prediction).
 *
 * Parameter exchange layout (FP32, sur_param_count values): for each layer in the
 * order e0a e0b e1a e1b e2a e2b e3a e3b d2a d2b d1a d1b d0a d0b out, the weights
 * w[co][ci][3][3] then the bias b[co]; the first layer takes ci = 16 input
 * channels (inputs 4..15 are zero), the last gives co = 1.  Images are FP32
 * NCHW: inputs [n][4][size][size], outputs and targets [n][size][size]. */
typedef struct sur_net sur_net;

/* size: image side, a multiple of 8; max_batch: images per device pass.
 * Allocates all device buffers; parameters start at zero (set them). */
lbm_status sur_create(int32_t size, int32_t max_batch, sur_net** out);
int64_t sur_param_count(const sur_net* n);
/* Sets the FP32 master parameters (exchange layout), resets Adam. */
lbm_status sur_set_params(sur_net* n, const float* params);
lbm_status sur_get_params(sur_net* n, float* params);
/* Prediction for count images (host buffers), in passes of max_batch. */
lbm_status sur_forward(sur_net* n, const float* inputs, int32_t count, float* outputs);
/* Mean-squared-error loss of count <= max_batch images against targets and the
 * gradient of every parameter (exchange layout; grads may be NULL). */
lbm_status sur_gradients(sur_net* n, const float* inputs, const float* targets, int32_t count,
                         float* grads, double* loss);
/* Copies a training set to the device (replacing any previous one). */
lbm_status sur_set_dataset(sur_net* n, const float* inputs, const float* targets, int32_t count);
/* steps Adam updates (lr; beta 0.9, 0.999; eps 1e-8) on minibatches of `batch`
 * images drawn with replacement from the dataset by SplitMix64 from seed; losses
 * (may be NULL) receives the loss of each step. */
lbm_status sur_train(sur_net* n, int32_t steps, int32_t batch, float lr, uint64_t seed, float* losses);

/* Inspection of the last pass, for checking each kernel on the exact operands it
 * used.  sur_trace(n, 1) allocates per-layer copies (about 150 MB at 256^2 and
 * batch 4) and makes every later backward pass keep each layer's output gradient
 * dz (as its weight gradient read it) and the gradients of the three pooled
 * branches; sur_trace(n, 0) frees them.  Tracing does not change any result. */
lbm_status sur_trace(sur_net* n, int32_t on);

/* Copies an internal tensor of the last forward (and, for the gradients, backward)
 * pass into out as FP32, NHWC [N][H][W][C] with C the channels of its buffer, and
 * its shape into shape[4] (out may be NULL to ask for the shape only; capacity is
 * out's length in floats).  BF16 tensors are converted exactly.  Names:
 *   forward: x0 (packed input, 16 ch), e0a, c0 ([up(d1) 64 | e0b 32]), p0, e1a,
 *     c1 ([up(d2) 96 | e1b 64]), p1, e2a, c2 ([up(e3) 128 | e2b 96]), p2, e3a, e3,
 *     d2a, d2, d1a, d1, d0a, d0 (BF16), y (FP32 prediction);
 *   backward: dc0, dc1, dc2 (FP32 gradients of the concatenations; the convolution
 *     that computes one sums its upsampled share over 2 x 2 blocks into the upsampling
 *     gradient at once and stores only the skip share, channels L..L+S-1 of a
 *     concatenation of L upsampled and S skip channels), and with tracing
 *     dz_<layer> for every layer (BF16; dz_out has 16 channels, channel 0 used) and
 *     dp_e3a, dp_e2a, dp_e1a (FP32 input gradients of the first convolution of
 *     levels 3, 2, 1).
 * LBM_EINVAL for an unknown name or a short buffer, LBM_ESTATE before any pass, for
 * a gradient before a backward pass, or for a traced tensor with tracing off. */
lbm_status sur_read(sur_net* n, const char* name, float* out, int64_t capacity, int64_t* shape);
void sur_destroy(sur_net* n);

/* ---- measurement -------------------------------------------------------- */

/* Bandwidth of a plain device-to-device copy of `bytes` (a multiple of 16)
 * repeated iters times: (read + written bytes) / time in GB/s, timed with HIP
 * events on a private stream.  Allocates and frees two device buffers. */
lbm_status lbm_copy_bandwidth(size_t bytes, int32_t iters, double* gbps);

/* ---- host thermodynamics tools (FP64) ---------------------------------- */

/* Critical point of an EOS (Sec. III reduced variables): dp0/drho = d2p0/drho2 = 0.
 * For PR and RKS alpha(Tc) = 1; for RK alpha = 1/sqrt(T). */
lbm_status lbm_critical_point(int32_t eos, double a, double b, double R, double* Tc,
                              double* rho_c, double* p_c);

/* Maxwell equal-area coexistence of the fluid in p (Sec. III, Fig. 1):
 * mu_b(rho_g) = mu_b(rho_l) and p0(rho_g) = p0(rho_l).  LBM_EDOMAIN if Tr >= 1. */
lbm_status lbm_coexistence(const lbm_params* p, double* rho_g, double* rho_l, double* p_sat,
                           double* mu_sat);

/* Spinodal densities of the fluid in p: dp0/drho < 0 for lo < rho < hi (the
 * unstable branch of Sec. III's p0).  lo = hi = 0 at or above Tc.  The FP16 and
 * BF16 deviation storage types evaluate psi'(rho) in FP64 inside this band and in
 * FP32 elsewhere. */
lbm_status lbm_spinodal(const lbm_params* p, double* lo, double* hi);

/* Bulk chemical potential psi'(rho) and pressure p0(rho) of the fluid in p at n
 * densities (host, FP64). */
lbm_status lbm_eos_eval(const lbm_params* p, int64_t n, const double* rho, double* mu_b,
                        double* p0);

/* Contact angle of a sessile drop (Sec. V): R = (4H^2 + L^2)/(8H),
 * tan(theta) = L / (2 (R - H)), evaluated as atan2 so that theta > 90 deg works.
 * rho is [ny][nx]; the interface is the rho_mid isoline; L is the liquid width on
 * base_row (edges linearly interpolated), H the height of the top crossing on the
 * column nearest the drop's centre of excess mass, measured from surface_y.
 * theta = 180 when the drop does not wet base_row.  Outputs may be NULL. */
lbm_status lbm_contact_angle(const double* rho, int32_t nx, int32_t ny, int32_t base_row,
                             double surface_y, double rho_mid, double* theta_deg, double* L,
                             double* H);

/* ---------------------------------------------------------------- warm-start host helpers
 * Host-only (no GPU work, callable from several threads at once) pieces of the
 * learned warm start: the warm field is a circular cap whose angle and bulk levels
 * are read off the network's predicted phase.  The paper defines none of these; the
 * cap's geometry is that of the contact-angle measurement of Sec. V. */

/* out[y][x] (host, nx * ny doubles) = (rho_in + rho_out)/2 - (rho_in - rho_out)/2 *
 * tanh(2 (r - radius) / width), r the distance of node (x, y) from (cx, cy).
 * LBM_EINVAL for empty sizes, a null pointer, width <= 0 or non-finite values. */
lbm_status lbm_warm_cap(int32_t nx, int32_t ny, double rho_in, double rho_out, double radius, double cx,
                        double cy, double width, double* out);

/* Logarithmic phase out[i] = ln(rho[i] / rho_g) / ln(rho_l / rho_g) (rho floored at 1e-300),
 * and its inverse rho[i] = rho_g exp(phi[i] ln(rho_l / rho_g)); n host values each.
 * LBM_EINVAL unless 0 < rho_g < rho_l. */
lbm_status lbm_warm_phase(int64_t n, const double* rho, double rho_g, double rho_l, float* out);
lbm_status lbm_warm_density(int64_t n, const float* phi, double rho_g, double rho_l, double* out);

/* One pass of the D2Q9-weighted average (4/9 centre, 1/9 axes, 1/36 diagonals) of the
 * predicted phase clipped to [lo, hi]; x periodic, rows clamped at the edges; host
 * [ny][nx] floats in and out (not aliased). */
lbm_status lbm_warm_smooth(int32_t nx, int32_t ny, const float* pred, float lo, float hi, float* out);

/* Liquid and vapour levels of a phase field: the medians of the nodes whose whole
 * 5 x 5 neighbourhood (periodic in x and y) lies above / below 1/2; 1 and 0 when no
 * node qualifies. */
lbm_status lbm_warm_bulk_phases(int32_t nx, int32_t ny, const float* phi, double* ph_l, double* ph_g);

#ifdef __cplusplus
}
#endif

#endif /* CPLBM_LBM_H */
