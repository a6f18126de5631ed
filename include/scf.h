/*
 * scf.h -- C ABI of the MI355X (gfx950) binary Shan-Chen capillary-filling library, libscf.so.
 *
 * The library advances the two-component pseudo-potential D2Q9 BGK lattice Boltzmann model of
 * S. Chibbaro, "Capillary filling with pseudo-potential binary Lattice-Boltzmann model"
 * (Sec. 2: eqs. lbe, feq1-feq3, forcing, forcingw; Sec. 3: the reservoir + capillary set-up of
 * Fig. 1) on one GPU, and reports the quantities the paper follows in time: the centre-line
 * interface position z(t), the precursor-film front and the per-component mass.
 *
 * Conventions shared by every call
 *  - Status: every int-returning call returns SCF_OK (0) or a negative SCF_E* code; the text of
 *    the last error of the calling thread is scf_last_error().
 *  - Memory: host arrays passed in are read during the call only and stay owned by the caller.
 *    Device memory is NOT allocated by the library: the caller passes one device workspace
 *    (dev_ws, at least scf_*workspace_bytes() bytes, 256-byte aligned) that must stay alive and
 *    untouched until the matching *_destroy.  The caller also passes the HIP stream (a
 *    hipStream_t cast to void*, NULL = the default stream); all device work is enqueued on it.
 *  - Geometry: a box nx x ny, periodic in x and y.  Rows y = 0 and y = ny-1 are solid for
 *    x in [x0, x1) (the coated capillary, bounce-back walls); elsewhere those rows are fluid
 *    (the reservoir).  Channel height H = ny - 2.  Liquid (component A) is expected to start
 *    at x < x0; observables are reported relative to x0.  An optional solid mask
 *    (scf_geometry.solid) replaces the rows by any set of solid nodes (rough walls, posts).
 *  - Field arrays are row-major (ny rows of nx values, x fastest), FP64 on the host.  The
 *    device state is FP32.
 *  - Threading: one context per stream; distinct contexts are independent.  Calls on one
 *    context must not overlap.
 */
#ifndef SCF_H
#define SCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SCF_OK = 0,
    SCF_EINVAL = -1,     /* bad argument: sizes, tau <= 1/2, NULL pointer, small workspace */
    SCF_ENOMEM = -2,     /* host allocation failed */
    SCF_EDEVICE = -3,    /* a HIP runtime call failed (message names it) */
    SCF_EUNSTABLE = -4,  /* the state holds a non-finite or negative (< -1e-3) density */
    SCF_ESTATE = -5      /* call not valid in the current state (e.g. checkpoint mismatch) */
};

/* Step variants (scf_set_variant). */
enum {
    SCF_VARIANT_FUSED = 0,     /* one kernel per step: pull, densities with an LDS halo, forces,
                                  equilibrium, collision, store (144 B per node update) */
    SCF_VARIANT_TWO_KERNEL = 1 /* density kernel, then pull + collide kernel reading the density
                                  field back (232 B per node update) */
};

typedef struct {
    int32_t nx, ny;    /* box size, nx >= 3, ny >= 3, nx < 2^20, ny < 2^20, and one population
                          buffer (18 planes of ny rows of nx rounded up to 64 FP32 values) at
                          most 4 GiB, about 59.6 M nodes per channel (the fused kernels address a
                          buffer with unsigned 32-bit byte offsets); larger problems are several
                          channels */
    int32_t x0, x1;    /* solid rows y = 0 and y = ny-1 for x in [x0, x1); x0 == x1: no walls */
    const uint8_t* solid;  /* optional host mask, ny*nx bytes row-major, non-zero = solid node.
                              When given it REPLACES the wall rows as the set of solid nodes
                              (bounce-back, psi = 0, and s = 1 in eq. forcingw all follow it);
                              x0, x1 then only place the observables (inlet x0, reservoir centre
                              x0/2).  Read during *_init only (copied); NULL: the wall rows.
                              A masked channel takes one more FP32 plane of workspace. */
} scf_geometry;

typedef struct {
    double G;          /* inter-component coupling of eq. forcing with psi_k = n_k, written with the
                          D2Q9 neighbour weights 1/9 (axis) and 1/36 (diagonal): the paper's
                          g_{AB} = G/9 on axis links and g_{AB}/4 on diagonal links; G > 0 repels */
    double gw[2];      /* wall couplings g_kw rho_w of eq. forcingw (same weights); < 0 attracts */
    double tau[2];     /* relaxation times tau_A, tau_B of eq. lbe, each > 1/2 */
    double alpha[2];   /* rest fractions alpha_k of eqs. feq1-feq3 (4/9: usual D2Q9), in [0, 1) */
    double mass[2];    /* molecular masses m_k, rho_k = m_k n_k (1 on the standard path), > 0 */
} scf_params;

typedef struct {
    int64_t t;            /* time step of the sample */
    double mass[2];       /* sum over fluid nodes of n_A and n_B (FP64 sum of FP32 values) */
    double z;             /* centre-line front: first downward zero crossing of n_A - n_B
                             scanning from x0/2, linearly refined, minus x0; NaN if none */
    double precursor;     /* mean of the two wall-row film fronts; NaN if either is absent */
    double precursor_lo;  /* row y = 1: first crossing of n_A through n_A(x0/2, centre)/3 */
    double precursor_hi;  /* row y = ny-2 */
    int32_t flags;        /* bit0: n_A - n_B < 0 at the reservoir centre (reservoir exhausted);
                             bit1: a non-finite density or one below -1e-3 at a fluid node */
    int32_t reserved;
} scf_obs;

/* Launch schedule of the fused step (see scf_set_tile). */
typedef struct {
    int32_t bx;           /* block width in nodes along x: 64, 128, 256 or 512 */
    int32_t cy;           /* rows per tile, >= 1 (>= ny: whole columns) */
    int32_t order;        /* tile order: SCF_ORDER_STRIPS (all row chunks of a strip, then the next
                             strip) or SCF_ORDER_BANDS (all strips of a row band, then the next
                             band), optionally | SCF_ORDER_XCD (each of the 8 XCDs takes a
                             contiguous eighth of that order instead of every 8th tile).
                             SCF_ORDER_PERSIST (| SCF_ORDER_XCD) instead launches one block per
                             resident slot (CUs x the kernel's occupancy, or blocks_per_cu) and
                             gives each block a contiguous run of the (channel, band, strip) tile
                             list, the runs balanced by rows: each channel's rows are cut into
                             round(ny / target) bands, with the band height `target` (from 16
                             rows up) that minimises the largest run (cy is then not used); with
                             SCF_ORDER_XCD each XCD takes a contiguous eighth of the runs */
    int32_t graph_steps;  /* steps per captured HIP graph, 0 = launch every step directly */
    int32_t fuse;         /* time steps per pass of the fused step: 1, or 2 (temporal blocking:
                             each launch advances two steps, its tiles are bx - 6 columns wide,
                             480 for bx = 512 and 224 for bx = 256 (edges on 128-byte lines), and
                             the intermediate populations stay on chip; an
                             odd remainder of a step count is done by one single step).  Same
                             results bit for bit. */
    int32_t blocks_per_cu; /* persistent schedules: blocks launched per compute unit, 0 = as many
                             as the kernel's occupancy allows; scf_get_tile reports the number
                             the two-step (fuse = 2) or single-step list uses.  Ignored otherwise. */
} scf_tile;

enum { SCF_ORDER_STRIPS = 0, SCF_ORDER_BANDS = 1, SCF_ORDER_XCD = 2, SCF_ORDER_PERSIST = 4 };

typedef struct scf_ctx scf_ctx;
typedef struct scf_batch scf_batch;

/* ---------------------------------------------------------------------------------------------
 * Single channel.
 * ------------------------------------------------------------------------------------------- */

/* Device workspace needed for one channel: two FP32 population buffers (2 x 2 x 9 planes),
 * a 2-plane density field, per-row partial sums and one observation record; each plane is
 * ny rows of nx rounded up to 64 floats.  0 if the geometry is invalid (including a channel
 * above the 4 GiB population-buffer limit of scf_geometry). */
size_t scf_workspace_bytes(const scf_geometry* geom);

/* Create a context and set every population to the rest equilibrium of eqs. feq1-feq3,
 * f_i = f_i^eq(n_k, u = 0) with n_k = rho_k / m_k (solid nodes ignored).  rhoA, rhoB: host
 * FP64 ny*nx arrays, copied.  Synchronises the stream before returning.
 * Errors: SCF_EINVAL (geometry, params, workspace), SCF_EDEVICE. */
int scf_init(scf_ctx** out, const scf_geometry* geom, const scf_params* params,
             const double* rhoA, const double* rhoB, void* dev_ws, size_t ws_bytes,
             void* hip_stream);

/* Advance nsteps >= 0 time steps of eq. lbe: densities, forces (eqs. forcing, forcingw),
 * common velocity, shifted equilibrium, BGK collision, streaming with half-way bounce-back.
 * Asynchronous on the stream; launches are replayed from a captured HIP graph when nsteps is
 * large enough.  Errors: SCF_EINVAL, SCF_EDEVICE (launch failure), SCF_EUNSTABLE (reported
 * lazily: the last scf_observe found flags bit1 set; the steps were still enqueued, and no
 * synchronisation is added to find out). */
int scf_step(scf_ctx* ctx, int64_t nsteps);

/* Observables of the current state (see scf_obs).  Enqueues two small kernels, copies one
 * record to the host and synchronises the stream.  Returns SCF_EUNSTABLE (with *out filled)
 * when flags bit1 is set. */
int scf_observe(scf_ctx* ctx, scf_obs* out);

/* Host copies of the current densities n_A, n_B (ny*nx each, FP64, 0 on solid nodes).
 * Synchronises the stream. */
int scf_get_density(scf_ctx* ctx, double* nA, double* nB);

/* Host copy of the current populations f[k][i][y][x] (2*9*ny*nx FP64, directions numbered as
 * in Sec. 2: 0 rest, 1-4 axis at 0/90/180/270 deg, 5-8 diagonals at 45/135/225/315 deg; solid
 * nodes 0).  Uses the idle population buffer as staging.  Synchronises the stream. */
int scf_get_populations(scf_ctx* ctx, double* f);

/* Select the step kernel (SCF_VARIANT_*).  Default SCF_VARIANT_FUSED. */
int scf_set_variant(scf_ctx* ctx, int32_t variant);

/* Set the launch schedule of the fused step: tiles of bx columns by cy rows (every other tile
 * of a strip walks its rows downward), taken by the blocks of one launch in the given order,
 * and one or two time steps per launch (fuse).  A new context starts with bx = 256, cy = 16,
 * order = SCF_ORDER_PERSIST | SCF_ORDER_XCD, graph_steps = 64, fuse = 2, blocks_per_cu = 0.  Schedules change only the order of work, never
 * the result.  Invalidates captured graphs.  Errors: SCF_EINVAL (bx not 64/128/256/512,
 * cy < 1, unknown order, graph_steps < 0, fuse not 1 or 2). */
int scf_set_tile(scf_ctx* ctx, const scf_tile* tile);
int scf_get_tile(const scf_ctx* ctx, scf_tile* tile);

/* Time candidate schedules (bx, cy, order, fuse) for `trial_steps` launches each, time the
 * best eight again with 4 x trial_steps launches, and keep the fastest per time step.  Every
 * trial launch reads the resident buffer and writes the idle one, so the state is unchanged.
 * The graph length is kept.  Writes the chosen schedule to *chosen if non-NULL. */
int scf_autotune(scf_ctx* ctx, int32_t trial_steps, scf_tile* chosen);

/* scf_autotune with a cache: cache_path names a text file of lines
 * "key bx cy order fuse blocks_per_cu ms_per_step", key a 64-bit hash (hex) of the device
 * (architecture name, compute units), the library's schedule version and the channels'
 * geometry class (nx, ny, x0, x1 and solid mask of every channel).  A line with this context's
 * key applies its schedule without timing; otherwise the schedules are timed as scf_autotune
 * does and one line is appended (the file is created if missing).  NULL cache_path: plain
 * scf_autotune.  Errors as scf_autotune, and SCF_EINVAL when the line cannot be written (the
 * tuned schedule is applied all the same). */
int scf_autotune_cached(scf_ctx* ctx, int32_t trial_steps, const char* cache_path, scf_tile* chosen);

/* Elapsed time step count of the context. */
int64_t scf_time(const scf_ctx* ctx);

/* Checkpoint: header (magic, version, geometry, params, t) and the FP32 post-collision
 * buffer, written to / read from a file.  scf_load requires the same geometry.
 * Errors: SCF_EINVAL (path), SCF_ESTATE (mismatch or bad file), SCF_EDEVICE. */
int scf_save(scf_ctx* ctx, const char* path);
int scf_load(scf_ctx* ctx, const char* path);

/* Release the context (host objects and graphs only; the workspace stays the caller's). */
void scf_destroy(scf_ctx* ctx);

/* Thread-local text of the last error, never NULL. */
const char* scf_last_error(void);

/* ---------------------------------------------------------------------------------------------
 * Batched: nchan independent channels advanced together, one launch per step over a packed
 * tile list of all channels (the calibration sweep: uneven H, L, wall couplings and tau).
 * ------------------------------------------------------------------------------------------- */

/* Workspace for nchan channels with room for max_samples observation records per channel. */
size_t scf_batch_workspace_bytes(int32_t nchan, const scf_geometry* geoms, int32_t max_samples);

/* geoms, params, rhoA[c], rhoB[c]: arrays of nchan entries (host).  Every sample_every >= 1
 * steps the observables of all channels are recorded on the device (up to max_samples each,
 * including the t = 0 record).  Errors as scf_init. */
int scf_batch_init(scf_batch** out, int32_t nchan, const scf_geometry* geoms,
                   const scf_params* params, const double* const* rhoA, const double* const* rhoB,
                   int32_t sample_every, int32_t max_samples, void* dev_ws, size_t ws_bytes,
                   void* hip_stream);

/* Advance every channel by nsteps, recording samples on the way.  Asynchronous.  Returns
 * SCF_EUNSTABLE (after enqueueing the steps) when the last scf_batch_observe found an unstable
 * sample. */
int scf_batch_step(scf_batch* b, int64_t nsteps);

/* Copy the recorded samples to out[c * max_samples + s] (nchan * max_samples records) and the
 * number recorded per channel to *nsamples.  Synchronises the stream.  Returns SCF_EUNSTABLE
 * if any recorded sample has flags bit1 set (all records are still written). */
int scf_batch_observe(scf_batch* b, scf_obs* out, int64_t* nsamples);

/* Host copy of channel c's densities (ny*nx FP64 each). */
int scf_batch_get_density(scf_batch* b, int32_t c, double* nA, double* nB);

/* Schedule of the batched step, as scf_set_tile / scf_get_tile. */
int scf_batch_set_tile(scf_batch* b, const scf_tile* tile);
int scf_batch_get_tile(const scf_batch* b, scf_tile* tile);

/* Autotune the batched step as scf_autotune, and with a cache as scf_autotune_cached (the key
 * covers every channel of the batch, in order). */
int scf_batch_autotune(scf_batch* b, int32_t trial_steps, scf_tile* chosen);
int scf_batch_autotune_cached(scf_batch* b, int32_t trial_steps, const char* cache_path, scf_tile* chosen);

void scf_batch_destroy(scf_batch* b);

/* ---------------------------------------------------------------------------------------------
 * Surrogate: a multilayer perceptron that maps sweep parameters and time to the front and
 * precursor positions, trained on trajectories of the batched LBM and used in its place inside
 * the training range.  d_in inputs -> `depth` hidden SiLU layers of `width` units -> 2 outputs.
 * Hidden-to-hidden layers run on BF16 MFMA with FP32 accumulation (forward and backward); the
 * first and output layers, master weights, gradients and Adam moments are FP32.
 * Inputs are normalised on the device by the mean and standard deviation of the data given to
 * scf_sur_set_data (identity before any data).  Loss: (1/2n) sum_rows w_row |y - t|^2.
 * Parameters are one FP32 vector, layer by layer: W (rows = outputs, row-major), then b.
 * ------------------------------------------------------------------------------------------- */

typedef struct scf_sur scf_sur;

typedef struct {
    int32_t d_in;        /* inputs per row, 1..32 */
    int32_t width;       /* hidden units per layer, a positive multiple of 64 */
    int32_t depth;       /* hidden layers, 1..16 */
    int32_t max_batch;   /* rows per pass, a positive multiple of 64 */
    int64_t max_data;    /* training rows the workspace holds */
    float lr, beta1, beta2, eps;   /* Adam */
    uint64_t seed;       /* parameter initialisation and minibatch draws */
} scf_sur_cfg;

/* Device workspace for a configuration; 0 if the configuration is invalid. */
size_t scf_sur_workspace_bytes(const scf_sur_cfg* cfg);

/* Create a network; weights are drawn on the device uniform in +-1/sqrt(fan_in) from cfg->seed,
 * biases are 0, Adam moments 0.  Workspace and stream as for scf_init.  Synchronises. */
int scf_sur_create(scf_sur** out, const scf_sur_cfg* cfg, void* dev_ws, size_t ws_bytes,
                   void* hip_stream);

/* Number of FP32 parameters (199 170 for 4 inputs, 256 x 4 hidden). */
int64_t scf_sur_param_count(const scf_sur* s);
int scf_sur_get_params(scf_sur* s, float* out);        /* host copy, param_count floats */
int scf_sur_set_params(scf_sur* s, const float* in);   /* also refreshes the BF16 copies */
int scf_sur_reset_optimizer(scf_sur* s);               /* Adam moments and step count to 0 */
int scf_sur_set_lr(scf_sur* s, float lr);              /* Adam step size for later updates, > 0 */

/* Copy n training rows (host: X n*d_in, T n*2, optional per-row weights w, NULL = 1) to the
 * device and compute there the per-input mean, standard deviation, min and max (the training
 * hull).  Errors: SCF_EINVAL (n outside [1, max_data]). */
int scf_sur_set_data(scf_sur* s, const float* X, const float* T, const float* w, int64_t n);
int scf_sur_get_norm(scf_sur* s, float* mean, float* stdv, float* lo, float* hi);   /* any may be NULL */
/* Set the input normalisation and the training hull directly (d_in floats each, stdv > 0), e.g.
 * for a network whose parameters were saved after training.  Errors: SCF_EINVAL. */
int scf_sur_set_norm(scf_sur* s, const float* mean, const float* stdv, const float* lo, const float* hi);

/* One forward and backward pass on an explicit batch (n <= max_batch rows, host arrays):
 * returns the loss and, if grad is non-NULL, the gradient (param_count floats). */
int scf_sur_grad(scf_sur* s, const float* X, const float* T, const float* w, int32_t n,
                 float* loss, float* grad);
/* The same pass followed by one Adam update. */
int scf_sur_step(scf_sur* s, const float* X, const float* T, const float* w, int32_t n,
                 float* loss);

/* `steps` Adam updates on minibatches of `batch` rows (a multiple of 64) drawn with replacement
 * from the stored data by a counter-based hash; each update is one replay of a captured HIP
 * graph.  Writes the last minibatch loss.  Errors: SCF_ESTATE without data. */
int scf_sur_train(scf_sur* s, int64_t steps, int32_t batch, float* last_loss);

/* Predictions for n rows (host X n*d_in -> Y n*2).  in_hull (optional, n bytes) is 1 where every
 * input lies inside [min, max] of the stored training inputs; callers answer the other rows with
 * the LBM. */
int scf_sur_predict(scf_sur* s, const float* X, int64_t n, float* Y, uint8_t* in_hull);

/* Allocation-free form of scf_sur_predict, for callers that cannot allocate device memory or
 * synchronise: code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  X (n*d_in floats), Y (n*2 floats) and in_hull (optional, n bytes: 1 where every
 * input lies inside the training hull, all 0 before any data or norm was set) are DEVICE
 * pointers owned by the caller.  The same layer kernels as scf_sur_predict give the same Y bit
 * for bit.  Their activations live in a library-owned device array of 20 MiB per GPU (held
 * until the process ends) instead of the workspace; one call takes rows_pad * (4 d_in +
 * 16 width) bytes of it (rows_pad = n rounded up to 64, plus alignment), so at width 256 and 5
 * inputs up to 5056 rows per call; larger n returns SCF_EINVAL and nothing is enqueued.
 * Asynchronous on the network's stream; no allocation, copy to or from the host, or
 * synchronisation.  The array keeps the last call's contents; every call writes the parts it
 * reads.  Calls that overlap on one GPU (any networks, any streams) race on the array.  Errors:
 * SCF_EINVAL (NULL, n < 0, n too large), SCF_EDEVICE (launch failure, or no array address on
 * the device current at scf_sur_create). */
int scf_sur_predict_noalloc(scf_sur* s, const float* X, int64_t n, float* Y, uint8_t* in_hull);

void scf_sur_destroy(scf_sur* s);

/* ---------------------------------------------------------------------------------------------
 * Three-dimensional capillary (D3Q19), the extension the paper names as future work
 * (Conclusions).  The step is that of Sec. 2 on the D3Q19 lattice: equilibrium
 * w_i n (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u) with w = 1/3 (rest), 1/18 (6 axis links), 1/36
 * (12 edge links); bulk and wall forces of eqs. forcing and forcingw with the same link weights;
 * common velocity, shifted equilibrium, BGK, pull streaming with half-way bounce-back.  The
 * weights' z-projection is D2Q9 with rest fraction 4/9, so a z-independent state evolves as the
 * 2-D model.  FP32 state.  By default one fused kernel per step: tiles of 64 x 4 (x, z) nodes walk
 * cy rows of y, keeping the densities of three y-slices in LDS; the two-kernel form (a density
 * field, then pull + collide) is selectable (scf3_set_schedule) and is the only one when one
 * component's 19 planes exceed 4 GiB (unsigned 32-bit buffer offsets).  Both give identical
 * results.
 * ------------------------------------------------------------------------------------------- */

typedef struct {
    int32_t nx, ny, nz;     /* box, periodic in x, y and z; 3 <= nx < 2^20, 3 <= ny, nz <= 65535 */
    int32_t x0, x1;         /* the capillary occupies x in [x0, x1) */
    int32_t walls_y;        /* non-zero: solid planes y = 0 and y = ny-1 over the capillary (a slit) */
    int32_t walls_z;        /* non-zero: solid planes z = 0 and z = nz-1 too (a square duct) */
} scf3_geometry;

typedef struct {
    int64_t t;
    double mass[2];         /* sum of n_k over fluid nodes (FP64) */
    double z;               /* front on the centre line (the up to four lines nearest
                               y = (ny-1)/2, z = (nz-1)/2, averaged): first downward crossing of
                               n_A - n_B scanning from x0/2, relative to x0; NaN if none */
    int32_t flags;          /* as scf_obs.flags */
    int32_t reserved;
} scf3_obs;

typedef struct scf3_ctx scf3_ctx;

/* Device workspace for one 3-D box: two FP32 population buffers (2 x 2 x 19 planes), a 2-plane
 * density field, per-row partial sums and one record; a plane is nz*ny rows of nx rounded up to
 * 64 floats.  0 if the geometry is invalid. */
size_t scf3_workspace_bytes(const scf3_geometry* geom);

/* Create a 3-D context at rest equilibrium.  params->alpha must be 4/9 for both components (the
 * D3Q19 equilibrium has fixed weights); G, gw, tau and mass as in scf_params.  rhoA, rhoB: host
 * FP64 nz*ny*nx arrays (x fastest), copied.  Workspace and stream as for scf_init.  Synchronises.
 * Errors: SCF_EINVAL, SCF_ENOMEM, SCF_EDEVICE. */
int scf3_init(scf3_ctx** out, const scf3_geometry* geom, const scf_params* params,
              const double* rhoA, const double* rhoB, void* dev_ws, size_t ws_bytes,
              void* hip_stream);

/* Advance nsteps >= 0 steps (one launch each, two in the two-kernel form; asynchronous on the
 * stream).  SCF_EUNSTABLE (after enqueueing) when the last scf3_observe found flags bit1 set. */
int scf3_step(scf3_ctx* ctx, int64_t nsteps);

/* Step schedule: fused = 1 (one kernel, cy >= 1 rows of y per tile, default 16 or the two-kernel
 * form where the fused one does not fit) or fused = 0 (two kernels, cy ignored).  The state is
 * unchanged; results do not depend on the schedule.  *_get_* writes the current one.
 * Errors: SCF_EINVAL (fused not 0/1, cy < 1, or fused = 1 where a component's 19 planes exceed
 * 4 GiB). */
int scf3_set_schedule(scf3_ctx* ctx, int32_t fused, int32_t cy);
int scf3_get_schedule(const scf3_ctx* ctx, int32_t* fused, int32_t* cy);

/* Observables of the current state; synchronises.  SCF_EUNSTABLE (with *out filled) when
 * flags bit1 is set. */
int scf3_observe(scf3_ctx* ctx, scf3_obs* out);

/* Host copies of n_A, n_B (nz*ny*nx each, FP64, 0 on solid nodes).  Synchronises. */
int scf3_get_density(scf3_ctx* ctx, double* nA, double* nB);

/* Host copy of the populations f[k][i][z][y][x] (2*19*nz*ny*nx FP64; i = 0 rest, 1-6 axis
 * +x,-x,+y,-y,+z,-z, 7-18 edges +x+y,-x-y,+x-y,-x+y,+x+z,-x-z,+x-z,-x+z,+y+z,-y-z,+y-z,-y+z;
 * solid nodes 0).  Uses the idle population buffer as staging.  Synchronises. */
int scf3_get_populations(scf3_ctx* ctx, double* f);

int64_t scf3_time(const scf3_ctx* ctx);
void scf3_destroy(scf3_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SCF_H */
