/*
 * swe.h -- C ABI of the MI355X shallow-water finite-volume library (libswe.so).
 *
 * Method: Delmas & Soulaimani, "Parallel high-order resolution of the
 * Shallow-water equations on real large-scale meshes with complex
 * bathymetries".  One explicit time step of the 2D shallow-water equations on
 * one sub-domain of an unstructured triangle mesh with k layers of ghost
 * cells: MUSCL reconstruction with a slope limiter (Sec. 6.2.3), hydrostatic
 * reconstruction with wet/dry treatment, HLLC (Sec. 6.2.1) or WAF
 * (Sec. 6.2.2) fluxes, the cell sum of eq. (vlap2) with bed source, Manning
 * friction and Euler / SSP-RK2 update (Sec. 6.1), the CFL step of Sec. 6.1,
 * and the on-device packing of the send buffers of Sec. 6.4 (receives land in
 * place because ghosts are numbered contiguously per owner, Sec. 3.3).
 *
 * Conventions
 *  - Every function returns an int status: SWE_OK (0) or a negative SWE_ERR_*.
 *    No exception crosses the ABI.  swe_last_error() gives a message for the
 *    last failure on a context; swe_strerror() names a code.
 *  - Host arrays passed in are copied; the caller keeps ownership.
 *  - Device pointers (where == SWE_DEVICE) are borrowed for the duration of
 *    the call only and must be valid on the context's device and ordered with
 *    the context's stream (the library synchronises the stream before it
 *    returns from any call that reads or writes caller memory).
 *  - All buffers the library allocates are owned by the context and released
 *    by swe_destroy().
 *  - Work is issued on the context's stream (one the library creates,
 *    default priority, non-blocking, or the caller's, swe_config.stream:
 *    then the caller's own work on that stream is ordered with the
 *    library's without synchronisation).  swe_step() is asynchronous; health
 *    errors (non-finite values, negative depths) are reported at the next
 *    synchronising call (swe_sync, swe_time, swe_read_state, swe_health).
 *  - One context per host thread; calls on one context are not thread-safe.
 *  - Cell layout: SoA arrays of n_total cells; the owned cells come first
 *    (indices [0, n_owned)), ghost cells after them, in one contiguous block
 *    per peer (see swe_subdomain_*).
 */
#ifndef SWE_H
#define SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWE_ABI_VERSION 5

/* status codes */
#define SWE_OK 0
#define SWE_ERR_ARG -1            /* bad argument (null pointer, bad size, bad enum) */
#define SWE_ERR_MESH -2           /* mesh fails validation at upload */
#define SWE_ERR_STATE -3          /* state missing or invalid (e.g. negative depth given) */
#define SWE_ERR_NONFINITE -4      /* a NaN/Inf appeared in an owned cell while stepping */
#define SWE_ERR_NEGATIVE_DEPTH -5 /* a depth below -eps appeared in an owned cell while stepping */
#define SWE_ERR_DEVICE -6         /* HIP runtime error */
#define SWE_ERR_OOM -7            /* an allocation failed (device; host in the toolkit) */
#define SWE_ERR_UNSUPPORTED -8    /* option not available in this build */

/* enums */
#define SWE_F32 0
#define SWE_F64 1
#define SWE_HLLC1 0       /* first-order HLLC (Sec. 6.2.1) */
#define SWE_MUSCL 1       /* MUSCL reconstruction + HLLC (Sec. 6.2.3) */
#define SWE_WAF 2         /* weighted average flux (Sec. 6.2.2) */
#define SWE_EULER 0
#define SWE_RK2 1         /* two-stage SSP Runge-Kutta (Heun) */
#define SWE_MINMOD 0      /* beta = 1 limiter (MINBEE) */
#define SWE_SUPERBEE 1    /* beta = 2 limiter */
#define SWE_VANALBADA 2
#define SWE_LEARNED 3     /* per-half-edge network phi in [0,1] x central slope */
#define SWE_ZEROSLOPE 4   /* slopes forced to zero (first order through the MUSCL path) */
#define SWE_WAF_SUPERBEE 0
#define SWE_WAF_GODUNOV 1   /* A = 1: WAF reduces to HLLC */
#define SWE_WAF_UNLIMITED 2 /* A = |c| */
#define SWE_HOST 0
#define SWE_DEVICE 1

/* boundary tags in cell_nbr (a negative entry instead of a neighbour index) */
#define SWE_BC_WALL -1
#define SWE_BC_TRANSMISSIVE -2
#define SWE_BC_INFLOW -3
#define SWE_BC_OUTFLOW -4   /* fixed stage */
#define SWE_BC_HALO -5      /* edge cut by the end of the ghost layers: transmissive */

/* health bits (swe_health) */
#define SWE_HEALTH_NONFINITE 1
#define SWE_HEALTH_NEGDEPTH 2
#define SWE_HEALTH_CLIPPED 4   /* a depth in [-eps, 0) was set to 0 */

typedef struct swe_ctx swe_ctx;
typedef struct swe_subdomain swe_subdomain;

/* Solver options.  Defaults from swe_config_default(). */
typedef struct {
    int abi_version;   /* SWE_ABI_VERSION */
    int precision;     /* SWE_F32 | SWE_F64: arithmetic and state type */
    int scheme;        /* SWE_HLLC1 | SWE_MUSCL | SWE_WAF */
    int integrator;    /* SWE_EULER | SWE_RK2 */
    int limiter;       /* SWE_MINMOD | SWE_SUPERBEE | SWE_VANALBADA | SWE_LEARNED | SWE_ZEROSLOPE */
    int waf_limiter;   /* SWE_WAF_* */
    int cfl_rule;      /* 0: min_i R_i/lambda_i;  1: min_i R_i / max_i lambda_i (printed form) */
    int device;        /* HIP device ordinal */
    double g;          /* gravity, default 9.81 */
    double cfl;        /* default 0.45 */
    double eps;        /* wet/dry threshold [m], default 1e-6 */
    double dt_max;     /* cap on the CFL step (<= 0: none); step used when no cell is wet */
    int block;         /* threads per block = cells per tile: 64, 128, 256 or 512 (0: 256,
                          64 for FP32 WAF with explicit Euler on the tiled kernel);
                          the one-thread-per-cell kernel, FP64 and WAF use at most 256
                          (FP64 WAF tiles at most 128) */
    int cell_kernel;   /* 1: one-thread-per-cell stage kernel for every scheme; 0: the
                          tiled kernels (HLLC1, MUSCL, and WAF with Euler steps; WAF with
                          RK2 uses the cell kernel) */
    void *stream;      /* NULL: the context creates its own stream (default priority,
                          non-blocking); else a hipStream_t on `device`, borrowed: all of
                          the context's work goes to it and it is never destroyed */
    int waves;         /* FP32 tiled kernel with 256-cell tiles (first-order HLLC and MUSCL
                          with a classic limiter): waves per SIMD it is built for, 6 or 7;
                          0 (default): 7 when that lets the chip hold every tile of a mesh
                          of up to two rounds at once, or when a launch spans 8 or more
                          rounds (then a persistent grid of 7 blocks per compute unit),
                          else 6.  Same results either way. */
    int phi_every;     /* SWE_LEARNED: phi is evaluated on the steps whose index since the
                          last set_state is a multiple of phi_every (1, 2, 3 or 6; 0: every
                          step), and on the first step after swe_limiter_set_weights or
                          swe_autotune; the steps between reuse the last phi.  Each
                          evaluation reads U^n of its own step, as with phi_every 1. */
    /* Optional allocator of the context's device buffers (both NULL: hipMalloc
     * and hipFree), e.g. a framework's caching allocator.  alloc(bytes, user)
     * returns memory on `device` usable by the context's stream, or NULL (the
     * call then fails with SWE_ERR_OOM); free(ptr, user) takes back a pointer
     * alloc returned, and is called only after the context's stream has
     * finished with it.  Both are called from the thread calling the library
     * (mesh upload, series and weight setting, autotune, destroy). */
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *alloc_user;
    int waf_positivity; /* WAF: 1 (default) keeps depths non-negative at wet/dry fronts:
                          an edge's mass flux out of a cell is at most 0.99 h R / (2 dt)
                          (R the inscribed radius, i.e. the edge's share L / P of the
                          cell's water per step); a WAF flux beyond it is blended
                          towards the HLLC flux of the same states; 0: plain WAF */
    int phi_in_stage;  /* SWE_LEARNED with the tiled kernel: 0 (default) evaluates the
                          network in a kernel of its own ahead of each step; 1 evaluates
                          it inside the step's first stage (phi stored for the second;
                          the far side of a tile-crossing edge evaluated where it is
                          needed), which saves that kernel's loads but adds its
                          arithmetic to a stage that is already half arithmetic-bound:
                          slower on the meshes measured.  Same results either way. */
} swe_config;

/* One sub-domain (or a whole mesh: n_owned == n_total, n_peers == 0).
 * Cell connectivity is the fixed-degree CSR of triangles: cell i owns the
 * three entries [3i, 3i+3) of cell_nodes and cell_nbr; local edge m of cell i
 * joins cell_nodes[3i+m] and cell_nodes[3i+(m+1)%3]. */
typedef struct {
    int32_t n_nodes;
    const double *node_xy;      /* [2*n_nodes] x,y */
    int32_t n_owned, n_total;   /* ghosts are [n_owned, n_total) */
    const int32_t *cell_nodes;  /* [3*n_total] counter-clockwise */
    const int64_t *cell_gid;    /* [n_total] global ids: each edge flux is computed with
                                   L = the cell of smaller gid (canonical orientation) */
    const int32_t *cell_nbr;    /* [3*n_total] local neighbour index, or a SWE_BC_* tag */
    const double *cell_b;       /* [n_total] bed elevation */
    const double *cell_manning; /* [n_total] Manning n (0: frictionless) */
    int32_t n_peers;
    const int32_t *peer_part;   /* [n_peers] ascending part ids (informative) */
    const int32_t *recv_off;    /* [n_peers+1]: ghost block q = [n_owned+recv_off[q], n_owned+recv_off[q+1]) */
    const int32_t *send_off;    /* [n_peers+1] */
    const int32_t *send_idx;    /* [send_off[n_peers]] local owned cells, per peer in the
                                   receiver's order */
    double inflow_q;            /* total inflow discharge [m^3/s] on SWE_BC_INFLOW edges */
    double inflow_length;       /* total length of the inflow edges of the WHOLE mesh
                                   (<= 0: computed from this mesh's owned cells) */
    double outflow_stage;       /* free-surface elevation on SWE_BC_OUTFLOW edges */
} swe_mesh;

/* ---- context ---------------------------------------------------------- */
void swe_config_default(swe_config *cfg);
int swe_create(const swe_config *cfg, swe_ctx **out);
void swe_destroy(swe_ctx *ctx);
const char *swe_last_error(const swe_ctx *ctx);
const char *swe_strerror(int code);

/* Copy a mesh to the device: validation (counter-clockwise cells, symmetric
 * neighbours, ghost and send ranges in bounds), geometry (areas, normals,
 * lengths, inscribed radii, MUSCL distances) and the device layout.
 * Replaces any previous mesh; the state must be set again afterwards.
 * SWE_ERR_MESH for a mesh without cells; SWE_ERR_UNSUPPORTED when a
 * per-cell array would exceed 4 GiB (more than about 89 million cells in
 * FP32, 44 million in FP64, per context).  Both size checks come before any
 * of the mesh's arrays is read. */
int swe_mesh_upload(swe_ctx *ctx, const swe_mesh *mesh);

/* Inflow hydrograph Q(t), piecewise linear through n points (clamped at the
 * ends), evaluated at each stage's time.  n = 0 restores the constant Q.
 * Waits for the context's stream (the series buffers are replaced). */
int swe_set_bc_series(swe_ctx *ctx, int n, const double *t, const double *q);

/* State of all n_total cells in the context's precision (float or double),
 * three SoA arrays.  set_state also sets the time and computes the CFL step
 * of the first step.  Negative or non-finite depths are rejected. */
int swe_set_state(swe_ctx *ctx, const void *h, const void *hu, const void *hv, int where,
                  double t);
int swe_read_state(swe_ctx *ctx, void *h, void *hu, void *hv, int where);

/* Solution output that overlaps the steps (Sec. 5.2: solutions written
 * while the solver keeps computing, the table of write modes): queues on the context's stream a copy of the state of all
 * n_total cells, as it stands after the steps queued so far, into three
 * device buffers of n_total values each in the context's precision, then
 * records done_event (a hipEvent_t, may be NULL) on that stream.  Returns
 * without waiting and without reporting health, so a copy to host memory
 * on another stream after done_event overlaps the following steps.
 * SWE_ERR_ARG if a buffer is not device memory of the context's device;
 * the buffers must not be reused before done_event has completed. */
int swe_snapshot(swe_ctx *ctx, void *h, void *hu, void *hv, void *done_event);

/* Batched ensemble: several independent meshes (no ghost cells), one
 * scenario each, concatenated in one context and stepped together by the
 * same kernel launches (one graph), each scenario with its own CFL step,
 * time, inflow and outflow.  State arrays of set_state / read_state are the
 * concatenation in the order given; swe_batch_offsets gives the first cell
 * of each scenario ([n_scen + 1] entries, may be NULL to get n_scen only).
 * 1 <= n_meshes <= 32768, else SWE_ERR_ARG. */
int swe_mesh_upload_batch(swe_ctx *ctx, int n_meshes, const swe_mesh *meshes);
int swe_set_bc_series_scenario(swe_ctx *ctx, int scenario, int n, const double *t,
                               const double *q);
int swe_batch_offsets(const swe_ctx *ctx, int32_t *n_scenarios, int32_t *offsets);
int swe_scenario_times(swe_ctx *ctx, double *t);  /* [n_scenarios]; syncs */

/* Autotuner: times n_steps CFL steps for each launch shape of the
 * configured stage kernel (64, 128, 256 or, FP32 tiled kernel only, 512
 * threads per block; one tile per block or a persistent grid of the blocks
 * the chip holds at once; with 256-cell FP32 tiles, builds for
 * 6 and 7 waves per SIMD) from the current state, keeps the fastest and
 * restores the state, clocks and time.  The choice never changes results
 * (the tiled kernel is bitwise independent of the tiling, and both builds
 * perform the same operations).
 * Outputs may be NULL; *persistent_grid is the chosen grid (-1: one tile per
 * block).  Untuned contexts sweep tiles with a persistent grid of the blocks
 * the chip holds at once when a launch has 8 or more rounds of tiles, and
 * launch one tile per block otherwise. */
int swe_autotune(swe_ctx *ctx, int n_steps, int *block, int *persistent_grid);

/* n_steps explicit steps, asynchronous on the context's stream.
 * dt_fixed > 0: every step uses that dt; otherwise the CFL step of Sec. 6.1
 * (computed on the device from the owned cells, never copied to the host). */
int swe_step(swe_ctx *ctx, int n_steps, double dt_fixed);

/* One step with the high-overlap schedule of Sec. 6.4 (the send cells are
 * computed first and their values leave while the interior is computed),
 * as one GPU does it: the pack is fused into the step's last stage kernel.
 * Each thread that computes a send cell's new state (the send cells are
 * local cells [0, max(send_idx) + 1), numbered first, so their tiles are
 * the first dispatched) also writes it to that cell's entries of
 * dev_sendbuf ([3][n_send] as swe_pack_ghosts lays it out), while other
 * tiles are still being computed; there is no pack launch.  The state,
 * clock and buffer equal those of swe_step(ctx, 1, dt_fixed) followed by
 * swe_pack_ghosts bitwise.  pack_done_event (a caller's hipEvent_t, may be
 * NULL) is recorded on the context stream once the buffer is complete, so
 * that a caller's exchange on another stream can wait for it.  Without send
 * cells this is swe_step(ctx, 1, dt_fixed).  Asynchronous; not captured in
 * the step graph.  SWE_ERR_ARG for a missing send buffer when n_send > 0. */
int swe_step_overlap(swe_ctx *ctx, double dt_fixed, void *dev_sendbuf, void *pack_done_event);

/* Capture and instantiate the launch graph swe_step replays for runs of
 * steps with this dt_fixed (dt_fixed <= 0: CFL mode), launching nothing, so
 * that a following swe_step pays no capture on the host.  swe_step builds
 * the same graph on first use when this was not called; a graph is rebuilt
 * when dt_fixed or the launch shape changes.  SWE_ERR_STATE without a state
 * (or without the network's weights for SWE_LEARNED). */
int swe_prepare(swe_ctx *ctx, double dt_fixed);

/* The kernel(s) one step launches under the context's configuration: *name
 * points to a static string (kernel names joined by '+'), and
 * *launches_per_step counts the launches of one step (e.g. 2 for the two
 * stage launches of RK2; a learned-limiter step that evaluates phi, where
 * phi_every > 1 skips the network's launch on the steps between).  For
 * measurement tools. */
int swe_step_kernel(const swe_ctx *ctx, const char **name, int *launches_per_step);

int swe_sync(swe_ctx *ctx);                 /* wait + report health */
int swe_time(swe_ctx *ctx, double *t);      /* simulated time (syncs) */
/* CFL step of the current state over the owned cells (syncs): the step
 * swe_step takes in CFL mode.  A sub-domain without a wet owned cell gives
 * dt_max, or 0 when none is configured (no bound from this part).
 * Sub-domains combine by a minimum (a min all-reduce) with cfl_rule 0:
 * each contributes +inf for 0, and an infinite result means no wet cell
 * anywhere (step 0, as one context would).  With cfl_rule 1 the global
 * step is not the minimum of the parts' steps. */
int swe_local_dt(swe_ctx *ctx, double *dt);
int swe_health(swe_ctx *ctx, int *bits);    /* SWE_HEALTH_* bits since the last set_state,
                                               over owned cells (a ghost cell's new state is
                                               provisional: the next exchange replaces it) */

/* Gather the owned cells listed in send_idx into dev_sendbuf, laid out
 * [3][n_send] (h, hu, hv; context precision), in CSR order of the peers.
 * Asynchronous on the context stream, after the steps queued before it: the
 * buffer is complete once that stream passes this point (swe_sync, or work
 * queued after it on the same stream, e.g. the exchange). */
int swe_pack_ghosts(swe_ctx *ctx, void *dev_sendbuf);
/* Copy dev_recvbuf, laid out [3][n_total - n_owned], into the ghost cells.
 * Asynchronous on the context stream: writes to dev_recvbuf issued on other
 * streams must be complete before this call, and the buffer must stay
 * unchanged until the stream passes it. */
int swe_unpack_ghosts(swe_ctx *ctx, const void *dev_recvbuf);
int swe_ghost_sizes(const swe_ctx *ctx, int32_t *n_send, int32_t *n_ghost);

/* Wall time of the kernels of the last swe_step call (ms, measured with HIP
 * events on the context stream; syncs). */
int swe_last_step_ms(swe_ctx *ctx, float *ms);

/* ---- learned slope limiter (an addition of this library) ---------------
 * A per-half-edge network 14 -> 32 -> 32 -> 1 (ReLU, ReLU, sigmoid) gives
 * phi in [0,1]; with limiter == SWE_LEARNED the MUSCL slope of a half-edge
 * becomes phi times the central slope (U_R - U_Lupw)/|x_R - x_Lupw| of
 * Sec. 6.2.3.  It falls back to the minmod slope when phi is outside [0,1]
 * or NaN or the reconstructed depth is negative, and to first order where
 * the classic limiter does (dry stencil cell, boundary edge).  phi is
 * evaluated once per time step (or every phi_every steps, see swe_config),
 * from the state the step starts from, and both RK2 stages use it.  Parameters
 * are 1569 floats: W1[32][14], b1[32], W2[32][32], b2[32], W3[32], b3. */
#define SWE_MLP_NPARAM 1569
#define SWE_PAIR_RECORD 40  /* floats per training record */
/* Store the parameters (host, FP32) rounded to BF16 for the matrix-core
 * inference kernel. */
int swe_limiter_set_weights(swe_ctx *ctx, const float *params);
/* phi of every half-edge of the current state into dev_phi[3*n_total]
 * (NaN where the half-edge is not reconstructed to second order: not
 * evaluated).  The phi that later steps reuse (phi_every > 1) is left as
 * it was. */
int swe_limiter_phi(swe_ctx *ctx, float *dev_phi);
/* Training records from a fine solution on the red refinement of the coarse
 * mesh (both contexts on one device, same precision).  dev_children
 * [4*n_total(coarse)]: fine local index of the four children of each coarse
 * cell (child k at parent node k, 3 the central one).  The coarse state is
 * set to the restriction (mean of the children) at t = 0, and dev_rec
 * [3*n_total(coarse)][40] receives per half-edge: features[14], cell values
 * (h, eta, u_n, u_t)[4], central slopes[4], the target distance d = d_mid / 2,
 * target[4] = mean of the two children touching the edge (their mean
 * centroid lies halfway from the cell centroid to the edge midpoint), valid
 * flag, the minmod interface values (h, eta, u_n, u_t)[4] at the edge
 * midpoint, backward slopes (q_c - q_upw)/d_up [4] and forward slopes
 * (q_R - q_c)/d_fwd [4].  Children out of range give SWE_ERR_ARG. */
int swe_limiter_pairs(swe_ctx *coarse, swe_ctx *fine, const int32_t *dev_children, float *dev_rec);

/* Trainer: FP32 master weights and Adam moments on one device.  The loss of
 * n records (indices dev_idx into dev_rec[n_rec][40]) is
 * (1/n) sum sum_v wv[v] (q_v + d clip(phi s_v, sb_v, sf_v) - t_v)^2 over
 * v = h, eta, u_n, u_t (d: the record's target distance; clip: the TVD
 * bound the solver applies to phi times the central slope, zero unless the
 * backward and forward slopes sb, sf share a sign, else of the sign of sf
 * and at most 2 min(|sb|, |sf|)), i.e. the misfit of the value the solver
 * reconstructs.  The gradient is zero where the clip does not pass phi s
 * through. */
typedef struct swe_trainer swe_trainer;
int swe_trainer_create(int device, const float *init_params, swe_trainer **out);
void swe_trainer_destroy(swe_trainer *tr);
/* loss and gradient (host [1569]) at the current weights, no update */
int swe_trainer_loss_grad(swe_trainer *tr, const float *dev_rec, int32_t n_rec,
                          const int32_t *dev_idx, int32_t n, const float *wv, float *loss,
                          float *grad_host);
/* one Adam step (beta 0.9 / 0.999, eps 1e-8) with learning rate lr */
int swe_trainer_step(swe_trainer *tr, const float *dev_rec, int32_t n_rec, const int32_t *dev_idx,
                     int32_t n, const float *wv, float lr, float *loss);
int swe_trainer_get_params(swe_trainer *tr, float *host_params);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): the loss and gradient of swe_trainer_loss_grad for parameters
 * given as a device array dev_params[1569] (FP32, the trainer's layout),
 * written to the caller's device buffer dev_grad_loss[1570] (gradient, then
 * the loss), queued on `stream` (a hipStream_t; NULL is the null stream) of
 * the current device, no host synchronisation.  It allocates nothing: the
 * per-block partial sums live in a static device array of this library
 * (512 blocks x 1570 floats, 3.2 MB per GPU, held until the process ends),
 * whose size does not depend on n (the grid is capped at 512 blocks, each
 * looping over chunks of 64 records), so no size is refused for want of
 * workspace.  Bitwise equal to swe_trainer_loss_grad with the same
 * parameters (same kernels, same grid, same reduction order).  Calls that
 * overlap on one GPU share that array and race: order them on one stream.
 * Errors: SWE_ERR_ARG for a null pointer or n, n_rec <= 0 (dev_idx entries
 * outside [0, n_rec) count as absent records, as in the trainer);
 * SWE_ERR_DEVICE when the array's address cannot be found or a launch
 * fails. */
int swe_trainer_loss_grad_static(const float *dev_params, const float *dev_rec, int32_t n_rec,
                                 const int32_t *dev_idx, int32_t n, const float *wv,
                                 float *dev_grad_loss, void *stream);

/* ---- host mesh toolkit (Sec. 3.1 - 3.3), CPU only ---------------------- */
/* Dual graph: cell across each local edge, -1 where none (global numbering).
 * Fails with SWE_ERR_MESH for an edge shared by more than two cells or by two
 * cells that traverse it in the same direction. */
int swe_dual_graph(int32_t n_nodes, int32_t n_cells, const int32_t *cell_nodes, int32_t *nbr);
/* Greedy breadth-first partition into P parts of sizes floor(n/P)+(p < n%P). */
int swe_partition_bfs(int32_t n_cells, const int32_t *nbr, int32_t P, int32_t *part);
/* Total length of the edges whose boundary tag bc[3*i+m] equals tag (for
 * the inflow length of a whole mesh before it is split into sub-domains). */
int swe_edge_length_sum(int32_t n_nodes, const double *node_xy, int32_t n_cells,
                        const int32_t *cell_nodes, const int8_t *bc, int32_t tag, double *out);
/* 32-bit Morton key of each cell centroid (16 bits per axis, x on even bits,
 * over the bounding box of all centroids). */
int swe_morton_keys(int32_t n_nodes, const double *node_xy, int32_t n_cells,
                    const int32_t *cell_nodes, uint32_t *key);
/* Part p with k ghost layers: local numbering (send cells, interior cells,
 * ghost blocks per peer), local neighbour table with boundary tags
 * (bc[3*n_cells] gives the tag of each edge that has no neighbour), receive
 * ranges and send lists.  The object owns its arrays. */
int swe_subdomain_build(int32_t n_nodes, const double *node_xy, int32_t n_cells,
                        const int32_t *cell_nodes, const int32_t *nbr, const int8_t *bc,
                        const int32_t *part, int32_t P, int32_t p, int32_t k,
                        swe_subdomain **out);
/* All P parts at once on n_threads host threads (<= 0: one per hardware
 * thread), out[P]: each part equals what swe_subdomain_build gives for it
 * (Sec. 3: ghost layers of every sub-domain generated in parallel; here the
 * parts of one shared-memory mesh are built concurrently).  On an error
 * every out[p] is NULL and the first error is returned; SWE_ERR_OOM when an
 * allocation fails.  The caller frees each part with swe_subdomain_free. */
int swe_subdomain_build_all(int32_t n_nodes, const double *node_xy, int32_t n_cells,
                            const int32_t *cell_nodes, const int32_t *nbr, const int8_t *bc,
                            const int32_t *part, int32_t P, int32_t k, int32_t n_threads,
                            swe_subdomain **out);
/* All P parts built the way Sec. 3.2 (Fig. `mainalg`) does it on
 * distributed memory, one worker per part on n_threads host threads: each
 * worker holds only its own cells (node ids, node coordinates, boundary
 * tags) and matches their edges itself (no global dual graph); the workers
 * share the bounding boxes of their nodes and centroids (all-gather), take
 * as potential neighbours the parts whose closed node boxes meet theirs,
 * build their k inner boundary layers (own cells within k edges of an edge
 * not shared with another own cell), exchange those layers once with their
 * potential neighbours, find ghost layer j as the received cells j edges
 * from their own cells, tell each owner which cells they receive (its send
 * lists) and number their cells as swe_subdomain_build does.  bc must tag
 * every edge on the domain boundary (negative); an edge tagged 0 is
 * interior, and one whose neighbour is not in the sub-domain becomes
 * SWE_BC_HALO.  When no part lies within k layers of a part whose box does
 * not meet its own, every out[p] equals swe_subdomain_build's; otherwise the
 * ghosts owned by such a far part are missed (the limitation the paper
 * states).  n_potential[P] (may be NULL) receives each part's number of
 * potential neighbours.  Errors as swe_subdomain_build_all (SWE_ERR_MESH for
 * an edge of more than two cells); on error every out[p] is NULL. */
int swe_subdomain_build_layers(int32_t n_nodes, const double *node_xy, int32_t n_cells,
                               const int32_t *cell_nodes, const int8_t *bc, const int32_t *part,
                               int32_t P, int32_t k, int32_t n_threads, swe_subdomain **out,
                               int32_t *n_potential);
typedef struct {
    int32_t n_owned, n_total, n_peers, n_send;
    const int32_t *l2g;       /* [n_total] global id of each local cell */
    const int32_t *layer;     /* [n_total] 0 owned, j for ghost layer j */
    const int32_t *owner;     /* [n_total] part of each local cell */
    const int32_t *nbr;       /* [3*n_total] local neighbour or SWE_BC_* tag */
    const int32_t *peers;     /* [n_peers] */
    const int32_t *recv_off;  /* [n_peers+1] */
    const int32_t *send_off;  /* [n_peers+1] */
    const int32_t *send_idx;  /* [n_send] */
} swe_subdomain_view;
int swe_subdomain_view_get(const swe_subdomain *sd, swe_subdomain_view *view);
void swe_subdomain_free(swe_subdomain *sd);

#ifdef __cplusplus
}
#endif
#endif /* SWE_H */
