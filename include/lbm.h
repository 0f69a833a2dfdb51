/*
 * lbm.h -- C ABI of the MI355X (gfx950) patch-and-block D3Q19 lattice
 * Boltzmann library.
 *
 * The method is the one of Feichtinger et al., "A Flexible Patch-Based Lattice
 * Boltzmann Parallelization Approach for Heterogeneous GPU-CPU Clusters":
 *   - D3Q19 BGK with the incompressible equilibrium of Eq. (2), populations
 *     stored shifted by w_i rho0 (Sec. 2.1);
 *   - pull streaming over two grids, SoA layout (Sec. 2.1, Sec. 3.2);
 *   - half-way bounce-back walls with an optional wall velocity (Sec. 2.1);
 *   - one Patch split into a Cartesian grid of Blocks, each with an
 *     axis-aligned bounding box and a BlockID (Sec. 4.2);
 *   - a time step is one Sweep: the ghost-layer exchange between Blocks plus
 *     the stream-collide kernel over every Block (Sec. 4, Sec. 4.4).
 * A body force (Guo forcing, u = j/rho0 + g/2) extends the method for
 * force-driven channels; with g = 0 it reduces exactly to the plain method.
 *
 * Conventions
 *   - Every call returns lbm_status.  No C++ exception crosses the ABI.
 *   - Cell arrays are global, x fastest: index c = (z*ny + y)*nx + x.
 *     Vector fields are SoA: u[a*N + c], a = 0,1,2.  Population arrays are
 *     [i][z][y][x] with the direction order
 *       0:(0,0,0) 1:(+1,0,0) 2:(-1,0,0) 3:(0,+1,0) 4:(0,-1,0) 5:(0,0,+1)
 *       6:(0,0,-1) 7:(+1,+1,0) 8:(-1,-1,0) 9:(+1,-1,0) 10:(-1,+1,0)
 *       11:(+1,0,+1) 12:(-1,0,-1) 13:(+1,0,-1) 14:(-1,0,+1) 15:(0,+1,+1)
 *       16:(0,-1,-1) 17:(0,+1,-1) 18:(0,-1,+1).
 *   - Walls lie half a cell outside the outermost cells of a WALL face.
 *   - Ownership: the context owns all device memory it allocates (through
 *     dev_alloc/dev_free when given, else hipMalloc/hipFree).  The caller
 *     owns every buffer it passes; none is retained after a call returns.
 *   - Ordering: work is enqueued on params.stream.  lbm_step is
 *     asynchronous; lbm_macroscopic, lbm_residual, lbm_sums, lbm_get_state
 *     and lbm_info synchronise that stream.
 *   - Errors: on LBM_EINVAL / LBM_ENOMEM the context is unchanged.
 *     LBM_EUNSTABLE is returned by a synchronising call that finds a
 *     non-finite FP64 sum; the state is then undefined.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef LBM_H_
#define LBM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = 1,    /* bad argument: parameters, tiling, sizes, NULL pointers */
  LBM_ENOMEM = 2,    /* device or host allocation failed */
  LBM_EDEVICE = 3,   /* a HIP call failed (message in lbm_last_error) */
  LBM_ESTATE = 4,    /* call not valid in the current state */
  LBM_EUNSTABLE = 5  /* non-finite values found by a reduction */
} lbm_status;

/* Storage precision of the populations.  F16S/BF16S store the shifted
 * values f~ = f - w_i rho0 (Sec. 2.1) in 16 bits, converted with
 * round-to-nearest-even, and always compute in FP32. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3 } lbm_precision;

/* Face kinds.  PERIODIC faces come in opposite pairs.  VELOCITY and
 * PRESSURE are open faces, on the faces of one axis (x, y or z; the other
 * face of that axis open or WALL): the boundary node one cell beyond the
 * face, next to the domain cell x_f, holds the post-collision
 * populations of the non-equilibrium extrapolation rule (Guo, Zheng and Shi,
 * 2002; on-GPU boundary conditions are the paper's stated future work,
 * Sec. 5.1 and the conclusion):
 *     f~_i(x_b) = feq~_i(drho_b, u_b) + f~*_i(x_f) - feq~_i(drho_f, u_f),
 * drho_f and u_f being the moments of x_f's last collision.  VELOCITY
 * prescribes u_b = wall_u[face] and takes drho_b = drho_f; PRESSURE
 * prescribes rho_b = face_rho[face] and takes u_b = u_f.  A link whose
 * source lies beyond a WALL face as well bounces back (walls take
 * precedence).  Open faces need two or more cells across them and no solid
 * cell on the face; the Blocks may be cut along and across the open axis (a
 * boundary node feeds the face cells of the Blocks next to it through their
 * ghost cells).  Contexts with open x faces run one cell per lane. */
typedef enum { LBM_PERIODIC = 0, LBM_WALL = 1, LBM_VELOCITY = 2, LBM_PRESSURE = 3 } lbm_face;

/* Half-open global cell box [lo, hi) of one Block (the Block AABB, Sec. 4.2). */
typedef struct { int32_t lo[3], hi[3]; } lbm_aabb;

typedef struct {
  int32_t dims[3];        /* nx, ny, nz of the single Patch, each >= 1 */
  int32_t face[6];        /* lbm_face of -x,+x,-y,+y,-z,+z: both faces of an axis
                             PERIODIC, or each WALL, VELOCITY or PRESSURE (the
                             last two on the faces of one axis only) */
  double wall_u[6][3];    /* WALL faces: wall velocity, tangential; VELOCITY faces: the
                             prescribed velocity (any direction); 0 on other faces */
  double tau;             /* BGK relaxation time, > 0.5 (nu = (tau - 1/2)/3) */
  double rho0;            /* reference density, > 0 (1 for all presets) */
  double force[3];        /* body force g per unit mass, lattice units */
  int32_t precision;      /* lbm_precision */
  int32_t fp64_math;      /* F32 storage: 1 = FP64 arithmetic, 0 = mixed (FP32 even part of the
                             collision; FP64 velocity, odd part and update); F64 storage
                             always FP64; F16S/BF16S always FP32 */
  void* stream;           /* hipStream_t; NULL = the null stream */
  void* (*dev_alloc)(size_t bytes, void* user);  /* optional device allocator */
  void (*dev_free)(void* ptr, void* user);
  void* alloc_user;
  int32_t row_pad;        /* x-row layout: 0 = automatic (rows rounded up to 128 bytes,
                             except FP32/FP64 rows of an odd number of 64-byte halves on
                             Blocks with an even y extent, packed two rows to three
                             128-byte lines); -1 = every row rounded up to 128 bytes;
                             n > 0 = rounded up, then n more 128-byte lines (layout only;
                             results do not depend on it; the sweep may store into the
                             padding, whose contents no call reads or returns) */
  double face_rho[6];     /* PRESSURE faces: the prescribed density (> 0); ignored
                             on other faces */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Kernel schedule of a context: how the Blocks are cut into work items and
 * launched (the role of the paper's per-Block kernel selection, Sec. 4.1). */
typedef struct {
  int32_t fused_exchange;  /* ghost exchange: 0 = a separate copy kernel after the sweep;
                              1 = the sweep writes every ghost value into the neighbours'
                              ghost layers itself; 2 = the sweep writes the x-face ghost
                              planes for rows off the y/z faces, the copy kernel the rest */
  int32_t item_cells;      /* target cells per work item (whole x-rows), >= 1 */
  int32_t wg_size;         /* threads per workgroup: 64, 128 or 256 */
  int32_t persistent;      /* 0: one workgroup per item; k > 0: k workgroups per
                              compute unit loop over the item list */
  int32_t graph_steps;     /* time steps per captured HIP graph; 0: plain launches */
  int32_t nontemporal;     /* 1: the sweep streams (non-temporal) its row stores; 0: ordinary
                              stores.  Loads and values written one per row (walls, x-ghost
                              planes) are ordinary either way.  Results do not depend on it. */
  int32_t cells_per_lane;  /* cells per lane along x: 0 = automatic (1); 1; or 2 (only for
                              F16S/BF16S and for F32 storage with FP64 arithmetic, with
                              every Block's x extent even and no open x face, else
                              LBM_EINVAL).  Results do not depend on it. */
} lbm_schedule;

typedef struct {
  int64_t n_cells;          /* nx*ny*nz */
  int64_t n_fluid;          /* cells that are not solid */
  int32_t n_blocks;
  int32_t n_items;          /* work items of the current schedule */
  int64_t steps;            /* time steps since the last (re)initialisation */
  int64_t device_bytes;     /* device memory held by the context */
  double bytes_per_update;  /* algorithmic HBM bytes per fluid-cell update:
                               19 loads + 19 stores of one stored value,
                               plus the link mask when obstacles exist */
  int32_t storage_bytes;    /* bytes per stored population */
  int32_t has_obstacles;
} lbm_info;

/* Create a context for the Patch p->dims split into nblocks Blocks.
 * The AABBs must tile the Patch exactly without overlap and form a
 * Cartesian grid (every distinct lo/hi per axis is a cut shared by all Blocks
 * it crosses); BlockID = index in `blocks`.  Block data live on the device;
 * the management data (AABB, BlockID, neighbour table) is also kept on the
 * host (Sec. 4.2).  State after creation: all fluid, rest equilibrium
 * f~ = 0.  Errors: LBM_EINVAL (bad parameters or tiling, or a Block one
 * of whose population arrays, ghost layers included, would reach 4 GiB:
 * about 530 M cells in FP64, 1070 M in FP32), LBM_ENOMEM, LBM_EDEVICE.
 * *out is set only on success. */
lbm_status lbm_create_blocks(const lbm_params* p, const lbm_aabb* blocks, int32_t nblocks,
                             lbm_ctx** out);

/* Solid mask on the host, nx*ny*nz bytes, x fastest, nonzero = solid;
 * NULL = all fluid.  Builds the per-cell link masks for half-way bounce-back
 * at obstacles (Sec. 2.1) and resets the state to rest (f~ = 0).
 * LBM_EINVAL for a solid cell on an open face, or for obstacles in a Block
 * six of whose population arrays would reach 4 GiB (about 89 M cells in
 * FP64, 178 M in FP32, 357 M in 16-bit storage). */
lbm_status lbm_set_geometry(lbm_ctx* c, const uint8_t* solid);

/* Warm start: f~ = feq~(rho - rho0, u) of Eq. (2) in every fluid cell, 0 in
 * solid cells.  Host arrays rho[N], u[3*N] (FP64).  Fills the ghost layers. */
lbm_status lbm_set_equilibrium(lbm_ctx* c, const double* rho, const double* u);

/* Enqueue n >= 0 time steps (each: stream-collide sweep over all Blocks plus
 * the ghost exchange, and with open faces the fill of their boundary nodes)
 * on the context stream.  Asynchronous. */
lbm_status lbm_step(lbm_ctx* c, int64_t n);
/* Advance n steps as persistent launches of steps_per_launch steps each (the
 * last one shorter): one workgroup per resident slot walks the Blocks' work
 * items (the block list) step after step, with the ghost exchange fused into
 * the sweep and a grid-wide barrier between steps (a cooperative launch:
 * every workgroup is resident).  Same results as lbm_step, bit for bit;
 * stream-ordered and asynchronous like lbm_step (Sec. 4: a Sweep is exchange
 * plus kernel; here one launch holds many of them).  LBM_EINVAL: n < 0,
 * steps_per_launch outside [1, 2^20], Blocks on the host CPU, open faces, or
 * a schedule with two cells per lane; LBM_EDEVICE if the cooperative launch
 * fails. */
lbm_status lbm_step_persistent(lbm_ctx* c, int64_t n, int32_t steps_per_launch);

/* Advances n steps (1 <= n <= 100000) exactly as lbm_step does, launched one
 * by one (no graphs), with a HIP event pair around every sweep launch and
 * the work after it (the separate ghost exchange and, with open faces, the
 * boundary-node fill) on params.stream; returns the mean duration of one
 * sweep launch and of the work after it (0 when the exchange is fused into
 * the sweep and no face is open), in milliseconds: the per-kernel durations
 * that bandwidth accounting divides by.  Synchronises. */
lbm_status lbm_step_timed(lbm_ctx* c, int64_t n, double* sweep_ms, double* exchange_ms);

/* Density and velocity used by the most recent collision (before any step:
 * the initial field), FP64: rho[N], u[3*N]; solid cells give rho0 and 0.
 * dst_is_device = 1: rho/u are device pointers.  Synchronises. */
lbm_status lbm_macroscopic(lbm_ctx* c, double* rho, double* u, int32_t dst_is_device);

/* r = ||u^n - u^(n-1)||_2 / ||u^n||_2 over fluid cells, FP64 (steady-state
 * measure).  Needs >= 2 steps since the last (re)initialisation, else
 * LBM_ESTATE.  Synchronises. */
lbm_status lbm_residual(lbm_ctx* c, double* r);

/* Velocity snapshot for residuals over several steps: stores u of the
 * current state (FP64, 4 N doubles of device memory, allocated on first use
 * through params.dev_alloc and kept until lbm_destroy).  Enqueued on
 * params.stream; lbm_set_geometry, lbm_set_equilibrium and lbm_set_state
 * discard the snapshot. */
lbm_status lbm_residual_mark(lbm_ctx* c);

/* r = ||u^n - u^m||_2 / ||u^n||_2 over fluid cells (FP64), u^m the snapshot of
 * lbm_residual_mark taken n - m steps ago (written to *nsteps when non-NULL).
 * With n - m even it is blind to the period-two population cycles that
 * bounce-back sustains in cells whose open links lie in one plane (their
 * momentum normal to that plane is reversed every step), which keep the
 * one-step residual of lbm_residual from decaying in random porous media.
 * LBM_ESTATE without a snapshot.  Synchronises. */
lbm_status lbm_residual_since_mark(lbm_ctx* c, double* r, int64_t* nsteps);

/* Global FP64 sums over fluid cells: mass = sum rho, mom = sum rho0 u. */
lbm_status lbm_sums(lbm_ctx* c, double* mass, double mom[3]);
/* lbm_sums for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, results and errors as lbm_sums, bit for bit, but the
 * reduction's scratch (per-workgroup partials and the final sums, at most
 * 6 x 1024 + 8 doubles; larger needs are refused with LBM_EINVAL) lives in
 * one static device array per GPU that the library holds until the process
 * ends, so the call allocates nothing (the context, made earlier, owns all
 * other device memory).  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents (nothing in it needs to start at zero):
 * calls that overlap on one GPU, from several threads or contexts, race.
 * Synchronises the context's stream.  LBM_EDEVICE if the array's address
 * cannot be obtained. */
lbm_status lbm_sums_noalloc(lbm_ctx* c, double* mass, double mom[3]);

/* Checkpoint: the current post-collision populations, 19 x N in [i][z][y][x],
 * host buffer; as_fp64 = 1: FP64 values, 0: the storage type's raw values
 * (8, 4 or 2 bytes each).  Solid cells read 0.  Synchronises. */
lbm_status lbm_get_state(lbm_ctx* c, void* f, int32_t as_fp64);

/* Restore a checkpoint of the same layout (solid entries are ignored and held
 * at 0).  The state is taken as post-collision; the step counter is reset to
 * 1 so that lbm_macroscopic reports its moments with the half-force shift. */
lbm_status lbm_set_state(lbm_ctx* c, const void* f, int32_t as_fp64);

/* Replace the state by the mean of the last two post-collision states (this
 * step's and the previous step's, which the two grids hold), value by value
 * in the storage format; ghost layers, wall slots and open-face boundary
 * nodes are then rebuilt from the mean.  Every part of the state that flips
 * sign from one step to the next cancels; the rest moves half a step back.
 * For starts from a state set from outside (the learned warm start sets an
 * equilibrium of predicted fields, Sec. 2.1's f^eq): such a state excites
 * period-two components that a few pore geometries hardly damp, so the
 * velocity keeps a step-to-step oscillation for tens of thousands of steps
 * while its two-step mean has converged.  One call after the first step
 * removes them.  Not an operation of the paper's method.
 * LBM_ESTATE without a step since the state was last set (creation,
 * lbm_set_geometry, lbm_set_equilibrium, lbm_set_state or this call);
 * LBM_EINVAL with host Blocks.  The step count is kept; lbm_residual needs
 * one more step.  Synchronises. */
lbm_status lbm_average_two_steps(lbm_ctx* c);

/* The schedule in force.  After lbm_create_blocks: fused_exchange = 0 for one
 * Block and 2 for several, item_cells = 512, wg_size = 256, persistent = 0,
 * graph_steps = 0, nontemporal = 1 (0 for grids of at most 192 MiB, which the
 * memory-side cache holds from one step to the next), cells_per_lane = 0. */
lbm_status lbm_get_schedule(lbm_ctx* c, lbm_schedule* s);
/* Validate and apply a schedule (rebuilds the item list and drops captured
 * graphs).  Results do not depend on the schedule, bit for bit. */
lbm_status lbm_set_schedule(lbm_ctx* c, const lbm_schedule* s);

/* Time candidate schedules for `trial_steps` steps each on this context and
 * apply the fastest.  The state is saved before and restored after, so the
 * simulation is unchanged.  cache_path (may be NULL) names a text file of
 * earlier choices keyed by the problem signature (device, storage and
 * arithmetic precision, obstacles, dimensions, the Block tiling, the six face
 * kinds and row_pad); a hit skips the trials, a line this context refuses is
 * skipped, and a new choice is appended.  The chosen schedule is written to
 * *chosen when non-NULL; the schedule's graph_steps is kept. */
lbm_status lbm_autotune(lbm_ctx* c, const char* cache_path, int32_t trial_steps,
                        lbm_schedule* chosen);

/* Heterogeneous runs (Sec. 4.5, Sec. 5.3): the Blocks in ids[0..n) run on
 * the host CPU, the rest on the GPU.  Each Block carries the hardware it runs
 * on; a host Block keeps both grids in pinned host memory (hipHostMalloc)
 * with the same layout as on the GPU, and `threads` host threads (0: up to
 * 16) sweep them while the GPU sweeps its Blocks.  Values that cross between
 * a host and a GPU Block each step go through exchange buffers of one format
 * that both sides pack and unpack; the ghost exchange among GPU Blocks
 * follows the schedule's fused_exchange, and steps are launched one by one
 * (graph_steps is not used): each step's exchange is followed on the stream
 * by the next GPU sweep while the host unpacks and sweeps.  lbm_step returns
 * after the last step's exchange has arrived (synchronous with host Blocks).  The host sweep repeats the GPU
 * arithmetic operation for operation, so results equal the all-GPU run bit
 * for bit.  n = 0 returns every Block to the GPU.  The state is carried
 * over; lbm_macroscopic, lbm_residual*, lbm_sums and lbm_get_state copy the
 * host Blocks' state to the device first.  Synchronises.
 * LBM_EINVAL: n < 0 or > the Block count, ids NULL with n > 0, an id out of
 * range or repeated, threads outside [0, 1024], F16S/BF16S storage, or open
 * faces (with n > 0); LBM_ENOMEM: host or device allocation failed (every
 * Block then stays on the GPU).  lbm_autotune refuses a context with host
 * Blocks. */
lbm_status lbm_set_host_blocks(lbm_ctx* c, const int32_t* ids, int32_t n, int32_t threads);

/* n steps (1 <= n <= 100000) of a context with host Blocks, with the mean
 * per step of: the GPU sweep (HIP events), the host sweep (wall clock, from
 * the GPU launch to the last host thread), the exchange phase (wall clock,
 * from the end of both sweeps) and the whole step (wall clock), in
 * milliseconds.  LBM_ESTATE without host Blocks.  Synchronises. */
lbm_status lbm_step_host_timed(lbm_ctx* c, int64_t n, double* gpu_sweep_ms, double* cpu_sweep_ms,
                               double* exchange_ms, double* step_ms);

/* Static load balance (Sec. 5.3: Blocks per process raised until the work
 * is balanced): times trial_steps steps with every Block on the GPU, then
 * the host sweep of the last Block of the list, and puts the last k Blocks
 * of the list on the host, k the largest for which the host's predicted
 * sweep time (fluid cells over its measured rate) stays within the GPU's;
 * if the measured step with that split is not faster than the GPU alone, k
 * is 0.  The split is applied (lbm_set_host_blocks with `threads`) and
 * *n_host = k; ms_gpu_only / ms_balanced (may be NULL) receive the measured
 * step times of the GPU alone and of the split tried (with k = 0: of one
 * host Block).  The state is saved before and restored after the trials.
 * LBM_EINVAL: NULL c or n_host, trial_steps outside [1, 10000], threads
 * outside [0, 1024], F16S/BF16S storage or open faces. */
lbm_status lbm_balance_host_blocks(lbm_ctx* c, int32_t threads, int32_t trial_steps, int32_t* n_host,
                                   double* ms_gpu_only, double* ms_balanced);

/* Static facts and counters of a context.  Synchronises. */
lbm_status lbm_info_get(lbm_ctx* c, lbm_info* info);

lbm_status lbm_destroy(lbm_ctx* c);
const char* lbm_strerror(lbm_status s);
/* Text of the last error detected on this thread (empty if none). */
const char* lbm_last_error(void);

/* Device copy-bandwidth probe: copies `bytes` (a multiple of 16) from src to
 * dst (device pointers) `reps` times on `stream` and returns the average
 * time per copy in milliseconds -- the attainable-bandwidth benchmark of
 * Sec. 3.1, written for gfx950. */
lbm_status lbm_bw_probe(void* dst, const void* src, size_t bytes, int32_t reps, void* stream,
                        double* ms_per_copy);

/* HBM bandwidth ceilings of plain access patterns (the patterns the sweep's
 * bandwidth is read against; Sec. 3.1's attainable-bandwidth benchmark
 * widened to several patterns).  kind:
 *   0 reads `a`; 1 writes `b`; 2 copies a -> b, grid-strided 16-byte accesses;
 *   3 copies a -> b in one contiguous chunk per workgroup;
 *   4 triad b = a0 + 3 a1 (a holds a0 then a1: 2 * bytes);
 *   5 the sweep's pattern without arithmetic: `bytes` per side cut into 19
 *     arrays (starts staggered by 768 bytes), every lane reads one word of
 *     all 19 arrays of a and writes them to the 19 arrays of b; the word is
 *     4 * unroll bytes (unroll 1, 2 or 4); needs bytes >= 19 * 8192;
 *   6 hipMemcpyAsync device to device (a -> b); 7 hipMemsetD32Async of b.
 * Bytes moved per pass: `bytes` for kinds 0, 1 and 7, 3 * bytes for kind 4,
 * 2 * bytes for the copies (kind 5: 2 * 19 * P, P the largest multiple of 4096
 * with 19 P + 13824 <= bytes).
 * Buffers are device buffers of that size (b is overwritten, a is only
 * read), `unroll` (1, 2, 4 or 8) independent accesses in flight per thread,
 * nontemporal = 1 for streaming loads and stores, `grid` workgroups of 256
 * threads (0: 16 per compute unit; ignored by kinds 6 and 7).  After one
 * warm-up pass, reps passes on `stream`; *ms = mean time per pass.
 * LBM_EINVAL on bad arguments (a may be NULL for kinds 1 and 7),
 * LBM_EDEVICE on a HIP error.  Synchronises. */
lbm_status lbm_hbm_probe(int32_t kind, int32_t unroll, int32_t nontemporal, const void* a, void* b,
                         size_t bytes, int32_t grid, int32_t reps, void* stream, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H_ */
