/*
 * ofmi.h -- C ABI of the MI355X dense pyramidal Lucas-Kanade velocimetry library.
 *
 * The library computes, for two frames of a particle-image sequence, a dense displacement
 * field with one vector per pixel (Gautier & Aider, Sec. 2.4): an image pyramid built by
 * reducing each frame by a factor of 4 in area per level, a zero initial displacement at the
 * coarsest level, a fixed number of Gauss-Newton iterations per level minimising a sum of
 * squared differences over an interrogation window of radius r, each level's result seeding
 * the next finer level.  The level count n_lev counts full resolution (eq. 1); n_iter is the
 * number of iterations per level (Sec. 2.4, Table 1).
 *
 * Operators fixed where the paper is silent (identical on every entry point):
 *   pyramid  separable 5-tap binomial [1 4 6 4 1]/16 (rows first, then columns),
 *            clamp-to-edge, keep even rows/columns, level sizes ceil(H/2) x ceil(W/2);
 *   seed     u <- 2 * bilinear(u_coarse, x/2, y/2) on the finer grid (same for v);
 *   warp     W2(x,y) = bilinear(I2, x+u, y+v), sample coordinates clamped into the image;
 *   gradient central differences of W2 with clamped neighbours;
 *   window   unweighted (2r+1)^2 box, truncated at the image border;
 *   step     each window pixel m is linearised around its own estimate u(m); with
 *            It = W2 - I1 - Ix u - Iy v and A,B,C,sx,sy the window sums of
 *            Ix^2, IxIy, Iy^2, Ix It, Iy It, the new estimate is u(x) + e where
 *            H e = -(sx + A u + B v, sy + B u + C v), H = [[A,B],[B,C]]: Cramer's rule when
 *            AC - B^2 > 1e-5 (A+C)^2, rank-1 pseudo-inverse H/(A+C)^2 when A+C > 0, else e = 0.
 *   iterations are Jacobi (each iteration reads the previous iteration's whole field).
 *
 * Conventions for every entry point:
 *   - Planes are row-major and dense: element (x, y) of an H x W plane is at index y*W + x
 *     (x = column, y = row).  u is the displacement along x, v along y, in level-0 pixels,
 *     from frame 1 to frame 2: I2(x + u, y + v) ~ I1(x, y).
 *   - Every plane pointer is a HIP device pointer on the device that was current when the
 *     object was created.  Frames are uint8 (or float32 with OF_FLAG_INPUT_F32) and are only
 *     read; u and v are float32 and are written.  The caller owns frames and outputs and keeps
 *     them alive until the work enqueued on `stream` has completed.  The library never frees
 *     caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Compute calls
 *     only enqueue work on it and never synchronise the host.
 *   - Objects (plan, batch, session) are not re-entrant: calls on one object must be ordered
 *     on one stream.  Distinct objects are independent.  *_destroy synchronises the device
 *     before freeing.
 *   - Errors: create functions return NULL and compute functions return a non-zero of_status;
 *     nothing is enqueued on an argument error.  of_last_error() gives the text of the last
 *     failure on the calling thread.  Device faults surface at the caller's next
 *     synchronisation.
 */
#ifndef OFMI_H
#define OFMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OF_API __attribute__((visibility("default")))

typedef enum {
  OF_OK = 0,
  OF_EINVAL = 1,   /* invalid argument; nothing enqueued */
  OF_ENOMEM = 2,   /* workspace too small or allocation failure */
  OF_EHIP = 3,     /* a HIP runtime call or kernel launch failed */
  OF_ESTATE = 4    /* object used in a state that does not allow the call */
} of_status;

/* Flags of the *_ex constructors. */
#define OF_FLAG_FP16_STORAGE (1u << 0) /* pyramid levels >= 1 stored in FP16; all math FP32 */
#define OF_FLAG_INPUT_F32    (1u << 1) /* frames are float32 instead of uint8 */
#define OF_FLAG_NO_GRAPH     (1u << 2) /* batches: launch kernels one by one instead of
                                          replaying a captured hipGraph of the schedule;
                                          plans: eager launches even with OF_FLAG_GRAPH */
#define OF_FLAG_NORMALIZE    (1u << 3) /* plans only: equalise both frames locally (see
                                          of_normalize; radius OF_NORMALIZE_RADIUS, eps
                                          OF_NORMALIZE_EPS) before the pyramid */
#define OF_FLAG_GAUSSIAN_WINDOW (1u << 4) /* plans, batches and servers: weight the window
                                          sums by separable Gaussian taps
                                          exp(-d^2 / (2 sigma^2)), sigma = r/2, over the same
                                          (2r+1)^2 support (a variant of the unweighted
                                          interrogation window of Sec. 2.4) */
#define OF_FLAG_GRAPH        (1u << 5) /* plans only: capture the schedule into a hipGraph
                                          per pointer tuple and replay it; plans launch kernels
                                          one by one otherwise (batches replay graphs unless
                                          OF_FLAG_NO_GRAPH; servers and sessions launch
                                          kernels one by one) */

/* Tile variants of the fused iteration kernel (launch configuration; results do not depend
 * on them).  NARROW: 5 threads per output column.  WIDE: 10 threads per output column with
 * per-thread item indices held in registers (shortest dependent path per band, for launches
 * of about one tile per CU).  WIDE_LEAN: 10 threads per output column, indices recomputed
 * every band (fewer live registers, so two workgroups share a CU, for launches of many
 * tiles). */
#define OF_TILE_NARROW 0
#define OF_TILE_WIDE 1
#define OF_TILE_WIDE_LEAN 2
/* Plans with the box window only: the wide variant on strips of 32 or 16 output columns
 * (instead of 64), for levels with fewer tiles than CUs: more, smaller tiles, each with a
 * shorter path per band. */
#define OF_TILE_WIDE32 3
#define OF_TILE_WIDE16 4
/* Plans with the box window and r <= 8 only: WIDE32 / WIDE16 with two bands per pass (20
 * threads per output column): a tile's priming band and first output band (a tile of one
 * output band is exactly these two) take one dependent path through the kernel instead of
 * two, for levels of about one tile per CU. */
#define OF_TILE_WIDE32X2 5
#define OF_TILE_WIDE16X2 6
/* WIDE32X2 with the item indices recomputed every pass (as WIDE_LEAN): 60-80 instead of
 * 96-134 VGPRs, so two or three workgroups share a CU, for levels with more tiles than CUs. */
#define OF_TILE_LEAN32X2 7

#define OF_MAX_LEVELS 12
#define OF_MAX_RADIUS 12
#define OF_MAX_ITERS 1000
#define OF_MAX_NORMALIZE_RADIUS 16
#define OF_NORMALIZE_RADIUS 5      /* the paper's local radius (Sec. 2.4) */
#define OF_NORMALIZE_EPS 1.0f      /* added to the local standard deviation (frame units) */

typedef struct of_plan of_plan;

/* Workspace bytes a plan needs (pyramids of both frames + flow ping-pong), 0 on invalid
 * parameters.  Parameters as of_plan_create_ex. */
OF_API size_t of_plan_workspace_bytes(int H, int W, int levels, int radius, int iters,
                                      unsigned flags);

/* Plan for one frame size: H x W frames (1 <= H, W < 2^24, H * W < 2^30; every plan, batch
 * and server checks these sizes), `levels` pyramid levels including full resolution
 * (1 <= levels <= min(OF_MAX_LEVELS, 1 + floor(log2(min(H, W))))), window radius
 * 0 <= radius <= OF_MAX_RADIUS, 0 <= iters <= OF_MAX_ITERS iterations per level (Sec. 2.4,
 * eq. 1).  uint8 frames, FP32 storage.  The plan allocates its own workspace.
 * Returns NULL on invalid parameters or allocation failure. */
OF_API of_plan* of_plan_create(int H, int W, int levels, int radius, int iters);

/* As of_plan_create with `flags` (OF_FLAG_*).  If `workspace` is non-NULL it must be a device
 * buffer of at least of_plan_workspace_bytes(...) bytes, 256-byte aligned, owned by the caller
 * and kept alive until of_plan_destroy; if NULL the plan allocates it. */
OF_API of_plan* of_plan_create_ex(int H, int W, int levels, int radius, int iters,
                                  unsigned flags, void* workspace, size_t workspace_bytes);

/* Dense flow from frame I1 to frame I2 (both H x W, uint8 or float32 per the plan's flags)
 * into u and v (H x W float32, 4-byte aligned, u != v).  Enqueues the pyramid build and the
 * levels x iters iterations on `stream`.  iters = 0 writes zeros.  Kernels are launched one
 * by one (measured as fast as graph replay or faster for one stream of pairs from 256^2 to
 * 1024^2).  With OF_FLAG_GRAPH (and neither OF_FLAG_NO_GRAPH nor kernel timing) the schedule
 * is captured once per distinct (I1, I2, u, v) into a hipGraph held by the plan (at most 64,
 * least recently used evicted) and replayed on `stream`, one call per pair for callers whose
 * host thread is the bottleneck; the first call for a pointer tuple pays the capture.
 * Errors: OF_EINVAL on a NULL plan or pointer or u == v (nothing enqueued); OF_EHIP if a
 * launch fails. */
OF_API of_status of_compute(of_plan* plan, const void* I1, const void* I2, float* u, float* v,
                            void* stream);

/* Releases the plan and the workspace it allocated.  NULL-safe. */
OF_API void of_plan_destroy(of_plan* plan);

/* --------------------------------------------------------------------- allocation-free form
 * For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): the flow of one pair without a plan object, with
 * the pyramids and field buffers in a fixed device scratch array inside the library
 * (OF_NOALLOC_SCRATCH_MIB MiB on each device that calls it, held until the process ends).
 * Parameters and results as of_plan_create_ex + of_compute in the default launch
 * configuration (bitwise the same), except: no plan, no masks, no graph flags (OF_FLAG_GRAPH
 * and OF_FLAG_NO_GRAPH give OF_EINVAL), kernels are launched one by one on `stream`.  No call
 * allocates or frees memory; the first call on a device looks up that device's copy of the
 * array.  Every call on one device uses the same array, so calls that may overlap on one
 * device (different streams, other threads) race and must be ordered by the caller; each
 * call writes every scratch byte it reads.  Errors: OF_EINVAL on invalid parameters or
 * pointers (nothing enqueued); OF_ENOMEM when of_plan_workspace_bytes(...) of these
 * parameters exceeds of_noalloc_scratch_bytes() (e.g. 1024 x 1024 FP32 at 4 levels needs
 * about 20 MB; 2048 x 2048 does not fit); OF_EHIP on a launch failure. */
#define OF_NOALLOC_SCRATCH_MIB 32
OF_API size_t of_noalloc_scratch_bytes(void);
OF_API of_status of_compute_noalloc(int H, int W, int levels, int radius, int iters,
                                    unsigned flags, const void* I1, const void* I2, float* u,
                                    float* v, void* stream);

/* Region-of-interest mask, the speed lever of Sec. 3.3 (skip obstacles and side walls):
 * `mask` is a DEVICE H x W uint8 plane, nonzero = compute.  The plan copies it (on `stream`,
 * after synchronising the device) and derives one mask per level: a coarser pixel is
 * unmasked when any of its (up to four) finer pixels is.  Every iteration then writes zero
 * flow at masked pixels; iteration tiles without an unmasked output pixel are not computed
 * (zero is written).  Unmasked pixels see the zero flow of masked neighbours, so results near
 * a mask edge differ from the unmasked computation.  mask == NULL removes the mask.  The first
 * call allocates the mask pyramid (freed by of_plan_destroy).  Drops captured graphs.
 * Errors: OF_EINVAL (NULL plan), OF_ENOMEM, OF_EHIP (e.g. `mask` not a device pointer). */
OF_API of_status of_plan_set_mask(of_plan* plan, const uint8_t* mask, void* stream);

/* Level count from eq. 1: the smallest L >= 1 with dmax / 2^(L-1) < 3 px, capped at the
 * largest count an H x W frame allows (1 + floor(log2(min(H, W))), at most OF_MAX_LEVELS).
 * dmax: the largest expected displacement in pixels.  Host only (no device call).  Returns 0
 * for invalid arguments (H or W < 1, dmax negative or not finite). */
OF_API int of_levels_for_displacement(float dmax, int H, int W);

/* Per-level launch configuration of a plan: bands[l] = tile height of the iteration kernel
 * in bands of 2r+1 rows (1..64), variant[l] = OF_TILE_* (defaults: 4 bands for levels of 2^19
 * pixels and more, else 1; levels of under 384 tiles of 64 columns at that height take WIDE32
 * with 4 bands, WIDE16X2 (under 128 tiles) or LEAN32X2 with 1 band (WIDE32 above r = 8, WIDE
 * with OF_FLAG_GAUSSIAN_WINDOW), larger ones WIDE_LEAN;
 * WIDE32, WIDE16 and the X2 variants are not available with OF_FLAG_GAUSSIAN_WINDOW, the X2
 * variants not above r = 8).  Arrays of `levels` entries.  set_config drops the plan's captured graphs; OF_EINVAL for values out
 * of range.  Results do not depend on the configuration. */
OF_API of_status of_plan_get_config(const of_plan* plan, int* bands, int* variant);
OF_API of_status of_plan_set_config(of_plan* plan, const int* bands, const int* variant);

/* Autotuner: for each level in turn, times that level's iteration launches for bands in
 * {1,2,3,4,8} x the tile variants the plan allows (eight with the box window and r <= 8, five
 * with the box window above, three with the Gaussian window)
 * on the given buffers (reps timed runs after one warm-up) and keeps the fastest.
 * Synchronises `stream`; writes u, v. */
OF_API of_status of_plan_autotune(of_plan* plan, const void* I1, const void* I2, float* u,
                                  float* v, void* stream, int reps);

/* Text of the last failure on the calling thread ("" if none). */
OF_API const char* of_last_error(void);

/* --------------------------------------------------------------------- kernel timing
 * Event timing for measurement, on the launch stream.  enable = OF_TIMING_LAUNCH: every
 * kernel launch of the plan is bracketed by a pair of hipEvents (kernel ids OF_KERNEL_ITERATE,
 * OF_KERNEL_REDUCE).  enable = OF_TIMING_LEVEL: one event pair around all pyramid launches of
 * a pair (OF_KERNEL_REDUCE) and one around the K iteration launches of each level l
 * (OF_KERNEL_LEVEL(l)), with no events between the launches of a span, so a span's time per
 * launch is the kernels' back-to-back duration.  0 switches timing off.
 * of_plan_read_timing waits for the recorded events of `kernel`, returns the totals since
 * the last read and resets them.
 *   kernel: OF_KERNEL_ITERATE (the fused iteration), OF_KERNEL_REDUCE (pyramid: one
 *   reduction, or one launch building 2 or 3 levels, for levels of up to 2^20 pixels), or
 *   OF_KERNEL_LEVEL(l) (level l's iteration launches, OF_TIMING_LEVEL only).
 *   total_ms: summed event-to-event time; launches: number of kernel launches timed; units:
 *   pixel-iterations (ITERATE, LEVEL) or output pixels (REDUCE); bytes: algorithmic HBM bytes
 *   of those launches (ITERATE, LEVEL: per pixel-iteration 2 frame elements + 16 bytes of u,v
 *   read and written; REDUCE: per frame the input plane once and every output plane once).
 *   Any out pointer may be NULL.
 * Errors: OF_EINVAL on a NULL plan, unknown mode or kernel; OF_EHIP if event creation fails. */
#define OF_KERNEL_ITERATE 0
#define OF_KERNEL_REDUCE 1
#define OF_KERNEL_LEVEL(l) (16 + (l))
#define OF_TIMING_LAUNCH 1
#define OF_TIMING_LEVEL 2
OF_API of_status of_plan_set_timing(of_plan* plan, int enable);
OF_API of_status of_plan_read_timing(of_plan* plan, int kernel, double* total_ms,
                                     long long* launches, double* units, double* bytes);

/* --------------------------------------------------------------------- batched form
 * Many frame pairs of different sizes with common levels, radius and iterations, computed
 * together: each pyramid step and each (level, iteration) phase of the method (Sec. 2.4) is
 * one launch whose workgroups stride over a work list of tiles of all pairs.  The paper runs
 * one field at a time and notes that fields are independent of one another (Sec. 3.3); the
 * batch exploits that independence on one device. */
typedef struct of_batch of_batch;

/* Argument blocks of a batch, held in its workspace: one per cached graph (OF_BATCH_GRAPHS
 * pointer sets) and a ring of OF_BATCH_EAGER_SLOTS for eager runs. */
#define OF_BATCH_GRAPHS 8
#define OF_BATCH_EAGER_SLOTS 4

/* Workspace bytes of a batch of n pairs of sizes H[i] x W[i] (host arrays), 0 on invalid
 * parameters (each pair as of_plan_create_ex; 1 <= n <= 65536): every pair's pyramids and
 * field buffers, the tile work lists and the argument blocks. */
OF_API size_t of_batch_workspace_bytes(int n, const int* H, const int* W, int levels, int radius,
                                       int iters, unsigned flags);

/* Batch object.  H, W: host arrays of n sizes (copied).  workspace as in of_plan_create_ex.
 * Set-up call: uploads the work lists and allocates pinned staging for the argument blocks.
 * Returns NULL on invalid parameters or allocation failure. */
OF_API of_batch* of_batch_create(int n, const int* H, const int* W, int levels, int radius,
                                 int iters, unsigned flags, void* workspace,
                                 size_t workspace_bytes);

/* Flow of every pair i: frames I1[i] -> I2[i] into u[i], v[i].  I1, I2, u, v are HOST arrays
 * of n DEVICE pointers, each plane laid out as for of_compute with pair i's size.  The whole
 * schedule is one hipGraph replay per call, captured on the first call with a given set of
 * pointers; its arguments are uploaded on `stream` (pinned staging, asynchronous) into one of
 * the OF_BATCH_GRAPHS argument blocks.  A ninth pointer set takes the block of the least
 * recently used graph, which is dropped once its last replay has completed (the call waits
 * for that replay).  Otherwise the call allocates nothing and does not wait.  With
 * OF_FLAG_NO_GRAPH or timing on, launches are eager and the arguments go through a ring of
 * OF_BATCH_EAGER_SLOTS blocks; when the next one is still read by an earlier run the call
 * returns OF_ESTATE and enqueues nothing.  Results are bitwise identical to of_compute on the
 * same pair with the same tile configuration (the window sums do not depend on the tiling).
 * Errors: OF_EINVAL for a NULL batch, array or buffer or u[i] == v[i]; OF_ESTATE (eager ring
 * busy); OF_EHIP on launch failure. */
OF_API of_status of_batch_compute(of_batch* b, const void* const* I1, const void* const* I2,
                                  float* const* u, float* const* v, void* stream);

/* Per-level launch configuration: bands[l] = tile height in bands of 2r+1 rows (1..64),
 * grid[l] = workgroups of the iteration launches (0 = one per tile, else a persistent grid
 * striding over the work list), variant[l] = OF_TILE_NARROW, _WIDE or _WIDE_LEAN, or -1 for
 * the default (WIDE for launches of under 384 tiles, else WIDE_LEAN).  Arrays of `levels` entries; `variant` may
 * be NULL (get: not returned; set: -1 for every level).  set_config rebuilds the work lists
 * and drops captured graphs. */
OF_API of_status of_batch_get_config(const of_batch* b, int* bands, int* grid, int* variant);
OF_API of_status of_batch_set_config(of_batch* b, const int* bands, const int* grid,
                                     const int* variant);

/* Autotuner: for each level in turn, times that level's iteration launches for every
 * candidate (bands in {1,2,4,8}, grid in {one per tile, 256, 512, 1024, 2048}, the three
 * tile variants) on the given buffers (reps timed runs after one warm-up) and keeps the
 * fastest.  Synchronises `stream`.  The chosen configuration is read back with
 * of_batch_get_config. */
OF_API of_status of_batch_autotune(of_batch* b, const void* const* I1, const void* const* I2,
                                   float* const* u, float* const* v, void* stream, int reps);

/* Region-of-interest masks of a batch (the masking lever of Sec. 3.3, as of_plan_set_mask):
 * masks is a HOST array of n DEVICE pointers, masks[i] an H[i] x W[i] uint8 plane (nonzero =
 * compute) or NULL for an unmasked pair; masks == NULL removes every mask.  The batch builds
 * each masked pair's mask pyramid and its tile flags (refreshed when the tile heights change):
 * tiles without an unmasked pixel are left out of every iteration launch (the last iteration
 * writes their zero flow), masked pixels get zero flow, results equal of_compute of a plan
 * with the same mask, bitwise.  Set-up call: waits for the device, drops the captured graphs,
 * allocates the mask memory (mask pyramid, tile flags, and four FP32 flow planes per level
 * >= 1 of each masked pair; freed by of_batch_destroy).
 * Errors: OF_EINVAL (NULL batch), OF_EHIP. */
OF_API of_status of_batch_set_masks(of_batch* b, const uint8_t* const* masks, void* stream);

/* Kernel timing of a batch, as of_plan_set_timing / of_plan_read_timing. */
OF_API of_status of_batch_set_timing(of_batch* b, int enable);
OF_API of_status of_batch_read_timing(of_batch* b, int kernel, double* total_ms,
                                      long long* launches, double* units, double* bytes);

/* Releases the batch (synchronises the device first).  NULL-safe. */
OF_API void of_batch_destroy(of_batch* b);

/* --------------------------------------------------------------------- serving form
 * Frame streams (e.g. a camera sequence) processed pair by pair: each stream is a session that
 * keeps its previous frame's pyramid resident on the device, so a new frame costs one new
 * pyramid plus the iterations (the paper's first computing scheme, Sec. 2.4, in which each
 * field needs only one newly acquired image to be processed).  Sessions of one parameter set
 * belong to a server, which admits new streams against an HBM budget and pushes the new
 * frames of many sessions together (one launch per pyramid step and per (level, iteration)
 * phase over all of their tiles; kernels are launched one by one).
 *
 * Push arguments travel through a ring of OF_SERVER_RING staging slots (pinned host and
 * device memory of the server), sized when a session opens for a push of every open session.
 * A push never allocates and never waits: when the slot it needs is still held by one of the
 * last OF_SERVER_RING pushes in flight, it returns OF_ESTATE and enqueues nothing (retry once
 * an earlier push has completed).  Pushes of one server must be ordered on one stream; the
 * server is internally locked, so concurrent calls from several threads serialise. */
typedef struct of_server of_server;
typedef struct of_session of_session;

#define OF_SERVER_RING 8

/* Device bytes one session of an H x W stream keeps resident (two frame pyramids including
 * level 0, four level-0 FP32 field planes); also the workspace size of of_session_create and
 * of_server_open_ex.  0 on invalid parameters, including the plan-only flags
 * OF_FLAG_NORMALIZE and OF_FLAG_GRAPH. */
OF_API size_t of_session_bytes(int H, int W, int levels, int radius, int iters, unsigned flags);

/* Server for streams sharing levels, radius, iters and flags (OF_FLAG_NO_GRAPH ignored).
 * hbm_budget_bytes bounds the resident bytes of all open sessions (0 = unbounded). */
OF_API of_server* of_server_create(int levels, int radius, int iters, unsigned flags,
                                   size_t hbm_budget_bytes);

/* Opens a session for an H x W stream.  Returns NULL (of_last_error says why) when the
 * parameters are invalid, when admitting it would exceed the HBM budget, or on allocation
 * failure.  Set-up call: it may grow the server's staging ring (after waiting for the device)
 * and allocates the session memory (hipMalloc). */
OF_API of_session* of_server_open(of_server* s, int H, int W);

/* As of_server_open with caller-owned session memory: `workspace` is a device buffer of at
 * least of_session_bytes(...) bytes, 256-byte aligned, kept alive until the session is closed
 * (NULL = the library allocates it). */
OF_API of_session* of_server_open_ex(of_server* s, int H, int W, void* workspace,
                                     size_t workspace_bytes);

/* Pushes the next frame of each of n distinct sessions of server s (host arrays of n
 * entries; frames[i] a device plane of session i's size and the server's frame type).  For a
 * session that already holds a frame, u[i], v[i] (device float32 planes) receive the flow
 * from its previous frame to frames[i] and has_flow[i] = 1; for a session's first frame only
 * its pyramid is built, u[i], v[i] are not touched (may be NULL) and has_flow[i] = 0.
 * frames[i] may be reused by the caller once the push's work on `stream` has completed.
 * Errors (nothing enqueued): OF_EINVAL for NULL arguments, a session of another server or a
 * session listed twice; OF_ESTATE when every staging slot is held by a push still in flight;
 * OF_EHIP on launch failure. */
OF_API of_status of_server_push(of_server* s, of_session* const* sessions, int n,
                                const void* const* frames, float* const* u, float* const* v,
                                int* has_flow, void* stream);

/* Sessions without an explicit server (the hot-path boundary's session entry points): the
 * session joins a library-held server of its parameter set on the current device (no budget;
 * retired with its last session).  workspace as in of_server_open_ex (NULL = the library
 * allocates).  Returns NULL on invalid parameters or allocation failure. */
OF_API of_session* of_session_create(int H, int W, int levels, int radius, int iters,
                                     unsigned flags, void* workspace, size_t workspace_bytes);

/* Region-of-interest mask of one stream (as of_plan_set_mask; Sec. 3.3): `mask` is a DEVICE
 * H x W uint8 plane of the session's size (nonzero = compute), NULL removes it.  Every later
 * push computes that session's flow with the mask: masked pixels get zero flow, tiles without
 * an unmasked pixel are left out of every iteration launch (the last iteration writes their
 * zero flow); equal to a plan with the same mask, bitwise.  Set-up call: waits for the device,
 * allocates the mask pyramid, tile flags and four FP32 flow planes per level >= 1 (freed with
 * the session) and clears the session's flow planes.
 * Errors: OF_EINVAL (NULL session), OF_EHIP. */
OF_API of_status of_session_set_mask(of_session* session, const uint8_t* mask, void* stream);

/* of_server_push for one session. */
OF_API of_status of_session_push(of_session* session, const void* frame, float* u, float* v,
                                 void* stream, int* has_flow);

/* Continuous batching over sessions: of_server_push of n sessions, which must all belong to
 * one server (the one of sessions[0]; sessions from of_session_create with equal parameters
 * on one device share one). */
OF_API of_status of_session_push_many(of_session* const* sessions, int n,
                                      const void* const* frames, float* const* u,
                                      float* const* v, int* has_flow, void* stream);

/* Resident bytes of one session / of all open sessions of a server. */
OF_API size_t of_session_resident_bytes(const of_session* session);
OF_API size_t of_server_resident_bytes(const of_server* s);

/* Closes one session of server s (synchronises the device, frees library-allocated session
 * memory, returns its budget). */
OF_API of_status of_server_close(of_server* s, of_session* session);

/* Closes a session (of either kind; as of_server_close).  NULL-safe. */
OF_API void of_session_destroy(of_session* session);

/* Destroys the server and every session still open.  NULL-safe; a no-op for the
 * library-held servers of of_session_create. */
OF_API void of_server_destroy(of_server* s);

/* --------------------------------------------------------------------- around the flow
 * Local equalisation of a raw frame (Sec. 2.4, eq. 2; the printed denominator is the root of
 * minus the variance, while the text divides by the local standard deviation, as here):
 * out = (in - m) / (sd + eps), m and sd the mean and standard deviation of `in` over the
 * (2r+1)^2 window truncated at the border (in-image pixels only), accumulated in FP64.
 * in: H x W uint8 (float32 with OF_FLAG_INPUT_F32) device plane; out: H x W float32 device
 * plane, distinct from in.  0 <= radius <= OF_MAX_NORMALIZE_RADIUS, eps >= 0.
 * Errors: OF_EINVAL on bad arguments (nothing enqueued). */
OF_API of_status of_normalize(const void* in, float* out, int H, int W, int radius, float eps,
                              unsigned flags, void* stream);

/* Field statistics for the recirculation-bubble surface (Sec. 3.2, eq. 3; denominator read
 * as the number of vectors, as the text says).  All pointers are device pointers.
 *   of_field_mean_update: mean <- mean + (x - mean) / (t + 1) over n elements (the mean of
 *     t + 1 fields from the mean of the first t).
 *   of_field_minmax: out2[0] = min x, out2[1] = max x; `work` is a caller-owned device
 *     scratch of 2 unsigned ints.
 *   of_count_at_most: *count (device uint64) = number of x[i] <= threshold.
 * The bubble surface is count / n with threshold (min + max) / 2 of the mean field. */
OF_API of_status of_field_mean_update(float* mean, const float* x, long long n, int t,
                                      void* stream);
OF_API of_status of_field_minmax(const float* x, long long n, float* out2, void* work,
                                 void* stream);
OF_API of_status of_count_at_most(const float* x, long long n, float threshold,
                                  unsigned long long* count, void* stream);

/* The bubble surface of a sequence of fields on the device, with no host read (Sec. 3.2,
 * eq. 3, for the real-time loop that feeds S_bubble to flow control).  The mean field is the
 * running time-mean of the fields so far; field t is thresholded with T_v = (min + max) / 2
 * of the mean of the fields before it (field 0 with its own).
 *   of_plan_set_bubble: device pointers to the threshold T_v (float) and a count (uint64);
 *     while set, every of_compute clears *count and its final iteration adds the number of
 *     level-0 u values <= *threshold it writes (a wave sum and one atomic per wave: no pass of
 *     its own).  NULL, NULL removes it.  Drops the plan's captured graphs.
 *   of_bubble_step, after field t of H x W = n vectors has been computed into u: *surface =
 *     S_bubble(t) (for t >= 1 from *count; for t = 0 counted here against field 0's own
 *     threshold), then mean <- mean + (u - mean) / (t + 1) (t = 0: mean <- u) and *threshold
 *     <- (min + max) / 2 of the new mean, ready for field t + 1.  work: device scratch of 2
 *     unsigned ints (caller-owned, reset by every call).  All pointers are device pointers;
 *     nothing is read back to the host.
 * Errors: OF_EINVAL on NULL or misaligned pointers, n < 1 or t < 0. */
OF_API of_status of_plan_set_bubble(of_plan* plan, const float* threshold,
                                    unsigned long long* count);
OF_API of_status of_bubble_step(float* mean, const float* u, long long n, int t,
                                unsigned long long* count, float* threshold, float* surface,
                                void* work, void* stream);

/* --------------------------------------------------------------------- stage entry points
 * One step of the method on caller buffers, for stage-by-stage checking.
 *   OF_STAGE_REDUCE:  one pyramid reduction (Sec. 2.4, factor 4 in area): in[0] is a level-`level`
 *     plane of the plan's frame 1 geometry (uint8 / float32 at level 0, per flags; float32 or
 *     FP16 above), out[0] receives the level-(level+1) plane (float32, or FP16 with
 *     OF_FLAG_FP16_STORAGE).
 *   OF_STAGE_ITERATE: one Gauss-Newton iteration at level `level`: in = {I1_l, I2_l, u, v},
 *     out = {u_new, v_new}; frames typed as for that level, fields float32 of the level size.
 * Errors: OF_EINVAL on a bad stage, level or NULL pointer. */
#define OF_STAGE_REDUCE 0
#define OF_STAGE_ITERATE 1
OF_API of_status of_debug_stage(of_plan* plan, int stage, int level, const void* const* in,
                                void* const* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* OFMI_H */
