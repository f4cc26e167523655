/*
 * rxgs.h -- C ABI of the MI355X multi-receiver Gaussian rasterizer.
 *
 * The library renders, for a batch of receivers, the spectrum that a set of
 * frozen 3-D Gaussians produces on an angular (azimuth x elevation) grid, as
 * RxGS (arXiv 2605.24290) defines it: Alg. 1 ("Multi-Receiver Spectrum
 * Rendering for One Transmitter") with its three stages -- projection and a
 * depth sort over (tile, depth) keys shared by the receivers of a view, one
 * batched radiance evaluation per (receiver, Gaussian), and front-to-back
 * alpha compositing per (tile, receiver) -- plus the backward pass of
 * App. D ("the backward kernel runs with the same gridDim.z = N") and a
 * continuous-batching server.
 *
 * Conventions shared by every entry point:
 *   - All functions return rxgs_status; no C++ exception crosses the ABI.
 *     On failure rxgs_last_error(ctx) returns a message valid until the next
 *     call on that context.
 *   - "device" pointers are HIP device memory on the context's device, owned
 *     by the caller; "host" pointers are ordinary host memory.
 *   - Work is enqueued on the caller's HIP stream (a hipStream_t passed as
 *     void*, NULL = the null stream).  rxgs_render waits once, after the
 *     projection, to size its buffers; every other device step is
 *     asynchronous.  Outputs are valid once the stream reaches that point.
 *   - A context is used by one host thread at a time; the server's submit,
 *     poll and cancel calls are thread-safe.
 *   - Arrays are row-major FP32 unless stated.
 *
 * Angular grid: row i is centred at elevation el0 + (i + 1/2) del_el,
 * column c at azimuth (c + 1/2) 2 pi / W, azimuth atan2(y, x) in [0, 2 pi)
 * and elevation measured from the horizontal plane (+z up).  The paper's
 * spatial-spectrum grid is 360 x 90 at 1 degree (App. E, Table 4).
 */
#ifndef RXGS_H
#define RXGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RXGS_OK = 0,
    RXGS_E_INVALID = 1,    /* bad argument: null pointer, size, non-finite value */
    RXGS_E_OOM = 2,        /* device or pinned host allocation failed */
    RXGS_E_DEVICE = 3,     /* a HIP call failed; the context should be destroyed */
    RXGS_E_STATE = 4,      /* call out of order (no scene, no MLP, stale saved state) */
    RXGS_E_BUSY = 5,       /* server queue full */
    RXGS_E_TIMEOUT = 6,    /* poll timed out; the ticket is still pending */
    RXGS_E_CANCELLED = 7   /* ticket was cancelled */
} rxgs_status;

typedef struct rxgs_ctx rxgs_ctx;
typedef struct rxgs_saved rxgs_saved;
typedef struct rxgs_server rxgs_server;

typedef struct {
    int32_t H;        /* rows (elevation), >= 1 */
    int32_t W;        /* columns (azimuth), >= 2, even */
    int32_t reserved; /* must be 0 */
    double el0;       /* elevation of the lower edge of row 0, radians */
    double del_el;    /* row pitch, radians (> 0) */
} rxgs_grid;

/* View modes.  TX: each transmitter is one view centred at it, shared by its
 * receivers (Alg. 1 stage 1 "computed once"; App. D "Transmitter-Side
 * Preprocessing").  RX: each receiver is its own view centred at its
 * position; keys are then (receiver, tile, depth). */
enum { RXGS_MODE_TX = 0, RXGS_MODE_RX = 1 };

/* Number of MLP parameters: W1 (64 x 68), b1 (64), W2 (64 x 64), b2 (64),
 * W3 (2 x 64), b3 (2), concatenated in that order, each row-major (out x in). */
#define RXGS_MLP_NPARAM 8706
#define RXGS_FEAT_DIM 32
#define RXGS_TILE 16

/* Create a context on HIP device `device` for one angular grid.  Its device
 * buffers come from hipMalloc.  Grids of at most 255 tiles place each tile
 * pair in its depth-ordered tile list directly; larger grids, or any grid
 * when the environment variable RXGS_PAIR_SORT=1 is set at creation, emit the
 * pairs in depth order and sort them stably by tile (the same lists).
 * Errors: E_INVALID (grid), E_DEVICE. */
rxgs_status rxgs_create(int device, const rxgs_grid *grid, rxgs_ctx **out);

/* Caller-supplied device allocator (e.g. a framework's caching allocator).
 * alloc returns `bytes` of device memory on `device` (256-byte aligned), or
 * NULL on failure (the library then reports E_OOM); free returns a block
 * with the size it was allocated with.  Both may be called from the thread
 * that calls into the context and from a server's worker thread.  Before
 * handing a block back the library waits until no queued device work uses
 * it (a device synchronisation), so a block may be reused on any stream. */
typedef void *(*rxgs_alloc_fn)(size_t bytes, int device, void *user);
typedef void (*rxgs_free_fn)(void *ptr, size_t bytes, int device, void *user);

/* rxgs_create whose every device buffer (scene, MLP, workspaces, saved
 * states, server slots) comes from alloc / free (both non-NULL); `user` is
 * passed through.  Pinned host staging still comes from hipHostMalloc.
 * Errors: those of rxgs_create, E_INVALID (NULL callback). */
rxgs_status rxgs_create_with_allocator(int device, const rxgs_grid *grid, rxgs_alloc_fn alloc,
                                       rxgs_free_fn free_fn, void *user, rxgs_ctx **out);

/* Destroy a context, its scene, MLP and internal workspaces.  Saved states
 * created from it must be destroyed first.  NULL is ignored. */
void rxgs_destroy(rxgs_ctx *ctx);

/* Last error message of the context ("" when none).  NULL ctx: the message
 * of the last failed rxgs_create on this thread. */
const char *rxgs_last_error(const rxgs_ctx *ctx);

/*
 * Upload the Gaussian scene (Sec. 2 eq. (1); App. E.1): K Gaussians with
 * means (K x 3, metres), log-space scales (K x 3), rotation quaternions
 * (K x 4, (w, x, y, z), normalised inside the renderer) and opacity logits
 * (K; opacity = sigmoid(logit)).  Radiance is either direct, radiance
 * (K x 2, Re/Im, the same for every receiver), or per-Gaussian features
 * (K x 32) fed to the conditioning MLP; at most one of the two is non-NULL.
 * With both NULL the scene is geometry only: rxgs_render refuses it
 * (E_STATE) unless K = 0, and rxgs_render_rxcond takes its radiance from a
 * conditioning model (rxgs_rxcond_upload).
 * The library copies everything into its own device buffers (the scene stays
 * resident for serving).  src_on_device: 1 if the pointers are device memory,
 * 0 for host memory.  Validates that every value is finite (E_INVALID).
 * K may be 0.  Invalidates earlier saved states (E_STATE on their backward).
 */
rxgs_status rxgs_scene_upload(rxgs_ctx *ctx, int64_t K, const float *means, const float *log_scales,
                              const float *quats, const float *logits, const float *radiance,
                              const float *features, int src_on_device, void *stream);

/*
 * Upload the receiver-conditioning MLP (RXGS_MLP_NPARAM floats, layout
 * above).  Its input is [gamma(r); f_k] where gamma(r)[12 d + 2 f] =
 * sin(2^f r_d) and gamma(r)[12 d + 2 f + 1] = cos(2^f r_d), d in {x, y, z},
 * f = 0..5 (the Fourier receiver encoding of Sec. 4.3.2 eq. rx_enc with the
 * 6 bands of App. E Table 4); hidden layers ReLU; output (Re, Im).
 * Layer 1 is evaluated as W1[:, :36] gamma(r_j) once per receiver plus
 * W1[:, 36:] f_k + b1 once per Gaussian (the global and local branches).
 * Layer 2, per (receiver, Gaussian), runs on FP16 matrix cores in split
 * precision (each FP32 operand as an FP16 (hi, lo) pair, three products
 * accumulated in FP32; relative error near 2^-21 per product) after an exact
 * power-of-two rescaling of W2 and, when the layer-1 activations exceed
 * 2^15, of the activations.  If that rescaling cannot be exact for the given
 * weights, or the environment variable RXGS_MLP_FP32=1 is set at upload,
 * layer 2 runs on FP32 matrix cores instead.
 */
rxgs_status rxgs_mlp_upload(rxgs_ctx *ctx, const float *params, int src_on_device, void *stream);

/* Saved forward state for the backward pass.  Buffers grow on demand and are
 * kept until rxgs_saved_destroy. */
rxgs_status rxgs_saved_create(rxgs_ctx *ctx, rxgs_saved **out);
void rxgs_saved_destroy(rxgs_saved *s);

/*
 * Render N receivers in one pass (Alg. 1; Sec. 4.4).
 *   mode    RXGS_MODE_TX or RXGS_MODE_RX.
 *   Q, tx   TX mode: Q >= 1 transmitters, tx device Q x 3; receivers
 *           rx_off[q] .. rx_off[q+1]-1 use transmitter q.  RX mode: tx and
 *           rx_off are ignored (may be NULL) and Q is ignored.
 *   rx_off  host, Q + 1 non-decreasing offsets, rx_off[0] = 0, rx_off[Q] = N.
 *   N, rx   N >= 0 receivers, device N x 3 (metres).
 *   C       device N x 2 x H x W output spectrum (Re plane, then Im plane).
 *   power   device N output, received power sum_p |C_p|^2 (App. A Def. 2
 *           aggregates over rays; here over the grid's pixels), or NULL.
 *   csum    device N x 2 output, coherent sum sum_p C_p, or NULL.
 *   amp     device N x H x W output amplitude sqrt(Re^2 + Im^2 + 1e-8) of every
 *           pixel (App. E.2, the stabilised |R|), or NULL.
 *   saved   state for rxgs_render_backward, or NULL (an internal workspace is
 *           used and nothing is kept).
 * Compositing per pixel (Alg. 1 stage 3): Gaussians of the view in ascending
 * (FP32 squared distance to the view centre, index) order; w = min(0.99,
 * o exp(-q/2)) with q the Mahalanobis distance of the pixel under the
 * projected covariance (+0.3 px^2); skipped when w < 1/255; C += T w s;
 * T <- T (1 - w); stop after the Gaussian that takes T below 1e-4.
 * Gaussians closer than 0.2 m to the view centre are culled.
 * Errors: E_INVALID, E_STATE (no scene, or MLP scene without an MLP), E_OOM,
 * E_DEVICE.  The call synchronises the stream once.
 */
rxgs_status rxgs_render(rxgs_ctx *ctx, int mode, int Q, const float *tx, const int32_t *rx_off,
                        int N, const float *rx, float *C, float *power, float *csum, float *amp,
                        rxgs_saved *saved, void *stream);

/*
 * rxgs_render for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments without a saved state, the same kernels and results, and no
 * device or host allocation in the call.  Its workspace is carved, in order,
 * from a static device array of RXGS_NOALLOC_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends (resolved per device by
 * rxgs_create, which also makes the call's pinned staging); the region is
 * rewound at every call.  Every context on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams, other threads, other
 * contexts) race; calls on one stream are ordered.  A render whose buffers
 * exceed the array fails with E_OOM ("scratch region exhausted") before any
 * output is written (work it had enqueued touched only the array).  The call
 * synchronises the stream once, like rxgs_render.  Errors: those of
 * rxgs_render; E_STATE if the context has no such workspace.
 */
#define RXGS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
rxgs_status rxgs_render_noalloc(rxgs_ctx *ctx, int mode, int Q, const float *tx, const int32_t *rx_off, int N,
                                const float *rx, float *C, float *power, float *csum, float *amp, void *stream);

/*
 * Coverage-map render: the receivers of rxgs_render (same arguments, no saved
 * state) streamed through consecutive chunks, each one rxgs_render call, the
 * largest whose workspace estimate (rxgs_workspace_estimate) fits
 * budget_bytes; budget_bytes <= 0 takes half the device memory free at the
 * call.  A chunk may split one transmitter's receivers (its view is then
 * projected and sorted once per chunk).  Every receiver's outputs are those
 * of rxgs_render up to the summation order of its blend workgroup (a chunk
 * of one receiver per view uses the one-receiver kernel).  The library's
 * internal workspace keeps the largest chunk's buffers until rxgs_destroy.
 * Writes the number of chunks to *n_chunks when it is not NULL.  Errors:
 * those of rxgs_render, and E_OOM when one receiver does not fit the budget.
 */
rxgs_status rxgs_render_chunked(rxgs_ctx *ctx, int mode, int Q, const float *tx, const int32_t *rx_off,
                                int N, const float *rx, float *C, float *power, float *csum, float *amp,
                                int64_t budget_bytes, int32_t *n_chunks, void *stream);

/* Gradient outputs of rxgs_render_backward (device pointers, caller-owned).
 * Any may be NULL to skip it; radiance is used for direct radiance scenes,
 * features and mlp for MLP scenes.  accumulate = 0: the outputs are
 * overwritten; 1: this backward's gradients are added to their contents (a
 * loss summed over several renders, e.g. several transmitters). */
typedef struct {
    float *means;        /* K x 3 */
    float *log_scales;   /* K x 3 */
    float *quats;        /* K x 4, gradient w.r.t. the raw (unnormalised) quaternion */
    float *logits;       /* K */
    float *radiance;     /* K x 2 */
    float *features;     /* K x 32 */
    float *mlp;          /* RXGS_MLP_NPARAM */
    int32_t accumulate;  /* 0 overwrite, 1 add */
} rxgs_grads;

/*
 * Backward pass of the last rxgs_render into `saved` (App. D: per-receiver
 * dL/ds, Gaussian-level gradients accumulated over receivers and pixels).
 *   C    device N x 2 x H x W, the forward's output (used for dL/dP and dL/damp).
 *   dC   device N x 2 x H x W, dL/dC, or NULL (zero).
 *   dP   device N, dL/dpower, or NULL.
 *   dA   device N x H x W, dL/damp for the amplitude output, or NULL.
 * Gradients flow through w = o exp(-q/2) when it is not clamped at 0.99, the
 * projected mean and covariance, the quaternion normalisation and the MLP
 * (ReLU derivative 0 at 0).  Float atomics make results vary in the last
 * bits from run to run.  Errors: E_INVALID, E_STATE, E_OOM, E_DEVICE.
 */
rxgs_status rxgs_render_backward(rxgs_ctx *ctx, const rxgs_saved *saved, const float *C,
                                 const float *dC, const float *dP, const float *dA,
                                 const rxgs_grads *grads, void *stream);

/* Sizes of a saved forward state. */
typedef struct {
    int64_t K;          /* Gaussians */
    int64_t K_pad;      /* per-view stride of record arrays (multiple of 4096) */
    int64_t V;          /* views */
    int64_t N;          /* receivers */
    int64_t D;          /* (view, tile, Gaussian) pairs */
    int64_t n_visible;  /* sum over views of Gaussians with a non-empty tile set */
    int64_t tiles;      /* tiles per view */
    int64_t tiles_x;    /* tile columns */
    int64_t n_composited_px;  /* (pixel, Gaussian) weights composited, counted once per
                                 receiver chunk that shares them (TX mode: up to 16
                                 receivers of a view share one weight evaluation) */
    int64_t n_composited;     /* the same counted once per receiver */
    int64_t n_evaluated_px;   /* (pixel, list entry) weights evaluated while the pixel was
                                 still compositing, once per receiver chunk */
    int64_t n_walked_px;      /* (pixel, list entry) slots walked by the waves (64 per
                                 entry and wave, terminated lanes included) */
    int64_t n_sort_fallbacks; /* radix-sort tiles (depth and pair sorts) whose bounded
                                 look-back wait expired and that counted the digits of
                                 their segment's earlier tiles directly instead (exact;
                                 normally 0) */
    int64_t workspace_bytes;  /* device bytes the render's workspace buffers asked for
                                 (what rxgs_workspace_estimate bounds, outputs aside) */
} rxgs_saved_info_t;

rxgs_status rxgs_saved_info(const rxgs_saved *s, rxgs_saved_info_t *out);

/* Copy an internal array of a saved state to a caller device or host buffer
 * (hipMemcpy semantics: the copy completes before return).  `what`:
 *   RXGS_EXPORT_BIN       V x K_pad x 4 f32: u, v, padded half-extents rup, rvp
 *   RXGS_EXPORT_KEYS      V x K_pad u32: FP32 depth-key bits (0xFFFFFFFF if culled)
 *   RXGS_EXPORT_OPACITY   V x K_pad f32: opacity used for culling
 *   RXGS_EXPORT_ORDER     V x K_pad i32: Gaussian index at each sorted position
 *                         s < NVIS[v] (later positions are undefined)
 *   RXGS_EXPORT_NVIS      V i32: visible Gaussians per view
 *   RXGS_EXPORT_PAIRS     D i32: sorted position (v * K_pad + s) of each pair
 *   RXGS_EXPORT_RANGES    V x tiles x 2 i32: [start, end) of each tile's pairs
 *   RXGS_EXPORT_RADIANCE  N x K_pad x 2 f32: radiance at each sorted position
 *                         s < NVIS[view of the receiver] (a render that evaluated
 *                         only the radiance its blend needed, see
 *                         rxgs_view_flags, evaluates the rest first, on the device)
 *   RXGS_EXPORT_TFINAL    S x H x W f32: final transmittance (S = V in TX mode, N in RX)
 *   RXGS_EXPORT_NLAST     S x H x W i32: entries of the tile list consumed
 *   RXGS_EXPORT_RECORDS   V x K_pad x 8 f32: the blend record at each sorted position
 *                         s < NVIS[v] (Alg. 1 stage 1 output): floor u, u - floor u,
 *                         floor v, v - floor v, then -log2(e)/2 a, -log2(e) b,
 *                         -log2(e)/2 c (the conic, inverse of the projected
 *                         covariance) and log2 o
 * `bytes` must be at least the size above; E_INVALID otherwise. */
enum {
    RXGS_EXPORT_BIN = 0, RXGS_EXPORT_KEYS = 1, RXGS_EXPORT_OPACITY = 2, RXGS_EXPORT_ORDER = 3,
    RXGS_EXPORT_NVIS = 4, RXGS_EXPORT_PAIRS = 5, RXGS_EXPORT_RANGES = 6,
    RXGS_EXPORT_RADIANCE = 7, RXGS_EXPORT_TFINAL = 8, RXGS_EXPORT_NLAST = 9, RXGS_EXPORT_RECORDS = 10
};
rxgs_status rxgs_saved_export(const rxgs_saved *s, int what, void *dst, int64_t bytes, int dst_on_device);

/*
 * Serving: a persistent request loop on one context (the use the paper
 * motivates with coverage maps, App. G.3 "Asymptotic scaling").  Each query is
 * one transmitter and n receivers; queries are rendered by a worker thread in
 * batches (several queries, each its own view in TX mode, fused into one
 * render) on `slots` HIP streams, so a batch is formed whenever a slot frees
 * up, from whatever has arrived (continuous batching), and batches on
 * different slots overlap on the device.  A batch takes queued queries in
 * arrival order while the receiver count, the query count and the estimated
 * device workspace stay within the limits; a query that alone exceeds them is
 * rejected at submit.  While a server runs, the context's scene and MLP must
 * not change and the context must not render from other threads.
 */
typedef struct {
    int64_t mem_budget_bytes;  /* device workspace for all slots; 0 = half of the free memory */
    int32_t max_rx_per_batch;  /* receivers fused into one render (>= 1) */
    int32_t max_queries_per_batch;
    int32_t slots;             /* batches in flight, 1..8 */
    int32_t mode;              /* RXGS_MODE_TX or RXGS_MODE_RX */
    int32_t queue_capacity;    /* queued queries; submit returns E_BUSY beyond */
    int32_t want_spectra;      /* 1: results include the N x 2 x H x W spectra */
} rxgs_server_opts;

typedef struct {
    double t_submit;           /* seconds, host monotonic clock */
    double t_start;            /* batch launched (the last attempt's) */
    double t_done;             /* results copied to host */
    int32_t batch_queries;     /* queries in the batch that carried it */
    int32_t batch_receivers;
    int32_t attempts;          /* batches that carried it (2: replayed once after a failed batch) */
    int32_t reserved;
} rxgs_ticket_info;

typedef struct {
    int64_t submitted, completed, cancelled, rejected, failed, batches, receivers;
    int64_t queued, in_flight;
    double busy_s;             /* summed wall time of batches on the device */
    int64_t failed_batches;    /* batches whose launch or device work failed */
    int64_t replayed;          /* tickets queued again after their batch failed */
    int64_t peak_slot_bytes;   /* largest device workspace one batch used (buffers it asked for) */
    int64_t over_estimate;     /* batches whose workspace exceeded the admission estimate */
} rxgs_server_stats_t;

/* Start the worker on a context with an uploaded scene (and MLP).  A batch
 * whose launch fails (e.g. the allocator returns NULL: E_OOM) or whose device
 * work reports an error has its slot reset (stream, event and workspace made
 * again) and its tickets queued again at the front, once; a ticket whose
 * second batch fails too is retired with that batch's status.  Other tickets
 * and the worker carry on.
 * Errors: E_INVALID (options), E_STATE (no scene / MLP), E_OOM, E_DEVICE. */
rxgs_status rxgs_server_start(rxgs_ctx *ctx, const rxgs_server_opts *opts, rxgs_server **out);

/* The same scheduler (admission, continuous batching, retirement, replay)
 * against a host-only executor instead of the GPU, for tests of the serving
 * logic without a device: a batch "renders" power_j = tx.x + r_j.x + 2 r_j.y +
 * 3 r_j.z for each of its receivers after delay_us microseconds; the launch
 * with index i (0-based, counting every launch) fails with E_OOM when
 * fail_launch_mask has bit i set (i < 64), and its work reports a device error
 * when fail_device_mask has bit i set.  K, H and W feed the admission estimate.
 * want_spectra must be 0. */
typedef struct {
    int64_t K;
    int32_t H, W;
    int32_t delay_us;
    int32_t reserved;
    uint64_t fail_launch_mask;
    uint64_t fail_device_mask;
} rxgs_host_executor;
rxgs_status rxgs_server_start_host(const rxgs_server_opts *opts, const rxgs_host_executor *exec,
                                   rxgs_server **out);
/* Queue one query: tx host 3 floats, rx_host n x 3 floats (copied).  Returns
 * a ticket.  Errors: E_INVALID (n < 1, n > max_rx_per_batch, non-finite,
 * workspace estimate above the per-slot budget), E_BUSY (queue full), E_STATE (stopped). */
rxgs_status rxgs_server_submit(rxgs_server *srv, const float *tx, int32_t n, const float *rx_host,
                               uint64_t *ticket);
/* Wait up to timeout_ms (< 0: forever) for a ticket; on success copy power
 * (n floats) and, if the server keeps spectra and C_host is not NULL, the
 * n x 2 x H x W spectra, fill info (may be NULL) and retire the ticket.
 * Errors: E_TIMEOUT (still pending), E_CANCELLED, E_INVALID (unknown ticket),
 * E_OOM or E_DEVICE (its batch failed twice; info is still filled). */
rxgs_status rxgs_server_poll(rxgs_server *srv, uint64_t ticket, float *power_host, float *C_host,
                             rxgs_ticket_info *info, int32_t timeout_ms);
/* Cancel a queued ticket (a ticket already on the device completes). */
rxgs_status rxgs_server_cancel(rxgs_server *srv, uint64_t ticket);
rxgs_status rxgs_server_stats(rxgs_server *srv, rxgs_server_stats_t *out);
/* Finish in-flight batches, cancel queued tickets, join the worker, free. */
rxgs_status rxgs_server_stop(rxgs_server *srv);

/*
 * Batch planning rule of the server, as a host function: given the receiver
 * counts of the queued queries in arrival order, return how many of them
 * (a prefix) the next batch takes and its workspace estimate.  Pure host
 * logic, no device access.
 */
int32_t rxgs_plan_batch(const int32_t *n_rx, int32_t n_queued, int32_t mode, int64_t K, int32_t H, int32_t W,
                        int64_t budget_bytes, int32_t max_rx, int32_t max_queries, int64_t *bytes_out);
/*
 * Device bytes of one render of Q queries and N receivers (mode, K Gaussians,
 * H x W grid): an upper bound of the sum of the render's workspace requests
 * (rxgs_saved_info.workspace_bytes) plus its inputs and outputs, given at most
 * RXGS_EST_PAIRS_PER_GAUSSIAN tile pairs per (view, Gaussian) on average,
 * the one term that depends on the scene (a Gaussian covers more tiles the
 * nearer it is to the view centre).  The server starts from that ratio and
 * raises it to 1.25 x the largest one a render has shown.
 */
#define RXGS_EST_PAIRS_PER_GAUSSIAN 8.0
int64_t rxgs_workspace_estimate(int32_t mode, int32_t Q, int32_t N, int64_t K, int32_t H, int32_t W);

/*
 * Stage timing.  While enabled, every pipeline stage of rxgs_render and
 * rxgs_render_backward is bracketed by HIP events recorded on the caller's
 * stream; rxgs_profile_read synchronises on them and returns, per stage,
 * the number of launches and the summed event-to-event time (ms).  Stage
 * names: project, sort_depth, emit_records, mlp_global, emit_pairs,
 * sort_pairs, ranges, mlp_items, blend_weights, mlp_local, mlp_pairs,
 * rad_direct, blend_fwd, reduce, redo_views (one launch per view redone over
 * all its entries, see rxgs_set_near_cut; the redone passes' own stages are
 * counted under their names), and the backward stages blend_bwd, mlp_bwd,
 * project_bwd, bwd_misc.  `reset` clears the totals after reading.  Errors:
 * E_INVALID, E_DEVICE.
 */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
} rxgs_stage_time;

rxgs_status rxgs_profile_enable(rxgs_ctx *ctx, int on);
rxgs_status rxgs_profile_read(rxgs_ctx *ctx, rxgs_stage_time *out, int max_entries, int *n_entries, int reset);

/*
 * Work counts of the profiled renders, counted on the device from the work
 * lists the kernels consume (Alg. 1 stage 2: the radiance of each receiver
 * at each sorted position): while profiling is enabled, every launch of the
 * pair MLP (or of the conditioned radiance) is followed by a small kernel that
 * adds up its work items.  mlp_items: work items evaluated (one view, 32
 * sorted positions, up to 16 receivers); mlp_pairs: (receiver, position)
 * radiance values evaluated; mlp_slots: (receiver, position slot) pairs the
 * matrix cores process, 32 per (work item, receiver), padding included.
 * The counts are read on `stream` (the renders' stream; the call waits for
 * it); `reset` clears them after reading.  Errors: E_INVALID, E_DEVICE.
 */
typedef struct {
    int64_t mlp_items;
    int64_t mlp_pairs;
    int64_t mlp_slots;
} rxgs_work_counts;

rxgs_status rxgs_profile_counts(rxgs_ctx *ctx, rxgs_work_counts *out, int reset, void *stream);

/*
 * Nearest-first emission (off by default).  Compositing stops at a pixel once
 * its transmittance falls below 1e-4 (Alg. 1, early termination), so where
 * every ray ends inside the scene a view's spectra depend only on its nearest
 * Gaussians.  With this on and more than 4096 Gaussians in the scene,
 * rxgs_render emits per view only its 4096 nearest depth-sorted entries,
 * then checks (one device-to-host copy and a stream synchronisation at the
 * end of the call) whether some pixel of a cut view stayed open; such views
 * are redone over all their entries (each alone without saved state, the
 * whole call again with it).  Results, and saved states, are the same as
 * with it off.  It pays only when views rarely keep an open pixel: a ray that
 * leaves the scene keeps its pixel open and forces the redo.  Errors:
 * E_INVALID (NULL ctx).
 */
rxgs_status rxgs_set_near_cut(rxgs_ctx *ctx, int on);

/*
 * Deterministic backward (off by default; on at rxgs_create when the
 * environment variable RXGS_DETERMINISTIC=1).  While on, renders into a saved
 * state evaluate every visible position's radiance (no radiance prefix), and
 * rxgs_render_backward on such a state sums every gradient in a fixed order
 * instead of with float atomics (App. D accumulates with atomicAdd): the
 * blend backward stores one partial per (pair, block of up to 4 receivers) at
 * the pair's emission slot, summing its waves in order, and gathers add them
 * per (view, position) and per (row, position) in emission order; the MLP
 * backward stores its per-Gaussian and per-receiver terms per marked position
 * block and gathers add them in view and block order; the projection
 * gradients of each Gaussian are summed over the views in order (FP64).  Two
 * backwards of the same inputs then give the same bits.  It needs about
 * (6 + 2 R_max) x 4 B per pair slot and 4 B per (view, Gaussian) more device
 * memory and one host wait.  Errors: E_INVALID (NULL ctx).
 */
rxgs_status rxgs_set_deterministic(rxgs_ctx *ctx, int on);

/* Views redone over all their entries since the context was created, or -1
 * for a NULL ctx. */
int64_t rxgs_views_redone(const rxgs_ctx *ctx);

/*
 * Per-view flags of the last rxgs_render (device-to-host copy, synchronous):
 * bit 0 the view's entries were cut (nearest-first emission; never with saved
 * state, which emits every entry), bit 1 a pixel stayed open after the cut;
 * with the radiance
 * prefix (the pair MLP first runs on each view's nearest sorted positions,
 * 4096 for TX views with fewer than 128 receivers, 8192 for RX views, when a
 * view has more visible), bit 3 some pixel composited a position past it
 * (those terms are added once their radiance exists) and bit 2 some pixel
 * composited more than 16 such positions (the view is blended again).  Copies
 * up to max_views words to out and writes the view count to *n_views when
 * not NULL.  Errors: E_INVALID, E_DEVICE.
 */
rxgs_status rxgs_view_flags(rxgs_ctx *ctx, uint32_t *out, int32_t max_views, int32_t *n_views);

/*
 * The paper's receiver-conditioned radiance (Sec. 4.3.2 eqs. rx_enc, film,
 * film_apply, transmittance, local, combined_local; App. E.2 and E.5; Alg. 1
 * stage 2).  Per Gaussian k a base coefficient phi_k[l][c] (complex) for each
 * basis component l = (deg, ord), index deg^2 + deg + ord, and channel c.
 * Per receiver j at r and Gaussian k at p, seen from the view centre c_v
 * along d = p - c_v:
 *   gamma(r) = [sin(w_i . r), cos(w_i . r)], i < 3F        (eq. rx_enc)
 *   (alpha_l, beta_l)[c] = MLP_g([gamma(r); deg/m, ord/m; e_l]),
 *       m = max(lmax, 1)                                    (eq. film)
 *   phi~ = (1 + alpha_l) phi_k + beta_l                    (eq. film_apply)
 *   q_s = p + t_s (r - p), t_s = 0.05 + 0.9 s / (S - 1); V(q) the occupancy of
 *   the voxel containing q (0 outside the grid); T = prod (1 - V(q_s)),
 *   rho = mean V(q_s)                                      (eq. transmittance)
 *   (alpha', beta')[c] = MLP_l([(r - p)/|r - p|; |r - p|; T; rho]), one pair
 *   per (receiver, Gaussian, channel) shared by all components (App. E.5:
 *   "per-Gaussian" scale and shift)                        (eq. local)
 *   s_c = sum_l ((1 + alpha') phi~_{l,c} + beta') B_l(d)   (eq. combined_local; App. E.2)
 * with complex products and B_l the basis: RXGS_BASIS_FLE the complex
 * Fourier-Legendre basis N_lm P_l^|m|(cos th) e^{i m ph} (App. E.2; N_lm the
 * orthonormal factor, P without the Condon-Shortley phase, th the polar angle
 * of d from +z, ph its azimuth); RXGS_BASIS_SH the real spherical harmonics
 * of the RF-3DGS backbone (Sec. 5): N P for m = 0, sqrt2 N P cos(m ph) for
 * m > 0, sqrt2 N P_l^|m| sin(|m| ph) for m < 0.  MLPs have three Linear
 * layers with ReLU after the first two (App. E.5).  The occupancy grid
 * (App. E.5) spans the box of the Gaussian means with G^3 voxels, voxel i at
 * lo + (i + 1/2)(hi - lo)/G per axis (an axis narrower than 1e-6 m gets
 * hi = lo + 1e-6), and holds V(x) = 1 - prod_k (1 - o_k exp(-|x - p_k|^2 /
 * (2 sigma_k^2))) over the Gaussians with |x - p_k| <= 2 sigma_k, o_k =
 * sigmoid(logit_k), sigma_k = the largest of its three scales.
 */
enum { RXGS_BASIS_FLE = 0, RXGS_BASIS_SH = 1 };
#define RXGS_RXCOND_EMB 16     /* component embedding width d_c (App. E Table 4) */
#define RXGS_RXCOND_HIDDEN 64  /* hidden width of both MLPs (Table 4: 64) */

typedef struct {
    int32_t basis;     /* RXGS_BASIS_FLE or RXGS_BASIS_SH */
    int32_t lmax;      /* largest degree, 0..12; L = (lmax + 1)^2 components */
    int32_t channels;  /* complex signal channels C, 1..32 (App. E.1: f in R^{L x C}) */
    int32_t bands;     /* Fourier bands F, 1..16: 3F frequency vectors */
    int32_t hidden;    /* must be RXGS_RXCOND_HIDDEN */
    int32_t probes;    /* occupancy probes S per (receiver, Gaussian), 2..64 */
    int32_t grid;      /* occupancy grid resolution G, 1..512 */
    int32_t reserved;  /* must be 0 */
} rxgs_rxcond_desc;

/* Number of conditioning parameters for a descriptor (-1 if invalid), in
 * this order, matrices row-major (out x in):
 *   w    3F x 3              Fourier frequency vectors w_i (eq. rx_enc)
 *   e    L x 16              component embeddings e_l
 *   global MLP  W1 (64 x (6F + 18)), b1 (64), W2 (64 x 64), b2 (64),
 *               W3 (4C x 64), b3 (4C); output row 4c + (alpha re, alpha im,
 *               beta re, beta im); input [gamma; deg/m, ord/m; e_l] with
 *               gamma[2i] = sin(w_i . r), gamma[2i + 1] = cos(w_i . r)
 *   local MLP   W1 (64 x 6), b1 (64), W2 (64 x 64), b2 (64), W3 (4C x 64),
 *               b3 (4C); output row 4c + (alpha' re, alpha' im, beta' re, beta' im) */
int64_t rxgs_rxcond_param_count(const rxgs_rxcond_desc *d);

/*
 * Upload a conditioning model for the current scene: coeffs K x L x C x 2
 * (Re, Im) base coefficients, params rxgs_rxcond_param_count floats.  Builds
 * the occupancy grid from the scene's means, log-scales and logits on the
 * device (once per upload: App. E.5 builds it once).  The call synchronises
 * the stream.  A later rxgs_scene_upload invalidates the model (E_STATE on
 * render until it is uploaded again).  Errors: E_INVALID (descriptor,
 * non-finite value), E_STATE (no scene), E_OOM, E_DEVICE.
 */
rxgs_status rxgs_rxcond_upload(rxgs_ctx *ctx, const rxgs_rxcond_desc *d, const float *coeffs,
                               const float *params, int src_on_device, void *stream);

/*
 * rxgs_render with the conditioned radiance above (Alg. 1 stages 2-3: every
 * (receiver, Gaussian) pair gets its coefficients modulated by both branches
 * and reduced against the basis of the view centre's direction, then each
 * channel is composited like a receiver of its own with the receiver's
 * weights).  Arguments as rxgs_render, with receiver-major channel rows:
 *   C      device N x C x 2 x H x W     power  device N x C, or NULL
 *   csum   device N x C x 2, or NULL   amp    device N x C x H x W, or NULL
 *   saved  state for rxgs_saved_export (its radiance rows are (receiver,
 *          channel)), or NULL; rxgs_render_backward refuses it (E_STATE).
 * Errors: those of rxgs_render; E_STATE without a current model.
 */
rxgs_status rxgs_render_rxcond(rxgs_ctx *ctx, int mode, int Q, const float *tx, const int32_t *rx_off, int N,
                               const float *rx, float *C, float *power, float *csum, float *amp,
                               rxgs_saved *saved, void *stream);

/* Copies of the model's derived arrays (synchronous):
 *   RXGS_RXCOND_OCCUPANCY  G^3 f32 occupancy values, x fastest
 *   RXGS_RXCOND_BOX        6 f64: lo[3], hi[3] of the grid
 * Errors: E_INVALID (kind, size), E_STATE (no model). */
enum { RXGS_RXCOND_OCCUPANCY = 0, RXGS_RXCOND_BOX = 1 };
rxgs_status rxgs_rxcond_export(rxgs_ctx *ctx, int what, void *dst, int64_t bytes, int dst_on_device);

/* Library version string. */
const char *rxgs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RXGS_H */
