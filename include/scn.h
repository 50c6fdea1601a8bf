/*
 * scn.h -- C ABI of libscn, a gfx950 (MI355X) implementation of the
 * data-parallel pixel stage that Scanner computation graphs run over frames
 * sampled from a video table (Poms et al., "Scanner: Efficient Video
 * Analysis at Scale", SIGGRAPH 2018).
 *
 * Concepts (paper Sec. 3):
 *   - a video is a table with one row per frame (Sec. 3, "Videos as logical
 *     tables"); here a table is a column of decoded NV12 frames resident in
 *     device memory;
 *   - sampling operations select rows by stride, index list or range
 *     (Sec. 3.2, "Sampling/spacing operations"); ranges also act as slices,
 *     boundaries that reset stencils (Sec. 3.2, "Slicing");
 *   - optical flow is a stencil S[0,1] operation (Sec. 3.2, "Stencil
 *     operations"), by default on the sampled sequence, i.e. between
 *     consecutive sampled rows of one slice, or on the original sequence
 *     before sampling (scn_sampling.stencil);
 *   - a job binds an operation to a table and its sampling (Sec. 3.1);
 *   - operations run over batches of elements (Sec. 3.3) and only the
 *     elements an output needs are ever read or computed (Sec. 4.2, unneeded
 *     element elimination);
 *   - scratch comes from a caller-owned memory pool (Sec. 4.1, custom GPU
 *     memory pools): no call allocates or frees device memory.
 *
 * Conventions shared by every entry point:
 *   - Every pointer named "device" is a HIP device pointer on the current
 *     device; "host" pointers are read before the call returns.
 *   - Every call is asynchronous on the given stream (a hipStream_t; NULL is
 *     the null stream).  Results are valid after the stream is synchronised.
 *   - Validation is complete before anything is enqueued.  On error nothing
 *     is enqueued, the status is negative and scn_last_error() explains why.
 *     HIP launch failures return SCN_EHIP; device faults surface at the
 *     caller's synchronisation.
 *   - Empty samplings (no rows, or no pairs for flow) return SCN_OK and
 *     enqueue nothing.
 *   - The caller owns every buffer.  `ws` is scratch device memory of
 *     `ws_bytes` bytes (size it with scn_workspace_bytes).  Every call made
 *     outside graph capture copies a small plan (row and pair tables) from
 *     host memory to the start of `ws`, ordered on its stream, so `ws` may
 *     hold anything between calls.  Calls that share one `ws` must be
 *     ordered on one stream (they overwrite each other's scratch).
 *   - HIP graph capture: a call made on a capturing stream records kernel
 *     launches only, no host-to-device copy.  It is accepted only if the last
 *     plan uploaded to the same `ws` (by an eager call) is exactly its own
 *     plan; otherwise it returns SCN_EINVAL with nothing recorded ("make the
 *     same call eagerly first").  The graph's kernels then read the plan
 *     that the workspace holds when the graph is replayed: between replays,
 *     do not run calls with a different plan on that `ws`, and do not write
 *     into its head, or re-run the eager call before replaying.
 *     scn_ws_forget(ws) drops the record of the last upload to `ws` (a later
 *     capture on it is refused until an eager call uploads again).
 */
#ifndef SCN_H
#define SCN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* scn_stream_t; /* hipStream_t */

typedef enum {
  SCN_OK = 0,
  SCN_EINVAL = -1,        /* an argument is invalid (null pointer, bad size, bad sampling) */
  SCN_EUNSUPPORTED = -2,  /* valid but not supported (odd width/height, too many levels) */
  SCN_ENOSPACE = -3,      /* ws_bytes is smaller than the minimum the call needs */
  SCN_EHIP = -4           /* a HIP runtime call failed */
} scn_status;

/* A video table: n_frames decoded NV12 uint8 frames in device memory.
 * Row f starts at frames + f * frame_bytes and holds the Y plane (height rows
 * of pitch bytes, the first width bytes used) followed by the interleaved
 * chroma plane (height/2 rows of pitch bytes: U0 V0 U1 V1 ...).
 * width and height are even and >= 2 and at most 32768; width <= pitch <=
 * 2^20; frame_bytes >= pitch * height * 3 / 2, and that Y + UV extent is at
 * most 2 GiB (kernels address a frame with 32-bit offsets).  Tables outside
 * these limits are refused with SCN_EUNSUPPORTED.
 * Only the rows a call reads are touched (its sampled rows, plus row s+1 of
 * each sampled row s with SCN_STENCIL_BEFORE), so only those rows need to be
 * backed by memory: a table may be a view of which a window of rows is
 * resident.  backed_count > 0 declares that only rows [backed_first,
 * backed_first + backed_count) are backed; every call then refuses with
 * SCN_EINVAL a job that would read another row.  backed_count == 0 (a
 * zero-initialised field) declares every row backed.  backed_first >= 0 and
 * backed_first + backed_count <= n_frames, else SCN_EINVAL. */
typedef struct {
  const uint8_t* frames; /* device */
  int32_t width, height, pitch, reserved;
  int64_t frame_bytes, n_frames;
  int64_t backed_first, backed_count;
} scn_table;

typedef enum { SCN_STRIDE = 0, SCN_GATHER = 1, SCN_RANGE = 2 } scn_sample_kind;

/* Sampling spec (paper Sec. 3.2; access patterns of Sec. 5.1.1).
 *   STRIDE: rows start, start+step, ... < stop (0 <= start <= stop <= n_frames, step >= 1).
 *   GATHER: idx holds n strictly increasing rows in [0, n_frames).
 *   RANGE:  idx holds n windows as 2n values begin_0, end_0, begin_1, ...;
 *           half-open, ascending and disjoint.  Each window is a slice:
 *           flow pairs never cross two windows.
 * idx is host memory. */
/* Where the S[0,1] stencil of FLOW sits relative to the sampling (Sec. 3.2,
 * composing stencils with sampling):
 *   SCN_STENCIL_AFTER (0): the stencil runs on the sampled sequence; pairs
 *     join consecutive sampled rows of one slice (flow at a low frame rate).
 *   SCN_STENCIL_BEFORE (1): the stencil runs on the original sequence and
 *     its outputs are sampled; each sampled row s gives the pair (s, s+1) of
 *     original rows (a sparse set of flow fields on original neighbours).  A
 *     sampled last row of the table gives no pair, and RANGE windows do not
 *     cut these pairs.  Row s+1 is read though it is not sampled. */
typedef enum { SCN_STENCIL_AFTER = 0, SCN_STENCIL_BEFORE = 1 } scn_stencil;

typedef struct {
  int32_t kind;
  int32_t stencil; /* scn_stencil; 0 in zero-initialised specs */
  int64_t start, step, stop;
  const int64_t* idx; /* host */
  int64_t n;
} scn_sampling;

typedef struct {
  const scn_table* table;       /* host */
  const scn_sampling* sampling; /* host */
} scn_job;

/* Pyramidal Horn-Schunck parameters (Horn & Schunck 1981, coarse to fine):
 * `levels` >= 1 pyramid levels (each level halves the size, rounding up;
 * the coarsest level must be at least 2x2), smoothness weight `alpha` > 0 in
 * luma code units, `iters` >= 0 Jacobi iterations at every level.
 * `sweeps_per_pass` and `tile_variant` select the Jacobi schedule: 0 and 0
 * let the library's autotuner choose (tuned once per level shape, see
 * SCN_TUNE_CACHE / SCN_TUNE in the implementation notes); sweeps_per_pass = 1
 * with tile_variant = 0 runs one sweep per launch; otherwise the `iters`
 * sweeps of a level run in ceil(iters / k) launches of nearly equal sweep
 * counts, k = sweeps_per_pass (1..63), on register tiles of variant 1..4
 * (128 x 128, 128 x 128, 128 x 64, 128 x 64 pixels), or on 128-column strips
 * streamed row by row with variants 5..18, where k is also capped at the
 * variant's largest sweep count (6, 8, 10, 10, 10, 10, 12, 12, 12, 12, 13,
 * 13, 17, 17; variants 8, 10, 12, 14, 16 and 18 stream bands of up to 1024
 * rows instead of 256; variants 9, 10, 13 and 14 keep six input rows in
 * flight instead of three).  Every schedule gives bitwise identical results.
 * Temporal warm start (scn_flow only; a bounded-state operation with warmup
 * W = 1, Sec. 3.2): with `warm_packet` G >= 2 the pairs of each slice are cut
 * into work packets of G consecutive pairs from the slice's first pair.  The
 * first pair of a packet is solved cold as above; each later pair is solved
 * at full resolution only, starting from its predecessor's flow (I2 warped
 * by it, the constraint linearised about it), with `warm_iters` >= 0 Jacobi
 * iterations.  Results depend on G, not on batching or chunking.  0 or 1:
 * every pair cold (warm_iters ignored).
 *
 * `solver` selects the method: SCN_SOLVER_HS (0, a zero-initialised field)
 * is the Horn-Schunck solver above.  SCN_SOLVER_FARNEBACK (1) is Farnebäck's
 * two-frame motion estimation by polynomial expansion (Farnebäck, SCIA 2003),
 * the FLOW kernel of the paper's microbenchmark (Sec. 5.1.2), on the same
 * pyramid and coarse-to-fine scheme: at every level each frame's
 * neighbourhoods are fitted by a quadratic t'A t + b't + c (weighted least
 * squares over the clamped (2 fb_poly_n + 1)^2 window, Gaussian applicability
 * with standard deviation fb_sigma); then `iters` times per level, from the
 * prior displacement d (the coarser level's result x 2 at the first
 * iteration, zero at the coarsest level), frame 2's coefficients are sampled
 * bilinearly at x + d, A = (A1 + A2(x + d)) / 2 and
 * db = -(b2(x + d) - b1) / 2 + A d, and the new displacement solves
 * (mean(A'A) + fb_lambda I) d = mean(A'db), the means taken over the clamped
 * (2 fb_win + 1)^2 box around each pixel.  alpha, sweeps_per_pass and
 * tile_variant are ignored; warm_packet must be 0 or 1.  Supported:
 * fb_poly_n = 2, fb_sigma in [0.5, 8], fb_win in [0, 8], fb_lambda in
 * (0, 1e6]; other values are SCN_EUNSUPPORTED (fb_poly_n) or SCN_EINVAL.
 * FP32 throughout; results do not depend on batching or chunking. */
enum { SCN_SOLVER_HS = 0, SCN_SOLVER_FARNEBACK = 1 };
typedef struct {
  int32_t levels;
  float alpha;
  int32_t iters;
  int32_t sweeps_per_pass;
  int32_t tile_variant;
  int32_t warm_packet;
  int32_t warm_iters;
  int32_t solver;
  int32_t fb_poly_n;
  float fb_sigma;
  int32_t fb_win;
  float fb_lambda;
} scn_flow_params;

enum { SCN_RGB24 = 0, SCN_GRAY8 = 1 };
enum {
  SCN_OP_CONVERT = 0,
  SCN_OP_HIST = 1,
  SCN_OP_FLOW = 2,
  SCN_OP_SURROGATE = 3,        /* scn_flow_surrogate (p = fallback parameters) */
  SCN_OP_SURROGATE_GRADS = 4,  /* scn_surrogate_grads */
  SCN_OP_SURROGATE_INFER = 5,  /* scn_surrogate_infer */
  SCN_OP_HIST_DIFF = 6         /* scn_hist_diff */
};

/* Number of sampled rows M of a job, or a negative scn_status. */
int64_t scn_count_rows(const scn_job* job);

/* Number of flow pairs P of a job (see scn_stencil), or a negative
 * scn_status. */
int64_t scn_count_pairs(const scn_job* job);

/* Workspace for an operation (SCN_OP_*) over `n_jobs` jobs: the size for
 * the fastest schedule (SCN_OP_FLOW and SCN_OP_SURROGATE also run in smaller
 * workspaces, down to a minimum, by processing pairs in chunks).  For
 * SCN_OP_CONVERT, SCN_OP_HIST and SCN_OP_HIST_DIFF n_jobs must be 1; p is the flow (or
 * fallback) parameters where needed.  Returns 0 on invalid arguments (see
 * scn_last_error). */
size_t scn_workspace_bytes(int32_t op, const scn_job* jobs, int32_t n_jobs, const scn_flow_params* p);

/* Gather the sampled rows of one job and convert them from NV12 to RGB24
 * (BT.601 limited range, Q14 fixed point, chroma replicated 2x2) or take
 * their luma (GRAY8), then resize bilinearly to out_w x out_h with
 * half-pixel centres and 8-bit weights (no resize when the sizes match).
 * This is the format conversion Sec. 4.3 counts as decoder post-processing
 * plus the Resize map of Sec. 3.1, applied only to sampled rows.
 * out: device, [M][out_h][out_w][3] (RGB24, R first) or [M][out_h][out_w]
 * (GRAY8), uint8, row-major, no padding.  out_w, out_h >= 1. */
scn_status scn_sample_convert(const scn_job* job, int32_t out_w, int32_t out_h, int32_t fmt,
                              uint8_t* out, void* ws, size_t ws_bytes, scn_stream_t stream);

/* HIST (Sec. 5.1.2): per sampled row, 16 uniform bins of width 16 per R, G, B
 * channel of the full-resolution BT.601 conversion.
 * hist: device, uint32 [M][3][16] (channel-major), overwritten. */
scn_status scn_hist(const scn_job* job, uint32_t* hist, void* ws, size_t ws_bytes,
                    scn_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): scn_hist
 * without a workspace.  Same kernels and same results as scn_hist; the
 * sampled-row table that scn_hist stages in `ws` goes to a fixed device array
 * of SCN_HIST_STATIC_MAX_ROWS int64 entries (512 KiB) that the library holds
 * on every GPU it runs on until the process ends.  No call allocates or frees
 * device memory.  Jobs selecting more than SCN_HIST_STATIC_MAX_ROWS rows are
 * refused with SCN_ENOSPACE.  Every call on one GPU shares that GPU's array
 * and overwrites the row table of the previous call: calls that overlap on
 * one GPU (different streams, or different host threads without ordering)
 * race, so order them on one stream.  Graph capture follows the workspace
 * rule above, with the array as the workspace.
 * hist: device, uint32 [M][3][16], overwritten. */
#define SCN_HIST_STATIC_MAX_ROWS 65536
scn_status scn_hist_static(const scn_job* job, uint32_t* hist, scn_stream_t stream);

/* Spacing (Sec. 3.2: the inverse of sampling, which aligns a sampled
 * sequence with the dense timeline): the index map of the job's FLOW outputs
 * (its pairs, in order) on the table's n_frames rows, output k placed at the
 * first row of its pair.  mode SCN_SPACE_NULL: map[t] = k at that row and -1
 * elsewhere; SCN_SPACE_REPEAT: map[t] = the last output placed at or before
 * row t (-1 before the first).  map: host, int64 [n_frames], overwritten.
 * Host only: enqueues nothing. */
typedef enum { SCN_SPACE_NULL = 0, SCN_SPACE_REPEAT = 1 } scn_space_mode;
scn_status scn_space_map(const scn_job* job, int32_t mode, int64_t* map);

/* Shot-boundary cue (Sec. 5.2.3: shot boundaries found from histogram
 * differences), a stencil S[0,1] over HIST's output (Sec. 3.2): for each
 * pair of consecutive sampled rows of a slice (the pairs of FLOW; none
 * crosses a RANGE window), d = sum over the 3 channels and 16 bins of
 * |h(second row) - h(first row)|, and cut = (d > threshold).  The job's
 * stencil must be SCN_STENCIL_AFTER (HIST has no output for unsampled rows;
 * else SCN_EINVAL).
 * hist: device, uint32 [M][3][16], the output of scn_hist for the same job
 * (read only).  diff: device, uint32 [P], overwritten.  cut: device, uint8
 * [P], overwritten, or NULL.  threshold: in pixel counts (d lies in
 * [0, 6 w h] and is even).  Frames above 715,827,882 pixels are
 * SCN_EUNSUPPORTED (d would not fit 32 bits).  P = 0 returns SCN_OK with no
 * work.  ws: scn_workspace_bytes(SCN_OP_HIST_DIFF, &job, 1, NULL) bytes. */
scn_status scn_hist_diff(const scn_job* job, const uint32_t* hist, uint32_t threshold, uint32_t* diff,
                         uint8_t* cut, void* ws, size_t ws_bytes, scn_stream_t stream);

/* FLOW (Sec. 3.2 stencil S[0,1], Sec. 5.1.2): dense pyramidal optical flow
 * (Horn-Schunck, or Farnebäck with p->solver), FP32, over the pairs of every job (consecutive sampled rows
 * of each slice, or original neighbours (s, s+1) of each sampled row s with
 * SCN_STENCIL_BEFORE).  Jobs may differ in resolution; all of their pairs
 * are computed by one batch of launches.  Each frame's pyramid is built
 * once and shared by the (at most two) pairs that use it.
 * flow[j]: device, float [P_j][2][H_j][W_j] (u plane then v plane, pixels
 * at full resolution, I1(x) ~ I2(x + (u, v))); may be NULL when P_j == 0. */
scn_status scn_flow(const scn_job* jobs, int32_t n_jobs, const scn_flow_params* p,
                    float* const* flow, void* ws, size_t ws_bytes, scn_stream_t stream);

/* ---- learned flow surrogate ---------------------------------------------
 * A learned model run as a graph operation (Sec. 3.1, Sec. 5.1.2 DNN) used
 * as a cheap FLOW with a conditional fallback to the full computation, the
 * pattern of the hyperlapse application's conditional matching
 * (Sec. 5.2.2).  Network: 3x3 convolutions conv1 2->32, conv2 32->64 stride
 * 2, conv3 64->96 stride 2, x2 nearest upsampling + conv4 96->64, x2 + conv5
 * 64->32, conv6 32->2; ReLU after conv1..conv5; BF16 weights and
 * activations, FP32 accumulation and bias.  Input: per pair, the 2x2 mean of
 * each frame's luma (round half up) as (v - 128)/64 (half resolution; frame
 * width and height must be multiples of 8, else SCN_EUNSUPPORTED).  Output:
 * half-resolution flow, upsampled x2 bilinearly (half-pixel centres) and
 * scaled by 2 to full-resolution pixels.
 * Parameters: scn_net_params() FP32 values, per layer the weights
 * [c_out][c_in][3][3] then the bias [c_out], conv1 first ("master" vector).
 * The network blob (scn_net_bytes() bytes, device, 256-byte aligned) holds
 * the BF16 weights in the kernels' layouts and the FP32 biases. */
size_t scn_net_bytes(void);
int32_t scn_net_params(void);

/* Convert FP32 master parameters (device) into a network blob (device). */
scn_status scn_net_pack(const float* master, void* net, scn_stream_t stream);

/* One Adam step (bias-corrected; `step` counts from 1) on the FP32 master
 * parameters with moment buffers m, v (device, scn_net_params() floats
 * each, zero before the first step) and gradients `grads`; also repacks the
 * updated parameters into `net`. */
scn_status scn_adam_step(float* master, float* m, float* v, const float* grads, int32_t step, float lr,
                         float beta1, float beta2, float eps, void* net, scn_stream_t stream);

/* Loss and gradients of one training batch: every pair of the jobs (one
 * resolution) is a sample; the loss is the mean over samples and
 * full-resolution pixels of sqrt(du^2 + dv^2 + 0.01^2) between the network's
 * full-resolution flow and targets[j] (device, [P_j][2][H][W], e.g. scn_flow's
 * output).  grads: device, scn_net_params() floats (overwritten); loss: device, 1 float. */
scn_status scn_surrogate_grads(const scn_job* jobs, int32_t n_jobs, const void* net, float* const* targets,
                               float* grads, float* loss, void* ws, size_t ws_bytes, scn_stream_t stream);

/* One training step (the trainer's inner loop as one call): the loss and
 * gradients of the batch exactly as scn_surrogate_grads, then the Adam step
 * exactly as scn_adam_step with step number `step` and learning rate `lr`,
 * which updates master, m and v and repacks `net`.  grads: device,
 * scn_net_params() floats of scratch (overwritten with the batch's
 * gradients); loss: device, 1 float.  Arguments of both parts are validated
 * before anything is enqueued.  ws: scn_workspace_bytes(
 * SCN_OP_SURROGATE_GRADS, ...) bytes. */
scn_status scn_surrogate_train_step(const scn_job* jobs, int32_t n_jobs, float* const* targets, float* master,
                                    float* m, float* v, float* grads, void* net, int32_t step, float lr, float beta1,
                                    float beta2, float eps, float* loss, void* ws, size_t ws_bytes,
                                    scn_stream_t stream);

/* The network's full-resolution flow for every pair (no gate, no fallback).
 * flow[j]: device, float [P_j][2][H][W]. */
scn_status scn_surrogate_infer(const scn_job* jobs, int32_t n_jobs, const void* net, float* const* flow, void* ws,
                               size_t ws_bytes, scn_stream_t stream);

/* FLOW with the surrogate and a residual gate: per pair the network's flow w
 * is kept if r = mean over pixels of |Y2(x + w) - Y1(x)| (luma, clamped
 * bilinear warp) is <= gate_tau, else the pair is recomputed by scn_flow's
 * plain Horn-Schunck solver with fallback_p (fallback_p->solver must be
 * SCN_SOLVER_HS, else SCN_EUNSUPPORTED).  The decision is taken on the
 * device (no host synchronisation).  flow[j]: device [P_j][2][H][W];
 * fell_back[j] (device, uint8 [P_j], may be NULL) receives 1 for recomputed
 * pairs; residual[j] (device, float [P_j], may be NULL) receives r. */
scn_status scn_flow_surrogate(const scn_job* jobs, int32_t n_jobs, const scn_flow_params* fallback_p, const void* net,
                              float gate_tau, float* const* flow, uint8_t* const* fell_back, float* const* residual,
                              void* ws, size_t ws_bytes, scn_stream_t stream);

/* Kernel timing for diagnostics and benchmarks.  scn_timing_enable(1, n)
 * creates a pool of 2n HIP events; while enabled, every kernel launch of the
 * library is bracketed by two events recorded on its stream (at most n
 * launches until the next scn_timing_reset).  scn_timing_read synchronises
 * those events and returns the summed duration and launch count of one
 * kernel class ("hist16", "nv12_rgb24", "nv12_resize", "luma_copy",
 * "pyr_down", "hs_setup", "hs_jacobi", "fb_poly", "fb_disp",
 * "conv_fwd", "conv_dx",
 * "conv_dw", "flow_up", "gate"), or of a finer class ("hs_jacobi_l0" ..
 * "hs_jacobi_l6" per pyramid level, "conv_fwd1" .. "conv_fwd6" per layer);
 * nested classes time the same launches.  It returns SCN_ENOSPACE if
 * launches were dropped because the pool was full.  Not thread-safe with
 * respect to concurrent enable/reset. */
scn_status scn_timing_enable(int32_t enable, int32_t max_launches);
scn_status scn_timing_reset(void);
scn_status scn_timing_read(const char* kernel, double* total_ms, int64_t* launches);
/* Summed work units of the recorded launches of one kernel class (same
 * classes and pool as scn_timing_read; no synchronisation).  The Jacobi
 * classes ("hs_jacobi", "hs_jacobi_l*") record, per pass over the planes
 * of a chunk, the level's pixels x the chunk's pairs, whatever the pass's
 * sweep count (every launch of the one-sweep schedule is a pass; a masked
 * fallback pass, whose pair count is known only on the device, records 0);
 * other classes record 0.  *units receives the sum;
 * SCN_EINVAL for NULL arguments, SCN_ENOSPACE if launches were dropped. */
scn_status scn_timing_units(const char* kernel, double* units);

/* Drop the record of the last plan uploaded to `ws` (for example before the
 * memory is freed; a capture on `ws` is then refused until an eager call). */
void scn_ws_forget(const void* ws);

/* Thread-local message for the last failing call on this thread ("" if none). */
const char* scn_last_error(void);

/* Library version string. */
const char* scn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SCN_H */
