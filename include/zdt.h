/*
 * zdt.h -- C ABI of the MI355X (gfx950) stereo hot path:
 *   ZNCC matching cost  ->  domain-transform (DT) aggregation  ->  WTA.
 *
 * Method: "Efficient Stereo Matching on Embedded GPUs with Zero-Means Cross
 * Correlation" (Chang et al., arXiv 2212.00476).  Each entry point cites the
 * passage that defines the operation it runs.
 *
 * Conventions shared by every entry point
 *   - Images are 8-bit grayscale, row-major, `pitch` bytes between rows.
 *     left = reference I_R, right = target I_T; a candidate pairs I_R(x,y)
 *     with I_T(x-d,y), d in [0, D) (Sec. III-A).
 *   - Every pixel read is clamped to the image (replicate border); target
 *     columns x-d+i < 0 read column 0.
 *   - A cost volume is [H][W][D] with d fastest (element (x,y,d) at
 *     ((y*W + x)*D + d)), stored as float32, float16, bfloat16, int16 or the
 *     8-bit code of an int16 (`vol_dtype`, zdt_dtype below).  The cost is
 *     1 - ZNCC in [0, 2] (times T for int16).
 *   - Pointers to images, volumes, disparities and workspace are DEVICE
 *     pointers owned by the caller; the library never frees or keeps them.
 *     `params` and the `applied_scale` output are HOST pointers.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     their kernels and return without synchronising.  Argument errors are
 *     reported synchronously with nothing enqueued; a failed launch returns
 *     ZDT_EHIP.  zdt_last_error() gives a message for the calling thread's
 *     last failure.
 *   - Calls that share a volume or workspace must be ordered by the caller
 *     (same stream, or events); calls on disjoint buffers may overlap.
 */
#ifndef ZDT_H
#define ZDT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum zdt_status {
  ZDT_OK = 0,
  ZDT_EINVAL = -1,          /* a parameter or pointer is invalid            */
  ZDT_ENOMEM = -2,          /* a host-side allocation failed                */
  ZDT_EHIP = -3,            /* a HIP call or kernel launch failed           */
  ZDT_EUNSUPPORTED = -4     /* valid, but outside what the library supports */
} zdt_status;

/* Volume element types.  ZDT_I16 and ZDT_I8 are the paper's narrow integer
 * volumes (Sec. IV-C) as its FastDT runs them (Sec. V-C, Table II): every DT
 * state but the last is the cost times T = 21 rounded to an int16 (round half
 * to even), as if each of the four passes stored its output; the states are
 * made nearly zero-mean by Eq. DT_new with d_arb = 0, subtracting the pass
 * input's d = 0 value at each pixel, in the first U2D pass for ZDT_I16 and
 * in the first R2L pass for ZDT_I8.  ZDT_I8 stores the R2L output (and the
 * output of every sweep but the last) as that int16's 8-bit code (six
 * significant bits plus a 2-bit position flag; only negative values are kept,
 * non-negative ones code to 0).  Volumes cross memory only between pass pairs;
 * the rounding of the L2R and U2D outputs happens in registers.  The
 * recursions run in float32.  They are approximations for bandwidth: the
 * paper's choice of T bounds the states only for few passes, so stereo_solve
 * refuses (ZDT_EUNSUPPORTED) parameters for which a stored state could leave
 * the int16 range (bound: 2T, times 1/(1-K) per pass, plus 1/2 per store). */
typedef enum zdt_dtype { ZDT_F32 = 0, ZDT_F16 = 1, ZDT_BF16 = 2, ZDT_I16 = 3, ZDT_I8 = 4 } zdt_dtype;

/* flags */
#define ZDT_FLAG_NORMALIZE 1     /* scale each DT pass by (1 - K); forced for F16/BF16 */
#define ZDT_FLAG_GUIDE_TARGET 2  /* DT weights from the target (right) image instead of the reference */

typedef struct zdt_params {
  int32_t width;        /* W >= 1                                                      */
  int32_t height;       /* H >= 1                                                      */
  int32_t pitch;        /* bytes between image rows, >= W                              */
  int32_t max_disp;     /* D >= 1; candidates d = 0 .. D-1                             */
  int32_t radius;       /* r, window side l = 2r+1; 0 <= r <= 7 (32-bit exact sums)     */
  float sigma_s;        /* DT spatial parameter, > 0 (Eq. a: a = K = exp(-1/sigma_s))  */
  float sigma_r;        /* DT range parameter in intensity/255 units, > 0; +inf turns  */
                        /* the range term off                                          */
  int32_t dt_iters;     /* I >= 0 sweeps of the four DT passes (0 = no aggregation)    */
  int32_t vol_dtype;    /* zdt_dtype of every cost volume the call reads or writes     */
  int32_t flags;        /* ZDT_FLAG_*                                                  */
  int32_t reserved[4];  /* must be zero                                                */
} zdt_params;

/* Bytes of device workspace that stereo_solve() needs besides its volume
 * (0 means `ws` may be NULL).  Returns 0 for invalid parameters as well; the
 * entry points report those. */
size_t zdt_workspace_size(const zdt_params* params);

/* Bytes of one cost volume for these parameters: W*H*D*sizeof(vol_dtype). */
size_t zdt_volume_size(const zdt_params* params);

/* Matching-cost volume (Sec. III-A, Eq. ZNCC, evaluated through the sum form
 * of Eq. OP_ZNCC from exact int32 window sums):
 *   cost(x,y,d) = 1 - clamp(ZNCC(x,y,d), -1, 1), written to `cost_hwd`.
 * A window of zero variance (on either side) gives ZNCC = 0, i.e. cost 1. */
int zncc_cost_volume(const zdt_params* params, const uint8_t* left, const uint8_t* right, void* cost_hwd,
                     void* stream);

/* DT aggregation in place on `cost_hwd` (Sec. III-B, Eqs. DT1-DT4 with the
 * edge weights of Eqs. k1-k4 / weight computed from `guide`):
 *   per sweep, for every d:  L along +x, R along -x, U along +y, D along -y,
 *   with W_L(x) = exp(-1/sigma_s - |G(x)-G(x-1)|/(255 sigma_r)), W_R(x) = W_L(x+1),
 *   and the same vertically; repeated dt_iters times.
 * `guide` is the reference image (the weights' image; the caller passes the
 * target to follow ZDT_FLAG_GUIDE_TARGET).  The recursion state is float32.
 * With ZDT_FLAG_NORMALIZE (always on for F16/BF16) every pass is scaled by
 * (1 - K); the volume returned is then s_total * C_agg with
 * s_total = (1-K)^(4*dt_iters), written to *applied_scale when it is not NULL
 * (1.0 without normalisation).  Scaling leaves the argmin unchanged. */
int dt_aggregate(const zdt_params* params, const uint8_t* guide, void* cost_hwd, double* applied_scale,
                 void* stream);

/* Winner-take-all (Sec. III-C, Eq. WTA1): disp(x,y) = the smallest d with
 * cost(x,y,d) = min_d' cost(x,y,d').  `disp_hw` is int32 [H][W]. */
int wta_disparity(const zdt_params* params, const void* cost_hwd, int32_t* disp_hw, void* stream);

/* The whole path for one pair: cost (Sec. III-A), DT (Sec. III-B), WTA
 * (Sec. III-C), with the cost fused into the first horizontal pass pair and the
 * WTA fused into the last vertical pass pair (the fusion boundaries of
 * Sec. V-C).  `vol_hwd` is a caller-owned volume of zdt_volume_size() bytes
 * used as the working volume; its contents on return are unspecified.  `ws`
 * holds zdt_workspace_size() bytes (may be NULL when that is 0).  With
 * dt_iters = 0 this is the WTA of the raw cost. */
int stereo_solve(const zdt_params* params, const uint8_t* left, const uint8_t* right, int32_t* disp_hw,
                 void* vol_hwd, void* ws, void* stream);

/* stereo_solve() for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * workspace comes from an array of ZDT_STATIC_WS_BYTES bytes that the library
 * holds on each GPU it runs on (until the process ends); the caller passes the
 * images, the disparity output and the working volume (zdt_volume_size()
 * bytes) as for stereo_solve().  Parameters whose zdt_workspace_size() exceeds
 * ZDT_STATIC_WS_BYTES give ZDT_EUNSUPPORTED (1280x384 with D = 128 fits in
 * every volume type).  The call makes no device or host allocation (the
 * array's device address is looked up once per GPU) and records no timing
 * events.  Every call on one GPU shares that GPU's array: calls that may
 * overlap on one GPU (other streams or threads) race and must be ordered by
 * the caller.  Nothing in the array needs to start at any value. */
#define ZDT_STATIC_WS_BYTES (32u << 20)
int stereo_solve_static_ws(const zdt_params* params, const uint8_t* left, const uint8_t* right, int32_t* disp_hw,
                           void* vol_hwd, void* stream);

/* One pair of a batch: its parameters and caller-owned device buffers, as for
 * stereo_solve() (vol: zdt_volume_size(&params) bytes, ws:
 * zdt_workspace_size(&params) bytes).  Jobs of one batch must not share a
 * volume, workspace or disparity buffer. */
typedef struct zdt_job {
  zdt_params params;
  const uint8_t* left;
  const uint8_t* right;
  int32_t* disp;
  void* vol;
  void* ws;
} zdt_job;

/* stereo_solve() for n pairs of mixed shapes, with the same results as n
 * separate calls.  The pairs are dealt, largest first, over two streams that
 * the library owns on the stream's GPU (default priority; created on the first
 * batch, kept until the process ends), forked from `stream` and joined back to
 * it with events: work enqueued on `stream` before the call is seen by every
 * pair, and work enqueued after it sees every result.  Pairs on the two streams
 * share the GPU, so one pair's launches fill the CUs while another's drain.
 * Batches from several host threads on one GPU are enqueued one at a time.
 * Under graph capture of `stream` the batch stays on `stream`, and jobs with
 * identical parameters share every launch: each stage (cost + L/R pair, U/D
 * pair, ...) runs as one grid over up to 32 of them.  (The paper solves one
 * pair at a time; its nearest analogue is the per-shape launch-configuration
 * sweep of Sec. V-B.)  All jobs are validated before anything is enqueued;
 * job i's error is reported with its index.  n = 0 does nothing. */
int stereo_solve_batch(const zdt_job* jobs, int32_t n, void* stream);

/* Graphs of a batch (serving loops): stereo_solve_batch(jobs, n) recorded
 * once on `stream` (hipStreamBeginCapture, thread-local mode) into an
 * executable HIP graph (hipGraphInstantiate) that zdt_graph_launch() replays
 * on any stream.  The jobs' device buffers and parameters are baked into the
 * graph: a replay solves whatever the images hold at that time, into the same
 * disparity buffers, so callers refill the images between replays (and order
 * replays that share buffers).  zdt_graph_create() first runs the batch once,
 * eagerly, on `stream` (which must not be the NULL stream) so that the capture
 * records launches only; the captured kernels include no memset.  The graph
 * object is owned by the caller (zdt_graph_destroy).  Same errors as
 * stereo_solve_batch(), ZDT_EHIP when capture or instantiation fails. */
typedef struct zdt_graph zdt_graph;
int zdt_graph_create(const zdt_job* jobs, int32_t n, void* stream, zdt_graph** out);
int zdt_graph_launch(zdt_graph* graph, void* stream);
int zdt_graph_destroy(zdt_graph* graph);

/* Semi-global matching over a cost volume: the aggregation of the paper's
 * system S1 (Sec. V-D, Table IV), where ZNCC costs multiplied by T feed SGM
 * with P1 = 18, P2 = 185.  The paper takes SGM from its reference [r7]; this
 * is its four-path form with constant penalties.  Along each of the paths
 * left-to-right, right-to-left, top-to-bottom and bottom-to-top, with q the
 * previous pixel of p on the path,
 *   L(p,d) = s*C(p,d) + min(L(q,d), L(q,d-1) + P1, L(q,d+1) + P1, m(q) + P2) - m(q),
 *   m(q) = min_k L(q,k),   L(p,d) = s*C(p,d) on a path's first pixel,
 * and sum_hwd(p,d) = the sum of the four L(p,d).  s is `cost_scale`.
 *   cost_hwd  [H][W][D] DEVICE volume of params->vol_dtype, ZDT_F32 or ZDT_F16
 *             (e.g. from zncc_cost_volume), read only; finite values
 *   sum_hwd   FP32 [H][W][D] DEVICE volume, written; must not overlap cost_hwd
 * Both volumes 16-byte aligned.  Other vol_dtypes or max_disp > 256 give
 * ZDT_EUNSUPPORTED; penalties outside 0 <= p1 <= p2 < inf, a cost_scale that
 * is negative or not finite, or NULL / misaligned / overlapping volumes give
 * ZDT_EINVAL.  The recursion runs in float32 whatever the cost type; rounding
 * aside the result is the four-path sum above.  wta_disparity() (with an F32
 * vol_dtype) on sum_hwd completes the system. */
int sgm_aggregate(const zdt_params* params, const void* cost_hwd, float* sum_hwd, float p1, float p2,
                  float cost_scale, void* stream);

/* sgm_aggregate() followed by the WTA (Eq. WTA1: the smallest d of minimum
 * sum), taken as the last two paths finish each pixel so that the final sums
 * are never stored: int32 disp_hw [H][W] (DEVICE).  sum_hwd is used as the
 * working volume; its contents on return are unspecified.  Same errors as
 * sgm_aggregate(), and ZDT_EINVAL for a NULL disp_hw. */
int sgm_disparity(const zdt_params* params, const void* cost_hwd, float* sum_hwd, int32_t* disp_hw, float p1,
                  float p2, float cost_scale, void* stream);

/* System S1 for one pair: zncc_cost_volume() into `cost_hwd`, then
 * sgm_disparity().  cost_hwd (W*H*D elements of vol_dtype, F32 or F16) and
 * sum_hwd (W*H*D floats) are caller-owned; their contents on return are
 * unspecified.  Same errors as sgm_disparity() and zncc_cost_volume(). */
int stereo_solve_sgm(const zdt_params* params, const uint8_t* left, const uint8_t* right, int32_t* disp_hw,
                     void* cost_hwd, float* sum_hwd, float p1, float p2, float cost_scale, void* stream);

/* Tile plan of the register-resident passes for one shape:
 *   h_lanes  lanes per horizontal segment: 32 (two segments per wave; the row
 *            must split into an even number <= 32 of segments of exactly
 *            h_seg values) or 64 (up to 16 segments of at most h_seg values)
 *   h_seg    compiled horizontal segment length: 8, 20, 40, 60 (32 lanes) or
 *            16, 40, 80 (64 lanes)
 *   v_lanes  lanes per vertical segment: 32 (two segments per wave, the
 *            column split into an even number <= 32 of segments of exactly
 *            v_seg rows) or 64 (up to 16 segments of at most v_seg rows)
 *   v_seg    compiled vertical segment length: 12, 24, 36 (32 lanes) or
 *            8, 12, 24, 48, 72 (64 lanes)
 * A plan changes only how rows and columns are cut into register-resident
 * segments; results agree with every other plan up to float32 rounding of the
 * segment-carry composition. */
typedef struct zdt_plan {
  int32_t h_lanes, h_seg, v_lanes, v_seg;
} zdt_plan;

/* Every plan that fits params' shape, the default first: writes up to `max` of
 * them to `out` (HOST array) and returns how many there are (< 0: error). */
int zdt_plan_candidates(const zdt_params* params, zdt_plan* out, int max);

/* The plan used for params' shape (W, H, D, r, vol_dtype): the one pinned by
 * zdt_set_plan() or zdt_autotune(), else the default. */
int zdt_get_plan(const zdt_params* params, zdt_plan* out);

/* Pin `plan` (a candidate for the shape, else ZDT_EINVAL) for every later call
 * on params' shape in this process; NULL returns the shape to its default.
 * Thread-safe; calls already enqueued keep the plan they were issued with. */
int zdt_set_plan(const zdt_params* params, const zdt_plan* plan);

/* Autotuner: if `cache_path` (may be NULL) holds a plan for the shape, pin it;
 * otherwise time stereo_solve() under every candidate plan on `stream` (two
 * warm-up and five timed runs each, on a synthetic pair in buffers it
 * allocates and frees), pin the fastest and append it to `cache_path`.  The
 * chosen plan is written to *chosen when that is not NULL.  Synchronises the
 * stream; not for use under stream capture. */
int zdt_autotune(const zdt_params* params, const char* cache_path, zdt_plan* chosen, void* stream);

/* Exact integer sums behind the cost (Sec. IV-B summation and the Pi_RT term
 * of Eq. OP_ZNCC), exposed for verification; any output pointer may be NULL:
 *   s_l, s_ll      [H][W]        sum of I_R and I_R^2 over the window at (x,y)
 *   s_t, s_tt      [H][W+D-1]    sum of I_T and I_T^2 over the window at x',
 *                                x' = -(D-1) .. W-1 stored at index x'+D-1
 *   s_rt           [H][W][D]     sum over the window of I_R(x+i,y+j) I_T(x-d+i,y+j)
 * All int32 and exact (every sum is below 2^31 for l <= 15). */
int zncc_window_sums(const zdt_params* params, const uint8_t* left, const uint8_t* right, int32_t* s_l,
                     int32_t* s_ll, int32_t* s_t, int32_t* s_tt, int32_t* s_rt, void* stream);

/* The same reference and target window sums by the paper's Method 2
 * (Sec. IV-B): integral images of the border-replicated image and of its
 * squares, integrating every row (a block-wide scan) and then every column,
 * and each window sum from four corners.  The integrals are kept in uint32 and
 * wrap on large images; a window's sum is below 2^31 and the four-corner
 * difference is exact modulo 2^32, so the results equal zncc_window_sums()'s
 * bit for bit.  Any output may be NULL; `ws` is DEVICE memory of
 * zdt_integral_workspace_size() bytes (4-byte aligned) holding the integral
 * images, overwritten.  W + D - 1 + 2r must not exceed 3072
 * (ZDT_EUNSUPPORTED). */
size_t zdt_integral_workspace_size(const zdt_params* params);
int zncc_window_sums_integral(const zdt_params* params, const uint8_t* left, const uint8_t* right, int32_t* s_l,
                              int32_t* s_ll, int32_t* s_t, int32_t* s_tt, void* ws, void* stream);

/* Test entry for the 8-bit code of ZDT_I8 volumes (Sec. IV-C, data encoding
 * and decoding): codes[i] = encode(values[i]) and decoded[i] =
 * decode(codes[i]) for i < n, on the device.  All three are DEVICE arrays. */
int zdt_i8_codec(const int16_t* values, uint8_t* codes, int16_t* decoded, int64_t n, void* stream);

/* Message for the calling thread's last non-OK return ("" if none). */
const char* zdt_last_error(void);

/* Kernel timing.  zdt_profile_enable(1) clears the records and makes every
 * later launch on any stream record a HIP event pair around itself on that
 * stream; zdt_profile_enable(0) stops recording.  zdt_profile_collect()
 * synchronises on the recorded events and returns the number of distinct
 * kernel names seen; zdt_profile_entry() reads one of them: its name (static
 * storage), the summed milliseconds and the number of launches. */
int zdt_profile_enable(int on);
int zdt_profile_collect(void);
int zdt_profile_entry(int index, const char** name, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* ZDT_H */
