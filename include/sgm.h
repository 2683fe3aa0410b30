/*
 * sgm.h -- C ABI of libsgm.so, the MI355X (gfx950) SGM stereo hot path.
 *
 * The calls follow the problem statement of Ruf et al., 2021, "ReS2tAC --
 * UAV-borne real-time SGM stereo optimized for embedded ARM and CUDA devices":
 * a rectified grey-value pair, a disparity range Gamma = {0 .. ndisp-1}, the
 * census/Hamming matching cost (Sec. 2.1.1, Eq. image_matching), the SGM path
 * aggregation (Sec. 2.1.2, Eq. sgm_path and Eq. sgm_path_aggr), and the
 * disparity selection with its post-processing (Eq. wta, Eq. right_disparity,
 * Eq. LR_check, the 3x3 median of Sec. 2.1.3).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every buffer pointer is a DEVICE pointer, allocated and owned by the
 *    caller.  Inputs are never written.  Outputs must not alias inputs.
 *  - Layout is row-major.  Maps are [height][width]; volumes are
 *    [height][width][ndisp] with the disparity index fastest (contiguous).
 *  - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL
 *    is the default stream).  No call allocates device memory or synchronises.
 *  - Every argument is validated before anything is enqueued.  On any error
 *    nothing is launched and nothing is written; the status tells why.
 *    Faults inside a launched kernel surface at the caller's next
 *    synchronisation of `stream`.
 *  - All arithmetic is integer; results are bit-exact and do not depend on
 *    launch shape, stream or timing.
 *  - Calls are reentrant; calls on different streams may run concurrently
 *    when their buffers are distinct.
 *  - Disparity maps are uint16 with SGM_INVALID (0xFFFF) marking invalid
 *    pixels.
 */
#ifndef SGM_H
#define SGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGM_INVALID 0xFFFFu
#define SGM_MAX_NDISP 256
#define SGM_MAX_SIDE 32768               /* width and height limit              */
#define SGM_MAX_VOLUME 2147483647LL      /* width * height * ndisp limit        */

typedef enum {
    SGM_OK = 0,
    SGM_ERR_ARG = -1,          /* null pointer, size or parameter out of range      */
    SGM_ERR_UNSUPPORTED = -2,  /* census window other than 5x5 or 9x7               */
    SGM_ERR_ALIGN = -3,        /* pointer not aligned as documented below           */
    SGM_ERR_HIP = -4,          /* a HIP launch failed; see sgm_last_hip_error()     */
    SGM_ERR_WORKSPACE = -5,    /* workspace missing or too small                    */
    SGM_ERR_TOO_LARGE = -6     /* frame needs more than SGM_NOALLOC_SCRATCH_BYTES   */
} sgm_status;

/*
 * Census transform (Sec. 2.2.1; centre omitted as in Sec. 2.3.1).
 * For every pixel p one bit [I(q) < I(p)] per neighbour q of a win_w x win_h
 * window (centre excluded), in raster order (rows top to bottom, columns left
 * to right), the first neighbour in the highest used bit; neighbours outside
 * the image read as 0 (the zero-valued margin).
 *   img         uint8 [height][pitch_bytes], 1-byte aligned, pitch_bytes >= width
 *   win_w,win_h (5,5) -> 24 bits, or (9,7) = 9 columns x 7 rows -> 62 bits
 *   census_out  uint64 [height][width], 8-byte aligned
 * Errors: SGM_ERR_ARG (null, width/height < 1, pitch < width),
 *         SGM_ERR_UNSUPPORTED (other windows), SGM_ERR_ALIGN.
 */
int32_t sgm_census(const uint8_t* img, int32_t width, int32_t height,
                   int32_t pitch_bytes, int32_t win_w, int32_t win_h,
                   uint64_t* census_out, void* stream);

/*
 * Census transform of both images of a pair in one launch (Sec. 2.2.1): the
 * same descriptors as sgm_census on left and on right, with one launch
 * latency instead of two.  Both images share width, height and pitch.
 *   left, right                       uint8 [height][pitch_bytes]
 *   census_left_out, census_right_out uint64 [height][width], 8-byte aligned,
 *                                     distinct buffers
 * Errors: as sgm_census; SGM_ERR_ARG also when the two outputs coincide.
 */
int32_t sgm_census_pair(const uint8_t* left, const uint8_t* right, int32_t width,
                        int32_t height, int32_t pitch_bytes, int32_t win_w, int32_t win_h,
                        uint64_t* census_left_out, uint64_t* census_right_out, void* stream);

/*
 * Matching-cost volume, Eq. (image_matching) with Phi the Hamming distance of
 * census descriptors (Sec. 2.1.1):
 *   C(x, y, d) = popcount(CL(x, y) ^ CR(x - d, y))   if x - d >= 0
 *              = 255 (0xFF, no match; Sec. 2.3.1)    otherwise
 *   census_left, census_right  uint64 [height][width], 8-byte aligned
 *   ndisp                      1 .. 256, width*height*ndisp <= SGM_MAX_VOLUME
 *   cost_out                   uint8 [height][width][ndisp], 16-byte aligned
 * Errors: SGM_ERR_ARG, SGM_ERR_ALIGN.
 */
int32_t sgm_cost(const uint64_t* census_left, const uint64_t* census_right,
                 int32_t width, int32_t height, int32_t ndisp,
                 uint8_t* cost_out, void* stream);

/*
 * Inverted, truncated normalised cross-correlation cost (Sec. 2.1.1,
 * Sec. 2.2.1), an alternative to sgm_census + sgm_cost:
 *   s = 1 - max(0, Phi_NCC) over win x win patches centred on (x, y) in the
 *   left image and (x - d, y) in the right image, with
 *   Phi = (n S_LR - S_L S_R) / (sqrt(n S_LL - S_L^2) * sqrt(n S_RR - S_R^2)),
 *   n = win^2 and S_* the integer sums over the two patches.
 *   Stored as round(255 s) (ties to even) in the same uint8 volume as
 *   sgm_cost, so the aggregation and selection calls apply unchanged.
 *   Pixels outside the image read as zero; a patch without variance gives
 *   cost 255, as does x - d < 0.  The float part is float32 with IEEE square
 *   root and division, evaluated as den = sqrt(vL) * sqrt(vR),
 *   phi = num / den, 255 * (1 - max(0, phi)); results are reproducible bit
 *   for bit.
 *   left, right  uint8 [height][pitch_bytes] device images
 *   win          5 or 9
 *   cost_out     uint8 [height][width][ndisp], 16-byte aligned
 * Errors: SGM_ERR_ARG, SGM_ERR_UNSUPPORTED (win), SGM_ERR_ALIGN.
 */
int32_t sgm_cost_ncc(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                     int32_t pitch_bytes, int32_t win, int32_t ndisp, uint8_t* cost_out,
                     void* stream);

/*
 * SGM aggregation, Eq. (sgm_path) and Eq. (sgm_path_aggr) (Sec. 2.1.2):
 *   L_r(p, d) = C(p, d) + min(L'(d), L'(d-1) + P1, L'(d+1) + P1, m' + P2) - m'
 *   with L' = L_r(p - r, .) and m' = min_d L'(d); L_r = C at the first pixel
 *   of a path; terms with d +- 1 outside Gamma drop out;
 *   S_bar(p, d) = sum over the path set of L_r(p, d).
 * Path sets: npaths = 4 -> the two horizontal and the two vertical paths
 * (Sec. 3.1.4); npaths = 8 adds the four diagonals.
 *   cost       uint8 [height][width][ndisp], 16-byte aligned
 *   p1, p2     penalties with 0 <= p1 <= p2 and npaths * (255 + p2) <= 65535,
 *              so that every S_bar fits uint16 exactly
 *   agg_out    uint16 [height][width][ndisp], 16-byte aligned
 *   work       device scratch of at least sgm_aggregate_work_bytes(...) bytes,
 *              16-byte aligned, holding one slice per pair of opposite path
 *              directions between the path pass and the sum; contents on
 *              return are unspecified
 * Errors: SGM_ERR_ARG (sizes, width*height*ndisp > SGM_MAX_VOLUME, npaths
 *         not 4/8, p1 > p2, overflow bound), SGM_ERR_WORKSPACE (work NULL or
 *         work_bytes too small), SGM_ERR_ALIGN.
 */
int32_t sgm_aggregate(const uint8_t* cost, int32_t width, int32_t height,
                      int32_t ndisp, int32_t npaths, int32_t p1, int32_t p2,
                      uint16_t* agg_out, void* work, size_t work_bytes,
                      void* stream);

/* Bytes of `work` that sgm_aggregate needs: npaths / 2 slices of
 * width*height*ndisp elements (rounded up to 256), 1 byte each when
 * p2 <= 127 (a pair's two penalty parts sum to at most 254), else 2.
 * 0 on invalid sizes or penalties. */
size_t sgm_aggregate_work_bytes(int32_t width, int32_t height, int32_t ndisp,
                                int32_t npaths, int32_t p2);

/*
 * Disparity selection and post-processing (Eq. wta, Eq. right_disparity,
 * Eq. LR_check, Sec. 2.1.3):
 *   D^L(p) = smallest d minimising S_bar(p, d)
 *   D^R(p) = smallest d minimising S_bar((px + d, py), d) over px + d < width
 *   LR check (lr_tolerance = t >= 0): D(p) = D^L(p) if px - D^L(p) >= 0 and
 *            |D^L(p) - D^R(px - D^L(p), py)| <= t, else SGM_INVALID;
 *            lr_tolerance < 0 skips the check (D = D^L).
 *   median3x3 = 1: every valid pixel takes the median of its 3x3 window, in
 *            which pixels outside the image and invalid pixels count as
 *            0xFFFF; invalid pixels stay invalid.  0 skips the median.
 *   agg             uint16 [height][width][ndisp], 16-byte aligned
 *   disp_out        uint16 [height][width], 4-byte aligned
 *   disp_right_out  uint16 [height][width] receiving D^R, or NULL
 *   work            uint16 scratch of sgm_wta_lrc_work_elems(width, height)
 *                   elements, 4-byte aligned; contents on return are
 *                   unspecified
 * Errors: SGM_ERR_ARG, SGM_ERR_ALIGN, SGM_ERR_WORKSPACE (work NULL).
 */
int32_t sgm_wta_lrc(const uint16_t* agg, int32_t width, int32_t height,
                    int32_t ndisp, int32_t lr_tolerance, int32_t median3x3,
                    uint16_t* disp_out, uint16_t* disp_right_out,
                    uint16_t* work, void* stream);

/* Number of uint16 elements sgm_wta_lrc needs in `work` (0 on bad sizes). */
size_t sgm_wta_lrc_work_elems(int32_t width, int32_t height);

/*
 * Streamlined aggregation: sgm_aggregate followed by sgm_wta_lrc in one call
 * whose path sum S_bar never reaches device memory.  The paper points to
 * fusing the last aggregation step with the disparity selection as a known
 * speed-up for GPU SGM (Sec. 4.2); here the path sum of Eq. (sgm_path_aggr)
 * is formed on chip inside the selection pass.  disp_out and disp_right_out
 * are bit-identical to those two calls with the same arguments.
 * The fused form applies when ndisp % 16 == 0 (any legal p2); other valid
 * arguments run the two unfused calls on the same workspace.
 *   cost, npaths, p1, p2          as for sgm_aggregate
 *   lr_tolerance, median3x3,
 *   disp_out, disp_right_out      as for sgm_wta_lrc
 *   work       device scratch of sgm_aggregate_select_work_bytes(...) bytes,
 *              256-byte aligned; contents on return are unspecified
 * Errors: SGM_ERR_ARG, SGM_ERR_WORKSPACE, SGM_ERR_ALIGN, SGM_ERR_HIP.
 */
int32_t sgm_aggregate_select(const uint8_t* cost, int32_t width, int32_t height,
                             int32_t ndisp, int32_t npaths, int32_t p1, int32_t p2,
                             int32_t lr_tolerance, int32_t median3x3,
                             uint16_t* disp_out, uint16_t* disp_right_out,
                             void* work, size_t work_bytes, void* stream);

/* Bytes of `work` that sgm_aggregate_select needs (0 on invalid arguments). */
size_t sgm_aggregate_select_work_bytes(int32_t width, int32_t height, int32_t ndisp,
                                       int32_t npaths, int32_t p2);

/*
 * sgm_aggregate_select without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * hosts that forbid hipMalloc).  The workspace is a fixed array of
 * SGM_NOALLOC_SCRATCH_BYTES inside this library, one per GPU, kept until the
 * process ends; the call itself allocates nothing.  Outputs are bit-identical
 * to sgm_aggregate_select with the same arguments.
 *   Arguments, layouts and ownership as for sgm_aggregate_select, without
 *   work / work_bytes; `stream` must belong to the current device.
 *   Every call on one GPU uses that GPU's one array: calls that overlap on
 *   one GPU (other streams, other host threads) race and must be ordered by
 *   the caller; calls queued on one stream are ordered already.
 * Errors: SGM_ERR_ARG, SGM_ERR_ALIGN, SGM_ERR_HIP (including the first
 *         look-up of the array on a device), SGM_ERR_TOO_LARGE when
 *         sgm_aggregate_select_work_bytes(...) > SGM_NOALLOC_SCRATCH_BYTES
 *         (1242 x 375 with D = 128 and 8 paths needs about 241 MB and fits);
 *         nothing is enqueued on error.
 */
#define SGM_NOALLOC_SCRATCH_BYTES (256u << 20)
int32_t sgm_aggregate_select_noalloc(const uint8_t* cost, int32_t width, int32_t height,
                                     int32_t ndisp, int32_t npaths, int32_t p1, int32_t p2,
                                     int32_t lr_tolerance, int32_t median3x3,
                                     uint16_t* disp_out, uint16_t* disp_right_out, void* stream);

/*
 * sgm_aggregate_select with subpixel refinement (Sec. 2.1.3): every pixel's
 * WTA disparity d gets the vertex offset of the parabola through S_bar at
 * d - 1, d, d + 1,
 *   off = (S(d-1) - S(d+1)) / (2 (S(d-1) - 2 S(d) + S(d+1))),  |off| <= 1/2,
 * with off = 0 at d = 0, d = ndisp - 1 and where the three costs are equal;
 * computed in float32 (IEEE division).  The LR check runs on the integer
 * maps exactly as in sgm_wta_lrc; pixels it keeps take d + off; the 3x3
 * median then runs over those float values, with pixels outside the image
 * and invalid pixels counting as +inf (a median of +inf is invalid).
 *   disp_out        float [height][width]; invalid pixels are -1.0f
 *   disp_right_out  uint16 [height][width] (D^R) or NULL
 *   work            sgm_aggregate_select_subpixel_work_bytes(...) bytes,
 *                   256-byte aligned
 * Other arguments and errors as for sgm_aggregate_select.
 */
int32_t sgm_aggregate_select_subpixel(const uint8_t* cost, int32_t width, int32_t height,
                                      int32_t ndisp, int32_t npaths, int32_t p1, int32_t p2,
                                      int32_t lr_tolerance, int32_t median3x3,
                                      float* disp_out, uint16_t* disp_right_out,
                                      void* work, size_t work_bytes, void* stream);

/* Bytes of `work` that sgm_aggregate_select_subpixel needs (0 on invalid
 * arguments). */
size_t sgm_aggregate_select_subpixel_work_bytes(int32_t width, int32_t height, int32_t ndisp,
                                                int32_t npaths, int32_t p2);

/* ---------------------------------------------------------------------------
 * Batched form: many rectified pairs, each with its own size and disparity
 * range, run as one hipGraph launch.  Each pair's outputs are bit-identical
 * to the four single-frame calls above with the same parameters.
 * ------------------------------------------------------------------------- */

/* Parameters shared by every pair of a batch (meanings as above). */
typedef struct {
    int32_t win_w, win_h;        /* census window: (5,5) or (9,7)               */
    int32_t npaths;              /* 4 or 8                                      */
    int32_t p1, p2;              /* 0 <= p1 <= p2, npaths * (255 + p2) <= 65535 */
    int32_t lr_tolerance;        /* < 0: no LR check                            */
    int32_t median3x3;           /* 0 or 1                                      */
} sgm_params;

/* One pair of a batch.  Device pointers owned by the caller; they must stay
 * valid, and their shapes unchanged, for the life of the plan. */
typedef struct {
    const uint8_t* left;         /* uint8 [height][pitch_bytes]                 */
    const uint8_t* right;        /* uint8 [height][pitch_bytes]                 */
    int32_t width, height, pitch_bytes;
    int32_t ndisp;               /* 1 .. 256                                    */
    uint16_t* disp_out;          /* uint16 [height][width], 4-byte aligned      */
    uint16_t* disp_right_out;    /* uint16 [height][width] (D^R) or NULL        */
} sgm_pair;

typedef struct sgm_plan sgm_plan;

/* Device workspace a plan needs for these pairs with this tuning table (the
 * same table as sgm_batch_plan_create; it decides how the frames are grouped
 * into launches): every pair's intermediates plus the plan's work-list
 * tables.  0 on invalid arguments. */
size_t sgm_batch_workspace_bytes(const sgm_pair* pairs, int32_t n,
                                 const sgm_params* params, const char* tune_table);

/*
 * Lays the intermediates out in `workspace` (256-byte aligned, at least
 * sgm_batch_workspace_bytes bytes, owned by the caller and kept alive with
 * the plan), copies the work lists to the device (a synchronous copy), and
 * captures the whole batch into a hipGraph on a stream of its own.
 * tune_table: NULL, or a flat JSON object (written by the project's tuner)
 * with two kinds of entries:
 *   "WxHxD": n   the path-kernel lane-layout variant for pairs of that shape
 *                (other shapes use the library's default for their size, as
 *                the single-frame calls do);
 *   "chains": n  how many streams inside the graph the pairs of 100k pixels
 *                and more are spread over, 1..8 (default 2); pairs on
 *                different streams may overlap.
 * Neither ever changes results.
 * Errors: SGM_ERR_ARG, SGM_ERR_WORKSPACE, SGM_ERR_ALIGN, SGM_ERR_HIP.
 */
int32_t sgm_batch_plan_create(const sgm_pair* pairs, int32_t n,
                              const sgm_params* params, void* workspace,
                              size_t workspace_bytes, const char* tune_table,
                              sgm_plan** plan_out);

/* Number of path-kernel lane-layout variants for this disparity range (the
 * values a tuning table may give), >= 1; 0 for ndisp outside 1..256. */
int32_t sgm_aggregate_variants(int32_t ndisp);

/* Enqueues the captured batch on `stream` (one hipGraphLaunch).  Replays of
 * one plan must not overlap. */
int32_t sgm_batch_run(sgm_plan* plan, void* stream);

/* Number of pairs of a plan (0 for NULL). */
int32_t sgm_batch_frames(const sgm_plan* plan);

/* Releases the graph and the plan's stream; the workspace stays the
 * caller's.  Accepts NULL. */
void sgm_batch_plan_destroy(sgm_plan* plan);

/* ---------------------------------------------------------------------------
 * Exact consistency check (Sec. 2.1.3, occlusion detection; Sec. 3.1.3):
 * D^R is not approximated from S_bar (Eq. right_disparity) but computed from
 * scratch: the pair is swapped and flipped horizontally and matched again by
 * the same census, cost, aggregation and WTA; that map, flipped back, is D^R
 * in Eq. (LR_check).  The whole path from the two images:
 *   D^L  = WTA of (left, right)
 *   D^R(x, y) = WTA of (flip(right), flip(left)) at (width - 1 - x, y),
 *               flip(I)(x, y) = I(width - 1 - x, y)
 *   then Eq. (LR_check) with params->lr_tolerance (< 0: no check) and the
 *   3x3 median as in sgm_wta_lrc.
 *   left, right     uint8 [height][pitch_bytes] device images
 *   params          census window, path set, penalties, tolerance, median
 *                   (as sgm_params of the batched form)
 *   disp_out        uint16 [height][width], 4-byte aligned
 *   disp_right_out  uint16 [height][width] receiving the exact D^R, or NULL
 *   work            device scratch of sgm_disparity_exact_lr_work_bytes(...)
 *                   bytes, 256-byte aligned; contents on return unspecified
 * Errors: SGM_ERR_ARG, SGM_ERR_UNSUPPORTED (window), SGM_ERR_WORKSPACE,
 *         SGM_ERR_ALIGN, SGM_ERR_HIP.
 * ------------------------------------------------------------------------- */
int32_t sgm_disparity_exact_lr(const uint8_t* left, const uint8_t* right,
                               int32_t width, int32_t height, int32_t pitch_bytes,
                               int32_t ndisp, const sgm_params* params,
                               uint16_t* disp_out, uint16_t* disp_right_out,
                               void* work, size_t work_bytes, void* stream);

/* Bytes of `work` that sgm_disparity_exact_lr needs (0 on invalid
 * arguments). */
size_t sgm_disparity_exact_lr_work_bytes(int32_t width, int32_t height, int32_t ndisp,
                                         const sgm_params* params);

/* Human-readable name of a status code. */
const char* sgm_status_string(int32_t status);

/* hipError_t of the most recent SGM_ERR_HIP on the calling thread. */
int32_t sgm_last_hip_error(void);

/* ABI version, incremented on every incompatible change. */
int32_t sgm_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SGM_H */
