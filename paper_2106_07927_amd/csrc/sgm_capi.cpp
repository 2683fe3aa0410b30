// sgm_capi.cpp -- the extern "C" entry points of include/sgm.h: argument
// validation, then the kernel launches.  Nothing here allocates memory or
// synchronises; every check happens before the first launch.
#include "sgm.h"

#include <hip/hip_runtime.h>

#include "sgm_internal.h"

namespace {

thread_local int32_t g_last_hip_error = 0;

constexpr int32_t kMaxSide = 32768;   // keeps every grid dimension in range

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

bool bad_size(int32_t width, int32_t height) {
    return width < 1 || height < 1 || width > kMaxSide || height > kMaxSide;
}

// volumes are addressed with 32-bit element offsets inside the kernels
bool bad_volume(int32_t width, int32_t height, int32_t ndisp) {
    return ndisp < 1 || ndisp > SGM_MAX_NDISP ||
           (int64_t)width * height * ndisp > (int64_t)SGM_MAX_VOLUME;
}

// P1 <= P2 makes the four-term recursion exact; the bound keeps every S_bar
// inside uint16
bool bad_penalties(int32_t npaths, int32_t p1, int32_t p2) {
    if (npaths != 4 && npaths != 8) return true;
    if (p1 < 0 || p2 < p1) return true;
    return (int64_t)npaths * (255 + (int64_t)p2) > 65535;
}

int32_t hip_status(hipError_t e) {
    if (e == hipSuccess) return SGM_OK;
    g_last_hip_error = (int32_t)e;
    return SGM_ERR_HIP;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Workspace of sgm_aggregate_select: path slices, S_bar (only where the fused
// selection does not apply), D^R keys, D^L.  Returns the total bytes.
size_t select_layout(int32_t width, int32_t height, int32_t ndisp, int32_t npaths, int32_t p2,
                     size_t* agg_off, size_t* keys_off, size_t* dl_off) {
    const size_t n = (size_t)width * height;
    size_t off = align256(sgm::aggregate_work_bytes(width, height, ndisp, npaths, p2));
    *agg_off = off;
    if (!sgm::fused_select_supported(ndisp, npaths, p2)) off += align256(2 * n * (size_t)ndisp);
    *keys_off = off;
    off += align256(4 * n);
    *dl_off = off;
    off += align256(2 * n);
    return off;
}

// The aggregation and selection of one frame: fused where it applies, else
// sgm_aggregate + sgm_wta_lrc with S_bar in f.agg.
hipError_t run_select(const sgm::Frame& f, hipStream_t s, bool fine = false) {
    if (sgm::fused_select_supported(f.ndisp, f.npaths, f.p2))
        return sgm::launch_aggregate_select(f, s, fine);
    const hipError_t e = sgm::launch_aggregate(f, s);
    if (e != hipSuccess) return e;
    return fine ? sgm::launch_wta_lrc_fine(f, s) : sgm::launch_wta_lrc(f, s);
}

bool good_params(const sgm_params* p) {
    if (!p) return false;
    if (!((p->win_w == 5 && p->win_h == 5) || (p->win_w == 9 && p->win_h == 7))) return false;
    if (bad_penalties(p->npaths, p->p1, p->p2)) return false;
    return p->median3x3 == 0 || p->median3x3 == 1;
}

// Workspace of the exact-check path, byte offsets.
struct ExactLayout {
    size_t ref, mat, census_left, census_right, cost, select, agg, keys, dl, disp_left,
        disp_flipped;
};

size_t exact_layout(int32_t width, int32_t height, int32_t ndisp, const sgm_params* p,
                    ExactLayout* l) {
    const size_t n = (size_t)width * height;
    size_t off = 0;
    l->ref = off;
    off += align256(n);
    l->mat = off;
    off += align256(n);
    l->census_left = off;
    off += align256(8 * n);
    l->census_right = off;
    off += align256(8 * n);
    l->cost = off;
    off += align256(n * (size_t)ndisp);
    l->select = off;
    off += select_layout(width, height, ndisp, p->npaths, p->p2, &l->agg, &l->keys, &l->dl);
    l->disp_left = off;
    off += align256(2 * n);
    l->disp_flipped = off;
    off += align256(2 * n);
    return off;
}

}  // namespace

namespace sgm {
// Records a HIP error for sgm_last_hip_error (other source files' entry points).
int32_t record_hip_error(hipError_t e) { return hip_status(e); }
}  // namespace sgm

extern "C" {

int32_t sgm_abi_version(void) { return 4; }

const char* sgm_status_string(int32_t status) {
    switch (status) {
        case SGM_OK: return "SGM_OK";
        case SGM_ERR_ARG: return "SGM_ERR_ARG: invalid argument";
        case SGM_ERR_UNSUPPORTED:
            return "SGM_ERR_UNSUPPORTED: window must be 5x5 or 9x7 (census) or 5 or 9 (NCC)";
        case SGM_ERR_ALIGN: return "SGM_ERR_ALIGN: misaligned buffer";
        case SGM_ERR_HIP: return "SGM_ERR_HIP: HIP launch failed";
        case SGM_ERR_WORKSPACE: return "SGM_ERR_WORKSPACE: workspace missing or too small";
        case SGM_ERR_TOO_LARGE:
            return "SGM_ERR_TOO_LARGE: the frame needs more than the fixed scratch "
                   "(SGM_NOALLOC_SCRATCH_BYTES)";
        default: return "unknown sgm status";
    }
}

int32_t sgm_last_hip_error(void) { return g_last_hip_error; }

int32_t sgm_census(const uint8_t* img, int32_t width, int32_t height, int32_t pitch_bytes,
                   int32_t win_w, int32_t win_h, uint64_t* census_out, void* stream) {
    if (!img || !census_out || bad_size(width, height) || pitch_bytes < width) return SGM_ERR_ARG;
    if (!((win_w == 5 && win_h == 5) || (win_w == 9 && win_h == 7))) return SGM_ERR_UNSUPPORTED;
    if (!aligned(census_out, 8)) return SGM_ERR_ALIGN;
    sgm::Frame f{};
    f.width = width;
    f.height = height;
    f.pitch = pitch_bytes;
    f.win_w = win_w;
    f.win_h = win_h;
    f.left = img;
    f.census_left = census_out;
    return hip_status(sgm::launch_census(f, false, as_stream(stream)));
}

int32_t sgm_census_pair(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                        int32_t pitch_bytes, int32_t win_w, int32_t win_h,
                        uint64_t* census_left_out, uint64_t* census_right_out, void* stream) {
    if (!left || !right || !census_left_out || !census_right_out || bad_size(width, height) ||
        pitch_bytes < width || census_left_out == census_right_out)
        return SGM_ERR_ARG;
    if (!((win_w == 5 && win_h == 5) || (win_w == 9 && win_h == 7))) return SGM_ERR_UNSUPPORTED;
    if (!aligned(census_left_out, 8) || !aligned(census_right_out, 8)) return SGM_ERR_ALIGN;
    sgm::Frame f{};
    f.width = width;
    f.height = height;
    f.pitch = pitch_bytes;
    f.win_w = win_w;
    f.win_h = win_h;
    f.left = left;
    f.right = right;
    f.census_left = census_left_out;
    f.census_right = census_right_out;
    return hip_status(sgm::launch_census_pair(f, as_stream(stream)));
}

int32_t sgm_cost(const uint64_t* census_left, const uint64_t* census_right, int32_t width,
                 int32_t height, int32_t ndisp, uint8_t* cost_out, void* stream) {
    if (!census_left || !census_right || !cost_out || bad_size(width, height)) return SGM_ERR_ARG;
    if (bad_volume(width, height, ndisp)) return SGM_ERR_ARG;
    if (!aligned(census_left, 8) || !aligned(census_right, 8) || !aligned(cost_out, 16))
        return SGM_ERR_ALIGN;
    sgm::Frame f{};
    f.width = width;
    f.height = height;
    f.ndisp = ndisp;
    f.census_left = const_cast<uint64_t*>(census_left);
    f.census_right = const_cast<uint64_t*>(census_right);
    f.cost = cost_out;
    return hip_status(sgm::launch_cost(f, as_stream(stream)));
}

int32_t sgm_cost_ncc(const uint8_t* left, const uint8_t* right, int32_t width, int32_t height,
                     int32_t pitch_bytes, int32_t win, int32_t ndisp, uint8_t* cost_out,
                     void* stream) {
    if (!left || !right || !cost_out || bad_size(width, height) || pitch_bytes < width)
        return SGM_ERR_ARG;
    if (bad_volume(width, height, ndisp)) return SGM_ERR_ARG;
    if (win != 5 && win != 9) return SGM_ERR_UNSUPPORTED;
    if (!aligned(cost_out, 16)) return SGM_ERR_ALIGN;
    return hip_status(sgm::launch_ncc_cost(left, right, width, height, pitch_bytes, win, ndisp,
                                           cost_out, as_stream(stream)));
}

size_t sgm_aggregate_work_bytes(int32_t width, int32_t height, int32_t ndisp, int32_t npaths,
                                int32_t p2) {
    if (bad_size(width, height) || bad_volume(width, height, ndisp) || bad_penalties(npaths, 0, p2))
        return 0;
    return sgm::aggregate_work_bytes(width, height, ndisp, npaths, p2);
}

int32_t sgm_aggregate(const uint8_t* cost, int32_t width, int32_t height, int32_t ndisp,
                      int32_t npaths, int32_t p1, int32_t p2, uint16_t* agg_out, void* work,
                      size_t work_bytes, void* stream) {
    if (!cost || !agg_out || bad_size(width, height)) return SGM_ERR_ARG;
    if (bad_volume(width, height, ndisp) || bad_penalties(npaths, p1, p2)) return SGM_ERR_ARG;
    if (!work || work_bytes < sgm::aggregate_work_bytes(width, height, ndisp, npaths, p2))
        return SGM_ERR_WORKSPACE;
    if (!aligned(cost, 16) || !aligned(agg_out, 16) || !aligned(work, 16)) return SGM_ERR_ALIGN;
    sgm::Frame f{};
    f.width = width;
    f.height = height;
    f.ndisp = ndisp;
    f.npaths = npaths;
    f.p1 = p1;
    f.p2 = p2;
    f.variant = -1;
    f.cost = const_cast<uint8_t*>(cost);
    f.slices = static_cast<uint8_t*>(work);
    f.slice_stride = sgm::aggregate_slice_elems(width, height, ndisp);
    f.agg = agg_out;
    return hip_status(sgm::launch_aggregate(f, as_stream(stream)));
}

size_t sgm_wta_lrc_work_elems(int32_t width, int32_t height) {
    if (bad_size(width, height)) return 0;
    return (size_t)3 * (size_t)width * (size_t)height;
}

int32_t sgm_wta_lrc(const uint16_t* agg, int32_t width, int32_t height, int32_t ndisp,
                    int32_t lr_tolerance, int32_t median3x3, uint16_t* disp_out,
                    uint16_t* disp_right_out, uint16_t* work, void* stream) {
    if (!agg || !disp_out || bad_size(width, height)) return SGM_ERR_ARG;
    if (bad_volume(width, height, ndisp)) return SGM_ERR_ARG;
    if (median3x3 != 0 && median3x3 != 1) return SGM_ERR_ARG;
    if (!work) return SGM_ERR_WORKSPACE;
    if (!aligned(agg, 16) || !aligned(disp_out, 4) || !aligned(work, 4) ||
        (disp_right_out && !aligned(disp_right_out, 4)))
        return SGM_ERR_ALIGN;
    const size_t n = (size_t)width * height;
    sgm::Frame f{};
    f.width = width;
    f.height = height;
    f.ndisp = ndisp;
    f.lr_tolerance = lr_tolerance;
    f.median3x3 = median3x3;
    f.agg = const_cast<uint16_t*>(agg);
    f.right_keys = reinterpret_cast<uint32_t*>(work);          // n uint32
    f.disp_left = work + 2 * n;                                 // n uint16
    f.disp = disp_out;
    f.disp_right = disp_right_out;
    return hip_status(sgm::launch_wta_lrc(f, as_stream(stream)));
}

size_t sgm_aggregate_select_work_bytes(int32_t width, int32_t height, int32_t ndisp,
                                       int32_t npaths, int32_t p2) {
    if (bad_size(width, height) || bad_volume(width, height, ndisp) || bad_penalties(npaths, 0, p2))
        return 0;
    size_t a, k, d;
    return select_layout(width, height, ndisp, npaths, p2, &a, &k, &d);
}

int32_t sgm_aggregate_select(const uint8_t* cost, int32_t width, int32_t height, int32_t ndisp,
                             int32_t npaths, int32_t p1, int32_t p2, int32_t lr_tolerance,
                             int32_t median3x3, uint16_t* disp_out, uint16_t* disp_right_out,
                             void* work, size_t work_bytes, void* stream) {
    if (!cost || !disp_out || bad_size(width, height)) return SGM_ERR_ARG;
    if (bad_volume(width, height, ndisp) || bad_penalties(npaths, p1, p2)) return SGM_ERR_ARG;
    if (median3x3 != 0 && median3x3 != 1) return SGM_ERR_ARG;
    size_t agg_off, keys_off, dl_off;
    const size_t need = select_layout(width, height, ndisp, npaths, p2, &agg_off, &keys_off, &dl_off);
    if (!work || work_bytes < need) return SGM_ERR_WORKSPACE;
    if (!aligned(cost, 16) || !aligned(work, 256) || !aligned(disp_out, 4) ||
        (disp_right_out && !aligned(disp_right_out, 4)))
        return SGM_ERR_ALIGN;
    char* base = static_cast<char*>(work);
    sgm::Frame f{};
    f.width = width;
    f.height = height;
    f.ndisp = ndisp;
    f.npaths = npaths;
    f.p1 = p1;
    f.p2 = p2;
    f.lr_tolerance = lr_tolerance;
    f.median3x3 = median3x3;
    f.variant = -1;
    f.cost = const_cast<uint8_t*>(cost);
    f.slices = reinterpret_cast<uint8_t*>(base);
    f.slice_stride = sgm::aggregate_slice_elems(width, height, ndisp);
    f.right_keys = reinterpret_cast<uint32_t*>(base + keys_off);
    f.disp_left = reinterpret_cast<uint16_t*>(base + dl_off);
    f.disp = disp_out;
    f.disp_right = disp_right_out;
    f.agg = reinterpret_cast<uint16_t*>(base + agg_off);
    return hip_status(run_select(f, as_stream(stream)));
}

size_t sgm_aggregate_select_subpixel_work_bytes(int32_t width, int32_t height, int32_t ndisp,
                                                int32_t npaths, int32_t p2) {
    const size_t base = sgm_aggregate_select_work_bytes(width, height, ndisp, npaths, p2);
    return base ? base + align256(4 * (size_t)width * height) : 0;
}

int32_t sgm_aggregate_select_subpixel(const uint8_t* cost, int32_t width, int32_t height,
                                      int32_t ndisp, int32_t npaths, int32_t p1, int32_t p2,
                                      int32_t lr_tolerance, int32_t median3x3, float* disp_out,
                                      uint16_t* disp_right_out, void* work, size_t work_bytes,
                                      void* stream) {
    if (!cost || !disp_out || bad_size(width, height)) return SGM_ERR_ARG;
    if (bad_volume(width, height, ndisp) || bad_penalties(npaths, p1, p2)) return SGM_ERR_ARG;
    if (median3x3 != 0 && median3x3 != 1) return SGM_ERR_ARG;
    size_t agg_off, keys_off, dl_off;
    const size_t fine_off = select_layout(width, height, ndisp, npaths, p2, &agg_off, &keys_off, &dl_off);
    const size_t need = fine_off + align256(4 * (size_t)width * height);
    if (!work || work_bytes < need) return SGM_ERR_WORKSPACE;
    if (!aligned(cost, 16) || !aligned(work, 256) || !aligned(disp_out, 4) ||
        (disp_right_out && !aligned(disp_right_out, 4)))
        return SGM_ERR_ALIGN;
    char* base = static_cast<char*>(work);
    sgm::Frame f{};
    f.width = width;
    f.height = height;
    f.ndisp = ndisp;
    f.npaths = npaths;
    f.p1 = p1;
    f.p2 = p2;
    f.lr_tolerance = lr_tolerance;
    f.median3x3 = median3x3;
    f.variant = -1;
    f.cost = const_cast<uint8_t*>(cost);
    f.slices = reinterpret_cast<uint8_t*>(base);
    f.slice_stride = sgm::aggregate_slice_elems(width, height, ndisp);
    f.agg = reinterpret_cast<uint16_t*>(base + agg_off);
    f.right_keys = reinterpret_cast<uint32_t*>(base + keys_off);
    f.disp_left = reinterpret_cast<uint16_t*>(base + dl_off);
    f.fine_left = reinterpret_cast<float*>(base + fine_off);
    f.disp_fine = disp_out;
    f.disp_right = disp_right_out;
    return hip_status(run_select(f, as_stream(stream), true));
}

size_t sgm_disparity_exact_lr_work_bytes(int32_t width, int32_t height, int32_t ndisp,
                                         const sgm_params* params) {
    if (bad_size(width, height) || bad_volume(width, height, ndisp) || !good_params(params)) return 0;
    ExactLayout l;
    return exact_layout(width, height, ndisp, params, &l);
}

int32_t sgm_disparity_exact_lr(const uint8_t* left, const uint8_t* right, int32_t width,
                               int32_t height, int32_t pitch_bytes, int32_t ndisp,
                               const sgm_params* params, uint16_t* disp_out,
                               uint16_t* disp_right_out, void* work, size_t work_bytes,
                               void* stream) {
    if (!left || !right || !disp_out || bad_size(width, height) || pitch_bytes < width)
        return SGM_ERR_ARG;
    if (bad_volume(width, height, ndisp) || !params) return SGM_ERR_ARG;
    if (!((params->win_w == 5 && params->win_h == 5) || (params->win_w == 9 && params->win_h == 7)))
        return SGM_ERR_UNSUPPORTED;
    if (!good_params(params)) return SGM_ERR_ARG;
    ExactLayout l;
    const size_t need = exact_layout(width, height, ndisp, params, &l);
    if (!work || work_bytes < need) return SGM_ERR_WORKSPACE;
    if (!aligned(work, 256) || !aligned(disp_out, 4) || (disp_right_out && !aligned(disp_right_out, 4)))
        return SGM_ERR_ALIGN;
    char* base = static_cast<char*>(work);
    const hipStream_t s = as_stream(stream);
    sgm::Frame f{};
    f.width = width;
    f.height = height;
    f.ndisp = ndisp;
    f.win_w = params->win_w;
    f.win_h = params->win_h;
    f.npaths = params->npaths;
    f.p1 = params->p1;
    f.p2 = params->p2;
    f.variant = -1;
    f.census_left = reinterpret_cast<uint64_t*>(base + l.census_left);
    f.census_right = reinterpret_cast<uint64_t*>(base + l.census_right);
    f.cost = reinterpret_cast<uint8_t*>(base + l.cost);
    f.slices = reinterpret_cast<uint8_t*>(base + l.select);
    f.slice_stride = sgm::aggregate_slice_elems(width, height, ndisp);
    f.agg = reinterpret_cast<uint16_t*>(base + l.select + l.agg);
    f.right_keys = reinterpret_cast<uint32_t*>(base + l.select + l.keys);
    f.disp_left = reinterpret_cast<uint16_t*>(base + l.select + l.dl);
    f.lr_tolerance = -1;            // both passes: plain WTA maps
    f.median3x3 = 0;
    f.disp_right = nullptr;
    uint16_t* dl = reinterpret_cast<uint16_t*>(base + l.disp_left);
    uint16_t* flipped = reinterpret_cast<uint16_t*>(base + l.disp_flipped);
    uint8_t* ref = reinterpret_cast<uint8_t*>(base + l.ref);
    uint8_t* mat = reinterpret_cast<uint8_t*>(base + l.mat);
    hipError_t e = hipSuccess;
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
        if (pass == 0) {
            f.left = left;
            f.right = right;
            f.pitch = pitch_bytes;
            f.disp = dl;
        } else {
            e = sgm::launch_flip_pair(left, right, width, height, pitch_bytes, ref, mat, s);
            f.left = ref;
            f.right = mat;
            f.pitch = width;
            f.disp = flipped;
        }
        if (e == hipSuccess) e = sgm::launch_census_pair(f, s);
        if (e == hipSuccess) e = sgm::launch_cost(f, s);
        if (e == hipSuccess) e = run_select(f, s);
    }
    if (e == hipSuccess)
        e = sgm::launch_check_exact(dl, flipped, width, height, params->lr_tolerance,
                                    params->median3x3, disp_out, disp_right_out, s);
    return hip_status(e);
}

}  // extern "C"
