// aggregate.hip -- the sum over paths of Eq. (sgm_path_aggr) (Sec. 2.1.2)
// from the pair slices the path pass writes (paths.hip), the choice of the
// path pass's lane layout, and its launch, gfx950.
//
// A pair slice holds, per volume element, A_r + A_-r (uint8, P2 <= 127) or
// L_r + L_-r (uint16) for one pair of opposite directions; merge_kernel forms
// S_bar = R C + sum of the uint8 slices, or the sum of the uint16 ones, for
// the four-call form.  The streamlined form sums the slices inside the
// selection pass instead (wta_lrc.hip).
#include "sgm_internal.h"

namespace sgm {
namespace {

// S_bar of the kMergeChunk elements of block lb from the pair slices: uint8
// slices hold A_r + A_-r, so S_bar = R C + sum of the R/2 slices; uint16
// slices hold L_r + L_-r, so S_bar = their sum.  Each thread sums 16
// consecutive elements.
template <int NS>
__device__ __forceinline__ void merge_u8_block(const Frame& f, int lb) {
    const size_t n = (size_t)f.width * f.height * f.ndisp;
    const size_t e0 = (size_t)lb * kMergeChunk + (size_t)threadIdx.x * 16;
    const uint8_t* cost = f.cost;
    const uint8_t* slices = f.slices;
    uint16_t* agg = f.agg;
    if (e0 + 16 <= n) {
        const size_t i = e0 / 16;
        const uint4 c = reinterpret_cast<const uint4*>(cost)[i];
        uint4 a[NS];
#pragma unroll
        for (int r = 0; r < NS; ++r) a[r] = load_once16(slices + (size_t)r * f.slice_stride + 16 * i);
        uint32_t s[8];
        merge16<NS, 2 * NS>(c, a, s);
        reinterpret_cast<uint4*>(agg)[2 * i] = make_uint4(s[0], s[1], s[2], s[3]);
        reinterpret_cast<uint4*>(agg)[2 * i + 1] = make_uint4(s[4], s[5], s[6], s[7]);
    } else {
        for (size_t e = e0; e < n && e < e0 + 16; ++e) {
            uint32_t s = (uint32_t)cost[e] * (2 * NS);
            for (int r = 0; r < NS; ++r) s += slices[(size_t)r * f.slice_stride + e];
            agg[e] = (uint16_t)s;
        }
    }
}

template <int NS>
__device__ __forceinline__ void merge_u16_block(const Frame& f, int lb) {
    const size_t n = (size_t)f.width * f.height * f.ndisp;
    const size_t e0 = (size_t)lb * kMergeChunk + (size_t)threadIdx.x * 16;
    const uint16_t* slices = reinterpret_cast<const uint16_t*>(f.slices);
    uint16_t* agg = f.agg;
    if (e0 + 16 <= n) {
        uint4 a[NS][2];
#pragma unroll
        for (int r = 0; r < NS; ++r) {
            a[r][0] = load_once16(slices + (size_t)r * f.slice_stride + e0);
            a[r][1] = load_once16(slices + (size_t)r * f.slice_stride + e0 + 8);
        }
        uint32_t s[8];
        wide_sum16<NS>(a, s);
        reinterpret_cast<uint4*>(agg)[e0 / 8] = make_uint4(s[0], s[1], s[2], s[3]);
        reinterpret_cast<uint4*>(agg)[e0 / 8 + 1] = make_uint4(s[4], s[5], s[6], s[7]);
    } else {
        for (size_t e = e0; e < n && e < e0 + 16; ++e) {
            uint32_t s = 0;
            for (int r = 0; r < NS; ++r) s += slices[(size_t)r * f.slice_stride + e];
            agg[e] = (uint16_t)s;
        }
    }
}

// MODE: 0 / 1 = uint16 slices of 4 / 8 paths, 2 / 3 = uint8 slices of 4 / 8
template <int MODE>
__device__ __forceinline__ void merge_block(const Frame& f, int lb) {
    if constexpr (MODE == 0) merge_u16_block<2>(f, lb);
    else if constexpr (MODE == 1) merge_u16_block<4>(f, lb);
    else if constexpr (MODE == 2) merge_u8_block<2>(f, lb);
    else merge_u8_block<4>(f, lb);
}

template <int MODE>
__global__ __launch_bounds__(256) void merge_kernel(Frame f) {
    merge_block<MODE>(f, blockIdx.x);
}

template <int MODE>
__global__ __launch_bounds__(256) void merge_batch_kernel(WorkList wl) {
    for (int b = blockIdx.x; b < wl.total; b += gridDim.x) {
        const int fi = find_frame(wl, b);
        merge_block<MODE>(wl.frames[fi], b - wl.starts[fi]);
    }
}

int merge_mode(int npaths, int p2) { return (slices_u8(p2) ? 2 : 0) + (npaths == 8 ? 1 : 0); }

}  // namespace

// Launch of the path pass for the layout `l`: the layout's kernels live in
// their own object (paths.hip, compiled per layout).
hipError_t launch_paths_any(const Frame* one, const WorkList* wl, int ndisp, int variant, bool u8,
                            int nblocks, hipStream_t stream) {
    const PathLayout l = path_layout(ndisp, variant);
#define SGM_CASE(K)                                                                                  \
    if (l.nreg_h == kPathLayouts[K].nreg_h && l.lpl_h == kPathLayouts[K].lpl_h &&                   \
        l.nreg_o == kPathLayouts[K].nreg_o && l.lpl_o == kPathLayouts[K].lpl_o)                     \
        return one ? launch_paths_layout_id<K>(*one, ndisp, u8, nblocks, stream)                     \
                   : launch_paths_batch_layout_id<K>(*wl, ndisp, u8, nblocks, stream);
    SGM_CASE(0)
    SGM_CASE(1)
    SGM_CASE(2)
    SGM_CASE(3)
    SGM_CASE(4)
    SGM_CASE(5)
    SGM_CASE(6)
    SGM_CASE(7)
    SGM_CASE(8)
    SGM_CASE(9)
    SGM_CASE(10)
    SGM_CASE(11)
#undef SGM_CASE
    return hipErrorInvalidValue;
}

// Lane layouts per disparity range.  Variant 0 is the default; the others
// trade the horizontal chains' per-step latency (more lanes per line) against
// total VALU work (more disparities per lane).  All give identical results.
int path_variants(int ndisp) {
    if (ndisp <= 32) return 1;
    if (ndisp <= 64) return 2;
    if (ndisp <= 128) return 3;
    return 2;
}

PathLayout path_layout(int ndisp, int variant) {
    if (ndisp <= 2) return {1, 1, 1, 1};
    if (ndisp <= 4) return {1, 2, 2, 1};
    if (ndisp <= 8) return {1, 4, 4, 1};
    if (ndisp <= 16) return {1, 8, 4, 2};
    if (ndisp <= 32) return {1, 16, 4, 4};
    if (ndisp <= 64) return variant == 1 ? PathLayout{2, 16, 4, 8} : PathLayout{1, 32, 4, 8};
    if (ndisp <= 128) {
        if (variant == 1) return {2, 32, 4, 16};
        if (variant == 2) return {1, 64, 8, 8};
        return {1, 64, 4, 16};
    }
    return variant == 1 ? PathLayout{4, 32, 8, 16} : PathLayout{2, 64, 8, 16};
}

// Variant used when none is asked for (variant < 0): the layout the tuner
// measured fastest for frames of this size class.  Large frames have enough
// horizontal lines to trade per-step latency for fewer instructions.
int default_variant(int width, int height, int ndisp) {
    const long px = (long)width * height;
    if (ndisp <= 32) return 0;
    if (ndisp > 128) return px >= 400000 ? 1 : 0;    // 1242x375, 1920x1080 at D = 256
    if (px >= 1500000) return 1;
    if (ndisp > 64 && px >= 400000) return 2;
    return 0;
}

int path_horizontal_blocks(int width, int height, int ndisp, int variant) {
    const PathLayout l = path_layout(ndisp, variant);
    return pair_blocks(0, width, height, l.lpl_h, l.lpl_o);
}

int path_blocks(int width, int height, int ndisp, int npaths, int variant) {
    const PathLayout l = path_layout(ndisp, variant);
    int nb = 0;
    for (int q = 0; q < npaths / 2; ++q) nb += pair_blocks(q, width, height, l.lpl_h, l.lpl_o);
    return nb;
}

// Slices start on 256-element boundaries so every vector access is aligned.
size_t aggregate_slice_elems(int width, int height, int ndisp) {
    const size_t n = (size_t)width * height * ndisp;
    return (n + 255) / 256 * 256;
}

size_t aggregate_work_bytes(int width, int height, int ndisp, int npaths, int p2) {
    return (size_t)(npaths / 2) * aggregate_slice_elems(width, height, ndisp) * (slices_u8(p2) ? 1 : 2);
}

hipError_t launch_paths(const Frame& f, hipStream_t stream) {
    const int variant = (f.variant >= 0 && f.variant < path_variants(f.ndisp))
                            ? f.variant
                            : default_variant(f.width, f.height, f.ndisp);
    const int nb = path_blocks(f.width, f.height, f.ndisp, f.npaths, variant);
    return launch_paths_any(&f, nullptr, f.ndisp, variant, slices_u8(f.p2), nb, stream);
}

hipError_t launch_aggregate(const Frame& f, hipStream_t stream) {
    hipError_t e = launch_paths(f, stream);
    if (e != hipSuccess) return e;
    const int mb = merge_blocks((size_t)f.width * f.height * f.ndisp);
    switch (merge_mode(f.npaths, f.p2)) {
        case 0: merge_kernel<0><<<mb, 256, 0, stream>>>(f); break;
        case 1: merge_kernel<1><<<mb, 256, 0, stream>>>(f); break;
        case 2: merge_kernel<2><<<mb, 256, 0, stream>>>(f); break;
        default: merge_kernel<3><<<mb, 256, 0, stream>>>(f); break;
    }
    return hipGetLastError();
}

hipError_t launch_paths_batch(const WorkList& wl, int ndisp, int npaths, int p2, int variant,
                              hipStream_t stream) {
    (void)npaths;
    if (variant < 0 || variant >= path_variants(ndisp)) variant = 0;
    return launch_paths_any(nullptr, &wl, ndisp, variant, slices_u8(p2), wl.total, stream);
}

hipError_t launch_merge_batch(const WorkList& wl, int npaths, int p2, hipStream_t stream) {
    const int grid = persistent_grid(wl.total);
    switch (merge_mode(npaths, p2)) {
        case 0: merge_batch_kernel<0><<<grid, 256, 0, stream>>>(wl); break;
        case 1: merge_batch_kernel<1><<<grid, 256, 0, stream>>>(wl); break;
        case 2: merge_batch_kernel<2><<<grid, 256, 0, stream>>>(wl); break;
        default: merge_batch_kernel<3><<<grid, 256, 0, stream>>>(wl); break;
    }
    return hipGetLastError();
}

}  // namespace sgm
