// sgm_internal.h -- shared pieces of the gfx950 kernels behind include/sgm.h.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>

namespace sgm {

// ---------------------------------------------------------------------------
// Packed 16-bit helpers.  Two uint16 lanes live in one 32-bit VGPR; the
// vector type makes clang emit v_pk_{add,sub,min,max}_u16.
// ---------------------------------------------------------------------------
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) { return as_u32(as_u16x2(a) + as_u16x2(b)); }
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) { return as_u32(as_u16x2(a) - as_u16x2(b)); }
__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b) {
    return as_u32(__builtin_elementwise_min(as_u16x2(a), as_u16x2(b)));
}
__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
    return as_u32(__builtin_elementwise_max(as_u16x2(a), as_u16x2(b)));
}
// (lo, hi) of the result = (hi of b, lo of a): the pair one element down.
__device__ __forceinline__ uint32_t pk_shift_in(uint32_t a, uint32_t b) {
    return __builtin_amdgcn_alignbit(a, b, 16);
}
__host__ __device__ __forceinline__ uint32_t pk_splat(uint32_t v16) { return v16 | (v16 << 16); }

// 16 bytes that the path reads exactly once (penalty slices, S_bar): a
// nontemporal load streams them past the caches, which keeps the lines that
// are read again (the cost volume) resident.
__device__ __forceinline__ uint4 load_once16(const void* p) {
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------------------------
// Path slices.  The path pass writes one slice per pair of opposite
// directions (r, -r).  With P2 <= 127 a slice holds A_r + A_-r, the sum of
// the two penalty parts A = L - C in [0, P2], as uint8 (exact: at most 254);
// otherwise it holds L_r + L_-r as uint16 (exact: npaths (255 + P2) < 2^16).
// ---------------------------------------------------------------------------
__host__ __device__ inline bool slices_u8(int p2) { return p2 <= 127; }

// Path sum of 16 consecutive volume elements (Eq. sgm_path_aggr) from NS
// uint8 pair slices: S = MUL * C + sum of the slices, MUL = npaths.  Bytes
// are split into even / odd 16-bit lanes, so plain 32-bit adds carry two
// sums per register with no carry between them (S <= 8 * 255 + 4 * 254 <
// 2^16).  `out` holds the 16 sums as packed pairs in memory order.
template <int NS, int MUL>
__device__ __forceinline__ void merge16(const uint4& c, const uint4 (&a)[NS], uint32_t (&out)[8]) {
    const uint32_t cw[4] = {c.x, c.y, c.z, c.w};
    uint32_t ev[4], od[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        ev[q] = (cw[q] & 0x00FF00FFu) * (uint32_t)MUL;
        od[q] = ((cw[q] >> 8) & 0x00FF00FFu) * (uint32_t)MUL;
    }
#pragma unroll
    for (int r = 0; r < NS; ++r) {
        const uint32_t aw[4] = {a[r].x, a[r].y, a[r].z, a[r].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ev[q] += aw[q] & 0x00FF00FFu;
            od[q] += (aw[q] >> 8) & 0x00FF00FFu;
        }
    }
    // interleave back: elements e0 o0 e1 o1 of every source word
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        out[2 * q] = __builtin_amdgcn_perm(od[q], ev[q], 0x05040100u);
        out[2 * q + 1] = __builtin_amdgcn_perm(od[q], ev[q], 0x07060302u);
    }
}

// Path sum of 16 consecutive volume elements from NS uint16 pair slices
// (two 16-byte blocks each): S = sum of the slices.
template <int NS>
__device__ __forceinline__ void wide_sum16(const uint4 (&a)[NS][2], uint32_t (&out)[8]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        uint32_t s[4] = {a[0][h].x, a[0][h].y, a[0][h].z, a[0][h].w};
#pragma unroll
        for (int r = 1; r < NS; ++r) {
            s[0] = pk_add(s[0], a[r][h].x);
            s[1] = pk_add(s[1], a[r][h].y);
            s[2] = pk_add(s[2], a[r][h].z);
            s[3] = pk_add(s[3], a[r][h].w);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) out[4 * h + q] = s[q];
    }
}

// ---------------------------------------------------------------------------
// DPP controls (GFX9 encoding).  All stay inside a 16-lane row.
// ---------------------------------------------------------------------------
enum : int {
    kDppQuadSwap1 = 0xB1,   // quad_perm [1,0,3,2]
    kDppQuadSwap2 = 0x4E,   // quad_perm [2,3,0,1]
    kDppRowShl1 = 0x101,
    kDppRowShr1 = 0x111,
    kDppRowRor1 = 0x121,
    kDppRowMirror = 0x140,
    kDppRowHalfMirror = 0x141,
};

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, 0xF, 0xF, false);
}

// Minimum over the GROUP consecutive lanes of an aligned group (GROUP a power
// of two, at most 16), returned to every lane of the group.
template <int GROUP>
__device__ __forceinline__ uint32_t group_min(uint32_t v) {
    if constexpr (GROUP >= 2) v = min(v, dpp<kDppQuadSwap1>(0u, v));
    if constexpr (GROUP >= 4) v = min(v, dpp<kDppQuadSwap2>(0u, v));
    if constexpr (GROUP >= 8) v = min(v, dpp<kDppRowHalfMirror>(0u, v));
    if constexpr (GROUP >= 16) v = min(v, dpp<kDppRowMirror>(0u, v));
    return v;
}

// Value of the next lane of the group; the group's last lane gets `edge`.
template <int GROUP>
__device__ __forceinline__ uint32_t group_next(uint32_t v, uint32_t edge, bool last) {
    if constexpr (GROUP == 1) {
        return edge;
    } else {
        uint32_t r = dpp<kDppRowShl1>(edge, v);
        if constexpr (GROUP < 16) r = last ? edge : r;
        return r;
    }
}

// Value of the previous lane of the group; the group's first lane gets `edge`.
template <int GROUP>
__device__ __forceinline__ uint32_t group_prev(uint32_t v, uint32_t edge, bool first) {
    if constexpr (GROUP == 1) {
        return edge;
    } else {
        uint32_t r = dpp<kDppRowShr1>(edge, v);
        if constexpr (GROUP < 16) r = first ? edge : r;
        return r;
    }
}

// ---------------------------------------------------------------------------
// One stereo frame: sizes, parameters and every device buffer of the path.
// Single-frame calls fill the fields their stage needs and pass the struct by
// value; batched launches read an array of them from device memory.
// ---------------------------------------------------------------------------
struct Frame {
    int32_t width, height, ndisp, pitch;
    int32_t win_w, win_h, npaths, p1, p2, lr_tolerance, median3x3;
    int32_t variant;                 // lane-layout variant of the path kernel (< 0: default)
    int32_t paths_fill_keys;         // the path kernel also sets right_keys to all ones
    const uint8_t* left;
    const uint8_t* right;
    uint64_t* census_left;
    uint64_t* census_right;
    uint8_t* cost;
    uint8_t* slices;                 // npaths path slices
    size_t slice_stride;             // elements between slices
    uint16_t* agg;
    uint32_t* right_keys;            // D^R keys, width*height
    uint16_t* disp_left;             // D^L, width*height
    uint16_t* disp;
    uint16_t* disp_right;            // may be null
    float* fine_left;                // subpixel forms: refined D^L, width*height
    float* disp_fine;                // subpixel forms: output map
};

// A launch over several frames: block b of the launch belongs to the frame f
// with starts[f] <= b < starts[f + 1] and is its block b - starts[f].
struct WorkList {
    const Frame* frames;
    const int32_t* starts;           // nframes + 1 entries
    int32_t nframes;
    int32_t total;                   // starts[nframes]
    // optional: total (frame, block) pairs giving the launch order of the
    // blocks (longest first); when set, block b of the launch is items[2b],
    // items[2b + 1] instead of the frame-major order of starts
    const int32_t* items;
};

__device__ __forceinline__ int find_frame(const WorkList& wl, int b) {
    int lo = 0, hi = wl.nframes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wl.starts[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Grid of a persistent launch: enough blocks to fill the GPU, never more than
// there is work.
inline int persistent_grid(int total_blocks, int per_cu = 8) {
    return std::max(1, std::min(total_blocks, 256 * per_cu));
}

// ---------------------------------------------------------------------------
// Stage geometry (blocks per frame), shared by host planning and kernels.
// ---------------------------------------------------------------------------
constexpr int kCensusTileW = 64;
constexpr int kCensusTileH = 16;
__host__ __device__ inline int census_blocks_x(int w) { return (w + kCensusTileW - 1) / kCensusTileW; }
__host__ __device__ inline int census_blocks(int w, int h) {
    return census_blocks_x(w) * ((h + kCensusTileH - 1) / kCensusTileH);
}

constexpr int kCostPix = 128;
__host__ __device__ inline int cost_blocks_x(int w) { return (w + kCostPix - 1) / kCostPix; }

constexpr int kSelectSeg = 128;   // pixels per wave segment
constexpr int kSelectWaves = 4;
__host__ __device__ inline int select_blocks_x(int w) {
    const int segs = (w + kSelectSeg - 1) / kSelectSeg;
    return (segs + kSelectWaves - 1) / kSelectWaves;
}

// pixels of one row per block of the fused path-sum + selection pass
// (at most 8192 volume elements per tile, so every thread sums two 16-byte
// blocks: 64 pixels up to D = 128, 32 beyond)
constexpr int kFusedTile = 64;
constexpr int kMaxFusedD = 256;
__host__ __device__ inline int fused_tile_px(int ndisp) { return ndisp > 128 ? 32 : kFusedTile; }
__host__ __device__ inline int fused_blocks_x(int w, int ndisp) {
    const int t = fused_tile_px(ndisp);
    return (w + t - 1) / t;
}

constexpr int kMedianTileW = 64;
constexpr int kMedianTileH = 4;
__host__ __device__ inline int median_blocks_x(int w) { return (w + kMedianTileW - 1) / kMedianTileW; }
__host__ __device__ inline int median_blocks(int w, int h) {
    return median_blocks_x(w) * ((h + kMedianTileH - 1) / kMedianTileH);
}

constexpr int kMergeChunk = 256 * 16;     // elements per merge block
__host__ __device__ inline int merge_blocks(size_t n) { return (int)((n + kMergeChunk - 1) / kMergeChunk); }

constexpr int kFillChunk = 256 * 16;
__host__ __device__ inline int fill_blocks(size_t n) { return (int)((n + kFillChunk - 1) / kFillChunk); }

// Lane layout of the path kernel for one disparity range and variant.
struct PathLayout {
    int nreg_h, lpl_h;    // horizontal lines
    int nreg_o, lpl_o;    // vertical and diagonal lines
};

// Every layout the library builds (paths.hip is compiled once per entry).
constexpr int kNumPathLayouts = 12;
constexpr PathLayout kPathLayouts[kNumPathLayouts] = {
    {1, 1, 1, 1}, {1, 2, 2, 1}, {1, 4, 4, 1}, {1, 8, 4, 2}, {1, 16, 4, 4}, {1, 32, 4, 8},
    {2, 16, 4, 8}, {1, 64, 4, 16}, {2, 32, 4, 16}, {1, 64, 8, 8}, {2, 64, 8, 16}, {4, 32, 8, 16},
};

// The path pass for layout kPathLayouts[ID] (paths.hip compiled per layout,
// in two objects): the single-frame kernel for one frame, or the work-list
// kernel for a batch.
template <int ID>
hipError_t launch_paths_layout_id(const Frame& one, int ndisp, bool u8, int nblocks, hipStream_t stream);
template <int ID>
hipError_t launch_paths_batch_layout_id(const WorkList& wl, int ndisp, bool u8, int nblocks,
                                        hipStream_t stream);
#define SGM_DECLARE_PATH_LAYOUT(K)                                                              \
    template <>                                                                                 \
    hipError_t launch_paths_layout_id<K>(const Frame&, int, bool, int, hipStream_t);            \
    template <>                                                                                 \
    hipError_t launch_paths_batch_layout_id<K>(const WorkList&, int, bool, int, hipStream_t);
SGM_DECLARE_PATH_LAYOUT(0)
SGM_DECLARE_PATH_LAYOUT(1)
SGM_DECLARE_PATH_LAYOUT(2)
SGM_DECLARE_PATH_LAYOUT(3)
SGM_DECLARE_PATH_LAYOUT(4)
SGM_DECLARE_PATH_LAYOUT(5)
SGM_DECLARE_PATH_LAYOUT(6)
SGM_DECLARE_PATH_LAYOUT(7)
SGM_DECLARE_PATH_LAYOUT(8)
SGM_DECLARE_PATH_LAYOUT(9)
SGM_DECLARE_PATH_LAYOUT(10)
SGM_DECLARE_PATH_LAYOUT(11)
#undef SGM_DECLARE_PATH_LAYOUT

// Pairs of opposite path directions.  Pair q's forward step r (the reverse
// wave walks -r): pairs 0, 1 are the 4-path set (Sec. 3.1.4), pairs 2, 3 add
// the diagonals.  Pair 0 has one line per row, the others one per column
// (the diagonals' lines wrap at the left / right border).
__host__ __device__ inline void pair_dir(int q, int* dx, int* dy) {
    constexpr int kDirs[4][2] = {{1, 0}, {0, 1}, {1, 1}, {-1, 1}};
    *dx = kDirs[q][0];
    *dy = kDirs[q][1];
}

__host__ __device__ inline int pair_lines(int q, int width, int height) { return q == 0 ? height : width; }

// Blocks of pair q in the path pass: one block (the forward and the reverse
// waves of two line groups) per two waves' worth of lines.
__host__ __device__ inline int pair_blocks(int q, int width, int height, int lpl_h, int lpl_o) {
    const int lpb = 2 * (64 / (q == 0 ? lpl_h : lpl_o));
    return (pair_lines(q, width, height) + lpb - 1) / lpb;
}
int path_variants(int ndisp);                       // number of variants (>= 1)
int default_variant(int width, int height, int ndisp);
PathLayout path_layout(int ndisp, int variant);
int path_blocks(int width, int height, int ndisp, int npaths, int variant);
// blocks of the horizontal directions, which come first in a frame's block order
int path_horizontal_blocks(int width, int height, int ndisp, int variant);
size_t aggregate_slice_elems(int width, int height, int ndisp);
size_t aggregate_work_bytes(int width, int height, int ndisp, int npaths, int p2);

// ---------------------------------------------------------------------------
// Launchers.  Single-frame forms take the frame by value; batched forms take
// a work list whose frames all share the template parameters of the stage
// (same window for census, same D for cost / paths / select).
// ---------------------------------------------------------------------------
hipError_t launch_census(const Frame& f, bool right, hipStream_t stream);
hipError_t launch_census_pair(const Frame& f, hipStream_t stream);
hipError_t launch_cost(const Frame& f, hipStream_t stream);
hipError_t launch_ncc_cost(const uint8_t* left, const uint8_t* right, int width, int height,
                           int pitch, int win, int ndisp, uint8_t* cost, hipStream_t stream);
hipError_t launch_aggregate(const Frame& f, hipStream_t stream);
hipError_t launch_wta_lrc(const Frame& f, hipStream_t stream);
// the path kernel of launch_aggregate alone (slices, no path sum)
hipError_t launch_paths(const Frame& f, hipStream_t stream);
// path sum fused with WTA / D^R / LR check / median, from the slices
bool fused_select_supported(int ndisp, int npaths, int p2);
hipError_t launch_aggregate_select(const Frame& f, hipStream_t stream, bool fine = false);
// selection with subpixel refinement from S_bar in f.agg (float output)
hipError_t launch_wta_lrc_fine(const Frame& f, hipStream_t stream);
// exact consistency check: the swapped, flipped pair and the check against
// its WTA map
hipError_t launch_flip_pair(const uint8_t* left, const uint8_t* right, int width, int height,
                            int pitch, uint8_t* ref, uint8_t* mat, hipStream_t stream);
hipError_t launch_check_exact(const uint16_t* disp_left, const uint16_t* flipped, int width,
                              int height, int tolerance, int median, uint16_t* disp,
                              uint16_t* disp_right, hipStream_t stream);

hipError_t launch_census_batch(const WorkList& wl, int win_w, int win_h, hipStream_t stream);
hipError_t launch_cost_batch(const WorkList& wl, int ndisp, hipStream_t stream);
hipError_t launch_paths_batch(const WorkList& wl, int ndisp, int npaths, int p2, int variant,
                              hipStream_t stream);
hipError_t launch_merge_batch(const WorkList& wl, int npaths, int p2, hipStream_t stream);
hipError_t launch_fill_keys_batch(const WorkList& wl, hipStream_t stream);
hipError_t launch_select_batch(const WorkList& wl, int ndisp, hipStream_t stream);
hipError_t launch_select_fused_batch(const WorkList& wl, int ndisp, int npaths, int p2,
                                     hipStream_t stream);
hipError_t launch_median_batch(const WorkList& wl, hipStream_t stream);

}  // namespace sgm
