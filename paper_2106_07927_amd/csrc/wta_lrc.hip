// wta_lrc.hip -- disparity selection and post-processing of Ruf et al. 2021:
// WTA (Eq. wta), the approximate right disparity map (Eq. right_disparity),
// the left-right consistency check (Eq. LR_check) and the 3x3 median
// (Sec. 2.1.3, Sec. 2.2.4), gfx950.
//
// Pass 1, D a multiple of 16: the tile pass of the fused selection
// (select_fused_kernel, below), fed S_bar itself as its one uint16 slice.
// Pass 1, other D (select_kernel): one wave walks a segment of one row, one
// pixel per step, reading that pixel's S_bar vector once and coalesced (lane j holds
// disparities j*EPL .. j*EPL+EPL-1); loads run a chunk of pixels ahead.
// Every value becomes a 32-bit key (S_bar << 8) | d, so a plain minimum
// yields the smallest cost and, among equal costs, the smallest d.
//  * D^L(x): each lane parks the minimum of its own keys for the step in an
//    LDS tile [step][lane]; every 64 steps lane i reduces row i, i.e. pixel i,
//    so the cross-lane reduction costs one LDS write and read per step.
//  * D^R(q) = min_d key(q + d, d): lane d keeps T_d, the running minimum for
//    q = x - d over the disparities d' <= d seen so far; each step every lane
//    takes its left neighbour's T (a one-lane shift) and folds in its own
//    key.  The lane holding d = D-1 then holds the complete minimum for
//    q = x - D + 1.  Those minima are gathered 64 at a time and merged with a
//    coalesced 32-bit atomicMin into a key map, as are the partial minima
//    left in the lanes at a segment's end, so S_bar is read exactly once,
//    in order, with no strided gather.
// Pass 2 (check_median_kernel): per 64x4 tile plus a one-pixel halo, applies
// the LR check into LDS, then the median over the 3x3 window with 0xFFFF for
// pixels outside the image and for invalid pixels.
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr uint16_t kInvalid = 0xFFFFu;

__device__ __forceinline__ uint32_t wave_shr1(uint32_t v, uint32_t edge) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x138, 0xF, 0xF, false);
}

// Raw S_bar words of one lane for one pixel: EPL consecutive disparities as
// uint16, unpacked only when used.
template <int EPL>
struct RawVals {
    static constexpr int kWords = (EPL + 1) / 2;
    uint32_t w[kWords];
};

template <int EPL, bool VEC>
__device__ __forceinline__ RawVals<EPL> load_vals(const uint16_t* __restrict__ agg, size_t pix,
                                                  int d0, int ndisp) {
    RawVals<EPL> r;
    const uint16_t* p = agg + pix * ndisp + (d0 < ndisp ? d0 : 0);
    // S_bar is read once: nontemporal loads
    if constexpr (VEC && EPL == 1) {
        r.w[0] = __builtin_nontemporal_load(p);
    } else if constexpr (VEC && EPL == 2) {
        r.w[0] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p));
    } else if constexpr (VEC && EPL == 4) {
        typedef uint32_t v2u __attribute__((ext_vector_type(2)));
        const v2u w = __builtin_nontemporal_load(reinterpret_cast<const v2u*>(p));
        r.w[0] = w.x;
        r.w[1] = w.y;
    } else {
#pragma unroll
        for (int i = 0; i < RawVals<EPL>::kWords; ++i) r.w[i] = 0;
#pragma unroll
        for (int e = 0; e < EPL; ++e)
            if (d0 + e < ndisp) r.w[e >> 1] |= (uint32_t)p[e] << (16 * (e & 1));
    }
    return r;
}

template <int EPL>
__device__ __forceinline__ uint32_t val(const RawVals<EPL>& r, int e) {
    return (e & 1) ? (r.w[e >> 1] >> 16) : (r.w[e >> 1] & 0xFFFFu);
}

// LDS of a selection block: the D^L tile of every wave (none with FINE).
template <bool FINE>
struct SelectTile {
    uint32_t key[kSelectWaves][64][65];
};
template <>
struct SelectTile<true> {
    uint32_t key[kSelectWaves][1][65];
};

// Minimum over the 64 lanes of the wave, returned to every lane.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = group_min<16>(v);
    auto s16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = min((uint32_t)s16[0], (uint32_t)s16[1]);
    auto s32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return min((uint32_t)s32[0], (uint32_t)s32[1]);
}

// S_bar of disparity d (wave-uniform) of the current pixel, from the lane
// that holds it.
template <int EPL>
__device__ __forceinline__ uint32_t value_of(const RawVals<EPL>& cv, int d) {
    const int ln = d / EPL;
    const int e = d - ln * EPL;
    uint32_t v = val<EPL>(cv, 0);
#pragma unroll
    for (int i = 1; i < EPL; ++i) v = (e == i) ? val<EPL>(cv, i) : v;
    return (uint32_t)__builtin_amdgcn_readlane((int)v, ln);
}

// Subpixel refinement (Sec. 2.1.3): d plus the vertex offset of the parabola
// through S_bar at d - 1, d, d + 1; no offset at either end of the range or
// when the three costs are equal.
__device__ __forceinline__ float refine(int d, uint32_t s_prev, uint32_t s_min, uint32_t s_next) {
    const float den = (float)s_prev - 2.0f * (float)s_min + (float)s_next;
    const float off = den > 0.0f ? ((float)s_prev - (float)s_next) / (2.0f * den) : 0.0f;
    return (float)d + off;
}

// Selection state of one wave over one row segment [x0, x1): the D^R chain,
// the D^L tile and the keys waiting to be merged.  With FINE, D^L comes from
// a wave-wide minimum at every pixel instead of the tile (the winner's
// neighbours are needed at once for the subpixel refinement), and the
// refined D^L is written beside it.
template <int EPL, bool FINE>
struct SelectWave {
    uint32_t (*tl)[65];
    uint16_t* disp_left;
    float* fine_left;
    uint32_t* right_keys;
    size_t row;
    int x0, x1, lane, d0, ndisp, dlast_lane, dlast_e;
    // D^R chain, one entry per disparity of the lane; a vector type so that
    // the wave-uniform pick of entry dlast_e stays in registers
    uint32_t T __attribute__((ext_vector_type(EPL)));
    uint32_t emit;                                 // lane i: D^R key emitted at step base + i
    uint32_t dl_slot;                              // FINE: lane i holds D^L of pixel base + i
    float fine_slot;                               //        and its refined value

    __device__ __forceinline__ void init(uint32_t (*tile)[65], uint16_t* dl, float* fl, uint32_t* rk,
                                         int width, int nd, int y, int seg_x0, int seg_x1) {
        tl = tile;
        disp_left = dl;
        fine_left = fl;
        right_keys = rk;
        row = (size_t)y * width;
        x0 = seg_x0;
        x1 = seg_x1;
        lane = threadIdx.x & 63;
        d0 = lane * EPL;
        ndisp = nd;
        dlast_lane = (nd - 1) / EPL;
        dlast_e = (nd - 1) % EPL;
#pragma unroll
        for (int e = 0; e < EPL; ++e) T[e] = kInf;
        emit = kInf;
        dl_slot = 0;
        fine_slot = 0.0f;
    }

    // one pixel x of the segment, S_bar words of this lane's disparities
    __device__ __forceinline__ void step(const RawVals<EPL>& cv, int x) {
        uint32_t key[EPL];
#pragma unroll
        for (int e = 0; e < EPL; ++e)
            key[e] = (d0 + e < ndisp) ? ((val<EPL>(cv, e) << 8) | (uint32_t)(d0 + e)) : kInf;
        uint32_t k = key[0];
#pragma unroll
        for (int e = 1; e < EPL; ++e) k = min(k, key[e]);
        const int slot = (x - x0) & 63;
        if constexpr (FINE) {
            const uint32_t best = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_min(k));
            const int d = (int)(best & 0xFFu);
            float f = (float)d;
            if (d > 0 && d < ndisp - 1)          // uniform
                f = refine(d, value_of<EPL>(cv, d - 1), best >> 8, value_of<EPL>(cv, d + 1));
            dl_slot = (lane == slot) ? (uint32_t)d : dl_slot;
            fine_slot = (lane == slot) ? f : fine_slot;
        } else {
            tl[slot][lane] = k;
        }
        // D^R chain: T_d <- min(T_{d-1}, key_d)
        const uint32_t carry = wave_shr1(T[EPL - 1], kInf);
#pragma unroll
        for (int e = EPL - 1; e >= 1; --e) T[e] = min(T[e - 1], key[e]);
        T[0] = min(lane == 0 ? kInf : carry, key[0]);
        const uint32_t done = __builtin_amdgcn_readlane(T[dlast_e], dlast_lane);
        emit = (lane == slot) ? done : emit;
        if (slot == 63 || x == x1 - 1) {
            const int base = x - slot;
            if constexpr (FINE) {
                if (lane <= slot) {
                    disp_left[row + base + lane] = (uint16_t)dl_slot;
                    fine_left[row + base + lane] = fine_slot;
                    const int q = base + lane - (ndisp - 1);
                    if (q >= 0) atomicMin(&right_keys[row + q], emit);
                }
            } else {
                // D^L of the pixels base .. x: lane i reduces row i of the tile
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane <= slot) {
                    uint32_t best = tl[lane][0];
#pragma unroll 8
                    for (int i = 1; i < 64; ++i) best = min(best, tl[lane][i]);
                    disp_left[row + base + lane] = (uint16_t)(best & 0xFFu);
                    const int q = base + lane - (ndisp - 1);
                    if (q >= 0) atomicMin(&right_keys[row + q], emit);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            emit = kInf;
        }
    }

    // partial minima still travelling through the lanes at the segment's end
    __device__ __forceinline__ void finish() {
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const int d = d0 + e;
            const int q = x1 - 1 - d;
            if (d < ndisp - 1 && q >= 0 && T[e] != kInf) atomicMin(&right_keys[row + q], T[e]);
        }
    }
};

// Segment of one wave: block (bx, y) of one frame; waves are independent.
template <int EPL, bool VEC, bool FINE>
__device__ __forceinline__ void select_block(SelectTile<FINE>& st, const uint16_t* __restrict__ agg,
                                             int width, int ndisp,
                                             uint16_t* __restrict__ disp_left,
                                             float* __restrict__ fine_left,
                                             uint32_t* __restrict__ right_keys, int bx, int y) {
    constexpr int K = 16;                      // pixels per load chunk
    const int wave = threadIdx.x >> 6;
    const int x0 = (bx * kSelectWaves + wave) * kSelectSeg;
    if (x0 >= width) return;                       // uniform per wave
    const int x1 = min(width, x0 + kSelectSeg);
    SelectWave<EPL, FINE> sw;
    sw.init(st.key[wave], disp_left, fine_left, right_keys, width, ndisp, y, x0, x1);

    int xl = x0;                                   // next pixel to load
    RawVals<EPL> nxt[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        nxt[j] = load_vals<EPL, VEC>(agg, sw.row + xl, sw.d0, ndisp);
        xl = min(xl + 1, x1 - 1);
    }
    for (int xc = x0; xc < x1; xc += K) {
        RawVals<EPL> cur[K];
#pragma unroll
        for (int j = 0; j < K; ++j) cur[j] = nxt[j];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            nxt[j] = load_vals<EPL, VEC>(agg, sw.row + xl, sw.d0, ndisp);
            xl = min(xl + 1, x1 - 1);
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int x = xc + j;
            if (x < x1) sw.step(cur[j], x);       // uniform
        }
    }
    sw.finish();
}

// ---- path sum fused with the selection pass --------------------------------
// A block owns a tile of one row: 64 pixels, or 32 when D > 128, so that the
// tile holds at most 8192 volume elements.
//  (1) Each of its 256 threads loads two blocks of 16 elements of the tile
//      from every pair slice (and, for uint8 slices, from the cost volume)
//      -- all loads issued before any is used -- and sums them into an LDS
//      copy of S_bar: one row of D values per pixel, padded by one dword so
//      that rows start in different banks.  S_bar never goes to HBM.
//  (2) 256 / tile threads per pixel take the minimum key (S_bar << 8) | d
//      over their share of the disparities; a DPP reduction gives D^L (and
//      with FINE the refined value, from the winner's two neighbours in LDS).
//  (3) One thread per right-view pixel q folds key(q + d, d) over the d with
//      q + d inside the tile and merges that partial minimum into the D^R key
//      map with atomicMin; the tiles holding q .. q + D - 1 complete it.
// Needs D % 16 == 0, so every block of 16 elements lies inside one pixel's
// vector.  NS pair slices: uint8 (S_bar = 2 NS C + sum) or uint16 (S_bar =
// sum).
template <int NS, bool U8, bool FINE>
__device__ __forceinline__ void select_tile_block(uint16_t* __restrict__ sb, const Frame& f, int bx,
                                                  int y) {
    const int width = f.width, ndisp = f.ndisp;
    const int tpx = fused_tile_px(ndisp);
    const int x0 = bx * tpx;
    const int npx = min(tpx, width - x0);
    const int rs = ndisp + 2;                      // LDS row stride (uint16)
    const size_t row = (size_t)y * width;
    const uint32_t e_tile = (uint32_t)(row + x0) * (uint32_t)ndisp;
    const uint32_t e_last = (uint32_t)(row + x0 + npx) * (uint32_t)ndisp - 16u;

    // (1) path sum into LDS.  Blocks past the row's last pixel re-read its
    // last block and land in LDS rows that are never read.  The slices are
    // read once (nontemporal loads); the cost volume keeps cached loads.
    const int nblk = tpx * ndisp / 16;             // <= 512
    if constexpr (U8) {
        uint4 c[2];
        uint4 a[2][NS];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            if (256 * i >= nblk) break;            // uniform: small D fits in one pass
            const uint32_t e = min(e_tile + 16u * (uint32_t)(threadIdx.x + 256 * i), e_last);
            c[i] = *reinterpret_cast<const uint4*>(f.cost + e);
#pragma unroll
            for (int r = 0; r < NS; ++r)
                a[i][r] = load_once16(f.slices + (size_t)r * f.slice_stride + e);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int b = threadIdx.x + 256 * i;
            if (b < nblk) {
                uint32_t sum[8];
                merge16<NS, 2 * NS>(c[i], a[i], sum);
                const int p = (16 * b) / ndisp;
                const int d = 16 * b - p * ndisp;
                uint32_t* dst = reinterpret_cast<uint32_t*>(sb + p * rs + d);
#pragma unroll
                for (int k = 0; k < 8; ++k) dst[k] = sum[k];
            }
        }
    } else {
        const uint16_t* slices = reinterpret_cast<const uint16_t*>(f.slices);
        uint4 a[2][NS][2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            if (256 * i >= nblk) break;
            const uint32_t e = min(e_tile + 16u * (uint32_t)(threadIdx.x + 256 * i), e_last);
#pragma unroll
            for (int r = 0; r < NS; ++r) {
                a[i][r][0] = load_once16(slices + (size_t)r * f.slice_stride + e);
                a[i][r][1] = load_once16(slices + (size_t)r * f.slice_stride + e + 8);
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int b = threadIdx.x + 256 * i;
            if (b < nblk) {
                uint32_t sum[8];
                wide_sum16<NS>(a[i], sum);
                const int p = (16 * b) / ndisp;
                const int d = 16 * b - p * ndisp;
                uint32_t* dst = reinterpret_cast<uint32_t*>(sb + p * rs + d);
#pragma unroll
                for (int k = 0; k < 8; ++k) dst[k] = sum[k];
            }
        }
    }
    __syncthreads();

    // (2) D^L: the tpp threads of pixel p each cover D / tpp disparities
    {
        const int tpp = 256 / tpx;                 // 4 or 8
        const int p = threadIdx.x / tpp, part = threadIdx.x % tpp;
        const int dq = ndisp / tpp;
        uint32_t best = kInf;
        if (p < npx) {
            const uint16_t* src = sb + p * rs + part * dq;
            for (int i = 0; i < dq; i += 2) {
                const uint32_t w = *reinterpret_cast<const uint32_t*>(src + i);
                const uint32_t d = (uint32_t)(part * dq + i);
                best = min(best, min(((w & 0xFFFFu) << 8) | d, ((w >> 16) << 8) | (d + 1)));
            }
        }
        best = min(best, dpp<kDppQuadSwap1>(kInf, best));
        best = min(best, dpp<kDppQuadSwap2>(kInf, best));
        if (tpp == 8) best = min(best, dpp<kDppRowHalfMirror>(kInf, best));
        if (part == 0 && p < npx) {
            const int d = (int)(best & 0xFFu);
            f.disp_left[row + x0 + p] = (uint16_t)d;
            if constexpr (FINE) {
                float v = (float)d;
                if (d > 0 && d < ndisp - 1)
                    v = refine(d, sb[p * rs + d - 1], best >> 8, sb[p * rs + d + 1]);
                f.fine_left[row + x0 + p] = v;
            }
        }
    }

    // (3) D^R partial minima: q = x0 - D + 1 + t; tile pixel k holds d = k + x0 - q
    const int nq = npx + ndisp - 1;
    for (int t = threadIdx.x; t < nq; t += blockDim.x) {
        const int q = x0 - ndisp + 1 + t;
        const int off = x0 - q;                    // d of tile pixel 0
        uint32_t best = kInf;
        const int k0 = max(0, -off), k1 = min(npx, ndisp - off);
        const uint16_t* src = sb + k0 * (rs + 1) + off;
        for (int k = k0; k < k1; ++k, src += rs + 1)
            best = min(best, ((uint32_t)*src << 8) | (uint32_t)(k + off));
        if (q >= 0) atomicMin(&f.right_keys[row + q], best);
    }
    __syncthreads();   // the LDS tile is reused by the next work item
}

// LDS of the fused pass: one row of D + 2 values per tile pixel, sized at launch
__host__ __device__ inline size_t fused_lds_bytes(int ndisp) {
    return (size_t)fused_tile_px(ndisp) * (size_t)(ndisp + 2) * sizeof(uint16_t);
}

template <int NS, bool U8, bool FINE>
__global__ __launch_bounds__(256) void select_fused_kernel(Frame f) {
    extern __shared__ uint16_t sb[];
    select_tile_block<NS, U8, FINE>(sb, f, blockIdx.x, blockIdx.y);
}

template <int NS, bool U8>
__global__ __launch_bounds__(256) void select_fused_batch_kernel(WorkList wl) {
    extern __shared__ uint16_t sb[];
    for (int b = blockIdx.x; b < wl.total; b += gridDim.x) {
        const int fi = find_frame(wl, b);
        const Frame& f = wl.frames[fi];
        const int lb = b - wl.starts[fi];
        const int bxs = fused_blocks_x(f.width, f.ndisp);
        select_tile_block<NS, U8, false>(sb, f, lb % bxs, lb / bxs);
    }
}

template <int EPL, bool VEC, bool FINE>
__global__ __launch_bounds__(64 * kSelectWaves) void select_kernel(Frame f) {
    __shared__ SelectTile<FINE> st;
    select_block<EPL, VEC, FINE>(st, f.agg, f.width, f.ndisp, f.disp_left, f.fine_left, f.right_keys,
                                 blockIdx.x, blockIdx.y);
}

template <int EPL, bool VEC>
__global__ __launch_bounds__(64 * kSelectWaves) void select_batch_kernel(WorkList wl) {
    __shared__ SelectTile<false> st;
    for (int b = blockIdx.x; b < wl.total; b += gridDim.x) {
        const int fi = find_frame(wl, b);
        const Frame& f = wl.frames[fi];
        const int lb = b - wl.starts[fi];
        const int bxs = select_blocks_x(f.width);
        select_block<EPL, VEC, false>(st, f.agg, f.width, f.ndisp, f.disp_left, nullptr, f.right_keys,
                                      lb % bxs, lb / bxs);
    }
}

// D^R keys start at "no candidate" (all ones).
__device__ __forceinline__ void fill_keys_block(const Frame& f, int lb) {
    const size_t n = (size_t)f.width * f.height;
    const size_t e0 = (size_t)lb * kFillChunk;
    for (size_t e = e0 + threadIdx.x; e < n && e < e0 + kFillChunk; e += blockDim.x) f.right_keys[e] = kInf;
}

__global__ __launch_bounds__(256) void fill_keys_kernel(Frame f) { fill_keys_block(f, blockIdx.x); }

__global__ __launch_bounds__(256) void fill_keys_batch_kernel(WorkList wl) {
    for (int b = blockIdx.x; b < wl.total; b += gridDim.x) {
        const int fi = find_frame(wl, b);
        fill_keys_block(wl.frames[fi], b - wl.starts[fi]);
    }
}

// Median of nine by the first five passes of a bubble-sort network (App. F).
__device__ __forceinline__ uint32_t median9(uint32_t v[9]) {
#pragma unroll
    for (int pass = 0; pass < 5; ++pass) {
#pragma unroll
        for (int i = 0; i < 8 - pass; ++i) {
            const uint32_t lo = min(v[i], v[i + 1]);
            const uint32_t hi = max(v[i], v[i + 1]);
            v[i] = lo;
            v[i + 1] = hi;
        }
    }
    return v[4];
}

constexpr int kTW = kMedianTileW, kTH = kMedianTileH;

struct MedianTile {
    uint16_t v[(kTH + 2) * (kTW + 2)];
};

// D^R of pixel (xr, row): from the key map of the approximate D^R, or, for the
// exact check, from the disparity map of the swapped, flipped pair.
struct RightSource {
    const uint32_t* keys;            // approximate: key & 0xFF
    const uint16_t* flipped;         // exact: flipped[row][width - 1 - xr]
    __device__ __forceinline__ int at(size_t row, int xr, int width) const {
        if (flipped) return flipped[row + (width - 1 - xr)];
        return (int)(keys[row + xr] & 0xFFu);
    }
};

__device__ __forceinline__ void check_median_block(MedianTile& mt, const uint16_t* __restrict__ disp_left,
                                                   RightSource rs, int width, int height,
                                                   int tolerance, int median,
                                                   uint16_t* __restrict__ disp,
                                                   uint16_t* __restrict__ disp_right, int bx, int by) {
    uint16_t* tile = mt.v;
    const int x0 = bx * kTW, y0 = by * kTH;
    for (int i = threadIdx.x; i < (kTH + 2) * (kTW + 2); i += 256) {
        const int ly = i / (kTW + 2), lx = i - ly * (kTW + 2);
        const int gx = x0 + lx - 1, gy = y0 + ly - 1;
        uint16_t v = kInvalid;
        if (gx >= 0 && gx < width && gy >= 0 && gy < height) {
            const size_t row = (size_t)gy * width;
            const int dl = disp_left[row + gx];
            v = (uint16_t)dl;
            if (tolerance >= 0) {
                const int xr = gx - dl;
                v = kInvalid;
                if (xr >= 0) {
                    const int dr = rs.at(row, xr, width);
                    const int diff = dl > dr ? dl - dr : dr - dl;
                    if (diff <= tolerance) v = (uint16_t)dl;
                }
            }
        }
        tile[i] = v;
    }
    __syncthreads();
    const int tx = threadIdx.x & (kTW - 1), ty = threadIdx.x / kTW;
    const int gx = x0 + tx, gy = y0 + ty;
    if (gx < width && gy < height) {
        const uint16_t* c = &tile[(ty + 1) * (kTW + 2) + tx + 1];
        uint16_t out = *c;
        if (median && out != kInvalid) {
            uint32_t v[9];
            int k = 0;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) v[k++] = c[dy * (kTW + 2) + dx];
            out = (uint16_t)median9(v);
        }
        const size_t row = (size_t)gy * width;
        disp[row + gx] = out;
        if (disp_right) disp_right[row + gx] = (uint16_t)rs.at(row, gx, width);
    }
    __syncthreads();   // the tile is reused by the next work item
}

__global__ __launch_bounds__(256) void check_median_kernel(Frame f) {
    __shared__ MedianTile mt;
    check_median_block(mt, f.disp_left, RightSource{f.right_keys, nullptr}, f.width, f.height,
                       f.lr_tolerance, f.median3x3, f.disp, f.disp_right, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void check_median_batch_kernel(WorkList wl) {
    __shared__ MedianTile mt;
    for (int b = blockIdx.x; b < wl.total; b += gridDim.x) {
        const int fi = find_frame(wl, b);
        const Frame& f = wl.frames[fi];
        const int lb = b - wl.starts[fi];
        const int bxs = median_blocks_x(f.width);
        check_median_block(mt, f.disp_left, RightSource{f.right_keys, nullptr}, f.width, f.height,
                           f.lr_tolerance, f.median3x3, f.disp, f.disp_right, lb % bxs, lb / bxs);
    }
}

// Exact consistency check: disp_left = D^L of the pair, flipped = the WTA map
// of the swapped, horizontally flipped pair (so D^R(xr) = flipped[W-1-xr]).
__global__ __launch_bounds__(256) void check_median_exact_kernel(const uint16_t* __restrict__ disp_left,
                                                                  const uint16_t* __restrict__ flipped,
                                                                  int width, int height, int tolerance,
                                                                  int median, uint16_t* __restrict__ disp,
                                                                  uint16_t* __restrict__ disp_right) {
    __shared__ MedianTile mt;
    check_median_block(mt, disp_left, RightSource{nullptr, flipped}, width, height, tolerance, median,
                       disp, disp_right, blockIdx.x, blockIdx.y);
}

// The swapped, horizontally flipped pair: ref[y][x] = right[y][W-1-x] (the
// new reference image), mat[y][x] = left[y][W-1-x].  Outputs have pitch W.
__global__ __launch_bounds__(256) void flip_pair_kernel(const uint8_t* __restrict__ left,
                                                        const uint8_t* __restrict__ right, int width,
                                                        int height, int pitch,
                                                        uint8_t* __restrict__ ref,
                                                        uint8_t* __restrict__ mat) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= width) return;
    const size_t src = (size_t)y * pitch + (width - 1 - x);
    const size_t dst = (size_t)y * width + x;
    ref[dst] = right[src];
    mat[dst] = left[src];
}

template <int EPL, bool VEC, bool FINE>
void launch_select_t(const Frame* one, const WorkList* wl, hipStream_t stream) {
    if (one) {
        const dim3 g(select_blocks_x(one->width), one->height);
        select_kernel<EPL, VEC, FINE><<<g, 64 * kSelectWaves, 0, stream>>>(*one);
    } else {
        select_batch_kernel<EPL, VEC><<<persistent_grid(wl->total, 2), 64 * kSelectWaves, 0, stream>>>(*wl);
    }
}

template <bool FINE>
void launch_select_any(const Frame* one, const WorkList* wl, int ndisp, hipStream_t stream) {
    if (ndisp <= 64) {
        launch_select_t<1, true, FINE>(one, wl, stream);
    } else if (ndisp <= 128) {
        if (ndisp % 2 == 0) launch_select_t<2, true, FINE>(one, wl, stream);
        else launch_select_t<2, false, FINE>(one, wl, stream);
    } else {
        if (ndisp % 4 == 0) launch_select_t<4, true, FINE>(one, wl, stream);
        else launch_select_t<4, false, FINE>(one, wl, stream);
    }
}

template <int NS, bool U8, bool FINE>
void launch_fused_t(const Frame* one, const WorkList* wl, int ndisp, hipStream_t stream) {
    const size_t lds = fused_lds_bytes(ndisp);
    if (one) {
        const dim3 g(fused_blocks_x(one->width, ndisp), one->height);
        select_fused_kernel<NS, U8, FINE><<<g, 256, lds, stream>>>(*one);
    } else {
        select_fused_batch_kernel<NS, U8><<<persistent_grid(wl->total), 256, lds, stream>>>(*wl);
    }
}

// frames of one launch share D (the LDS size depends on it)
template <bool FINE>
void launch_fused_any(const Frame* one, const WorkList* wl, int ndisp, int npaths, int p2,
                      hipStream_t stream) {
    const bool u8 = slices_u8(p2);
    if (npaths == 4) {
        if (u8) launch_fused_t<2, true, FINE>(one, wl, ndisp, stream);
        else launch_fused_t<2, false, FINE>(one, wl, ndisp, stream);
    } else {
        if (u8) launch_fused_t<4, true, FINE>(one, wl, ndisp, stream);
        else launch_fused_t<4, false, FINE>(one, wl, ndisp, stream);
    }
}

// ---- subpixel output: LR check on the integer maps, then the median over
// the refined values (pixels outside the image and invalid pixels count as
// +inf; a median of +inf is invalid).  Invalid pixels are -1.0f.
constexpr float kInvalidF = -1.0f;

struct MedianTileF {
    float v[(kTH + 2) * (kTW + 2)];
};

__device__ __forceinline__ float median9f(float v[9]) {
#pragma unroll
    for (int pass = 0; pass < 5; ++pass) {
#pragma unroll
        for (int i = 0; i < 8 - pass; ++i) {
            const float lo = fminf(v[i], v[i + 1]);
            const float hi = fmaxf(v[i], v[i + 1]);
            v[i] = lo;
            v[i + 1] = hi;
        }
    }
    return v[4];
}

__global__ __launch_bounds__(256) void check_median_fine_kernel(Frame f) {
    __shared__ MedianTileF mt;
    float* tile = mt.v;
    const int width = f.width, height = f.height, tolerance = f.lr_tolerance;
    const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * kTH;
    for (int i = threadIdx.x; i < (kTH + 2) * (kTW + 2); i += 256) {
        const int ly = i / (kTW + 2), lx = i - ly * (kTW + 2);
        const int gx = x0 + lx - 1, gy = y0 + ly - 1;
        float v = INFINITY;
        if (gx >= 0 && gx < width && gy >= 0 && gy < height) {
            const size_t row = (size_t)gy * width;
            const int dl = f.disp_left[row + gx];
            bool ok = true;
            if (tolerance >= 0) {
                const int xr = gx - dl;
                ok = false;
                if (xr >= 0) {
                    const int dr = (int)(f.right_keys[row + xr] & 0xFFu);
                    const int diff = dl > dr ? dl - dr : dr - dl;
                    ok = diff <= tolerance;
                }
            }
            if (ok) v = f.fine_left[row + gx];
        }
        tile[i] = v;
    }
    __syncthreads();
    const int tx = threadIdx.x & (kTW - 1), ty = threadIdx.x / kTW;
    const int gx = x0 + tx, gy = y0 + ty;
    if (gx < width && gy < height) {
        const float* c = &tile[(ty + 1) * (kTW + 2) + tx + 1];
        float out = *c;
        if (f.median3x3 && out != INFINITY) {
            float v[9];
            int k = 0;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) v[k++] = c[dy * (kTW + 2) + dx];
            out = median9f(v);
        }
        const size_t idx = (size_t)gy * width + gx;
        f.disp_fine[idx] = out == INFINITY ? kInvalidF : out;
        if (f.disp_right) f.disp_right[idx] = (uint16_t)(f.right_keys[idx] & 0xFFu);
    }
}

}  // namespace

bool fused_select_supported(int ndisp, int npaths, int p2) {
    (void)p2;
    return ndisp % 16 == 0 && ndisp <= 256 && (npaths == 4 || npaths == 8);
}

hipError_t launch_aggregate_select(const Frame& f, hipStream_t stream, bool fine) {
    Frame g = f;
    g.paths_fill_keys = 1;                     // the path kernel clears the D^R keys
    hipError_t e = launch_paths(g, stream);
    if (e != hipSuccess) return e;
    if (fine) launch_fused_any<true>(&f, nullptr, f.ndisp, f.npaths, f.p2, stream);
    else launch_fused_any<false>(&f, nullptr, f.ndisp, f.npaths, f.p2, stream);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2(median_blocks_x(f.width), (f.height + kTH - 1) / kTH);
    if (fine) check_median_fine_kernel<<<g2, 256, 0, stream>>>(f);
    else check_median_kernel<<<g2, 256, 0, stream>>>(f);
    return hipGetLastError();
}

hipError_t launch_select_fused_batch(const WorkList& wl, int ndisp, int npaths, int p2,
                                     hipStream_t stream) {
    launch_fused_any<false>(nullptr, &wl, ndisp, npaths, p2, stream);
    return hipGetLastError();
}

hipError_t launch_wta_lrc_fine(const Frame& f, hipStream_t stream) {
    const size_t n = (size_t)f.width * f.height;
    fill_keys_kernel<<<fill_blocks(n), 256, 0, stream>>>(f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    launch_select_any<true>(&f, nullptr, f.ndisp, stream);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2(median_blocks_x(f.width), (f.height + kTH - 1) / kTH);
    check_median_fine_kernel<<<g2, 256, 0, stream>>>(f);
    return hipGetLastError();
}

hipError_t launch_wta_lrc(const Frame& f, hipStream_t stream) {
    const size_t n = (size_t)f.width * f.height;
    fill_keys_kernel<<<fill_blocks(n), 256, 0, stream>>>(f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (f.ndisp % 16 == 0) {
        // the fused selection's tile pass, fed S_bar itself as its one
        // uint16 "slice" (the sum of one slice is the slice): S_bar is read
        // once, in 16-byte blocks, instead of by the row-segment pass
        Frame g = f;
        g.slices = reinterpret_cast<uint8_t*>(f.agg);
        g.slice_stride = 0;
        launch_fused_t<1, false, false>(&g, nullptr, f.ndisp, stream);
    } else {
        launch_select_any<false>(&f, nullptr, f.ndisp, stream);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2(median_blocks_x(f.width), (f.height + kTH - 1) / kTH);
    check_median_kernel<<<g2, 256, 0, stream>>>(f);
    return hipGetLastError();
}

hipError_t launch_flip_pair(const uint8_t* left, const uint8_t* right, int width, int height,
                            int pitch, uint8_t* ref, uint8_t* mat, hipStream_t stream) {
    const dim3 g((width + 255) / 256, height);
    flip_pair_kernel<<<g, 256, 0, stream>>>(left, right, width, height, pitch, ref, mat);
    return hipGetLastError();
}

hipError_t launch_check_exact(const uint16_t* disp_left, const uint16_t* flipped, int width,
                              int height, int tolerance, int median, uint16_t* disp,
                              uint16_t* disp_right, hipStream_t stream) {
    const dim3 g(median_blocks_x(width), (height + kTH - 1) / kTH);
    check_median_exact_kernel<<<g, 256, 0, stream>>>(disp_left, flipped, width, height, tolerance,
                                                      median, disp, disp_right);
    return hipGetLastError();
}

hipError_t launch_fill_keys_batch(const WorkList& wl, hipStream_t stream) {
    fill_keys_batch_kernel<<<persistent_grid(wl.total), 256, 0, stream>>>(wl);
    return hipGetLastError();
}

hipError_t launch_select_batch(const WorkList& wl, int ndisp, hipStream_t stream) {
    launch_select_any<false>(nullptr, &wl, ndisp, stream);
    return hipGetLastError();
}

hipError_t launch_median_batch(const WorkList& wl, hipStream_t stream) {
    check_median_batch_kernel<<<persistent_grid(wl.total), 256, 0, stream>>>(wl);
    return hipGetLastError();
}

}  // namespace sgm
