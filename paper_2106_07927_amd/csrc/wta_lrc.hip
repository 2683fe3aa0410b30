// wta_lrc.hip -- disparity selection and post-processing of Ruf et al. 2021:
// WTA (Eq. wta), the approximate right disparity map (Eq. right_disparity),
// the left-right consistency check (Eq. LR_check) and the 3x3 median
// (Sec. 2.1.3, Sec. 2.2.4), gfx950.
//
// Pass 1 (select_kernel): one wave walks a segment of one row, one pixel per
// step, reading that pixel's S_bar vector once and coalesced (lane j holds
// disparities j*EPL .. j*EPL+EPL-1).  Every value becomes a 32-bit key
// (S_bar << 8) | d, so a plain minimum yields the smallest cost and, among
// equal costs, the smallest d.
//  * D^L(x): all-reduce of the keys over the wave (DPP + permlane swaps).
//  * D^R(q) = min_d key(q + d, d): lane d keeps T_d, the running minimum for
//    q = x - d over the disparities d' <= d seen so far; each step every lane
//    takes its left neighbour's T (a one-lane shift) and folds in its own
//    key.  The lane holding d = D-1 then holds the complete minimum for
//    q = x - D + 1.  Partial minima left at a segment's end are merged with
//    the next segment's through a 32-bit atomicMin on a key map, so S_bar is
//    read exactly once, in order, with no strided gather.
// Pass 2 (check_median_kernel): per 64x4 tile plus a one-pixel halo, applies
// the LR check into LDS, then the median over the 3x3 window with 0xFFFF for
// pixels outside the image and for invalid pixels.
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr uint16_t kInvalid = 0xFFFFu;
constexpr int kSeg = 128;          // pixels per wave segment
constexpr int kSegWaves = 4;

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = group_min<16>(v);
    auto s16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = min((uint32_t)s16[0], (uint32_t)s16[1]);
    auto s32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return min((uint32_t)s32[0], (uint32_t)s32[1]);
}

__device__ __forceinline__ uint32_t wave_shr1(uint32_t v, uint32_t edge) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x138, 0xF, 0xF, false);
}

template <int EPL>
__global__ __launch_bounds__(64 * kSegWaves) void select_kernel(const uint16_t* __restrict__ agg,
                                                                int width, int ndisp,
                                                                uint16_t* __restrict__ disp_left,
                                                                uint32_t* __restrict__ right_keys) {
    const int lane = threadIdx.x & 63;
    const int seg = blockIdx.x * kSegWaves + (threadIdx.x >> 6);
    const int y = blockIdx.y;
    const int x0 = seg * kSeg;
    if (x0 >= width) return;                       // uniform per wave
    const int x1 = min(width, x0 + kSeg);
    const size_t row = (size_t)y * width;
    const int dlast_lane = (ndisp - 1) / EPL;
    const int dlast_e = (ndisp - 1) % EPL;

    uint32_t T[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) T[e] = kInf;
    uint32_t dl_keep = 0;

    for (int x = x0; x < x1; ++x) {
        const uint16_t* px = agg + (row + x) * ndisp;
        uint32_t key[EPL];
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const int d = lane * EPL + e;
            key[e] = d < ndisp ? (((uint32_t)px[d] << 8) | (uint32_t)d) : kInf;
        }
        // D^L
        uint32_t k = key[0];
#pragma unroll
        for (int e = 1; e < EPL; ++e) k = min(k, key[e]);
        k = wave_min(k);
        const int slot = (x - x0) & 63;
        if (lane == slot) dl_keep = k & 0xFFu;
        if (slot == 63 || x == x1 - 1) {
            if (lane <= slot) disp_left[row + (x - slot) + lane] = (uint16_t)dl_keep;
        }
        // D^R chain: T_d <- min(T_{d-1}, key_d)
        const uint32_t carry = wave_shr1(T[EPL - 1], kInf);
#pragma unroll
        for (int e = EPL - 1; e >= 1; --e) T[e] = min(T[e - 1], key[e]);
        T[0] = min(lane == 0 ? kInf : carry, key[0]);
        if (lane == dlast_lane) {
            const int q = x - (ndisp - 1);
            if (q >= 0) atomicMin(&right_keys[row + q], T[dlast_e]);
        }
    }
    // partial minima still travelling through the lanes
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const int d = lane * EPL + e;
        const int q = x1 - 1 - d;
        if (d < ndisp - 1 && q >= 0 && T[e] != kInf) atomicMin(&right_keys[row + q], T[e]);
    }
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
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

constexpr int kTW = 64, kTH = 4;

__global__ __launch_bounds__(256) void check_median_kernel(const uint16_t* __restrict__ disp_left,
                                                           const uint32_t* __restrict__ right_keys,
                                                           int width, int height, int tolerance,
                                                           int median,
                                                           uint16_t* __restrict__ disp,
                                                           uint16_t* __restrict__ disp_right) {
    __shared__ uint16_t tile[(kTH + 2) * (kTW + 2)];
    const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * kTH;
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
                    const int dr = (int)(right_keys[row + xr] & 0xFFu);
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
    if (gx >= width || gy >= height) return;
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
    const size_t idx = (size_t)gy * width + gx;
    disp[idx] = out;
    if (disp_right) disp_right[idx] = (uint16_t)(right_keys[idx] & 0xFFu);
}

}  // namespace

hipError_t launch_wta_lrc(const uint16_t* agg, int width, int height, int ndisp,
                          int lr_tolerance, int median3x3, uint16_t* disp,
                          uint16_t* disp_right, uint16_t* work, hipStream_t stream) {
    const size_t n = (size_t)width * height;
    uint32_t* keys = reinterpret_cast<uint32_t*>(work);     // n uint32
    uint16_t* dl = work + 2 * n;                              // n uint16
    {
        const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
        fill_u32_kernel<<<blocks, 256, 0, stream>>>(keys, n, kInf);
    }
    const int segs = (width + kSeg - 1) / kSeg;
    const dim3 g1((segs + kSegWaves - 1) / kSegWaves, height);
    if (ndisp <= 64) select_kernel<1><<<g1, 64 * kSegWaves, 0, stream>>>(agg, width, ndisp, dl, keys);
    else if (ndisp <= 128) select_kernel<2><<<g1, 64 * kSegWaves, 0, stream>>>(agg, width, ndisp, dl, keys);
    else select_kernel<4><<<g1, 64 * kSegWaves, 0, stream>>>(agg, width, ndisp, dl, keys);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2((width + kTW - 1) / kTW, (height + kTH - 1) / kTH);
    check_median_kernel<<<g2, 256, 0, stream>>>(dl, keys, width, height, lr_tolerance,
                                                 median3x3, disp, disp_right);
    return hipGetLastError();
}

}  // namespace sgm
