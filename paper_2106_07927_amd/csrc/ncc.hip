// ncc.hip -- inverted, truncated normalised cross-correlation matching cost
// (Sec. 2.1.1, Sec. 2.2.1 of Ruf et al. 2021), gfx950.
//
//   s = 1 - max(0, Phi),  Phi = (n S_LR - S_L S_R) / (sqrt(n S_LL - S_L^2) sqrt(n S_RR - S_R^2))
//
// over win x win patches (n = win^2), stored as the uint8 cost round(255 s).
// Pixels outside the image read as zero (the zero margin of the census
// window); a patch without variance has no correlation (cost 255); x - d < 0
// costs 255.  The window sums are exact integers; the float part runs in
// float32 with IEEE square root and division in a fixed order, so the
// quantised cost is reproducible bit for bit.
//
// A 256-thread block owns 64 pixels of one row and every disparity.  It
// stages the window columns of both images in LDS -- each column's win bytes
// packed into dwords so that one v_dot4_u32_u8 multiplies four rows -- plus
// each column's sum and sum of squares.  Per-pixel patch sums (the mean and
// variance terms of the paper's per-pixel struct) follow from sliding sums
// over the columns.  A thread then takes one disparity d and 32 consecutive
// pixels: it slides the cross sum S_LR along x, one new column product per
// pixel, and evaluates the cost.  Consecutive threads take consecutive d, so
// every byte store of a wave is 64 consecutive bytes of the volume.
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr int kNccTile = 64;                   // pixels of a row per block
constexpr int kNccRun = 32;                    // pixels per thread and disparity
constexpr int kMaxD = 256;

template <int WIN>
struct NccTile {
    static constexpr int R = (WIN - 1) / 2;
    static constexpr int CW = (WIN + 3) / 4;   // dwords per packed column
    static constexpr int LCOLS = kNccTile + 2 * R;
    static constexpr int RCOLS = kNccTile + kMaxD - 1 + 2 * R;
    uint32_t lcol[LCOLS][CW];
    uint32_t rcol[RCOLS][CW];
    int32_t lsum[LCOLS], lsq[LCOLS];
    int32_t rsum[RCOLS], rsq[RCOLS];
    int32_t ls[kNccTile];                      // S_L per tile pixel
    float lsig[kNccTile];                      // sqrt(n S_LL - S_L^2), 0 if flat
    int32_t rs[kNccTile + kMaxD - 1];          // S_R per right pixel x0 - D + 1 + i
    float rsig[kNccTile + kMaxD - 1];
};

// Column c of a staged image: rows y - R .. y + R at image column gx.
template <int WIN>
__device__ __forceinline__ void stage_column(const uint8_t* __restrict__ img, int width, int height,
                                             int pitch, int gx, int y, uint32_t (&col)[NccTile<WIN>::CW],
                                             int32_t& sum, int32_t& sq) {
    constexpr int R = NccTile<WIN>::R;
#pragma unroll
    for (int k = 0; k < NccTile<WIN>::CW; ++k) col[k] = 0;
    int s = 0, q = 0;
#pragma unroll
    for (int i = 0; i < WIN; ++i) {
        const int gy = y - R + i;
        uint32_t v = 0;
        if (gx >= 0 && gx < width && gy >= 0 && gy < height) v = img[(size_t)gy * pitch + gx];
        col[i >> 2] |= v << (8 * (i & 3));
        s += (int)v;
        q += (int)(v * v);
    }
    sum = s;
    sq = q;
}

template <int WIN>
__device__ __forceinline__ uint32_t column_dot(const uint32_t (&a)[NccTile<WIN>::CW],
                                               const uint32_t (&b)[NccTile<WIN>::CW]) {
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < NccTile<WIN>::CW; ++k) acc = __builtin_amdgcn_udot4(a[k], b[k], acc, false);
    return acc;
}

// sqrt(n SS - S^2) as float32 (IEEE square root), 0 for a patch without
// variance.
__device__ __forceinline__ float patch_sigma(int n, int32_t s, int32_t ss) {
    const int32_t v = n * ss - s * s;
    return v > 0 ? sqrtf((float)v) : 0.0f;
}

#pragma clang fp contract(off)
__device__ __forceinline__ uint8_t ncc_cost_value(int n, int32_t slr, int32_t sl, int32_t sr,
                                                  float sigl, float sigr) {
    if (sigl == 0.0f || sigr == 0.0f) return 255;
    const int32_t num = n * slr - sl * sr;
    const float den = sigl * sigr;
    const float phi = (float)num / den;
    const float s = 1.0f - (phi > 0.0f ? phi : 0.0f);
    float v = rintf(255.0f * s);
    v = v < 0.0f ? 0.0f : (v > 255.0f ? 255.0f : v);
    return (uint8_t)v;
}

template <int WIN>
__global__ __launch_bounds__(256) void ncc_cost_kernel(const uint8_t* __restrict__ left,
                                                       const uint8_t* __restrict__ right, int width,
                                                       int height, int pitch, int ndisp,
                                                       uint8_t* __restrict__ cost) {
    using T = NccTile<WIN>;
    constexpr int R = T::R;
    constexpr int N = WIN * WIN;
    __shared__ T t;
    const int x0 = blockIdx.x * kNccTile;
    const int y = blockIdx.y;
    const int npx = min(kNccTile, width - x0);
    const int rbase = x0 - ndisp + 1 - R;      // image column of rcol[0]
    const int nr = npx + ndisp - 1 + 2 * R;

    // stage the window columns
    for (int c = threadIdx.x; c < npx + 2 * R; c += blockDim.x)
        stage_column<WIN>(left, width, height, pitch, x0 - R + c, y, t.lcol[c], t.lsum[c], t.lsq[c]);
    for (int c = threadIdx.x; c < nr; c += blockDim.x)
        stage_column<WIN>(right, width, height, pitch, rbase + c, y, t.rcol[c], t.rsum[c], t.rsq[c]);
    __syncthreads();

    // patch sums and deviations
    for (int p = threadIdx.x; p < npx; p += blockDim.x) {
        int32_t s = 0, q = 0;
#pragma unroll
        for (int k = 0; k < WIN; ++k) {
            s += t.lsum[p + k];
            q += t.lsq[p + k];
        }
        t.ls[p] = s;
        t.lsig[p] = patch_sigma(N, s, q);
    }
    for (int p = threadIdx.x; p < npx + ndisp - 1; p += blockDim.x) {
        int32_t s = 0, q = 0;
#pragma unroll
        for (int k = 0; k < WIN; ++k) {
            s += t.rsum[p + k];
            q += t.rsq[p + k];
        }
        t.rs[p] = s;
        t.rsig[p] = patch_sigma(N, s, q);
    }
    __syncthreads();

    // costs: item = (run, d); right pixel x - d is rs index p + D - 1 - d
    const int runs = (npx + kNccRun - 1) / kNccRun;
    uint8_t* out = cost + ((size_t)y * width + x0) * ndisp;
    for (int item = threadIdx.x; item < runs * ndisp; item += blockDim.x) {
        const int d = item % ndisp;
        const int p0 = (item / ndisp) * kNccRun;
        const int p1 = min(npx, p0 + kNccRun);
        const int off = ndisp - 1 - d;          // rcol index of left column c is c + off
        uint32_t win[WIN];                      // column products of the current window
        int32_t slr = 0;
#pragma unroll
        for (int k = 0; k < WIN - 1; ++k) {
            win[k] = column_dot<WIN>(t.lcol[p0 + k], t.rcol[p0 + k + off]);
            slr += (int32_t)win[k];
        }
        for (int p = p0; p < p1; ++p) {
            const uint32_t fresh = column_dot<WIN>(t.lcol[p + WIN - 1], t.rcol[p + WIN - 1 + off]);
            slr += (int32_t)fresh;
            uint8_t c = 255;
            if (x0 + p - d >= 0)
                c = ncc_cost_value(N, slr, t.ls[p], t.rs[p + off], t.lsig[p], t.rsig[p + off]);
            out[(size_t)p * ndisp + d] = c;
            // slide: drop the window's first column, keep the rest in order
            slr -= (int32_t)win[0];
#pragma unroll
            for (int k = 0; k < WIN - 2; ++k) win[k] = win[k + 1];
            win[WIN - 2] = fresh;
        }
    }
}

}  // namespace

hipError_t launch_ncc_cost(const uint8_t* left, const uint8_t* right, int width, int height,
                           int pitch, int win, int ndisp, uint8_t* cost, hipStream_t stream) {
    const dim3 grid((width + kNccTile - 1) / kNccTile, height);
    if (win == 5) ncc_cost_kernel<5><<<grid, 256, 0, stream>>>(left, right, width, height, pitch, ndisp, cost);
    else ncc_cost_kernel<9><<<grid, 256, 0, stream>>>(left, right, width, height, pitch, ndisp, cost);
    return hipGetLastError();
}

}  // namespace sgm
