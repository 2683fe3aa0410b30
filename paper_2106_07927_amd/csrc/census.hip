// census.hip -- census transform (Sec. 2.2.1 of Ruf et al. 2021; centre
// omitted as in Sec. 2.3.1), gfx950.
//
// A 256-thread workgroup owns a 64 x 16 output tile.  The tile plus its
// (RX, RY) halo is staged once through LDS with the zero margin applied at the
// image border; every thread then computes four pixels, one column and four
// rows apart, reading the window from LDS.  Output: one uint64 per pixel,
// written coalesced along x.
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr int kTileW = 64;
constexpr int kTileH = 16;
constexpr int kThreads = 256;

template <int RX, int RY>
__global__ __launch_bounds__(kThreads) void census_kernel(const uint8_t* __restrict__ img,
                                                          int width, int height, int pitch,
                                                          uint64_t* __restrict__ out) {
    constexpr int LW = kTileW + 2 * RX;
    constexpr int LH = kTileH + 2 * RY;
    constexpr int LWP = (LW + 3) & ~3;
    __shared__ uint8_t tile[LH * LWP];

    const int x0 = blockIdx.x * kTileW;
    const int y0 = blockIdx.y * kTileH;
    for (int i = threadIdx.x; i < LW * LH; i += kThreads) {
        const int ly = i / LW, lx = i - ly * LW;
        const int gx = x0 + lx - RX, gy = y0 + ly - RY;
        uint8_t v = 0;
        if (gx >= 0 && gx < width && gy >= 0 && gy < height) v = img[(size_t)gy * pitch + gx];
        tile[ly * LWP + lx] = v;
    }
    __syncthreads();

    const int tx = threadIdx.x & (kTileW - 1);
    const int ty0 = threadIdx.x / kTileW;
    const int gx = x0 + tx;
    if (gx >= width) return;
#pragma unroll
    for (int r = 0; r < kTileH / (kThreads / kTileW); ++r) {
        const int ty = ty0 + r * (kThreads / kTileW);
        const int gy = y0 + ty;
        if (gy >= height) break;
        const uint8_t* c = &tile[(ty + RY) * LWP + tx + RX];
        const uint32_t centre = *c;
        // bits shifted in raster order: the first neighbour ends highest
        uint32_t hi = 0, lo = 0;
        int n = 0;
        constexpr int kBits = (2 * RX + 1) * (2 * RY + 1) - 1;
        constexpr int kHiBits = kBits > 32 ? kBits - 32 : 0;
#pragma unroll
        for (int dy = -RY; dy <= RY; ++dy) {
#pragma unroll
            for (int dx = -RX; dx <= RX; ++dx) {
                if (dx == 0 && dy == 0) continue;
                const uint32_t bit = (uint32_t)c[dy * LWP + dx] < centre ? 1u : 0u;
                if (n < kHiBits) hi = (hi << 1) | bit;
                else lo = (lo << 1) | bit;
                ++n;
            }
        }
        out[(size_t)gy * width + gx] = ((uint64_t)hi << 32) | lo;
    }
}

}  // namespace

hipError_t launch_census(const uint8_t* img, int width, int height, int pitch,
                         int win_w, int win_h, uint64_t* out, hipStream_t stream) {
    const dim3 grid((width + kTileW - 1) / kTileW, (height + kTileH - 1) / kTileH);
    if (win_w == 5 && win_h == 5) {
        census_kernel<2, 2><<<grid, kThreads, 0, stream>>>(img, width, height, pitch, out);
    } else {
        census_kernel<4, 3><<<grid, kThreads, 0, stream>>>(img, width, height, pitch, out);
    }
    return hipGetLastError();
}

}  // namespace sgm
