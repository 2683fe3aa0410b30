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

constexpr int kThreads = 256;

template <int RX, int RY>
struct CensusTile {
    static constexpr int LW = kCensusTileW + 2 * RX;
    static constexpr int LH = kCensusTileH + 2 * RY;
    static constexpr int LWP = (LW + 3) & ~3;
    uint8_t px[LH * LWP];
};

// Tile (bx, by) of one image.  Every thread passes the same barriers.
template <int RX, int RY>
__device__ __forceinline__ void census_tile(CensusTile<RX, RY>& t, const uint8_t* __restrict__ img,
                                            int width, int height, int pitch,
                                            uint64_t* __restrict__ out, int bx, int by) {
    using T = CensusTile<RX, RY>;
    const int x0 = bx * kCensusTileW;
    const int y0 = by * kCensusTileH;
    for (int i = threadIdx.x; i < T::LW * T::LH; i += kThreads) {
        const int ly = i / T::LW, lx = i - ly * T::LW;
        const int gx = x0 + lx - RX, gy = y0 + ly - RY;
        uint8_t v = 0;
        if (gx >= 0 && gx < width && gy >= 0 && gy < height) v = img[(size_t)gy * pitch + gx];
        t.px[ly * T::LWP + lx] = v;
    }
    __syncthreads();

    const int tx = threadIdx.x & (kCensusTileW - 1);
    const int ty0 = threadIdx.x / kCensusTileW;
    const int gx = x0 + tx;
    if (gx < width) {
#pragma unroll
        for (int r = 0; r < kCensusTileH / (kThreads / kCensusTileW); ++r) {
            const int ty = ty0 + r * (kThreads / kCensusTileW);
            const int gy = y0 + ty;
            if (gy < height) {
                const uint8_t* c = &t.px[(ty + RY) * T::LWP + tx + RX];
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
                        const uint32_t bit = (uint32_t)c[dy * T::LWP + dx] < centre ? 1u : 0u;
                        if (n < kHiBits) hi = (hi << 1) | bit;
                        else lo = (lo << 1) | bit;
                        ++n;
                    }
                }
                out[(size_t)gy * width + gx] = ((uint64_t)hi << 32) | lo;
            }
        }
    }
    __syncthreads();   // the tile is reused by the next work item
}

template <int RX, int RY>
__global__ __launch_bounds__(kThreads) void census_kernel(const uint8_t* __restrict__ img, int width,
                                                          int height, int pitch,
                                                          uint64_t* __restrict__ out) {
    __shared__ CensusTile<RX, RY> tile;
    census_tile<RX, RY>(tile, img, width, height, pitch, out, blockIdx.x, blockIdx.y);
}

// Both images of every frame of the work list: block b of a frame is tile b
// of the left image, tile b - census_blocks(w, h) of the right one.
template <int RX, int RY>
__global__ __launch_bounds__(kThreads) void census_batch_kernel(WorkList wl) {
    __shared__ CensusTile<RX, RY> tile;
    for (int b = blockIdx.x; b < wl.total; b += gridDim.x) {
        const int fi = find_frame(wl, b);
        const Frame& f = wl.frames[fi];
        int lb = b - wl.starts[fi];
        const int nb = census_blocks(f.width, f.height);
        const bool right = lb >= nb;
        lb -= right ? nb : 0;
        const int bxs = census_blocks_x(f.width);
        census_tile<RX, RY>(tile, right ? f.right : f.left, f.width, f.height, f.pitch,
                            right ? f.census_right : f.census_left, lb % bxs, lb / bxs);
    }
}

}  // namespace

hipError_t launch_census(const Frame& f, bool right, hipStream_t stream) {
    const dim3 grid(census_blocks_x(f.width), (f.height + kCensusTileH - 1) / kCensusTileH);
    const uint8_t* img = right ? f.right : f.left;
    uint64_t* out = right ? f.census_right : f.census_left;
    if (f.win_w == 5 && f.win_h == 5) {
        census_kernel<2, 2><<<grid, kThreads, 0, stream>>>(img, f.width, f.height, f.pitch, out);
    } else {
        census_kernel<4, 3><<<grid, kThreads, 0, stream>>>(img, f.width, f.height, f.pitch, out);
    }
    return hipGetLastError();
}

hipError_t launch_census_batch(const WorkList& wl, int win_w, int win_h, hipStream_t stream) {
    const int grid = persistent_grid(wl.total);
    if (win_w == 5 && win_h == 5) census_batch_kernel<2, 2><<<grid, kThreads, 0, stream>>>(wl);
    else census_batch_kernel<4, 3><<<grid, kThreads, 0, stream>>>(wl);
    return hipGetLastError();
}

}  // namespace sgm
