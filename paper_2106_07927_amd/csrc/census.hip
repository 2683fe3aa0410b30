// census.hip -- census transform (Sec. 2.2.1 of Ruf et al. 2021; centre
// omitted as in Sec. 2.3.1), gfx950.
//
// A 256-thread workgroup owns a 64 x 16 output tile.  The tile plus its
// (RX, RY) halo is staged once through LDS with the zero margin applied at the
// image border; every thread then computes four consecutive pixels of one row
// with packed byte compares (four comparisons per instruction group).
// Output: one uint64 per pixel, written coalesced along x.
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr int kThreads = 256;

template <int RX, int RY>
struct CensusTile {
    static constexpr int LW = kCensusTileW + 2 * RX;
    static constexpr int LH = kCensusTileH + 2 * RY;
    static constexpr int LWP = (LW + 3) & ~3;
    alignas(16) uint8_t px[LH * LWP];          // rows start on dword boundaries
};

// Unsigned per-byte a < b for four byte pairs at once, result in bit 7 of
// every byte: with t = (a | 0x80) - (b & 0x7F) per byte (never borrows out of
// the byte), a < b iff (a7 < b7) or (a7 == b7 and bit 7 of t is clear).  One
// v_bitop3 evaluates that; its table is f(0xF0, 0xCC, 0xAA) for inputs
// (a, b, t).
__device__ __forceinline__ uint32_t bytes_less(uint32_t a, uint32_t b_low7, uint32_t b) {
    const uint32_t t = (a | 0x80808080u) - b_low7;
    return __builtin_amdgcn_bitop3_b32(a, b, t, 0x4D);
}

// Tile (bx, by) of one image.  Every thread passes the same barriers.  A
// thread owns four consecutive pixels of one tile row: for every window
// offset it compares the four neighbour bytes against the four centres at
// once (bytes_less) and files the four result bits into per-pixel bytes, so
// that after all offsets byte j of acc[g] holds bits 8g .. 8g+7 of pixel j's
// descriptor (counted from the top of a 64-bit word whose leading unused bits
// are zero); a byte transpose then gives each pixel its uint64.
template <int RX, int RY>
__device__ __forceinline__ void census_tile(CensusTile<RX, RY>& t, const uint8_t* __restrict__ img,
                                            int width, int height, int pitch,
                                            uint64_t* __restrict__ out, int bx, int by) {
    using T = CensusTile<RX, RY>;
    const int x0 = bx * kCensusTileW;
    const int y0 = by * kCensusTileH;
    // Every load of the tile is issued before the first LDS write, so staging
    // costs one memory round trip: each position reads the clamped pixel
    // (always inside the image), and a tile that reaches past the border
    // then overwrites those positions with the zero margin.
    constexpr int kN = T::LW * T::LH;
    constexpr int kIt = (kN + kThreads - 1) / kThreads;
    uint32_t v[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = min((int)threadIdx.x + it * kThreads, kN - 1);
        const int ly = i / T::LW, lx = i - ly * T::LW;
        const int cx = min(max(x0 + lx - RX, 0), width - 1), cy = min(max(y0 + ly - RY, 0), height - 1);
        v[it] = img[(size_t)cy * pitch + cx];
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = min((int)threadIdx.x + it * kThreads, kN - 1);   // equal values where clamped
        const int ly = i / T::LW, lx = i - ly * T::LW;
        t.px[ly * T::LWP + lx] = (uint8_t)v[it];
    }
    if (x0 < RX || y0 < RY || x0 + T::LW - RX > width || y0 + T::LH - RY > height) {
        __syncthreads();
        for (int i = threadIdx.x; i < kN; i += kThreads) {
            const int ly = i / T::LW, lx = i - ly * T::LW;
            const int gx = x0 + lx - RX, gy = y0 + ly - RY;
            if (gx < 0 || gx >= width || gy < 0 || gy >= height) t.px[ly * T::LWP + lx] = 0;
        }
    }
    __syncthreads();

    constexpr int kBits = (2 * RX + 1) * (2 * RY + 1) - 1;
    constexpr int kLead = 64 - kBits;                  // unused top bits of the uint64
    constexpr int kWords = (4 + 2 * RX + 3) / 4;       // dwords covering a quad's window row
    const int q = threadIdx.x & 15;                    // quad of the tile row
    const int ty = threadIdx.x >> 4;                   // tile row
    const int gy = y0 + ty;
    const int gx = x0 + 4 * q;
    uint32_t acc[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) acc[g] = 0;
    // the centres: columns 4q + RX .. 4q + RX + 3 of LDS row ty + RY
    const uint32_t* crow = reinterpret_cast<const uint32_t*>(&t.px[(ty + RY) * T::LWP + 4 * q]);
    const uint32_t centre = __builtin_amdgcn_alignbyte(crow[RX / 4 + 1], crow[RX / 4], RX % 4);
    const uint32_t centre_low7 = centre & 0x7F7F7F7Fu;
    int n = 0;
#pragma unroll
    for (int dy = -RY; dy <= RY; ++dy) {
        const uint32_t* row = reinterpret_cast<const uint32_t*>(&t.px[(ty + RY + dy) * T::LWP + 4 * q]);
        uint32_t w[kWords + 1];
#pragma unroll
        for (int k = 0; k < kWords; ++k) w[k] = row[k];
        w[kWords] = 0;
#pragma unroll
        for (int dx = -RX; dx <= RX; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int c = RX + dx;                     // first column of the four neighbours
            const uint32_t nb = __builtin_amdgcn_alignbyte(w[c / 4 + 1], w[c / 4], c % 4);
            const uint32_t lt = bytes_less(nb, centre_low7, centre);
            const int pos = kLead + n;                 // bit index from the top
            const int sh = pos & 7;
            acc[pos >> 3] |= (lt >> sh) & (0x80808080u >> sh);
            ++n;
        }
    }
    // byte transpose: pixel j takes byte j of acc[0..7] (acc[0] the top byte)
    uint64_t d[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t hi = 0, lo = 0;
#pragma unroll
        for (int g = 0; g < 4; ++g) hi |= ((acc[g] >> (8 * j)) & 0xFFu) << (8 * (3 - g));
#pragma unroll
        for (int g = 4; g < 8; ++g) lo |= ((acc[g] >> (8 * j)) & 0xFFu) << (8 * (7 - g));
        d[j] = ((uint64_t)hi << 32) | lo;
    }
    if (gy < height) {
        uint64_t* o = out + (size_t)gy * width + gx;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (gx + j < width) o[j] = d[j];
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

// Both images of one frame in one launch: blockIdx.z selects the image.
template <int RX, int RY>
__global__ __launch_bounds__(kThreads) void census_pair_kernel(Frame f) {
    __shared__ CensusTile<RX, RY> tile;
    const bool right = blockIdx.z != 0;
    census_tile<RX, RY>(tile, right ? f.right : f.left, f.width, f.height, f.pitch,
                        right ? f.census_right : f.census_left, blockIdx.x, blockIdx.y);
}

}  // namespace

hipError_t launch_census_pair(const Frame& f, hipStream_t stream) {
    const dim3 grid(census_blocks_x(f.width), (f.height + kCensusTileH - 1) / kCensusTileH, 2);
    if (f.win_w == 5 && f.win_h == 5) census_pair_kernel<2, 2><<<grid, kThreads, 0, stream>>>(f);
    else census_pair_kernel<4, 3><<<grid, kThreads, 0, stream>>>(f);
    return hipGetLastError();
}

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
