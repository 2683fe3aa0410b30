// cost.hip -- Hamming matching-cost volume, Eq. (image_matching) of Ruf et
// al. 2021 with the census Hamming distance (Sec. 2.1.1) and the 0xFF value
// for matches left of the image (Sec. 2.3.1), gfx950.
//
// A workgroup owns a run of kCostPix pixels of one row.  It stages the left
// descriptors of the run and the right descriptors of [x0 - D + 1, x0 + kCostPix)
// in LDS, so every right descriptor is read from HBM once per run.  When D is
// a multiple of 4 each thread produces 4 consecutive disparities for a run of
// PPG pixels (XOR + two v_bcnt each, packed into one dword), keeping the
// PPG + 3 right descriptors it needs in registers; consecutive threads write
// consecutive dwords, so the uint8 volume is written fully coalesced.
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr int kMaxD = 256;

struct CostTile {
    uint64_t sl[kCostPix];
    uint64_t sr[kCostPix + kMaxD - 1];
};

__device__ __forceinline__ int stage_row(CostTile& t, const uint64_t* __restrict__ cl,
                                         const uint64_t* __restrict__ cr, int width, int ndisp,
                                         int x0, int y) {
    const int npix = min(kCostPix, width - x0);
    const uint64_t* rowl = cl + (size_t)y * width;
    const uint64_t* rowr = cr + (size_t)y * width;
    const int rbase = x0 - (ndisp - 1);
    // entries [0, npix) of the left row, then [0, npix + D - 1) of the right
    // one; all loads are issued before the first LDS write (one round trip)
    const int nl = npix, n = npix + npix + ndisp - 1;
    constexpr int kIt = (kCostPix + kCostPix + kMaxD - 1 + 127) / 128;   // blocks of >= 128 threads
    uint64_t v[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = (int)threadIdx.x + it * (int)blockDim.x;
        v[it] = 0ull;
        if (i < nl) {
            v[it] = rowl[x0 + i];
        } else if (i < n) {
            const int x = rbase + (i - nl);
            if (x >= 0) v[it] = rowr[x];
        }
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = (int)threadIdx.x + it * (int)blockDim.x;
        if (i < nl) t.sl[i] = v[it];
        else if (i < n) t.sr[i - nl] = v[it];
    }
    __syncthreads();
    return npix;
}

// D a multiple of 4.  Thread (q, g) produces disparities 4q .. 4q+3 for the
// PPG consecutive pixels of group g; the right descriptors it needs,
// CR(x - d) for those pixels and disparities, are PPG + 3 consecutive LDS
// entries, read once into registers and reused across the run.  FULL: the
// run holds kCostPix pixels and starts at x0 >= D - 1, so no pixel lies past
// the row's end and no disparity reaches left of the image (no checks).
template <int PPG, bool FULL>
__device__ __forceinline__ void cost_tile_vec4(const CostTile& t, int npix, int ndisp,
                                               uint32_t* __restrict__ out, int x0) {
    const int dwords = ndisp >> 2;                 // dwords per pixel
    const int q = threadIdx.x % dwords;
    const int g = threadIdx.x / dwords;
    const int d0 = q * 4;
    const int p0 = g * PPG;
    if (!FULL && p0 >= npix) return;
    // sr index of CR(x - d) for pixel p: p + ndisp - 1 - d
    const int rb = p0 + ndisp - 1 - d0 - 3;
    uint64_t r[PPG + 3];
#pragma unroll
    for (int k = 0; k < PPG + 3; ++k) r[k] = (FULL || rb + k < npix + ndisp - 1) ? t.sr[rb + k] : 0ull;
    uint32_t* o = out + p0 * dwords + q;
#pragma unroll
    for (int i = 0; i < PPG; ++i) {
        const int p = p0 + i;
        if (FULL || p < npix) {
            const uint64_t l = t.sl[p];
            uint32_t c0 = __popcll(l ^ r[i + 3]);
            uint32_t c1 = __popcll(l ^ r[i + 2]);
            uint32_t c2 = __popcll(l ^ r[i + 1]);
            uint32_t c3 = __popcll(l ^ r[i]);
            if (!FULL) {
                const int x = x0 + p;
                if (x < d0 + 3) {                       // some of d0..d0+3 exceed x
                    c0 = (x - d0 >= 0) ? c0 : 255u;
                    c1 = (x - d0 - 1 >= 0) ? c1 : 255u;
                    c2 = (x - d0 - 2 >= 0) ? c2 : 255u;
                    c3 = (x - d0 - 3 >= 0) ? c3 : 255u;
                }
            }
            // bytes c0..c3 (each <= 255): two shift-ors and one byte permute
            o[i * dwords] = __builtin_amdgcn_perm(c2 | (c3 << 8), c0 | (c1 << 8), 0x05040100u);
        }
    }
}

template <int PPG>
__device__ __forceinline__ void cost_run_vec4(CostTile& t, const uint64_t* __restrict__ cl,
                                              const uint64_t* __restrict__ cr, int width,
                                              int ndisp, uint8_t* __restrict__ cost, int bx, int y) {
    const int x0 = bx * kCostPix;
    const int npix = stage_row(t, cl, cr, width, ndisp, x0, y);
    uint32_t* out = reinterpret_cast<uint32_t*>(cost + ((size_t)y * width + x0) * ndisp);
    if (npix == kCostPix && x0 >= ndisp - 1) cost_tile_vec4<PPG, true>(t, npix, ndisp, out, x0);
    else cost_tile_vec4<PPG, false>(t, npix, ndisp, out, x0);
    __syncthreads();   // the tile is reused by the next work item
}

// Any D: one byte per thread.
__device__ __forceinline__ void cost_run_bytes(CostTile& t, const uint64_t* __restrict__ cl,
                                               const uint64_t* __restrict__ cr, int width,
                                               int ndisp, uint8_t* __restrict__ cost, int bx, int y) {
    const int x0 = bx * kCostPix;
    const int npix = stage_row(t, cl, cr, width, ndisp, x0, y);
    uint8_t* out = cost + ((size_t)y * width + x0) * ndisp;
    for (int b = threadIdx.x; b < npix * ndisp; b += blockDim.x) {
        const int p = b / ndisp, d = b - p * ndisp;
        const int x = x0 + p;
        out[b] = (x - d >= 0) ? (uint8_t)__popcll(t.sl[p] ^ t.sr[p + ndisp - 1 - d]) : (uint8_t)255;
    }
    __syncthreads();
}

template <int PPG>
__global__ __launch_bounds__(256) void cost_kernel_vec4(const uint64_t* __restrict__ cl,
                                                        const uint64_t* __restrict__ cr, int width,
                                                        int ndisp, uint8_t* __restrict__ cost) {
    __shared__ CostTile t;
    cost_run_vec4<PPG>(t, cl, cr, width, ndisp, cost, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void cost_kernel_bytes(const uint64_t* __restrict__ cl,
                                                         const uint64_t* __restrict__ cr, int width,
                                                         int ndisp, uint8_t* __restrict__ cost) {
    __shared__ CostTile t;
    cost_run_bytes(t, cl, cr, width, ndisp, cost, blockIdx.x, blockIdx.y);
}

template <int PPG>
__global__ __launch_bounds__(256) void cost_batch_vec4(WorkList wl) {
    __shared__ CostTile t;
    for (int b = blockIdx.x; b < wl.total; b += gridDim.x) {
        const int fi = find_frame(wl, b);
        const Frame& f = wl.frames[fi];
        const int lb = b - wl.starts[fi];
        const int bxs = cost_blocks_x(f.width);
        cost_run_vec4<PPG>(t, f.census_left, f.census_right, f.width, f.ndisp, f.cost, lb % bxs,
                           lb / bxs);
    }
}

__global__ __launch_bounds__(256) void cost_batch_bytes(WorkList wl) {
    __shared__ CostTile t;
    for (int b = blockIdx.x; b < wl.total; b += gridDim.x) {
        const int fi = find_frame(wl, b);
        const Frame& f = wl.frames[fi];
        const int lb = b - wl.starts[fi];
        const int bxs = cost_blocks_x(f.width);
        cost_run_bytes(t, f.census_left, f.census_right, f.width, f.ndisp, f.cost, lb % bxs, lb / bxs);
    }
}

// pixels per thread group and threads per block for D a multiple of 4
void vec4_shape(int ndisp, int* ppg, int* threads) {
    const int dwords = ndisp / 4;
    const int need = (kCostPix * dwords + 255) / 256;          // pixels per group, at least
    *ppg = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : need <= 16 ? 16 : 32;
    *threads = dwords * ((kCostPix + *ppg - 1) / *ppg);
}

}  // namespace

hipError_t launch_cost(const Frame& f, hipStream_t stream) {
    const dim3 grid(cost_blocks_x(f.width), f.height);
    const uint64_t* cl = f.census_left;
    const uint64_t* cr = f.census_right;
    if ((f.ndisp & 3) == 0) {
        int ppg, threads;
        vec4_shape(f.ndisp, &ppg, &threads);
#define SGM_COST(P) cost_kernel_vec4<P><<<grid, threads, 0, stream>>>(cl, cr, f.width, f.ndisp, f.cost)
        if (ppg == 1) SGM_COST(1);
        else if (ppg == 2) SGM_COST(2);
        else if (ppg == 4) SGM_COST(4);
        else if (ppg == 8) SGM_COST(8);
        else if (ppg == 16) SGM_COST(16);
        else SGM_COST(32);
#undef SGM_COST
    } else {
        cost_kernel_bytes<<<grid, 256, 0, stream>>>(cl, cr, f.width, f.ndisp, f.cost);
    }
    return hipGetLastError();
}

hipError_t launch_cost_batch(const WorkList& wl, int ndisp, hipStream_t stream) {
    const int grid = persistent_grid(wl.total);
    if ((ndisp & 3) == 0) {
        int ppg, threads;
        vec4_shape(ndisp, &ppg, &threads);
#define SGM_COST(P) cost_batch_vec4<P><<<grid, threads, 0, stream>>>(wl)
        if (ppg == 1) SGM_COST(1);
        else if (ppg == 2) SGM_COST(2);
        else if (ppg == 4) SGM_COST(4);
        else if (ppg == 8) SGM_COST(8);
        else if (ppg == 16) SGM_COST(16);
        else SGM_COST(32);
#undef SGM_COST
    } else {
        cost_batch_bytes<<<grid, 256, 0, stream>>>(wl);
    }
    return hipGetLastError();
}

}  // namespace sgm
