// cost.hip -- Hamming matching-cost volume, Eq. (image_matching) of Ruf et
// al. 2021 with the census Hamming distance (Sec. 2.1.1) and the 0xFF value
// for matches left of the image (Sec. 2.3.1), gfx950.
//
// A workgroup owns a run of kPix pixels of one row.  It stages the left
// descriptors of the run and the right descriptors of [x0 - D + 1, x0 + kPix)
// in LDS, so every right descriptor is read from HBM once per run.  When D is
// a multiple of 4 each thread produces 4 consecutive disparities of one pixel
// (XOR + two v_bcnt, packed into one dword) and consecutive threads write
// consecutive dwords, so the uint8 volume is written fully coalesced.
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr int kPix = 128;
constexpr int kMaxD = 256;

// D a multiple of 4.  Thread (q, g) produces disparities 4q .. 4q+3 for the
// PPG consecutive pixels of group g; the right descriptors it needs,
// CR(x - d) for those pixels and disparities, are PPG + 3 consecutive LDS
// entries, read once into registers and reused across the run.
template <int PPG>
__global__ __launch_bounds__(256) void cost_kernel_vec4(const uint64_t* __restrict__ cl,
                                                        const uint64_t* __restrict__ cr,
                                                        int width, int ndisp,
                                                        uint8_t* __restrict__ cost) {
    __shared__ uint64_t sl[kPix];
    __shared__ uint64_t sr[kPix + kMaxD - 1];
    const int y = blockIdx.y;
    const int x0 = blockIdx.x * kPix;
    const int npix = min(kPix, width - x0);
    const uint64_t* rowl = cl + (size_t)y * width;
    const uint64_t* rowr = cr + (size_t)y * width;
    const int rbase = x0 - (ndisp - 1);
    for (int i = threadIdx.x; i < npix; i += blockDim.x) sl[i] = rowl[x0 + i];
    for (int i = threadIdx.x; i < npix + ndisp - 1; i += blockDim.x) {
        const int x = rbase + i;
        sr[i] = (x >= 0) ? rowr[x] : 0ull;
    }
    __syncthreads();

    const int dwords = ndisp >> 2;                 // dwords per pixel
    const int q = threadIdx.x % dwords;
    const int g = threadIdx.x / dwords;
    const int d0 = q * 4;
    const int p0 = g * PPG;
    if (p0 >= npix) return;
    // sr index of CR(x - d) for pixel p: p + ndisp - 1 - d
    const int rb = p0 + ndisp - 1 - d0 - 3;
    uint64_t r[PPG + 3];
#pragma unroll
    for (int k = 0; k < PPG + 3; ++k) r[k] = (rb + k < npix + ndisp - 1) ? sr[rb + k] : 0ull;
    uint32_t* out = reinterpret_cast<uint32_t*>(cost + ((size_t)y * width + x0) * ndisp);
#pragma unroll
    for (int i = 0; i < PPG; ++i) {
        const int p = p0 + i;
        if (p < npix) {
            const uint64_t l = sl[p];
            uint32_t c0 = __popcll(l ^ r[i + 3]);
            uint32_t c1 = __popcll(l ^ r[i + 2]);
            uint32_t c2 = __popcll(l ^ r[i + 1]);
            uint32_t c3 = __popcll(l ^ r[i]);
            const int x = x0 + p;
            if (x < d0 + 3) {                       // some of d0..d0+3 exceed x
                c0 = (x - d0 >= 0) ? c0 : 255u;
                c1 = (x - d0 - 1 >= 0) ? c1 : 255u;
                c2 = (x - d0 - 2 >= 0) ? c2 : 255u;
                c3 = (x - d0 - 3 >= 0) ? c3 : 255u;
            }
            out[p * dwords + q] = c0 | (c1 << 8) | (c2 << 16) | (c3 << 24);
        }
    }
}

// Any D: one byte per thread.
__global__ __launch_bounds__(256) void cost_kernel_bytes(const uint64_t* __restrict__ cl,
                                                         const uint64_t* __restrict__ cr,
                                                         int width, int ndisp,
                                                         uint8_t* __restrict__ cost) {
    __shared__ uint64_t sl[kPix];
    __shared__ uint64_t sr[kPix + kMaxD - 1];
    const int y = blockIdx.y;
    const int x0 = blockIdx.x * kPix;
    const int npix = min(kPix, width - x0);
    const uint64_t* rowl = cl + (size_t)y * width;
    const uint64_t* rowr = cr + (size_t)y * width;
    const int rbase = x0 - (ndisp - 1);
    for (int i = threadIdx.x; i < npix; i += blockDim.x) sl[i] = rowl[x0 + i];
    for (int i = threadIdx.x; i < npix + ndisp - 1; i += blockDim.x) {
        const int x = rbase + i;
        sr[i] = (x >= 0) ? rowr[x] : 0ull;
    }
    __syncthreads();
    uint8_t* out = cost + ((size_t)y * width + x0) * ndisp;
    for (int b = threadIdx.x; b < npix * ndisp; b += blockDim.x) {
        const int p = b / ndisp, d = b - p * ndisp;
        const int x = x0 + p;
        out[b] = (x - d >= 0) ? (uint8_t)__popcll(sl[p] ^ sr[p + ndisp - 1 - d]) : (uint8_t)255;
    }
}

}  // namespace

hipError_t launch_cost(const uint64_t* cl, const uint64_t* cr, int width, int height,
                       int ndisp, uint8_t* cost, hipStream_t stream) {
    const dim3 grid((width + kPix - 1) / kPix, height);
    if ((ndisp & 3) == 0) {
        // groups of PPG pixels; at most 256 threads cover all dwords of kPix pixels
        const int dwords = ndisp / 4;
        const int need = (kPix * dwords + 255) / 256;             // pixels per group, at least
        const int ppg = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : need <= 16 ? 16 : 32;
        const int threads = dwords * ((kPix + ppg - 1) / ppg);
        if (ppg == 1) cost_kernel_vec4<1><<<grid, threads, 0, stream>>>(cl, cr, width, ndisp, cost);
        else if (ppg == 2) cost_kernel_vec4<2><<<grid, threads, 0, stream>>>(cl, cr, width, ndisp, cost);
        else if (ppg == 4) cost_kernel_vec4<4><<<grid, threads, 0, stream>>>(cl, cr, width, ndisp, cost);
        else if (ppg == 8) cost_kernel_vec4<8><<<grid, threads, 0, stream>>>(cl, cr, width, ndisp, cost);
        else if (ppg == 16) cost_kernel_vec4<16><<<grid, threads, 0, stream>>>(cl, cr, width, ndisp, cost);
        else cost_kernel_vec4<32><<<grid, threads, 0, stream>>>(cl, cr, width, ndisp, cost);
    } else {
        cost_kernel_bytes<<<grid, 256, 0, stream>>>(cl, cr, width, ndisp, cost);
    }
    return hipGetLastError();
}

}  // namespace sgm
