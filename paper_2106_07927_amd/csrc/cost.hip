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

constexpr int kPix = 64;
constexpr int kMaxD = 256;

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
    const int per_pass = blockDim.x / dwords;      // pixels per pass
    const int q = threadIdx.x % dwords;
    const int p0 = threadIdx.x / dwords;
    if (p0 >= per_pass) return;
    const int d0 = q * 4;
    uint32_t* out = reinterpret_cast<uint32_t*>(cost + ((size_t)y * width + x0) * ndisp);
    for (int p = p0; p < npix; p += per_pass) {
        const uint64_t l = sl[p];
        const int x = x0 + p;
        // sr index of the right pixel x - d is p + (ndisp - 1) - d
        const int base = p + ndisp - 1 - d0;
        uint32_t c0 = __popcll(l ^ sr[base]);
        uint32_t c1 = __popcll(l ^ sr[base - 1]);
        uint32_t c2 = __popcll(l ^ sr[base - 2]);
        uint32_t c3 = __popcll(l ^ sr[base - 3]);
        if (x < d0 + 3) {                           // some of d0..d0+3 exceed x
            c0 = (x - d0 >= 0) ? c0 : 255u;
            c1 = (x - d0 - 1 >= 0) ? c1 : 255u;
            c2 = (x - d0 - 2 >= 0) ? c2 : 255u;
            c3 = (x - d0 - 3 >= 0) ? c3 : 255u;
        }
        out[p * dwords + q] = c0 | (c1 << 8) | (c2 << 16) | (c3 << 24);
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
        const int dwords = ndisp / 4;
        const int threads = dwords * (dwords >= 256 ? 1 : 256 / dwords);
        cost_kernel_vec4<<<grid, threads, 0, stream>>>(cl, cr, width, ndisp, cost);
    } else {
        cost_kernel_bytes<<<grid, 256, 0, stream>>>(cl, cr, width, ndisp, cost);
    }
    return hipGetLastError();
}

}  // namespace sgm
