// sgm_internal.h -- shared pieces of the gfx950 kernels behind include/sgm.h.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
// Host-side launchers (one per kernel family).  All return hipError_t.
// ---------------------------------------------------------------------------
hipError_t launch_census(const uint8_t* img, int width, int height, int pitch,
                         int win_w, int win_h, uint64_t* out, hipStream_t stream);
hipError_t launch_cost(const uint64_t* cl, const uint64_t* cr, int width, int height,
                       int ndisp, uint8_t* cost, hipStream_t stream);
size_t aggregate_work_bytes(int width, int height, int ndisp, int npaths, int p2);
hipError_t launch_aggregate(const uint8_t* cost, int width, int height, int ndisp,
                            int npaths, int p1, int p2, uint16_t* agg, void* work,
                            hipStream_t stream);
hipError_t launch_wta_lrc(const uint16_t* agg, int width, int height, int ndisp,
                          int lr_tolerance, int median3x3, uint16_t* disp,
                          uint16_t* disp_right, uint16_t* work, hipStream_t stream);

}  // namespace sgm
