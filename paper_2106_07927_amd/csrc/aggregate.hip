// aggregate.hip -- SGM path aggregation, Eq. (sgm_path) and Eq. (sgm_path_aggr)
// of Ruf et al. 2021 (Sec. 2.1.2), gfx950.
//
// Every path direction r splits the image into independent lines (rows for
// the horizontal paths, columns for the vertical ones, and for the diagonals
// W "wrapped" lines that take one pixel per row and restart at the border, as
// the paper's CUDA scheme does in Sec. 2.2.2, so every diagonal line has the
// same length H).  One launch covers all paths of the set, each block owning
// a run of lines of one direction.
//
// A line is owned by LPL consecutive lanes of a wave; each lane keeps 2*NREG
// disparities of the line's current path vector as packed uint16 pairs in
// NREG VGPRs.  Per pixel step:
//   * the cost bytes of the step were loaded PF steps earlier (prefetch ring);
//   * the state is kept normalised, N = L' - m', so the recursion reads
//       L(d) = C(d) + min(N(d), min(N(d-1), N(d+1)) + P1, P2);
//     min(N(d-1), N(d+1)) comes from Q_k = min(P_k, P_k+1) and one alignbit per
//     register, with a single DPP lane shift each way per step;
//   * m = min_d L(d) is a per-lane v_pk_min_u16 tree followed by a DPP
//     all-reduce over the line's lanes;
//   * L is added into S_bar with 32-bit atomics on packed pairs.  They are
//     exact: no partial sum exceeds 16 bits (the ABI checks
//     npaths * (255 + P2) <= 65535), so no carry crosses a half, and integer
//     addition makes the result independent of the order.
// Disparities beyond D (padding lanes) hold 0x7FFF, which never wins a
// minimum and, as a neighbour, never beats the P2 term.
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr uint32_t kBig = 0x7FFFu;
constexpr uint32_t kBig2 = 0x7FFF7FFFu;
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

struct DirTask {
    int dx, dy;      // step r: the predecessor of p is p - r
    int nlines;      // independent lines of this direction
    int nsteps;      // pixels per line
    int block0;      // first block of this direction in the grid
};

struct DirTable {
    DirTask t[8];
    int ndir;
};

// ---- cross-lane helpers for groups of 32 and 64 lanes ---------------------
template <int GROUP>
__device__ __forceinline__ uint32_t line_min(uint32_t v) {
    if constexpr (GROUP <= 16) {
        return group_min<GROUP>(v);
    } else {
        v = group_min<16>(v);
        // rows (0,1) and (2,3) exchange, then the two halves of the wave
        auto s16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        v = min((uint32_t)s16[0], (uint32_t)s16[1]);
        if constexpr (GROUP == 64) {
            auto s32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
            v = min((uint32_t)s32[0], (uint32_t)s32[1]);
        }
        return v;
    }
}

template <int GROUP>
__device__ __forceinline__ uint32_t line_next(uint32_t v, uint32_t edge, bool last) {
    if constexpr (GROUP <= 16) {
        return group_next<GROUP>(v, edge, last);
    } else {
        uint32_t r = (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x130, 0xF, 0xF, false);
        return last ? edge : r;   // wave_shl:1
    }
}

template <int GROUP>
__device__ __forceinline__ uint32_t line_prev(uint32_t v, uint32_t edge, bool first) {
    if constexpr (GROUP <= 16) {
        return group_prev<GROUP>(v, edge, first);
    } else {
        uint32_t r = (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x138, 0xF, 0xF, false);
        return first ? edge : r;  // wave_shr:1
    }
}

// ---- cost vector of one lane for one pixel: 2*NREG bytes ------------------
template <int NREG>
struct CostVec {
    static constexpr int kWords = (NREG + 1) / 2;
    uint32_t w[kWords];
};

template <int NREG, bool ALIGNED>
__device__ __forceinline__ CostVec<NREG> load_cost(const uint8_t* __restrict__ cost,
                                                   size_t off, int d0, int ndisp) {
    CostVec<NREG> c;
#pragma unroll
    for (int i = 0; i < CostVec<NREG>::kWords; ++i) c.w[i] = 0;
    if constexpr (ALIGNED) {
        if (d0 < ndisp) {
            const uint8_t* p = cost + off;
            if constexpr (NREG == 1) {
                c.w[0] = *reinterpret_cast<const uint16_t*>(p);
            } else if constexpr (NREG == 2) {
                c.w[0] = *reinterpret_cast<const uint32_t*>(p);
            } else if constexpr (NREG == 4) {
                const uint2 v = *reinterpret_cast<const uint2*>(p);
                c.w[0] = v.x;
                c.w[1] = v.y;
            } else {
                const uint4 v = *reinterpret_cast<const uint4*>(p);
                c.w[0] = v.x;
                c.w[1] = v.y;
                c.w[2] = v.z;
                c.w[3] = v.w;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < 2 * NREG; ++e) {
            if (d0 + e < ndisp) c.w[e >> 2] |= (uint32_t)cost[off + e] << (8 * (e & 3));
        }
    }
    return c;
}

// bytes 2k, 2k+1 of the vector, zero-extended into a packed pair
template <int NREG>
__device__ __forceinline__ uint32_t cost_pair(const CostVec<NREG>& c, int k) {
    const uint32_t sel = (k & 1) ? 0x0c030c02u : 0x0c010c00u;
    return __builtin_amdgcn_perm(0u, c.w[k >> 1], sel);
}

template <int NREG, bool ALIGNED>
__device__ __forceinline__ void add_atomic(uint16_t* __restrict__ agg, size_t off, int d0,
                                           int ndisp, const uint32_t (&L)[NREG]) {
    if constexpr (ALIGNED) {
        if (d0 < ndisp) {
            uint32_t* p = reinterpret_cast<uint32_t*>(agg + off);
#pragma unroll
            for (int k = 0; k < NREG; ++k) atomicAdd(p + k, L[k]);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 2 * NREG; ++e) {
            if (d0 + e < ndisp) {
                const size_t idx = off + e;
                const uint32_t v = (e & 1) ? (L[e >> 1] >> 16) : (L[e >> 1] & 0xFFFFu);
                uint32_t* word = reinterpret_cast<uint32_t*>(agg) + (idx >> 1);
                atomicAdd(word, v << (16 * (idx & 1)));
            }
        }
    }
}

// One wave's lines of one direction, the whole way along.
template <int NREG, int LPL, int PF, bool ALIGNED>
__device__ __forceinline__ void run_lines(const uint8_t* __restrict__ cost,
                                          uint16_t* __restrict__ agg, int width, int height,
                                          int ndisp, uint32_t p1x2, uint32_t p2x2,
                                          const DirTask& task, int wave_in_dir) {
    constexpr int DPL = 2 * NREG;
    constexpr int LPW = 64 / LPL;
    const int lane = threadIdx.x & 63;
    const int sub = lane % LPL;
    const int line = wave_in_dir * LPW + lane / LPL;
    const bool valid = line < task.nlines;
    const int lc = valid ? line : task.nlines - 1;
    const int d0 = sub * DPL;
    const bool first_lane = sub == 0;
    const bool last_lane = sub == LPL - 1;
    const int dx = task.dx, dy = task.dy;
    const bool diag = dx != 0 && dy != 0;

    // padding: 0x7FFF in every element with d >= D
    uint32_t pad[NREG];
#pragma unroll
    for (int k = 0; k < NREG; ++k) {
        const uint32_t lo = (d0 + 2 * k < ndisp) ? 0u : kBig;
        const uint32_t hi = (d0 + 2 * k + 1 < ndisp) ? 0u : kBig;
        pad[k] = lo | (hi << 16);
    }

    // start pixel of the line
    int x, y;
    if (dy == 0) {
        y = lc;
        x = dx > 0 ? 0 : width - 1;
    } else {
        x = lc;
        y = dy > 0 ? 0 : height - 1;
    }
    int xa = x, ya = y;   // look-ahead position for the prefetch
    const int nsteps = task.nsteps;
    auto advance = [&](int& px, int& py) {
        px += dx;
        py += dy;
        if (diag) {
            if (px == width) px = 0;
            else if (px < 0) px = width - 1;
        }
    };

    CostVec<NREG> ring[PF];
#pragma unroll
    for (int j = 0; j < PF; ++j) {
        if (j < nsteps) ring[j] = load_cost<NREG, ALIGNED>(cost, ((size_t)ya * width + xa) * ndisp + d0, d0, ndisp);
        advance(xa, ya);
    }

    uint32_t P[NREG];
#pragma unroll
    for (int k = 0; k < NREG; ++k) P[k] = pad[k];
    const int restart_x = dx > 0 ? 0 : width - 1;

    for (int s0 = 0; s0 < nsteps; s0 += PF) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int s = s0 + j;
            if (s >= nsteps) break;
            const CostVec<NREG> c = ring[j];
            if (s + PF < nsteps) {
                ring[j] = load_cost<NREG, ALIGNED>(cost, ((size_t)ya * width + xa) * ndisp + d0, d0, ndisp);
            }
            advance(xa, ya);

            // a diagonal line restarts where it wrapped to the other border
            if (diag && s > 0 && x == restart_x) {
#pragma unroll
                for (int k = 0; k < NREG; ++k) P[k] = pad[k];
            }

            // min(N(d-1), N(d+1)) for every register
            uint32_t Q[NREG];
            const uint32_t nxt = line_next<LPL>(P[0], kBig2, last_lane);
#pragma unroll
            for (int k = 0; k + 1 < NREG; ++k) Q[k] = pk_min(P[k], P[k + 1]);
            Q[NREG - 1] = pk_min(P[NREG - 1], nxt);
            const uint32_t qprev = line_prev<LPL>(Q[NREG - 1], P[0], first_lane);

            uint32_t L[NREG];
#pragma unroll
            for (int k = 0; k < NREG; ++k) {
                const uint32_t M = pk_shift_in(Q[k], k == 0 ? qprev : Q[k - 1]);
                uint32_t a = pk_add(M, p1x2);
                a = pk_min(a, P[k]);
                a = pk_min(a, p2x2);
                a = pk_add(a, cost_pair<NREG>(c, k));
                if (ALIGNED ? (LPL * DPL > ndisp) : true) a = pk_max(a, pad[k]);
                L[k] = a;
            }

            uint32_t mm = L[0];
#pragma unroll
            for (int k = 1; k < NREG; ++k) mm = pk_min(mm, L[k]);
            uint32_t m = min(mm & 0xFFFFu, mm >> 16);
            m = line_min<LPL>(m);
            const uint32_t m2 = pk_splat(m);

            if (valid) add_atomic<NREG, ALIGNED>(agg, ((size_t)y * width + x) * ndisp + d0, d0, ndisp, L);

#pragma unroll
            for (int k = 0; k < NREG; ++k) P[k] = pk_sub(L[k], m2);
            advance(x, y);
        }
    }
}

template <int NREG_H, int LPL_H, int NREG_O, int LPL_O, int PF, bool AL_H, bool AL_O>
__global__ __launch_bounds__(kThreads) void aggregate_kernel(const uint8_t* __restrict__ cost,
                                                             uint16_t* __restrict__ agg,
                                                             int width, int height, int ndisp,
                                                             uint32_t p1x2, uint32_t p2x2,
                                                             DirTable tab) {
    int di = 0;
#pragma unroll
    for (int i = 1; i < 8; ++i)
        if (i < tab.ndir && (int)blockIdx.x >= tab.t[i].block0) di = i;
    const DirTask task = tab.t[di];
    const int wave_in_dir = ((int)blockIdx.x - task.block0) * kWaves + (int)(threadIdx.x >> 6);
    if (task.dy == 0) {
        __builtin_amdgcn_s_setprio(2);   // the long horizontal chains go first
        run_lines<NREG_H, LPL_H, PF, AL_H>(cost, agg, width, height, ndisp, p1x2, p2x2, task, wave_in_dir);
    } else {
        run_lines<NREG_O, LPL_O, PF, AL_O>(cost, agg, width, height, ndisp, p1x2, p2x2, task, wave_in_dir);
    }
}

__global__ __launch_bounds__(256) void fill_zero_kernel(uint4* __restrict__ p, size_t n16,
                                                        uint16_t* __restrict__ tail, size_t ntail) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0)
        for (size_t i = threadIdx.x; i < ntail; i += blockDim.x) tail[i] = 0;
}

// Lane layout per disparity range: (NREG, LPL) so that LPL * 2 * NREG >= D.
struct Layout {
    int nreg, lpl;
};

Layout layout_other(int ndisp) {
    if (ndisp <= 2) return {1, 1};
    if (ndisp <= 4) return {2, 1};
    if (ndisp <= 8) return {4, 1};
    if (ndisp <= 16) return {4, 2};
    if (ndisp <= 32) return {4, 4};
    if (ndisp <= 64) return {4, 8};
    if (ndisp <= 128) return {4, 16};
    return {8, 16};
}

Layout layout_horizontal(int ndisp) {
    if (ndisp <= 2) return {1, 1};
    if (ndisp <= 4) return {1, 2};
    if (ndisp <= 8) return {1, 4};
    if (ndisp <= 16) return {1, 8};
    if (ndisp <= 32) return {1, 16};
    if (ndisp <= 64) return {1, 32};
    if (ndisp <= 128) return {1, 64};
    return {2, 64};
}

template <int NREG_H, int LPL_H, int NREG_O, int LPL_O>
hipError_t launch_variant(const uint8_t* cost, int width, int height, int ndisp,
                          uint32_t p1x2, uint32_t p2x2, uint16_t* agg, const DirTable& tab,
                          int nblocks, hipStream_t stream) {
    constexpr int PF = 4;
    const bool al_h = ndisp % (2 * NREG_H) == 0;
    const bool al_o = ndisp % (2 * NREG_O) == 0;
#define SGM_AGG_LAUNCH(AH, AO)                                                                  \
    aggregate_kernel<NREG_H, LPL_H, NREG_O, LPL_O, PF, AH, AO>                                   \
        <<<nblocks, kThreads, 0, stream>>>(cost, agg, width, height, ndisp, p1x2, p2x2, tab)
    if (al_h && al_o) SGM_AGG_LAUNCH(true, true);
    else if (al_h) SGM_AGG_LAUNCH(true, false);
    else if (al_o) SGM_AGG_LAUNCH(false, true);
    else SGM_AGG_LAUNCH(false, false);
#undef SGM_AGG_LAUNCH
    return hipGetLastError();
}

}  // namespace

hipError_t launch_aggregate(const uint8_t* cost, int width, int height, int ndisp,
                            int npaths, int p1, int p2, uint16_t* agg, hipStream_t stream) {
    // S_bar starts at zero; the paths add into it.
    const size_t n = (size_t)width * height * ndisp;
    const size_t n16 = n / 8;
    {
        const int blocks = (int)std::min<size_t>((n16 + 255) / 256 + 1, 4096);
        fill_zero_kernel<<<blocks, 256, 0, stream>>>(reinterpret_cast<uint4*>(agg), n16,
                                                    agg + n16 * 8, n - n16 * 8);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }

    static const int kDirs[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1},
                                    {1, 1}, {-1, 1}, {1, -1}, {-1, -1}};
    const Layout lh = layout_horizontal(ndisp);
    const Layout lo = layout_other(ndisp);
    DirTable tab{};
    int nblocks = 0;
    tab.ndir = npaths;
    for (int i = 0; i < npaths; ++i) {
        DirTask& t = tab.t[i];
        t.dx = kDirs[i][0];
        t.dy = kDirs[i][1];
        const bool horiz = t.dy == 0;
        t.nlines = horiz ? height : width;
        t.nsteps = horiz ? width : height;
        const int lpl = horiz ? lh.lpl : lo.lpl;
        const int lines_per_block = kWaves * (64 / lpl);
        t.block0 = nblocks;
        nblocks += (t.nlines + lines_per_block - 1) / lines_per_block;
    }
    const uint32_t p1x2 = pk_splat((uint32_t)p1);
    const uint32_t p2x2 = pk_splat((uint32_t)p2);

#define SGM_AGG_CASE(NH, LH, NO, LO)                                                          \
    if (lh.nreg == NH && lh.lpl == LH && lo.nreg == NO && lo.lpl == LO)                      \
        return launch_variant<NH, LH, NO, LO>(cost, width, height, ndisp, p1x2, p2x2, agg,   \
                                              tab, nblocks, stream);
    SGM_AGG_CASE(1, 1, 1, 1)
    SGM_AGG_CASE(1, 2, 2, 1)
    SGM_AGG_CASE(1, 4, 4, 1)
    SGM_AGG_CASE(1, 8, 4, 2)
    SGM_AGG_CASE(1, 16, 4, 4)
    SGM_AGG_CASE(1, 32, 4, 8)
    SGM_AGG_CASE(1, 64, 4, 16)
    SGM_AGG_CASE(2, 64, 8, 16)
#undef SGM_AGG_CASE
    return hipErrorInvalidValue;
}

}  // namespace sgm
