// aggregate.hip -- SGM path aggregation, Eq. (sgm_path) and Eq. (sgm_path_aggr)
// of Ruf et al. 2021 (Sec. 2.1.2), gfx950.
//
// Lines.  Every path direction r splits the image into independent lines:
// rows for the horizontal paths, columns for the vertical ones, and for the
// diagonals W "wrapped" lines that take one pixel per row and restart when
// they cross the left/right border -- the paper's CUDA scheme (Sec. 2.2.2) --
// so every diagonal line is H pixels long.  One launch (paths_kernel) runs
// every direction of the set at once, each block owning a run of lines of one
// direction; the long horizontal chains, which bound the launch, get priority.
//
// Lanes.  A line is owned by LPL consecutive lanes; each lane keeps 2*NREG
// disparities of the path vector as packed uint16 pairs.  The state is the
// previous pixel's path vector L' (each value C + A <= 255 + P2), and one
// step reads
//     L(d) = C(d) + min(X(d), m' + P2) - m',
//     X(d) = min(L'(d), min(L'(d-1), L'(d+1)) + P1),  m' = min_d L'(d);
// min(L'(d-1), L'(d+1)) comes from Q_k = min(L'_k, L'_k+1) and one alignbit
// per register, with one DPP lane shift each way per step; m' is a
// v_pk_min_u16 tree plus a DPP / permlane all-reduce over the line's lanes,
// which runs beside X instead of ahead of it.  Disparities beyond D (padding)
// hold 0x7FFF: never a minimum, and as a neighbour never below m' + P2.
//
// Memory.  On this GPU family one counter tracks both loads and stores, so a
// loop that prefetches while it stores would wait for every store each step.
// The loop therefore runs in chunks of K steps: at a chunk boundary it waits
// once, issues the loads of the next chunk, and computes the K steps from
// registers.  No branch guards a load (positions past a line's end are
// clamped to its last pixel).
//
// Sum over paths.  Paths visit a pixel in different orders, so their values
// meet in memory: each path writes its own slice, then merge_kernel forms
// S_bar.  With P2 <= 255 a path writes only its penalty part
//     A_r(p, d) = L_r(p, d) - C(p, d) = min(N(d), N(d +- 1) + P1, P2) in [0, P2]
// as uint8 (exact), and S_bar = R * C + sum_r A_r; otherwise it writes L_r as
// uint16 and S_bar = sum_r L_r.  32-bit atomics on packed pairs would also be
// exact, but device-wide atomics run an order of magnitude slower here than
// the two plain passes.
#include "sgm_internal.h"

namespace sgm {
namespace {

constexpr uint32_t kBig = 0x7FFFu;
constexpr uint32_t kBig2 = 0x7FFF7FFFu;
constexpr int kWaves = 4;                 // waves per block of the path kernel
constexpr int kThreads = 64 * kWaves;

enum Kind : int { kHorizontal = 0, kVertical = 1, kDiagonal = 2 };

// Steps per chunk of the path loop, by lane layout (horizontal lines with one
// / more packed registers per lane, other lines with <= 4 / 8 registers).
// Halving them times the same on the 1242x375, D = 128 frame; 1.5x as many
// no longer fit the registers of the 8-register layout.
constexpr int kStepsH1 = 32, kStepsH2 = 16;
constexpr int kStepsO4 = 16, kStepsO8 = 8;

struct DirTask {
    int dx, dy;      // step r: the predecessor of p is p - r
    int nlines;      // independent lines of this direction
    int nsteps;      // pixels per line
};

// The path set in launch order: the long horizontal chains first, so their
// blocks are dispatched first.  4 paths: LR, RL, TB, BT; 8 adds the diagonals.
__host__ __device__ inline void path_dir(int i, int* dx, int* dy) {
    constexpr int kDirs[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1},
                                 {1, 1}, {-1, 1}, {1, -1}, {-1, -1}};
    *dx = kDirs[i][0];
    *dy = kDirs[i][1];
}

// Blocks of direction i: lines / (lines per block).
__host__ __device__ inline int dir_blocks(int i, int width, int height, int lpl_h, int lpl_o) {
    int dx, dy;
    path_dir(i, &dx, &dy);
    const bool horiz = dy == 0;
    const int nlines = horiz ? height : width;
    const int lines_per_block = kWaves * (64 / (horiz ? lpl_h : lpl_o));
    return (nlines + lines_per_block - 1) / lines_per_block;
}

// Direction and first block of block lb of a frame.
__device__ __forceinline__ DirTask find_dir(int lb, int width, int height, int npaths, int lpl_h,
                                            int lpl_o, int* block0, int* index) {
    int start = 0, i = 0;
    for (; i < npaths - 1; ++i) {
        const int nb = dir_blocks(i, width, height, lpl_h, lpl_o);
        if (lb < start + nb) break;
        start += nb;
    }
    DirTask t;
    path_dir(i, &t.dx, &t.dy);
    const bool horiz = t.dy == 0;
    t.nlines = horiz ? height : width;
    t.nsteps = horiz ? width : height;
    *block0 = start;
    *index = i;
    return t;
}

// ---- cross-lane helpers for lines of up to 64 lanes -----------------------
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
        const uint32_t r = (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x130, 0xF, 0xF, false);
        if constexpr (GROUP == 64) return r;        // wave_shl:1, lane 63 keeps `edge`
        else return last ? edge : r;
    }
}

template <int GROUP>
__device__ __forceinline__ uint32_t line_prev(uint32_t v, uint32_t edge, bool first) {
    if constexpr (GROUP <= 16) {
        return group_prev<GROUP>(v, edge, first);
    } else {
        const uint32_t r = (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x138, 0xF, 0xF, false);
        if constexpr (GROUP == 64) return r;        // wave_shr:1, lane 0 keeps `edge`
        else return first ? edge : r;
    }
}

// ---- cost bytes of one lane for one pixel: 2*NREG bytes --------------------
template <int NREG>
struct CostVec {
    static constexpr int kWords = (NREG + 1) / 2;
    uint32_t w[kWords];
};

template <int NREG, bool ALIGNED>
__device__ __forceinline__ CostVec<NREG> load_cost(const uint8_t* __restrict__ cost, uint32_t off,
                                                   int d0, int ndisp) {
    CostVec<NREG> c;
    if constexpr (ALIGNED) {
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
    } else {
#pragma unroll
        for (int i = 0; i < CostVec<NREG>::kWords; ++i) c.w[i] = 0;
#pragma unroll
        for (int e = 0; e < 2 * NREG; ++e)
            if (d0 + e < ndisp) c.w[e >> 2] |= (uint32_t)cost[off + e] << (8 * (e & 3));
    }
    return c;
}

// bytes 2k, 2k+1 of the vector, zero-extended into a packed pair
template <int NREG>
__device__ __forceinline__ uint32_t cost_pair(const CostVec<NREG>& c, int k) {
    return __builtin_amdgcn_perm(0u, c.w[k >> 1], (k & 1) ? 0x0c030c02u : 0x0c010c00u);
}

// Raw buffer over a uint8 slice: the hardware range check drops a store at
// a byte offset >= `bytes`, so lanes that must not write (padding
// disparities, lines past the direction's end) carry kNoWrite added to their
// offsets and store unconditionally, without an exec-mask branch per step.
// Valid offsets are < 2^31 (volume limit), so biased ones stay in
// [2^31, 2^32) and never wrap back into range.
constexpr uint32_t kNoWrite = 0x80000000u;
constexpr int kRawBufferWord3 = 0x00020000;     // 32-bit data format, no swizzle

__device__ __forceinline__ __amdgpu_buffer_rsrc_t slice_rsrc(void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, kRawBufferWord3);
}

// Writes the step's output of one lane: penalty bytes through the slice's
// buffer resource (U8; `off` is the byte offset of the lane's first
// disparity, biased for a lane that never writes, `eoff` the per-element
// offsets of the unaligned form, and `past` = kNoWrite on the steps after a
// line's end, OR-ed in last so that it cannot cancel a bias), or path values
// (uint16) through a plain pointer, guarded by `write` and `past`.
template <int NREG, bool ALIGNED, bool U8>
__device__ __forceinline__ void store_out(__amdgpu_buffer_rsrc_t rs, uint16_t* __restrict__ wide,
                                          uint32_t off, uint32_t past, bool write, int d0, int ndisp,
                                          const uint32_t (&eoff)[2 * NREG],
                                          const uint32_t (&A)[NREG], const uint32_t (&L)[NREG]) {
    if constexpr (U8) {
        if constexpr (ALIGNED) {
            off |= past;
            if constexpr (NREG == 1) {
                __builtin_amdgcn_raw_buffer_store_b16((uint16_t)__builtin_amdgcn_perm(0u, A[0], 0x0c0c0200u),
                                                      rs, off, 0, 0);
            } else if constexpr (NREG == 2) {
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_amdgcn_perm(A[1], A[0], 0x06040200u), rs, off,
                                                      0, 0);
            } else if constexpr (NREG == 4) {
                typedef uint32_t v2 __attribute__((ext_vector_type(2)));
                v2 v;
                v.x = __builtin_amdgcn_perm(A[1], A[0], 0x06040200u);
                v.y = __builtin_amdgcn_perm(A[3], A[2], 0x06040200u);
                __builtin_amdgcn_raw_buffer_store_b64(v, rs, off, 0, 0);
            } else {
                typedef uint32_t v4 __attribute__((ext_vector_type(4)));
                v4 v;
                v.x = __builtin_amdgcn_perm(A[1], A[0], 0x06040200u);
                v.y = __builtin_amdgcn_perm(A[3], A[2], 0x06040200u);
                v.z = __builtin_amdgcn_perm(A[5], A[4], 0x06040200u);
                v.w = __builtin_amdgcn_perm(A[7], A[6], 0x06040200u);
                __builtin_amdgcn_raw_buffer_store_b128(v, rs, off, 0, 0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 2 * NREG; ++e)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)((e & 1) ? (A[e >> 1] >> 16) : A[e >> 1]), rs,
                                                     (off + eoff[e]) | past, 0, 0);
        }
    } else {
        if (!write || past) return;
        uint16_t* p = wide + off;
        if constexpr (ALIGNED) {
            uint32_t* q = reinterpret_cast<uint32_t*>(p);
#pragma unroll
            for (int k = 0; k < NREG; ++k) q[k] = L[k];
        } else {
#pragma unroll
            for (int e = 0; e < 2 * NREG; ++e)
                if (d0 + e < ndisp) p[e] = (uint16_t)((e & 1) ? (L[e >> 1] >> 16) : L[e >> 1]);
        }
    }
}

// One wave's lines of one direction, the whole way along.  Positions are
// carried as volume offsets that advance by one uniform stride per step;
// only a diagonal line tracks its column, to wrap at the border.
template <int KIND, int NREG, int LPL, int K, bool ALIGNED, bool PADDED, bool U8>
__device__ __forceinline__ void run_lines(const uint8_t* __restrict__ cost, void* __restrict__ slice,
                                          uint32_t slice_bytes, int width, int height, int ndisp,
                                          uint32_t p1x2, uint32_t p2x2, const DirTask& task,
                                          int wave_in_dir) {
    constexpr int DPL = 2 * NREG;
    constexpr int LPW = 64 / LPL;
    const int lane = threadIdx.x & 63;
    const int sub = lane % LPL;
    const int line = wave_in_dir * LPW + lane / LPL;
    const bool line_ok = line < task.nlines;
    const int lc = line_ok ? line : task.nlines - 1;
    const bool d_ok = sub * DPL < ndisp;
    const int d0 = d_ok ? sub * DPL : 0;             // padding lanes read d = 0
    const bool write = line_ok && d_ok;
    const bool first_lane = sub == 0;
    const bool last_lane = sub == LPL - 1;
    const int dx = task.dx, dy = task.dy;
    const int nsteps = task.nsteps;
    const __amdgpu_buffer_rsrc_t rs = slice_rsrc(slice, slice_bytes);
    uint16_t* const wide = static_cast<uint16_t*>(slice);

    uint32_t pad[NREG];
#pragma unroll
    for (int k = 0; k < NREG; ++k) {
        const uint32_t lo = (sub * DPL + 2 * k < ndisp) ? 0u : kBig;
        const uint32_t hi = (sub * DPL + 2 * k + 1 < ndisp) ? 0u : kBig;
        pad[k] = lo | (hi << 16);
    }
    // the no-write bias goes either on the lane's offset (aligned stores) or
    // on each element's offset (unaligned ones), never on both: two biases
    // would wrap back into range
    uint32_t eoff[DPL];
#pragma unroll
    for (int e = 0; e < DPL; ++e) eoff[e] = (uint32_t)e + ((write && d0 + e < ndisp) ? 0u : kNoWrite);

    // first pixel of the line, the per-step stride of the volume offset and,
    // for a diagonal, the stride of the step that wraps to the other border
    int x, y;
    if constexpr (KIND == kHorizontal) {
        y = lc;
        x = dx > 0 ? 0 : width - 1;
    } else {
        x = lc;
        y = dy > 0 ? 0 : height - 1;
    }
    const int32_t stride = (dy * width + dx) * ndisp;
    const int32_t stride_wrap = (dy * width + dx - dx * width) * ndisp;
    const int last_x = dx > 0 ? width - 1 : 0;        // a diagonal wraps after this column
    const int restart_x = dx > 0 ? 0 : width - 1;
    const uint32_t off0 = ((uint32_t)y * (uint32_t)width + (uint32_t)x) * (uint32_t)ndisp + (uint32_t)d0;
    uint32_t soff = off0 + ((U8 && ALIGNED && !write) ? kNoWrite : 0u);  // store side
    uint32_t aoff = off0;                                       // prefetch side (cost bytes)
    int xa = x, sa = 0;

    // advance one step along the line; returns true when a diagonal wraps
    auto advance = [&](uint32_t& off, int& px) {
        if constexpr (KIND == kDiagonal) {
            const bool wrap = px == last_x;
            off += (uint32_t)(wrap ? stride_wrap : stride);
            px = wrap ? restart_x : px + dx;
            return wrap;
        } else {
            off += (uint32_t)stride;
            return false;
        }
    };
    auto fetch = [&]() {
        const CostVec<NREG> c = load_cost<NREG, ALIGNED>(cost, aoff, d0, ndisp);
        if (sa + 1 < nsteps) advance(aoff, xa);      // stay on the last pixel past the end
        ++sa;
        return c;
    };

    CostVec<NREG> nxt[K];
#pragma unroll
    for (int j = 0; j < K; ++j) nxt[j] = fetch();

    // Path values of the previous pixel, L' (not normalised: every valid one
    // is C + A <= 255 + P2, padding holds 0x7FFF).  The line's minimum m' is
    // needed only at the end of a step,
    //     A(d) = min(X(d), m' + P2) - m',  X(d) = min(L'(d), min(L'(d-1), L'(d+1)) + P1),
    // so the cross-lane reduction for m' runs beside the neighbour terms X
    // rather than ahead of them on the step's dependency chain.  At a line's
    // start (and a diagonal's restart) L' = padding: m' = 0 and A = 0.
    uint32_t Lp[NREG];
#pragma unroll
    for (int k = 0; k < NREG; ++k) Lp[k] = pad[k];
    bool restart = false;                             // the line re-entered at the other border

    const int nchunks = (nsteps + K - 1) / K;
    for (int chunk = 0; chunk < nchunks; ++chunk) {
        CostVec<NREG> cur[K];
#pragma unroll
        for (int j = 0; j < K; ++j) cur[j] = nxt[j];
#pragma unroll
        for (int j = 0; j < K; ++j) nxt[j] = fetch();
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int s = chunk * K + j;
            if constexpr (KIND == kDiagonal) {
                // one step in a line's H wraps; skip the selects on the others
                if (__builtin_amdgcn_ballot_w64(restart)) {
#pragma unroll
                    for (int k = 0; k < NREG; ++k) Lp[k] = restart ? pad[k] : Lp[k];
                }
            }
            // m' over the line
            uint32_t mm = Lp[0];
#pragma unroll
            for (int k = 1; k < NREG; ++k) mm = pk_min(mm, Lp[k]);
            const uint32_t m = line_min<LPL>(min(mm & 0xFFFFu, mm >> 16));

            // X(d), independent of m'
            uint32_t Q[NREG];
            const uint32_t nxt0 = line_next<LPL>(Lp[0], kBig2, last_lane);
#pragma unroll
            for (int k = 0; k + 1 < NREG; ++k) Q[k] = pk_min(Lp[k], Lp[k + 1]);
            Q[NREG - 1] = pk_min(Lp[NREG - 1], nxt0);
            const uint32_t qprev = line_prev<LPL>(Q[NREG - 1], Lp[0], first_lane);
            uint32_t X[NREG];
#pragma unroll
            for (int k = 0; k < NREG; ++k)
                X[k] = pk_min(pk_add(pk_shift_in(Q[k], k == 0 ? qprev : Q[k - 1]), p1x2), Lp[k]);

            const uint32_t m2 = pk_splat(m);
            const uint32_t cap = pk_add(m2, p2x2);
            uint32_t A[NREG], L[NREG];
#pragma unroll
            for (int k = 0; k < NREG; ++k) {
                const uint32_t a = pk_sub(pk_min(X[k], cap), m2);
                A[k] = a;
                uint32_t l = pk_add(a, cost_pair<NREG>(cur[j], k));
                if constexpr (PADDED) l = pk_max(l, pad[k]);
                L[k] = l;
            }

            // every step stores, past a line's end out of range: a store
            // count the compiler can see lets each chunk wait for its loads
            // only, not for the stores issued after them
            store_out<NREG, ALIGNED, U8>(rs, wide, soff, s < nsteps ? 0u : kNoWrite, write, d0, ndisp,
                                         eoff, A, L);
            restart = advance(soff, x);
#pragma unroll
            for (int k = 0; k < NREG; ++k) Lp[k] = L[k];
        }
    }
}

// Block lb of the path pass of one frame.
template <int NH, int LH, int NO, int LO, bool ALH, bool PDH, bool ALO, bool PDO, bool U8>
__device__ __forceinline__ void paths_block(const Frame& f, int lb) {
    // steps per chunk: enough to cover a memory round trip, few enough to
    // keep two chunks of cost bytes in registers
    constexpr int KH = NH == 1 ? kStepsH1 : kStepsH2;
    constexpr int KO = NO <= 4 ? kStepsO4 : kStepsO8;
    if (f.paths_fill_keys) {
        // the D^R key map of the selection that follows starts at "no
        // candidate"; every block clears an equal share of it
        int nb = 0;
        for (int i = 0; i < f.npaths; ++i) nb += dir_blocks(i, f.width, f.height, LH, LO);
        const size_t n = (size_t)f.width * f.height;
        const size_t per = (n + nb - 1) / nb;
        const size_t e1 = min(n, (size_t)(lb + 1) * per);
        for (size_t e = (size_t)lb * per + threadIdx.x; e < e1; e += blockDim.x) f.right_keys[e] = 0xFFFFFFFFu;
    }
    int block0, di;
    const DirTask task = find_dir(lb, f.width, f.height, f.npaths, LH, LO, &block0, &di);
    const int wave_in_dir = (lb - block0) * kWaves + (int)(threadIdx.x >> 6);
    void* slice = f.slices + (size_t)di * f.slice_stride * (U8 ? 1 : 2);
    // bytes of this path's slice: the range the buffer stores check
    const uint32_t slice_bytes = (uint32_t)((size_t)f.width * f.height * f.ndisp);
    const uint32_t p1x2 = pk_splat((uint32_t)f.p1);
    const uint32_t p2x2 = pk_splat((uint32_t)f.p2);
    if (task.dy == 0) {
        __builtin_amdgcn_s_setprio(2);
        run_lines<kHorizontal, NH, LH, KH, ALH, PDH, U8>(f.cost, slice, slice_bytes, f.width, f.height,
                                                         f.ndisp, p1x2, p2x2, task, wave_in_dir);
        __builtin_amdgcn_s_setprio(0);
    } else if (task.dx == 0) {
        run_lines<kVertical, NO, LO, KO, ALO, PDO, U8>(f.cost, slice, slice_bytes, f.width, f.height,
                                                       f.ndisp, p1x2, p2x2, task, wave_in_dir);
    } else {
        run_lines<kDiagonal, NO, LO, KO, ALO, PDO, U8>(f.cost, slice, slice_bytes, f.width, f.height,
                                                       f.ndisp, p1x2, p2x2, task, wave_in_dir);
    }
}

template <int NH, int LH, int NO, int LO, bool ALH, bool PDH, bool ALO, bool PDO, bool U8>
__global__ __launch_bounds__(kThreads) void paths_kernel(Frame f) {
    paths_block<NH, LH, NO, LO, ALH, PDH, ALO, PDO, U8>(f, blockIdx.x);
}

template <int NH, int LH, int NO, int LO, bool ALH, bool PDH, bool ALO, bool PDO, bool U8>
__global__ __launch_bounds__(kThreads) void paths_batch_kernel(WorkList wl) {
    for (int b = blockIdx.x; b < wl.total; b += gridDim.x) {
        if (wl.items) {
            paths_block<NH, LH, NO, LO, ALH, PDH, ALO, PDO, U8>(wl.frames[wl.items[2 * b]],
                                                               wl.items[2 * b + 1]);
        } else {
            const int fi = find_frame(wl, b);
            paths_block<NH, LH, NO, LO, ALH, PDH, ALO, PDO, U8>(wl.frames[fi], b - wl.starts[fi]);
        }
    }
}

// S_bar = R * C + sum_r A_r over uint8 penalty slices, for the kMergeChunk
// elements of block lb; each thread sums 16 consecutive elements.
template <int NP, bool PAIR>
__device__ __forceinline__ void merge_u8_block(const Frame& f, int lb) {
    const size_t n = (size_t)f.width * f.height * f.ndisp;
    const size_t e0 = (size_t)lb * kMergeChunk + (size_t)threadIdx.x * 16;
    const uint8_t* cost = f.cost;
    const uint8_t* slices = f.slices;
    uint16_t* agg = f.agg;
    if (e0 + 16 <= n) {
        const size_t i = e0 / 16;
        const uint4 c = reinterpret_cast<const uint4*>(cost)[i];
        uint4 a[NP];
#pragma unroll
        for (int r = 0; r < NP; ++r) a[r] = load_once16(slices + (size_t)r * f.slice_stride + 16 * i);
        uint32_t s[8];
        merge16<NP, PAIR>(c, a, s);
        reinterpret_cast<uint4*>(agg)[2 * i] = make_uint4(s[0], s[1], s[2], s[3]);
        reinterpret_cast<uint4*>(agg)[2 * i + 1] = make_uint4(s[4], s[5], s[6], s[7]);
    } else {
        for (size_t e = e0; e < n && e < e0 + 16; ++e) {
            uint32_t s = (uint32_t)cost[e] * NP;
            for (int r = 0; r < NP; ++r) s += slices[(size_t)r * f.slice_stride + e];
            agg[e] = (uint16_t)s;
        }
    }
}

// S_bar = sum_r L_r over uint16 path slices, 16 elements per thread.
__device__ __forceinline__ void merge_u16_block(const Frame& f, int lb) {
    const size_t n = (size_t)f.width * f.height * f.ndisp;
    const size_t e0 = (size_t)lb * kMergeChunk + (size_t)threadIdx.x * 16;
    const uint16_t* slices = reinterpret_cast<const uint16_t*>(f.slices);
    uint16_t* agg = f.agg;
    if (e0 + 16 <= n) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const size_t i = e0 / 8 + h;
            // cached loads: nontemporal ones measured 13 % slower here
            uint4 s = reinterpret_cast<const uint4*>(slices)[i];
            for (int r = 1; r < f.npaths; ++r) {
                const uint4 a = reinterpret_cast<const uint4*>(slices + (size_t)r * f.slice_stride)[i];
                s.x = pk_add(s.x, a.x);
                s.y = pk_add(s.y, a.y);
                s.z = pk_add(s.z, a.z);
                s.w = pk_add(s.w, a.w);
            }
            reinterpret_cast<uint4*>(agg)[i] = s;
        }
    } else {
        for (size_t e = e0; e < n && e < e0 + 16; ++e) {
            uint32_t s = 0;
            for (int r = 0; r < f.npaths; ++r) s += slices[(size_t)r * f.slice_stride + e];
            agg[e] = (uint16_t)s;
        }
    }
}

// MODE: 0 = uint16 slices, 1 / 2 = uint8 slices of 4 / 8 paths, 3 / 4 = the
// same with P2 <= 127 (bytewise pair sums)
template <int MODE>
__device__ __forceinline__ void merge_block(const Frame& f, int lb) {
    if constexpr (MODE == 0) merge_u16_block(f, lb);
    else merge_u8_block<(MODE == 1 || MODE == 3) ? 4 : 8, (MODE >= 3)>(f, lb);
}

template <int MODE>
__global__ __launch_bounds__(256) void merge_kernel(Frame f) {
    merge_block<MODE>(f, blockIdx.x);
}

template <int MODE>
__global__ __launch_bounds__(256) void merge_batch_kernel(WorkList wl) {
    for (int b = blockIdx.x; b < wl.total; b += gridDim.x) {
        const int fi = find_frame(wl, b);
        merge_block<MODE>(wl.frames[fi], b - wl.starts[fi]);
    }
}

int merge_mode(int npaths, int p2) {
    if (p2 > 255) return 0;
    return (npaths == 4 ? 1 : 2) + (p2 <= 127 ? 2 : 0);
}

// Path-kernel launch for one lane layout; `batch` selects the persistent
// work-list form.
template <int NH, int LH, int NO, int LO>
hipError_t launch_paths_layout(const Frame* one, const WorkList* wl, int ndisp, bool u8,
                               int nblocks, hipStream_t stream) {
    const bool alh = ndisp % (2 * NH) == 0;
    const bool alo = ndisp % (2 * NO) == 0;
    const bool pdh = LH * 2 * NH > ndisp;
    const bool pdo = LO * 2 * NO > ndisp;
    // an ordered item list is dispatched one block per item, so the hardware
    // hands out the longest lines first
    const int grid = (one || wl->items) ? nblocks : persistent_grid(nblocks);
#define SGM_PATHS(A, B, C, D, U)                                                                   \
    do {                                                                                           \
        if (one) paths_kernel<NH, LH, NO, LO, A, B, C, D, U><<<grid, kThreads, 0, stream>>>(*one); \
        else paths_batch_kernel<NH, LH, NO, LO, A, B, C, D, U><<<grid, kThreads, 0, stream>>>(*wl); \
    } while (0)
    if (alh && alo) {
        if (!pdh && !pdo) {
            if (u8) SGM_PATHS(true, false, true, false, true);
            else SGM_PATHS(true, false, true, false, false);
        } else {
            if (u8) SGM_PATHS(true, true, true, true, true);
            else SGM_PATHS(true, true, true, true, false);
        }
    } else {
        if (u8) SGM_PATHS(false, true, false, true, true);
        else SGM_PATHS(false, true, false, true, false);
    }
#undef SGM_PATHS
    return hipGetLastError();
}

hipError_t launch_paths_any(const Frame* one, const WorkList* wl, int ndisp, int variant, bool u8,
                            int nblocks, hipStream_t stream) {
    const PathLayout l = path_layout(ndisp, variant);
#define SGM_CASE(NH, LH, NO, LO)                                                          \
    if (l.nreg_h == NH && l.lpl_h == LH && l.nreg_o == NO && l.lpl_o == LO)              \
        return launch_paths_layout<NH, LH, NO, LO>(one, wl, ndisp, u8, nblocks, stream);
    SGM_CASE(1, 1, 1, 1)
    SGM_CASE(1, 2, 2, 1)
    SGM_CASE(1, 4, 4, 1)
    SGM_CASE(1, 8, 4, 2)
    SGM_CASE(1, 16, 4, 4)
    SGM_CASE(1, 32, 4, 8)
    SGM_CASE(2, 16, 4, 8)
    SGM_CASE(1, 64, 4, 16)
    SGM_CASE(2, 32, 4, 16)
    SGM_CASE(1, 64, 8, 8)
    SGM_CASE(2, 64, 8, 16)
    SGM_CASE(4, 32, 8, 16)
#undef SGM_CASE
    return hipErrorInvalidValue;
}

}  // namespace

// Lane layouts per disparity range.  Variant 0 is the default; the others
// trade the horizontal chains' per-step latency (more lanes per line) against
// total VALU work (more disparities per lane).  All give identical results.
int path_variants(int ndisp) {
    if (ndisp <= 32) return 1;
    if (ndisp <= 64) return 2;
    if (ndisp <= 128) return 3;
    return 2;
}

PathLayout path_layout(int ndisp, int variant) {
    if (ndisp <= 2) return {1, 1, 1, 1};
    if (ndisp <= 4) return {1, 2, 2, 1};
    if (ndisp <= 8) return {1, 4, 4, 1};
    if (ndisp <= 16) return {1, 8, 4, 2};
    if (ndisp <= 32) return {1, 16, 4, 4};
    if (ndisp <= 64) return variant == 1 ? PathLayout{2, 16, 4, 8} : PathLayout{1, 32, 4, 8};
    if (ndisp <= 128) {
        if (variant == 1) return {2, 32, 4, 16};
        if (variant == 2) return {1, 64, 8, 8};
        return {1, 64, 4, 16};
    }
    return variant == 1 ? PathLayout{4, 32, 8, 16} : PathLayout{2, 64, 8, 16};
}

// Variant used when none is asked for (variant < 0): the layout the tuner
// measured fastest for frames of this size class.  Large frames have enough
// horizontal lines to trade per-step latency for fewer instructions.
int default_variant(int width, int height, int ndisp) {
    const long px = (long)width * height;
    if (ndisp <= 32 || ndisp > 128) return 0;
    if (px >= 1500000) return 1;
    if (ndisp > 64 && px >= 400000) return 2;
    return 0;
}

int path_horizontal_blocks(int width, int height, int ndisp, int variant) {
    const PathLayout l = path_layout(ndisp, variant);
    return dir_blocks(0, width, height, l.lpl_h, l.lpl_o) + dir_blocks(1, width, height, l.lpl_h, l.lpl_o);
}

int path_blocks(int width, int height, int ndisp, int npaths, int variant) {
    const PathLayout l = path_layout(ndisp, variant);
    int nb = 0;
    for (int i = 0; i < npaths; ++i) nb += dir_blocks(i, width, height, l.lpl_h, l.lpl_o);
    return nb;
}

// Slices start on 256-element boundaries so every vector access is aligned.
size_t aggregate_slice_elems(int width, int height, int ndisp) {
    const size_t n = (size_t)width * height * ndisp;
    return (n + 255) / 256 * 256;
}

size_t aggregate_work_bytes(int width, int height, int ndisp, int npaths, int p2) {
    return (size_t)npaths * aggregate_slice_elems(width, height, ndisp) * (p2 <= 255 ? 1 : 2);
}

hipError_t launch_paths(const Frame& f, hipStream_t stream) {
    const int variant = (f.variant >= 0 && f.variant < path_variants(f.ndisp))
                            ? f.variant
                            : default_variant(f.width, f.height, f.ndisp);
    const int nb = path_blocks(f.width, f.height, f.ndisp, f.npaths, variant);
    return launch_paths_any(&f, nullptr, f.ndisp, variant, f.p2 <= 255, nb, stream);
}

hipError_t launch_aggregate(const Frame& f, hipStream_t stream) {
    hipError_t e = launch_paths(f, stream);
    if (e != hipSuccess) return e;
    const int mb = merge_blocks((size_t)f.width * f.height * f.ndisp);
    switch (merge_mode(f.npaths, f.p2)) {
        case 0: merge_kernel<0><<<mb, 256, 0, stream>>>(f); break;
        case 1: merge_kernel<1><<<mb, 256, 0, stream>>>(f); break;
        case 2: merge_kernel<2><<<mb, 256, 0, stream>>>(f); break;
        case 3: merge_kernel<3><<<mb, 256, 0, stream>>>(f); break;
        default: merge_kernel<4><<<mb, 256, 0, stream>>>(f); break;
    }
    return hipGetLastError();
}

hipError_t launch_paths_batch(const WorkList& wl, int ndisp, int npaths, int p2, int variant,
                              hipStream_t stream) {
    (void)npaths;
    if (variant < 0 || variant >= path_variants(ndisp)) variant = 0;
    return launch_paths_any(nullptr, &wl, ndisp, variant, p2 <= 255, wl.total, stream);
}

hipError_t launch_merge_batch(const WorkList& wl, int npaths, int p2, hipStream_t stream) {
    const int grid = persistent_grid(wl.total);
    switch (merge_mode(npaths, p2)) {
        case 0: merge_batch_kernel<0><<<grid, 256, 0, stream>>>(wl); break;
        case 1: merge_batch_kernel<1><<<grid, 256, 0, stream>>>(wl); break;
        case 2: merge_batch_kernel<2><<<grid, 256, 0, stream>>>(wl); break;
        case 3: merge_batch_kernel<3><<<grid, 256, 0, stream>>>(wl); break;
        default: merge_batch_kernel<4><<<grid, 256, 0, stream>>>(wl); break;
    }
    return hipGetLastError();
}

}  // namespace sgm
