// paths.hip -- the path pass of the SGM aggregation, Eq. (sgm_path) and Eq. (sgm_path_aggr)
// of Ruf et al. 2021 (Sec. 2.1.2), gfx950.
//
// This file is compiled once per lane layout (-DSGM_PATH_LAYOUT=<index into
// kPathLayouts>) and per form (-DSGM_PATH_PART=0: the single-frame kernel,
// 1: the work-list kernel), so the kernels build in parallel; aggregate.hip
// holds the pass that sums the slices and picks the layout.
//
// Lines.  Every path direction r splits the image into independent lines:
// rows for the horizontal paths, columns for the vertical ones, and for the
// diagonals W "wrapped" lines that take one pixel per row and restart when
// they cross the left/right border -- the paper's CUDA scheme (Sec. 2.2.2) --
// so every diagonal line is H pixels long.  The path set is taken as pairs of
// opposite directions (r, -r): (LR, RL), (TB, BT), (TLBR, BRTL), (TRBL, BLTR).
// Both directions of a pair cover the same lines, in opposite orders (for a
// diagonal, the same wrapped pixel sequence backwards).
//
// Pairs.  A block holds a forward wave that walks r along a group of lines
// and a reverse wave that walks -r along the same lines (two such pairs per
// block).  Each writes its
// penalty part A (or L, see below) for its own first half of every line
// into the pair's slice; after a workgroup barrier each adds the value the
// other wave left at the pixels of its second half and writes the sum.  So a
// pair slice holds, exactly, A_r + A_-r at every pixel: with P2 <= 127 both
// lie in [0, P2] and the sum fits a byte; otherwise the slice is uint16 and
// holds L_r + L_-r.  The selection then reads R/2 slices, not R.  Both waves
// run the same number of steps T = n + delta (a multiple of the chunk length
// K): the forward wave's extra steps come after its line's end, the reverse
// wave's before its start, so that each wave's barrier falls on a chunk
// boundary of its own.  Extra steps load whatever their offset holds (the
// loads are range-checked buffer loads), never store, and the reverse wave
// restarts its recursion after them.
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
// once, issues the loads of the next chunk (cost bytes, and in the second
// half the partner's values), and computes the K steps from registers.
// Cost and partner loads and the slice stores go through raw buffer
// resources: offsets past the volume read as zero and stores there are
// dropped, so positions beyond a line need no clamping; a lane or step that
// must not write carries kNoWrite added to its offset.
#include "sgm_internal.h"

#include <type_traits>

namespace sgm {
namespace {

constexpr uint32_t kBig = 0x7FFFu;
constexpr uint32_t kBig2 = 0x7FFF7FFFu;
// A block is four waves: the forward waves of two line groups, then their
// reverse waves.  Four-wave blocks put one wave on each SIMD of a compute
// unit; two-wave blocks let the dispatcher stack waves of the long
// horizontal lines on the same SIMD (measured: 227 -> 197 us per frame at
// 1242x375, D = 128).
constexpr int kThreads = 256;

enum Kind : int { kHorizontal = 0, kVertical = 1, kDiagonal = 2 };

// Steps per chunk of the path loop, by lane layout (horizontal lines with one
// / more packed registers per lane, other lines with <= 4 / 8 registers).
constexpr int kStepsH1 = 32, kStepsH2 = 16;
constexpr int kStepsO4 = 16, kStepsO8 = 8;

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

// Minimum over all 64 lanes as a wave-uniform value: row reductions, the
// row_bcast:15 / row_bcast:31 steps that carry it to lane 63, one readlane.
// The result lives in a scalar register, so the splat and the cap that
// follow run on the scalar unit, off the vector chain of the step.
__device__ __forceinline__ uint32_t wave_min_uniform(uint32_t v) {
    v = group_min<16>(v);
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)v, 0x142, 0xA, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)v, 0x143, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
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

// ---- bytes of one lane for one pixel: 2*NREG bytes --------------------------
template <int NREG>
struct ByteVec {
    static constexpr int kWords = (NREG + 1) / 2;
    uint32_t w[kWords];
};

// uint16 values of one lane for one pixel: 2*NREG values
template <int NREG>
struct WideVec {
    uint32_t w[NREG];
};

typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr uint32_t kNoWrite = 0x80000000u;
constexpr int kRawBufferWord3 = 0x00020000;     // 32-bit data format, no swizzle

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             kRawBufferWord3);
}

// 2*NREG bytes at byte offset `off` (out of range: zero)
template <int NREG, bool ALIGNED>
__device__ __forceinline__ ByteVec<NREG> load_bytes(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    ByteVec<NREG> c;
    if constexpr (ALIGNED) {
        if constexpr (NREG == 1) {
            c.w[0] = __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
        } else if constexpr (NREG == 2) {
            c.w[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        } else if constexpr (NREG == 4) {
            const v2u v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
            c.w[0] = v.x;
            c.w[1] = v.y;
        } else {
            const v4u v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
            c.w[0] = v.x;
            c.w[1] = v.y;
            c.w[2] = v.z;
            c.w[3] = v.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < ByteVec<NREG>::kWords; ++i) c.w[i] = 0;
#pragma unroll
        for (int e = 0; e < 2 * NREG; ++e)
            c.w[e >> 2] |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, off + e, 0, 0) << (8 * (e & 3));
    }
    return c;
}

// 2*NREG uint16 values at byte offset `off` (out of range: zero)
template <int NREG, bool ALIGNED>
__device__ __forceinline__ WideVec<NREG> load_wide(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    WideVec<NREG> v;
    if constexpr (ALIGNED && NREG == 1) {
        v.w[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    } else if constexpr (ALIGNED && NREG == 2) {
        const v2u a = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
        v.w[0] = a.x;
        v.w[1] = a.y;
    } else if constexpr (ALIGNED && NREG % 4 == 0) {
#pragma unroll
        for (int q = 0; q < NREG / 4; ++q) {
            const v4u a = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16 * q, 0, 0);
            v.w[4 * q] = a.x;
            v.w[4 * q + 1] = a.y;
            v.w[4 * q + 2] = a.z;
            v.w[4 * q + 3] = a.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NREG; ++k)
            v.w[k] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, off + 4 * k, 0, 0) |
                     ((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, off + 4 * k + 2, 0, 0) << 16);
    }
    return v;
}

// bytes 2k, 2k+1 of the vector, zero-extended into a packed pair
template <int NREG>
__device__ __forceinline__ uint32_t cost_pair(const ByteVec<NREG>& c, int k) {
    return __builtin_amdgcn_perm(0u, c.w[k >> 1], (k & 1) ? 0x0c030c02u : 0x0c010c00u);
}

// Partner values a wave adds before storing: bytes (uint8 slices) or packed
// uint16 pairs (wide slices); zero in a wave's first half.
template <int NREG, bool U8>
struct Partner;
template <int NREG>
struct Partner<NREG, true> {
    ByteVec<NREG> v;
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int i = 0; i < ByteVec<NREG>::kWords; ++i) v.w[i] = 0;
    }
    template <bool ALIGNED>
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t elem) {
        v = load_bytes<NREG, ALIGNED>(rs, elem);
    }
};
template <int NREG>
struct Partner<NREG, false> {
    WideVec<NREG> v;
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int i = 0; i < NREG; ++i) v.w[i] = 0;
    }
    template <bool ALIGNED>
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t elem) {
        v = load_wide<NREG, ALIGNED>(rs, 2u * elem);
    }
};


// Stores one lane's step: uint8 slices take the penalty bytes A plus the
// partner's bytes (each byte sum <= 2 P2 <= 254: no carry between bytes);
// wide slices take the path values L plus the partner's, as uint16.  `off`
// is the element offset of the lane's first disparity, kNoWrite for a step
// outside the line.  For aligned uint8 stores `bias` is the lane's no-write
// bias; for unaligned ones `ebias` holds one per element, OR-ed (never
// added) onto the offset so that two biases cannot wrap back into range.
// Wide stores are guarded by a branch instead: their byte offsets use all
// 32 bits.
template <int NREG, bool ALIGNED, bool U8>
__device__ __forceinline__ void store_step(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t bias,
                                           bool write, const uint32_t (&ebias)[2 * NREG],
                                           const uint32_t (&A)[NREG], const uint32_t (&L)[NREG],
                                           const Partner<NREG, U8>& part) {
    if constexpr (U8) {
        constexpr int W = ByteVec<NREG>::kWords;
        uint32_t pk[W];
        if constexpr (NREG == 1) {
            pk[0] = __builtin_amdgcn_perm(0u, A[0], 0x0c0c0200u);
        } else {
#pragma unroll
            for (int i = 0; i < W; ++i) pk[i] = __builtin_amdgcn_perm(A[2 * i + 1], A[2 * i], 0x06040200u);
        }
#pragma unroll
        for (int i = 0; i < W; ++i) pk[i] += part.v.w[i];
        if constexpr (ALIGNED) {
            const uint32_t o = off | bias;
            if constexpr (NREG == 1) {
                __builtin_amdgcn_raw_buffer_store_b16((uint16_t)pk[0], rs, o, 0, 0);
            } else if constexpr (NREG == 2) {
                __builtin_amdgcn_raw_buffer_store_b32(pk[0], rs, o, 0, 0);
            } else if constexpr (NREG == 4) {
                v2u v;
                v.x = pk[0];
                v.y = pk[1];
                __builtin_amdgcn_raw_buffer_store_b64(v, rs, o, 0, 0);
            } else {
                v4u v;
                v.x = pk[0];
                v.y = pk[1];
                v.z = pk[2];
                v.w = pk[3];
                __builtin_amdgcn_raw_buffer_store_b128(v, rs, o, 0, 0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 2 * NREG; ++e)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(pk[e >> 2] >> (8 * (e & 3))), rs,
                                                     (off | ebias[e]) + (uint32_t)e, 0, 0);
        }
    } else {
        if (!write || off >= kNoWrite) return;
        uint32_t s[NREG];
#pragma unroll
        for (int k = 0; k < NREG; ++k) s[k] = pk_add(L[k], part.v.w[k]);
        const uint32_t boff = 2u * off;
        if constexpr (ALIGNED && NREG == 1) {
            __builtin_amdgcn_raw_buffer_store_b32(s[0], rs, boff, 0, 0);
        } else if constexpr (ALIGNED && NREG == 2) {
            v2u v;
            v.x = s[0];
            v.y = s[1];
            __builtin_amdgcn_raw_buffer_store_b64(v, rs, boff, 0, 0);
        } else if constexpr (ALIGNED && NREG % 4 == 0) {
#pragma unroll
            for (int q = 0; q < NREG / 4; ++q) {
                v4u v;
                v.x = s[4 * q];
                v.y = s[4 * q + 1];
                v.z = s[4 * q + 2];
                v.w = s[4 * q + 3];
                __builtin_amdgcn_raw_buffer_store_b128(v, rs, boff + 16 * q, 0, 0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 2 * NREG; ++e)
                if (ebias[e] == 0)
                    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(s[e >> 1] >> (16 * (e & 1))), rs,
                                                          boff + 2 * e, 0, 0);
        }
    }
}

// One step of the recursion for one lane: A (penalty part) and the new L',
// both as packed uint16 pairs.
template <int NREG, int LPL, bool PADDED>
__device__ __forceinline__ void path_step(uint32_t (&Lp)[NREG], const ByteVec<NREG>& c, uint32_t p1x2,
                                          uint32_t p2x2, const uint32_t (&pad)[NREG], bool first_lane,
                                          bool last_lane, uint32_t (&A)[NREG]) {
    // m' over the line
    uint32_t mm = Lp[0];
#pragma unroll
    for (int k = 1; k < NREG; ++k) mm = pk_min(mm, Lp[k]);
    uint32_t m;
    if constexpr (LPL == 64) m = wave_min_uniform(min(mm & 0xFFFFu, mm >> 16));
    else m = line_min<LPL>(min(mm & 0xFFFFu, mm >> 16));

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
    const uint32_t cap = m2 + p2x2;              // no carry crosses the halves: m' + P2 < 2^16
#pragma unroll
    for (int k = 0; k < NREG; ++k) {
        const uint32_t a = pk_sub(pk_min(X[k], cap), m2);
        A[k] = a;
        uint32_t l = pk_add(a, cost_pair<NREG>(c, k));
        if constexpr (PADDED) l = pk_max(l, pad[k]);
        Lp[k] = l;
    }
}

// Chunk schedule of one line pair of n pixels: both waves run T = n + delta
// steps (T a multiple of K).  The forward wave's step s is its pixel s; the
// reverse wave's step s is its pixel s - delta.  The forward wave writes its
// own values for steps [0, split_fwd), the reverse wave for steps
// [0, split_rev) -- together every pixel of the line exactly once, with each
// split on a chunk boundary -- and then each completes the pixels the other
// wrote.
struct Schedule {
    int T, delta, split_fwd, split_rev;
    __host__ __device__ Schedule(int n, int K) {
        delta = (K - n % K) % K;
        T = n + delta;
        split_fwd = K * (T / (2 * K));
        split_rev = T - split_fwd;
    }
};

__device__ __forceinline__ void pair_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Position of one lane along its line: the element offset of the next step to
// lay out and, for a diagonal, its column.  A diagonal's steps come with
// their restart flags: the recursion starts afresh there (the line re-entered
// at the other border, or the reverse wave's first pixel after its extra
// steps).  Other lines restart only at the reverse wave's first pixel, which
// the loop handles itself.
template <int KIND>
struct Walker {
    int t;                 // own pixel index of the next step (< 0: before the line)
    int n;                 // pixels of the line
    uint32_t e;            // element offset of pixel t (valid for 0 <= t < n)
    int x;                 // diagonal: column of pixel t
    bool wrapped;          // diagonal: pixel t starts a new segment
    bool restart_first;    // pixel 0 follows extra steps
    int32_t stride, stride_wrap;
    int last_x, restart_x, sdx;

    // offset of the next step, kNoWrite outside the line (CHECKED: the step
    // may lie outside it); advances
    template <bool CHECKED>
    __device__ __forceinline__ uint32_t next(bool& restart) {
        uint32_t off;
        if (CHECKED && (t < 0 || t >= n)) {
            off = kNoWrite;
            restart = false;
        } else {
            off = e;
            if constexpr (KIND == kDiagonal) {
                restart = wrapped;
                wrapped = x == last_x;
                e += (uint32_t)(wrapped ? stride_wrap : stride);
                x = wrapped ? restart_x : x + sdx;
                if (CHECKED && t == 0) restart = restart || restart_first;
            } else {
                restart = false;
                e += (uint32_t)stride;
            }
        }
        ++t;
        return off;
    }
};

// One wave of a line pair, the whole way along.  The offsets of the steps of
// the next chunk are laid out one chunk ahead and serve its cost loads,
// partner loads and stores.
template <int KIND, int NREG, int LPL, int K, bool ALIGNED, bool PADDED, bool U8>
__device__ __forceinline__ void run_wave(const Frame& f, uint8_t* __restrict__ slice, int q, bool fwd,
                                         int group) {
    constexpr int DPL = 2 * NREG;
    constexpr int LPW = 64 / LPL;
    const int width = f.width, height = f.height, ndisp = f.ndisp;
    const int lane = threadIdx.x & 63;
    const int sub = lane % LPL;
    const int nlines = pair_lines(q, width, height);
    const int line = group * LPW + lane / LPL;
    const bool line_ok = line < nlines;
    const int lc = line_ok ? line : nlines - 1;
    const bool d_ok = sub * DPL < ndisp;
    const int d0 = d_ok ? sub * DPL : 0;             // padding lanes read d = 0
    const bool write = line_ok && d_ok;
    const bool first_lane = sub == 0;
    const bool last_lane = sub == LPL - 1;
    const int n = KIND == kHorizontal ? width : height;
    const Schedule sch(n, K);
    const int dlt = fwd ? 0 : sch.delta;             // pixel of step s = s - dlt
    const int nchunks = sch.T / K;
    const int c_split = (fwd ? sch.split_fwd : sch.split_rev) / K;
    // the forward wave's last chunk holds steps past its line's end
    const int c_last_checked = (fwd && sch.delta > 0) ? nchunks - 1 : -1;

    const uint32_t vol = (uint32_t)((size_t)width * height * ndisp);
    const __amdgpu_buffer_rsrc_t rc = buffer_rsrc(f.cost, vol);
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(slice, U8 ? vol : 2u * vol);
    const uint32_t p1x2 = pk_splat((uint32_t)f.p1);
    const uint32_t p2x2 = pk_splat((uint32_t)f.p2);

    uint32_t pad[NREG];
#pragma unroll
    for (int k = 0; k < NREG; ++k) {
        const uint32_t lo = (sub * DPL + 2 * k < ndisp) ? 0u : kBig;
        const uint32_t hi = (sub * DPL + 2 * k + 1 < ndisp) ? 0u : kBig;
        pad[k] = lo | (hi << 16);
    }
    uint32_t ebias[DPL];
#pragma unroll
    for (int e = 0; e < DPL; ++e) ebias[e] = (write && d0 + e < ndisp) ? 0u : kNoWrite;
    const uint32_t lane_bias = (U8 && ALIGNED && !write) ? kNoWrite : 0u;

    // the wave's own direction and first pixel; the reverse wave starts where
    // the forward line ends
    int dx, dy;
    pair_dir(q, &dx, &dy);
    const int sdx = fwd ? dx : -dx, sdy = fwd ? dy : -dy;
    int x0, y0;
    if constexpr (KIND == kHorizontal) {
        y0 = lc;
        x0 = sdx > 0 ? 0 : width - 1;
    } else if constexpr (KIND == kVertical) {
        x0 = lc;
        y0 = sdy > 0 ? 0 : height - 1;
    } else {
        y0 = sdy > 0 ? 0 : height - 1;
        const int e = fwd ? lc : (lc + dx * (height - 1)) % width;
        x0 = e < 0 ? e + width : e;
    }
    Walker<KIND> wk;
    wk.t = -dlt;
    wk.n = n;
    wk.e = ((uint32_t)y0 * (uint32_t)width + (uint32_t)x0) * (uint32_t)ndisp + (uint32_t)d0;
    wk.x = x0;
    wk.wrapped = false;
    wk.restart_first = dlt > 0;
    wk.stride = (sdy * width + sdx) * ndisp;
    wk.stride_wrap = (sdy * width + sdx - sdx * width) * ndisp;
    wk.last_x = sdx > 0 ? width - 1 : 0;
    wk.restart_x = sdx > 0 ? 0 : width - 1;
    wk.sdx = sdx;

    // the next chunk: step offsets, restart flags, cost bytes, partner values
    uint32_t offs_n[K];
    bool rst_n[K];
    ByteVec<NREG> cn[K];
    Partner<NREG, U8> pn[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        offs_n[j] = wk.template next<true>(rst_n[j]);
        cn[j] = load_bytes<NREG, ALIGNED>(rc, offs_n[j]);
        pn[j].clear();
    }

    // L' of the previous pixel; padding at a line's start
    uint32_t Lp[NREG];
#pragma unroll
    for (int k = 0; k < NREG; ++k) Lp[k] = pad[k];

    // one chunk; CHECK: some step of it may restart the recursion
    auto chunk = [&](int c, auto check) {
        constexpr bool CHECK = decltype(check)::value;
        uint32_t offs[K];
        bool rst[K];
        ByteVec<NREG> cur[K];
        Partner<NREG, U8> pc[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            offs[j] = offs_n[j];
            rst[j] = rst_n[j];
            cur[j] = cn[j];
            pc[j] = pn[j];
        }
        if (c == c_split) {
            // the other wave has written the pixels this one completes
            pair_barrier();
#pragma unroll
            for (int j = 0; j < K; ++j) pc[j].template load<ALIGNED>(rs, offs[j]);
        }
        if (c + 1 < nchunks) {
            if (c + 1 == c_last_checked) {
#pragma unroll
                for (int j = 0; j < K; ++j) offs_n[j] = wk.template next<true>(rst_n[j]);
            } else {
#pragma unroll
                for (int j = 0; j < K; ++j) offs_n[j] = wk.template next<false>(rst_n[j]);
            }
#pragma unroll
            for (int j = 0; j < K; ++j) cn[j] = load_bytes<NREG, ALIGNED>(rc, offs_n[j]);
            if (c >= c_split) {
#pragma unroll
                for (int j = 0; j < K; ++j) pn[j].template load<ALIGNED>(rs, offs_n[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if constexpr (CHECK && KIND == kDiagonal) {
                // a restart is rare; skip the selects on the other steps
                if (__builtin_amdgcn_ballot_w64(rst[j])) {
#pragma unroll
                    for (int k = 0; k < NREG; ++k) Lp[k] = rst[j] ? pad[k] : Lp[k];
                }
            } else if constexpr (CHECK) {
                // the reverse wave's first pixel after its extra steps
                if (j == dlt) {
#pragma unroll
                    for (int k = 0; k < NREG; ++k) Lp[k] = pad[k];
                }
            }
            uint32_t A[NREG];
            path_step<NREG, LPL, PADDED>(Lp, cur[j], p1x2, p2x2, pad, first_lane, last_lane, A);
            store_step<NREG, ALIGNED, U8>(rs, offs[j], lane_bias, write, ebias, A, Lp, pc[j]);
        }
    };
    for (int c = 0; c < nchunks; ++c) {
        if (KIND == kDiagonal || (c == 0 && dlt > 0)) chunk(c, std::true_type{});
        else chunk(c, std::false_type{});
    }
    if (c_split == nchunks) pair_barrier();
}

// Block lb of the path pass of one frame: pair q, line groups 2g and 2g + 1;
// waves 0, 1 walk the forward direction along them, waves 2, 3 the reverse
// one.
template <int NH, int LH, int NO, int LO, bool ALH, bool PDH, bool ALO, bool PDO, bool U8>
__device__ __forceinline__ void paths_block(const Frame& f, int lb) {
    // steps per chunk: enough to cover a memory round trip, few enough to
    // keep two chunks of cost bytes and partner values in registers
    constexpr int KH = NH == 1 ? kStepsH1 : kStepsH2;
    constexpr int KO = NO <= 4 ? kStepsO4 : kStepsO8;
    const int npairs = f.npaths / 2;
    if (f.paths_fill_keys) {
        // the D^R key map of the selection that follows starts at "no
        // candidate"; every block clears an equal share of it
        int nb = 0;
        for (int q = 0; q < npairs; ++q) nb += pair_blocks(q, f.width, f.height, LH, LO);
        const size_t n = (size_t)f.width * f.height;
        const size_t per = (n + nb - 1) / nb;
        const size_t e1 = min(n, (size_t)(lb + 1) * per);
        for (size_t e = (size_t)lb * per + threadIdx.x; e < e1; e += blockDim.x) f.right_keys[e] = 0xFFFFFFFFu;
    }
    int q = 0, start = 0;
    for (; q < npairs - 1; ++q) {
        const int nb = pair_blocks(q, f.width, f.height, LH, LO);
        if (lb < start + nb) break;
        start += nb;
    }
    const int group = 2 * (lb - start) + ((threadIdx.x >> 6) & 1);
    const bool fwd = threadIdx.x < 128;
    uint8_t* slice = f.slices + (size_t)q * f.slice_stride * (U8 ? 1 : 2);
    if (q == 0) {
        __builtin_amdgcn_s_setprio(2);
        run_wave<kHorizontal, NH, LH, KH, ALH, PDH, U8>(f, slice, q, fwd, group);
        __builtin_amdgcn_s_setprio(0);
    } else if (q == 1) {
        run_wave<kVertical, NO, LO, KO, ALO, PDO, U8>(f, slice, q, fwd, group);
    } else {
        run_wave<kDiagonal, NO, LO, KO, ALO, PDO, U8>(f, slice, q, fwd, group);
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

// Path-kernel launches for one lane layout: the single-frame kernel, or the
// persistent work-list form.  The two are compiled in separate objects
// (SGM_PATH_PART 0 and 1), so the library's longest compile splits in two.
struct LayoutFlags {
    bool alh, alo, padded;
};

__host__ inline LayoutFlags layout_flags(int nh, int lh, int no, int lo, int ndisp) {
    return {ndisp % (2 * nh) == 0, ndisp % (2 * no) == 0, lh * 2 * nh > ndisp || lo * 2 * no > ndisp};
}

#if SGM_PATH_PART == 0
template <int NH, int LH, int NO, int LO>
hipError_t launch_paths_single(const Frame& one, int ndisp, bool u8, int nblocks, hipStream_t stream) {
    const LayoutFlags fl = layout_flags(NH, LH, NO, LO, ndisp);
#define SGM_PATHS(A, B, C, D, U) \
    paths_kernel<NH, LH, NO, LO, A, B, C, D, U><<<nblocks, kThreads, 0, stream>>>(one)
    if (fl.alh && fl.alo) {
        if (!fl.padded) {
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
#else
template <int NH, int LH, int NO, int LO>
hipError_t launch_paths_worklist(const WorkList& wl, int ndisp, bool u8, int nblocks, hipStream_t stream) {
    const LayoutFlags fl = layout_flags(NH, LH, NO, LO, ndisp);
    // an ordered item list is dispatched one block per item, so the hardware
    // hands out the longest lines first
    const int grid = wl.items ? nblocks : persistent_grid(nblocks);
#define SGM_PATHS(A, B, C, D, U) \
    paths_batch_kernel<NH, LH, NO, LO, A, B, C, D, U><<<grid, kThreads, 0, stream>>>(wl)
    if (fl.alh && fl.alo) {
        if (!fl.padded) {
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
#endif

}  // namespace

#ifndef SGM_PATH_LAYOUT
#error "paths.hip is compiled once per lane layout: -DSGM_PATH_LAYOUT=<index>"
#endif
#if !defined(SGM_PATH_PART) || (SGM_PATH_PART != 0 && SGM_PATH_PART != 1)
#error "paths.hip is compiled in two parts: -DSGM_PATH_PART=0 (single frame) or 1 (work list)"
#endif

#if SGM_PATH_PART == 0
template <>
hipError_t launch_paths_layout_id<SGM_PATH_LAYOUT>(const Frame& one, int ndisp, bool u8, int nblocks,
                                                   hipStream_t stream) {
    constexpr PathLayout L = kPathLayouts[SGM_PATH_LAYOUT];
    return launch_paths_single<L.nreg_h, L.lpl_h, L.nreg_o, L.lpl_o>(one, ndisp, u8, nblocks, stream);
}
#else
template <>
hipError_t launch_paths_batch_layout_id<SGM_PATH_LAYOUT>(const WorkList& wl, int ndisp, bool u8,
                                                         int nblocks, hipStream_t stream) {
    constexpr PathLayout L = kPathLayouts[SGM_PATH_LAYOUT];
    return launch_paths_worklist<L.nreg_h, L.lpl_h, L.nreg_o, L.lpl_o>(wl, ndisp, u8, nblocks, stream);
}
#endif

}  // namespace sgm
