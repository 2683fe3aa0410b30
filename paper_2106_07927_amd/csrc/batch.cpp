// batch.cpp -- many stereo pairs of uneven size and disparity range in one
// hipGraph launch (the batched form of the path).
//
// Plan creation lays every frame's intermediates out in the caller's
// workspace, groups the frames by what the kernels are compiled for
// (disparity range, and for the path pass the lane-layout variant chosen by
// the tuning table), writes one device work list per stage and group, and
// captures the whole sequence into a hipGraph:
//     census (all frames, both images) -> cost (per D) -> paths (per D and
//     variant) -> D^R key fill (all) -> path sum fused with the selection
//     (per D) -> LR check + median (all)
// Frames whose disparity range rules out the fused selection (D % 16 != 0)
// take merge (S_bar in the workspace) and the plain selection instead.
// Every stage is one persistent launch that walks its work list of
// (frame, block) items; the blocks of a frame are exactly those of the
// single-frame call, so each frame's results are bit-identical to it.
// Only frames below kSmallPixels go through these work lists: there a
// stage's blocks of many frames fill the GPU where one frame's would not.
// A larger frame already fills it and runs faster through the single-frame
// kernels, so the graph launches those for it, spread over a number of
// streams forked and joined inside the graph (the tuning table's "chains").
// Running the plan is one hipGraphLaunch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "sgm.h"
#include "sgm_internal.h"

struct sgm_plan {
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t nframes = 0;
};

namespace sgm {
namespace {

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Bytes of one frame's intermediates, in workspace order.
struct FrameLayout {
    size_t census, cost, slices, agg, keys, dl, total;
};

FrameLayout frame_layout(int w, int h, int nd, int npaths, int p2) {
    const size_t n = (size_t)w * h;
    FrameLayout l{};
    l.census = align256(8 * n);
    l.cost = align256(n * nd);
    l.slices = align256(aggregate_work_bytes(w, h, nd, npaths, p2));
    l.agg = fused_select_supported(nd, npaths, p2) ? 0 : align256(2 * n * nd);
    l.keys = align256(4 * n);
    l.dl = align256(2 * n);
    l.total = 2 * l.census + l.cost + l.slices + l.agg + l.keys + l.dl;
    return l;
}

// Streams for the large frames inside the graph when the table names none,
// and the most it may name.  Frames of one stream run one after another;
// frames on different streams overlap, which fills the compute units that
// one frame's path pass leaves idle in its tail.
constexpr int kDefaultChains = 2;
constexpr int kMaxChains = 8;

// Looks up the integer value of "key" in a flat JSON object; `absent` when
// the key is missing.
int table_int(const char* table, const char* key, int absent) {
    if (!table) return absent;
    const char* p = strstr(table, key);
    if (!p) return absent;
    p = strchr(p + strlen(key), ':');
    if (!p) return absent;
    return (int)strtol(p + 1, nullptr, 10);
}

// "WxHxD": lane-layout variant of the path pass for that frame shape.
int tuned_variant(const char* table, int w, int h, int nd) {
    char key[64];
    snprintf(key, sizeof(key), "\"%dx%dx%d\"", w, h, nd);
    return table_int(table, key, -1);
}

// "chains": streams inside the graph for the large frames (1..kMaxChains).
int tuned_chains(const char* table) {
    const int c = table_int(table, "\"chains\"", kDefaultChains);
    return std::max(1, std::min(kMaxChains, c));
}

enum Stage { kCensus, kCost, kPaths, kMerge, kFill, kSelect, kFused, kMedian, kStages };

int stage_blocks(Stage st, const Frame& f) {
    const size_t n = (size_t)f.width * f.height;
    switch (st) {
        case kCensus: return 2 * census_blocks(f.width, f.height);
        case kCost: return cost_blocks_x(f.width) * f.height;
        case kPaths: return path_blocks(f.width, f.height, f.ndisp, f.npaths, f.variant);
        case kMerge: return merge_blocks(n * f.ndisp);
        case kFill: return fill_blocks(n);
        case kSelect: return select_blocks_x(f.width) * f.height;
        case kFused: return fused_blocks_x(f.width, f.ndisp) * f.height;
        case kMedian: return median_blocks(f.width, f.height);
        default: return 0;
    }
}

constexpr long kSmallPixels = 100000;

bool small_frame(const Frame& f) { return (long)f.width * f.height < kSmallPixels; }

// One launch: a stage over a group of frames (indices into the frame table).
struct Launch {
    Stage stage;
    int ndisp, variant;
    std::vector<int> frames;
    size_t frames_off = 0, starts_off = 0;   // workspace offsets of its tables
    size_t items_off = 0;                    // path stage: ordered (frame, block) list
    WorkList wl{};
};

}  // namespace
}  // namespace sgm

using namespace sgm;

namespace {

bool valid_params(const sgm_params* p) {
    if (!p) return false;
    if (!((p->win_w == 5 && p->win_h == 5) || (p->win_w == 9 && p->win_h == 7))) return false;
    if (p->npaths != 4 && p->npaths != 8) return false;
    if (p->p1 < 0 || p->p2 < p->p1) return false;
    if ((int64_t)p->npaths * (255 + (int64_t)p->p2) > 65535) return false;
    return p->median3x3 == 0 || p->median3x3 == 1;
}

bool valid_pair(const sgm_pair& q) {
    if (!q.left || !q.right || !q.disp_out) return false;
    if (q.width < 1 || q.height < 1 || q.width > SGM_MAX_SIDE || q.height > SGM_MAX_SIDE) return false;
    if (q.pitch_bytes < q.width || q.ndisp < 1 || q.ndisp > SGM_MAX_NDISP) return false;
    if ((int64_t)q.width * q.height * q.ndisp > (int64_t)SGM_MAX_VOLUME) return false;
    if ((reinterpret_cast<uintptr_t>(q.disp_out) & 3) != 0) return false;
    if (q.disp_right_out && (reinterpret_cast<uintptr_t>(q.disp_right_out) & 3) != 0) return false;
    return true;
}

// Builds the frame table and the launch list; returns the workspace bytes.
size_t build_layout(const sgm_pair* pairs, int32_t n, const sgm_params* p, const char* tune_table,
                    std::vector<Frame>* frames, std::vector<Launch>* launches, size_t* tables_off) {
    frames->clear();
    launches->clear();
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        const sgm_pair& q = pairs[i];
        Frame f{};
        f.width = q.width;
        f.height = q.height;
        f.ndisp = q.ndisp;
        f.pitch = q.pitch_bytes;
        f.win_w = p->win_w;
        f.win_h = p->win_h;
        f.npaths = p->npaths;
        f.p1 = p->p1;
        f.p2 = p->p2;
        f.lr_tolerance = p->lr_tolerance;
        f.median3x3 = p->median3x3;
        const int tv = tuned_variant(tune_table, q.width, q.height, q.ndisp);
        f.variant = (tv >= 0 && tv < path_variants(q.ndisp)) ? tv
                                                             : default_variant(q.width, q.height, q.ndisp);
        f.left = q.left;
        f.right = q.right;
        f.disp = q.disp_out;
        f.disp_right = q.disp_right_out;
        f.slice_stride = aggregate_slice_elems(q.width, q.height, q.ndisp);
        // workspace offsets are stored in the pointers for now, rebased later
        const FrameLayout l = frame_layout(q.width, q.height, q.ndisp, p->npaths, p->p2);
        f.census_left = reinterpret_cast<uint64_t*>(off);
        f.census_right = reinterpret_cast<uint64_t*>(off + l.census);
        f.cost = reinterpret_cast<uint8_t*>(off + 2 * l.census);
        f.slices = reinterpret_cast<uint8_t*>(off + 2 * l.census + l.cost);
        f.agg = reinterpret_cast<uint16_t*>(off + 2 * l.census + l.cost + l.slices);
        f.right_keys = reinterpret_cast<uint32_t*>(off + 2 * l.census + l.cost + l.slices + l.agg);
        f.disp_left = reinterpret_cast<uint16_t*>(off + 2 * l.census + l.cost + l.slices + l.agg + l.keys);
        off += l.total;
        frames->push_back(f);
    }
    // work-list launch groups over the small frames, in stage order
    std::vector<int> all;
    for (int i = 0; i < n; ++i)
        if (small_frame((*frames)[i])) all.push_back(i);
    if (!all.empty()) {
        std::map<int, std::vector<int>> by_d;
        std::map<std::pair<int, int>, std::vector<int>> by_dv;
        std::vector<int> unfused;
        for (int i : all) {
            by_d[(*frames)[i].ndisp].push_back(i);
            by_dv[{(*frames)[i].ndisp, (*frames)[i].variant}].push_back(i);
            if (!fused_select_supported((*frames)[i].ndisp, p->npaths, p->p2)) unfused.push_back(i);
        }
        launches->push_back({kCensus, 0, 0, all});
        for (auto& kv : by_d) launches->push_back({kCost, kv.first, 0, kv.second});
        for (auto& kv : by_dv) launches->push_back({kPaths, kv.first.first, kv.first.second, kv.second});
        if (!unfused.empty()) launches->push_back({kMerge, 0, 0, unfused});
        launches->push_back({kFill, 0, 0, all});
        for (auto& kv : by_d) {
            const bool fused = fused_select_supported(kv.first, p->npaths, p->p2);
            launches->push_back({fused ? kFused : kSelect, kv.first, 0, kv.second});
        }
        launches->push_back({kMedian, 0, 0, all});
    }
    // tables: one frame table per launch (frames of the group, in order) and
    // its block starts
    *tables_off = off;
    for (Launch& L : *launches) {
        L.frames_off = off;
        off += align256(L.frames.size() * sizeof(Frame));
        L.starts_off = off;
        off += align256((L.frames.size() + 1) * sizeof(int32_t));
        if (L.stage == kPaths) {
            size_t items = 0;
            for (int k : L.frames) items += stage_blocks(kPaths, (*frames)[k]);
            L.items_off = off;
            off += align256(2 * items * sizeof(int32_t));
        }
    }
    return off;
}

}  // namespace

extern "C" {

size_t sgm_batch_workspace_bytes(const sgm_pair* pairs, int32_t n, const sgm_params* params,
                                 const char* tune_table) {
    if (!pairs || n < 1 || !valid_params(params)) return 0;
    for (int i = 0; i < n; ++i)
        if (!valid_pair(pairs[i])) return 0;
    std::vector<Frame> frames;
    std::vector<Launch> launches;
    size_t tables_off;
    return build_layout(pairs, n, params, tune_table, &frames, &launches, &tables_off);
}

int32_t sgm_batch_plan_create(const sgm_pair* pairs, int32_t n, const sgm_params* params,
                              void* workspace, size_t workspace_bytes, const char* tune_table,
                              sgm_plan** plan_out) {
    if (!plan_out) return SGM_ERR_ARG;
    *plan_out = nullptr;
    if (!pairs || n < 1 || !valid_params(params)) return SGM_ERR_ARG;
    for (int i = 0; i < n; ++i)
        if (!valid_pair(pairs[i])) return SGM_ERR_ARG;
    std::vector<Frame> frames;
    std::vector<Launch> launches;
    size_t tables_off;
    const size_t need = build_layout(pairs, n, params, tune_table, &frames, &launches, &tables_off);
    if (!workspace || workspace_bytes < need) return SGM_ERR_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return SGM_ERR_ALIGN;

    // rebase the intermediate buffers onto the workspace
    char* base = static_cast<char*>(workspace);
    for (Frame& f : frames) {
        f.census_left = reinterpret_cast<uint64_t*>(base + reinterpret_cast<uintptr_t>(f.census_left));
        f.census_right = reinterpret_cast<uint64_t*>(base + reinterpret_cast<uintptr_t>(f.census_right));
        f.cost = reinterpret_cast<uint8_t*>(base + reinterpret_cast<uintptr_t>(f.cost));
        f.slices = reinterpret_cast<uint8_t*>(base + reinterpret_cast<uintptr_t>(f.slices));
        f.agg = fused_select_supported(f.ndisp, f.npaths, f.p2)
                    ? nullptr
                    : reinterpret_cast<uint16_t*>(base + reinterpret_cast<uintptr_t>(f.agg));
        f.right_keys = reinterpret_cast<uint32_t*>(base + reinterpret_cast<uintptr_t>(f.right_keys));
        f.disp_left = reinterpret_cast<uint16_t*>(base + reinterpret_cast<uintptr_t>(f.disp_left));
    }
    // work-list tables: copied to the device once, here
    std::vector<char> host(need - tables_off, 0);
    for (Launch& L : launches) {
        Frame* ft = reinterpret_cast<Frame*>(host.data() + (L.frames_off - tables_off));
        int32_t* st = reinterpret_cast<int32_t*>(host.data() + (L.starts_off - tables_off));
        int32_t acc = 0;
        for (size_t k = 0; k < L.frames.size(); ++k) {
            ft[k] = frames[L.frames[k]];
            st[k] = acc;
            acc += stage_blocks(L.stage, ft[k]);
        }
        st[L.frames.size()] = acc;
        L.wl.frames = reinterpret_cast<const Frame*>(base + L.frames_off);
        L.wl.starts = reinterpret_cast<const int32_t*>(base + L.starts_off);
        L.wl.nframes = (int32_t)L.frames.size();
        L.wl.total = acc;
        L.wl.items = nullptr;
        if (L.stage == kPaths) {
            // every block of the group, longest lines first: a block walks
            // W steps on the horizontal paths and H steps on the others
            struct Item { int32_t steps, frame, block; };
            std::vector<Item> items;
            for (size_t k = 0; k < L.frames.size(); ++k) {
                const Frame& f = ft[k];
                const int nh = path_horizontal_blocks(f.width, f.height, f.ndisp, f.variant);
                const int nb = stage_blocks(kPaths, f);
                for (int b = 0; b < nb; ++b)
                    items.push_back({b < nh ? f.width : f.height, (int32_t)k, b});
            }
            std::stable_sort(items.begin(), items.end(),
                             [](const Item& a, const Item& b) { return a.steps > b.steps; });
            int32_t* it = reinterpret_cast<int32_t*>(host.data() + (L.items_off - tables_off));
            for (size_t i = 0; i < items.size(); ++i) {
                it[2 * i] = items[i].frame;
                it[2 * i + 1] = items[i].block;
            }
            L.wl.items = reinterpret_cast<const int32_t*>(base + L.items_off);
        }
    }
    hipError_t e = hipMemcpy(base + tables_off, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return SGM_ERR_HIP;
    }

    sgm_plan* plan = new sgm_plan();
    plan->nframes = n;
    // streams of the graph: the work lists on the first; the large frames,
    // by descending volume, each to the stream with the least volume so far
    std::vector<int> large;
    for (int i = 0; i < n; ++i)
        if (!small_frame(frames[i])) large.push_back(i);
    auto vol = [&](int i) { return (double)frames[i].width * frames[i].height * frames[i].ndisp; };
    std::stable_sort(large.begin(), large.end(), [&](int a, int b) { return vol(a) > vol(b); });
    const int nchains =
        std::max(1, std::min<int>(tuned_chains(tune_table), (int)large.size() + (launches.empty() ? 0 : 1)));
    std::vector<std::vector<int>> chain_frames(nchains);
    std::vector<double> load(nchains, 0.0);
    if (!launches.empty()) {
        for (int i = 0; i < n; ++i)
            if (small_frame(frames[i])) load[0] += vol(i);
    }
    for (int i : large) {
        const int c = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        chain_frames[c].push_back(i);
        load[c] += vol(i);
    }
    std::vector<hipStream_t> side(nchains, nullptr);
    std::vector<hipEvent_t> ev;                     // fork and joins
    auto new_event = [&](hipEvent_t* out) {
        hipError_t r = hipEventCreateWithFlags(out, hipEventDisableTiming);
        if (r == hipSuccess) ev.push_back(*out);
        return r;
    };
    e = hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking);
    for (int c = 0; c < nchains && e == hipSuccess; ++c) e = hipStreamCreateWithFlags(&side[c], hipStreamNonBlocking);
    hipEvent_t fork = nullptr;
    if (e == hipSuccess) e = new_event(&fork);
    if (e == hipSuccess) e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t ce = hipEventRecord(fork, plan->capture_stream);
        for (int c = 0; c < nchains && ce == hipSuccess; ++c) ce = hipStreamWaitEvent(side[c], fork, 0);
        for (size_t k = 0; k < launches.size() && ce == hipSuccess; ++k) {
            const Launch& L = launches[k];
            hipStream_t s = side[0];
            switch (L.stage) {
                case kCensus: ce = launch_census_batch(L.wl, params->win_w, params->win_h, s); break;
                case kCost: ce = launch_cost_batch(L.wl, L.ndisp, s); break;
                case kPaths:
                    ce = launch_paths_batch(L.wl, L.ndisp, params->npaths, params->p2, L.variant, s);
                    break;
                case kMerge: ce = launch_merge_batch(L.wl, params->npaths, params->p2, s); break;
                case kFill: ce = launch_fill_keys_batch(L.wl, s); break;
                case kSelect: ce = launch_select_batch(L.wl, L.ndisp, s); break;
                case kFused: ce = launch_select_fused_batch(L.wl, L.ndisp, params->npaths, params->p2, s); break;
                case kMedian: ce = launch_median_batch(L.wl, s); break;
                default: break;
            }
        }
        for (int c = 0; c < nchains && ce == hipSuccess; ++c) {
            hipStream_t s = side[c];
            for (int i : chain_frames[c]) {
                const Frame& f = frames[i];
                if (ce == hipSuccess) ce = launch_census_pair(f, s);
                if (ce == hipSuccess) ce = launch_cost(f, s);
                if (ce != hipSuccess) break;
                if (fused_select_supported(f.ndisp, f.npaths, f.p2)) {
                    ce = launch_aggregate_select(f, s);
                } else {
                    ce = launch_aggregate(f, s);
                    if (ce == hipSuccess) ce = launch_wta_lrc(f, s);
                }
            }
            hipEvent_t je = nullptr;
            if (ce == hipSuccess) ce = new_event(&je);
            if (ce == hipSuccess) ce = hipEventRecord(je, s);
            if (ce == hipSuccess) ce = hipStreamWaitEvent(plan->capture_stream, je, 0);
        }
        if (e == hipSuccess) e = ce;
        hipError_t ee = hipStreamEndCapture(plan->capture_stream, &plan->graph);
        if (e == hipSuccess) e = ee;
    }
    for (hipEvent_t x : ev) (void)hipEventDestroy(x);
    for (hipStream_t x : side)
        if (x) (void)hipStreamDestroy(x);
    if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        sgm_batch_plan_destroy(plan);
        (void)hipGetLastError();
        return SGM_ERR_HIP;
    }
    *plan_out = plan;
    return SGM_OK;
}

int32_t sgm_batch_run(sgm_plan* plan, void* stream) {
    if (!plan || !plan->exec) return SGM_ERR_ARG;
    const hipError_t e = hipGraphLaunch(plan->exec, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return SGM_ERR_HIP;
    }
    return SGM_OK;
}

int32_t sgm_batch_frames(const sgm_plan* plan) { return plan ? plan->nframes : 0; }

int32_t sgm_aggregate_variants(int32_t ndisp) {
    if (ndisp < 1 || ndisp > SGM_MAX_NDISP) return 0;
    return path_variants(ndisp);
}

void sgm_batch_plan_destroy(sgm_plan* plan) {
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
    delete plan;
}

}  // extern "C"
