// fmb_api.cpp -- host side of the C ABI declared in include/fmb.h.
//
// Holds the scene / batch descriptors, cuts the work into items (see
// fmb_internal.h), owns the device workspace (item lists, partial gradients, work
// counters), launches the kernels of fmb_kernels.hip on the caller's stream, captures
// HIP graphs for batches, times the tile variants (autotuner) and records kernel
// timings with HIP events.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "fmb.h"
#include "fmb_internal.h"

namespace fmb {
int num_fwd_variants();
int fwd_variant_rays(int v);
int num_bwd_variants();
int bwd_variant_rt(int v);
int bwd_variant_ray_tile(int v);
int bwd_variant_tiles(int v);
int block_size();
hipError_t launch_fwd(int variant, int flags, int grid, hipStream_t st, const Params &P, const FwdOut &O,
                      const FwdItem *items, int n, const int *order, int *counter);
hipError_t launch_bwd(int variant, int flags, int grid, hipStream_t st, const Params &P, const BwdIn &I,
                      const BwdItem *items, int n, const int *order, int *counter, float *partial, float *bpart);
hipError_t launch_fin(int n_tasks, int n_groups, int max_gc, int max_nval, hipStream_t st, const Params &P,
                      const FinTask *tasks,
                      const FinGroup *groups, const float *partial, const float *bpart, double *stage,
                      double *stage_beta, float *g_means, float *g_prec, float *g_weights, float *g_colors,
                      float *g_betas);
hipError_t launch_fill(int *p, int n, int value, hipStream_t st);
hipError_t launch_loss(int p, const float *depth, const float *alpha, const float *flow, const float *color,
                       const float *depth_t, const float *alpha_t, const float *flow_t, const float *color_t,
                       float w_depth, float w_flow, int flow_norm, int flow_cols, float w_color, float *g_depth,
                       float *g_alpha, float *g_flow, float *g_color, float *block_loss, hipStream_t st);
hipError_t launch_validate(const Params &P, int n_total, int n_scenes, int *flags, hipStream_t st);
hipError_t launch_fwdc(int flags, int n_items, hipStream_t st, const Params &P, const FwdOut &O,
                       const BwdItem *items, const int *order);
hipError_t launch_stat(int n_items, int n_tasks, int max_gc, hipStream_t st, const Params &P, const float *loss,
                       const float *stash, const BwdItem *items, const StatTask *tasks, float *partial,
                       const int64_t *rays_per_scene, float *lbar);
hipError_t launch_statc(int n_items, hipStream_t st, const Params &P, const float *loss, const float *stash,
                        const BwdItem *items, float *partial);
hipError_t launch_bwdc(int flags, int n_items, hipStream_t st, const Params &P, const BwdIn &I,
                       const BwdItem *items, const int *order, float *partial, float *beta_partial, int max_n);
hipError_t occupancy_fwd(int variant, int flags, int *blocks_per_cu);
hipError_t occupancy_bwd(int variant, int flags, int *blocks_per_cu);
hipError_t scratch_base(void **out);
size_t scratch_bytes();
}  // namespace fmb

using namespace fmb;

namespace {
constexpr int kFlagNrm = 1, kFlagFlw = 2, kFlagPer = 4, kFlagCol = 8, kFlagBig = 16;

// Gradient outputs of a backward call.
struct Grads {
    float *means, *prec, *weights, *colors, *betas;
};
}  // namespace

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                                 \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess)                                                                     \
            return fail(e_ == hipErrorOutOfMemory ? FMB_ERR_OOM : FMB_ERR_HIP,                    \
                        std::string(#x) + ": " + hipGetErrorString(e_));                          \
    } while (0)

#define CHECK_ARG(cond, msg)                                                                      \
    do {                                                                                          \
        if (!(cond)) return fail(FMB_ERR_INVALID_ARG, msg);                                       \
    } while (0)

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// View record with its ray tiles: 8 x 8 pixel tiles for images at least 8 pixels wide, else runs
// of 64 consecutive rays (also every view of explicit rays, stored as h x 1).
ViewRec view_rec(int32_t h, int32_t w, int64_t ray_off, int32_t scene)
{
    ViewRec v{h, w, (int32_t)ray_off, scene, 0, 0};
    if (w >= 8) {
        v.tiles_x = (w + 7) / 8;
        v.tiles = v.tiles_x * ((h + 7) / 8);
    } else {
        v.tiles = (int32_t)(((int64_t)h * w + 63) / 64);
    }
    return v;
}

// Size limits (FMB_MAX_* in fmb.h).  Ray indices are 32-bit in the kernels (per-ray output offsets
// are formed in 64 bits); the 2^24 rays of headroom keep every tile or span end (spans are at most
// 2^22 rays) inside int.  Gaussian and view counts keep 16 x index inside int.
constexpr int64_t kMaxRays = FMB_MAX_RAYS;
constexpr int64_t kMaxGaussians = FMB_MAX_GAUSSIANS;
constexpr int64_t kMaxViews = FMB_MAX_VIEWS;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n)
    {
        if (n <= bytes && p) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, n > 0 ? n : 16);
        if (e == hipSuccess) bytes = n > 0 ? n : 16;
        return e;
    }
    template <class T>
    hipError_t upload(const std::vector<T> &v)
    {
        hipError_t e = ensure(v.size() * sizeof(T));
        if (e != hipSuccess || v.empty()) return e;
        return hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------------------------------
// Kernel timing with HIP events
// ---------------------------------------------------------------------------------------

struct Timing {
    std::mutex mu;
    bool enabled = false;
    struct Rec {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double ms[3] = {0, 0, 0};
    long count[3] = {0, 0, 0};

    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void drain()
    {
        for (auto &r : pending) {
            float t = 0.0f;
            if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
                ms[r.kind] += t;
                count[r.kind] += 1;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
};
Timing g_timing;

bool stream_capturing(hipStream_t st)
{
    hipStreamCaptureStatus s = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &s) != hipSuccess) return false;
    return s != hipStreamCaptureStatusNone;
}

struct TimedSpan {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    int kind;
    bool on = false;
    TimedSpan(hipStream_t s, int k) : st(s), kind(k)
    {
        if (!g_timing.enabled || stream_capturing(st)) return;
        std::lock_guard<std::mutex> lk(g_timing.mu);
        a = g_timing.get();
        b = g_timing.get();
        if (a && b && hipEventRecord(a, st) == hipSuccess) on = true;
    }
    void stop()
    {
        if (!on) return;
        on = false;
        if (hipEventRecord(b, st) != hipSuccess) return;
        std::lock_guard<std::mutex> lk(g_timing.mu);
        g_timing.pending.push_back({a, b, kind});
        if (g_timing.pending.size() > 4096) g_timing.drain();
    }
};

// ---------------------------------------------------------------------------------------
// Job: S scenes, their views, work items and workspace
// ---------------------------------------------------------------------------------------

struct Job {
    int S = 0, V = 0;
    int n_total = 0;
    int64_t P = 0;
    std::vector<SceneRec> scenes;
    std::vector<ViewRec> views;
    std::vector<float> eta;
    std::vector<int64_t> ray_off_scene;
    Params prm{};
    bool has_flow = false;
    bool cams_set = false;
    int model = FMB_MODEL_BLEND;
    int device = 0, n_cu = 0;
    DevBuf d_scenes, d_views, d_eta, d_counter;

    // forward work
    int fwd_variant = 1, fwd_built = -1, n_fitems = 0;
    bool launch_fixed = false;  // variants set by the caller or the autotuner
    DevBuf d_fitems, d_forder;
    // backward work
    int bwd_variant = 8, bwd_built = -1, n_bitems = 0, n_tasks = 0, n_groups = 0;
    int fin_max_gc = 1, fin_max_nval = 1;  // largest chunk and first-stage record (finalize grid)
    DevBuf d_bitems, d_border, d_tasks, d_groups, d_partial, d_bpart, d_stage, d_stage_beta;
    size_t partial_floats = 0;

    hipGraphExec_t gexec[2] = {nullptr, nullptr};  // captured forward, backward

    // Captured graphs hold the kernel arguments of their launches: the Params (colours, flow
    // targets), the item lists, their counts and the workspace addresses.  Every change of
    // those (a rebuilt item list, a moved buffer, new Params) drops them, so a stale graph is
    // never replayed: fmb_batch_graph_launch then reports FMB_ERR_STATE.
    void drop_graphs()
    {
        for (auto &g : gexec) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    }
    ~Job() { drop_graphs(); }

    int max_scene_n() const
    {
        int m = 0;
        for (const auto &sc : scenes) m = std::max(m, sc.n);
        return m;
    }

    int init_device()
    {
        HIPCHK(hipGetDevice(&device));
        HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device));
        HIPCHK(d_counter.ensure(4 * sizeof(int)));
        return FMB_OK;
    }

    int upload_descriptors()
    {
        HIPCHK(d_scenes.upload(scenes));
        HIPCHK(d_views.upload(views));
        HIPCHK(d_eta.upload(eta));
        prm.scenes = d_scenes.as<SceneRec>();
        prm.views = d_views.as<ViewRec>();
        prm.eta = d_eta.as<float>();
        // untuned default: 512 rays per forward item, or 256 where that leaves fewer than two
        // items per compute unit (a 64 x 64 view: 16 items instead of 8)
        if (!launch_fixed) fwd_variant = P < 2LL * n_cu * fwd_variant_rays(1) ? 0 : 1;
        return FMB_OK;
    }

    int build_fwd(int variant)
    {
        if (fwd_built == variant) return FMB_OK;
        drop_graphs();  // the forward graph's items (and possibly their buffer) change
        const int R = fwd_variant_rays(variant);  // rays of an item: R / 64 tiles
        std::vector<FwdItem> items;
        std::vector<double> cost;
        for (int k = 0; k < V; ++k) {
            const int64_t hw = (int64_t)views[k].h * views[k].w;
            const int n = scenes[views[k].scene].n;
            for (int t0 = 0; t0 < views[k].tiles; t0 += R / 64) {
                items.push_back({k, t0});
                cost.push_back((double)n * std::min<int64_t>(R, hw - 64 * (int64_t)t0));
            }
        }
        std::vector<int> order(items.size());
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        HIPCHK(d_fitems.upload(items));
        HIPCHK(d_forder.upload(order));
        n_fitems = (int)items.size();
        fwd_built = variant;
        return FMB_OK;
    }

    static void chunking(int n, int block, int &gc, int &slots)
    {
        if (n >= block) {
            gc = block;
            slots = 1;
            return;
        }
        double best = 0.0;
        int bc = 1;
        std::vector<double> util(9, 0.0);
        for (int c = 1; c <= 8; ++c) {
            const int g = (n + c - 1) / c;
            const int sl = block / g;
            util[c] = (double)n * sl / ((double)c * block);
            best = std::max(best, util[c]);
        }
        for (int c = 1; c <= 8; ++c)
            if (util[c] >= 0.92 * best) {
                bc = c;
                break;
            }
        gc = (n + bc - 1) / bc;
        slots = block / gc;
    }

    // Backward items (and, for the compositing model, the forward items too).  The key
    // records the model, the colour record size and the blend backward's variant.
    int bwd_key(int variant, bool colour) const
    {
        return model == FMB_MODEL_COMPOSITE ? (colour ? 3 : 1) : (variant * 2 + (colour ? 1 : 0)) * 2;
    }

    // The backward's work plan, built on the host: items (LPT order), finalize tasks and groups, and
    // the sizes of the partial records and reduction stages.
    struct BwdPlan {
        int key = -1;
        std::vector<BwdItem> items;
        std::vector<int> order;
        std::vector<FinTask> tasks;
        std::vector<FinGroup> groups;
        size_t poff = 0, soff = 0;  // partial floats, first-stage doubles
        int max_gc = 1, max_nval = 1;
    };
    BwdPlan na_plan;  // the plan of the last fmb_backward_noalloc call (host memory only)

    int build_bwd(int variant, bool colour)
    {
        const int key = bwd_key(variant, colour);
        if (bwd_built == key) return FMB_OK;
        drop_graphs();  // items, partial records and the finalize plan change (and may move)
        BwdPlan pl;
        int rc = plan_bwd(variant, colour, pl);
        if (rc) return rc;
        HIPCHK(d_bitems.upload(pl.items));
        HIPCHK(d_border.upload(pl.order));
        HIPCHK(d_tasks.upload(pl.tasks));
        HIPCHK(d_groups.upload(pl.groups));
        HIPCHK(d_stage.ensure(std::max<size_t>(pl.soff, 1) * sizeof(double)));
        HIPCHK(d_stage_beta.ensure(std::max<size_t>(2 * pl.groups.size(), 2) * sizeof(double)));
        n_groups = (int)pl.groups.size();
        fin_max_gc = pl.max_gc;
        fin_max_nval = pl.max_nval;
        HIPCHK(d_partial.ensure(std::max<size_t>(pl.poff, 1) * sizeof(float)));
        HIPCHK(d_bpart.ensure(std::max<size_t>(2 * pl.items.size(), 2) * sizeof(float)));
        partial_floats = pl.poff;
        n_bitems = (int)pl.items.size();
        n_tasks = (int)pl.tasks.size();
        bwd_built = key;
        return FMB_OK;
    }

    int plan_bwd(int variant, bool colour, BwdPlan &pl)
    {
        const int key = bwd_key(variant, colour);
        const bool comp = model == FMB_MODEL_COMPOSITE;
        const int rec = colour ? kPartialColor : kPartial;
        const int RT = bwd_variant_rt(variant);
        const int ray_tile = comp ? 0 : bwd_variant_ray_tile(variant);
        // ray tiles per item of the tiled kernels (the compositing kernels are tiled too)
        const int tiles = comp ? kCompTiles : bwd_variant_tiles(variant);
        const int B = block_size();
        std::vector<int> gcs(S), sls(S), spans(S), min_span(S);
        for (int s = 0; s < S; ++s) {
            if (tiles > 0) {
                // tiled kernels: the whole scene per item, `tiles` ray tiles (ViewRec) per item
                gcs[s] = scenes[s].n;
                sls[s] = 1;
                min_span[s] = spans[s] = tiles;
            } else if (ray_tile > 0) {
                // ray-lane kernel: the whole scene per item, two ray tiles per item to start
                gcs[s] = scenes[s].n;
                sls[s] = 1;
                min_span[s] = ray_tile;
                spans[s] = 2 * ray_tile;
            } else {
                chunking(scenes[s].n, B, gcs[s], sls[s]);
                min_span[s] = RT;
                spans[s] = std::max(RT, ((256 * sls[s] + RT - 1) / RT) * RT);
            }
        }
        // Span of rays per item, chosen per scene only (so a scene is cut the same way alone
        // and inside a batch): about 256 rays per lane, at most 16384 and, where the scene is
        // small, at least 2048 items.
        for (int s = 0; s < S && tiles == 0; ++s) {
            const int chunks = (scenes[s].n + gcs[s] - 1) / gcs[s];
            auto count_items = [&](int span) {
                int64_t c = 0;
                for (int k = scenes[s].view_off; k < scenes[s].view_off + scenes[s].n_views; ++k) {
                    const int hw = views[k].h * views[k].w;
                    c += (int64_t)chunks * ((hw + span - 1) / span);
                }
                return c;
            };
            while (count_items(spans[s]) > 16384 && spans[s] < (1 << 22)) spans[s] *= 2;
            while (count_items(spans[s]) < 2048 && spans[s] > min_span[s]) spans[s] /= 2;
        }
        std::vector<BwdItem> items;
        std::vector<FinTask> tasks;
        std::vector<int> tasks_item_begin, tasks_item_end;
        std::vector<double> cost;
        size_t poff = 0;
        for (int s = 0; s < S; ++s) {
            const int gc = gcs[s], sl = sls[s], span = spans[s];
            const int n = scenes[s].n;
            for (int g0 = 0; g0 < n; g0 += gc) {
                FinTask t{};
                t.scene = s;
                t.g0 = g0;
                t.gc = std::min(gc, n - g0);
                tasks_item_begin.push_back((int)items.size());
                for (int k = scenes[s].view_off; k < scenes[s].view_off + scenes[s].n_views; ++k) {
                    // ray0 and span count rays, or for the tiled kernel ray tiles
                    const int hw = views[k].h * views[k].w;
                    const int lim = tiles > 0 ? views[k].tiles : hw;
                    for (int r0 = 0; r0 < lim; r0 += span) {
                        BwdItem it{};
                        it.view = k;
                        it.ray0 = r0;
                        it.span = span;
                        it.g0 = g0;
                        it.gc = gc;
                        it.slots = sl;
                        if (poff > (size_t)INT32_MAX - (size_t)gc * rec)
                            return fail(FMB_ERR_SHAPE, "backward partial buffer exceeds 2^31 floats");
                        it.poff = (int)poff;
                        it.seq = (int)items.size();
                        poff += (size_t)gc * rec;
                        items.push_back(it);
                        cost.push_back((double)t.gc * (tiles > 0 ? std::min<int64_t>(64LL * span, hw - 64LL * r0)
                                                                 : std::min(span, hw - r0)));
                    }
                }
                tasks_item_end.push_back((int)items.size());
                t.beta = (g0 == 0) ? 1 : 0;
                t.rec = rec;
                tasks.push_back(t);
            }
        }
        // first-stage reduction groups: runs of kGroupItems items inside each chunk
        std::vector<FinGroup> groups;
        size_t soff = 0;
        int scene_first_group = 0, cur_scene = -1;
        for (auto &t : tasks) {
            if (t.scene != cur_scene) {
                cur_scene = t.scene;
                scene_first_group = (int)groups.size();
            }
            const int ib = tasks_item_begin[&t - &tasks[0]], ie = tasks_item_end[&t - &tasks[0]];
            t.group_begin = (int)groups.size();
            // about sqrt(items) items per group so both stages sum similar counts
            const int gsz = std::max(kGroupItems, (int)std::ceil(std::sqrt((double)(ie - ib))));
            for (int a = ib; a < ie; a += gsz) {
                FinGroup g{};
                g.item_begin = a;
                g.item_end = std::min(ie, a + gsz);
                g.poff = items[a].poff;
                g.nval = items[a].gc * rec;
                g.soff = (int)soff;
                soff += (size_t)g.nval;
                groups.push_back(g);
            }
            t.group_end = (int)groups.size();
            t.sgroup_begin = scene_first_group;
        }
        for (auto &t : tasks) {
            int e = 0;
            for (auto &u : tasks)
                if (u.scene == t.scene) e = std::max(e, u.group_end);
            t.sgroup_end = e;
        }
        std::vector<int> order(items.size());
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        pl.key = key;
        pl.max_gc = 1;
        pl.max_nval = 1;
        for (const auto &t : tasks) pl.max_gc = std::max(pl.max_gc, t.gc);
        for (const auto &g : groups) pl.max_nval = std::max(pl.max_nval, g.nval);
        pl.items = std::move(items);
        pl.order = std::move(order);
        pl.tasks = std::move(tasks);
        pl.groups = std::move(groups);
        pl.poff = poff;
        pl.soff = soff;
        return FMB_OK;
    }

    // split statistic: its own items (runs of ray tiles of one view against the whole scene, for
    // both models) and buffers, so captured graphs of the passes stay valid
    int stat_built = -1, n_sitems = 0, n_stasks = 0, stat_max_gc = 0;
    DevBuf d_sitems, d_stasks, d_spartial, d_srays;

    int build_stat()
    {
        if (stat_built == model) return FMB_OK;
        const bool comp = model == FMB_MODEL_COMPOSITE;
        std::vector<BwdItem> items;
        std::vector<StatTask> tasks;
        std::vector<int64_t> rays(S, 0);
        size_t poff = 0;
        stat_max_gc = 0;
        for (int s = 0; s < S; ++s) {
            const int n = scenes[s].n;
            const int gc = n, sl = 1;
            const int span = comp ? kCompTiles : kStatTiles;  // ray tiles (ViewRec) per item
            stat_max_gc = std::max(stat_max_gc, gc);
            for (int k = scenes[s].view_off; k < scenes[s].view_off + scenes[s].n_views; ++k)
                rays[s] += (int64_t)views[k].h * views[k].w;
            for (int g0 = 0; g0 < n; g0 += gc) {
                StatTask t{};
                t.scene = s;
                t.g0 = g0;
                t.gc = std::min(gc, n - g0);
                t.item_begin = (int)items.size();
                for (int k = scenes[s].view_off; k < scenes[s].view_off + scenes[s].n_views; ++k) {
                    // ray0 and span count ray tiles
                    const int lim = views[k].tiles;
                    for (int r0 = 0; r0 < lim; r0 += span) {
                        BwdItem it{};
                        it.view = k;
                        it.ray0 = r0;
                        it.span = span;
                        it.g0 = g0;
                        it.gc = gc;
                        it.slots = sl;
                        if (poff > (size_t)INT32_MAX - (size_t)gc)
                            return fail(FMB_ERR_SHAPE, "split statistic partials exceed 2^31 floats");
                        it.poff = (int)poff;
                        it.seq = (int)items.size();
                        poff += (size_t)gc;
                        items.push_back(it);
                    }
                }
                t.item_end = (int)items.size();
                tasks.push_back(t);
            }
        }
        HIPCHK(d_sitems.upload(items));
        HIPCHK(d_stasks.upload(tasks));
        HIPCHK(d_srays.upload(rays));
        HIPCHK(d_spartial.ensure(std::max<size_t>(poff, 1) * sizeof(float)));
        n_sitems = (int)items.size();
        n_stasks = (int)tasks.size();
        stat_built = model;
        return FMB_OK;
    }

    int split_statistic(const float *loss, const float *stash, float *lbar, hipStream_t st)
    {
        if (!cams_set) return fail(FMB_ERR_STATE, "split statistic before cameras were set");
        CHECK_ARG(loss && stash && lbar, "loss, stash and lbar must be non-NULL");
        CHECK_ARG(aligned(stash, 16), "stash must be 16-byte aligned");
        int rc = build_stat();
        if (rc) return rc;
        if (model == FMB_MODEL_COMPOSITE) {
            HIPCHK(launch_statc(n_sitems, st, prm, loss, stash, d_sitems.as<BwdItem>(),
                                d_spartial.as<float>()));
            HIPCHK(launch_stat(0, n_stasks, stat_max_gc, st, prm, loss, stash, d_sitems.as<BwdItem>(),
                               d_stasks.as<StatTask>(), d_spartial.as<float>(), d_srays.as<int64_t>(), lbar));
        } else {
            HIPCHK(launch_stat(n_sitems, n_stasks, stat_max_gc, st, prm, loss, stash, d_sitems.as<BwdItem>(),
                               d_stasks.as<StatTask>(), d_spartial.as<float>(), d_srays.as<int64_t>(), lbar));
        }
        return FMB_OK;
    }

    std::map<int, int> occ_f, occ_b;  // blocks per CU of the persistent kernels
    int persist_mult[2] = {1, 1};     // persistent grid = mult x occupancy x CUs (fwd, bwd)

    int grid_fwd(int flags, int &grid)
    {
        const int key = fwd_variant * 16 + (flags | kFlagPer);
        auto it = occ_f.find(key);
        if (it == occ_f.end()) {
            int o = 0;
            HIPCHK(occupancy_fwd(fwd_variant, flags | kFlagPer, &o));
            it = occ_f.emplace(key, std::max(1, o)).first;
        }
        grid = std::max(1, std::min(n_fitems, persist_mult[0] * it->second * n_cu));
        return FMB_OK;
    }

    int grid_bwd(int variant, int flags, int &grid)
    {
        const int key = variant * 16 + (flags | kFlagPer);
        auto it = occ_b.find(key);
        if (it == occ_b.end()) {
            int o = 0;
            HIPCHK(occupancy_bwd(variant, flags | kFlagPer, &o));
            it = occ_b.emplace(key, std::max(1, o)).first;
        }
        grid = std::max(1, std::min(n_bitems, persist_mult[1] * it->second * n_cu));
        return FMB_OK;
    }

    // The backward variant a call runs: the tiled variants take no normal cotangent, so such calls
    // run the Gaussian-lane variant 2 instead.
    int bwd_run_variant(const BwdIn &I) const
    {
        return bwd_variant_tiles(bwd_variant) > 0 && I.g_normal ? 2 : bwd_variant;
    }

    static int fwd_flags(const FwdOut &O, bool persist)
    {
        return (O.normal ? kFlagNrm : 0) | (O.flow ? kFlagFlw : 0) | (persist ? kFlagPer : 0) |
               (O.color ? kFlagCol : 0);
    }
    // The blend forward's flags: with a scene of more than a block's count of Gaussians, the kernel
    // form that takes such scenes in pre-culled rounds.
    int blend_fwd_flags(const FwdOut &O, bool persist) const
    {
        return fwd_flags(O, persist) | (max_scene_n() > block_size() ? kFlagBig : 0);
    }
    // The blend backward's flags for variant v: for the tiled variants with a scene of more than a
    // block's count of Gaussians, the kernel form that takes such scenes in pre-culled rounds.
    int blend_bwd_flags(const BwdIn &I, bool persist, int v) const
    {
        return bwd_flags(I, persist) | (bwd_variant_tiles(v) > 0 && max_scene_n() > block_size() ? kFlagBig : 0);
    }
    static int bwd_flags(const BwdIn &I, bool persist)
    {
        return (I.g_normal ? kFlagNrm : 0) | (I.g_flow ? kFlagFlw : 0) | (persist ? kFlagPer : 0) |
               (I.g_color ? kFlagCol : 0);
    }

    int forward(const FwdOut &O, bool persist, hipStream_t st)
    {
        if (!cams_set) return fail(FMB_ERR_STATE, "render before cameras were set");
        CHECK_ARG(O.depth && O.alpha, "depth and alpha outputs are required");
        CHECK_ARG(!O.flow || has_flow, "flow output given but the cameras have no second pose");
        CHECK_ARG(!O.color || prm.colors, "colour output given but no colours were set");
        CHECK_ARG(!O.stash || aligned(O.stash, 16), "stash must be 16-byte aligned");
        if (model == FMB_MODEL_COMPOSITE) {
            // items shared with the backward pass: keep whichever colour record is built
            int rc = (bwd_built == 1 || bwd_built == 3) ? FMB_OK : build_bwd(bwd_variant, prm.colors != nullptr);
            if (rc) return rc;
            TimedSpan ts(st, 0);
            HIPCHK(launch_fwdc(fwd_flags(O, false), n_bitems, st, prm, O, d_bitems.as<BwdItem>(), d_border.as<int>()));
            ts.stop();
            return FMB_OK;
        }
        int rc = build_fwd(fwd_variant);
        if (rc) return rc;
        const int flags = blend_fwd_flags(O, persist);
        int grid = n_fitems;
        if (persist) {
            if ((rc = grid_fwd(flags, grid))) return rc;
            HIPCHK(launch_fill(d_counter.as<int>(), 1, 0, st));
        }
        TimedSpan ts(st, 0);
        HIPCHK(launch_fwd(fwd_variant, flags, grid, st, prm, O, d_fitems.as<FwdItem>(), n_fitems,
                          persist ? d_forder.as<int>() : nullptr, persist ? d_counter.as<int>() : nullptr));
        ts.stop();
        return FMB_OK;
    }

    int backward(const BwdIn &I, const Grads &G, bool persist, hipStream_t st)
    {
        if (!cams_set) return fail(FMB_ERR_STATE, "backward before cameras were set");
        CHECK_ARG(I.depth && I.stash, "depth and stash from the forward pass are required");
        CHECK_ARG(aligned(I.stash, 16), "stash must be 16-byte aligned");
        CHECK_ARG(G.means && G.prec && G.weights && G.betas, "gradient outputs are required");
        CHECK_ARG(!I.g_flow || has_flow, "flow cotangent given but the cameras have no second pose");
        CHECK_ARG(!I.g_color || (prm.colors && I.color), "colour cotangent needs colours and the colour output");
        const int bv = bwd_run_variant(I);
        int rc = build_bwd(bv, I.g_color != nullptr);
        if (rc) return rc;
        if (model == FMB_MODEL_COMPOSITE) {
            TimedSpan tb(st, 1);
            HIPCHK(launch_bwdc(bwd_flags(I, false), n_bitems, st, prm, I, d_bitems.as<BwdItem>(), d_border.as<int>(),
                               d_partial.as<float>(), d_bpart.as<float>(), max_scene_n()));
            tb.stop();
        } else {
            const int flags = blend_bwd_flags(I, persist, bv);
            int grid = n_bitems;
            if (persist) {
                if ((rc = grid_bwd(bv, flags, grid))) return rc;
                HIPCHK(launch_fill(d_counter.as<int>() + 1, 1, 0, st));
            }
            TimedSpan tb(st, 1);
            HIPCHK(launch_bwd(bv, flags, grid, st, prm, I, d_bitems.as<BwdItem>(), n_bitems,
                              persist ? d_border.as<int>() : nullptr, persist ? d_counter.as<int>() + 1 : nullptr,
                              d_partial.as<float>(), d_bpart.as<float>()));
            tb.stop();
        }
        TimedSpan tf(st, 2);
        HIPCHK(launch_fin(n_tasks, n_groups, fin_max_gc, fin_max_nval, st, prm, d_tasks.as<FinTask>(), d_groups.as<FinGroup>(),
                          d_partial.as<float>(), d_bpart.as<float>(), d_stage.as<double>(),
                          d_stage_beta.as<double>(), G.means, G.prec, G.weights, G.colors, G.betas));
        tf.stop();
        return FMB_OK;
    }

    // fmb_backward without a device allocation: the work plan (built on the host and kept there) is
    // copied into the library's fixed scratch array on the call's stream, and the same kernels run
    // over it with the same one-shot launches, so the results equal fmb_backward's bit for bit.
    int backward_noalloc(const BwdIn &I, const Grads &G, hipStream_t st)
    {
        if (!cams_set) return fail(FMB_ERR_STATE, "backward before cameras were set");
        CHECK_ARG(I.depth && I.stash, "depth and stash from the forward pass are required");
        CHECK_ARG(aligned(I.stash, 16), "stash must be 16-byte aligned");
        CHECK_ARG(G.means && G.prec && G.weights && G.betas, "gradient outputs are required");
        CHECK_ARG(!I.g_flow || has_flow, "flow cotangent given but the cameras have no second pose");
        CHECK_ARG(!I.g_color || (prm.colors && I.color), "colour cotangent needs colours and the colour output");
        const bool colour = I.g_color != nullptr;
        const int bv = bwd_run_variant(I);
        if (na_plan.key != bwd_key(bv, colour)) {
            int rc = plan_bwd(bv, colour, na_plan);
            if (rc) return rc;
        }
        const BwdPlan &pl = na_plan;
        // sections of the scratch array, each 256-byte aligned
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t at = off;
            off = (off + bytes + 255) & ~size_t(255);
            return at;
        };
        const size_t o_items = take(pl.items.size() * sizeof(BwdItem));
        const size_t o_tasks = take(pl.tasks.size() * sizeof(FinTask));
        const size_t o_groups = take(pl.groups.size() * sizeof(FinGroup));
        const size_t o_part = take(std::max<size_t>(pl.poff, 1) * sizeof(float));
        const size_t o_bpart = take(std::max<size_t>(2 * pl.items.size(), 2) * sizeof(float));
        const size_t o_stage = take(std::max<size_t>(pl.soff, 1) * sizeof(double));
        const size_t o_sbeta = take(std::max<size_t>(2 * pl.groups.size(), 2) * sizeof(double));
        if (off > scratch_bytes()) {
            std::ostringstream m;
            m << "the scene's backward needs " << off << " bytes of workspace; fmb_backward_noalloc has "
              << scratch_bytes() << " (FMB_NOALLOC_SCRATCH_BYTES): use fmb_backward";
            return fail(FMB_ERR_SHAPE, m.str());
        }
        int dev = -1;
        HIPCHK(hipGetDevice(&dev));
        if (dev != device) return fail(FMB_ERR_STATE, "the scene's device must be the current device");
        void *base = nullptr;
        HIPCHK(scratch_base(&base));
        char *b = static_cast<char *>(base);
        HIPCHK(hipMemcpyAsync(b + o_items, pl.items.data(), pl.items.size() * sizeof(BwdItem), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(b + o_tasks, pl.tasks.data(), pl.tasks.size() * sizeof(FinTask), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(b + o_groups, pl.groups.data(), pl.groups.size() * sizeof(FinGroup),
                              hipMemcpyHostToDevice, st));
        const BwdItem *items = reinterpret_cast<const BwdItem *>(b + o_items);
        float *part = reinterpret_cast<float *>(b + o_part);
        float *bpart = reinterpret_cast<float *>(b + o_bpart);
        const int n_items = (int)pl.items.size();
        if (model == FMB_MODEL_COMPOSITE) {
            TimedSpan tb(st, 1);
            HIPCHK(launch_bwdc(bwd_flags(I, false), n_items, st, prm, I, items, nullptr, part, bpart, max_scene_n()));
            tb.stop();
        } else {
            TimedSpan tb(st, 1);
            HIPCHK(launch_bwd(bv, blend_bwd_flags(I, false, bv), n_items, st, prm, I, items, n_items, nullptr, nullptr,
                              part, bpart));
            tb.stop();
        }
        TimedSpan tf(st, 2);
        HIPCHK(launch_fin((int)pl.tasks.size(), (int)pl.groups.size(), pl.max_gc, pl.max_nval, st, prm,
                          reinterpret_cast<const FinTask *>(b + o_tasks), reinterpret_cast<const FinGroup *>(b + o_groups),
                          part, bpart, reinterpret_cast<double *>(b + o_stage), reinterpret_cast<double *>(b + o_sbeta),
                          G.means, G.prec, G.weights, G.colors, G.betas));
        tf.stop();
        return FMB_OK;
    }
};

int check_params(const float *means, const float *prec, const float *weights, const float *betas)
{
    CHECK_ARG(means && prec && weights && betas, "scene parameter pointers must be non-NULL");
    CHECK_ARG(aligned(means, 4) && aligned(prec, 4) && aligned(weights, 4) && aligned(betas, 4),
              "scene parameters must be 4-byte aligned");
    return FMB_OK;
}

int check_cams(const float *w2c, const float *intr, const int32_t *hw, int v, const float *w2c_b,
               const float *intr_b, int64_t &p)
{
    CHECK_ARG(w2c && intr && hw, "w2c, intr and hw must be non-NULL");
    CHECK_ARG(aligned(w2c, 4) && aligned(intr, 4), "camera arrays must be 4-byte aligned");
    CHECK_ARG((w2c_b == nullptr) == (intr_b == nullptr), "w2c_b and intr_b must both be given or both NULL");
    if (v > kMaxViews) return fail(FMB_ERR_SHAPE, "more than FMB_MAX_VIEWS views");
    p = 0;
    for (int k = 0; k < v; ++k) {
        CHECK_ARG(hw[2 * k] >= 1 && hw[2 * k + 1] >= 1, "image sizes must be >= 1");
        p += (int64_t)hw[2 * k] * hw[2 * k + 1];
        if (p > kMaxRays) return fail(FMB_ERR_SHAPE, "more than FMB_MAX_RAYS rays");
    }
    return FMB_OK;
}

}  // namespace

struct fmb_scene {
    Job job;
    int32_t n = 0;
};
struct fmb_batch {
    Job job;
};

extern "C" {

int fmb_abi_version(void) { return FMB_ABI_VERSION; }

const char *fmb_last_error(void) { return g_err.c_str(); }

int fmb_scene_create(fmb_scene **out, int32_t n, const float *means, const float *prec, const float *weights,
                     const float *betas, float eta)
{
    g_err.clear();
    CHECK_ARG(out, "out must be non-NULL");
    *out = nullptr;
    CHECK_ARG(n >= 1, "n must be >= 1");
    CHECK_ARG(std::isfinite(eta) && eta > 0.0f, "eta must be finite and > 0");
    int rc = check_params(means, prec, weights, betas);
    if (rc) return rc;
    if (n > kMaxGaussians) return fail(FMB_ERR_SHAPE, "more than FMB_MAX_GAUSSIANS Gaussians");
    fmb_scene *s = new (std::nothrow) fmb_scene();
    if (!s) return fail(FMB_ERR_OOM, "host allocation failed");
    s->n = n;
    Job &j = s->job;
    j.S = 1;
    j.n_total = n;
    j.scenes.push_back({n, 0, 0, 0});
    j.eta.push_back(eta);
    j.prm.means = means;
    j.prm.prec = prec;
    j.prm.weights = weights;
    j.prm.betas = betas;
    if ((rc = j.init_device()) || (rc = j.upload_descriptors())) {
        delete s;
        return rc;
    }
    *out = s;
    return FMB_OK;
}

int fmb_scene_rebind(fmb_scene *s, const float *means, const float *prec, const float *weights,
                     const float *betas)
{
    g_err.clear();
    CHECK_ARG(s, "scene must be non-NULL");
    int rc = check_params(means, prec, weights, betas);
    if (rc) return rc;
    s->job.prm.means = means;
    s->job.prm.prec = prec;
    s->job.prm.weights = weights;
    s->job.prm.betas = betas;
    return FMB_OK;
}

int fmb_scene_destroy(fmb_scene *s)
{
    g_err.clear();
    delete s;
    return FMB_OK;
}

int fmb_set_cameras(fmb_scene *s, int32_t v, const float *w2c, const float *intr, const int32_t *hw,
                    const float *w2c_b, const float *intr_b)
{
    g_err.clear();
    CHECK_ARG(s, "scene must be non-NULL");
    CHECK_ARG(v >= 1, "v must be >= 1");
    int64_t p = 0;
    int rc = check_cams(w2c, intr, hw, v, w2c_b, intr_b, p);
    if (rc) return rc;
    Job &j = s->job;
    j.V = v;
    j.P = p;
    j.views.clear();
    int64_t off = 0;
    for (int k = 0; k < v; ++k) {
        j.views.push_back(view_rec(hw[2 * k], hw[2 * k + 1], off, 0));
        off += (int64_t)hw[2 * k] * hw[2 * k + 1];
    }
    j.scenes[0].view_off = 0;
    j.scenes[0].n_views = v;
    j.prm.w2c = w2c;
    j.prm.intr = intr;
    j.prm.w2c_b = w2c_b;
    j.prm.intr_b = intr_b;
    j.prm.w2c_c = j.prm.intr_c = nullptr;
    j.prm.dirs = nullptr;
    j.has_flow = w2c_b != nullptr;
    j.fwd_built = j.bwd_built = j.stat_built = -1;
    j.cams_set = false;
    if ((rc = j.upload_descriptors())) return rc;
    j.cams_set = true;
    return FMB_OK;
}

int fmb_set_rays(fmb_scene *s, int32_t v, const float *w2c, const float *intr, const int32_t *counts,
                 const float *dirs, const float *w2c_b, const float *intr_b)
{
    g_err.clear();
    CHECK_ARG(s, "scene must be non-NULL");
    CHECK_ARG(v >= 1, "v must be >= 1");
    CHECK_ARG(counts && dirs && w2c && intr, "w2c, intr, counts and dirs must be non-NULL");
    CHECK_ARG(aligned(w2c, 4) && aligned(intr, 4) && aligned(dirs, 4), "arrays must be 4-byte aligned");
    CHECK_ARG((w2c_b == nullptr) == (intr_b == nullptr), "w2c_b and intr_b must both be given or both NULL");
    if (v > kMaxViews) return fail(FMB_ERR_SHAPE, "more than FMB_MAX_VIEWS views");
    int64_t p = 0;
    for (int k = 0; k < v; ++k) {
        CHECK_ARG(counts[k] >= 0, "ray counts must be >= 0");
        p += counts[k];
        if (p > kMaxRays) return fail(FMB_ERR_SHAPE, "more than FMB_MAX_RAYS rays");
    }
    CHECK_ARG(p >= 1, "at least one ray is needed");
    Job &j = s->job;
    j.V = v;
    j.P = p;
    j.views.clear();
    int64_t off = 0;
    for (int k = 0; k < v; ++k) {
        j.views.push_back(view_rec(counts[k], 1, off, 0));
        off += counts[k];
    }
    j.scenes[0].view_off = 0;
    j.scenes[0].n_views = v;
    j.prm.w2c = w2c;
    j.prm.intr = intr;
    j.prm.w2c_b = w2c_b;
    j.prm.intr_b = intr_b;
    j.prm.w2c_c = j.prm.intr_c = nullptr;
    j.prm.dirs = dirs;
    j.has_flow = w2c_b != nullptr;
    j.fwd_built = j.bwd_built = j.stat_built = -1;
    j.cams_set = false;
    int rc = j.upload_descriptors();
    if (rc) return rc;
    j.cams_set = true;
    return FMB_OK;
}

int64_t fmb_num_rays(const fmb_scene *s) { return (s && s->job.cams_set) ? s->job.P : 0; }

int fmb_set_flow_pose2(fmb_scene *s, fmb_batch *b, const float *w2c_c, const float *intr_c)
{
    g_err.clear();
    CHECK_ARG((s != nullptr) != (b != nullptr), "exactly one of scene and batch must be given");
    CHECK_ARG((w2c_c == nullptr) == (intr_c == nullptr), "w2c_c and intr_c must both be given or both NULL");
    CHECK_ARG(!w2c_c || (aligned(w2c_c, 4) && aligned(intr_c, 4)), "camera arrays must be 4-byte aligned");
    Job &j = s ? s->job : b->job;
    if (!j.cams_set) return fail(FMB_ERR_STATE, "set the cameras first");
    CHECK_ARG(!w2c_c || j.has_flow, "a second flow target needs the first one (w2c_b, intr_b)");
    if (j.prm.w2c_c != w2c_c || j.prm.intr_c != intr_c) j.drop_graphs();
    j.prm.w2c_c = w2c_c;
    j.prm.intr_c = intr_c;
    return FMB_OK;
}

int fmb_set_model(fmb_scene *s, fmb_batch *b, int32_t model)
{
    g_err.clear();
    CHECK_ARG((s != nullptr) != (b != nullptr), "exactly one of scene and batch must be given");
    CHECK_ARG(model == FMB_MODEL_BLEND || model == FMB_MODEL_COMPOSITE, "model must be FMB_MODEL_BLEND or "
                                                                        "FMB_MODEL_COMPOSITE");
    Job &j = s ? s->job : b->job;
    if (model != j.model) {
        j.model = model;
        j.bwd_built = -1;
        j.drop_graphs();
    }
    return FMB_OK;
}

int fmb_set_colors(fmb_scene *s, fmb_batch *b, const float *colors)
{
    g_err.clear();
    CHECK_ARG((s != nullptr) != (b != nullptr), "exactly one of scene and batch must be given");
    CHECK_ARG(!colors || aligned(colors, 4), "colors must be 4-byte aligned");
    Job &j = s ? s->job : b->job;
    if (j.prm.colors != colors) j.drop_graphs();
    j.prm.colors = colors;
    return FMB_OK;
}

int fmb_render(fmb_scene *s, float *depth, float *alpha, float *normal, float *flow, float *color, float *stash,
               void *stream)
{
    g_err.clear();
    CHECK_ARG(s, "scene must be non-NULL");
    return s->job.forward(FwdOut{depth, alpha, normal, flow, color, stash}, false, (hipStream_t)stream);
}

int fmb_backward(fmb_scene *s, const float *g_depth, const float *g_alpha, const float *g_normal,
                 const float *g_flow, const float *g_color, const float *depth, const float *color,
                 const float *stash, float *g_means, float *g_prec, float *g_weights, float *g_colors,
                 float *g_betas, void *stream)
{
    g_err.clear();
    CHECK_ARG(s, "scene must be non-NULL");
    return s->job.backward(BwdIn{g_depth, g_alpha, g_normal, g_flow, g_color, depth, color, stash},
                           Grads{g_means, g_prec, g_weights, g_colors, g_betas}, false, (hipStream_t)stream);
}

int fmb_backward_noalloc(fmb_scene *s, const float *g_depth, const float *g_alpha, const float *g_normal,
                         const float *g_flow, const float *g_color, const float *depth, const float *color,
                         const float *stash, float *g_means, float *g_prec, float *g_weights, float *g_colors,
                         float *g_betas, void *stream)
{
    g_err.clear();
    CHECK_ARG(s, "scene must be non-NULL");
    return s->job.backward_noalloc(BwdIn{g_depth, g_alpha, g_normal, g_flow, g_color, depth, color, stash},
                                   Grads{g_means, g_prec, g_weights, g_colors, g_betas}, (hipStream_t)stream);
}

int fmb_batch_create(fmb_batch **out, int32_t s, const int32_t *n_host, const int32_t *v_host, const float *means,
                     const float *prec, const float *weights, const float *betas, const float *eta,
                     const float *w2c, const float *intr, const int32_t *hw, const float *w2c_b,
                     const float *intr_b)
{
    g_err.clear();
    CHECK_ARG(out, "out must be non-NULL");
    *out = nullptr;
    CHECK_ARG(s >= 1, "s must be >= 1");
    CHECK_ARG(n_host && v_host && eta, "n_host, v_host and eta must be non-NULL");
    int rc = check_params(means, prec, weights, betas);
    if (rc) return rc;
    int64_t n_total = 0, v_total = 0;
    for (int i = 0; i < s; ++i) {
        CHECK_ARG(n_host[i] >= 1 && v_host[i] >= 1, "every scene needs >= 1 Gaussian and >= 1 view");
        CHECK_ARG(std::isfinite(eta[i]) && eta[i] > 0.0f, "eta must be finite and > 0");
        n_total += n_host[i];
        v_total += v_host[i];
    }
    if (n_total > kMaxGaussians) return fail(FMB_ERR_SHAPE, "more than FMB_MAX_GAUSSIANS Gaussians in the batch");
    if (v_total > kMaxViews) return fail(FMB_ERR_SHAPE, "more than FMB_MAX_VIEWS views in the batch");
    int64_t p = 0;
    if ((rc = check_cams(w2c, intr, hw, (int)v_total, w2c_b, intr_b, p))) return rc;
    fmb_batch *b = new (std::nothrow) fmb_batch();
    if (!b) return fail(FMB_ERR_OOM, "host allocation failed");
    Job &j = b->job;
    j.S = s;
    j.V = (int)v_total;
    j.P = p;
    j.n_total = (int)n_total;
    int goff = 0, voff = 0;
    int64_t roff = 0;
    for (int i = 0; i < s; ++i) {
        j.scenes.push_back({n_host[i], goff, voff, v_host[i]});
        j.eta.push_back(eta[i]);
        j.ray_off_scene.push_back(roff);
        for (int k = 0; k < v_host[i]; ++k) {
            const int kk = voff + k;
            j.views.push_back(view_rec(hw[2 * kk], hw[2 * kk + 1], roff, i));
            roff += (int64_t)hw[2 * kk] * hw[2 * kk + 1];
        }
        goff += n_host[i];
        voff += v_host[i];
    }
    j.ray_off_scene.push_back(roff);
    j.prm.means = means;
    j.prm.prec = prec;
    j.prm.weights = weights;
    j.prm.betas = betas;
    j.prm.w2c = w2c;
    j.prm.intr = intr;
    j.prm.w2c_b = w2c_b;
    j.prm.intr_b = intr_b;
    j.has_flow = w2c_b != nullptr;
    if ((rc = j.init_device()) || (rc = j.upload_descriptors())) {
        delete b;
        return rc;
    }
    j.cams_set = true;
    *out = b;
    return FMB_OK;
}

int fmb_batch_destroy(fmb_batch *b)
{
    g_err.clear();
    delete b;
    return FMB_OK;
}

int64_t fmb_batch_num_rays(const fmb_batch *b) { return b ? b->job.P : 0; }

int64_t fmb_batch_ray_offset(const fmb_batch *b, int32_t i)
{
    if (!b || i < 0 || i > b->job.S) return -1;
    return b->job.ray_off_scene[i];
}

int64_t fmb_batch_gauss_offset(const fmb_batch *b, int32_t i)
{
    if (!b || i < 0 || i > b->job.S) return -1;
    return i == b->job.S ? b->job.n_total : b->job.scenes[i].gauss_off;
}

int fmb_batch_forward(fmb_batch *b, float *depth, float *alpha, float *normal, float *flow, float *color,
                      float *stash, void *stream)
{
    g_err.clear();
    CHECK_ARG(b, "batch must be non-NULL");
    return b->job.forward(FwdOut{depth, alpha, normal, flow, color, stash}, true, (hipStream_t)stream);
}

int fmb_batch_forward_loss(fmb_batch *b, float *depth, float *alpha, float *normal, float *flow, float *color,
                           float *stash, const float *depth_t, const float *alpha_t, float w_depth,
                           float *g_depth, float *g_alpha, void *stream)
{
    g_err.clear();
    CHECK_ARG(b, "batch must be non-NULL");
    CHECK_ARG(depth_t && alpha_t && g_depth && g_alpha, "targets and cotangent outputs must be non-NULL");
    CHECK_ARG(std::isfinite(w_depth), "w_depth must be finite");
    FwdOut O{depth, alpha, normal, flow, color, stash};
    O.depth_t = depth_t;
    O.alpha_t = alpha_t;
    O.g_depth = g_depth;
    O.g_alpha = g_alpha;
    O.w_depth = w_depth;
    O.inv_p = 1.0f / (float)b->job.P;  // as the loss kernel forms it
    return b->job.forward(O, true, (hipStream_t)stream);
}

int fmb_batch_backward(fmb_batch *b, const float *g_depth, const float *g_alpha, const float *g_normal,
                       const float *g_flow, const float *g_color, const float *depth, const float *color,
                       const float *stash, float *g_means, float *g_prec, float *g_weights, float *g_colors,
                       float *g_betas, void *stream)
{
    g_err.clear();
    CHECK_ARG(b, "batch must be non-NULL");
    return b->job.backward(BwdIn{g_depth, g_alpha, g_normal, g_flow, g_color, depth, color, stash},
                           Grads{g_means, g_prec, g_weights, g_colors, g_betas}, true, (hipStream_t)stream);
}

int fmb_batch_capture(fmb_batch *b, float *depth, float *alpha, float *normal, float *flow, float *color,
                      float *stash, const float *g_depth, const float *g_alpha, const float *g_normal,
                      const float *g_flow, const float *g_color, float *g_means, float *g_prec, float *g_weights,
                      float *g_colors, float *g_betas, void *stream)
{
    g_err.clear();
    CHECK_ARG(b, "batch must be non-NULL");
    CHECK_ARG(stash, "capture needs the stash buffer");
    hipStream_t st = (hipStream_t)stream;
    if (st == nullptr) return fail(FMB_ERR_CAPTURE, "graph capture needs a non-default stream");
    if (stream_capturing(st)) return fail(FMB_ERR_CAPTURE, "stream is already capturing");
    Job &j = b->job;
    const FwdOut O{depth, alpha, normal, flow, color, stash};
    const BwdIn I{g_depth, g_alpha, g_normal, g_flow, g_color, depth, color, stash};
    const Grads G{g_means, g_prec, g_weights, g_colors, g_betas};
    // item lists and occupancy are prepared outside the capture (they use synchronous copies)
    int rc = j.build_bwd(j.bwd_run_variant(I), g_color != nullptr);
    if (j.model == FMB_MODEL_BLEND) {
        int gdummy = 0;
        if (!rc) rc = j.build_fwd(j.fwd_variant);
        if (!rc) rc = j.grid_fwd(j.blend_fwd_flags(O, true), gdummy);
        if (!rc) rc = j.grid_bwd(j.bwd_run_variant(I), j.blend_bwd_flags(I, true, j.bwd_run_variant(I)), gdummy);
    }
    if (rc) return rc;
    j.drop_graphs();
    for (int which = 0; which < 2; ++which) {
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int r = which == 0 ? j.forward(O, true, st) : j.backward(I, G, true, st);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (r) {
            if (g) (void)hipGraphDestroy(g);
            j.drop_graphs();
            return r;
        }
        if (e != hipSuccess) {
            j.drop_graphs();
            return fail(FMB_ERR_CAPTURE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        }
        hipError_t ei = hipGraphInstantiate(&j.gexec[which], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            j.drop_graphs();
            return fail(FMB_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        }
    }
    return FMB_OK;
}

int fmb_batch_graph_launch(fmb_batch *b, int32_t which, void *stream)
{
    g_err.clear();
    CHECK_ARG(b, "batch must be non-NULL");
    CHECK_ARG(which >= 0 && which <= 2, "which must be 0 (forward), 1 (backward) or 2 (both)");
    Job &j = b->job;
    if (!j.gexec[0] || !j.gexec[1]) return fail(FMB_ERR_STATE, "no captured graph");
    hipStream_t st = (hipStream_t)stream;
    if (which != 1) {
        TimedSpan t(st, 0);
        HIPCHK(hipGraphLaunch(j.gexec[0], st));
        t.stop();
    }
    if (which != 0) {
        TimedSpan t(st, 1);
        HIPCHK(hipGraphLaunch(j.gexec[1], st));
        t.stop();
    }
    return FMB_OK;
}

int fmb_validate(fmb_scene *s, int32_t *bad_host, void *stream)
{
    g_err.clear();
    CHECK_ARG(s && bad_host, "scene and bad_host must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    Job &j = s->job;
    int rc = FMB_OK;
    HIPCHK(launch_fill(j.d_counter.as<int>() + 2, 1, 0, st));
    HIPCHK(launch_validate(j.prm, j.n_total, j.S, j.d_counter.as<int>() + 2, st));
    int flags = 0;
    HIPCHK(hipMemcpyAsync(&flags, j.d_counter.as<int>() + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *bad_host = flags;
    return rc;
}

int fmb_split_statistic(fmb_scene *s, fmb_batch *b, const float *loss, const float *stash, float *lbar,
                        void *stream)
{
    g_err.clear();
    CHECK_ARG((s != nullptr) != (b != nullptr), "exactly one of scene and batch must be given");
    return (s ? s->job : b->job).split_statistic(loss, stash, lbar, (hipStream_t)stream);
}

int fmb_set_config(fmb_scene *s, fmb_batch *b, int32_t fwd_variant, int32_t bwd_variant, int32_t fwd_grid_mult,
                   int32_t bwd_grid_mult)
{
    g_err.clear();
    CHECK_ARG((s != nullptr) != (b != nullptr), "exactly one of scene and batch must be given");
    CHECK_ARG(fwd_variant >= 0 && fwd_variant < num_fwd_variants(), "forward variant out of range");
    CHECK_ARG(bwd_variant >= 0 && bwd_variant < num_bwd_variants(), "backward variant out of range");
    CHECK_ARG(fwd_grid_mult >= 1 && fwd_grid_mult <= 2 && bwd_grid_mult >= 1 && bwd_grid_mult <= 2,
              "grid multipliers must be 1 or 2");
    Job &j = s ? s->job : b->job;
    j.fwd_variant = fwd_variant;
    j.bwd_variant = bwd_variant;
    j.launch_fixed = true;
    j.persist_mult[0] = fwd_grid_mult;
    j.persist_mult[1] = bwd_grid_mult;
    j.drop_graphs();
    return FMB_OK;
}

int fmb_get_config(const fmb_scene *s, const fmb_batch *b, int32_t *out)
{
    g_err.clear();
    CHECK_ARG((s != nullptr) != (b != nullptr), "exactly one of scene and batch must be given");
    CHECK_ARG(out, "out must be non-NULL");
    const Job &j = s ? s->job : b->job;
    out[0] = j.fwd_variant;
    out[1] = fwd_variant_rays(j.fwd_variant);
    out[2] = j.bwd_variant;
    out[3] = bwd_variant_rt(j.bwd_variant) > 0 ? bwd_variant_rt(j.bwd_variant)
             : bwd_variant_tiles(j.bwd_variant) > 0 ? 64 * bwd_variant_tiles(j.bwd_variant)
                                                    : bwd_variant_ray_tile(j.bwd_variant);
    out[4] = j.persist_mult[0];
    out[5] = j.persist_mult[1];
    // item counts of the lists built for the configuration in use (0 until built)
    const bool comp = j.model == FMB_MODEL_COMPOSITE;
    const bool bwd_cur = comp ? (j.bwd_built == 1 || j.bwd_built == 3)
                              : (j.bwd_built >= 0 && j.bwd_built % 2 == 0 && j.bwd_built / 4 == j.bwd_variant);
    out[6] = comp ? (bwd_cur ? j.n_bitems : 0) : (j.fwd_built == j.fwd_variant ? j.n_fitems : 0);
    out[7] = bwd_cur ? j.n_bitems : 0;
    return FMB_OK;
}

int fmb_timing_enable(int enable)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.enabled = enable != 0;
    return FMB_OK;
}

int fmb_kernel_times(double *out6, int reset)
{
    g_err.clear();
    CHECK_ARG(out6, "out6 must be non-NULL");
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.drain();
    for (int k = 0; k < 3; ++k) {
        out6[k] = g_timing.ms[k];
        out6[3 + k] = (double)g_timing.count[k];
    }
    if (reset) {
        for (int k = 0; k < 3; ++k) {
            g_timing.ms[k] = 0.0;
            g_timing.count[k] = 0;
        }
    }
    return FMB_OK;
}

// ---------------------------------------------------------------------------------------
// Autotuner: time every (forward variant) x (backward variant) on the real shapes.
// ---------------------------------------------------------------------------------------

static std::string tune_key(const Job &j, int fflags, int unused, int cot_mask)
{
    hipDeviceProp_t prop{};
    (void)hipGetDeviceProperties(&prop, j.device);
    std::ostringstream k;
    k << prop.gcnArchName << ":cu" << j.n_cu << ":v5:S" << j.S << ":V" << j.V << ":P" << j.P << ":N" << j.n_total
      << ":out" << fflags << ":cot" << cot_mask;
    (void)unused;
    return k.str();
}

int fmb_autotune(fmb_scene *s, fmb_batch *b, float *depth, float *alpha, float *normal, float *flow, float *color,
                 float *stash, const float *g_depth, const float *g_alpha, const float *g_normal,
                 const float *g_flow, const float *g_color, float *g_means, float *g_prec, float *g_weights,
                 float *g_colors, float *g_betas, const char *cache_path, void *stream)
{
    g_err.clear();
    CHECK_ARG((s != nullptr) != (b != nullptr), "exactly one of scene and batch must be given");
    CHECK_ARG(depth && alpha && stash && g_means && g_prec && g_weights && g_betas, "buffers are required");
    Job &j = s ? s->job : b->job;
    const bool persist = b != nullptr;
    hipStream_t st = (hipStream_t)stream;
    if (!j.cams_set) return fail(FMB_ERR_STATE, "autotune before cameras were set");
    if (j.model == FMB_MODEL_COMPOSITE) return FMB_OK;  // one launch configuration
    j.drop_graphs();  // the variants and grids may change
    const FwdOut O{depth, alpha, normal, flow, color, stash};
    const BwdIn I{g_depth, g_alpha, g_normal, g_flow, g_color, depth, color, stash};
    const Grads G{g_means, g_prec, g_weights, g_colors, g_betas};
    const int cot_mask = (g_depth ? 1 : 0) | (g_alpha ? 2 : 0) | (g_normal ? 4 : 0) | (g_flow ? 8 : 0) |
                         (g_color ? 16 : 0);
    const std::string key = tune_key(j, Job::fwd_flags(O, false), 0, cot_mask);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            int fv = -1, bv = -1, mf = 1, mb = 1;
            if (ls >> k >> fv >> bv >> mf >> mb && k == key && fv >= 0 && fv < num_fwd_variants() && bv >= 0 &&
                bv < num_bwd_variants() && mf >= 1 && mf <= 2 && mb >= 1 && mb <= 2) {
                j.fwd_variant = fv;
                j.bwd_variant = bv;
                j.persist_mult[0] = mf;
                j.persist_mult[1] = mb;
                j.launch_fixed = true;
                return FMB_OK;
            }
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // one untimed launch (it builds the variant's item lists), then kTuneLaunches timed back to back
    constexpr int kTuneLaunches = 10;
    auto time_it = [&](auto &&fn, float &ms) -> int {
        int rc = fn();
        if (rc) return rc;
        HIPCHK(hipEventRecord(e0, st));
        for (int r = 0; r < kTuneLaunches; ++r)
            if ((rc = fn())) return rc;
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        return FMB_OK;
    };
    int rc = FMB_OK;
    float best_f = 1e30f, best_b = 1e30f;
    int bf = j.fwd_variant, bb = j.bwd_variant;
    const int n_mult = persist ? 2 : 1;
    int bmf = 1, bmb = 1;
    for (int v = 0; v < num_fwd_variants() && !rc; ++v)
        for (int m = 1; m <= n_mult && !rc; ++m) {
            j.fwd_variant = v;
            j.persist_mult[0] = m;
            float ms = 0.0f;
            rc = time_it([&]() { return j.forward(O, persist, st); }, ms);
            if (!rc && ms < best_f) {
                best_f = ms;
                bf = v;
                bmf = m;
            }
        }
    j.fwd_variant = bf;
    j.persist_mult[0] = bmf;
    if (!rc) rc = j.forward(O, persist, st);
    for (int v = 0; v < num_bwd_variants() && !rc; ++v)
        for (int m = 1; m <= n_mult && !rc; ++m) {
            j.bwd_variant = v;
            j.persist_mult[1] = m;
            float ms = 0.0f;
            rc = time_it([&]() { return j.backward(I, G, persist, st); }, ms);
            if (!rc && ms < best_b) {
                best_b = ms;
                bb = v;
                bmb = m;
            }
        }
    j.bwd_variant = bb;
    j.persist_mult[1] = bmb;
    j.launch_fixed = true;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (cache_path) {
        std::ofstream outf(cache_path, std::ios::app);
        if (outf) outf << key << " " << bf << " " << bb << " " << bmf << " " << bmb << "\n";
    }
    return FMB_OK;
}

int fmb_loss_grad(int64_t p, const float *depth, const float *alpha, const float *flow, const float *color,
                  const float *depth_t, const float *alpha_t, const float *flow_t, const float *color_t,
                  float w_depth, float w_flow, int32_t flow_norm, int32_t flow_cols, float w_color,
                  float *g_depth, float *g_alpha, float *g_flow, float *g_color, float *block_loss, void *stream)
{
    g_err.clear();
    CHECK_ARG(p >= 1, "p must be >= 1");
    if (p > kMaxRays) return fail(FMB_ERR_SHAPE, "more than FMB_MAX_RAYS rays");
    CHECK_ARG(depth && alpha && depth_t && alpha_t && g_depth && g_alpha, "required pointer is NULL");
    CHECK_ARG((flow == nullptr) == (flow_t == nullptr) && (flow == nullptr) == (g_flow == nullptr),
              "flow, flow_t and g_flow must all be given or all be NULL");
    CHECK_ARG((color == nullptr) == (color_t == nullptr) && (color == nullptr) == (g_color == nullptr),
              "color, color_t and g_color must all be given or all be NULL");
    CHECK_ARG(flow_norm == 1 || flow_norm == 2, "flow_norm must be 1 or 2");
    CHECK_ARG(flow_cols == 2 || flow_cols == 4, "flow_cols must be 2 or 4");
    HIPCHK(launch_loss((int)p, depth, alpha, flow, color, depth_t, alpha_t, flow_t, color_t, w_depth, w_flow,
                       flow_norm, flow_cols, w_color, g_depth, g_alpha, g_flow, g_color, block_loss, (hipStream_t)stream));
    return FMB_OK;
}

}  // extern "C"
