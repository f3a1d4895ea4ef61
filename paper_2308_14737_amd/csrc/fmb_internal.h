// fmb_internal.h -- descriptors shared by the host library and the gfx950 kernels.
//
// A render job is always a "batch": S scenes, each with its own Gaussians, blend
// parameters and views.  A single scene is the batch S = 1, so the plain and the
// persistent kernels run the same per-item code.
//
// Work is cut into items:
//   forward item  = (view, first of BLOCK*RPT/64 consecutive ray tiles of that view, see ViewRec)
//   backward item = (view, first ray of a span of rays, Gaussian chunk) plus the
//                   (chunk size, slots) thread mapping and the offset of its partial
//                   gradient record.
#pragma once
#include <stdint.h>

namespace fmb {

// log2(e): the kernels keep log-densities in base 2 so that exp() is one v_exp_f32.
constexpr double kLog2e = 1.4426950408889634073599246810019;
// 0/0 guard of every vector normalisation: |y| is sqrt(y.y + kEpsN).
constexpr float kEpsN = 1e-30f;
// Base-2 log of the smallest blend weight (relative to the ray's running maximum) that the
// kernels evaluate: 2^-150 is below half of FP32's smallest subnormal, so such a weight is
// exactly zero and its terms are skipped.
constexpr float kSkipLog2 = -150.0f;
// Base-2 log of the smallest density whose alpha term D_bar delta the tiled backward evaluates
// where a tile has no weight above zero: a pair below it adds at most 2^-48 |D_bar| to its
// Gaussian's sums, so even 2^21 rays (a 1080p view) change a Gaussian's record by less than
// 2^-27 |D_bar|, far below the terms of the rays that see it.
constexpr float kDensSkipLog2 = -48.0f;

struct ViewRec {       // one per view of the batch
    int32_t h, w;      // image size (explicit rays: h = ray count, w = 1)
    int32_t ray_off;   // global index of the view's first ray
    int32_t scene;     // owning scene
    // Ray tiles of 64 rays, the unit of a wave: 8 x 8 pixel tiles (row-major over tiles) for views
    // at least 8 pixels wide (tiles_x tiles per tile row), else runs of 64 consecutive rays
    // (tiles_x = 0).  `tiles` counts them.
    int32_t tiles_x, tiles;
};

struct SceneRec {
    int32_t n;         // Gaussians
    int32_t gauss_off; // first Gaussian in the concatenated parameter arrays
    int32_t view_off;  // first view
    int32_t n_views;
};

struct FwdItem {       // 8 bytes
    int32_t view;
    int32_t tile0;     // first ray tile (see ViewRec) of the view
};

struct BwdItem {       // 32 bytes
    int32_t view;
    int32_t ray0;      // first local ray of the span
    int32_t span;      // rays in the span (clipped to the view by the kernel)
    int32_t g0;        // first Gaussian (scene-local) of the chunk
    int32_t gc;        // Gaussians in the chunk (<= block size)
    int32_t slots;     // ray slots: thread t works on Gaussian t % gc, rays t / gc mod slots
    int32_t poff;      // offset (floats) of this item's partial record [gc][kPartial]
    int32_t seq;       // canonical item index (beta partials)
};

struct FinTask {       // one per (scene, Gaussian chunk)
    int32_t scene;
    int32_t g0;        // scene-local first Gaussian
    int32_t gc;        // valid Gaussians of the chunk
    int32_t group_begin, group_end;  // first-stage groups of this chunk's items
    int32_t beta;      // 1 if this task also reduces the scene's beta partials
    int32_t sgroup_begin, sgroup_end;  // all groups of the scene (beta partials)
    int32_t rec;       // floats per Gaussian in the partial records (kPartial or kPartialColor)
    int32_t pad[3];
};

// First stage of the deterministic gradient reduction: a group of consecutive
// canonical items of one chunk, summed (FP64, item order) into stage[soff ...].
struct FinGroup {
    int32_t item_begin, item_end;
    int32_t poff;      // partial offset (floats) of item_begin; items of a chunk are contiguous
    int32_t nval;      // gc * kPartial values per item (gc = item chunk size)
    int32_t soff;      // offset (doubles) of the group's sums in the stage buffer
    int32_t pad[3];
};
constexpr int kGroupItems = 32;  // minimum items per first-stage group

// Split statistic (one value per Gaussian and item): the items of a (scene, Gaussian chunk)
// are consecutive, [item_begin, item_end), and their partial sums are added in that order.
struct StatTask {
    int32_t scene;
    int32_t g0, gc;                 // scene-local first Gaussian and chunk size
    int32_t item_begin, item_end;
    int32_t pad[3];
};

constexpr int kPartial = 10;       // per-Gaussian partial: dU (6), sum rho (3), dlog(lambda) (1)
constexpr int kPartialColor = 13;  // ... and dL/d(colour) (3)

// Zero-parameter (alpha-compositing) renderer: ray tiles (ViewRec) per work item, one wave per
// item.
constexpr int kCompTiles = 16;
constexpr int kStatTiles = 16;  // ray tiles (ViewRec) per item of the blend model's split statistic

// Kernel argument blocks (passed by value).
struct Params {
    const float *means, *prec, *weights, *betas;   // concatenated over scenes; betas [S,2]
    const float *eta;                               // device [S]
    const float *w2c, *intr, *w2c_b, *intr_b;       // per global view
    const float *w2c_c, *intr_c;                    // optional second flow target per view, or NULL
    const float *dirs;                              // explicit ray directions [P,3] or NULL (pixel rays)
    const float *colors;                            // unconstrained colours [N,3] or NULL
    const ViewRec *views;
    const SceneRec *scenes;
};

struct FwdOut {
    float *depth, *alpha, *normal, *flow, *color, *stash;
    // Optional, in the per-ray epilogue: the gradient of the loss's depth and alpha terms
    // against targets (what the loss kernel writes for them), over p rays (inv_p = 1/p).
    const float *depth_t = nullptr, *alpha_t = nullptr;
    float *g_depth = nullptr, *g_alpha = nullptr;
    float w_depth = 0.0f, inv_p = 0.0f;
};

struct BwdIn {
    const float *g_depth, *g_alpha, *g_normal, *g_flow, *g_color;
    const float *depth, *color, *stash;
};

}  // namespace fmb
