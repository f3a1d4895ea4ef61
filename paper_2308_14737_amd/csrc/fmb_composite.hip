// fmb_composite.hip -- gfx950 kernels of the zero-parameter Fuzzy Metaballs renderer
// (alpha compositing, Keselman & Hebert, WACV 2024, Sec. 3.3, Eq. 9-10).
//
// Weights: w_i = T_i (1 - exp(-delta_i)), T_i = exp(-sum_j delta_j [t_j < t_i]), blended by
// Eq. (3) for depth, normals and colour; alpha is Eq. (8) as in the two-parameter model.  The
// weights enter Eq. (3) as base-2 logarithms,
//   log2 w_i = -log2(e) F_i + log2(1 - exp(-delta_i)),   F_i = sum_{t_j < t_i} delta_j,
// normalised by their running maximum like the two-parameter weights, so rays far from every
// Gaussian keep finite weights.  The strict inequality is taken literally: intersections at
// equal depth do not attenuate one another.
//
// Layout: one ray per lane, one 8 x 8 pixel tile (ViewRec's ray tiles) per wave, one wave per
// block; an item is a run of consecutive tiles of one view, and the Gaussians are staged through
// LDS in tiles of kCompTG entries (once per item when the scene fits one tile).
//
// Front sums without a sort: F_i only needs the densities in front of t_i, and of those only the
// significant ones (density above 2^sig, comp_sig_log2: the rest total below 2^-24, FP32's
// rounding of T_i).  A lane keeps its ray's significant intersections, with their depths, in
// registers and forms F_i as a sum of exact 0/1 steps over them: per pair the cost is the count of
// significant intersections around the tile (about ten on the benchmark scenes), not N.  Slots are
// filled in Gaussian order at positions uniform over the wave -- a lane for which the slot's
// Gaussian is not significant leaves density 0 there -- so that filling a slot is a register move
// and the step sums run a count uniform over the wave.
//
// Depth windows: a pass fills at most kCompSlots slots.  When more Gaussians are significant for
// the tile, a lane that meets one more than the slots hold records the nearest such depth, and the
// pass covers only the depths in front of it: the lane's window [lo, hi).  The next pass starts at
// hi, with the window's densities (and those at its lower edge, which do not attenuate one another)
// added to the lane's base sum.  Every pair is blended in the window that holds its depth.  Almost
// every tile of the benchmark scenes takes one window; a tile whose rays pass hundreds of Gaussians
// takes several, so the renderer takes any N.
//
// Backward (same layout): with z_i = log w_i and z_bar_i = wt_i (lin_i - kappa) the softmax
// adjoint (wt_i the normalised weight, lin_i the pair's share of the cotangents), delta_j enters
// z_i of every pair behind it, so
//   d_bar(log delta_j) = z_bar_j delta_j / expm1(delta_j) + delta_j (D_bar - B_j),
//   B_j = sum_{t_i > t_j} z_bar_i,   t_bar_j = wt_j tf_bar,
// and the rest is the two-parameter renderer's per-pair adjoint.  B_j is summed over the
// significant intersections (one pass over the slots' Gaussians forms their z_bar), by the same
// step sums; across windows the z_bar of the windows behind come from a first sweep.  The pairs
// left out carry normalised weights below 2^-24 of the ray's largest, and delta_j B_j is itself
// below 2^-24 of z_bar_j where every density of the ray is insignificant.  Each wave sums its pairs'
// terms over its 64 rays for every Gaussian it touches (a fixed butterfly), adds them to the item's
// record in LDS in tile order, and the records go to the deterministic two-stage finalize.
#include "fmb_device.h"

namespace fmb {

constexpr int kCompSlots = 48;  // significant intersections a lane holds per depth window
constexpr int kCompTG = 128;    // Gaussians staged per LDS tile
// Waves per SIMD the kernels are compiled for: the slots take 2 kCompSlots VGPRs (3 kCompSlots
// in the backward).  With 48 slots rather than 32 the dense tiles of the benchmark scenes take one
// window instead of several, which costs less than the lost occupancy.  The forward is held to
// three waves (168 VGPRs, with about 48 values spilled to scratch), which
// is faster than two waves without spills; the backward (and the split statistic) keep two.
constexpr int kFwdcWaves = 3, kBwdcWaves = 2, kStatcWaves = 2;

// log2(1 - exp(-delta)) with log2(delta) = d2.
__device__ __forceinline__ float log2_opacity(float delta, float d2)
{
    const float series = fmaf((float)kLog2e * delta, fmaf(delta, fmaf(delta * delta, -1.0f / 2880.0f, 1.0f / 24.0f), -0.5f), d2);
    const float direct = __builtin_amdgcn_logf(1.0f - exp2_(-(float)kLog2e * delta));
    return delta < 0.0625f ? series : direct;
}

// delta / expm1(delta) = d log(1 - exp(-delta)) / d log(delta).
__device__ __forceinline__ float opacity_slope(float delta)
{
    const float series = fmaf(delta, fmaf(delta, fmaf(delta * delta, -1.0f / 720.0f, 1.0f / 12.0f), -0.5f), 1.0f);
    const float em = exp2_(-(float)kLog2e * delta);
    const float direct = delta * em * rcp_(1.0f - em);
    return delta < 0.0625f ? series : direct;
}

// Depths are kept and compared scaled by 2^100: clamp(b - a, 0, 1) of two scaled depths is 1
// exactly when a < b and 0 when a >= b, for every pair of depths below 2^27 in magnitude whose
// difference is at least 2^-100, i.e. any two distinct depths this renderer meets.
constexpr float kDepthScale = 0x1p100f;

__device__ __forceinline__ float before(float a, float b) { return __builtin_amdgcn_fmed3f(b - a, 0.0f, 1.0f); }

// Base-2 log of the smallest significant density of a scene of n Gaussians: the densities left
// out of a front sum total less than n 2^sig <= 2^-36 (and 2^sig <= 2^-30).
__device__ __forceinline__ float comp_sig_log2(int n)
{
    const int lg = n > 1 ? 32 - __clz(n - 1) : 0;  // ceil(log2 n)
    return fminf(-30.0f, -36.0f - (float)lg);
}

// A ray whose largest base-2 log weight is at least this takes only its significant pairs: the
// others weigh less than n 2^sig <= 2^-36 together, below 2^-24 of its sum of weights.
constexpr float kCompHitLog2 = -12.0f;

// Base-2 log of the smallest normalised weight (and density) whose pair terms are evaluated: the
// weights of Eq. (9) fall off only as fast as the densities, so pairs far from a ray keep weights far
// above FP32's zero, but all pairs below 2^skip together move a ray's sums by less than
// n 2^skip <= 2^-26 of their value (and 2^skip <= 2^-40).
__device__ __forceinline__ float comp_skip_log2(int n)
{
    const int lg = n > 1 ? 32 - __clz(n - 1) : 0;  // ceil(log2 n)
    return fminf(-40.0f, -26.0f - (float)lg);
}

// A lane's slots: scaled depth and density of the significant intersection of the slot's
// Gaussian (density 0 where that Gaussian is not significant for the lane, or not in its window).
// They are register vectors (slots 0..31 in the first, 32..47 in the second), read at
// compile-time positions and written at the wave-uniform fill position by one indirect register
// move; slot k holds the window's k-th Gaussian in staging order, and the slots from ns on hold
// zeros.
typedef float CompV32 __attribute__((ext_vector_type(32)));
typedef float CompV16 __attribute__((ext_vector_type(16)));
static_assert(kCompSlots == 48, "the slot vectors hold 32 + 16 slots");
struct CompList {
    CompV32 t0, d0;
    CompV16 t1, d1;
};
// a value per slot (the backward's z_bar of the slots' pairs)
struct CompZ {
    CompV32 z0;
    CompV16 z1;
};

__device__ __forceinline__ float slot_t(const CompList &L, int k) { return k < 32 ? L.t0[k] : L.t1[k - 32]; }
__device__ __forceinline__ float slot_d(const CompList &L, int k) { return k < 32 ? L.d0[k] : L.d1[k - 32]; }
__device__ __forceinline__ float slot_z(const CompZ &z, int k) { return k < 32 ? z.z0[k] : z.z1[k - 32]; }

__device__ __forceinline__ void slot_set_d(CompList &L, int k, float d)
{
    if (k < 32)
        L.d0[k] = d;
    else
        L.d1[k - 32] = d;
}

__device__ __forceinline__ void slot_set(CompList &L, int k, float t, float d)
{
    if (k < 32) {
        L.t0[k] = t;
        L.d0[k] = d;
    } else {
        L.t1[k - 32] = t;
        L.d1[k - 32] = d;
    }
}

__device__ __forceinline__ void slot_set_z(CompZ &z, int k, float v)
{
    if (k < 32)
        z.z0[k] = v;
    else
        z.z1[k - 32] = v;
}

// A lane's depth window (scaled depths): pairs with lo <= t < hi are taken in the current pass;
// base sums the significant densities in front of lo, tie those at lo.
struct CompWin {
    float lo, hi, base, tie;
};

__device__ __forceinline__ void comp_clear(CompList &L)
{
    L.t0 = (CompV32)(0.0f);
    L.d0 = (CompV32)(0.0f);
    L.t1 = (CompV16)(0.0f);
    L.d1 = (CompV16)(0.0f);
}

// Step sums over the slots in use, eight slots at a time (template recursion, so that every slot
// index is a compile-time register index); ns is uniform, so the early exits are scalar branches,
// and the unused slots of a group add zeros.  The even and the odd slots go to two sums (two
// independent chains).
constexpr int kSlotGroup = 8;
template <int K>
struct SlotSums {
    // sum of the densities of the slots in front of ts
    __device__ static __forceinline__ void front(const CompList &L, int ns, float ts, float &f, float &g)
    {
        if (K >= ns) return;
#pragma unroll
        for (int k = K; k < K + kSlotGroup; k += 2) {
            f = fmaf(before(slot_t(L, k), ts), slot_d(L, k), f);
            g = fmaf(before(slot_t(L, k + 1), ts), slot_d(L, k + 1), g);
        }
        SlotSums<K + kSlotGroup>::front(L, ns, ts, f, g);
    }
    // sum of z over the slots behind ts
    __device__ static __forceinline__ void behind(const CompList &L, const CompZ &z, int ns, float ts, float &b,
                                                  float &c)
    {
        if (K >= ns) return;
#pragma unroll
        for (int k = K; k < K + kSlotGroup; k += 2) {
            b = fmaf(before(ts, slot_t(L, k)), slot_z(z, k), b);
            c = fmaf(before(ts, slot_t(L, k + 1)), slot_z(z, k + 1), c);
        }
        SlotSums<K + kSlotGroup>::behind(L, z, ns, ts, b, c);
    }
};
template <>
struct SlotSums<kCompSlots> {
    __device__ static __forceinline__ void front(const CompList &, int, float, float &, float &) {}
    __device__ static __forceinline__ void behind(const CompList &, const CompZ &, int, float, float &, float &) {}
};
static_assert(kCompSlots % kSlotGroup == 0 && kSlotGroup % 2 == 0, "whole slot groups, of pairs");

// F at scaled depth ts inside window w: base, the densities at lo (if ts > lo), and the slots
// in front of ts.
__device__ __forceinline__ float comp_front(const CompList &L, int ns, const CompWin &w, float ts)
{
    float f = ts > w.lo ? w.base + w.tie : w.base, g = 0.0f;
    SlotSums<0>::front(L, ns, ts, f, g);
    return f + g;
}

// Sum of z over the slots behind ts.
__device__ __forceinline__ float comp_behind(const CompList &L, const CompZ &z, int ns, float ts)
{
    float b = 0.0f, c = 0.0f;
    SlotSums<0>::behind(L, z, ns, ts, b, c);
    return b + c;
}

// z_bar of the slots' pairs without a normal or colour cotangent, from the slots alone: the pair's
// weight 2^(lw - M2) / S with lw = -log2(e) F + log2(1 - exp(-delta)) at the slot's depth and
// density, times (tf_bar t - kappa); 0 where the slot is empty for the lane.  A loop over the slots
// in use (each read and written by an indirect register move at the uniform index k) rather than
// one unrolled over every slot: the unrolled form, a front sum per slot, was 70 KB of the adjoint
// kernel's 118 KB of code (same speed on the benchmark scenes).
__device__ __forceinline__ float slot_zf(float f, float dl, float ts, float M2, float invS, float tfb, float kap);

__device__ __forceinline__ float slot_z_plain(const CompList &L, int ns, const CompWin &w, float M2, float invS,
                                              float tfb, float kap, float dl, float ts)
{
    if (!(dl > 0.0f)) return 0.0f;
    return slot_zf(comp_front(L, ns, w, ts), dl, ts, M2, invS, tfb, kap);
}

__device__ __forceinline__ void slots_z_plain(const CompList &L, CompZ &zs, int ns, const CompWin &w, float M2,
                                              float invS, float tfb, float kap)
{
    // (one loop per register vector, so that each writes a single vector in place)
#pragma unroll 1
    for (int k = 0; k < min(ns, 32); ++k)
        zs.z0[k] = slot_z_plain(L, ns, w, M2, invS, tfb, kap, L.d0[k], L.t0[k]);
#pragma unroll 1
    for (int k = 32; k < ns; ++k)
        zs.z1[k - 32] = slot_z_plain(L, ns, w, M2, invS, tfb, kap, L.d1[k - 32], L.t1[k - 32]);
}

// z_bar of a slot's pair from its front sum F, density and depth (0 where the slot is empty).
__device__ __forceinline__ float slot_zf(float f, float dl, float ts, float M2, float invS, float tfb, float kap)
{
    if (!(dl > 0.0f)) return 0.0f;
    const float lw = fmaf(-(float)kLog2e, f, log2_opacity(dl, __builtin_amdgcn_logf(dl)));
    return exp2_(lw - M2) * invS * fmaf(tfb, ts * (1.0f / kDepthScale), -kap);
}

// The same z_bar for a tile of one window whose pairs are all slots' (no normal or colour
// cotangent): first every slot's front sum F into zs, then every slot's z_bar into its density
// register.  The adjoint of such a tile then takes a pair's front sum from zs and the sums of z_bar
// behind it from the density registers: the slots' densities are needed only for the front sums,
// and a second front sum per pair is saved.  The values are those slots_z_plain and comp_front
// form, bit for bit.
__device__ __forceinline__ void slots_fz_plain(CompList &L, CompZ &zs, int ns, const CompWin &w, float M2,
                                               float invS, float tfb, float kap)
{
#pragma unroll 1
    for (int k = 0; k < min(ns, 32); ++k) zs.z0[k] = comp_front(L, ns, w, L.t0[k]);
#pragma unroll 1
    for (int k = 32; k < ns; ++k) zs.z1[k - 32] = comp_front(L, ns, w, L.t1[k - 32]);
#pragma unroll 1
    for (int k = 0; k < min(ns, 32); ++k) L.d0[k] = slot_zf(zs.z0[k], L.d0[k], L.t0[k], M2, invS, tfb, kap);
#pragma unroll 1
    for (int k = 32; k < ns; ++k)
        L.d1[k - 32] = slot_zf(zs.z1[k - 32], L.d1[k - 32], L.t1[k - 32], M2, invS, tfb, kap);
}

// Entries of Gaussians [gb, gb + cnt) of the scene into LDS, EW float4 each: the entry, the terms
// of the m estimate (make_entry_est) and, with EW = 6, the colour.
constexpr int kCompEst = 4, kCompCol = 5;  // float4 offsets within an LDS entry
template <int EW>
__device__ __forceinline__ void comp_stage(const Params &P, const SceneRec &sr, int gb, int cnt, const double o[3],
                                           float4 *__restrict__ ents)
{
    __syncthreads();  // the previous tile is consumed
    for (int q = threadIdx.x; q < cnt; q += 64) {
        const int gi = sr.gauss_off + gb + q;
        make_entry_est(P.means + 3 * gi, P.prec + 6 * gi, P.weights[gi], o, &ents[EW * q]);
        if (EW == 6) ents[EW * q + kCompCol] = colour_entry(P.colors + 3 * gi);
    }
    __syncthreads();
}

// Upper bound of the pair's log2 density from the one-FMA lower bound of m (pair_m_low), with the
// peak already formed (pair_geo_peak returned vc).
__device__ __forceinline__ float comp_d2_hi(const Ent &g, const float4 &est, float vc, float t, float hm)
{
    return fmaf(hm, pair_m_low(est, vc, t), g.l2l);
}

template <int EW>
__device__ __forceinline__ Ent comp_ent(const float4 *__restrict__ ents, int i)
{
    return ent_from(ents[EW * i], ents[EW * i + 1], ents[EW * i + 2], ents[EW * i + 3]);
}

// Cone of a wave's rays: unit centre direction (uniform over the wave) and the cosine of the
// largest angle between it and a ray of the wave.
struct TileCone {
    float c0, c1, c2, ca;
};

__device__ __forceinline__ float wave_sum_f(float x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ TileCone comp_cone(float v0, float v1, float v2, bool valid)
{
    float c0 = wave_sum_f(valid ? v0 : 0.0f), c1 = wave_sum_f(valid ? v1 : 0.0f), c2 = wave_sum_f(valid ? v2 : 0.0f);
    c0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c0)));
    c1 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c1)));
    c2 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c2)));
    const float inv = rsq_(fmaf(c0, c0, fmaf(c1, c1, fmaf(c2, c2, kEpsN))));
    TileCone tc;
    tc.c0 = c0 * inv;
    tc.c1 = c1 * inv;
    tc.c2 = c2 * inv;
    float ca = valid ? fmaf(tc.c0, v0, fmaf(tc.c1, v1, tc.c2 * v2)) : 1.0f;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) ca = fminf(ca, __shfl_xor(ca, off, 64));
    // margins for the rounding of the directions and of the cone
    tc.ca = fminf(ca, 1.0f) - 1e-5f;
    return tc;
}

// Staged Gaussians [0, cnt) whose log2 density can exceed thr on some ray of the cone (the bound of
// tile_bounds from the cone's centre ray and radius), as two 64-bit masks (lane j tests Gaussians
// j and 64 + j).
__device__ __forceinline__ void comp_cull(const float4 *__restrict__ ents, int ew, int cnt, const TileCone &tc,
                                          float thr, unsigned long long mask[2])
{
    static_assert(kCompTG == 128, "two 64-bit masks per staged tile");
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int i = 64 * c + (int)threadIdx.x;
        bool keep = false;
        if (i < cnt) {
            const Ent g = ent_from(ents[ew * i], ents[ew * i + 1], ents[ew * i + 2], ents[ew * i + 3]);
            // the largest distance of a unit ray direction of the cone from its centre: |v - c|^2 = 2 - 2 cos
            const float rho = sqrtf(fmaxf(0.0f, 2.0f - 2.0f * tc.ca)) * (1.0f + 1e-4f) + 1e-6f;
            float d2_hi, z_hi;
            tile_bounds(g, ents[ew * i + kCompEst], make_float4(tc.c0, tc.c1, tc.c2, rho), (float)(-0.5 * kLog2e),
                        0.0f, 0.0f, d2_hi, z_hi);
            keep = !(d2_hi <= thr);  // (a NaN bound keeps the Gaussian)
        }
        mask[c] = wave_ballot(keep);
    }
}

// The slots of window w: every Gaussian significant for some lane of the wave, with a depth behind
// lo for that lane, takes the next slot; the densities at lo go to w.tie (and each such pair, whose
// front sum is w.base, to on_tie(g, q, density, staged index)); a lane that meets one more than the
// slots hold lowers w.hi to its depth, and its slots at or behind w.hi are cleared (they belong to a
// later window).  Returns the slot count (uniform); slot_g (if given) receives the slots'
// scene-local Gaussian indices.
template <int EW, class OnTie>
__device__ __forceinline__ int comp_collect(const Params &P, const SceneRec &sr, const double o[3],
                                            float4 *__restrict__ ents, bool resident, float v0, float v1,
                                            float v2, float hm, float sig2, const TileCone &tc, CompWin &w,
                                            CompList &L, int *__restrict__ slot_g, OnTie on_tie)
{
    int ns = 0;
    bool t_inf = false;  // a slot of this lane holds an infinite scaled depth
    comp_clear(L);
    for (int gb = 0; gb < sr.n; gb += kCompTG) {
        const int cnt = min(kCompTG, sr.n - gb);
        if (!resident) comp_stage<EW>(P, sr, gb, cnt, o, ents);
        // only the Gaussians that can be significant on some ray of the wave
        unsigned long long mask[2];
        comp_cull(ents, EW, cnt, tc, sig2, mask);
        // the pair's share of the window: tie, slot or (a full list) the end of the window
        auto take = [&](const Ent &g, const Geo &q, int i) {
            const bool sig = q.d2 > sig2;
            if (!wave_any(sig)) return;
            const float ts = q.t * kDepthScale;
            const float dl = exp2_(q.d2);
            if (sig && ts == w.lo) {
                w.tie += dl;
                on_tie(g, q, dl, i);
            }
            const bool cand = sig && ts > w.lo;
            if (!wave_any(cand)) return;
            if (ns < kCompSlots) {
                slot_set(L, ns, ts, cand ? dl : 0.0f);
                t_inf = t_inf || (cand && ts == INFINITY);
                if (threadIdx.x == 0) slot_g[ns] = gb + i;
                ns = __builtin_amdgcn_readfirstlane(ns + 1);
            } else if (cand) {
                w.hi = fminf(w.hi, ts);
            }
        };
        // two candidates a step, their geometry computed together (two independent chains)
        for (int c = 0; c < 2; ++c) {
            unsigned long long mk = mask[c];
            while (mk) {
                const int ia = 64 * c + __builtin_ctzll(mk);
                mk &= mk - 1;
                const bool two = mk != 0;
                const int ib = two ? 64 * c + __builtin_ctzll(mk) : ia;
                if (two) mk &= mk - 1;
                const Ent ga = comp_ent<EW>(ents, ia), gb2 = comp_ent<EW>(ents, ib);
                Geo qa, qb;
                const float vca = pair_geo_peak(ga, v0, v1, v2, qa), vcb = pair_geo_peak(gb2, v0, v1, v2, qb);
                // the residual only where the density bound allows a significant pair
                if (wave_any(comp_d2_hi(ga, ents[EW * ia + kCompEst], vca, qa.t, hm) > sig2)) {
                    pair_geo_resid(ga, v0, v1, v2, hm, 0.0f, 0.0f, qa);
                    take(ga, qa, ia);
                }
                if (two && wave_any(comp_d2_hi(gb2, ents[EW * ib + kCompEst], vcb, qb.t, hm) > sig2)) {
                    pair_geo_resid(gb2, v0, v1, v2, hm, 0.0f, 0.0f, qb);
                    take(gb2, qb, ib);
                }
            }
        }
    }
    // (where no lane's window was cut, only a slot at an infinite scaled depth can be at or behind hi)
    if (wave_any(w.hi != INFINITY || t_inf)) {
#pragma unroll
        for (int k = 0; k < kCompSlots; ++k) slot_set_d(L, k, slot_t(L, k) >= w.hi ? 0.0f : slot_d(L, k));
    }
    return ns;
}

// Moves window w past hi (or marks the lane done); returns true while the lane has depths left.
__device__ __forceinline__ bool comp_next(CompWin &w, const CompList &L, int ns)
{
    if (w.hi == INFINITY) {
        w.lo = INFINITY;
        return false;
    }
    float s = w.tie;
#pragma unroll
    for (int k = 0; k < kCompSlots; ++k) s += slot_d(L, k);
    w.base += s;
    w.lo = w.hi;
    w.hi = INFINITY;
    w.tie = 0.0f;
    return true;
}

// ------------------------------------------------------------------------------------
// Forward
// ------------------------------------------------------------------------------------

template <int F>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kFwdcWaves))) void fwdc_kernel(Params P, FwdOut O, const BwdItem *__restrict__ items,
                                                                                                      const int *__restrict__ order)
{
    constexpr bool NORMALS = (F & kNrm) != 0, COLOR = (F & kCol) != 0;
    constexpr int EW = COLOR ? 6 : 5;
    __shared__ float4 ents[kCompTG * EW];
    __shared__ int slot_g[kCompSlots];
    const int lane = threadIdx.x;
    const BwdItem item = ld_uniform(items + (order ? ld_uniform(order + blockIdx.x) : (int)blockIdx.x));
    const ViewRec vr = ld_uniform(P.views + item.view);
    const SceneRec sr = ld_uniform(P.scenes + vr.scene);
    const CamRec cam = cam_of(P, item.view);
    const float *e = cam.e, *kk = cam.k;
    double o[3];
    cam_centre(e, o);
    const float o0 = (float)o[0], o1 = (float)o[1], o2 = (float)o[2];
    const float hm = (float)(-0.5 * kLog2e);
    const float sig2 = comp_sig_log2(sr.n), skip2 = comp_skip_log2(sr.n);
    const bool resident = sr.n <= kCompTG;
    if (resident) comp_stage<EW>(P, sr, 0, sr.n, o, ents);
    const int nt = min(item.span, vr.tiles - item.ray0);  // ray0: the item's first tile

    for (int tt = 0; tt < nt; ++tt) {
        int row, col;
        const int loc = tile_local(vr, item.ray0 + tt, lane, row, col);
        const bool valid = loc >= 0;
        float v0, v1, v2;
        tile_ray_dir(P, vr, e, kk, valid ? loc : 0, valid ? row : 0, valid ? col : 0, v0, v1, v2);
        float at = 0.0f, dt = 0.0f;  // loss targets, loaded ahead of the epilogue
        if (O.g_depth && valid) {
            at = O.alpha_t[vr.ray_off + loc];
            dt = O.depth_t[vr.ray_off + loc];
        }
        const TileCone tc = comp_cone(v0, v1, v2, valid);
        float M, S, T, N0, N1, N2, C0, C1, C2, D;
        auto reset = [&]() {
            M = -INFINITY;
            S = T = N0 = N1 = N2 = C0 = C1 = C2 = D = 0.0f;
        };
        reset();
        CompWin w{valid ? -INFINITY : INFINITY, INFINITY, 0.0f, 0.0f};
        CompList L;
        // blends pair (g, q) of this lane at front sum fs; ci: the staged index of its colour
        auto blend = [&](const Ent &g, Geo &q, float fs, int ci) {
            const float delta = exp2_(q.d2);
            D += delta;
            const float lw = fmaf(-(float)kLog2e, fs, log2_opacity(delta, q.d2));
            if (lw > M) {  // new running maximum: rescale the sums
                const float sc = exp2_(M - lw);
                S *= sc;
                T *= sc;
                N0 *= sc;
                N1 *= sc;
                N2 *= sc;
                C0 *= sc;
                C1 *= sc;
                C2 *= sc;
                M = lw;
            }
            const float ew = exp2_(lw - M);
            S += ew;
            T = fmaf(ew, q.t, T);
            if (NORMALS) {
                pair_refine(q);
                const PairNormal pn = pair_normal(g, q, 0.0f, 0.0f, 0.0f);
                N0 = fmaf(ew, pn.n0, N0);
                N1 = fmaf(ew, pn.n1, N1);
                N2 = fmaf(ew, pn.n2, N2);
            }
            if (COLOR) {
                const float4 cc = ents[EW * ci + kCompCol];
                C0 = fmaf(ew, cc.x, C0);
                C1 = fmaf(ew, cc.y, C1);
                C2 = fmaf(ew, cc.z, C2);
            }
        };
        const auto no_tie = [](const Ent &, const Geo &, float, int) {};
        int ns = comp_collect<EW>(P, sr, o, ents, resident, v0, v1, v2, hm, sig2, tc, w, L, slot_g, no_tie);

        // A tile of one window whose rays all weigh at least 2^kCompHitLog2 somewhere blends only the
        // significant pairs (the slots' Gaussians), each ray its own.
        bool done = false;
        // (a ray without a significant intersection cannot qualify)
        float own = 0.0f;
#pragma unroll
        for (int k = 0; k < kCompSlots; ++k) own += slot_d(L, k);
        if (resident && ns > 0 && !wave_any(w.hi != INFINITY) && wave_all(!valid || own > 0.0f)) {
            for (int s = 0; s < ns; s += 2) {  // two slots a step (two independent chains)
                const bool two = s + 1 < ns;
                const int ia = slot_g[s], ib = two ? slot_g[s + 1] : ia;
                const Ent ga = comp_ent<EW>(ents, ia), gb = comp_ent<EW>(ents, ib);
                Geo qa, qb;
                pair_geo_coarse(ga, v0, v1, v2, hm, 0.0f, 0.0f, qa);
                pair_geo_coarse(gb, v0, v1, v2, hm, 0.0f, 0.0f, qb);
                if (valid && qa.d2 > sig2) blend(ga, qa, comp_front(L, ns, w, qa.t * kDepthScale), ia);
                if (two && valid && qb.d2 > sig2) blend(gb, qb, comp_front(L, ns, w, qb.t * kDepthScale), ib);
            }
            done = wave_all(!valid || M >= kCompHitLog2);
            if (!done) reset();
        }
        // Otherwise every pair of every window (a tile that sees background or several windows).
        while (!done) {
            for (int gb = 0; gb < sr.n; gb += kCompTG) {
                const int cnt = min(kCompTG, sr.n - gb);
                if (!resident) comp_stage<EW>(P, sr, gb, cnt, o, ents);
                for (int i = 0; i < cnt; i += 2) {  // two Gaussians a step (two independent chains)
                    const bool two = i + 1 < cnt;
                    const int ib = two ? i + 1 : i;
                    const Ent ga = comp_ent<EW>(ents, i), gb = comp_ent<EW>(ents, ib);
                    Geo qa, qb;
                    const float vca = pair_geo_peak(ga, v0, v1, v2, qa), vcb = pair_geo_peak(gb, v0, v1, v2, qb);
                    // a pair of this window whose weight (at most its density) is not below
                    // 2^skip2 of the running maximum (nor is its density below 2^skip2, as M <= 0);
                    // the density bound rules most pairs out before the residual
                    const float tsa = qa.t * kDepthScale, tsb = qb.t * kDepthScale;
                    const bool ina = tsa >= w.lo && tsa < w.hi, inb = two && tsb >= w.lo && tsb < w.hi;
                    if (wave_any(ina && comp_d2_hi(ga, ents[EW * i + kCompEst], vca, qa.t, hm) - M >= skip2)) {
                        pair_geo_resid(ga, v0, v1, v2, hm, 0.0f, 0.0f, qa);
                        const bool la = ina && qa.d2 - M >= skip2;
                        if (wave_any(la) && la) blend(ga, qa, comp_front(L, ns, w, tsa), i);
                    }
                    if (wave_any(inb && comp_d2_hi(gb, ents[EW * ib + kCompEst], vcb, qb.t, hm) - M >= skip2)) {
                        pair_geo_resid(gb, v0, v1, v2, hm, 0.0f, 0.0f, qb);
                        const bool lb = inb && qb.d2 - M >= skip2;
                        if (wave_any(lb) && lb) blend(gb, qb, comp_front(L, ns, w, tsb), ib);
                    }
                }
            }
            const bool more = comp_next(w, L, ns);
            if (!wave_any(more)) break;
            ns = comp_collect<EW>(P, sr, o, ents, resident, v0, v1, v2, hm, sig2, tc, w, L, slot_g, no_tie);
        }
        if (valid)
            write_ray<F>(P, O, item.view, vr.ray_off + loc, e, kk, o0, o1, o2, v0, v1, v2, M, S, T, N0, N1, N2, C0,
                         C1, C2, D, at, dt);
    }
}

// ------------------------------------------------------------------------------------
// Backward
// ------------------------------------------------------------------------------------

template <int F>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kBwdcWaves))) void bwdc_kernel(Params P, BwdIn I, const BwdItem *__restrict__ items,
                                                  const int *__restrict__ order, float *__restrict__ partial,
                                                  float *__restrict__ beta_partial)
{
    constexpr bool NORMALS = (F & kNrm) != 0, COLOR = (F & kCol) != 0;
    // without a normal cotangent the pairs take the offset form of the adjoint
    // (pair_adjoint_offset), which needs neither the refined peak nor r
    constexpr bool PLAIN = !NORMALS;
    constexpr int EW = COLOR ? 6 : 5;
    constexpr int REC = COLOR ? kPartialColor : kPartial;   // partial record per Gaussian
    // the sums per Gaussian: (H, Bv, L) of the offset form or the general record, then colour
    constexpr int LREC = (PLAIN ? kOffsetAcc : kPartial) + (COLOR ? 3 : 0);
    static_assert(LREC <= 16, "one 16-value wave sum per pair");
    __shared__ float4 ents[kCompTG * EW];
    // the slots' entries, for scenes beyond one LDS tile (dynamic: launched without it when every
    // scene is resident, so that more blocks share a compute unit)
    extern __shared__ float4 sents[];
    __shared__ float rec[kCompTG * LREC];      // the item's sums of the staged Gaussians
    __shared__ int slot_g[kCompSlots];
    __shared__ int touched[kCompTG];
    const int lane = threadIdx.x;
    const BwdItem item = ld_uniform(items + (order ? ld_uniform(order + blockIdx.x) : (int)blockIdx.x));
    const ViewRec vr = ld_uniform(P.views + item.view);
    const SceneRec sr = ld_uniform(P.scenes + vr.scene);
    const CamRec cam = cam_of(P, item.view);
    const float *e = cam.e, *kk = cam.k;
    double o[3];
    cam_centre(e, o);
    const float o0 = (float)o[0], o1 = (float)o[1], o2 = (float)o[2];
    const float hm = (float)(-0.5 * kLog2e);
    const float sig2 = comp_sig_log2(sr.n), skip2 = comp_skip_log2(sr.n);
    const int n = sr.n;
    const bool resident = n <= kCompTG;
    float *__restrict__ prec_out = partial + item.poff;
    if (resident) {
        comp_stage<EW>(P, sr, 0, n, o, ents);
        for (int q = lane; q < n * LREC; q += 64) rec[q] = 0.0f;
    } else {
        // the record is summed in place over the item's tiles and windows, one staged tile at a time
        for (int q = lane; q < n * REC; q += 64) prec_out[q] = 0.0f;
    }
    __syncthreads();
    const int nt = min(item.span, vr.tiles - item.ray0);

    for (int tt = 0; tt < nt; ++tt) {
        int row, col;
        const int loc = tile_local(vr, item.ray0 + tt, lane, row, col);
        const bool valid = loc >= 0;
        float4 pr[4];
        ray_prologue<F>(P, I, item.view, vr, e, kk, o0, o1, o2, valid ? loc : 0, valid, 0.0f, 0.0f, pr);
        const float v0 = pr[0].x, v1 = pr[0].y, v2 = pr[0].z, M2 = pr[0].w;
        const float invS = pr[1].x, tfb = pr[1].y, nb0 = pr[1].z, nb1 = pr[1].w;
        const float nb2 = pr[2].x, kap = pr[2].y, Db = pr[2].z;
        const float cb0 = pr[3].x, cb1 = pr[3].y, cb2 = pr[3].z;
        // a normalised weight 2^(lw - M2) / S is below 2^skip2 where lw < M2 + log2 S + skip2,
        // and lw is at most the log2 density
        const float wskip = valid ? M2 - __builtin_amdgcn_logf(invS) + skip2 : INFINITY;
        // the least cutoff of the wave's rays (pairs below a ray's cutoff are not taken)
        float lim_min = valid ? fminf(skip2, wskip) : INFINITY;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lim_min = fminf(lim_min, __shfl_xor(lim_min, off, 64));
        const CompWin w0{valid ? -INFINITY : INFINITY, INFINITY, 0.0f, 0.0f};
        CompWin w = w0;
        CompList L;
        CompZ zs;
        const TileCone tc = comp_cone(v0, v1, v2, valid);

        // z_bar of the slots' own pairs (the lanes' significant intersections of the window)
        auto slots_z = [&](int ns) {
            zs.z0 = (CompV32)(0.0f);
            zs.z1 = (CompV16)(0.0f);
            if (PLAIN && !COLOR) {
                // z_bar = wt (tf_bar t - kappa) needs only the slot's depth and density (a colour
                // cotangent adds C_bar . c of the slot's Gaussian: the general form below)
                slots_z_plain(L, zs, ns, w, M2, invS, tfb, kap);
                return;
            }
            if (!resident) {
                __syncthreads();
                if (lane < ns) {
                    const int gi = sr.gauss_off + slot_g[lane];
                    make_entry_est(P.means + 3 * gi, P.prec + 6 * gi, P.weights[gi], o, &sents[EW * lane]);
                    if (COLOR) sents[EW * lane + kCompCol] = colour_entry(P.colors + 3 * gi);
                }
                __syncthreads();
            }
            const float4 *src = resident ? ents : sents;
            // z_bar of the lane's pair (g, q) when the slot holds it: significant and in the window
            auto own_z = [&](const Ent &g, Geo &q, int gs, int k) {
                const float ts = q.t * kDepthScale;
                const bool own = q.d2 > sig2 && ts > w.lo && ts < w.hi;
                float z = 0.0f;
                if (wave_any(own) && own) {
                    const float lw = fmaf(-(float)kLog2e, comp_front(L, ns, w, ts), log2_opacity(exp2_(q.d2), q.d2));
                    const float wt = exp2_(lw - M2) * invS;
                    float lin = tfb * q.t;
                    if (NORMALS) {
                        pair_refine(q);
                        lin += pair_normal(g, q, nb0, nb1, nb2).nN;
                    }
                    if (COLOR) {
                        const float4 cc = src[EW * gs + kCompCol];
                        lin = fmaf(cb0, cc.x, fmaf(cb1, cc.y, fmaf(cb2, cc.z, lin)));
                    }
                    z = wt * (lin - kap);
                }
                slot_set_z(zs, k, z);
            };
            for (int s = 0; s < ns; s += 2) {  // two slots a step (two independent chains)
                const bool two = s + 1 < ns;
                const int ga_i = resident ? slot_g[s] : s;
                const int gb_i = two ? (resident ? slot_g[s + 1] : s + 1) : ga_i;
                const Ent ga = comp_ent<EW>(src, ga_i), gb = comp_ent<EW>(src, gb_i);
                Geo qa, qb;
                pair_geo_coarse(ga, v0, v1, v2, hm, 0.0f, 0.0f, qa);
                pair_geo_coarse(gb, v0, v1, v2, hm, 0.0f, 0.0f, qb);
                own_z(ga, qa, ga_i, s);
                if (two) own_z(gb, qb, gb_i, s + 1);
            }
        };

        // z_bar of the significant pairs at a window's lower edge (the depth where the previous
        // window stopped): they take no slot, and their front sum is the window's base
        float ztie = 0.0f;
        auto on_tie = [&](const Ent &g, const Geo &q0, float dl, int i) {
            Geo q = q0;
            const float lw = fmaf(-(float)kLog2e, w.base, log2_opacity(dl, q.d2));
            const float wt = exp2_(lw - M2) * invS;
            float lin = tfb * q.t;
            if (NORMALS) {
                pair_refine(q);
                lin += pair_normal(g, q, nb0, nb1, nb2).nN;
            }
            if (COLOR) {
                const float4 cc = ents[EW * i + kCompCol];
                lin = fmaf(cb0, cc.x, fmaf(cb1, cc.y, fmaf(cb2, cc.z, lin)));
            }
            ztie = fmaf(wt, lin - kap, ztie);
        };
        // sum of z_bar over the window's significant pairs: the slots' and the lower edge's
        auto window_z = [&](int ns) {
            float s = ztie;
#pragma unroll
            for (int k = 0; k < kCompSlots; ++k) s += slot_z(zs, k);
            return s;
        };

        // First sweep, for tiles that take several windows: the sum of z_bar over all significant
        // intersections of each ray, so that a window knows the z_bar of the windows behind it.
        int ns = comp_collect<EW>(P, sr, o, ents, resident, v0, v1, v2, hm, sig2, tc, w, L, slot_g, on_tie);
        float zall = 0.0f;
        if (wave_any(w.hi != INFINITY)) {
            bool more = true;
            for (;;) {
                slots_z(ns);
                zall += window_z(ns);
                more = comp_next(w, L, ns);
                if (!wave_any(more)) break;
                ztie = 0.0f;
                ns = comp_collect<EW>(P, sr, o, ents, resident, v0, v1, v2, hm, sig2, tc, w, L, slot_g, on_tie);
            }
            w = w0;
            ztie = 0.0f;
            ns = comp_collect<EW>(P, sr, o, ents, resident, v0, v1, v2, hm, sig2, tc, w, L, slot_g, on_tie);
        }

        // A tile of one window whose rays all weigh at least 2^kCompHitLog2 somewhere (the forward's
        // test, on its stashed maximum) takes only the slots' Gaussians, each ray its own pairs.
        const bool hit_tile = resident && ns > 0 && !wave_any(w.hi != INFINITY) && wave_all(!valid || M2 >= kCompHitLog2);

        // Adjoint terms of this lane's pair (g, q) of Gaussian staged at index i (live: the lane
        // has the pair), summed over the wave and added to the Gaussian's sums rec[LREC r ...].
        // With from_slots (a tile of slots_fz_plain) the pair's front sum is fs and z_bar of the
        // slots is in the density registers.
        auto pair_terms = [&](const Ent &g, Geo &q, float ts, bool live, int i, int r, float zafter, bool from_slots,
                              float fs) {
            PairAcc acc;
            OffsetAcc oacc;
            float aC0 = 0.0f, aC1 = 0.0f, aC2 = 0.0f;
            if (live) {
                const float delta = exp2_(q.d2);
                const float lw = fmaf(-(float)kLog2e, from_slots ? fs : comp_front(L, ns, w, ts), log2_opacity(delta, q.d2));
                const float wt = exp2_(lw - M2) * invS;
                PairNormal pn{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                if (NORMALS) {
                    pair_refine(q);
                    pn = pair_normal(g, q, nb0, nb1, nb2);
                }
                float lin = fmaf(tfb, q.t, pn.nN);
                if (COLOR) {
                    const float4 cc = ents[EW * i + kCompCol];
                    lin = fmaf(cb0, cc.x, fmaf(cb1, cc.y, fmaf(cb2, cc.z, lin)));
                    aC0 = wt * cb0;
                    aC1 = wt * cb1;
                    aC2 = wt * cb2;
                }
                const float zb = wt * (lin - kap);
                const float bsum = zafter + (from_slots ? comp_behind(L, CompZ{L.d0, L.d1}, ns, ts)
                                                        : comp_behind(L, zs, ns, ts));
                const float db = fmaf(zb, opacity_slope(delta), delta * (Db - bsum));
                const float tb = wt * tfb;
                if (PLAIN)
                    pair_adjoint_offset(q, v0, v1, v2, tb, db, oacc);
                else
                    pair_adjoint<NORMALS>(g, q, v0, v1, v2, wt, pn, nb0, nb1, nb2, tb, db, acc);
            }
            float x[16];
            if (PLAIN) {
                offset_acc_store(oacc, x);
            } else {
                x[0] = acc.u0; x[1] = acc.u1; x[2] = acc.u2; x[3] = acc.u3; x[4] = acc.u4; x[5] = acc.u5;
                x[6] = acc.p0; x[7] = acc.p1; x[8] = acc.p2; x[9] = acc.l;
            }
            constexpr int B0 = PLAIN ? kOffsetAcc : kPartial;
#pragma unroll
            for (int c = B0; c < 16; ++c) x[c] = 0.0f;
            if (COLOR) {
                x[B0] = aC0;
                x[B0 + 1] = aC1;
                x[B0 + 2] = aC2;
            }
            const float tot = wave_sum16(x, lane);
            const int idx = wave16_index(lane);
            if ((lane & 3) == 0 && idx < LREC) rec[LREC * r + idx] += tot;
        };

        float zthrough = 0.0f;
        for (;;) {
            // (a tile of one window whose pairs are all slots': the slots keep F and z_bar)
            const bool fz = PLAIN && !COLOR && hit_tile;
            if (fz) {
                slots_fz_plain(L, zs, ns, w, M2, invS, tfb, kap);
            } else {
                slots_z(ns);
                zthrough += window_z(ns);
            }
            // z_bar of the significant intersections behind this window
            const float zafter = w.hi == INFINITY ? 0.0f : zall - zthrough;

            if (hit_tile) {
                for (int s = 0; s < ns; ++s) {
                    const int ia = slot_g[s];
                    const Ent ga = comp_ent<EW>(ents, ia);
                    Geo qa;
                    pair_geo_coarse(ga, v0, v1, v2, hm, 0.0f, 0.0f, qa);
                    // the pair of slot s is the slot's own (its front sum is F of the slot)
                    const float fa = fz ? slot_z(zs, s) : 0.0f;
                    pair_terms(ga, qa, qa.t * kDepthScale, valid && qa.d2 > sig2, ia, ia, zafter, fz, fa);
                }
            } else {
                for (int gb = 0; gb < n; gb += kCompTG) {
                    const int cnt = min(kCompTG, n - gb);
                    if (!resident) {
                        comp_stage<EW>(P, sr, gb, cnt, o, ents);
                        for (int q = lane; q < cnt * LREC; q += 64) rec[q] = 0.0f;
                        for (int q = lane; q < cnt; q += 64) touched[q] = 0;
                        __syncthreads();
                    }
                    // only the Gaussians whose density can reach some lane's cutoff on the tile
                    // (the tile bound of comp_cull), two a step (two independent chains)
                    unsigned long long fm[2];
                    comp_cull(ents, EW, cnt, tc, lim_min, fm);
                    for (int c = 0; c < 2; ++c) {
                      unsigned long long mk = fm[c];
                      while (mk) {
                        const int i = 64 * c + __builtin_ctzll(mk);
                        mk &= mk - 1;
                        const bool two = mk != 0;
                        const int ib = two ? 64 * c + __builtin_ctzll(mk) : i;
                        if (two) mk &= mk - 1;
                        const Ent ga = comp_ent<EW>(ents, i), gb = comp_ent<EW>(ents, ib);
                        Geo qa, qb;
                        const float vca = pair_geo_peak(ga, v0, v1, v2, qa), vcb = pair_geo_peak(gb, v0, v1, v2, qb);
                        // a pair of this window with a normalised weight or a density not below
                        // 2^skip2 (the density bound rules most pairs out before the residual)
                        const float tsa = qa.t * kDepthScale, tsb = qb.t * kDepthScale;
                        const float lim = fminf(skip2, wskip);
                        const bool ina = tsa >= w.lo && tsa < w.hi, inb = two && tsb >= w.lo && tsb < w.hi;
                        if (wave_any(ina && comp_d2_hi(ga, ents[EW * i + kCompEst], vca, qa.t, hm) >= lim)) {
                            pair_geo_resid(ga, v0, v1, v2, hm, 0.0f, 0.0f, qa);
                            const bool la = ina && qa.d2 >= lim;
                            if (wave_any(la)) {
                                pair_terms(ga, qa, tsa, la, i, i, zafter, false, 0.0f);
                                if (!resident && lane == 0) touched[i] = 1;
                            }
                        }
                        if (wave_any(inb && comp_d2_hi(gb, ents[EW * ib + kCompEst], vcb, qb.t, hm) >= lim)) {
                            pair_geo_resid(gb, v0, v1, v2, hm, 0.0f, 0.0f, qb);
                            const bool lb = inb && qb.d2 >= lim;
                            if (wave_any(lb)) {
                                pair_terms(gb, qb, tsb, lb, ib, ib, zafter, false, 0.0f);
                                if (!resident && lane == 0) touched[ib] = 1;
                            }
                        }
                      }
                    }
                    if (!resident) {
                        // add the tile's sums of this window to the item's record
                        __syncthreads();
                        for (int qq = lane; qq < cnt; qq += 64) {
                            if (!touched[qq]) continue;
                            const int gg = sr.gauss_off + gb + qq;
                            float r[kPartialColor];
                            if (PLAIN)
                                write_partial_offset(r, rec + LREC * qq, REC, P.prec + 6 * gg, P.means + 3 * gg, o);
                            else
                                write_partial(r, rec + LREC * qq, REC, P.means + 3 * gg, o);
                            float *dst = prec_out + REC * (gb + qq);
                            for (int c = 0; c < REC; ++c) dst[c] += r[c];
                        }
                    }
                }
            }
            const bool more = comp_next(w, L, ns);
            if (!wave_any(more)) break;
            ztie = 0.0f;
            ns = comp_collect<EW>(P, sr, o, ents, resident, v0, v1, v2, hm, sig2, tc, w, L, slot_g, on_tie);
        }
    }

    if (resident) {
        __syncthreads();
        for (int q = lane; q < n; q += 64) {
            const int gg = sr.gauss_off + q;
            if (PLAIN)
                write_partial_offset(prec_out + REC * q, rec + LREC * q, REC, P.prec + 6 * gg, P.means + 3 * gg, o);
            else
                write_partial(prec_out + REC * q, rec + LREC * q, REC, P.means + 3 * gg, o);
        }
    }
    if (lane < 2) beta_partial[2 * item.seq + lane] = 0.0f;  // the model has no blend parameters
}

// ------------------------------------------------------------------------------------
// Split statistic (Sec. 8) with the compositing weights: lbar_i = (1/M) sum_j L_j w_ji, summed
// here per item and Gaussian; the running maximum and 1/S come from the forward's stash.
// ------------------------------------------------------------------------------------

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kStatcWaves))) void statc_kernel(Params P, const float *__restrict__ loss,
                                                   const float *__restrict__ stash,
                                                   const BwdItem *__restrict__ items, float *__restrict__ partial)
{
    constexpr int EW = 5;
    const int *order = nullptr;
    __shared__ float4 ents[kCompTG * EW];
    __shared__ float rec[kCompTG];
    __shared__ int slot_g[kCompSlots];
    const int lane = threadIdx.x;
    const BwdItem item = ld_uniform(items + (order ? ld_uniform(order + blockIdx.x) : (int)blockIdx.x));
    const ViewRec vr = ld_uniform(P.views + item.view);
    const SceneRec sr = ld_uniform(P.scenes + vr.scene);
    const CamRec cam = cam_of(P, item.view);
    const float *e = cam.e, *kk = cam.k;
    double o[3];
    cam_centre(e, o);
    const float hm = (float)(-0.5 * kLog2e);
    const float sig2 = comp_sig_log2(sr.n), skip2 = comp_skip_log2(sr.n);
    const int n = sr.n;
    const bool resident = n <= kCompTG;
    float *__restrict__ out = partial + item.poff;
    if (resident) {
        comp_stage<EW>(P, sr, 0, n, o, ents);
        for (int q = lane; q < n; q += 64) rec[q] = 0.0f;
    } else {
        for (int q = lane; q < n; q += 64) out[q] = 0.0f;
    }
    __syncthreads();
    const int nt = min(item.span, vr.tiles - item.ray0);
    for (int tt = 0; tt < nt; ++tt) {
        int row, col;
        const int loc = tile_local(vr, item.ray0 + tt, lane, row, col);
        const bool valid = loc >= 0;
        float v0, v1, v2;
        tile_ray_dir(P, vr, e, kk, valid ? loc : 0, valid ? row : 0, valid ? col : 0, v0, v1, v2);
        float M2 = INFINITY, invS = 0.0f, lr = 0.0f;
        if (valid) {
            const size_t r = (size_t)vr.ray_off + loc;
            const float4 s0 = reinterpret_cast<const float4 *>(stash)[2 * r];
            M2 = s0.x;
            invS = s0.y;
            lr = loss[r];
        }
        const float wskip = valid ? M2 - __builtin_amdgcn_logf(invS) + skip2 : INFINITY;
        CompWin w{valid ? -INFINITY : INFINITY, INFINITY, 0.0f, 0.0f};
        CompList L;
        const TileCone tc = comp_cone(v0, v1, v2, valid);
        const auto no_tie = [](const Ent &, const Geo &, float, int) {};
        for (bool first = true;; first = false) {
            const int ns = comp_collect<EW>(P, sr, o, ents, resident, v0, v1, v2, hm, sig2, tc, w, L, slot_g, no_tie);
            // as in the forward: a tile of one window whose rays all weigh at least 2^kCompHitLog2
            // somewhere takes only the slots' Gaussians
            if (first && resident && ns > 0 && !wave_any(w.hi != INFINITY) && wave_all(!valid || M2 >= kCompHitLog2)) {
                for (int s = 0; s < ns; ++s) {
                    const int gi = slot_g[s];
                    const Ent g = comp_ent<EW>(ents, gi);
                    Geo q;
                    pair_geo_coarse(g, v0, v1, v2, hm, 0.0f, 0.0f, q);
                    const float ts = q.t * kDepthScale;
                    float x = 0.0f;
                    if (valid && q.d2 > sig2) {
                        const float lw = fmaf(-(float)kLog2e, comp_front(L, ns, w, ts), log2_opacity(exp2_(q.d2), q.d2));
                        x = lr * (exp2_(lw - M2) * invS);
                    }
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
                    if (lane == 0) rec[gi] += x;
                }
                break;
            }
            for (int gb = 0; gb < n; gb += kCompTG) {
                const int cnt = min(kCompTG, n - gb);
                if (!resident) {
                    comp_stage<EW>(P, sr, gb, cnt, o, ents);
                    for (int q = lane; q < cnt; q += 64) rec[q] = 0.0f;
                    __syncthreads();
                }
                for (int i = 0; i < cnt; ++i) {
                    const Ent g = comp_ent<EW>(ents, i);
                    Geo q;
                    pair_geo_coarse(g, v0, v1, v2, hm, 0.0f, 0.0f, q);
                    const float ts = q.t * kDepthScale;
                    const bool live = ts >= w.lo && ts < w.hi && q.d2 >= wskip;
                    if (!wave_any(live)) continue;
                    float x = 0.0f;
                    if (live) {
                        const float lw = fmaf(-(float)kLog2e, comp_front(L, ns, w, ts), log2_opacity(exp2_(q.d2), q.d2));
                        x = lr * (exp2_(lw - M2) * invS);
                    }
                    // sum over the wave in a fixed order
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
                    if (lane == 0) rec[i] += x;
                }
                if (!resident) {
                    __syncthreads();
                    for (int q = lane; q < cnt; q += 64) out[gb + q] += rec[q];
                }
            }
            const bool more = comp_next(w, L, ns);
            if (!wave_any(more)) break;
        }
    }
    if (resident) {
        __syncthreads();
        for (int q = lane; q < n; q += 64) out[q] = rec[q];
    }
}

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------

#define FMB_COMP_DISPATCH(flags, CALL)                                                                     \
    switch (flags) {                                                                                      \
    case 0: CALL(0); break;                                                                               \
    case 1: CALL(1); break;                                                                               \
    case 2: CALL(2); break;                                                                               \
    case 3: CALL(3); break;                                                                               \
    case 8: CALL(8); break;                                                                               \
    case 9: CALL(9); break;                                                                               \
    case 10: CALL(10); break;                                                                             \
    case 11: CALL(11); break;                                                                             \
    default: return hipErrorInvalidValue;                                                                 \
    }

#define FMB_FWDC_CALL(F_) hipLaunchKernelGGL((fwdc_kernel<F_>), dim3(n_items), dim3(64), 0, st, P, O, items, order)
#define FMB_BWDC_CALL(F_)                                                                                 \
    hipLaunchKernelGGL((bwdc_kernel<F_>), dim3(n_items), dim3(64), dyn, st, P, I, items, order, partial,    \
                       beta_partial)

// Blocks take the items in `order` (longest first) where given, else in item order.
hipError_t launch_fwdc(int flags, int n_items, hipStream_t st, const Params &P, const FwdOut &O,
                       const BwdItem *items, const int *order)
{
    flags &= ~kPer;
    if (n_items < 1) return hipSuccess;
    FMB_COMP_DISPATCH(flags, FMB_FWDC_CALL)
    return hipGetLastError();
}

// max_n: the largest scene of the batch (the slots' entries are staged only beyond one LDS tile).
hipError_t launch_bwdc(int flags, int n_items, hipStream_t st, const Params &P, const BwdIn &I,
                       const BwdItem *items, const int *order, float *partial, float *beta_partial, int max_n)
{
    flags &= ~kPer;
    if (n_items < 1) return hipSuccess;
    const size_t dyn = max_n > kCompTG ? (size_t)kCompSlots * 6 * sizeof(float4) : 0;
    FMB_COMP_DISPATCH(flags, FMB_BWDC_CALL)
    return hipGetLastError();
}

hipError_t launch_statc(int n_items, hipStream_t st, const Params &P, const float *loss, const float *stash,
                        const BwdItem *items, float *partial)
{
    if (n_items < 1) return hipSuccess;
    hipLaunchKernelGGL(statc_kernel, dim3(n_items), dim3(64), 0, st, P, loss, stash, items, partial);
    return hipGetLastError();
}

}  // namespace fmb
