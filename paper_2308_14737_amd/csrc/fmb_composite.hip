// fmb_composite.hip -- gfx950 kernels of the zero-parameter Fuzzy Metaballs renderer
// (alpha compositing, Keselman & Hebert, WACV 2024, Sec. 3.3, Eq. 9-10).
//
// Weights: w_i = T_i (1 - exp(-delta_i)), T_i = exp(-sum_j delta_j [t_j < t_i]), blended by
// Eq. (3) for depth, normals and colour; alpha is Eq. (8) as in the two-parameter model.
//
// Layout: one ray per segment of `seg` consecutive lanes of a wave, seg the smallest power of
// two >= N / 2 (at most 64; N / 3 in the forward at three Gaussians per lane, KM = 3); lane l
// of the segment holds Gaussians l, l + seg, ... (ke <= KM of them: two up to N = 128, three
// in the forward up to N = 192).  The segment writes its (t_i, delta_i) to LDS and every lane sums, for each of its
// Gaussians, the densities of the Gaussians strictly in front of it: an O(N) loop of LDS
// broadcasts per pair and no sort, with the strict inequality of Eq. (10) taken literally
// (Gaussians at equal depth do not attenuate one another).  Segment sums (max, weights,
// blended values) are butterflies over the segment's lanes.  A block of 256 lanes handles
// 4 * 64 / seg rays per step and loops over the rays of its item.
//
// Numerics: the weights enter Eq. (3) as base-2 logarithms,
//   log2 w_i = -log2(e) sum_{t_j < t_i} delta_j + log2(1 - exp(-delta_i)),
// shifted by their maximum over the ray, so rays far from every Gaussian keep finite weights;
// log2(1 - exp(-delta)) = log2(delta) + log2(e) (-delta/2 + delta^2/24 - delta^4/2880) below
// delta = 1/16 (truncation < 1e-12 relative), log2(1 - 2^(-delta log2 e)) above.
//
// Backward (per ray, same layout): with z_i = log w_i and z_bar_i = wt_i (tf_bar t_i +
// Nb.n_i + Cb.c_i - kappa) the softmax adjoint, delta_j enters every z_i behind it, so
//   d_bar_j = z_bar_j delta_j / expm1(delta_j) + delta_j (D_bar - sum_{t_j < t_i} z_bar_i),
//   t_bar_j = wt_j tf_bar (the indicator is piecewise constant),
// the second sum again an O(N) LDS loop; the rest of the per-pair adjoint is shared with the
// two-parameter renderer.  Partial gradients per item go to the same deterministic finalize.
#include "fmb_device.h"

namespace fmb {

constexpr int kCompBlock = 256;

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

// Lane exchanges within groups of 4, 8 and 16 lanes (DPP): quad_perm [1,0,3,2] and [2,3,0,1],
// and the mirror of each half-row (8 lanes) and row (16 lanes).  After the quad steps every
// lane of a quad holds the same value, so the mirrors pair each group with its neighbour.
template <int CTRL>
__device__ __forceinline__ float dpp_(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Sum (max) over the aligned group of `seg` lanes, left in every lane of the group.
__device__ __forceinline__ float seg_sum(float x, int seg)
{
    if (seg > 1) x += dpp_<0xB1>(x);
    if (seg > 2) x += dpp_<0x4E>(x);
    if (seg > 4) x += dpp_<0x141>(x);
    if (seg > 8) x += dpp_<0x140>(x);
    if (seg > 16) x += __shfl_xor(x, 16, 64);
    if (seg > 32) x += __shfl_xor(x, 32, 64);
    return x;
}

// Sums of eight values over the aligned group of `seg` >= 8 lanes, scattered over its lanes:
// three halving exchanges (each lane keeps half of its values and adds its partner's copy of
// that half, lanes seg/2, seg/4, seg/8 apart), then a sum over the remaining groups of seg/8
// lanes.  Lane l of the segment ends with the total of value seg8_index(l, seg) -- half the
// exchanges of eight separate sums, and no DPP (which issues at half rate).
__device__ __forceinline__ int seg8_index(int sl, int seg)
{
    return ((sl & (seg >> 1)) ? 4 : 0) + ((sl & (seg >> 2)) ? 2 : 0) + ((sl & (seg >> 3)) ? 1 : 0);
}

__device__ __forceinline__ float seg_sum8(const float x[8], int sl, int seg)
{
    float y[4], z[2];
    int o = seg >> 1;
    bool up = (sl & o) != 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] = (up ? x[i + 4] : x[i]) + __shfl_xor(up ? x[i] : x[i + 4], o, 64);
    o >>= 1;
    up = (sl & o) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) z[i] = (up ? y[i + 2] : y[i]) + __shfl_xor(up ? y[i] : y[i + 2], o, 64);
    o >>= 1;
    up = (sl & o) != 0;
    const float w = (up ? z[1] : z[0]) + __shfl_xor(up ? z[0] : z[1], o, 64);
    return seg_sum(w, seg >> 3);
}

__device__ __forceinline__ float seg_max(float x, int seg)
{
    if (seg > 1) x = fmaxf(x, dpp_<0xB1>(x));
    if (seg > 2) x = fmaxf(x, dpp_<0x4E>(x));
    if (seg > 4) x = fmaxf(x, dpp_<0x141>(x));
    if (seg > 8) x = fmaxf(x, dpp_<0x140>(x));
    if (seg > 16) x = fmaxf(x, __shfl_xor(x, 16, 64));
    if (seg > 32) x = fmaxf(x, __shfl_xor(x, 32, 64));
    return x;
}

// Orders the LDS accesses of one wave around this point, for data that only lanes of the same
// wave share (a segment's slots, a wave's epilogue records): the LDS performs one wave's
// operations in program order, and the fence and barrier keep the compiler from moving them
// across.  No block barrier, so the waves of a block do not wait for one another.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane geometry of a scene with n Gaussians.
struct CompLanes {
    int seg, ke;        // lanes per ray, Gaussians per lane
    int sl, sg, rpw;    // lane within the segment, segment within the wave, rays per wave
    int sbase;          // first LDS slot of the segment
};

template <int KM>
__device__ __forceinline__ CompLanes comp_lanes(int n)
{
    CompLanes c;
    c.seg = comp_seg(n, KM == 3 ? 3 : 2);
    c.ke = (n + c.seg - 1) / c.seg;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    c.sl = lane & (c.seg - 1);
    c.sg = lane / c.seg;
    c.rpw = 64 / c.seg;
    c.sbase = (wave * 64 + c.sg * c.seg) * KM;
    return c;
}

// Entries of the lane's Gaussians; a slot past the last Gaussian takes the last one's entry
// (finite arithmetic, zero weight and density).
template <int KM, bool COLOR>
__device__ __forceinline__ void comp_entries(const Params &P, const SceneRec &sr, const CompLanes &c,
                                             const double o[3], Ent g[KM], float4 cc[KM], bool gv[KM])
{
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        gv[k] = false;
        if (k < c.ke) {
            const int j = k * c.seg + c.sl;
            gv[k] = j < sr.n;
            const int gg = sr.gauss_off + (gv[k] ? j : sr.n - 1);
            float4 q[4];
            make_entry(P.means + 3 * gg, P.prec + 6 * gg, P.weights[gg], o, q);
            g[k] = ent_from(q[0], q[1], q[2], q[3]);
            if (COLOR) cc[k] = colour_entry(P.colors + 3 * gg);
        }
    }
}

// Densities below this are left out of the front sums: with at most 256 Gaussians they change a
// sum by less than 2^-22, so a log2 weight -log2(e) F + log2(1 - e^-delta) by less than
// 3.5e-7 (FP32 rounding of the weight itself), while about three quarters of the pairs of a
// typical ray have a density below it (the ray passes more than ~6 standard deviations away).
constexpr float kCompMinDensity = 0x1p-30f;
// Likewise, softmax adjoints z_bar_i of pairs whose normalised weight is below this are left out
// of the adjoint's sums over the Gaussians behind: |z_bar_i| <= w_i |lin_i - kappa| while a ray's
// largest term is at least (1/N) |lin - kappa|, so with N <= 256 a sum moves by less than
// N^2 2^-40 < 6e-8 of the ray's scale; about three quarters of the pairs fall below it.
constexpr float kCompMinWeight = 0x1p-40f;

// Depths are compared in the slot loops as clamp((t_k - t_j) * 2^100, 0, 1) (one subtraction
// with the clamp modifier on pre-scaled depths, then an FMA): 1 exactly when t_k > t_j, 0 when
// t_k <= t_j, for every pair of depths below 2^27 in magnitude whose difference is at least
// 2^-100, i.e. any two distinct depths this renderer meets.
constexpr float kDepthScale = 0x1p100f;

// Writes the segment's pairs (t_j kDepthScale, x_j) with x_j != 0 (DENSITY: x_j > kCompMinDensity) to its
// LDS slots, in Gaussian order, and (0, 0) to the rest of its seg * KM slots; returns the
// largest such count over the wave's segments, the same in every lane.  Terms left out add
// nothing (or below rounding) to the sums below, so the slot loops run that wave-uniform count
// (a scalar loop) and skip the Gaussians that cannot contribute.  The zero fill and the packed
// writes are LDS writes of one wave, which the LDS performs in program order.
template <int KM, bool DENSITY>
__device__ __forceinline__ int compact_slots(float2 *__restrict__ slots, const CompLanes &c, const Geo q[KM],
                                             const float x[KM])
{
    const int l0 = (threadIdx.x & 63) - c.sl;  // first lane of the segment
    const unsigned long long segmask = c.seg == 64 ? ~0ull : ((1ull << c.seg) - 1ull);
    const unsigned long long below = (1ull << c.sl) - 1ull;
#pragma unroll
    for (int k = 0; k < KM; ++k) slots[c.sl + k * c.seg] = make_float2(0.0f, 0.0f);
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        if (k < c.ke) {
            const bool nz = DENSITY ? x[k] > kCompMinDensity : x[k] != 0.0f;
            const unsigned long long bits = (__ballot(nz) >> l0) & segmask;
            if (nz) slots[cnt + __popcll(bits & below)] = make_float2(q[k].t * kDepthScale, x[k]);
            cnt += __popcll(bits);
        }
    }
    for (int off = c.seg; off < 64; off <<= 1) cnt = max(cnt, __shfl_xor(cnt, off, 64));
    return __builtin_amdgcn_readfirstlane(cnt);
}

// For each of the lane's Gaussians k: the sum of x_j over the first n slots with t_j < t_k
// (AFTER = false) or t_j > t_k, one pass over the slots for all of them.
template <int KM, bool AFTER>
__device__ __forceinline__ void ordered_sums(const float2 *__restrict__ slots, int n, const CompLanes &c,
                                             const Geo q[KM], float out[KM])
{
    float t[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        out[k] = 0.0f;
        t[k] = q[k].t * kDepthScale;
    }
    // 1 if slot depth ts is before (AFTER: behind) t, else 0
    auto step = [](float ts, float tk) {
        return __builtin_amdgcn_fmed3f(AFTER ? ts - tk : tk - ts, 0.0f, 1.0f);
    };
    int j = 0;
    for (; j + 4 <= n; j += 4) {
        const float2 a = slots[j], b = slots[j + 1], cc = slots[j + 2], d = slots[j + 3];
#pragma unroll
        for (int k = 0; k < KM; ++k) {  // k >= ke: computed and not used
            out[k] = fmaf(step(a.x, t[k]), a.y, out[k]);
            out[k] = fmaf(step(b.x, t[k]), b.y, out[k]);
            out[k] = fmaf(step(cc.x, t[k]), cc.y, out[k]);
            out[k] = fmaf(step(d.x, t[k]), d.y, out[k]);
        }
    }
    for (; j < n; ++j) {
        const float2 a = slots[j];
#pragma unroll
        for (int k = 0; k < KM; ++k) out[k] = fmaf(step(a.x, t[k]), a.y, out[k]);
    }
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k >= c.ke) out[k] = 0.0f;
}

// ------------------------------------------------------------------------------------
// Forward
// ------------------------------------------------------------------------------------

// Per-ray results wait in LDS (one record per ray) until the wave holds 64 of them; then
// each lane writes one ray's outputs.
constexpr int kEpiRec = 12;  // local ray index, M, S, T, N (3), C (3), D

template <int KM, int F>
__global__ __launch_bounds__(kCompBlock) void fwdc_kernel(Params P, FwdOut O, const BwdItem *__restrict__ items)
{
    constexpr bool NORMALS = (F & kNrm) != 0, COLOR = (F & kCol) != 0;
    __shared__ float2 tdl[kCompBlock * KM];
    __shared__ float epi[kCompBlock * kEpiRec];
    const BwdItem item = items[blockIdx.x];
    const ViewRec vr = P.views[item.view];
    const SceneRec sr = P.scenes[vr.scene];
    const int n = sr.n;
    const CompLanes c = comp_lanes<KM>(n);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float *__restrict__ e = P.w2c + 12 * item.view;
    const float *__restrict__ kk = P.intr + 4 * item.view;
    double o[3];
    cam_centre(e, o);
    const float o0 = (float)o[0], o1 = (float)o[1], o2 = (float)o[2];
    const float hm = (float)(-0.5 * kLog2e);
    Ent g[KM];
    float4 cc[KM];
    bool gv[KM];
    comp_entries<KM, COLOR>(P, sr, c, o, g, cc, gv);
    const int hw = vr.h * vr.w;
    const int end = min(item.ray0 + item.span, hw);
    float *__restrict__ my_epi = epi + wave * 64 * kEpiRec;
    int filled = 0;  // records waiting in this wave's slice (the same in every wave)

    for (int base = item.ray0; base < end; base += 4 * c.rpw) {
        const int local = base + wave * c.rpw + c.sg;
        const bool valid = local < end;
        float v0, v1, v2;
        ray_dir(P, vr, e, kk, valid ? local : end - 1, v0, v1, v2);
        Geo q[KM];
        float dl[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            if (k < c.ke) {
                pair_geo(g[k], v0, v1, v2, hm, 0.0f, 0.0f, q[k]);
                dl[k] = gv[k] ? exp2_(q[k].d2) : 0.0f;
            } else {
                dl[k] = 0.0f;
            }
        }
        wave_sync();  // the previous step is done with the slots
        const int cnt = compact_slots<KM, true>(tdl + c.sbase, c, q, dl);
        wave_sync();
        float front[KM];
        ordered_sums<KM, false>(tdl + c.sbase, cnt, c, q, front);
        float l2[KM];
        float mx = -INFINITY;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            l2[k] = -INFINITY;
            if (k < c.ke && gv[k]) l2[k] = fmaf(-(float)kLog2e, front[k], log2_opacity(dl[k], q[k].d2));
            mx = fmaxf(mx, l2[k]);
        }
        mx = seg_max(mx, c.seg);
        float S = 0, T = 0, N0 = 0, N1 = 0, N2 = 0, C0 = 0, C1 = 0, C2 = 0, D = 0;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            if (k < c.ke) {
                const float ew = exp2_(l2[k] - mx);  // 0 for an empty slot
                S += ew;
                T = fmaf(ew, q[k].t, T);
                D += dl[k];
                if (NORMALS) {
                    const PairNormal pn = pair_normal(g[k], q[k], 0.0f, 0.0f, 0.0f);
                    N0 = fmaf(ew, pn.n0, N0);
                    N1 = fmaf(ew, pn.n1, N1);
                    N2 = fmaf(ew, pn.n2, N2);
                }
                if (COLOR) {
                    C0 = fmaf(ew, cc[k].x, C0);
                    C1 = fmaf(ew, cc[k].y, C1);
                    C2 = fmaf(ew, cc[k].z, C2);
                }
            }
        }
        float *r = my_epi + (filled + c.sg) * kEpiRec;
        if (c.seg >= 8) {
            // S, T, D, N, C0, C1 scattered over the segment, each written by the lanes that hold it
            const float x[8] = {S, T, D, N0, N1, N2, C0, C1};
            const float v = seg_sum8(x, c.sl, c.seg);
            if (COLOR) C2 = seg_sum(C2, c.seg);
            if ((c.sl & ((c.seg >> 3) - 1)) == 0) {
                const int i = seg8_index(c.sl, c.seg);
                r[i < 2 ? 2 + i : (i == 2 ? 10 : 1 + i)] = v;  // S, T at 2, 3; D at 10; N, C0, C1 at 4..8
            }
            if (c.sl == 0) {
                r[0] = __int_as_float(valid ? local : -1);
                r[1] = mx;
                r[9] = C2;
            }
        } else {
            S = seg_sum(S, c.seg);
            T = seg_sum(T, c.seg);
            D = seg_sum(D, c.seg);
            if (NORMALS) {
                N0 = seg_sum(N0, c.seg);
                N1 = seg_sum(N1, c.seg);
                N2 = seg_sum(N2, c.seg);
            }
            if (COLOR) {
                C0 = seg_sum(C0, c.seg);
                C1 = seg_sum(C1, c.seg);
                C2 = seg_sum(C2, c.seg);
            }
            if (c.sl == 0) {
                r[0] = __int_as_float(valid ? local : -1);
                r[1] = mx; r[2] = S; r[3] = T; r[4] = N0; r[5] = N1; r[6] = N2;
                r[7] = C0; r[8] = C1; r[9] = C2; r[10] = D;
            }
        }
        filled += c.rpw;
        if (filled == 64 || base + 4 * c.rpw >= end) {
            wave_sync();
            if (lane < filled) {
                const float *r = my_epi + lane * kEpiRec;
                const int rl = __float_as_int(r[0]);
                if (rl >= 0) {
                    float at = 0.0f, dt = 0.0f;  // loss targets, loaded ahead of the direction
                    if (O.g_depth) {
                        at = O.alpha_t[vr.ray_off + rl];
                        dt = O.depth_t[vr.ray_off + rl];
                    }
                    float w0, w1, w2;
                    ray_dir(P, vr, e, kk, rl, w0, w1, w2);
                    write_ray<F>(P, O, item.view, vr.ray_off + rl, e, kk, o0, o1, o2, w0, w1, w2, r[1], r[2], r[3],
                                 r[4], r[5], r[6], r[7], r[8], r[9], r[10], at, dt);
                }
            }
            wave_sync();
            filled = 0;
        }
    }
}

// ------------------------------------------------------------------------------------
// Backward
// ------------------------------------------------------------------------------------

// Waves per SIMD the compositing adjoint is compiled for: five for the plain form at two
// Gaussians per lane (96 VGPRs; it spills 11-16 of its 112-119 and still runs 6 % faster than
// at four waves), else what its registers give.
constexpr int bwdc_min_waves(int km, int f) { return km == 2 && (f & (kNrm | kCol)) == 0 ? 5 : 1; }

template <int KM, int F>
__global__ __launch_bounds__(kCompBlock) __attribute__((amdgpu_waves_per_eu(bwdc_min_waves(KM, F)))) void bwdc_kernel(Params P, BwdIn I, const BwdItem *__restrict__ items,
                                                          float *__restrict__ partial, float *__restrict__ beta_partial)
{
    constexpr bool NORMALS = (F & kNrm) != 0, COLOR = (F & kCol) != 0;
    // without a normal cotangent the pairs take the offset form of the adjoint
    // (pair_adjoint_offset), which needs neither the refined peak nor r
    constexpr bool PLAIN = !NORMALS;
    constexpr int RW = COLOR ? 4 : 3;                        // float4 per staged ray
    constexpr int REC = COLOR ? kPartialColor : kPartial;   // partial record per Gaussian
    // a lane's sums per Gaussian: (H, Bv, L) of the offset form or the general record, then colour
    constexpr int LREC = PLAIN ? kOffsetAcc + (COLOR ? 3 : 0) : REC;
    constexpr int RAYS4 = kCompBlock * RW;
    constexpr int RED4 = (kCompBlock * KM * LREC + 3) / 4;
    __shared__ float4 smem[RAYS4 > RED4 ? RAYS4 : RED4];     // staged rays, then the reduction
    __shared__ float2 tdl[kCompBlock * KM];
    const int tid = threadIdx.x;
    const BwdItem item = items[blockIdx.x];
    const ViewRec vr = P.views[item.view];
    const SceneRec sr = P.scenes[vr.scene];
    const int n = sr.n;
    const CompLanes c = comp_lanes<KM>(n);
    const int wave = tid >> 6;
    const float *__restrict__ e = P.w2c + 12 * item.view;
    const float *__restrict__ kk = P.intr + 4 * item.view;
    double o[3];
    cam_centre(e, o);
    const float o0 = (float)o[0], o1 = (float)o[1], o2 = (float)o[2];
    const float hm = (float)(-0.5 * kLog2e);
    Ent g[KM];
    float4 cc[KM];
    bool gv[KM];
    comp_entries<KM, COLOR>(P, sr, c, o, g, cc, gv);
    PairAcc acc[KM];
    OffsetAcc pacc[KM];
    float aC[KM][3];
#pragma unroll
    for (int k = 0; k < KM; ++k) aC[k][0] = aC[k][1] = aC[k][2] = 0.0f;
    const int hw = vr.h * vr.w;
    const int end = min(item.ray0 + item.span, hw);
    const int step = 4 * c.rpw;

    // rays are staged kCompBlock at a time (one prologue per thread), then taken a step of
    // 4 * 64 / seg rays at a time
    for (int sb = item.ray0; sb < end; sb += kCompBlock) {
        __syncthreads();  // the previous stage is done with the staged rays
        {
            float4 pr[4];
            ray_prologue<F>(P, I, item.view, vr, e, kk, o0, o1, o2, sb + tid, sb + tid < end, 0.0f, 0.0f, pr);
#pragma unroll
            for (int w = 0; w < RW; ++w) smem[RW * tid + w] = pr[w];
        }
        __syncthreads();  // the staged rays are visible to every wave
        for (int s0 = 0; s0 < kCompBlock && sb + s0 < end; s0 += step) {
            wave_sync();  // the previous step is done with the slots
            const int ry = s0 + wave * c.rpw + c.sg;
            const float4 x0 = smem[RW * ry], x1 = smem[RW * ry + 1], x2 = smem[RW * ry + 2];
            float4 x3 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (COLOR) x3 = smem[RW * ry + 3];
            const float v0 = x0.x, v1 = x0.y, v2 = x0.z, M2 = x0.w, invS = x1.x, tfb = x1.y;
            const float nb0 = x1.z, nb1 = x1.w, nb2 = x2.x, kap = x2.y, Db = x2.z;
            Geo q[KM];
            float dl[KM];
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                dl[k] = 0.0f;
                if (k < c.ke) {
                    if (PLAIN)
                        pair_geo_coarse(g[k], v0, v1, v2, hm, 0.0f, 0.0f, q[k]);
                    else
                        pair_geo(g[k], v0, v1, v2, hm, 0.0f, 0.0f, q[k]);
                    dl[k] = gv[k] ? exp2_(q[k].d2) : 0.0f;
                }
            }
            const int cnt = compact_slots<KM, true>(tdl + c.sbase, c, q, dl);
            wave_sync();
            float front[KM];
            ordered_sums<KM, false>(tdl + c.sbase, cnt, c, q, front);
            float wt[KM], zb[KM];
            PairNormal pn[KM];
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                wt[k] = zb[k] = 0.0f;
                pn[k] = PairNormal{0, 0, 0, 0, 0};
                if (k < c.ke) {
                    if (gv[k]) wt[k] = exp2_(fmaf(-(float)kLog2e, front[k], log2_opacity(dl[k], q[k].d2)) - M2) * invS;
                    if (NORMALS) pn[k] = pair_normal(g[k], q[k], nb0, nb1, nb2);
                    float lin = fmaf(tfb, q[k].t, pn[k].nN);
                    if (COLOR) lin = fmaf(x3.x, cc[k].x, fmaf(x3.y, cc[k].y, fmaf(x3.z, cc[k].z, lin)));
                    zb[k] = wt[k] * (lin - kap);
                }
            }
            wave_sync();  // the segment is done reading (t, delta)
            float zp[KM];  // the terms of the behind sums
#pragma unroll
            for (int k = 0; k < KM; ++k) zp[k] = wt[k] >= kCompMinWeight ? zb[k] : 0.0f;
            const int cnt_b = compact_slots<KM, false>(tdl + c.sbase, c, q, zp);
            wave_sync();
            float behind[KM];
            ordered_sums<KM, true>(tdl + c.sbase, cnt_b, c, q, behind);
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (k < c.ke) {
                    const float db = fmaf(zb[k], opacity_slope(dl[k]), dl[k] * (Db - behind[k]));
                    const float tb = wt[k] * tfb;
                    if (COLOR) {
                        aC[k][0] = fmaf(wt[k], x3.x, aC[k][0]);
                        aC[k][1] = fmaf(wt[k], x3.y, aC[k][1]);
                        aC[k][2] = fmaf(wt[k], x3.z, aC[k][2]);
                    }
                    if (PLAIN)
                        pair_adjoint_offset(q[k], v0, v1, v2, tb, db, pacc[k]);
                    else
                        pair_adjoint<NORMALS>(g[k], q[k], v0, v1, v2, wt[k], pn[k], nb0, nb1, nb2, tb, db, acc[k]);
                }
            }
        }
    }

    // deterministic reduction over the block's segments: Gaussian j's record sums the lanes
    // holding it in wave order, then segment order
    __syncthreads();
    float *red = reinterpret_cast<float *>(smem);
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        float *my = red + (tid * KM + k) * LREC;
        if (PLAIN) {
            offset_acc_store(pacc[k], my);
        } else {
            const PairAcc &a = acc[k];
            my[0] = a.u0; my[1] = a.u1; my[2] = a.u2; my[3] = a.u3; my[4] = a.u4; my[5] = a.u5;
            my[6] = a.p0; my[7] = a.p1; my[8] = a.p2; my[9] = a.l;
        }
        if (COLOR) {
            my[LREC - 3] = aC[k][0]; my[LREC - 2] = aC[k][1]; my[LREC - 1] = aC[k][2];
        }
    }
    __syncthreads();
    if (tid < n) {
        const int k = tid / c.seg, l = tid % c.seg;
        float sum[LREC];
#pragma unroll
        for (int v = 0; v < LREC; ++v) sum[v] = 0.0f;
        for (int w = 0; w < kCompBlock / 64; ++w)
            for (int s = 0; s < c.rpw; ++s) {
                const float *src = red + ((w * 64 + s * c.seg + l) * KM + k) * LREC;
#pragma unroll
                for (int v = 0; v < LREC; ++v) sum[v] += src[v];
            }
        const int gg = sr.gauss_off + tid;
        if (PLAIN)
            write_partial_offset(partial + item.poff + REC * tid, sum, REC, P.prec + 6 * gg, P.means + 3 * gg, o);
        else
            write_partial(partial + item.poff + REC * tid, sum, REC, P.means + 3 * gg, o);
    }
    if (tid < 2) beta_partial[2 * item.seq + tid] = 0.0f;  // the model has no blend parameters
}

// ------------------------------------------------------------------------------------
// Split statistic (Sec. 8) with the compositing weights: lbar_i = (1/M) sum_j L_j w_ji,
// same layout as the backward; the running maximum and 1/S come from the forward's stash.
// ------------------------------------------------------------------------------------

template <int KM>
__global__ __launch_bounds__(kCompBlock) void statc_kernel(Params P, const float *__restrict__ loss,
                                                           const float *__restrict__ stash,
                                                           const BwdItem *__restrict__ items,
                                                           float *__restrict__ partial)
{
    __shared__ float4 rays[kCompBlock * 2];
    __shared__ float2 tdl[kCompBlock * KM];
    __shared__ float red[kCompBlock * KM];
    const int tid = threadIdx.x;
    const BwdItem item = items[blockIdx.x];
    const ViewRec vr = P.views[item.view];
    const SceneRec sr = P.scenes[vr.scene];
    const int n = sr.n;
    const CompLanes c = comp_lanes<KM>(n);
    const int wave = tid >> 6;
    const float *__restrict__ e = P.w2c + 12 * item.view;
    const float *__restrict__ kk = P.intr + 4 * item.view;
    double o[3];
    cam_centre(e, o);
    const float hm = (float)(-0.5 * kLog2e);
    Ent g[KM];
    float4 cc[KM];
    bool gv[KM];
    comp_entries<KM, false>(P, sr, c, o, g, cc, gv);
    float acc[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) acc[k] = 0.0f;
    const int hw = vr.h * vr.w;
    const int end = min(item.ray0 + item.span, hw);
    const int step = 4 * c.rpw;
    for (int base = item.ray0; base < end; base += step) {
        __syncthreads();
        if (tid < step) {
            const int local = base + tid;
            float4 a = make_float4(0.0f, 0.0f, 1.0f, INFINITY), b = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (local < end) {
                const int r = vr.ray_off + local;
                float v0, v1, v2;
                ray_dir(P, vr, e, kk, local, v0, v1, v2);
                const float4 s0 = reinterpret_cast<const float4 *>(stash)[2 * (size_t)r];
                a = make_float4(v0, v1, v2, s0.x);
                b = make_float4(s0.y, loss[r], 0.0f, 0.0f);
            }
            rays[2 * tid] = a;
            rays[2 * tid + 1] = b;
        }
        __syncthreads();
        const int ry = wave * c.rpw + c.sg;
        const float4 x0 = rays[2 * ry], x1 = rays[2 * ry + 1];
        Geo q[KM];
        float dl[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            dl[k] = 0.0f;
            if (k < c.ke) {
                pair_geo(g[k], x0.x, x0.y, x0.z, hm, 0.0f, 0.0f, q[k]);
                dl[k] = gv[k] ? exp2_(q[k].d2) : 0.0f;
            }
        }
        const int cnt = compact_slots<KM, true>(tdl + c.sbase, c, q, dl);
        __syncthreads();
        float front[KM];
        ordered_sums<KM, false>(tdl + c.sbase, cnt, c, q, front);
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            if (k < c.ke && gv[k]) {
                const float wt = exp2_(fmaf(-(float)kLog2e, front[k], log2_opacity(dl[k], q[k].d2)) - x0.w) * x1.x;
                acc[k] = fmaf(x1.y, wt, acc[k]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KM; ++k) red[tid * KM + k] = acc[k];
    __syncthreads();
    if (tid < n) {
        const int k = tid / c.seg, l = tid % c.seg;
        float sum = 0.0f;
        for (int w = 0; w < kCompBlock / 64; ++w)
            for (int sgi = 0; sgi < c.rpw; ++sgi) sum += red[(w * 64 + sgi * c.seg + l) * KM + k];
        partial[item.poff + tid] = sum;
    }
}

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------

#define FMB_COMP_DISPATCH(KM_, flags, CALL)                                                                \
    switch (flags) {                                                                                      \
    case 0: CALL(KM_, 0); break;                                                                          \
    case 1: CALL(KM_, 1); break;                                                                          \
    case 2: CALL(KM_, 2); break;                                                                          \
    case 3: CALL(KM_, 3); break;                                                                          \
    case 8: CALL(KM_, 8); break;                                                                          \
    case 9: CALL(KM_, 9); break;                                                                          \
    case 10: CALL(KM_, 10); break;                                                                        \
    case 11: CALL(KM_, 11); break;                                                                        \
    default: return hipErrorInvalidValue;                                                                 \
    }

#define FMB_FWDC_CALL(KM_, F_)                                                                            \
    hipLaunchKernelGGL((fwdc_kernel<KM_, F_>), dim3(n_items), dim3(kCompBlock), 0, st, P, O, items)
#define FMB_BWDC_CALL(KM_, F_)                                                                            \
    hipLaunchKernelGGL((bwdc_kernel<KM_, F_>), dim3(n_items), dim3(kCompBlock), 0, st, P, I, items, partial, \
                       beta_partial)

hipError_t launch_fwdc(int km, int flags, int n_items, hipStream_t st, const Params &P, const FwdOut &O,
                       const BwdItem *items)
{
    flags &= ~kPer;
    if (n_items < 1) return hipSuccess;
    if (km == 1) {
        FMB_COMP_DISPATCH(1, flags, FMB_FWDC_CALL)
    } else if (km == 2) {
        FMB_COMP_DISPATCH(2, flags, FMB_FWDC_CALL)
    } else if (km == 3) {
        FMB_COMP_DISPATCH(3, flags, FMB_FWDC_CALL)
    } else if (km == 4) {
        FMB_COMP_DISPATCH(4, flags, FMB_FWDC_CALL)
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bwdc(int km, int flags, int n_items, hipStream_t st, const Params &P, const BwdIn &I,
                       const BwdItem *items, float *partial, float *beta_partial)
{
    flags &= ~kPer;
    if (n_items < 1) return hipSuccess;
    if (km == 1) {
        FMB_COMP_DISPATCH(1, flags, FMB_BWDC_CALL)
    } else if (km == 2) {
        FMB_COMP_DISPATCH(2, flags, FMB_BWDC_CALL)
    } else if (km == 4) {
        FMB_COMP_DISPATCH(4, flags, FMB_BWDC_CALL)
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_statc(int km, int n_items, hipStream_t st, const Params &P, const float *loss, const float *stash,
                        const BwdItem *items, float *partial)
{
    if (n_items < 1) return hipSuccess;
    if (km == 1)
        hipLaunchKernelGGL((statc_kernel<1>), dim3(n_items), dim3(kCompBlock), 0, st, P, loss, stash, items, partial);
    else if (km == 2)
        hipLaunchKernelGGL((statc_kernel<2>), dim3(n_items), dim3(kCompBlock), 0, st, P, loss, stash, items, partial);
    else if (km == 4)
        hipLaunchKernelGGL((statc_kernel<4>), dim3(n_items), dim3(kCompBlock), 0, st, P, loss, stash, items, partial);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace fmb
