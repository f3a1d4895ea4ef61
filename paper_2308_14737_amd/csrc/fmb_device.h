// fmb_device.h -- device helpers shared by the gfx950 kernels of both renderers: the
// (view, Gaussian) entry formed in FP64, rays and projections, the geometry of one
// (ray, Gaussian) pair, the per-ray adjoint prologue and the per-pair adjoint that maps
// (dL/dt_i, dL/dd_i, dL/dn_i) to the Gaussian's parameters.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fmb_internal.h"

namespace fmb {

// ------------------------------------------------------------------------------------
// Small helpers
// ------------------------------------------------------------------------------------

__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float exp2_(float x) { return __builtin_amdgcn_exp2f(x); }

struct Ent {  // one (view, Gaussian) entry: 16 floats = 4 x float4 in LDS
    float u00, u01, u02, u11, u12, u22;  // packed upper U
    float mh0, mh1, mh2;                 // mu - o rounded to float ("high part")
    float ul0, ul1, ul2;                 // U (mu - o - high part): the low part, through U
    float c0, c1, c2;                    // Sigma^-1 (mu - o)
    float l2l;                           // log2 lambda
};

__device__ __forceinline__ Ent ent_from(const float4 a, const float4 b, const float4 c, const float4 d)
{
    return Ent{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w};
}

// Block-uniform, read-only metadata (work items, view and scene records, cameras, betas):
// a load through the constant address space becomes a scalar load whose result stays in
// SGPRs.  Inside a persistent loop the kernel's own stores would otherwise keep the compiler
// from proving the records unchanged, and it would fall back to vector loads and VGPRs.  No
// kernel writes these arrays.
template <class T>
__device__ __forceinline__ T ld_uniform(const T *p)
{
    static_assert(sizeof(T) % 4 == 0 && alignof(T) >= 4, "records of 32-bit words");
    const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)p;
    uint32_t w[sizeof(T) / 4];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = q[i];
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}

// Wave votes over the active lanes.  The predicate goes to the ballot as the lane mask its
// comparison already produces; the int-predicate forms widen it to a 0/1 integer per lane and
// compare that again (two extra vector instructions per vote).
__device__ __forceinline__ unsigned long long wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }
__device__ __forceinline__ bool wave_all(bool p) { return __builtin_amdgcn_ballot_w64(!p) == 0; }

struct CamRec {  // world-to-camera [R | T] row-major, then (fx, fy, cx, cy)
    float e[12];
    float k[4];
};

__device__ __forceinline__ CamRec cam_of(const Params &P, int view)
{
    CamRec c;
#pragma unroll
    for (int i = 0; i < 12; ++i) c.e[i] = ld_uniform(P.w2c + 12 * view + i);
#pragma unroll
    for (int i = 0; i < 4; ++i) c.k[i] = ld_uniform(P.intr + 4 * view + i);
    return c;
}

// Camera centre o = -R^T T in double.
__device__ __forceinline__ void cam_centre(const float *__restrict__ e, double o[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
        o[a] = -((double)e[a] * (double)e[3] + (double)e[4 + a] * (double)e[7] +
                 (double)e[8 + a] * (double)e[11]);
}

// (view, Gaussian) entry in double, rounded to float.  mu - o is split as hi + lo; the
// pair loop forms U (t v - mu') as U (t v - hi) - U lo, so only U lo is stored.  log2 lambda
// is the FP32 log2 (within an ulp of the rounded double): the FP64 routine's polynomial
// constants would be hoisted out of a persistent loop and held in VGPRs for the whole kernel.
__device__ __forceinline__ void make_entry(const float *__restrict__ mu, const float *__restrict__ u,
                                           float lam, const double o[3], float4 out[4])
{
    const double m0 = (double)mu[0] - o[0], m1 = (double)mu[1] - o[1], m2 = (double)mu[2] - o[2];
    const float h0 = (float)m0, h1 = (float)m1, h2 = (float)m2;
    const double l0 = m0 - (double)h0, l1 = m1 - (double)h1, l2 = m2 - (double)h2;
    const double U00 = u[0], U01 = u[1], U02 = u[2], U11 = u[3], U12 = u[4], U22 = u[5];
    const double b0 = U00 * m0 + U01 * m1 + U02 * m2;
    const double b1 = U11 * m1 + U12 * m2;
    const double b2 = U22 * m2;
    const double c0 = U00 * b0;
    const double c1 = U01 * b0 + U11 * b1;
    const double c2 = U02 * b0 + U12 * b1 + U22 * b2;
    const double ul0 = U00 * l0 + U01 * l1 + U02 * l2, ul1 = U11 * l1 + U12 * l2, ul2 = U22 * l2;
    out[0] = make_float4(u[0], u[1], u[2], u[3]);
    out[1] = make_float4(u[4], u[5], h0, h1);
    out[2] = make_float4(h2, (float)ul0, (float)ul1, (float)ul2);
    out[3] = make_float4((float)c0, (float)c1, (float)c2, log2f(lam));
}

// The entry and, as a fifth float4, (|U mu'|^2, |Sigma^-1 mu'|_1, 0, 0): the terms of the one-FMA
// estimate of the squared Mahalanobis distance m = |U mu'|^2 - (v.c) t and of its error bound
// (pair_m_low).
__device__ __forceinline__ void make_entry_est(const float *__restrict__ mu, const float *__restrict__ u,
                                               float lam, const double o[3], float4 out[5])
{
    make_entry(mu, u, lam, o, out);
    const double m0 = (double)mu[0] - o[0], m1 = (double)mu[1] - o[1], m2 = (double)mu[2] - o[2];
    const double U00 = u[0], U01 = u[1], U02 = u[2], U11 = u[3], U12 = u[4], U22 = u[5];
    const double b0 = U00 * m0 + U01 * m1 + U02 * m2;
    const double b1 = U11 * m1 + U12 * m2;
    const double b2 = U22 * m2;
    const double c0 = U00 * b0, c1 = U01 * b0 + U11 * b1, c2 = U02 * b0 + U12 * b1 + U22 * b2;
    out[4] = make_float4((float)(b0 * b0 + b1 * b1 + b2 * b2), (float)(fabs(c0) + fabs(c1) + fabs(c2)), 0.0f,
                         0.0f);
}

// Unit direction of the ray through the centre of pixel (row, col).
__device__ __forceinline__ void pixel_dir(const float *__restrict__ e, const float *__restrict__ k, int row,
                                          int col, float &v0, float &v1, float &v2)
{
    const float dx = ((float)col + 0.5f - k[2]) / k[0];
    const float dy = ((float)row + 0.5f - k[3]) / k[1];
    const float x = fmaf(e[0], dx, fmaf(e[4], dy, e[8]));
    const float y = fmaf(e[1], dx, fmaf(e[5], dy, e[9]));
    const float z = fmaf(e[2], dx, fmaf(e[6], dy, e[10]));
    const float inv = 1.0f / sqrtf(fmaf(x, x, fmaf(y, y, z * z)));
    v0 = x * inv;
    v1 = y * inv;
    v2 = z * inv;
}

// Direction of ray `local` of view `vr`: the pixel ray, or the given direction normalised.
__device__ __forceinline__ void ray_dir(const Params &P, const ViewRec &vr, const float *__restrict__ e,
                                        const float *__restrict__ k, int local, float &v0, float &v1, float &v2)
{
    if (P.dirs) {
        const float *d = P.dirs + 3 * ((size_t)vr.ray_off + local);
        const float x = d[0], y = d[1], z = d[2];
        const float inv = 1.0f / sqrtf(fmaf(x, x, fmaf(y, y, z * z)));
        v0 = x * inv;
        v1 = y * inv;
        v2 = z * inv;
    } else {
        pixel_dir(e, k, local / vr.w, local % vr.w, v0, v1, v2);
    }
}

// Ray `lane` of ray tile `tile` of view `vr` (see ViewRec): its local index (row-major pixel
// index, or explicit-ray index), or -1 past the view's edge; `row` and `col` give the pixel of an
// 8 x 8 tile.  `tile` is uniform over the wave.
__device__ __forceinline__ int tile_local(const ViewRec &vr, int tile, int lane, int &row, int &col)
{
    if (vr.tiles_x > 0) {
        const int ty = tile / vr.tiles_x, tx = tile - ty * vr.tiles_x;
        row = 8 * ty + (lane >> 3);
        col = 8 * tx + (lane & 7);
        return (tile < vr.tiles && row < vr.h && col < vr.w) ? row * vr.w + col : -1;
    }
    const int local = 64 * tile + lane;
    row = col = 0;
    return local < vr.h * vr.w ? local : -1;
}

// Direction of the ray of a tile lane with local index `local` >= 0 (tile_local's row and col).
__device__ __forceinline__ void tile_ray_dir(const Params &P, const ViewRec &vr, const float *__restrict__ e,
                                             const float *__restrict__ k, int local, int row, int col, float &v0,
                                             float &v1, float &v2)
{
    if (!P.dirs && vr.tiles_x > 0)
        pixel_dir(e, k, row, col, v0, v1, v2);
    else
        ray_dir(P, vr, e, k, local, v0, v1, v2);
}

__device__ __forceinline__ void project(const float *__restrict__ e, const float *__restrict__ k, float p0,
                                        float p1, float p2, float &u, float &v)
{
    const float q0 = fmaf(e[0], p0, fmaf(e[1], p1, fmaf(e[2], p2, e[3])));
    const float q1 = fmaf(e[4], p0, fmaf(e[5], p1, fmaf(e[6], p2, e[7])));
    const float q2 = fmaf(e[8], p0, fmaf(e[9], p1, fmaf(e[10], p2, e[11])));
    const float iz = 1.0f / q2;
    u = fmaf(k[0] * q0, iz, k[2]);
    v = fmaf(k[1] * q1, iz, k[3]);
}

// Geometry of one (ray, Gaussian) pair.
struct Geo {
    float a0, a1, a2, raa;  // a = U v, 1/(a.a)
    float t;                // peak depth
    float w0, w1, w2;       // t v - mu' (the high part of mu'): the peak point relative to the mean
    float r0, r1, r2;       // r = U (t v - mu'), at the refined peak after pair_refine
    float d2, z2;           // log2 density, log2 blend weight
};

// The peak t = v.c / a.a and r = U (t v - mu') with mu' = hi + lo as U (t v - hi) - U lo, then
// m = r.r, the log2 density d2 and the log2 weight z2.  The rounding error of t is below
// cond(Sigma^-1) times a few ulp (v.c is a dot product whose terms are at most that factor
// larger than the sum); it enters m only to second order (m is minimal at the peak), so t is
// the pair's depth and d2 and z2 are final here.
// The first half of pair_geo_coarse: a, 1/(a.a) and the peak t; returns v.c.
__device__ __forceinline__ float pair_geo_peak(const Ent &g, float v0, float v1, float v2, Geo &q)
{
    q.a0 = fmaf(g.u00, v0, fmaf(g.u01, v1, g.u02 * v2));
    q.a1 = fmaf(g.u11, v1, g.u12 * v2);
    q.a2 = g.u22 * v2;
    const float aa = fmaf(q.a0, q.a0, fmaf(q.a1, q.a1, q.a2 * q.a2));
    const float vc = fmaf(v0, g.c0, fmaf(v1, g.c1, v2 * g.c2));
    q.raa = rcp_(aa);
    q.t = vc * q.raa;
    return vc;
}

// The second half: w = t v - hi, r = U w - U lo, the log2 density d2 and weight z2.
__device__ __forceinline__ void pair_geo_resid(const Ent &g, float v0, float v1, float v2, float hm, float b1,
                                               float nc2, Geo &q)
{
    q.w0 = fmaf(q.t, v0, -g.mh0);
    q.w1 = fmaf(q.t, v1, -g.mh1);
    q.w2 = fmaf(q.t, v2, -g.mh2);
    q.r0 = fmaf(g.u00, q.w0, fmaf(g.u01, q.w1, fmaf(g.u02, q.w2, -g.ul0)));
    q.r1 = fmaf(g.u11, q.w1, fmaf(g.u12, q.w2, -g.ul1));
    q.r2 = fmaf(g.u22, q.w2, -g.ul2);
    const float m = fmaf(q.r0, q.r0, fmaf(q.r1, q.r1, q.r2 * q.r2));
    q.d2 = fmaf(hm, m, g.l2l);
    q.z2 = fmaf(b1, q.d2, nc2 * q.t);
}

// A lower bound of the m that pair_geo_resid forms, from the entry's fifth float4 est and v.c:
// m = |U mu'|^2 - (v.c)^2 / (a.a) estimated as est.x - (v.c) t in one FMA.  Its rounding error is a
// few units of 2^-24 (|U mu'|^2 + |Sigma^-1 mu'|_1 |t|) (the terms that cancel; (v.c) t is at most
// |U mu'|^2), and the residual form's own error is smaller still, so 2^-17 of that sum bounds both.
__device__ __forceinline__ float pair_m_low(const float4 &est, float vc, float t)
{
    constexpr float kErr = 0x1p-17f;
    return fmaf(-kErr, fmaf(est.y, fabsf(t), est.x), fmaf(-vc, t, est.x));
}

// Upper bounds of the log2 density and of beta1 log2(density) + |nc2| |t| over every ray of a
// tile, from the tile's unit centre direction c and the largest distance rho of its unit ray
// directions from c (tc = (c, rho)), for the Gaussian of entry g (est: its m estimate terms).
// For a ray v, any depth t gives |U(t v - mu')| >= |U(t c - mu')| - |U|_2 |t| |v - c|, so the
// ray's m is at least (sqrt(m_c) - |U|_2 t_max rho)^2 with m_c the centre ray's m (from below, as
// pair_m_low bounds it) and t_max >= |t| = |(U v).(U mu')| / |U v|^2 <= |U mu'| |U^-1|_2; the
// 2-norms are bounded by sqrt(|.|_1 |.|_inf).  The slack terms cover the FP32 rounding of the bound.
__device__ __forceinline__ void tile_bounds(const Ent &g, const float4 &est, const float4 &tc, float hm, float b1,
                                            float nc2, float &d2_hi, float &z_hi)
{
    Geo qc;
    const float vc = pair_geo_peak(g, tc.x, tc.y, tc.z, qc);
    const float mc = fmaxf(pair_m_low(est, vc, qc.t), 0.0f);
    const float a00 = fabsf(g.u00), a01 = fabsf(g.u01), a02 = fabsf(g.u02);
    const float a11 = fabsf(g.u11), a12 = fabsf(g.u12), a22 = fabsf(g.u22);
    const float u2 = sqrtf(fmaxf(a00, fmaxf(a01 + a11, a02 + a12 + a22)) * fmaxf(a00 + a01 + a02, fmaxf(a11 + a12, a22)));
    // U^-1 of the upper-triangular U
    const float i00 = rcp_(g.u00), i11 = rcp_(g.u11), i22 = rcp_(g.u22);
    const float i01 = -g.u01 * i00 * i11, i12 = -g.u12 * i11 * i22;
    const float i02 = (g.u01 * g.u12 - g.u02 * g.u11) * i00 * i11 * i22;
    const float c1 = fmaxf(fabsf(i00), fmaxf(fabsf(i01) + fabsf(i11), fabsf(i02) + fabsf(i12) + fabsf(i22)));
    const float r1 = fmaxf(fabsf(i00) + fabsf(i01) + fabsf(i02), fmaxf(fabsf(i11) + fabsf(i12), fabsf(i22)));
    const float tmax = sqrtf(est.x * c1 * r1) * (1.0f + 1e-4f);
    const float lo = fmaxf(0.0f, sqrtf(mc) * (1.0f - 1e-4f) - u2 * tmax * tc.w * (1.0f + 1e-4f));
    d2_hi = fmaf(hm, lo * lo * (1.0f - 1e-4f), g.l2l) + 1e-3f;
    z_hi = fmaf(b1, d2_hi, fabsf(nc2) * tmax);
}

__device__ __forceinline__ void pair_geo_coarse(const Ent &g, float v0, float v1, float v2, float hm, float b1,
                                                float nc2, Geo &q)
{
    pair_geo_peak(g, v0, v1, v2, q);
    pair_geo_resid(g, v0, v1, v2, hm, b1, nc2, q);
}

// The residual at the refined peak: one Newton step on t -> |U (t v - mu')|^2 (exactly
// quadratic), dt = (a.r)/(a.a), applied to r only.  r, unlike m, has a first-order error in t,
// and the normal g = U^T r amplifies it by |U|; after the step a.r = 0 to rounding, which the
// general adjoint relies on.  The depth stays t (its own error is ~1e-6 relative), so every
// kernel blends and differentiates the same depth.
__device__ __forceinline__ void pair_refine(Geo &q)
{
    const float dt = fmaf(q.a0, q.r0, fmaf(q.a1, q.r1, q.a2 * q.r2)) * q.raa;
    q.r0 = fmaf(-dt, q.a0, q.r0);
    q.r1 = fmaf(-dt, q.a1, q.r1);
    q.r2 = fmaf(-dt, q.a2, q.r2);
}

__device__ __forceinline__ void pair_geo(const Ent &g, float v0, float v1, float v2, float hm, float b1,
                                         float nc2, Geo &q)
{
    pair_geo_coarse(g, v0, v1, v2, hm, b1, nc2, q);
    pair_refine(q);
}

// Per-item blend constants of a scene: hm = -log2(e)/2, b1 = beta1, nc2 = -beta2 log2(e)/eta.
struct Blend {
    float hm, b1, nc2, cb;  // cb = beta2 / eta (natural units, backward)
    float inv_eta;
};

__device__ __forceinline__ Blend blend_of(const Params &P, int s)
{
    const double b1 = ld_uniform(P.betas + 2 * s), b2 = ld_uniform(P.betas + 2 * s + 1);
    const double eta = ld_uniform(P.eta + s);
    Blend b;
    b.hm = (float)(-0.5 * kLog2e);
    b.b1 = (float)b1;
    b.nc2 = (float)(-b2 * kLog2e / eta);
    b.cb = (float)(b2 / eta);
    b.inv_eta = (float)(1.0 / eta);
    return b;
}

// ------------------------------------------------------------------------------------
// Kernel variants: F is a bit set of the outputs/cotangents a launch handles.
// ------------------------------------------------------------------------------------

constexpr int kNrm = 1;  // normals (Eq. 17)
constexpr int kFlw = 2;  // flow to a second pose (Sec. 5)
constexpr int kPer = 4;  // persistent work queue
constexpr int kCol = 8;  // per-Gaussian colour blended by Eq. (3)
constexpr int kBig = 16;  // forward: scenes beyond a block's count of Gaussians take pre-culled rounds

// Colour of a Gaussian: sigmoid of the unconstrained parameters (double, rounded).
__device__ __forceinline__ float4 colour_entry(const float *__restrict__ q)
{
    return make_float4((float)(1.0 / (1.0 + exp(-(double)q[0]))), (float)(1.0 / (1.0 + exp(-(double)q[1]))),
                       (float)(1.0 / (1.0 + exp(-(double)q[2]))), 0.0f);
}

// Gradient of one ray's loss terms with respect to its alpha and depth (Sec. 4: binary cross
// entropy of alpha, clamped to [1e-6, 1 - 1e-6], against the target mask, and the mask-weighted
// L1 depth term with weight w_depth), each divided by the ray count (inv_p = 1/p).  The loss
// kernel and the forward's fused epilogue both use it, so their cotangents agree bit for bit.
__device__ __forceinline__ void loss_grad_ray(float a, float at, float d, float dt, float w_depth, float inv_p,
                                              float &ga, float &gd)
{
    const float ac = fminf(fmaxf(a, 1e-6f), 1.0f - 1e-6f);
    const bool inside = a >= 1e-6f && a <= 1.0f - 1e-6f;
    ga = inside ? (ac - at) / (ac * (1.0f - ac)) * inv_p : 0.0f;
    const float dd = d - dt;
    gd = w_depth * at * (float)((dd > 0.0f) - (dd < 0.0f)) * inv_p;
}

// Outputs of ray r (global index) of view `view` from its blended sums, common to both
// renderers: S = sum of the weights scaled by 2^-M (M the running maximum of their base-2
// logarithms), T = sum w t, N = sum w n, C = sum w c (same scale) and D = sum delta.  Writes
// depth = T/S (Eq. 3), alpha (Eq. 8), the unit normal, the flow to the second (and third)
// pose, the colour and the stash (M, 1/S, N/S, D, 0, 0).
template <int F>
__device__ __forceinline__ void write_ray(const Params &P, const FwdOut &O, int view, int r,
                                          const float *__restrict__ e, const float *__restrict__ kk, float o0,
                                          float o1, float o2, float v0, float v1, float v2, float M, float S,
                                          float T, float N0, float N1, float N2, float C0, float C1, float C2,
                                          float D, float alpha_t = 0.0f, float depth_t = 0.0f)
{
    constexpr bool NORMALS = (F & kNrm) != 0, FLOW = (F & kFlw) != 0, COLOR = (F & kCol) != 0;
    const size_t r3 = 3 * (size_t)r;  // per-ray offsets in 64 bits: 3 r overflows int above 7.2e8 rays
    const float invS = 1.0f / S;
    const float tf = T * invS;
    const float n0 = N0 * invS, n1 = N1 * invS, n2 = N2 * invS;
    const float alpha = -expm1f(-D);
    O.depth[r] = tf;
    O.alpha[r] = alpha;
    if (O.g_depth) {  // the targets alpha_t, depth_t of ray r, loaded by the caller
        float ga, gd;
        loss_grad_ray(alpha, alpha_t, tf, depth_t, O.w_depth, O.inv_p, ga, gd);
        O.g_alpha[r] = ga;
        O.g_depth[r] = gd;
    }
    if (NORMALS) {
        const float inn = 1.0f / sqrtf(fmaf(n0, n0, fmaf(n1, n1, fmaf(n2, n2, kEpsN))));
        O.normal[r3 + 0] = n0 * inn;
        O.normal[r3 + 1] = n1 * inn;
        O.normal[r3 + 2] = n2 * inn;
    }
    if (FLOW) {
        // flow to the second pose (and, if given, to a third: forward and backward flow)
        const float p0 = fmaf(tf, v0, o0), p1 = fmaf(tf, v1, o1), p2 = fmaf(tf, v2, o2);
        float ub, vb, ua, va;
        project(P.w2c_b + 12 * view, P.intr_b + 4 * view, p0, p1, p2, ub, vb);
        project(e, kk, p0, p1, p2, ua, va);
        const int fk = P.w2c_c ? 4 : 2;
        float *fl = O.flow + (size_t)fk * r;
        fl[0] = ub - ua;
        fl[1] = vb - va;
        if (P.w2c_c) {
            float uc, vc;
            project(P.w2c_c + 12 * view, P.intr_c + 4 * view, p0, p1, p2, uc, vc);
            fl[2] = uc - ua;
            fl[3] = vc - va;
        }
    }
    if (COLOR) {
        O.color[r3 + 0] = C0 * invS;
        O.color[r3 + 1] = C1 * invS;
        O.color[r3 + 2] = C2 * invS;
    }
    if (O.stash) {
        float4 *st = reinterpret_cast<float4 *>(O.stash) + 2 * (size_t)r;
        st[0] = make_float4(M, invS, n0, n1);
        st[1] = make_float4(n2, D, 0.0f, 0.0f);
    }
}

// ------------------------------------------------------------------------------------
// Adjoint helpers
// ------------------------------------------------------------------------------------

// g . d pi(p + t v)/dt at t = 0 for camera e (world-to-camera) and intrinsics k.
__device__ __forceinline__ float flow_dot(const float *__restrict__ e, const float *__restrict__ k, float p0,
                                          float p1, float p2, float v0, float v1, float v2,
                                          const float *__restrict__ g)
{
    const float q0 = fmaf(e[0], p0, fmaf(e[1], p1, fmaf(e[2], p2, e[3])));
    const float q1 = fmaf(e[4], p0, fmaf(e[5], p1, fmaf(e[6], p2, e[7])));
    const float q2 = fmaf(e[8], p0, fmaf(e[9], p1, fmaf(e[10], p2, e[11])));
    const float u0 = fmaf(e[0], v0, fmaf(e[1], v1, e[2] * v2));
    const float u1 = fmaf(e[4], v0, fmaf(e[5], v1, e[6] * v2));
    const float u2 = fmaf(e[8], v0, fmaf(e[9], v1, e[10] * v2));
    const float iz = 1.0f / q2;
    const float j0 = k[0] * (u0 - q0 * iz * u2) * iz;
    const float j1 = k[1] * (u1 - q1 * iz * u2) * iz;
    return fmaf(g[0], j0, g[1] * j1);
}

// Per-ray adjoint prologue:
//   (v0, v1, v2, M2) (invS, tf_bar, Nb0, Nb1) (Nb2, kappa, D_bar, t_f) (Cb0, Cb1, Cb2, dc)
// with tf_bar = dL/dt_f (depth + flow), Nb = dL/dN for the unnormalised blended normal,
// Cb = dL/dC for the blended colour, kappa = tf_bar t_f + Nb.N + Cb.C, and
// D_bar = dL/d(sum delta) = g_alpha exp(-D).  t_f and dc centre the blend-parameter sums: the
// softmax adjoints z_bar_i of a ray sum to zero, so sum z_bar_i (t_i - t_f) and
// sum z_bar_i (d2_i - dc) equal sum z_bar_i t_i and sum z_bar_i d2_i, without the rounding
// residual of sum z_bar_i times a large depth or log-density; dc = (M2 - nc2 t_f) / b1 is the
// log2 density of a Gaussian at depth t_f with the ray's largest weight (0 without b1).
template <int F>
__device__ __forceinline__ void ray_prologue(const Params &P, const BwdIn &I, int view, const ViewRec &vr,
                                             const float *__restrict__ e, const float *__restrict__ kk,
                                             const float o0, const float o1, const float o2, int local,
                                             bool valid, float b1, float nc2, float4 out[4])
{
    constexpr bool NORMALS = (F & kNrm) != 0, FLOW = (F & kFlw) != 0, COLOR = (F & kCol) != 0;
    if (!valid) {
        out[0] = make_float4(0.0f, 0.0f, 1.0f, INFINITY);
        out[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        out[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        out[3] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    float v0, v1, v2;
    ray_dir(P, vr, e, kk, local, v0, v1, v2);
    const int r = vr.ray_off + local;
    const size_t r3 = 3 * (size_t)r;  // 64-bit per-ray offsets (3 r overflows int above 7.2e8 rays)
    const float tf = I.depth[r];
    const float4 s0 = reinterpret_cast<const float4 *>(I.stash)[2 * (size_t)r];
    const float4 s1 = reinterpret_cast<const float4 *>(I.stash)[2 * (size_t)r + 1];
    const float Nx = s0.z, Ny = s0.w, Nz = s1.x, Dsum = s1.y;
    float tfb = I.g_depth ? I.g_depth[r] : 0.0f;
    if (FLOW) {
        // flow = pi_B(p) - pi_A(p), p = o + t_f v; pi_A(o + t v) does not depend on t, so
        // d flow / d t_f = J_B R_B v (and likewise for the optional third pose).
        const float p0 = fmaf(tf, v0, o0), p1 = fmaf(tf, v1, o1), p2 = fmaf(tf, v2, o2);
        const int fk = P.w2c_c ? 4 : 2;
        const float *gfl = I.g_flow + (size_t)fk * r;
        tfb += flow_dot(P.w2c_b + 12 * view, P.intr_b + 4 * view, p0, p1, p2, v0, v1, v2, gfl);
        if (P.w2c_c)
            tfb += flow_dot(P.w2c_c + 12 * view, P.intr_c + 4 * view, p0, p1, p2, v0, v1, v2, gfl + 2);
    }
    const float Db = I.g_alpha ? I.g_alpha[r] * expf(-Dsum) : 0.0f;
    float nb0 = 0.0f, nb1 = 0.0f, nb2 = 0.0f;
    if (NORMALS) {
        const float s = sqrtf(fmaf(Nx, Nx, fmaf(Ny, Ny, fmaf(Nz, Nz, kEpsN))));
        const float is = 1.0f / s;
        const float f0 = Nx * is, f1 = Ny * is, f2 = Nz * is;
        const float g0 = I.g_normal[r3], g1 = I.g_normal[r3 + 1], g2 = I.g_normal[r3 + 2];
        const float dp = fmaf(f0, g0, fmaf(f1, g1, f2 * g2));
        nb0 = (g0 - f0 * dp) * is;
        nb1 = (g1 - f1 * dp) * is;
        nb2 = (g2 - f2 * dp) * is;
    }
    float kap = fmaf(tfb, tf, fmaf(nb0, Nx, fmaf(nb1, Ny, nb2 * Nz)));
    float cb0 = 0.0f, cb1 = 0.0f, cb2 = 0.0f;
    if (COLOR) {
        cb0 = I.g_color[r3];
        cb1 = I.g_color[r3 + 1];
        cb2 = I.g_color[r3 + 2];
        kap = fmaf(cb0, I.color[r3], fmaf(cb1, I.color[r3 + 1], fmaf(cb2, I.color[r3 + 2], kap)));
    }
    float dc = (s0.x - nc2 * tf) * (1.0f / b1);
    if (!isfinite(dc)) dc = 0.0f;
    out[0] = make_float4(v0, v1, v2, s0.x);
    out[1] = make_float4(s0.y, tfb, nb0, nb1);
    out[2] = make_float4(nb2, kap, Db, tf);
    out[3] = make_float4(cb0, cb1, cb2, dc);
}

// Normal of Eq. (17) for one pair: g = U^T r = Sigma^-1 x, n = g / |g|, and n . Nb for the
// per-ray normal cotangent Nb.
struct PairNormal {
    float n0, n1, n2;  // unit normal
    float rs;          // 1 / |g|
    float nN;          // n . Nb
};

__device__ __forceinline__ PairNormal pair_normal(const Ent &g, const Geo &q, float nb0, float nb1, float nb2)
{
    const float g0 = g.u00 * q.r0;
    const float g1 = fmaf(g.u01, q.r0, g.u11 * q.r1);
    const float g2 = fmaf(g.u02, q.r0, fmaf(g.u12, q.r1, g.u22 * q.r2));
    PairNormal pn;
    pn.rs = rsq_(fmaf(g0, g0, fmaf(g1, g1, fmaf(g2, g2, kEpsN))));
    pn.n0 = g0 * pn.rs;
    pn.n1 = g1 * pn.rs;
    pn.n2 = g2 * pn.rs;
    pn.nN = fmaf(pn.n0, nb0, fmaf(pn.n1, nb1, pn.n2 * nb2));
    return pn;
}

// Per-Gaussian gradient accumulator of one lane: dL/dU (upper, without the -(sum rho) mu'^T
// term), sum rho = dL/d(U mu') and dL/dlog(lambda).
struct PairAcc {
    float u0 = 0, u1 = 0, u2 = 0, u3 = 0, u4 = 0, u5 = 0;
    float p0 = 0, p1 = 0, p2 = 0;
    float l = 0;
};

// Adjoint of one pair given tb = dL/dt_i (peak depth), db = dL/dd_i (log density) and the
// normal's cotangent wt * Nb.  r_bar = U g_bar - d_bar r with g_bar = wt (Nb - n (n.Nb)) / |g|;
// the peak-depth adjoint tau = (t_bar + a.r_bar) / (a.a) uses a.r = 0 at the peak, and
// rho = r_bar - tau a.  U_bar = sum r g_bar^T + rho w^T - tau r v^T with w = t v - mu' is
// accumulated as sum r g_bar^T + (t rho - tau r) v^T; the -(sum rho) mu'^T term is applied
// once per item.
template <bool NORMALS>
__device__ __forceinline__ void pair_adjoint(const Ent &g, const Geo &q, float v0, float v1, float v2, float wt,
                                             const PairNormal &pn, float nb0, float nb1, float nb2, float tb,
                                             float db, PairAcc &a)
{
    a.l += db;
    float gb0 = 0, gb1 = 0, gb2 = 0, ug0 = 0, ug1 = 0, ug2 = 0, tau;
    if (NORMALS) {
        const float ws = wt * pn.rs;
        gb0 = ws * fmaf(-pn.n0, pn.nN, nb0);
        gb1 = ws * fmaf(-pn.n1, pn.nN, nb1);
        gb2 = ws * fmaf(-pn.n2, pn.nN, nb2);
        ug0 = fmaf(g.u00, gb0, fmaf(g.u01, gb1, g.u02 * gb2));
        ug1 = fmaf(g.u11, gb1, g.u12 * gb2);
        ug2 = g.u22 * gb2;
        tau = fmaf(q.a0, ug0, fmaf(q.a1, ug1, fmaf(q.a2, ug2, tb))) * q.raa;
    } else {
        tau = tb * q.raa;
    }
    const float p0 = fmaf(-tau, q.a0, fmaf(-db, q.r0, ug0));
    const float p1 = fmaf(-tau, q.a1, fmaf(-db, q.r1, ug1));
    const float p2 = fmaf(-tau, q.a2, fmaf(-db, q.r2, ug2));
    const float k0 = fmaf(q.t, p0, -tau * q.r0);
    const float k1 = fmaf(q.t, p1, -tau * q.r1);
    const float k2 = fmaf(q.t, p2, -tau * q.r2);
    if (NORMALS) {
        a.u0 = fmaf(q.r0, gb0, a.u0);
        a.u1 = fmaf(q.r0, gb1, a.u1);
        a.u2 = fmaf(q.r0, gb2, a.u2);
        a.u3 = fmaf(q.r1, gb1, a.u3);
        a.u4 = fmaf(q.r1, gb2, a.u4);
        a.u5 = fmaf(q.r2, gb2, a.u5);
    }
    a.u0 = fmaf(k0, v0, a.u0);
    a.u1 = fmaf(k0, v1, a.u1);
    a.u2 = fmaf(k0, v2, a.u2);
    a.u3 = fmaf(k1, v1, a.u3);
    a.u4 = fmaf(k1, v2, a.u4);
    a.u5 = fmaf(k2, v2, a.u5);
    a.p0 += p0;
    a.p1 += p1;
    a.p2 += p2;
}

// Adjoint of one pair without a normal cotangent, summed in terms of the peak's offset from the
// mean.  With w = t v - mu' (the peak point relative to the mean, r = U w), tau = tb / (a.a) and
// rho = -tau a - db r (the general adjoint with no normal term), the pair adds
//   rho w^T - tau r v^T = U X,   X = -tau (w v^T + v w^T) - db w w^T = -(h w^T + w h^T),
//   h = tau v + (db / 2) w,
// to dL/dU, and -U (tau v + db w) = U (db mu' - beta v), beta = tau + db t, to sum rho.  A lane
// therefore sums H = sum h w^T (9), Bv = sum beta v (3) and L = sum db, and write_partial_offset
// forms dU = -U (H + H^T) and sum rho = L U mu' - U Bv once per (item, Gaussian) in double.
// Every summand of H is of the size of the pair's own contribution.  Expanding w w^T into monomials
// of v instead (the same sums over A = sum alpha v v^T, Bv and L with alpha = -t (2 tau + db t),
// the record U A + b Bv^T - (L b - U Bv) mu'^T, b = U mu') is fewer operations per pair but cancels
// by (|mu'| / |w|)^2 ~ |b|^2 / |r|^2: for Gaussians a few thousandths wide seen from a few units
// away its FP32 sums leave errors of 1e-3 of dL/dU.  Sum rho cancels only linearly (|mu'| / |w|).  The envelope
// condition a.r = 0 enters only through terms of relative size |t - t_peak| |a| / |r|, so neither
// t nor r needs the Newton step, and w is the high part t v - hi (the low part of mu' is below
// 2^-24 |mu'|).
struct OffsetAcc {
    float h00 = 0, h01 = 0, h02 = 0, h10 = 0, h11 = 0, h12 = 0, h20 = 0, h21 = 0, h22 = 0;
    float b0 = 0, b1 = 0, b2 = 0;
    float l = 0;
};
constexpr int kOffsetAcc = 13;  // floats of an OffsetAcc

__device__ __forceinline__ void pair_adjoint_offset(const Geo &q, float v0, float v1, float v2, float tb, float db,
                                                    OffsetAcc &a)
{
    const float tau = tb * q.raa;
    const float dh = 0.5f * db;
    const float h0 = fmaf(tau, v0, dh * q.w0);
    const float h1 = fmaf(tau, v1, dh * q.w1);
    const float h2 = fmaf(tau, v2, dh * q.w2);
    a.h00 = fmaf(h0, q.w0, a.h00);
    a.h01 = fmaf(h0, q.w1, a.h01);
    a.h02 = fmaf(h0, q.w2, a.h02);
    a.h10 = fmaf(h1, q.w0, a.h10);
    a.h11 = fmaf(h1, q.w1, a.h11);
    a.h12 = fmaf(h1, q.w2, a.h12);
    a.h20 = fmaf(h2, q.w0, a.h20);
    a.h21 = fmaf(h2, q.w1, a.h21);
    a.h22 = fmaf(h2, q.w2, a.h22);
    const float be = fmaf(db, q.t, tau);
    a.b0 = fmaf(be, v0, a.b0);
    a.b1 = fmaf(be, v1, a.b1);
    a.b2 = fmaf(be, v2, a.b2);
    a.l += db;
}

__device__ __forceinline__ void offset_acc_store(const OffsetAcc &a, float *my)
{
    my[0] = a.h00; my[1] = a.h01; my[2] = a.h02; my[3] = a.h10; my[4] = a.h11; my[5] = a.h12;
    my[6] = a.h20; my[7] = a.h21; my[8] = a.h22; my[9] = a.b0; my[10] = a.b1; my[11] = a.b2; my[12] = a.l;
}

// Partial record of one Gaussian from the sums (H, Bv, L) of pair_adjoint_offset (acc[0..12]), in
// double: dU = U X with X = -(H + H^T) (upper triangle), sum rho = L b - U Bv with b = U mu',
// dL/dlog(lambda) = L, then the remaining values (colour, acc[13..]) as given.
__device__ __forceinline__ void write_partial_offset(float *__restrict__ dst, const float *acc, int rec,
                                                     const float *__restrict__ prec, const float *__restrict__ mu,
                                                     const double o[3])
{
    const double u00 = prec[0], u01 = prec[1], u02 = prec[2], u11 = prec[3], u12 = prec[4], u22 = prec[5];
    const double m0 = (double)mu[0] - o[0], m1 = (double)mu[1] - o[1], m2 = (double)mu[2] - o[2];
    const double X00 = -2.0 * (double)acc[0], X11 = -2.0 * (double)acc[4], X22 = -2.0 * (double)acc[8];
    const double X01 = -((double)acc[1] + (double)acc[3]);
    const double X02 = -((double)acc[2] + (double)acc[6]);
    const double X12 = -((double)acc[5] + (double)acc[7]);
    const double B0 = acc[9], B1 = acc[10], B2 = acc[11], L = acc[12];
    const double b0 = u00 * m0 + u01 * m1 + u02 * m2, b1 = u11 * m1 + u12 * m2, b2 = u22 * m2;
    dst[0] = (float)(u00 * X00 + u01 * X01 + u02 * X02);
    dst[1] = (float)(u00 * X01 + u01 * X11 + u02 * X12);
    dst[2] = (float)(u00 * X02 + u01 * X12 + u02 * X22);
    dst[3] = (float)(u11 * X11 + u12 * X12);
    dst[4] = (float)(u11 * X12 + u12 * X22);
    dst[5] = (float)(u22 * X22);
    dst[6] = (float)(L * b0 - (u00 * B0 + u01 * B1 + u02 * B2));
    dst[7] = (float)(L * b1 - (u11 * B1 + u12 * B2));
    dst[8] = (float)(L * b2 - u22 * B2);
    dst[9] = (float)L;
    for (int c = 10; c < rec; ++c) dst[c] = acc[c + kOffsetAcc - 10];
}

// Write one Gaussian's partial record: dU with the -(sum rho) mu'^T term applied in double
// (mu' = mu - o), then sum rho, dL/dlog(lambda) and the remaining values as given.
__device__ __forceinline__ void write_partial(float *__restrict__ dst, const float *acc, int rec,
                                              const float *__restrict__ mu, const double o[3])
{
    const double m0 = (double)mu[0] - o[0], m1 = (double)mu[1] - o[1], m2 = (double)mu[2] - o[2];
    const double r0 = acc[6], r1 = acc[7], r2 = acc[8];
    dst[0] = (float)((double)acc[0] - r0 * m0);
    dst[1] = (float)((double)acc[1] - r0 * m1);
    dst[2] = (float)((double)acc[2] - r0 * m2);
    dst[3] = (float)((double)acc[3] - r1 * m1);
    dst[4] = (float)((double)acc[4] - r1 * m2);
    dst[5] = (float)((double)acc[5] - r2 * m2);
    for (int c = 6; c < rec; ++c) dst[c] = acc[c];
}

// Sum over the wave of 16 values, scattered: halving exchanges between lanes 32, 16, 8 and 4 apart
// (each lane keeps half of its values and adds its partner's copy of that half), then a sum over
// groups of 4 lanes.  Lane l ends with the total of value wave16_index(l); the order of the
// additions is fixed.  The first two exchanges are gfx950's permlane32/permlane16 swaps (the upper
// half of one register trades places with the lower half of another, so one instruction serves two
// values and no lane select is needed); the rest are DPP moves within rows: rotation by 8, the
// mirror of each half-row (any pairing across the two halves serves a sum), then the quad.
__device__ __forceinline__ int wave16_index(int lane)
{
    return ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum16(const float x[16], int lane)
{
    float y[8], z[4], u[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[i]), __float_as_uint(x[i + 8]), false, false);
        y[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(y[i]), __float_as_uint(y[i + 4]), false, false);
        z[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    bool up = (lane & 8) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) u[i] = (up ? z[i + 2] : z[i]) + dpp_mov<0x128>(up ? z[i] : z[i + 2]);  // row_ror:8
    up = (lane & 4) != 0;
    float s = (up ? u[1] : u[0]) + dpp_mov<0x141>(up ? u[0] : u[1]);  // row_half_mirror
    s += dpp_mov<0x4E>(s);  // quad_perm [2, 3, 0, 1]
    s += dpp_mov<0xB1>(s);  // quad_perm [1, 0, 3, 2]
    return s;
}

}  // namespace fmb
