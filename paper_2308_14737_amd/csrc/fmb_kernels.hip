// fmb_kernels.hip -- gfx950 kernels of the sort-free two-parameter Fuzzy Metaballs
// renderer (Keselman & Hebert, WACV 2024, Sec. 3.1-3.2, 5, 6).
//
// Layout of the work (see fmb_internal.h):
//   * forward: one lane per ray (RPT rays per lane), Gaussians staged through LDS in
//     tiles of TG; each (view, Gaussian) entry is formed on the fly in FP64 when the
//     tile is loaded (mean relative to the camera centre as a float hi/lo pair, the
//     precision-weighted mean c = Sigma^-1 (mu - o), log2 lambda).  The softmax of the
//     blend weights (Eq. 7 in Eq. 3) runs online in FP32 registers in base 2.
//   * backward: one lane per (Gaussian, ray slot); rays of the item's span are staged
//     through LDS with their per-ray adjoint prologue; every lane recomputes its pairs
//     and accumulates its Gaussian's gradient in registers -- no per-pair cross-lane
//     reduction and no P x N storage.  Partial gradients per item are reduced
//     deterministically by the finalize kernel.
//   * persistent variants pull items from a device counter (reset by a fill kernel)
//     in the order given by the host (largest item first).
//
// Per pair (ray o + t v with |v| = 1, Gaussian mu, U, lambda; mu' = mu - o):
//   a = U v, t = v.c / a.a (peak of the density along the ray, Sec. 3.1),
//   r = U (t v - mu') formed as U (t v - hi) - U lo, one Newton refinement of t on
//   |U(t v - mu')|^2, m = r.r, d = log lambda - m/2 (Eq. 2), delta = e^d (Eq. 4),
//   z = beta1 d - (beta2/eta) t (log of Eq. 7), g = U^T r = Sigma^-1 x (Eq. 17).
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

// Camera centre o = -R^T T in double.
__device__ __forceinline__ void cam_centre(const float *__restrict__ e, double o[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
        o[a] = -((double)e[a] * (double)e[3] + (double)e[4 + a] * (double)e[7] +
                 (double)e[8 + a] * (double)e[11]);
}

// (view, Gaussian) entry in double, rounded to float.  mu - o is split as hi + lo; the
// pair loop forms U (t v - mu') as U (t v - hi) - U lo, so only U lo is stored.
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
    out[3] = make_float4((float)c0, (float)c1, (float)c2, (float)log2((double)lam));
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
    float t;                // refined peak depth
    float r0, r1, r2;       // r = U (t v - mu')
    float d2, z2;           // log2 density, log2 blend weight
};

__device__ __forceinline__ void pair_geo(const Ent &g, float v0, float v1, float v2, float hm, float b1,
                                         float nc2, Geo &q)
{
    q.a0 = fmaf(g.u00, v0, fmaf(g.u01, v1, g.u02 * v2));
    q.a1 = fmaf(g.u11, v1, g.u12 * v2);
    q.a2 = g.u22 * v2;
    const float aa = fmaf(q.a0, q.a0, fmaf(q.a1, q.a1, q.a2 * q.a2));
    const float vc = fmaf(v0, g.c0, fmaf(v1, g.c1, v2 * g.c2));
    q.raa = rcp_(aa);
    const float t0 = vc * q.raa;
    const float w0 = fmaf(t0, v0, -g.mh0);
    const float w1 = fmaf(t0, v1, -g.mh1);
    const float w2 = fmaf(t0, v2, -g.mh2);
    const float r0 = fmaf(g.u00, w0, fmaf(g.u01, w1, fmaf(g.u02, w2, -g.ul0)));
    const float r1 = fmaf(g.u11, w1, fmaf(g.u12, w2, -g.ul1));
    const float r2 = fmaf(g.u22, w2, -g.ul2);
    // one Newton step on t -> |U (t v - mu')|^2 (exactly quadratic): dt = (a.r)/(a.a)
    const float dt = fmaf(q.a0, r0, fmaf(q.a1, r1, q.a2 * r2)) * q.raa;
    q.t = t0 - dt;
    q.r0 = fmaf(-dt, q.a0, r0);
    q.r1 = fmaf(-dt, q.a1, r1);
    q.r2 = fmaf(-dt, q.a2, r2);
    const float m = fmaf(q.r0, q.r0, fmaf(q.r1, q.r1, q.r2 * q.r2));
    q.d2 = fmaf(hm, m, g.l2l);
    q.z2 = fmaf(b1, q.d2, nc2 * q.t);
}

// Per-item blend constants of a scene: hm = -log2(e)/2, b1 = beta1, nc2 = -beta2 log2(e)/eta.
struct Blend {
    float hm, b1, nc2, cb;  // cb = beta2 / eta (natural units, backward)
    float inv_eta;
};

__device__ __forceinline__ Blend blend_of(const Params &P, int s)
{
    const double b1 = P.betas[2 * s], b2 = P.betas[2 * s + 1], eta = P.eta[s];
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

// Colour of a Gaussian: sigmoid of the unconstrained parameters (double, rounded).
__device__ __forceinline__ float4 colour_entry(const float *__restrict__ q)
{
    return make_float4((float)(1.0 / (1.0 + exp(-(double)q[0]))), (float)(1.0 / (1.0 + exp(-(double)q[1]))),
                       (float)(1.0 / (1.0 + exp(-(double)q[2]))), 0.0f);
}

// ------------------------------------------------------------------------------------
// Forward
// ------------------------------------------------------------------------------------

template <int BLOCK, int RPT, int TG, int F>
__global__ __launch_bounds__(BLOCK) void fwd_kernel(Params P, FwdOut O, const FwdItem *__restrict__ items,
                                                   int n_items, const int *__restrict__ order,
                                                   int *__restrict__ counter)
{
    constexpr bool NORMALS = (F & kNrm) != 0, FLOW = (F & kFlw) != 0, PERSIST = (F & kPer) != 0;
    constexpr bool COLOR = (F & kCol) != 0;
    constexpr int EW = COLOR ? 5 : 4;  // float4 per LDS entry
    __shared__ float4 tile[TG * EW];
    __shared__ int s_item;
    int pos = blockIdx.x;
    for (;;) {
        if (PERSIST) {
            __syncthreads();  // everyone is done with s_item and the tile of the last item
            if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
            __syncthreads();
            pos = s_item;
        }
        if (pos >= n_items) break;
        const int it = order ? order[pos] : pos;
        const FwdItem item = items[it];
        const ViewRec vr = P.views[item.view];
        const SceneRec sr = P.scenes[vr.scene];
        const float *__restrict__ e = P.w2c + 12 * item.view;
        const float *__restrict__ kk = P.intr + 4 * item.view;
        double o[3];
        cam_centre(e, o);
        const Blend bl = blend_of(P, vr.scene);
        const int hw = vr.h * vr.w;

        float v0[RPT], v1[RPT], v2[RPT];
        float M[RPT], S[RPT], T[RPT], N0[RPT], N1[RPT], N2[RPT], D[RPT], C0[RPT], C1[RPT], C2[RPT];
        int loc[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            loc[j] = item.ray0 + (int)threadIdx.x + j * BLOCK;
            const int lc = loc[j] < hw ? loc[j] : hw - 1;
            ray_dir(P, vr, e, kk, lc, v0[j], v1[j], v2[j]);
            M[j] = -INFINITY;
            S[j] = T[j] = N0[j] = N1[j] = N2[j] = D[j] = C0[j] = C1[j] = C2[j] = 0.0f;
        }

        for (int gb = 0; gb < sr.n; gb += TG) {
            const int cnt = min(TG, sr.n - gb);
            if (gb > 0 || !PERSIST) __syncthreads();
            for (int q = threadIdx.x; q < cnt; q += BLOCK) {
                const int gi = sr.gauss_off + gb + q;
                make_entry(P.means + 3 * gi, P.prec + 6 * gi, P.weights[gi], o, &tile[EW * q]);
                if (COLOR) tile[EW * q + 4] = colour_entry(P.colors + 3 * gi);
            }
            __syncthreads();
#pragma unroll 2
            for (int i = 0; i < cnt; ++i) {
                const Ent g = ent_from(tile[EW * i], tile[EW * i + 1], tile[EW * i + 2], tile[EW * i + 3]);
                float4 cc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (COLOR) cc = tile[EW * i + 4];
#pragma unroll
                for (int j = 0; j < RPT; ++j) {
                    Geo q;
                    pair_geo(g, v0[j], v1[j], v2[j], bl.hm, bl.b1, bl.nc2, q);
                    const float delta = exp2_(q.d2);
                    if (q.z2 > M[j]) {  // new running maximum: rescale the sums (rare)
                        const float sc = exp2_(M[j] - q.z2);
                        S[j] *= sc;
                        T[j] *= sc;
                        if (NORMALS) {
                            N0[j] *= sc;
                            N1[j] *= sc;
                            N2[j] *= sc;
                        }
                        if (COLOR) {
                            C0[j] *= sc;
                            C1[j] *= sc;
                            C2[j] *= sc;
                        }
                        M[j] = q.z2;
                    }
                    const float ew = exp2_(q.z2 - M[j]);
                    S[j] += ew;
                    T[j] = fmaf(ew, q.t, T[j]);
                    D[j] += delta;
                    if (NORMALS) {
                        const float g0 = g.u00 * q.r0;
                        const float g1 = fmaf(g.u01, q.r0, g.u11 * q.r1);
                        const float g2 = fmaf(g.u02, q.r0, fmaf(g.u12, q.r1, g.u22 * q.r2));
                        const float es = ew * rsq_(fmaf(g0, g0, fmaf(g1, g1, fmaf(g2, g2, kEpsN))));
                        N0[j] = fmaf(es, g0, N0[j]);
                        N1[j] = fmaf(es, g1, N1[j]);
                        N2[j] = fmaf(es, g2, N2[j]);
                    }
                    if (COLOR) {
                        C0[j] = fmaf(ew, cc.x, C0[j]);
                        C1[j] = fmaf(ew, cc.y, C1[j]);
                        C2[j] = fmaf(ew, cc.z, C2[j]);
                    }
                }
            }
        }

        const float o0 = (float)o[0], o1 = (float)o[1], o2 = (float)o[2];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            if (loc[j] >= hw) continue;
            const int r = vr.ray_off + loc[j];
            const float invS = 1.0f / S[j];
            const float tf = T[j] * invS;
            const float n0 = N0[j] * invS, n1 = N1[j] * invS, n2 = N2[j] * invS;
            O.depth[r] = tf;
            O.alpha[r] = -expm1f(-D[j]);
            if (NORMALS) {
                const float inn = 1.0f / sqrtf(fmaf(n0, n0, fmaf(n1, n1, fmaf(n2, n2, kEpsN))));
                O.normal[3 * r + 0] = n0 * inn;
                O.normal[3 * r + 1] = n1 * inn;
                O.normal[3 * r + 2] = n2 * inn;
            }
            if (FLOW) {
                // flow to the second pose (and, if given, to a third: forward and backward flow)
                const float p0 = fmaf(tf, v0[j], o0), p1 = fmaf(tf, v1[j], o1), p2 = fmaf(tf, v2[j], o2);
                float ub, vb, ua, va;
                project(P.w2c_b + 12 * item.view, P.intr_b + 4 * item.view, p0, p1, p2, ub, vb);
                project(e, kk, p0, p1, p2, ua, va);
                const int fk = P.w2c_c ? 4 : 2;
                O.flow[fk * r + 0] = ub - ua;
                O.flow[fk * r + 1] = vb - va;
                if (P.w2c_c) {
                    float uc, vc;
                    project(P.w2c_c + 12 * item.view, P.intr_c + 4 * item.view, p0, p1, p2, uc, vc);
                    O.flow[fk * r + 2] = uc - ua;
                    O.flow[fk * r + 3] = vc - va;
                }
            }
            if (COLOR) {
                O.color[3 * r + 0] = C0[j] * invS;
                O.color[3 * r + 1] = C1[j] * invS;
                O.color[3 * r + 2] = C2[j] * invS;
            }
            if (O.stash) {
                float4 *st = reinterpret_cast<float4 *>(O.stash) + 2 * (size_t)r;
                st[0] = make_float4(M[j], invS, n0, n1);
                st[1] = make_float4(n2, D[j], 0.0f, 0.0f);
            }
        }
        if (!PERSIST) break;
    }
}

// ------------------------------------------------------------------------------------
// Backward
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

// Per-ray adjoint prologue, staged in LDS as RW float4:
//   (v0, v1, v2, M2) (invS, tf_bar, Nb0, Nb1) (Nb2, kappa, D_bar, 0) [(Cb0, Cb1, Cb2, 0)]
// with tf_bar = dL/dt_f (depth + flow), Nb = dL/dN for the unnormalised blended normal,
// Cb = dL/dC for the blended colour, kappa = tf_bar t_f + Nb.N + Cb.C, and
// D_bar = dL/d(sum delta) = g_alpha exp(-D).
template <int F>
__device__ __forceinline__ void ray_prologue(const Params &P, const BwdIn &I, int view, const ViewRec &vr,
                                             const float *__restrict__ e, const float *__restrict__ kk,
                                             const float o0, const float o1, const float o2, int local,
                                             bool valid, float4 out[4])
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
        tfb += flow_dot(P.w2c_b + 12 * view, P.intr_b + 4 * view, p0, p1, p2, v0, v1, v2, I.g_flow + fk * r);
        if (P.w2c_c)
            tfb += flow_dot(P.w2c_c + 12 * view, P.intr_c + 4 * view, p0, p1, p2, v0, v1, v2, I.g_flow + fk * r + 2);
    }
    const float Db = I.g_alpha ? I.g_alpha[r] * expf(-Dsum) : 0.0f;
    float nb0 = 0.0f, nb1 = 0.0f, nb2 = 0.0f;
    if (NORMALS) {
        const float s = sqrtf(fmaf(Nx, Nx, fmaf(Ny, Ny, fmaf(Nz, Nz, kEpsN))));
        const float is = 1.0f / s;
        const float f0 = Nx * is, f1 = Ny * is, f2 = Nz * is;
        const float g0 = I.g_normal[3 * r], g1 = I.g_normal[3 * r + 1], g2 = I.g_normal[3 * r + 2];
        const float dp = fmaf(f0, g0, fmaf(f1, g1, f2 * g2));
        nb0 = (g0 - f0 * dp) * is;
        nb1 = (g1 - f1 * dp) * is;
        nb2 = (g2 - f2 * dp) * is;
    }
    float kap = fmaf(tfb, tf, fmaf(nb0, Nx, fmaf(nb1, Ny, nb2 * Nz)));
    float cb0 = 0.0f, cb1 = 0.0f, cb2 = 0.0f;
    if (COLOR) {
        cb0 = I.g_color[3 * r];
        cb1 = I.g_color[3 * r + 1];
        cb2 = I.g_color[3 * r + 2];
        kap = fmaf(cb0, I.color[3 * r], fmaf(cb1, I.color[3 * r + 1], fmaf(cb2, I.color[3 * r + 2], kap)));
    }
    out[0] = make_float4(v0, v1, v2, s0.x);
    out[1] = make_float4(s0.y, tfb, nb0, nb1);
    out[2] = make_float4(nb2, kap, Db, 0.0f);
    out[3] = make_float4(cb0, cb1, cb2, 0.0f);
}

template <int BLOCK, int RT, int F>
__global__ __launch_bounds__(BLOCK) void bwd_kernel(Params P, BwdIn I, const BwdItem *__restrict__ items,
                                                   int n_items, const int *__restrict__ order,
                                                   int *__restrict__ counter, float *__restrict__ partial,
                                                   float *__restrict__ beta_partial)
{
    constexpr bool NORMALS = (F & kNrm) != 0, PERSIST = (F & kPer) != 0, COLOR = (F & kCol) != 0;
    constexpr int RW = COLOR ? 4 : 3;             // float4 per staged ray
    constexpr int REC = COLOR ? kPartialColor : kPartial;  // partial record per Gaussian
    constexpr int RS = REC + 2;                   // reduction record per lane (+ two betas)
    __shared__ float4 rays[RT * RW];
    __shared__ float red[BLOCK * RS];
    __shared__ int s_item;
    int pos = blockIdx.x;
    const int tid = threadIdx.x;
    for (;;) {
        if (PERSIST) {
            __syncthreads();
            if (tid == 0) s_item = atomicAdd(counter, 1);
            __syncthreads();
            pos = s_item;
        }
        if (pos >= n_items) break;
        const int it = order ? order[pos] : pos;
        const BwdItem item = items[it];
        const ViewRec vr = P.views[item.view];
        const SceneRec sr = P.scenes[vr.scene];
        const float *__restrict__ e = P.w2c + 12 * item.view;
        const float *__restrict__ kk = P.intr + 4 * item.view;
        double o[3];
        cam_centre(e, o);
        const float o0 = (float)o[0], o1 = (float)o[1], o2 = (float)o[2];
        const Blend bl = blend_of(P, vr.scene);
        const int hw = vr.h * vr.w;
        const int end = min(item.ray0 + item.span, hw);

        const int gi = tid % item.gc;
        const int slot = tid / item.gc;
        const bool active = slot < item.slots && item.g0 + gi < sr.n;
        Ent g;
        float4 cc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (active) {
            const int gg = sr.gauss_off + item.g0 + gi;
            float4 q[4];
            make_entry(P.means + 3 * gg, P.prec + 6 * gg, P.weights[gg], o, q);
            g = ent_from(q[0], q[1], q[2], q[3]);
            if (COLOR) cc = colour_entry(P.colors + 3 * gg);
        }
        float aU0 = 0, aU1 = 0, aU2 = 0, aU3 = 0, aU4 = 0, aU5 = 0;
        float aP0 = 0, aP1 = 0, aP2 = 0, aL = 0, aB1 = 0, aB2 = 0;
        float aC0 = 0, aC1 = 0, aC2 = 0;

        for (int r0 = item.ray0; r0 < end; r0 += RT) {
            const int cnt = min(RT, end - r0);
            __syncthreads();
            for (int q = tid; q < RT; q += BLOCK) {
                float4 pr[4];
                ray_prologue<F>(P, I, item.view, vr, e, kk, o0, o1, o2, r0 + q, q < cnt, pr);
#pragma unroll
                for (int k = 0; k < RW; ++k) rays[RW * q + k] = pr[k];
            }
            __syncthreads();
            if (active) {
                for (int j = slot; j < cnt; j += item.slots) {
                    const float4 x0 = rays[RW * j], x1 = rays[RW * j + 1], x2 = rays[RW * j + 2];
                    float4 x3 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (COLOR) x3 = rays[RW * j + 3];
                    const float v0 = x0.x, v1 = x0.y, v2 = x0.z;
                    Geo q;
                    pair_geo(g, v0, v1, v2, bl.hm, bl.b1, bl.nc2, q);
                    const float delta = exp2_(q.d2);
                    const float wt = exp2_(q.z2 - x0.w) * x1.x;   // normalised blend weight
                    const float tfb = x1.y;
                    // recompute the normal of Eq. (17)
                    float n0 = 0, n1 = 0, n2 = 0, rs = 0, nN = 0;
                    float g0 = 0, g1 = 0, g2 = 0;
                    if (NORMALS) {
                        g0 = g.u00 * q.r0;
                        g1 = fmaf(g.u01, q.r0, g.u11 * q.r1);
                        g2 = fmaf(g.u02, q.r0, fmaf(g.u12, q.r1, g.u22 * q.r2));
                        rs = rsq_(fmaf(g0, g0, fmaf(g1, g1, fmaf(g2, g2, kEpsN))));
                        n0 = g0 * rs;
                        n1 = g1 * rs;
                        n2 = g2 * rs;
                        nN = fmaf(n0, x1.z, fmaf(n1, x1.w, n2 * x2.x));
                    }
                    // softmax adjoint: z_bar = wt (tf_bar t + Nb.n + Cb.c - kappa)
                    float lin = fmaf(tfb, q.t, nN);
                    if (COLOR) {
                        lin = fmaf(x3.x, cc.x, fmaf(x3.y, cc.y, fmaf(x3.z, cc.z, lin)));
                        aC0 = fmaf(wt, x3.x, aC0);
                        aC1 = fmaf(wt, x3.y, aC1);
                        aC2 = fmaf(wt, x3.z, aC2);
                    }
                    const float zb = wt * (lin - x2.y);
                    const float tb = fmaf(-bl.cb, zb, wt * tfb);
                    const float db = fmaf(bl.b1, zb, x2.z * delta);
                    aB1 = fmaf(zb, q.d2, aB1);
                    aB2 = fmaf(zb, q.t, aB2);
                    aL += db;
                    // r_bar = U g_bar - d_bar r with g_bar = wt (Nb - n (n.Nb)) / |g|; the peak-depth
                    // adjoint tau = (t_bar + a.r_bar) / (a.a) uses a.r = 0 at the peak, and
                    // rho = r_bar - tau a.  U_bar = sum r g_bar^T + rho w^T - tau r v^T with
                    // w = t v - mu' is accumulated as sum r g_bar^T + (t rho - tau r) v^T; the
                    // -(sum rho) mu'^T term is applied once per item.
                    float gb0 = 0, gb1 = 0, gb2 = 0, ug0 = 0, ug1 = 0, ug2 = 0, tau;
                    if (NORMALS) {
                        const float ws = wt * rs;
                        gb0 = ws * fmaf(-n0, nN, x1.z);
                        gb1 = ws * fmaf(-n1, nN, x1.w);
                        gb2 = ws * fmaf(-n2, nN, x2.x);
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
                        aU0 = fmaf(q.r0, gb0, aU0);
                        aU1 = fmaf(q.r0, gb1, aU1);
                        aU2 = fmaf(q.r0, gb2, aU2);
                        aU3 = fmaf(q.r1, gb1, aU3);
                        aU4 = fmaf(q.r1, gb2, aU4);
                        aU5 = fmaf(q.r2, gb2, aU5);
                    }
                    aU0 = fmaf(k0, v0, aU0);
                    aU1 = fmaf(k0, v1, aU1);
                    aU2 = fmaf(k0, v2, aU2);
                    aU3 = fmaf(k1, v1, aU3);
                    aU4 = fmaf(k1, v2, aU4);
                    aU5 = fmaf(k2, v2, aU5);
                    aP0 += p0;
                    aP1 += p1;
                    aP2 += p2;
                }
            }
        }

        // deterministic block reduction: Gaussian partials over the slots, betas over all lanes
        __syncthreads();
        {
            float *my = red + RS * tid;
            my[0] = aU0; my[1] = aU1; my[2] = aU2; my[3] = aU3; my[4] = aU4; my[5] = aU5;
            my[6] = aP0; my[7] = aP1; my[8] = aP2; my[9] = aL;
            if (COLOR) {
                my[10] = aC0; my[11] = aC1; my[12] = aC2;
            }
            my[REC] = aB1; my[REC + 1] = aB2;
        }
        __syncthreads();
        if (slot == 0 && gi < item.gc && item.g0 + gi < sr.n) {
            float acc[REC];
#pragma unroll
            for (int c = 0; c < REC; ++c) acc[c] = red[RS * gi + c];
            for (int s = 1; s < item.slots; ++s) {
#pragma unroll
                for (int c = 0; c < REC; ++c) acc[c] += red[RS * (s * item.gc + gi) + c];
            }
            // U_bar -= (sum rho) mu'^T (upper triangle), mu' = mu - o in double
            const float *mu = P.means + 3 * (sr.gauss_off + item.g0 + gi);
            const double m0 = (double)mu[0] - o[0], m1 = (double)mu[1] - o[1], m2 = (double)mu[2] - o[2];
            const double r0 = acc[6], r1 = acc[7], r2 = acc[8];
            float *dst = partial + item.poff + REC * gi;
            dst[0] = (float)((double)acc[0] - r0 * m0);
            dst[1] = (float)((double)acc[1] - r0 * m1);
            dst[2] = (float)((double)acc[2] - r0 * m2);
            dst[3] = (float)((double)acc[3] - r1 * m1);
            dst[4] = (float)((double)acc[4] - r1 * m2);
            dst[5] = (float)((double)acc[5] - r2 * m2);
#pragma unroll
            for (int c = 6; c < REC; ++c) dst[c] = acc[c];
        }
        if (tid < 64) {
            // lane l sums lanes l, l+64, ... in order, then a fixed butterfly over the wave
            float s1 = 0.0f, s2 = 0.0f;
            for (int k = tid; k < BLOCK; k += 64) {
                s1 += red[RS * k + REC];
                s2 += red[RS * k + REC + 1];
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                s1 += __shfl_xor(s1, off, 64);
                s2 += __shfl_xor(s2, off, 64);
            }
            if (tid == 0) {
                beta_partial[2 * item.seq] = s1;
                beta_partial[2 * item.seq + 1] = s2;
            }
        }
        if (!PERSIST) break;
    }
}

// ------------------------------------------------------------------------------------
// Finalize, in two deterministic stages.
//   stage 1: each group of <= kGroupItems consecutive items of a chunk is summed in item
//            order in FP64 (all values of the chunk's partial record, and the betas);
//   stage 2: each chunk sums its groups in order, maps the peak-depth adjoint to the means
//            (dL/dmu = -U^T sum rho), the log-weight adjoint to the weights
//            (dL/dlambda = dL/dlog(lambda) / lambda), and the first chunk of a scene
//            reduces the scene's betas.
// ------------------------------------------------------------------------------------

// Sum n strided values src[0], src[stride], ... in index order (FP64), issuing the loads
// eight at a time so that they are in flight together; the association is fixed.
template <typename T>
__device__ __forceinline__ double ordered_sum(const T *__restrict__ src, int n, int stride)
{
    double s = 0.0;
    int i = 0;
    for (; i + 8 <= n; i += 8) {
        T x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = src[(size_t)(i + k) * stride];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += (double)x[k];
    }
    for (; i < n; ++i) s += (double)src[(size_t)i * stride];
    return s;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void fin1_kernel(const FinGroup *__restrict__ groups,
                                                    const float *__restrict__ partial,
                                                    const float *__restrict__ beta_partial,
                                                    double *__restrict__ stage, double *__restrict__ stage_beta)
{
    const FinGroup gr = groups[blockIdx.x];
    const int tid = threadIdx.x;
    const int n = gr.item_end - gr.item_begin;
    for (int v = tid; v < gr.nval; v += BLOCK) stage[gr.soff + v] = ordered_sum(partial + gr.poff + v, n, gr.nval);
    if (tid < 2) stage_beta[2 * blockIdx.x + tid] = ordered_sum(beta_partial + 2 * gr.item_begin + tid, n, 2);
}

// Second stage: block (task, slice) finishes kFinSlice Gaussians of a chunk.
constexpr int kFinSlice = 25;

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void fin2_kernel(Params P, const FinTask *__restrict__ tasks,
                                                    const FinGroup *__restrict__ groups,
                                                    const double *__restrict__ stage,
                                                    const double *__restrict__ stage_beta,
                                                    float *__restrict__ g_means, float *__restrict__ g_prec,
                                                    float *__restrict__ g_weights, float *__restrict__ g_colors,
                                                    float *__restrict__ g_betas)
{
    __shared__ double sums[kFinSlice * kPartialColor];
    const FinTask task = tasks[blockIdx.x];
    const int g_lo = blockIdx.y * kFinSlice;
    if (g_lo >= task.gc) return;
    const int ng = min(kFinSlice, task.gc - g_lo);
    const int rec = task.rec;
    const SceneRec sr = P.scenes[task.scene];
    const int tid = threadIdx.x;
    for (int tv = tid; tv < ng * rec; tv += BLOCK) {
        const int v = g_lo * rec + tv;
        double s = 0.0;
        int gi = task.group_begin;
        for (; gi + 8 <= task.group_end; gi += 8) {
            double x[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = stage[groups[gi + k].soff + v];
#pragma unroll
            for (int k = 0; k < 8; ++k) s += x[k];
        }
        for (; gi < task.group_end; ++gi) s += stage[groups[gi].soff + v];
        sums[tv] = s;
    }
    __syncthreads();
    if (tid < ng) {
        const int gg = sr.gauss_off + task.g0 + g_lo + tid;
        const double *sm = sums + rec * tid;
        const float *u = P.prec + 6 * gg;
        float *gp = g_prec + 6 * gg;
#pragma unroll
        for (int c = 0; c < 6; ++c) gp[c] = (float)sm[c];
        const double r0 = sm[6], r1 = sm[7], r2 = sm[8];
        g_means[3 * gg + 0] = (float)(-(double)u[0] * r0);
        g_means[3 * gg + 1] = (float)(-((double)u[1] * r0 + (double)u[3] * r1));
        g_means[3 * gg + 2] = (float)(-((double)u[2] * r0 + (double)u[4] * r1 + (double)u[5] * r2));
        g_weights[gg] = (float)(sm[9] / (double)P.weights[gg]);
        if (rec == kPartialColor && g_colors) {
            // colour = sigmoid(q): dL/dq = dL/dc c (1 - c)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double col = 1.0 / (1.0 + exp(-(double)P.colors[3 * gg + c]));
                g_colors[3 * gg + c] = (float)(sm[10 + c] * col * (1.0 - col));
            }
        }
    }
    if (task.beta && blockIdx.y == 0 && tid < 2) {
        const double sb = ordered_sum(stage_beta + 2 * task.sgroup_begin + tid, task.sgroup_end - task.sgroup_begin, 2);
        // beta1_bar = sum z_bar d (d = d2 / log2 e); beta2_bar = -sum z_bar t / eta
        g_betas[2 * task.scene + tid] = tid == 0 ? (float)(sb / kLog2e) : (float)(-sb / (double)P.eta[task.scene]);
    }
}

// Gradient of the Sec. 4 reconstruction loss (mask BCE, mask-weighted L1 depth, mask-weighted
// flow term) with respect to one render's outputs; per-block loss partials in fixed order.
constexpr int kLossBlock = 1024;

__global__ __launch_bounds__(kLossBlock) void loss_kernel(int p, const float *__restrict__ depth,
                                                         const float *__restrict__ alpha,
                                                         const float *__restrict__ flow,
                                                         const float *__restrict__ color,
                                                         const float *__restrict__ depth_t,
                                                         const float *__restrict__ alpha_t,
                                                         const float *__restrict__ flow_t,
                                                         const float *__restrict__ color_t, float w_depth,
                                                         float w_flow, int flow_norm, int flow_cols,
                                                         float w_color, float *__restrict__ g_depth, float *__restrict__ g_alpha,
                                                         float *__restrict__ g_flow, float *__restrict__ g_color,
                                                         float *__restrict__ block_loss)
{
    __shared__ float red[kLossBlock / 64];
    const int r = blockIdx.x * kLossBlock + threadIdx.x;
    const float inv_p = 1.0f / (float)p;
    float l = 0.0f;
    if (r < p) {
        const float at = alpha_t[r];
        const float a = alpha[r];
        const float ac = fminf(fmaxf(a, 1e-6f), 1.0f - 1e-6f);
        const bool inside = a >= 1e-6f && a <= 1.0f - 1e-6f;
        g_alpha[r] = inside ? (ac - at) / (ac * (1.0f - ac)) * inv_p : 0.0f;
        const float dd = depth[r] - depth_t[r];
        g_depth[r] = w_depth * at * (float)((dd > 0.0f) - (dd < 0.0f)) * inv_p;
        l = -(at * logf(ac) + (1.0f - at) * logf(1.0f - ac)) + w_depth * at * fabsf(dd);
        if (flow) {
            for (int c = 0; c < flow_cols; ++c) {
                const float f = flow[flow_cols * r + c] - flow_t[flow_cols * r + c];
                if (flow_norm == 1) {
                    g_flow[flow_cols * r + c] = w_flow * at * (float)((f > 0.0f) - (f < 0.0f)) * inv_p;
                    l += w_flow * at * fabsf(f);
                } else {
                    g_flow[flow_cols * r + c] = 2.0f * w_flow * at * f * inv_p;
                    l += w_flow * at * f * f;
                }
            }
        }
        if (color) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float dc = color[3 * r + c] - color_t[3 * r + c];
                g_color[3 * r + c] = w_color * at * (float)((dc > 0.0f) - (dc < 0.0f)) * inv_p;
                l += w_color * at * fabsf(dc);
            }
        }
        l *= inv_p;
    }
    if (block_loss) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
        __syncthreads();
        if (threadIdx.x == 0) {
            float s = 0.0f;
            for (int k = 0; k < kLossBlock / 64; ++k) s += red[k];
            block_loss[blockIdx.x] = s;
        }
    }
}

hipError_t launch_loss(int p, const float *depth, const float *alpha, const float *flow, const float *color,
                       const float *depth_t, const float *alpha_t, const float *flow_t, const float *color_t,
                       float w_depth, float w_flow, int flow_norm, int flow_cols, float w_color, float *g_depth,
                       float *g_alpha, float *g_flow, float *g_color, float *block_loss, hipStream_t st)
{
    hipLaunchKernelGGL(loss_kernel, dim3((p + kLossBlock - 1) / kLossBlock), dim3(kLossBlock), 0, st, p, depth, alpha,
                       flow, color, depth_t, alpha_t, flow_t, color_t, w_depth, w_flow, flow_norm, flow_cols, w_color, g_depth,
                       g_alpha, g_flow, g_color, block_loss);
    return hipGetLastError();
}

__global__ void fill_int_kernel(int *p, int n, int value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// Parameter validation: bit 1 non-finite, 2 weight <= 0, 4 zero diagonal of U, 8 bad beta.
__global__ void validate_kernel(Params P, int n_total, int n_scenes, int *flags)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int f = 0;
    if (i < n_total) {
        for (int a = 0; a < 3; ++a)
            if (!isfinite(P.means[3 * i + a])) f |= 1;
        for (int a = 0; a < 6; ++a)
            if (!isfinite(P.prec[6 * i + a])) f |= 1;
        const float w = P.weights[i];
        if (!isfinite(w)) f |= 1;
        if (!(w > 0.0f)) f |= 2;
        if (P.prec[6 * i] == 0.0f || P.prec[6 * i + 3] == 0.0f || P.prec[6 * i + 5] == 0.0f) f |= 4;
    }
    if (i < n_scenes) {
        if (!isfinite(P.betas[2 * i]) || !isfinite(P.betas[2 * i + 1])) f |= 8;
    }
    if (f) atomicOr(flags, f);
}

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------

constexpr int kBlock = 256;

struct FwdVariant {
    int rpt, tg;
};
static const FwdVariant kFwdVariants[] = {{1, 128}, {2, 128}, {2, 256}, {4, 128}};
static const int kBwdRT[] = {64, 128, 256};

// F dispatch: calls body<F>() for the runtime flag set f (0..15).
#define FMB_DISPATCH_F(f, CALL)                                                                            \
    switch (f) {                                                                                           \
    case 0: CALL(0); break;   case 1: CALL(1); break;   case 2: CALL(2); break;   case 3: CALL(3); break;   \
    case 4: CALL(4); break;   case 5: CALL(5); break;   case 6: CALL(6); break;   case 7: CALL(7); break;   \
    case 8: CALL(8); break;   case 9: CALL(9); break;   case 10: CALL(10); break; case 11: CALL(11); break; \
    case 12: CALL(12); break; case 13: CALL(13); break; case 14: CALL(14); break; case 15: CALL(15); break; \
    default: return hipErrorInvalidValue;                                                                  \
    }

template <int RPT, int TG>
static hipError_t launch_fwd_v(int f, int grid, hipStream_t st, const Params &P, const FwdOut &O,
                               const FwdItem *items, int n, const int *order, int *counter)
{
#define FMB_FWD_CALL(F)                                                                                    \
    hipLaunchKernelGGL((fwd_kernel<kBlock, RPT, TG, F>), dim3(grid), dim3(kBlock), 0, st, P, O, items, n, order, \
                       counter)
    FMB_DISPATCH_F(f, FMB_FWD_CALL)
#undef FMB_FWD_CALL
    return hipGetLastError();
}

template <int RT>
static hipError_t launch_bwd_v(int f, int grid, hipStream_t st, const Params &P, const BwdIn &I,
                               const BwdItem *items, int n, const int *order, int *counter, float *partial,
                               float *bpart)
{
#define FMB_BWD_CALL(F)                                                                                    \
    hipLaunchKernelGGL((bwd_kernel<kBlock, RT, F>), dim3(grid), dim3(kBlock), 0, st, P, I, items, n, order,     \
                       counter, partial, bpart)
    FMB_DISPATCH_F(f, FMB_BWD_CALL)
#undef FMB_BWD_CALL
    return hipGetLastError();
}

int num_fwd_variants() { return (int)(sizeof kFwdVariants / sizeof kFwdVariants[0]); }
int fwd_variant_rays(int v) { return kBlock * kFwdVariants[v].rpt; }
int num_bwd_variants() { return (int)(sizeof kBwdRT / sizeof kBwdRT[0]); }
int bwd_variant_rt(int v) { return kBwdRT[v]; }
int block_size() { return kBlock; }

// flags: bit 0 normals, 1 flow, 2 persistent, 3 colour
hipError_t launch_fwd(int variant, int flags, int grid, hipStream_t st, const Params &P, const FwdOut &O,
                      const FwdItem *items, int n, const int *order, int *counter)
{
    switch (variant) {
    case 0: return launch_fwd_v<1, 128>(flags, grid, st, P, O, items, n, order, counter);
    case 1: return launch_fwd_v<2, 128>(flags, grid, st, P, O, items, n, order, counter);
    case 2: return launch_fwd_v<2, 256>(flags, grid, st, P, O, items, n, order, counter);
    case 3: return launch_fwd_v<4, 128>(flags, grid, st, P, O, items, n, order, counter);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bwd(int variant, int flags, int grid, hipStream_t st, const Params &P, const BwdIn &I,
                      const BwdItem *items, int n, const int *order, int *counter, float *partial, float *bpart)
{
    switch (variant) {
    case 0: return launch_bwd_v<64>(flags, grid, st, P, I, items, n, order, counter, partial, bpart);
    case 1: return launch_bwd_v<128>(flags, grid, st, P, I, items, n, order, counter, partial, bpart);
    case 2: return launch_bwd_v<256>(flags, grid, st, P, I, items, n, order, counter, partial, bpart);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fin(int n_tasks, int n_groups, hipStream_t st, const Params &P, const FinTask *tasks,
                      const FinGroup *groups, const float *partial, const float *bpart, double *stage,
                      double *stage_beta, float *g_means, float *g_prec, float *g_weights, float *g_colors,
                      float *g_betas)
{
    hipLaunchKernelGGL((fin1_kernel<256>), dim3(n_groups), dim3(256), 0, st, groups, partial, bpart, stage,
                       stage_beta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fin2_kernel<256>), dim3(n_tasks, (kBlock + kFinSlice - 1) / kFinSlice), dim3(256), 0, st, P,
                       tasks, groups, stage, stage_beta, g_means, g_prec, g_weights, g_colors, g_betas);
    return hipGetLastError();
}

hipError_t launch_fill(int *p, int n, int value, hipStream_t st)
{
    hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, value);
    return hipGetLastError();
}

hipError_t launch_validate(const Params &P, int n_total, int n_scenes, int *flags, hipStream_t st)
{
    const int n = n_total > n_scenes ? n_total : n_scenes;
    hipLaunchKernelGGL(validate_kernel, dim3((n + 255) / 256), dim3(256), 0, st, P, n_total, n_scenes, flags);
    return hipGetLastError();
}

template <typename K>
static hipError_t occ(K kernel, int *blocks)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, kernel, kBlock, 0);
}

// Occupancy of the persistent kernels (flags include kPer).
hipError_t occupancy_fwd(int variant, int flags, int *blocks_per_cu)
{
#define FMB_OCC_F(F) return occ(fwd_kernel<kBlock, RPT, TG, F>, blocks_per_cu)
#define FMB_OCC_V(RPT_, TG_)                                                                               \
    {                                                                                                      \
        constexpr int RPT = RPT_, TG = TG_;                                                                \
        FMB_DISPATCH_F(flags, FMB_OCC_F)                                                                   \
    }
    switch (variant) {
    case 0: FMB_OCC_V(1, 128)
    case 1: FMB_OCC_V(2, 128)
    case 2: FMB_OCC_V(2, 256)
    case 3: FMB_OCC_V(4, 128)
    default: return hipErrorInvalidValue;
    }
#undef FMB_OCC_V
#undef FMB_OCC_F
    return hipErrorInvalidValue;
}

hipError_t occupancy_bwd(int variant, int flags, int *blocks_per_cu)
{
#define FMB_OCC_F(F) return occ(bwd_kernel<kBlock, RT, F>, blocks_per_cu)
#define FMB_OCC_V(RT_)                                                                                     \
    {                                                                                                      \
        constexpr int RT = RT_;                                                                            \
        FMB_DISPATCH_F(flags, FMB_OCC_F)                                                                   \
    }
    switch (variant) {
    case 0: FMB_OCC_V(64)
    case 1: FMB_OCC_V(128)
    case 2: FMB_OCC_V(256)
    default: return hipErrorInvalidValue;
    }
#undef FMB_OCC_V
#undef FMB_OCC_F
    return hipErrorInvalidValue;
}

}  // namespace fmb
