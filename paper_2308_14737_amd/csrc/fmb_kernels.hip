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
//     reduction and no P x N storage (without a normal cotangent in the offset form of
//     pair_adjoint_offset).  Partial gradients per item are reduced deterministically by
//     the finalize kernel.
//   * persistent variants pull items from a device counter (reset by a fill kernel)
//     in the order given by the host (largest item first).
//
// Per pair (ray o + t v with |v| = 1, Gaussian mu, U, lambda; mu' = mu - o):
//   a = U v, t = v.c / a.a (peak of the density along the ray, Sec. 3.1),
//   r = U (t v - mu') formed as U (t v - hi) - U lo, m = r.r, d = log lambda - m/2 (Eq. 2),
//   delta = e^d (Eq. 4), z = beta1 d - (beta2/eta) t (log of Eq. 7); where a normal is
//   needed, one Newton step on |U(t v - mu')|^2 moves r to the peak, g = U^T r =
//   Sigma^-1 x (Eq. 17).
#include "fmb_device.h"

namespace fmb {

// ------------------------------------------------------------------------------------
// Forward
// ------------------------------------------------------------------------------------

template <int BLOCK, int RPT, int TG, int F>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void fwd_kernel(Params P, FwdOut O, const FwdItem *__restrict__ items,
                                                   int n_items, const int *__restrict__ order,
                                                   int *__restrict__ counter)
{
    constexpr bool NORMALS = (F & kNrm) != 0, PERSIST = (F & kPer) != 0;
    constexpr bool COLOR = (F & kCol) != 0, BIG = (F & kBig) != 0;
    constexpr int EW = COLOR ? 6 : 5;  // float4 per LDS entry: the entry, the m estimate terms, colour
    __shared__ float4 tile[TG * EW];
    // the first sweep's weight bound of each (Gaussian, ray tile) for the second sweep (-inf where
    // the first sweep took the pair): per wave, per group of 64 / RPT Gaussians, per lane
    __shared__ float zsave[BLOCK / 64][TG * RPT];
    // scenes beyond BLOCK Gaussians: the item's tile cones, the waves' least running maxima and
    // counts of survivors, and a round's survivors
    __shared__ float4 icones[BIG ? BLOCK / 64 * RPT : 1];
    __shared__ float wmin[BIG ? BLOCK / 64 : 1];
    __shared__ int wcnt[BIG ? BLOCK / 64 : 1];
    __shared__ int slist[BIG ? BLOCK : 1];
    __shared__ int s_item;
    int pos = blockIdx.x;
    for (;;) {
        if (PERSIST) {
            __syncthreads();  // everyone is done with s_item and the tile of the last item
            if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
            __syncthreads();
            pos = __builtin_amdgcn_readfirstlane(s_item);  // block-uniform: keep the item in SGPRs
        }
        if (pos >= n_items) break;
        const int it = order ? ld_uniform(order + pos) : pos;
        const FwdItem item = ld_uniform(items + it);
        const ViewRec vr = ld_uniform(P.views + item.view);
        const SceneRec sr = ld_uniform(P.scenes + vr.scene);
        const CamRec cam = cam_of(P, item.view);
        const float *e = cam.e, *kk = cam.k;
        double o[3];
        cam_centre(e, o);
        const Blend bl = blend_of(P, vr.scene);
        const bool b1_pos = bl.b1 >= 0.0f;  // the weight bound needs beta1 >= 0
        // ray j of a lane: lane `lane` of tile tile0 + j * NW + wave (8 x 8 pixels where the view is
        // wide enough: a wave's rays stay close together, so the exact skip of zero weights below
        // is uniform over the wave more often)
        constexpr int NW = BLOCK / 64;
        const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;

        float v0[RPT], v1[RPT], v2[RPT];
        float M[RPT], S[RPT], T[RPT], N0[RPT], N1[RPT], N2[RPT], D[RPT], C0[RPT], C1[RPT], C2[RPT];
        float at[RPT], dt[RPT];  // loss targets, loaded now so that the epilogue does not wait
        int loc[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            int row, col;
            loc[j] = tile_local(vr, item.tile0 + j * NW + wave, lane, row, col);
            const int lc = loc[j] >= 0 ? loc[j] : 0;  // a lane past the edge takes ray 0 (not written)
            tile_ray_dir(P, vr, e, kk, lc, loc[j] >= 0 ? row : 0, loc[j] >= 0 ? col : 0, v0[j], v1[j], v2[j]);
            M[j] = -INFINITY;
            S[j] = T[j] = N0[j] = N1[j] = N2[j] = D[j] = C0[j] = C1[j] = C2[j] = 0.0f;
            at[j] = dt[j] = 0.0f;
            if (O.g_depth) {
                at[j] = O.alpha_t[vr.ray_off + lc];
                dt[j] = O.depth_t[vr.ray_off + lc];
            }
        }
        // The cone of each of the wave's ray tiles (unit centre direction, largest |v - c|), for the
        // bound of tile_bounds: lane l bounds Gaussian l / RPT on ray tile l % RPT (cl: its cone).
        const int jl = lane % RPT;
        float4 cl = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const bool ok = loc[j] >= 0;
            float c0 = ok ? v0[j] : 0.0f, c1 = ok ? v1[j] : 0.0f, c2 = ok ? v2[j] : 0.0f;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                c0 += __shfl_xor(c0, off, 64);
                c1 += __shfl_xor(c1, off, 64);
                c2 += __shfl_xor(c2, off, 64);
            }
            const float inv = rsq_(fmaf(c0, c0, fmaf(c1, c1, fmaf(c2, c2, kEpsN))));
            c0 *= inv;
            c1 *= inv;
            c2 *= inv;
            const float e0 = v0[j] - c0, e1 = v1[j] - c1, e2 = v2[j] - c2;
            float rho = ok ? sqrtf(fmaf(e0, e0, fmaf(e1, e1, e2 * e2))) : 0.0f;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) rho = fmaxf(rho, __shfl_xor(rho, off, 64));
            if (jl == j) cl = make_float4(c0, c1, c2, rho * (1.0f + 1e-4f) + 1e-6f);
        }

        // A scene of more than BLOCK Gaussians is taken in rounds of BLOCK: each Gaussian of the
        // round is first bounded on a cone around all the item's tiles, and only those whose
        // density can reach 2^kDensSkipLog2 there, or whose weight can be above FP32's zero
        // against the least running maximum of the item's rays so far, are staged, in scene order
        // (slist).  The running maxima only grow, so a Gaussian left out is one whose every pair
        // the tests below would skip when its turn came: the sums are those of the full order.
        // Smaller scenes take one round of all their Gaussians (and launches without kBig, whose
        // scenes are all small, have no such rounds).
        const bool sparse = BIG && sr.n > BLOCK;
        if (sparse && lane < RPT) icones[wave * RPT + lane] = cl;
        for (int rb = 0; rb < sr.n; rb += sparse ? BLOCK : sr.n) {
          int total = sr.n;
          if (sparse) {
            float mm = INFINITY;
#pragma unroll
            for (int j = 0; j < RPT; ++j) mm = loc[j] >= 0 ? fminf(mm, M[j]) : mm;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) mm = fminf(mm, __shfl_xor(mm, off, 64));
            __syncthreads();  // the previous round's list and staged tile are consumed
            if (lane == 0) wmin[wave] = mm;
            __syncthreads();  // tile cones and least maxima visible
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, imin = INFINITY;
            for (int t = 0; t < NW * RPT; ++t) {
                s0 += icones[t].x;  // (a tile without a ray in the view has centre 0)
                s1 += icones[t].y;
                s2 += icones[t].z;
            }
            for (int w = 0; w < NW; ++w) imin = fminf(imin, wmin[w]);
            const float si = rsq_(fmaf(s0, s0, fmaf(s1, s1, fmaf(s2, s2, kEpsN))));
            s0 *= si;
            s1 *= si;
            s2 *= si;
            float irho = 0.0f;  // |v - c| <= |v - c_t| + |c_t - c| for a ray v of tile t
            for (int t = 0; t < NW * RPT; ++t) {
                const float4 ct = icones[t];
                if (fmaf(ct.x, ct.x, fmaf(ct.y, ct.y, ct.z * ct.z)) < 0.25f) continue;
                const float d0 = ct.x - s0, d1 = ct.y - s1, d2 = ct.z - s2;
                irho = fmaxf(irho, sqrtf(fmaf(d0, d0, fmaf(d1, d1, d2 * d2))) + ct.w);
            }
            const float4 icone = make_float4(s0, s1, s2, irho * (1.0f + 1e-4f) + 1e-6f);
            const int gl = rb + (int)threadIdx.x;
            bool keep = false;
            if (gl < sr.n) {
                const int gg = sr.gauss_off + gl;
                float4 q[5];
                make_entry_est(P.means + 3 * gg, P.prec + 6 * gg, P.weights[gg], o, q);
                float d2_hi, z_hi;
                tile_bounds(ent_from(q[0], q[1], q[2], q[3]), q[4], icone, bl.hm, bl.b1, bl.nc2, d2_hi, z_hi);
                // (written so that a NaN bound keeps the Gaussian)
                keep = !(b1_pos && d2_hi < kDensSkipLog2 && z_hi - imin < kSkipLog2);
            }
            const unsigned long long bal = wave_ballot(keep);
            if (lane == 0) wcnt[wave] = __popcll(bal);
            __syncthreads();
            int off = 0;
            total = 0;
            for (int w = 0; w < NW; ++w) {
                const int c = wcnt[w];
                off += w < wave ? c : 0;
                total += c;
            }
            if (keep) slist[off + __popcll(bal & ((1ull << lane) - 1ull))] = gl;
          }
        for (int gb = 0; gb < total; gb += TG) {
            const int cnt = min(TG, total - gb);
            if (gb > 0 || !PERSIST || sparse) __syncthreads();
            for (int q = threadIdx.x; q < cnt; q += BLOCK) {
                const int gi = sr.gauss_off + (sparse ? slist[gb + q] : gb + q);
                make_entry_est(P.means + 3 * gi, P.prec + 6 * gi, P.weights[gi], o, &tile[EW * q]);
                if (COLOR) tile[EW * q + 5] = colour_entry(P.colors + 3 * gi);
            }
            __syncthreads();
            // Two sweeps over the staged Gaussians, GP at a time.  The first takes the (Gaussian, ray
            // tile) pairs whose density can reach 2^kDensSkipLog2 on some ray of the tile -- these
            // hold every ray's largest weights -- and the second the others, except where the tile's
            // least running maximum then rules out a weight above FP32's zero (tile_bounds; a pair
            // of neither sweep is one the per-pair test below would skip).  Without beta1 >= 0 the
            // weight bound does not hold and the first sweep takes every pair.
            constexpr int GP = 64 / RPT;
            float mmin = -INFINITY;  // the least running maximum of lane's bound tile (second sweep)
            for (int sweep = 0; sweep < 2; ++sweep) {
              if (sweep == 1) {
#pragma unroll
                for (int j = 0; j < RPT; ++j) {
                    float mm = loc[j] >= 0 ? M[j] : INFINITY;
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) mm = fminf(mm, __shfl_xor(mm, off, 64));
                    if (jl == j) mmin = mm;
                }
              }
              for (int ib = 0; ib < cnt; ib += GP) {
                const int il = ib + lane / RPT;
                float *const zs = &zsave[wave][ib * RPT + lane];
                bool need = false;
                if (il < cnt) {
                    if (sweep == 0) {
                        const Ent gl = ent_from(tile[EW * il], tile[EW * il + 1], tile[EW * il + 2], tile[EW * il + 3]);
                        float d2h, zh;
                        tile_bounds(gl, tile[EW * il + 4], cl, bl.hm, bl.b1, bl.nc2, d2h, zh);
                        // (comparisons written so that a NaN bound keeps the pair)
                        need = !(b1_pos && d2h < kDensSkipLog2);
                        *zs = need ? -INFINITY : zh;
                    } else {
                        const float zh = *zs;
                        need = zh != -INFINITY && !(zh - mmin < kSkipLog2);
                    }
                }
                const unsigned long long nm = wave_ballot(need);
                if (nm == 0ull) continue;
                const int kn = min(GP, cnt - ib);
#pragma unroll 2
              for (int k = 0; k < kn; ++k) {
                const unsigned bits = (unsigned)(nm >> (k * RPT)) & ((1u << RPT) - 1u);
                if (bits == 0u) continue;
                const int i = ib + k;
                const Ent g = ent_from(tile[EW * i], tile[EW * i + 1], tile[EW * i + 2], tile[EW * i + 3]);
                const float4 est = tile[EW * i + 4];
                float4 cc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (COLOR) cc = tile[EW * i + 5];
#pragma unroll
                for (int j = 0; j < RPT; ++j) {
                    if (!((bits >> j) & 1u)) continue;  // no ray of tile j needs the pair
                    Geo q;
                    const float vc = pair_geo_peak(g, v0[j], v1[j], v2[j], q);
                    {
                        // upper bounds of the log2 density and weight from a lower bound of m (one
                        // FMA): a pair below both cutoffs adds a weight that is zero in FP32 and a
                        // density below 2^kDensSkipLog2 to alpha's sum, and skips the residual
                        const float d2_hi = fmaf(bl.hm, pair_m_low(est, vc, q.t), g.l2l);
                        const float zr_hi = b1_pos ? fmaf(bl.b1, d2_hi, fmaf(bl.nc2, q.t, -M[j])) : INFINITY;
                        if (zr_hi < kSkipLog2 && d2_hi < kDensSkipLog2) continue;
                    }
                    pair_geo_resid(g, v0[j], v1[j], v2[j], bl.hm, bl.b1, bl.nc2, q);
                    const float delta = exp2_(q.d2);
                    D[j] += delta;
                    // log2 of the weight relative to the running maximum, b1 d2 + (nc2 t - M)
                    float zr = fmaf(bl.b1, q.d2, fmaf(bl.nc2, q.t, -M[j]));
                    // A weight below 2^-150 of the running maximum is zero in FP32: its terms are
                    // skipped (the branch is uniform over a wave for most distant Gaussians).
                    if (zr < kSkipLog2) continue;
                    pair_refine(q);
                    if (zr > 0.0f) {  // new running maximum: rescale the sums (rare)
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
                        zr = 0.0f;
                    }
                    const float ew = exp2_(zr);
                    S[j] += ew;
                    T[j] = fmaf(ew, q.t, T[j]);
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
            }
        }
        }

        const float o0 = (float)o[0], o1 = (float)o[1], o2 = (float)o[2];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            if (loc[j] < 0) continue;
            write_ray<F>(P, O, item.view, vr.ray_off + loc[j], e, kk, o0, o1, o2, v0[j], v1[j], v2[j], M[j], S[j],
                         T[j], N0[j], N1[j], N2[j], C0[j], C1[j], C2[j], D[j], at[j], dt[j]);
        }
        if (!PERSIST) break;
    }
}

// ------------------------------------------------------------------------------------
// Backward
// ------------------------------------------------------------------------------------


// Waves per SIMD the Gaussian-lane backward is compiled for: six (at most 80 VGPRs) where the
// variant fits without spilling, else what its registers give.
constexpr int bwd_min_waves(int F)
{
    return ((F & kCol) ? F == kCol : !((F & kFlw) && (F & kPer))) ? 6 : 1;
}

template <int BLOCK, int RT, int F>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(bwd_min_waves(F)))) void bwd_kernel(Params P, BwdIn I, const BwdItem *__restrict__ items,
                                                   int n_items, const int *__restrict__ order,
                                                   int *__restrict__ counter, float *__restrict__ partial,
                                                   float *__restrict__ beta_partial)
{
    constexpr bool NORMALS = (F & kNrm) != 0, PERSIST = (F & kPer) != 0, COLOR = (F & kCol) != 0;
    // Without a normal cotangent the pairs take pair_adjoint_offset: the staged ray is
    // (v, M2) (invS, tf_bar, kappa, D_bar) (t_f, dc, 0, 0) [(Cb, 0)]; with one it is the prologue
    // as written by ray_prologue (four float4).
    constexpr bool PLAIN = !NORMALS;
    constexpr int RW = PLAIN ? (COLOR ? 4 : 3) : 4;  // float4 per staged ray
    constexpr int REC = COLOR ? kPartialColor : kPartial;  // partial record per Gaussian
    // a lane's sums: (H, Bv, L) of the offset form or the general record, then the colour sums
    constexpr int LREC = PLAIN ? kOffsetAcc + (COLOR ? 3 : 0) : REC;
    constexpr int RS = LREC + 2;                  // reduction record per lane (+ two betas)
    // the staged rays and, after an item's pair loop, the reduction records share the LDS
    constexpr int SM4 = RT * RW > BLOCK * RS / 4 ? RT * RW : (BLOCK * RS + 3) / 4;
    __shared__ float4 smem[SM4];
    float4 *rays = smem;
    float *red = reinterpret_cast<float *>(smem);
    __shared__ int s_item;
    int pos = blockIdx.x;
    const int tid = threadIdx.x;
    for (;;) {
        if (PERSIST) {
            __syncthreads();
            if (tid == 0) s_item = atomicAdd(counter, 1);
            __syncthreads();
            pos = __builtin_amdgcn_readfirstlane(s_item);  // block-uniform: keep the item in SGPRs
        }
        if (pos >= n_items) break;
        const int it = order ? ld_uniform(order + pos) : pos;
        const BwdItem item = ld_uniform(items + it);
        const ViewRec vr = ld_uniform(P.views + item.view);
        const SceneRec sr = ld_uniform(P.scenes + vr.scene);
        const CamRec cam = cam_of(P, item.view);
        const float *e = cam.e, *kk = cam.k;
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
        float aB1 = 0, aB2 = 0;
        float aC0 = 0, aC1 = 0, aC2 = 0;
        // The item's rays RT at a time: staged with their prologue, then `pair` runs over this lane's
        // rays slot, slot + slots, ... (walked by address: one induction variable).
        auto passes = [&](auto &&pair) {
            for (int r0 = item.ray0; r0 < end; r0 += RT) {
                const int cnt = min(RT, end - r0);
                __syncthreads();
                for (int q = tid; q < RT; q += BLOCK) {
                    float4 pr[4];
                    ray_prologue<F>(P, I, item.view, vr, e, kk, o0, o1, o2, r0 + q, q < cnt, bl.b1, bl.nc2, pr);
                    if (PLAIN) {
                        rays[RW * q] = pr[0];
                        rays[RW * q + 1] = make_float4(pr[1].x, pr[1].y, pr[2].y, pr[2].z);
                        rays[RW * q + 2] = make_float4(pr[2].w, pr[3].w, 0.0f, 0.0f);
                        if (COLOR) rays[RW * q + 3] = pr[3];
                    } else {
#pragma unroll
                        for (int k = 0; k < RW; ++k) rays[RW * q + k] = pr[k];
                    }
                }
                __syncthreads();
                if (active) {
                    const float4 *const rend = rays + RW * cnt;
                    for (const float4 *rp = rays + RW * slot; rp < rend; rp += RW * item.slots) pair(rp);
                }
            }
            __syncthreads();  // every lane is done with the staged rays (the LDS is reused below)
        };
        // One pair without a normal cotangent, accumulated in the offset form.
        auto plain_pair = [&](const float4 *rp, OffsetAcc &acc) {
            const float4 x0 = rp[0], x1 = rp[1], x2 = rp[2];
            float4 x4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (COLOR) x4 = rp[3];
            const float v0 = x0.x, v1 = x0.y, v2 = x0.z;
            Geo q;
            pair_geo_coarse(g, v0, v1, v2, bl.hm, bl.b1, bl.nc2, q);
            const float delta = exp2_(q.d2);
            // normalised blend weight 2^(z2 - M) / S, with z2 - M = b1 d2 + (nc2 t - M)
            const float wt = exp2_(fmaf(bl.b1, q.d2, fmaf(bl.nc2, q.t, -x0.w))) * x1.x;
            const float tfb = x1.y;
            float lin = tfb * q.t;
            if (COLOR) {
                lin = fmaf(x4.x, cc.x, fmaf(x4.y, cc.y, fmaf(x4.z, cc.z, lin)));
                aC0 = fmaf(wt, x4.x, aC0);
                aC1 = fmaf(wt, x4.y, aC1);
                aC2 = fmaf(wt, x4.z, aC2);
            }
            const float zb = wt * (lin - x1.z);
            const float tb = fmaf(-bl.cb, zb, wt * tfb);
            const float db = fmaf(bl.b1, zb, x1.w * delta);
            aB1 = fmaf(zb, q.d2 - x2.y, aB1);
            aB2 = fmaf(zb, q.t - x2.x, aB2);
            pair_adjoint_offset(q, v0, v1, v2, tb, db, acc);
        };
        float *my = red + RS * tid;
        if (!PLAIN) {
            PairAcc acc;
            passes([&](const float4 *rp) {
                const float4 x0 = rp[0], x1 = rp[1], x2 = rp[2], x3 = rp[3];
                const float v0 = x0.x, v1 = x0.y, v2 = x0.z;
                Geo q;
                pair_geo(g, v0, v1, v2, bl.hm, bl.b1, bl.nc2, q);
                const float delta = exp2_(q.d2);
                const float wt = exp2_(q.z2 - x0.w) * x1.x;   // normalised blend weight
                const float tfb = x1.y;
                PairNormal pn{0, 0, 0, 0, 0};
                if (NORMALS) pn = pair_normal(g, q, x1.z, x1.w, x2.x);
                // softmax adjoint: z_bar = wt (tf_bar t + Nb.n + Cb.c - kappa)
                float lin = fmaf(tfb, q.t, pn.nN);
                if (COLOR) {
                    lin = fmaf(x3.x, cc.x, fmaf(x3.y, cc.y, fmaf(x3.z, cc.z, lin)));
                    aC0 = fmaf(wt, x3.x, aC0);
                    aC1 = fmaf(wt, x3.y, aC1);
                    aC2 = fmaf(wt, x3.z, aC2);
                }
                const float zb = wt * (lin - x2.y);
                // z = beta1 d - (beta2/eta) t
                const float tb = fmaf(-bl.cb, zb, wt * tfb);
                const float db = fmaf(bl.b1, zb, x2.z * delta);
                aB1 = fmaf(zb, q.d2 - x3.w, aB1);
                aB2 = fmaf(zb, q.t - x2.w, aB2);
                pair_adjoint<NORMALS>(g, q, v0, v1, v2, wt, pn, x1.z, x1.w, x2.x, tb, db, acc);
            });
            my[0] = acc.u0; my[1] = acc.u1; my[2] = acc.u2; my[3] = acc.u3; my[4] = acc.u4; my[5] = acc.u5;
            my[6] = acc.p0; my[7] = acc.p1; my[8] = acc.p2; my[9] = acc.l;
        } else {
            OffsetAcc acc;
            passes([&](const float4 *rp) { plain_pair(rp, acc); });
            offset_acc_store(acc, my);
        }

        // deterministic block reduction: Gaussian partials over the slots, betas over all lanes
        if (COLOR) {
            my[LREC - 3] = aC0; my[LREC - 2] = aC1; my[LREC - 1] = aC2;
        }
        my[LREC] = aB1; my[LREC + 1] = aB2;
        __syncthreads();
        if (slot == 0 && gi < item.gc && item.g0 + gi < sr.n) {
            float sum[LREC];
#pragma unroll
            for (int c = 0; c < LREC; ++c) sum[c] = red[RS * gi + c];
            for (int s = 1; s < item.slots; ++s) {
#pragma unroll
                for (int c = 0; c < LREC; ++c) sum[c] += red[RS * (s * item.gc + gi) + c];
            }
            const int gg = sr.gauss_off + item.g0 + gi;
            if (PLAIN)
                write_partial_offset(partial + item.poff + REC * gi, sum, REC, P.prec + 6 * gg, P.means + 3 * gg, o);
            else
                write_partial(partial + item.poff + REC * gi, sum, REC, P.means + 3 * gg, o);
        }
        if (tid < 64) {
            // lane l sums lanes l, l+64, ... in order, then a fixed butterfly over the wave
            float s1 = 0.0f, s2 = 0.0f;
            for (int k = tid; k < BLOCK; k += 64) {
                s1 += red[RS * k + LREC];
                s2 += red[RS * k + LREC + 1];
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
// Backward, ray-lane layout: one lane per ray (RPT rays per lane) as in the forward pass,
// the item's Gaussians staged through LDS in tiles of TG.  For each Gaussian the lanes'
// terms are summed over the wave (butterfly) and the wave sums in LDS, over the item's ray
// tiles, so an item writes one partial record per Gaussian of its scene.  A Gaussian whose
// blend weight is exactly zero (below 2^-150 of the ray's maximum) on every ray of the wave
// takes only the density term of alpha, and one whose density is zero too is skipped.
// ------------------------------------------------------------------------------------

__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

template <int BLOCK, int RPT, int TG, int F>
__global__ __launch_bounds__(BLOCK) void bwdr_kernel(Params P, BwdIn I, const BwdItem *__restrict__ items,
                                                    int n_items, const int *__restrict__ order,
                                                    int *__restrict__ counter, float *__restrict__ partial,
                                                    float *__restrict__ beta_partial)
{
    constexpr bool NORMALS = (F & kNrm) != 0, PERSIST = (F & kPer) != 0, COLOR = (F & kCol) != 0;
    // without a normal cotangent the pairs take the offset form (pair_adjoint_offset)
    constexpr bool PLAIN = !NORMALS;
    constexpr int EW = COLOR ? 5 : 4;                       // float4 per LDS entry
    constexpr int REC = COLOR ? kPartialColor : kPartial;  // partial record per Gaussian
    // sums per Gaussian and wave: (H, Bv, L) of the offset form or the general record, then colour
    constexpr int LREC = PLAIN ? kOffsetAcc + (COLOR ? 3 : 0) : REC;
    constexpr int NW = BLOCK / 64;
    __shared__ float4 tile[TG * EW];
    __shared__ float wsum[NW * TG * LREC];  // per wave, per Gaussian of the tile
    __shared__ float bsum[NW * 2];
    __shared__ int s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int pos = blockIdx.x;
    for (;;) {
        if (PERSIST) {
            __syncthreads();
            if (tid == 0) s_item = atomicAdd(counter, 1);
            __syncthreads();
            pos = __builtin_amdgcn_readfirstlane(s_item);  // block-uniform: keep the item in SGPRs
        }
        if (pos >= n_items) break;
        const int it = order ? ld_uniform(order + pos) : pos;
        const BwdItem item = ld_uniform(items + it);
        const ViewRec vr = ld_uniform(P.views + item.view);
        const SceneRec sr = ld_uniform(P.scenes + vr.scene);
        const CamRec cam = cam_of(P, item.view);
        const float *e = cam.e, *kk = cam.k;
        double o[3];
        cam_centre(e, o);
        const float o0 = (float)o[0], o1 = (float)o[1], o2 = (float)o[2];
        const Blend bl = blend_of(P, vr.scene);
        const int hw = vr.h * vr.w;
        const int end = min(item.ray0 + item.span, hw);
        float aB1 = 0.0f, aB2 = 0.0f;

        for (int gb = 0; gb < sr.n; gb += TG) {
            const int cnt = min(TG, sr.n - gb);
            __syncthreads();  // the previous tile's entries and sums are no longer read
            for (int q = tid; q < cnt; q += BLOCK) {
                const int gi = sr.gauss_off + gb + q;
                make_entry(P.means + 3 * gi, P.prec + 6 * gi, P.weights[gi], o, &tile[EW * q]);
                if (COLOR) tile[EW * q + 4] = colour_entry(P.colors + 3 * gi);
            }
            for (int q = tid; q < NW * TG * LREC; q += BLOCK) wsum[q] = 0.0f;
            __syncthreads();
            for (int rb = item.ray0; rb < end; rb += BLOCK * RPT) {
                float4 x0[RPT], x1[RPT], x2[RPT], x3[RPT];
#pragma unroll
                for (int j = 0; j < RPT; ++j) {
                    const int local = rb + tid + j * BLOCK;
                    float4 pr[4];
                    ray_prologue<F>(P, I, item.view, vr, e, kk, o0, o1, o2, local, local < end, bl.b1, bl.nc2, pr);
                    x0[j] = pr[0];
                    x1[j] = pr[1];
                    x2[j] = pr[2];
                    x3[j] = pr[3];
                }
                for (int i = 0; i < cnt; ++i) {
                    const Ent g = ent_from(tile[EW * i], tile[EW * i + 1], tile[EW * i + 2], tile[EW * i + 3]);
                    float4 cc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (COLOR) cc = tile[EW * i + 4];
                    Geo q[RPT];
                    float delta[RPT], wt[RPT];
                    bool need_w = false, need_d = false;
#pragma unroll
                    for (int j = 0; j < RPT; ++j) {
                        if (PLAIN)
                            pair_geo_coarse(g, x0[j].x, x0[j].y, x0[j].z, bl.hm, bl.b1, bl.nc2, q[j]);
                        else
                            pair_geo(g, x0[j].x, x0[j].y, x0[j].z, bl.hm, bl.b1, bl.nc2, q[j]);
                        delta[j] = exp2_(q[j].d2);
                        const bool w_on = q[j].z2 - x0[j].w >= kSkipLog2;
                        wt[j] = w_on ? exp2_(q[j].z2 - x0[j].w) * x1[j].x : 0.0f;
                        need_w |= w_on;
                        need_d |= x2[j].z * delta[j] != 0.0f;
                    }
                    PairAcc a;
                    OffsetAcc pa;
                    float aC0 = 0.0f, aC1 = 0.0f, aC2 = 0.0f;
                    if (wave_any(need_w)) {
#pragma unroll
                        for (int j = 0; j < RPT; ++j) {
                            const float tfb = x1[j].y;
                            PairNormal pn{0, 0, 0, 0, 0};
                            if (NORMALS) pn = pair_normal(g, q[j], x1[j].z, x1[j].w, x2[j].x);
                            float lin = fmaf(tfb, q[j].t, pn.nN);
                            if (COLOR) {
                                lin = fmaf(x3[j].x, cc.x, fmaf(x3[j].y, cc.y, fmaf(x3[j].z, cc.z, lin)));
                                aC0 = fmaf(wt[j], x3[j].x, aC0);
                                aC1 = fmaf(wt[j], x3[j].y, aC1);
                                aC2 = fmaf(wt[j], x3[j].z, aC2);
                            }
                            const float zb = wt[j] * (lin - x2[j].y);
                            const float tb = fmaf(-bl.cb, zb, wt[j] * tfb);
                            const float db = fmaf(bl.b1, zb, x2[j].z * delta[j]);
                            aB1 = fmaf(zb, q[j].d2 - x3[j].w, aB1);
                            aB2 = fmaf(zb, q[j].t - x2[j].w, aB2);
                            if (PLAIN) {
                                pair_adjoint_offset(q[j], x0[j].x, x0[j].y, x0[j].z, tb, db, pa);
                            } else {
                                pair_adjoint<NORMALS>(g, q[j], x0[j].x, x0[j].y, x0[j].z, wt[j], pn, x1[j].z,
                                                      x1[j].w, x2[j].x, tb, db, a);
                            }
                        }
                    } else if (wave_any(need_d)) {
                        // zero weight on every ray of the wave: only d(alpha)/d(delta) remains
#pragma unroll
                        for (int j = 0; j < RPT; ++j) {
                            if (PLAIN) {
                                pair_adjoint_offset(q[j], x0[j].x, x0[j].y, x0[j].z, 0.0f, x2[j].z * delta[j], pa);
                            } else {
                                const PairNormal pn{0, 0, 0, 0, 0};
                                pair_adjoint<false>(g, q[j], x0[j].x, x0[j].y, x0[j].z, 0.0f, pn, 0.0f, 0.0f, 0.0f,
                                                    0.0f, x2[j].z * delta[j], a);
                            }
                        }
                    } else {
                        continue;  // no term of this Gaussian on this wave's rays
                    }
                    float v[LREC];
                    if (PLAIN) {
                        offset_acc_store(pa, v);
                    } else {
                        v[0] = a.u0; v[1] = a.u1; v[2] = a.u2; v[3] = a.u3; v[4] = a.u4; v[5] = a.u5;
                        v[6] = a.p0; v[7] = a.p1; v[8] = a.p2; v[9] = a.l;
                    }
                    if (COLOR) {
                        v[LREC - 3] = aC0; v[LREC - 2] = aC1; v[LREC - 1] = aC2;
                    }
#pragma unroll
                    for (int c = 0; c < LREC; ++c) v[c] = wave_sum(v[c]);
                    if (lane == 0) {
                        float *dst = wsum + (wave * TG + i) * LREC;
#pragma unroll
                        for (int c = 0; c < LREC; ++c) dst[c] += v[c];
                    }
                }
            }
            __syncthreads();
            // the tile's partial records: waves summed in order, -(sum rho) mu'^T applied in double
            for (int q = tid; q < cnt; q += BLOCK) {
                float sum[LREC];
#pragma unroll
                for (int c = 0; c < LREC; ++c) sum[c] = wsum[q * LREC + c];
                for (int w = 1; w < NW; ++w) {
#pragma unroll
                    for (int c = 0; c < LREC; ++c) sum[c] += wsum[(w * TG + q) * LREC + c];
                }
                const int gg = sr.gauss_off + gb + q;
                if (PLAIN)
                    write_partial_offset(partial + item.poff + REC * (gb + q), sum, REC, P.prec + 6 * gg, P.means + 3 * gg, o);
                else
                    write_partial(partial + item.poff + REC * (gb + q), sum, REC, P.means + 3 * gg, o);
            }
        }
        // betas: lanes summed over the wave, then the waves in order
        aB1 = wave_sum(aB1);
        aB2 = wave_sum(aB2);
        if (lane == 0) {
            bsum[2 * wave] = aB1;
            bsum[2 * wave + 1] = aB2;
        }
        __syncthreads();
        if (tid < 2) {
            float sb = 0.0f;
            for (int w = 0; w < NW; ++w) sb += bsum[2 * w + tid];
            beta_partial[2 * item.seq + tid] = sb;
        }
        if (!PERSIST) break;
    }
}

// ------------------------------------------------------------------------------------
// Backward, tiled ray-lane layout (no normal cotangent): an item is T ray tiles of
// one view (8 x 8 pixels, see ViewRec) against every Gaussian of its scene.  The item's rays
// are staged in LDS with their adjoint prologue; each wave takes every NW-th Gaussian and walks
// the T tiles with a lane per ray, so a lane sums that Gaussian's terms over T rays before one
// scattered reduction over the wave.  A tile on which the Gaussian's blend weight is exactly
// zero on every ray takes only the density term of alpha, and one whose density is zero too
// adds nothing -- both decided uniformly over the wave (on the 16-scene batch about 58 % and
// 34 % of (tile, Gaussian) pairs).
// ------------------------------------------------------------------------------------

template <int BLOCK, int T, int TG, int F>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void bwdt_kernel(
    Params P, BwdIn I, const BwdItem *__restrict__ items, int n_items, const int *__restrict__ order,
    int *__restrict__ counter, float *__restrict__ partial, float *__restrict__ beta_partial)
{
    static_assert((F & kNrm) == 0, "the tiled backward takes no normal cotangent");
    constexpr bool PERSIST = (F & kPer) != 0, COLOR = (F & kCol) != 0, BIG = (F & kBig) != 0;
    constexpr int NW = BLOCK / 64;
    constexpr int RAYS = 64 * T;
    static_assert(T <= 32 && 64 % T == 0, "a 32-bit mask of the item's ray tiles, whole tile sets per wave");
    constexpr int RW = COLOR ? 3 : 2;                         // float4 per staged ray
    constexpr int EW = COLOR ? 6 : 5;                         // float4 per staged Gaussian
    constexpr int LREC = kOffsetAcc + (COLOR ? 3 : 0);        // sums per Gaussian
    constexpr int REC = COLOR ? kPartialColor : kPartial;     // partial record per Gaussian
    // per ray: (v, M2 + log2 S), (tf_bar, D_bar, dc, t_f) [, (C_bar, C_bar . C)]
    __shared__ float4 rays[RW * RAYS];
    __shared__ float4 tcone[T];               // per ray tile: unit centre direction, largest |v - c|
    __shared__ float tnorm[T];                // per ray tile: least M2 + log2 S over its rays
    __shared__ int tdb[T];                    // per ray tile: 1 if some ray has D_bar != 0, else 0
    __shared__ float4 ents[EW * TG];          // the Gaussian tile's entries (m estimate terms, colour)
    __shared__ float rec[LREC * TG];          // (H, Bv, L) [and the colour sums] of each Gaussian
    __shared__ float bsum[2 * NW];
    __shared__ int slist[BIG ? BLOCK : 1];    // scenes beyond BLOCK Gaussians: a round's survivors
    __shared__ int wcnt[BIG ? NW : 1];
    __shared__ int s_item;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int pos = blockIdx.x;
    for (;;) {
        if (PERSIST) {
            __syncthreads();
            if (tid == 0) s_item = atomicAdd(counter, 1);
            __syncthreads();
            pos = __builtin_amdgcn_readfirstlane(s_item);  // block-uniform: keep the item in SGPRs
        }
        if (pos >= n_items) break;
        const int it = order ? ld_uniform(order + pos) : pos;
        const BwdItem item = ld_uniform(items + it);
        const ViewRec vr = ld_uniform(P.views + item.view);
        const SceneRec sr = ld_uniform(P.scenes + vr.scene);
        const CamRec cam = cam_of(P, item.view);
        const float *e = cam.e, *kk = cam.k;
        double o[3];
        cam_centre(e, o);
        const float o0 = (float)o[0], o1 = (float)o[1], o2 = (float)o[2];
        const Blend bl = blend_of(P, vr.scene);
        const bool b1_pos = bl.b1 >= 0.0f;  // the weight bound needs beta1 >= 0
        const int nt = min(T, vr.tiles - item.ray0);  // the item's tiles: ray0 is its first tile

        __syncthreads();  // the previous item is done with the staged rays
        for (int q = tid; q < RAYS; q += BLOCK) {
            int row, col;
            const int local = (q >> 6) < nt ? tile_local(vr, item.ray0 + (q >> 6), q & 63, row, col) : -1;
            float4 pr[4];
            ray_prologue<F>(P, I, item.view, vr, e, kk, o0, o1, o2, local >= 0 ? local : 0, local >= 0, bl.b1, bl.nc2,
                            pr);
            // the weight 2^(z2 - M2) / S as 2^(z2 - M2 - log2 S); a ray past the edge has M2 = inf, S = inf
            rays[RW * q] = make_float4(pr[0].x, pr[0].y, pr[0].z, pr[0].w - __builtin_amdgcn_logf(pr[1].x));
            rays[RW * q + 1] = make_float4(pr[1].y, pr[2].z, pr[3].w, pr[2].w);
            if (COLOR) {
                // the colour cotangent and its product with the blended colour (kappa's colour part)
                float kc = 0.0f;
                if (local >= 0) {
                    const size_t r3 = 3 * ((size_t)vr.ray_off + local);
                    kc = fmaf(pr[3].x, I.color[r3], fmaf(pr[3].y, I.color[r3 + 1], pr[3].z * I.color[r3 + 2]));
                }
                rays[RW * q + 2] = make_float4(pr[3].x, pr[3].y, pr[3].z, kc);
            }
        }
        __syncthreads();
        // each ray tile's cone (centre direction and radius) and least normaliser, for the bound
        // that lets a wave pass over the tiles on which a Gaussian can neither weigh above FP32's
        // zero nor add a density above 2^kDensSkipLog2 (tile_bounds)
        for (int tt = wave; tt < nt; tt += NW) {
            int row, col;
            const bool ok = tile_local(vr, item.ray0 + tt, lane, row, col) >= 0;
            const float4 x0 = rays[RW * (64 * tt + lane)];
            const int db_flag = wave_any(rays[RW * (64 * tt + lane) + 1].y != 0.0f) ? 1 : 0;
            float c0 = wave_sum(ok ? x0.x : 0.0f), c1 = wave_sum(ok ? x0.y : 0.0f), c2 = wave_sum(ok ? x0.z : 0.0f);
            const float inv = rsq_(fmaf(c0, c0, fmaf(c1, c1, fmaf(c2, c2, kEpsN))));
            c0 *= inv;
            c1 *= inv;
            c2 *= inv;
            const float e0 = x0.x - c0, e1 = x0.y - c1, e2 = x0.z - c2;
            float rho = ok ? sqrtf(fmaf(e0, e0, fmaf(e1, e1, e2 * e2))) : 0.0f;
            float nmin = ok ? x0.w : INFINITY;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                rho = fmaxf(rho, __shfl_xor(rho, off, 64));
                nmin = fminf(nmin, __shfl_xor(nmin, off, 64));
            }
            if (lane == 0) {
                tcone[tt] = make_float4(c0, c1, c2, rho * (1.0f + 1e-4f) + 1e-6f);
                tnorm[tt] = nmin;
                tdb[tt] = db_flag;
            }
        }
        float aB1 = 0.0f, aB2 = 0.0f;
        unsigned db_any = 0;  // bit t: some ray of tile t has a density cotangent
        bool db_set = false;
        // A scene of more than BLOCK Gaussians is taken in rounds of BLOCK: each Gaussian of the
        // round is first bounded on the whole item (tile_bounds on a cone around all its tiles,
        // against their least normaliser), and only those that can matter on some tile are staged,
        // TG at a time, in scene order (slist: their scene-local indices); the others' records are
        // zero, as the per-tile bounds would have left them.  Smaller scenes take one round of all
        // their Gaussians in order (and launches without kBig, whose scenes are all small, have no
        // such rounds).
        const bool sparse = BIG && sr.n > BLOCK;
        for (int rb = 0; rb < sr.n; rb += sparse ? BLOCK : sr.n) {
          int total = sr.n;
          if (sparse) {
            __syncthreads();  // cones visible; the previous round's list and entries are consumed
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, inorm = INFINITY;
            for (int t = 0; t < nt; ++t) {
                s0 += tcone[t].x;
                s1 += tcone[t].y;
                s2 += tcone[t].z;
                inorm = fminf(inorm, tnorm[t]);
            }
            const float si = rsq_(fmaf(s0, s0, fmaf(s1, s1, fmaf(s2, s2, kEpsN))));
            s0 *= si;
            s1 *= si;
            s2 *= si;
            float irho = 0.0f;  // |v - c| <= |v - c_t| + |c_t - c| for a ray v of tile t
            for (int t = 0; t < nt; ++t) {
                const float4 ct = tcone[t];
                const float d0 = ct.x - s0, d1 = ct.y - s1, d2 = ct.z - s2;
                irho = fmaxf(irho, sqrtf(fmaf(d0, d0, fmaf(d1, d1, d2 * d2))) + ct.w);
            }
            const float4 icone = make_float4(s0, s1, s2, irho * (1.0f + 1e-4f) + 1e-6f);
            // the round's records start as zeros, written contiguously by all threads (the
            // survivors' are overwritten after the barriers below)
            {
                float *dst = partial + item.poff + REC * rb;
                const int nz = REC * min(BLOCK, sr.n - rb);
                for (int c = tid; c < nz; c += BLOCK) dst[c] = 0.0f;
            }
            const int gl = rb + tid;
            bool keep = false;
            if (gl < sr.n) {
                const int gg = sr.gauss_off + gl;
                float4 q[5];
                make_entry_est(P.means + 3 * gg, P.prec + 6 * gg, P.weights[gg], o, q);
                float d2_hi, z_hi;
                tile_bounds(ent_from(q[0], q[1], q[2], q[3]), q[4], icone, bl.hm, bl.b1, bl.nc2, d2_hi, z_hi);
                // (written so that a NaN bound keeps the Gaussian)
                keep = !(b1_pos && z_hi - inorm < kSkipLog2 && d2_hi < kDensSkipLog2);
            }
            const unsigned long long bal = wave_ballot(keep);
            if (lane == 0) wcnt[wave] = __popcll(bal);
            __syncthreads();
            int off = 0;
            total = 0;
            for (int w = 0; w < NW; ++w) {
                const int c = wcnt[w];
                off += w < wave ? c : 0;
                total += c;
            }
            if (keep) slist[off + __popcll(bal & ((1ull << lane) - 1ull))] = gl;
          }
          for (int gb = 0; gb < total; gb += TG) {
            const int cnt = min(TG, total - gb);
            __syncthreads();  // staged rays (and the list) visible; the previous tile's entries and sums are consumed
            for (int q = tid; q < cnt; q += BLOCK) {
                const int gi = sr.gauss_off + (sparse ? slist[gb + q] : gb + q);
                make_entry_est(P.means + 3 * gi, P.prec + 6 * gi, P.weights[gi], o, &ents[EW * q]);
                if (COLOR) ents[EW * q + 5] = colour_entry(P.colors + 3 * gi);
            }
            __syncthreads();
            if (!db_set) {  // (uniform: the first batch of the item)
                db_any = (unsigned)wave_ballot(lane < nt && tdb[lane] != 0);
                db_set = true;
            }
            // The wave takes Gaussians i0, i0 + NW, ... and bounds GPB of them on the item's tiles in
            // one pass (lane: tile lane % T of Gaussian i0 + (lane / T) NW), then walks them in order.
            constexpr int GPB = 64 / T;
            for (int i0 = wave; i0 < cnt; i0 += GPB * NW) {
              unsigned long long tmasks;  // bits [T k, T k + T): the tiles Gaussian i0 + k NW can matter on
              {
                const int ik = i0 + (lane / T) * NW, tl = lane % T;
                bool need = false;
                if (tl < nt && ik < cnt) {
                    const Ent gk = ent_from(ents[EW * ik], ents[EW * ik + 1], ents[EW * ik + 2], ents[EW * ik + 3]);
                    float d2_hi, z_hi;
                    tile_bounds(gk, ents[EW * ik + 4], tcone[tl], bl.hm, bl.b1, bl.nc2, d2_hi, z_hi);
                    // (written so that a NaN bound keeps the tile)
                    need = !(b1_pos && z_hi - tnorm[tl] < kSkipLog2 && d2_hi < kDensSkipLog2);
                }
                tmasks = wave_ballot(need);
              }
              for (int k = 0; k < GPB; ++k) {
                const int i = i0 + k * NW;
                if (i >= cnt) break;
                unsigned tmask = (unsigned)(tmasks >> (T * k));
                if (T < 32) tmask &= (1u << (T % 32)) - 1u;
                if (tmask == 0u) {
                    // no tile of the item takes a term of this Gaussian: its sums are zero
                    if (lane < LREC) rec[LREC * i + lane] = 0.0f;
                    continue;
                }
                const Ent g = ent_from(ents[EW * i], ents[EW * i + 1], ents[EW * i + 2], ents[EW * i + 3]);
                const float4 est = ents[EW * i + 4];
                float4 cc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (COLOR) cc = ents[EW * i + 5];
                OffsetAcc acc;
                float aC0 = 0.0f, aC1 = 0.0f, aC2 = 0.0f;  // colour sums: wt C_bar
#pragma unroll 1
                while (tmask) {
                    const int t = __builtin_ctz(tmask);
                    tmask &= tmask - 1;
                    const float4 x0 = rays[RW * (64 * t + lane)], x1 = rays[RW * (64 * t + lane) + 1];
                    Geo q;
                    const float vc = pair_geo_peak(g, x0.x, x0.y, x0.z, q);
                    {
                        // upper bounds of the log2 density and of the log2 weight from a lower bound
                        // of m (one FMA): a tile they put below both cutoffs everywhere is one the exact
                        // test below would skip, and it skips the residual as well
                        // (each vote on a single comparison; the tile's density-cotangent flag
                        // loosens the second to rays without one, which the exact test excludes)
                        const float d2_hi = fmaf(bl.hm, pair_m_low(est, vc, q.t), g.l2l);
                        const bool w_hi = !b1_pos || wave_any(fmaf(bl.b1, d2_hi, fmaf(bl.nc2, q.t, -x0.w)) >= kSkipLog2);
                        if (!w_hi && !(((db_any >> t) & 1u) && wave_any(d2_hi >= kDensSkipLog2))) continue;
                    }
                    pair_geo_resid(g, x0.x, x0.y, x0.z, bl.hm, bl.b1, bl.nc2, q);
                    // log2 of the normalised weight, and the density term D_bar delta
                    const float zr = fmaf(bl.b1, q.d2, fmaf(bl.nc2, q.t, -x0.w));
                    // a weight below 2^-150 rounds to zero in FP32, and a density below 2^kDensSkipLog2
                    // adds nothing measurable: such a tile skips the exponential and the adjoint
                    // (the density test only where no weight is left)
                    const bool any_w = wave_any(zr >= kSkipLog2);
                    if (any_w || wave_any(q.d2 >= kDensSkipLog2 && x1.y != 0.0f)) {
                        const float dd = x1.y * exp2_(q.d2);
                        // with zero weights on every ray of the tile only the density term remains:
                        // t_bar = 0, d_bar = D_bar delta (the offset form then adds exactly that)
                        float tb = 0.0f, db = dd;
                        if (any_w) {
                            // z_bar = wt (tf_bar t - kappa) with kappa = tf_bar t_f [+ C_bar . C, and
                            // C_bar . c added to the pair's share]
                            const float x = q.t - x1.w;
                            const float wt = exp2_(zr);
                            const float wtf = wt * x1.x;
                            float zb = wtf * x;
                            if (COLOR) {
                                const float4 x2 = rays[RW * (64 * t + lane) + 2];
                                zb = fmaf(wt, fmaf(x2.x, cc.x, fmaf(x2.y, cc.y, fmaf(x2.z, cc.z, -x2.w))), zb);
                                aC0 = fmaf(wt, x2.x, aC0);
                                aC1 = fmaf(wt, x2.y, aC1);
                                aC2 = fmaf(wt, x2.z, aC2);
                            }
                            tb = fmaf(-bl.cb, zb, wtf);
                            db = fmaf(bl.b1, zb, dd);
                            aB1 = fmaf(zb, q.d2 - x1.z, aB1);
                            aB2 = fmaf(zb, x, aB2);
                        }
                        // one accumulation for both cases, so the sums stay in their registers
                        pair_adjoint_offset(q, x0.x, x0.y, x0.z, tb, db, acc);
                    }
                }
                float v[16];
                offset_acc_store(acc, v);
                v[13] = aC0;
                v[14] = aC1;
                v[15] = aC2;
                static_assert(kOffsetAcc + 3 <= 16, "one 16-value wave sum per Gaussian");
                const float tot = wave_sum16(v, lane);
                const int idx = wave16_index(lane);
                if ((lane & 3) == 0 && idx < LREC) rec[LREC * i + idx] = tot;
              }
            }
            __syncthreads();
            for (int q = tid; q < cnt; q += BLOCK) {
                const int gl = sparse ? slist[gb + q] : gb + q;
                const int gg = sr.gauss_off + gl;
                write_partial_offset(partial + item.poff + REC * gl, rec + LREC * q, REC,
                                     P.prec + 6 * gg, P.means + 3 * gg, o);
            }
          }
        }
        // betas: lanes summed over the wave, then the waves in order
        aB1 = wave_sum(aB1);
        aB2 = wave_sum(aB2);
        if (lane == 0) {
            bsum[2 * wave] = aB1;
            bsum[2 * wave + 1] = aB2;
        }
        __syncthreads();
        if (tid < 2) {
            float sb = 0.0f;
            for (int w = 0; w < NW; ++w) sb += bsum[2 * w + tid];
            beta_partial[2 * item.seq + tid] = sb;
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

// First stage: block (group, slice) sums the values slice * BLOCK + tid, + BLOCK * slices, ...
// of a group's records (a record of a whole large scene spreads over many blocks).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void fin1_kernel(const FinGroup *__restrict__ groups,
                                                    const float *__restrict__ partial,
                                                    const float *__restrict__ beta_partial,
                                                    double *__restrict__ stage, double *__restrict__ stage_beta)
{
    const FinGroup gr = groups[blockIdx.x];
    const int tid = threadIdx.x;
    const int n = gr.item_end - gr.item_begin;
    for (int v = blockIdx.y * BLOCK + tid; v < gr.nval; v += BLOCK * gridDim.y)
        stage[gr.soff + v] = ordered_sum(partial + gr.poff + v, n, gr.nval);
    if (blockIdx.y == 0 && tid < 2)
        stage_beta[2 * blockIdx.x + tid] = ordered_sum(beta_partial + 2 * gr.item_begin + tid, n, 2);
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

// ------------------------------------------------------------------------------------
// Split statistic (Sec. 8): lbar_i = (1/M) sum_j L_j w_ji over a scene's M rays, w_ji the
// normalised blend weights of Eq. (3) (Eq. 7 here), read back from the forward pass's stash.
// Tiled like the backward (bwdt_kernel): an item is T ray tiles of one view against every
// Gaussian of its scene.  The rays are staged in LDS with M2 + log2 S (so that z2 minus it is the
// log2 of the normalised weight) and their loss value; each wave bounds GPB Gaussians at a time on
// the item's tiles (tile_bounds against the tile's least M2 + log2 S) and, for each Gaussian, sums
// L w over the rays of the tiles where some weight can be above FP32's zero (the one-FMA bound
// of m per pair first), then reduces over the wave into the item's record of one float per
// Gaussian.
// ------------------------------------------------------------------------------------

template <int BLOCK, int T, int TG>
__global__ __launch_bounds__(BLOCK) void statt_kernel(Params P, const float *__restrict__ loss,
                                                     const float *__restrict__ stash,
                                                     const BwdItem *__restrict__ items, float *__restrict__ partial)
{
    static_assert(T <= 32 && 64 % T == 0, "a 32-bit mask of the item's ray tiles, whole tile sets per wave");
    constexpr int NW = BLOCK / 64, RAYS = 64 * T, GPB = 64 / T;
    __shared__ float4 rays[RAYS];   // per ray: (v, M2 + log2 S)
    __shared__ float lossv[RAYS];   // per ray: its loss value
    __shared__ float4 tcone[T];     // per ray tile: unit centre direction, largest |v - c|
    __shared__ float tnorm[T];      // per ray tile: least M2 + log2 S over its rays
    __shared__ float4 ents[5 * TG];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const BwdItem item = ld_uniform(items + blockIdx.x);
    const ViewRec vr = ld_uniform(P.views + item.view);
    const SceneRec sr = ld_uniform(P.scenes + vr.scene);
    const CamRec cam = cam_of(P, item.view);
    const float *e = cam.e, *kk = cam.k;
    double o[3];
    cam_centre(e, o);
    const Blend bl = blend_of(P, vr.scene);
    const bool b1_pos = bl.b1 >= 0.0f;  // the weight bounds need beta1 >= 0
    const int nt = min(T, vr.tiles - item.ray0);  // the item's tiles: ray0 is its first tile

    for (int q = tid; q < RAYS; q += BLOCK) {
        int row = 0, col = 0;
        const int local = (q >> 6) < nt ? tile_local(vr, item.ray0 + (q >> 6), q & 63, row, col) : -1;
        float v0 = 0.0f, v1 = 0.0f, v2 = 1.0f, wo = INFINITY, lr = 0.0f;  // a ray past the edge weighs 0
        if (local >= 0) {
            tile_ray_dir(P, vr, e, kk, local, row, col, v0, v1, v2);
            const size_t r = (size_t)vr.ray_off + local;
            const float4 s0 = reinterpret_cast<const float4 *>(stash)[2 * r];
            wo = s0.x - __builtin_amdgcn_logf(s0.y);  // M2 + log2 S (s0.y = 1 / S)
            lr = loss[r];
        }
        rays[q] = make_float4(v0, v1, v2, wo);
        lossv[q] = lr;
    }
    __syncthreads();
    for (int tt = wave; tt < nt; tt += NW) {
        int row, col;
        const bool ok = tile_local(vr, item.ray0 + tt, lane, row, col) >= 0;
        const float4 x0 = rays[64 * tt + lane];
        float c0 = wave_sum(ok ? x0.x : 0.0f), c1 = wave_sum(ok ? x0.y : 0.0f), c2 = wave_sum(ok ? x0.z : 0.0f);
        const float inv = rsq_(fmaf(c0, c0, fmaf(c1, c1, fmaf(c2, c2, kEpsN))));
        c0 *= inv;
        c1 *= inv;
        c2 *= inv;
        const float e0 = x0.x - c0, e1 = x0.y - c1, e2 = x0.z - c2;
        float rho = ok ? sqrtf(fmaf(e0, e0, fmaf(e1, e1, e2 * e2))) : 0.0f;
        float nmin = ok ? x0.w : INFINITY;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            rho = fmaxf(rho, __shfl_xor(rho, off, 64));
            nmin = fminf(nmin, __shfl_xor(nmin, off, 64));
        }
        if (lane == 0) {
            tcone[tt] = make_float4(c0, c1, c2, rho * (1.0f + 1e-4f) + 1e-6f);
            tnorm[tt] = nmin;
        }
    }
    float *__restrict__ out = partial + item.poff;
    for (int gb = 0; gb < sr.n; gb += TG) {
        const int cnt = min(TG, sr.n - gb);
        __syncthreads();  // staged rays and cones visible; the previous tile's entries are consumed
        for (int q = tid; q < cnt; q += BLOCK) {
            const int gi = sr.gauss_off + gb + q;
            make_entry_est(P.means + 3 * gi, P.prec + 6 * gi, P.weights[gi], o, &ents[5 * q]);
        }
        __syncthreads();
        for (int i0 = wave; i0 < cnt; i0 += GPB * NW) {
            unsigned long long tmasks;  // bits [T k, T k + T): the tiles Gaussian i0 + k NW can weigh on
            {
                const int ik = i0 + (lane / T) * NW, tl = lane % T;
                bool need = false;
                if (tl < nt && ik < cnt) {
                    const Ent gk = ent_from(ents[5 * ik], ents[5 * ik + 1], ents[5 * ik + 2], ents[5 * ik + 3]);
                    float d2_hi, z_hi;
                    tile_bounds(gk, ents[5 * ik + 4], tcone[tl], bl.hm, bl.b1, bl.nc2, d2_hi, z_hi);
                    // (written so that a NaN bound keeps the tile)
                    need = !(b1_pos && z_hi - tnorm[tl] < kSkipLog2);
                }
                tmasks = wave_ballot(need);
            }
            for (int k = 0; k < GPB; ++k) {
                const int i = i0 + k * NW;
                if (i >= cnt) break;
                unsigned tmask = (unsigned)(tmasks >> (T * k));
                if (T < 32) tmask &= (1u << (T % 32)) - 1u;
                float acc = 0.0f;
                if (tmask != 0u) {
                    const Ent g = ent_from(ents[5 * i], ents[5 * i + 1], ents[5 * i + 2], ents[5 * i + 3]);
                    const float4 est = ents[5 * i + 4];
#pragma unroll 1
                    while (tmask) {
                        const int t = __builtin_ctz(tmask);
                        tmask &= tmask - 1;
                        const float4 x0 = rays[64 * t + lane];
                        Geo q;
                        const float vc = pair_geo_peak(g, x0.x, x0.y, x0.z, q);
                        if (b1_pos) {
                            // an upper bound of the log2 weight from a lower bound of m (one FMA)
                            const float d2_hi = fmaf(bl.hm, pair_m_low(est, vc, q.t), g.l2l);
                            if (!wave_any(fmaf(bl.b1, d2_hi, fmaf(bl.nc2, q.t, -x0.w)) >= kSkipLog2)) continue;
                        }
                        pair_geo_resid(g, x0.x, x0.y, x0.z, bl.hm, bl.b1, bl.nc2, q);
                        const float zr = fmaf(bl.b1, q.d2, fmaf(bl.nc2, q.t, -x0.w));
                        if (zr >= kSkipLog2) acc = fmaf(lossv[64 * t + lane], exp2_(zr), acc);
                    }
                    acc = wave_sum(acc);
                }
                if (lane == 0) out[gb + i] = acc;
            }
        }
    }
}

// lbar of one Gaussian of a (scene, chunk) per block: thread j adds the partial sums of items
// j, j + 256, ... in double, then a fixed tree over the threads, divided by the scene's ray
// count (the same order on every call).
__global__ __launch_bounds__(256) void stat_fin_kernel(Params P, const StatTask *__restrict__ tasks,
                                                      const BwdItem *__restrict__ items,
                                                      const float *__restrict__ partial,
                                                      const int64_t *__restrict__ rays_per_scene,
                                                      float *__restrict__ lbar)
{
    __shared__ double red[256];
    const StatTask t = tasks[blockIdx.x];
    const int g = blockIdx.y;
    if (g >= t.gc) return;  // uniform over the block
    double s = 0.0;
    for (int it = t.item_begin + (int)threadIdx.x; it < t.item_end; it += 256)
        s += (double)partial[items[it].poff + g];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const SceneRec sr = P.scenes[t.scene];
        lbar[sr.gauss_off + t.g0 + g] = (float)(red[0] / (double)rays_per_scene[t.scene]);
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
    // 64-bit ray index: the products flow_cols r and 3 r overflow int above 5.4e8 rays
    const int64_t r = (int64_t)blockIdx.x * kLossBlock + threadIdx.x;
    const float inv_p = 1.0f / (float)p;
    float l = 0.0f;
    if (r < p) {
        const float at = alpha_t[r];
        const float a = alpha[r];
        const float ac = fminf(fmaxf(a, 1e-6f), 1.0f - 1e-6f);
        const float dd = depth[r] - depth_t[r];
        float ga, gd;
        loss_grad_ray(a, at, depth[r], depth_t[r], w_depth, inv_p, ga, gd);
        g_alpha[r] = ga;
        g_depth[r] = gd;
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
// Backward variants: 0-2 the Gaussian-lane kernel with RT rays staged per pass; 3-5 the
// ray-lane kernel with (RPT rays per lane, TG Gaussians per tile).
static const int kBwdRT[] = {64, 128, 256};
struct BwdRayVariant {
    int rpt, tg;
};
static const BwdRayVariant kBwdRay[] = {{2, 64}, {4, 64}, {4, 128}};
constexpr int kNumBwdGauss = (int)(sizeof kBwdRT / sizeof kBwdRT[0]);
constexpr int kNumBwdRay = (int)(sizeof kBwdRay / sizeof kBwdRay[0]);
// Variants 6-8: the tiled ray-lane kernel with T ray tiles per item (Gaussians staged 64 at a time);
// without a normal cotangent only (the host runs variant 2 for that).
// (256 threads per block for variants 6 and 7; variant 8 has eight waves share an item's 16 staged
// tiles, 512 threads)
static const int kBwdTiles[] = {8, 16, 16};
constexpr int kNumBwdTiled = (int)(sizeof kBwdTiles / sizeof kBwdTiles[0]);
constexpr int kBwdTiledFirst = kNumBwdGauss + kNumBwdRay;

// F dispatch: calls body<F>() for the runtime flag set f (0..15).
#define FMB_DISPATCH_F(f, CALL)                                                                            \
    switch (f) {                                                                                           \
    case 0: CALL(0); break;   case 1: CALL(1); break;   case 2: CALL(2); break;   case 3: CALL(3); break;   \
    case 4: CALL(4); break;   case 5: CALL(5); break;   case 6: CALL(6); break;   case 7: CALL(7); break;   \
    case 8: CALL(8); break;   case 9: CALL(9); break;   case 10: CALL(10); break; case 11: CALL(11); break; \
    case 12: CALL(12); break; case 13: CALL(13); break; case 14: CALL(14); break; case 15: CALL(15); break; \
    default: return hipErrorInvalidValue;                                                                  \
    }

// ... and over the forward's flag sets with kBig (16..31).
#define FMB_DISPATCH_F32(f, CALL)                                                                          \
    if ((f) < 16) {                                                                                        \
        FMB_DISPATCH_F(f, CALL)                                                                            \
    } else {                                                                                               \
        switch (f) {                                                                                       \
        case 16: CALL(16); break; case 17: CALL(17); break; case 18: CALL(18); break; case 19: CALL(19); break; \
        case 20: CALL(20); break; case 21: CALL(21); break; case 22: CALL(22); break; case 23: CALL(23); break; \
        case 24: CALL(24); break; case 25: CALL(25); break; case 26: CALL(26); break; case 27: CALL(27); break; \
        case 28: CALL(28); break; case 29: CALL(29); break; case 30: CALL(30); break; case 31: CALL(31); break; \
        default: return hipErrorInvalidValue;                                                              \
        }                                                                                                  \
    }

template <int RPT, int TG>
static hipError_t launch_fwd_v(int f, int grid, hipStream_t st, const Params &P, const FwdOut &O,
                               const FwdItem *items, int n, const int *order, int *counter)
{
#define FMB_FWD_CALL(F)                                                                                    \
    hipLaunchKernelGGL((fwd_kernel<kBlock, RPT, TG, F>), dim3(grid), dim3(kBlock), 0, st, P, O, items, n, order, \
                       counter)
    FMB_DISPATCH_F32(f, FMB_FWD_CALL)
#undef FMB_FWD_CALL
    return hipGetLastError();
}

template <int RPT, int TG>
static hipError_t launch_bwdr_v(int f, int grid, hipStream_t st, const Params &P, const BwdIn &I,
                                const BwdItem *items, int n, const int *order, int *counter, float *partial,
                                float *bpart)
{
#define FMB_BWDR_CALL(F)                                                                                   \
    hipLaunchKernelGGL((bwdr_kernel<kBlock, RPT, TG, F>), dim3(grid), dim3(kBlock), 0, st, P, I, items, n,      \
                       order, counter, partial, bpart)
    FMB_DISPATCH_F(f, FMB_BWDR_CALL)
#undef FMB_BWDR_CALL
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

template <int BLK, int T>
static hipError_t launch_bwdt_v(int f, int grid, hipStream_t st, const Params &P, const BwdIn &I,
                                const BwdItem *items, int n, const int *order, int *counter, float *partial,
                                float *bpart)
{
#define FMB_BWDT_CALL(F)                                                                                   \
    hipLaunchKernelGGL((bwdt_kernel<BLK, T, 64, F>), dim3(grid), dim3(BLK), 0, st, P, I, items, n, order,   \
                       counter, partial, bpart)
    switch (f) {
    case 0: FMB_BWDT_CALL(0); break;
    case kFlw: FMB_BWDT_CALL(kFlw); break;
    case kPer: FMB_BWDT_CALL(kPer); break;
    case kFlw | kPer: FMB_BWDT_CALL(kFlw | kPer); break;
    case kCol: FMB_BWDT_CALL(kCol); break;
    case kCol | kFlw: FMB_BWDT_CALL(kCol | kFlw); break;
    case kCol | kPer: FMB_BWDT_CALL(kCol | kPer); break;
    case kCol | kFlw | kPer: FMB_BWDT_CALL(kCol | kFlw | kPer); break;
    case kBig: FMB_BWDT_CALL(kBig); break;
    case kBig | kFlw: FMB_BWDT_CALL(kBig | kFlw); break;
    case kBig | kPer: FMB_BWDT_CALL(kBig | kPer); break;
    case kBig | kFlw | kPer: FMB_BWDT_CALL(kBig | kFlw | kPer); break;
    case kBig | kCol: FMB_BWDT_CALL(kBig | kCol); break;
    case kBig | kCol | kFlw: FMB_BWDT_CALL(kBig | kCol | kFlw); break;
    case kBig | kCol | kPer: FMB_BWDT_CALL(kBig | kCol | kPer); break;
    case kBig | kCol | kFlw | kPer: FMB_BWDT_CALL(kBig | kCol | kFlw | kPer); break;
    default: return hipErrorInvalidValue;
    }
#undef FMB_BWDT_CALL
    return hipGetLastError();
}

int num_fwd_variants() { return (int)(sizeof kFwdVariants / sizeof kFwdVariants[0]); }
int fwd_variant_rays(int v) { return kBlock * kFwdVariants[v].rpt; }
int num_bwd_variants() { return kNumBwdGauss + kNumBwdRay + kNumBwdTiled; }
// Tiled variants 6-8: ray tiles per item (0 for the others); they take no normal cotangent.
int bwd_variant_tiles(int v) { return v >= kBwdTiledFirst && v < num_bwd_variants() ? kBwdTiles[v - kBwdTiledFirst] : 0; }
// Gaussian-lane variants: rays staged per pass; others: 0.
int bwd_variant_rt(int v) { return v < kNumBwdGauss ? kBwdRT[v] : 0; }
// Ray-lane variants 3-5: rays per block tile (BLOCK * RPT); others: 0.
int bwd_variant_ray_tile(int v) { return v >= kNumBwdGauss ? kBlock * kBwdRay[v - kNumBwdGauss].rpt : 0; }
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
    case 3: return launch_bwdr_v<2, 64>(flags, grid, st, P, I, items, n, order, counter, partial, bpart);
    case 4: return launch_bwdr_v<4, 64>(flags, grid, st, P, I, items, n, order, counter, partial, bpart);
    case 5: return launch_bwdr_v<4, 128>(flags, grid, st, P, I, items, n, order, counter, partial, bpart);
    case 6: return launch_bwdt_v<256, 8>(flags, grid, st, P, I, items, n, order, counter, partial, bpart);
    case 7: return launch_bwdt_v<256, 16>(flags, grid, st, P, I, items, n, order, counter, partial, bpart);
    case 8: return launch_bwdt_v<512, 16>(flags, grid, st, P, I, items, n, order, counter, partial, bpart);
    default: return hipErrorInvalidValue;
    }
}

// max_gc: the largest chunk of any task (a whole scene for the ray-lane backward); max_nval: the
// largest first-stage record of any group.
hipError_t launch_fin(int n_tasks, int n_groups, int max_gc, int max_nval, hipStream_t st, const Params &P,
                      const FinTask *tasks, const FinGroup *groups, const float *partial, const float *bpart,
                      double *stage, double *stage_beta, float *g_means, float *g_prec, float *g_weights,
                      float *g_colors, float *g_betas)
{
    if (max_gc < 1 || max_nval < 1) return hipErrorInvalidValue;
    const int slices = (max_nval + 255) / 256 < 65535 ? (max_nval + 255) / 256 : 65535;
    hipLaunchKernelGGL((fin1_kernel<256>), dim3(n_groups, slices), dim3(256), 0, st, groups, partial, bpart, stage,
                       stage_beta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int gslices = (max_gc + kFinSlice - 1) / kFinSlice;
    if (gslices > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((fin2_kernel<256>), dim3(n_tasks, gslices), dim3(256), 0, st, P, tasks, groups, stage,
                       stage_beta, g_means, g_prec, g_weights, g_colors, g_betas);
    return hipGetLastError();
}

hipError_t launch_stat(int n_items, int n_tasks, int max_gc, hipStream_t st, const Params &P, const float *loss,
                       const float *stash, const BwdItem *items, const StatTask *tasks, float *partial,
                       const int64_t *rays_per_scene, float *lbar)
{
    if (n_items > 0)
        hipLaunchKernelGGL((statt_kernel<512, kStatTiles, 64>), dim3(n_items), dim3(512), 0, st, P, loss, stash, items,
                           partial);
    if (n_tasks > 0)
        hipLaunchKernelGGL(stat_fin_kernel, dim3(n_tasks, max_gc), dim3(256), 0, st, P, tasks, items, partial,
                           rays_per_scene, lbar);
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
        FMB_DISPATCH_F32(flags, FMB_OCC_F)                                                                 \
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
    default: break;
    }
#undef FMB_OCC_V
#undef FMB_OCC_F
#define FMB_OCC_F(F) return occ(bwdr_kernel<kBlock, RPT, TG, F>, blocks_per_cu)
#define FMB_OCC_V(RPT_, TG_)                                                                               \
    {                                                                                                      \
        constexpr int RPT = RPT_, TG = TG_;                                                                \
        FMB_DISPATCH_F(flags, FMB_OCC_F)                                                                   \
    }
    switch (variant) {
    case 3: FMB_OCC_V(2, 64)
    case 4: FMB_OCC_V(4, 64)
    case 5: FMB_OCC_V(4, 128)
    default: break;
    }
#undef FMB_OCC_V
#undef FMB_OCC_F
    auto occb = [&](auto kernel, int blk) { return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kernel, blk, 0); };
    // the persistent forms the batch launches (flow, colour and the large-scene form as given)
#define FMB_OCC_T(BLK, T)                                                                                  \
    switch (flags & (kFlw | kCol | kBig)) {                                                                \
    case 0: return occb(bwdt_kernel<BLK, T, 64, kPer>, BLK);                                              \
    case kFlw: return occb(bwdt_kernel<BLK, T, 64, kFlw | kPer>, BLK);                                    \
    case kCol: return occb(bwdt_kernel<BLK, T, 64, kCol | kPer>, BLK);                                    \
    case kCol | kFlw: return occb(bwdt_kernel<BLK, T, 64, kCol | kFlw | kPer>, BLK);                      \
    case kBig: return occb(bwdt_kernel<BLK, T, 64, kBig | kPer>, BLK);                                    \
    case kBig | kFlw: return occb(bwdt_kernel<BLK, T, 64, kBig | kFlw | kPer>, BLK);                      \
    case kBig | kCol: return occb(bwdt_kernel<BLK, T, 64, kBig | kCol | kPer>, BLK);                      \
    default: return occb(bwdt_kernel<BLK, T, 64, kBig | kCol | kFlw | kPer>, BLK);                        \
    }
    if (variant == 6) FMB_OCC_T(256, 8)
    if (variant == 7) FMB_OCC_T(256, 16)
    if (variant == 8) FMB_OCC_T(512, 16)
#undef FMB_OCC_T
    return hipErrorInvalidValue;
}

}  // namespace fmb
