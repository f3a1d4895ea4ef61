// fmb_split.cpp -- host-side removal and splitting of Gaussians (Sec. 8).
//
// Runs once per optimisation stage on the n Gaussians (no rays), so it is plain double
// precision host code on host arrays.  The GPU part of the procedure, the per-Gaussian mean
// loss over a batch of rays, is fmb_split_statistic.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "fmb.h"

namespace {

void mean_std(int32_t n, const float *x, double &mean, double &sd)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += x[i];
    mean = s / n;
    double v = 0.0;
    for (int32_t i = 0; i < n; ++i) v += (x[i] - mean) * (x[i] - mean);
    sd = sqrt(v / n);
}

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations: a = V diag(w) V^T,
// eigenvectors in the columns of V.
void sym_eig3(const double a_in[9], double w[3], double V[9])
{
    double a[9];
    memcpy(a, a_in, sizeof a);
    for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        const double diag = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = a[3 * p + q];
                if (apq == 0.0) continue;
                const double theta = (a[3 * q + q] - a[3 * p + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                // a <- J^T a J with the rotation J in the (p, q) plane
                for (int k = 0; k < 3; ++k) {
                    const double akp = a[3 * k + p], akq = a[3 * k + q];
                    a[3 * k + p] = c * akp - s * akq;
                    a[3 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = a[3 * p + k], aqk = a[3 * q + k];
                    a[3 * p + k] = c * apk - s * aqk;
                    a[3 * q + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[3 * k + p], vkq = V[3 * k + q];
                    V[3 * k + p] = c * vkp - s * vkq;
                    V[3 * k + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < 3; ++i) w[i] = a[4 * i];
}

// Upper-triangular U with positive diagonal and U^T U = a (a symmetric positive definite).
bool upper_factor(const double a[9], double u[6])
{
    // a = L L^T with L lower, then U = L^T
    const double l00 = sqrt(a[0]);
    if (!(l00 > 0.0)) return false;
    const double l10 = a[3] / l00, l20 = a[6] / l00;
    const double d1 = a[4] - l10 * l10;
    if (!(d1 > 0.0)) return false;
    const double l11 = sqrt(d1);
    const double l21 = (a[7] - l20 * l10) / l11;
    const double d2 = a[8] - l20 * l20 - l21 * l21;
    if (!(d2 > 0.0)) return false;
    const double l22 = sqrt(d2);
    u[0] = l00;
    u[1] = l10;
    u[2] = l20;
    u[3] = l11;
    u[4] = l21;
    u[5] = l22;
    return true;
}

}  // namespace

extern "C" {

int fmb_prune_mask(int32_t n, const float *weights, float z, uint8_t *remove)
{
    if (n < 1 || !weights || !remove) return FMB_ERR_INVALID_ARG;
    double mean, sd;
    mean_std(n, weights, mean, sd);
    const double lim = mean - (double)z * sd;
    for (int32_t i = 0; i < n; ++i) remove[i] = (double)weights[i] <= lim ? 1 : 0;
    return FMB_OK;
}

int fmb_split_mask(int32_t n, const float *lbar, float z, uint8_t *split)
{
    if (n < 1 || !lbar || !split) return FMB_ERR_INVALID_ARG;
    double mean, sd;
    mean_std(n, lbar, mean, sd);
    const double lim = mean + (double)z * sd;
    for (int32_t i = 0; i < n; ++i) split[i] = (double)lbar[i] >= lim ? 1 : 0;
    return FMB_OK;
}

int fmb_split_gaussians(int32_t n, const float *means, const float *prec, const float *weights,
                        const float *colors, const float *noise_w, const float *noise_c, float *out_means,
                        float *out_prec, float *out_weights, float *out_colors)
{
    if (n < 0 || (n > 0 && (!means || !prec || !weights || !noise_w || !out_means || !out_prec || !out_weights)))
        return FMB_ERR_INVALID_ARG;
    if ((colors == nullptr) != (out_colors == nullptr) || (colors && !noise_c)) return FMB_ERR_INVALID_ARG;
    const double shift = sqrt(2.0 / M_PI), shrink = sqrt(1.0 - 2.0 / M_PI);
    for (int32_t i = 0; i < n; ++i) {
        const float *u = prec + 6 * (size_t)i;
        // Sigma^-1 = U^T U, U upper triangular (packed row-major)
        const double U[9] = {u[0], u[1], u[2], 0.0, u[3], u[4], 0.0, 0.0, u[5]};
        double A[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += U[3 * k + r] * U[3 * k + c];
                A[3 * r + c] = s;
            }
        // eigenvalues of Sigma^-1 are 1 / sigma_k^2; the dominant axis has the smallest one
        double w[3], V[9];
        sym_eig3(A, w, V);
        int k1 = 0;
        for (int k = 1; k < 3; ++k)
            if (w[k] < w[k1]) k1 = k;
        if (!(w[k1] > 0.0)) return FMB_ERR_INVALID_ARG;
        double v1[3] = {V[k1], V[3 + k1], V[6 + k1]};
        // sign convention: the largest-magnitude component of v1 is positive
        int big = 0;
        for (int k = 1; k < 3; ++k)
            if (fabs(v1[k]) > fabs(v1[big])) big = k;
        if (v1[big] < 0.0)
            for (double &x : v1) x = -x;
        const double sigma1 = 1.0 / sqrt(w[k1]);
        // children share Sigma' = Sigma with sigma1 scaled by sqrt(1 - 2/pi):
        // Sigma'^-1 = A + (1/(shrink^2) - 1) w1 v1 v1^T
        double A2[9];
        const double extra = (1.0 / (shrink * shrink) - 1.0) * w[k1];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) A2[3 * r + c] = A[3 * r + c] + extra * v1[r] * v1[c];
        double u2[6];
        if (!upper_factor(A2, u2)) return FMB_ERR_INVALID_ARG;
        for (int child = 0; child < 2; ++child) {
            const size_t o = 2 * (size_t)i + child;
            const double sgn = child == 0 ? 1.0 : -1.0;
            for (int a = 0; a < 3; ++a)
                out_means[3 * o + a] = (float)((double)means[3 * (size_t)i + a] + sgn * sigma1 * shift * v1[a]);
            for (int a = 0; a < 6; ++a) out_prec[6 * o + a] = (float)u2[a];
            out_weights[o] = (float)((double)weights[i] * exp((double)noise_w[o]));
            if (colors)
                for (int a = 0; a < 3; ++a)
                    out_colors[3 * o + a] = (float)((double)colors[3 * (size_t)i + a] + (double)noise_c[3 * o + a]);
        }
    }
    return FMB_OK;
}

}  // extern "C"
