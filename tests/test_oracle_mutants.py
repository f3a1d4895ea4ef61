"""Planted mistakes in copies of the oracle: each must fail at least one pin.

Every mutant is a one-line slip of the kind a reimplementation makes (a sign, a
transposed operand, a dropped factor or term, a swapped index).  The copy is built
in a temporary directory; the committed oracle is never modified.
"""

import os
import subprocess

import pytest

import oracle as O
from tests import oracle_pins as P

SRC = os.path.join(os.path.dirname(O.lib_path()), "fmb_oracle.c")

MUTANTS = {
    "beta2_sign": ("q->z = b1 * q->d - (b2 / eta) * q->t;", "q->z = b1 * q->d + (b2 / eta) * q->t;"),
    "eta_times": ("q->z = b1 * q->d - (b2 / eta) * q->t;", "q->z = b1 * q->d - (b2 * eta) * q->t;"),
    "precision_UUt": ("s += U[k * 3 + a] * U[k * 3 + b];", "s += U[a * 3 + k] * U[b * 3 + k];"),
    "half_dropped": ("q->d = g->loglam - 0.5 * q->m;", "q->d = g->loglam - q->m;"),
    "flow_sign": ("ry->flow[0] = ub[0] - ua[0];", "ry->flow[0] = ua[0] - ub[0];"),
    "pixel_centre": ("((double)col[r] + 0.5 - k[2]) / k[0]", "((double)col[r] - k[2]) / k[0]"),
    "fx_fy_swap": ("((double)row[r] + 0.5 - k[3]) / k[1]", "((double)row[r] + 0.5 - k[3]) / k[0]"),
    "unweighted_normal": ("r->N[a] += wt[i] * q[i].n[a];", "r->N[a] += q[i].n[a];"),
    "weighted_density": ("r->D += q[i].delta;", "r->D += wt[i] * q[i].delta;"),
    "centre_R_not_RT": ("c[a] = -(e[0 * 4 + a] * e[3] + e[1 * 4 + a] * e[7] + e[2 * 4 + a] * e[11]);",
                        "c[a] = -(e[a * 4 + 0] * e[3] + e[a * 4 + 1] * e[7] + e[a * 4 + 2] * e[11]);"),
    "adj_den_dropped": ("+ den_bar * v[a] * v[b];", ";"),
    "adj_beta1_uses_t": ("gb[0] += z_bar * pq->d;", "gb[0] += z_bar * pq->t;"),
    "adj_normal_projection_dropped": ("g_bar[a] = (n_bar[a] - pq->n[a] * sg) / pq->gn;",
                                      "g_bar[a] = n_bar[a] / pq->gn;"),
    "adj_softmax_mean_dropped": ("double z_bar = wt[i] * (w_bar - mean_wbar);",
                                 "double z_bar = wt[i] * w_bar;"),
    "adj_flow_rows_swapped": ("gfl[0] * (Jb[a] - Ja[a]) + gfl[1] * (Jb[3 + a] - Ja[3 + a])",
                              "gfl[1] * (Jb[a] - Ja[a]) + gfl[0] * (Jb[3 + a] - Ja[3 + a])"),
    "colour_unweighted": ("for (int a = 0; a < 3; ++a) r->C[a] += wt[i] * g[i].col[a];",
                          "for (int a = 0; a < 3; ++a) r->C[a] += g[i].col[a];"),
    "adj_colour_no_sigmoid_slope": ("s.col[j] * g[i].col[j] * (1.0 - g[i].col[j])", "s.col[j]"),
    "adj_U_fold_transposed": ("t += g[i].U[a * 3 + k] * Bs[k * 3 + b];",
                              "t += g[i].U[k * 3 + a] * Bs[k * 3 + b];"),
    "composite_non_strict": ("if (q[j].t < q[i].t) before += q[j].delta;",
                             "if (q[j].t <= q[i].t) before += q[j].delta;"),
    "composite_back_to_front": ("if (q[j].t < q[i].t) before += q[j].delta;",
                                "if (q[j].t > q[i].t) before += q[j].delta;"),
    "composite_density_not_opacity": ("q[i].z = -before + log_opacity(q[i].delta, q[i].d);",
                                      "q[i].z = -before + q[i].d;"),
    "composite_tiny_branch_drops_d": ("return delta < 1e-300 ? d : log(-expm1(-delta));",
                                      "return delta < 1e-300 ? 0.0 : log(-expm1(-delta));"),
    "adj_composite_wrong_side": ("if (pq->t < q[k].t) later += zbar[k];",
                                 "if (pq->t > q[k].t) later += zbar[k];"),
    "adj_composite_slope_dropped": ("d_bar = z_bar * log_opacity_slope(pq->delta);", "d_bar = z_bar;"),
    "split_mean_over_gaussians": ("lbar[i] = s / (double)p;", "lbar[i] = s / (double)n;"),
    "dir_rays_unnormalised": ("double nn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);", "double nn = 1.0;"),
    "dir_rays_first_view": ("cam_centre(w2c + 12 * (int64_t)view[r], orig + 3 * r);", "cam_centre(w2c, orig + 3 * r);"),
    "split_unweighted": ("acc[(size_t)tid * n + i] += loss[r] * wt[i];", "acc[(size_t)tid * n + i] += loss[r];"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    c = tmp_path / f"{name}.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", str(so), str(c),
                    "-lm"], check=True)
    return str(so)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, oracle_lib, name):
    old, new = MUTANTS[name]
    so = _build_mutant(tmp_path, name, old, new)
    prev = O.oracle.use_library(so)
    caught = []
    try:
        for pin in P.ALL_PINS:
            try:
                pin()
            except (AssertionError, ValueError, FloatingPointError, ZeroDivisionError):
                caught.append(pin.__name__)
                break
    finally:
        O.oracle.restore_library(prev)
    assert caught, f"planted mistake {name!r} passed every pin"
