"""Benchmark: ray x Gaussian pairs per second, forward + backward, batched vs plain.

One step is one pass of the whole hot path over the uneven 16-scene batch
(N ~ U{10..100} Gaussians, 4..32 views of 64^2 / 128^2 / 256^2 per scene, seed 3):
forward render (depth, alpha, normals) of every pixel ray against every Gaussian of
its scene, the loss cotangents (alpha-weighted L1 depth + BCE alpha against targets
rendered from a perturbed copy of each scene), and the adjoint pass producing the
gradients of means, precision factors, weights and both blend parameters.

The timed value replays one HIP graph of the whole step (persistent forward kernel, loss
cotangents, persistent backward + finalize kernels), captured from the stream the library
calls run on; the batch's own captured forward and backward graphs are timed too.  The same
steps are also timed with one plain launch sequence per scene (`plain_value`).  Kernel
durations for the roofline come from HIP events recorded around each kernel launch on its
stream.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic floating-point operations per (ray, Gaussian) pair, counted from the
# method's per-pair formulas (add/sub/mul/compare = 1, fused multiply-add = 2, exp /
# reciprocal / rsqrt = 1), excluding the backward's recomputation of the forward pair
# terms and the extra precision steps (hi/lo mean, Newton refinement of the peak).
FLOPS_FWD_NORMALS = 76     # intersection, density, weight, online blend, normal blend
FLOPS_FWD_PLAIN = 54       # without the normal terms
FLOPS_ADJ_NORMALS = 92     # adjoint with a normal cotangent
FLOPS_ADJ_PLAIN = 61       # adjoint of depth/alpha/flow cotangents only
# Zero-parameter (alpha-compositing) kernels, counted as the sort-based method computes them: per
# pair the same geometry as the blend model up to the density, the log opacity log(1 - exp(-delta))
# instead of the blend exponent and the normal blend (81); per ray a comparison sort of its N
# intersections (N ceil(log2 N) compares) and an exclusive prefix sum of the densities (N adds) for
# the transmittances.  The backward's adjoint per pair (73, with the opacity slope) adds the suffix
# sum of z_bar over the intersections behind (1 add per pair) and reuses the forward's order.
FLOPS_COMP_FWD_NORMALS = 81   # + ceil(log2 N) + 1 per pair
FLOPS_COMP_ADJ_PLAIN = 73     # + 1 per pair
# The paper's GPU timing of a whole iteration (forward and backward, 40 Gaussians): 377.6 ns per
# ray with alpha compositing against 226.6 ns with the weighted blend (Tab. 2).
PAPER_COMP_OVER_BLEND = 377.6 / 226.6
PEAK_FP32 = 157.3e12       # MI355X FP32 vector peak (published; 256 CUs x 128 FMA lanes x 2.4 GHz)


KERNEL_SOURCES = ("fmb_kernels.hip", "fmb_device.h", "fmb_internal.h", "fmb_api.cpp")


def kernel_source_sha256():
    """SHA-256 over the sources of the blend-model kernels and of the work items they are launched
    over (the host code that cuts items), in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2308_14737_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def bwd_kernel_name(variant):
    """The backward kernel a backward tile variant launches (the variant tables of the library)."""
    if variant < 3:
        return "bwd_kernel (persistent, Gaussian lanes)"
    if variant < 6:
        return "bwdr_kernel (persistent, ray lanes)"
    return "bwdt_kernel (persistent, 8x8 ray tiles per wave)"


def _profile_values(name, bwd_variant):
    """key: value lines of a committed rocprofv3 summary under profiles/, or {} if the kernel
    sources have changed since it was taken or it covers another backward variant."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        vals = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith(("#", "|", " ")):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
        if vals.get("kernel_source_sha256") != kernel_source_sha256() or \
                vals.get("bwd_variant") != str(bwd_variant):
            return {}
        return vals
    except OSError:
        return {}


def measured_traffic(bwd_variant):
    """HBM bytes per launch of the persistent backward kernel, from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, if it was taken of this variant's kernel as it is now."""
    try:
        return float(_profile_values("batch16_bwd_traffic.md", bwd_variant)["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def executed(pairs, bwd_ms, bwd_variant):
    """FP32 arithmetic the backward kernel executes per pair (rocprofv3 counters, including the
    recomputed pair terms), and the resulting rate, if the committed counters are current."""
    vals = _profile_values("batch16_valu.md", bwd_variant)
    try:
        fl = float(vals["bwd_executed_flops_per_pair"])
    except (KeyError, ValueError):
        return {"executed_flops_per_pair": None, "executed_frac": None}
    return {"executed_flops_per_pair": fl, "executed_frac": pairs * fl / (bwd_ms * 1e-3) / PEAK_FP32}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches only")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the colour, two-way flow and split-statistic legs")
    ap.add_argument("--no-composite", action="store_true",
                    help="skip the alpha-compositing (zero-parameter) leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy a 256 MiB buffer once (a kernel of known traffic for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def host_cpu():
    """CPU model, logical CPUs of the host and those this process may use (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(w, seconds):
    """Time the FP64 oracle (as it stands) on the same workload, scene after scene (passes over
    the batch repeated) until about `seconds` of work; returns pairs/s of forward + backward."""
    import numpy as np

    import oracle as O
    # the threads OpenMP is given (OMP_NUM_THREADS where it is set, e.g. a host's CPU share per
    # GPU), else every core this process may run on
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = max(1, min(int(os.environ.get("OMP_NUM_THREADS") or avail), avail))
    pairs = scenes = 0
    g = np.random.Generator(np.random.PCG64(9))
    t0 = time.perf_counter()
    while time.perf_counter() - t0 <= seconds:
        for sc, cams in zip(w.scenes, w.cameras):
            cot = {"depth": g.standard_normal(cams.n_rays), "alpha": g.standard_normal(cams.n_rays),
                   "normal": None, "flow": None}
            O.render_workload_view(sc, cams, w.betas, w.eta, n_threads=threads, cot=cot)
            pairs += cams.n_rays * sc.n
            scenes += 1
            if time.perf_counter() - t0 > seconds:
                break
    dt = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "host": host_cpu(), "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"),
            "sample": f"FP64 oracle forward (depth, alpha, normals) + backward (depth and alpha "
                      f"cotangents), all rays of {scenes} scenes taken in order, passes over the "
                      f"16-scene batch repeated: {pairs} pairs in {dt:.2f} s on {threads} threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (sharding the rays or "
              "scenes across GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2308_14737_amd as fmb
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = W.make_config("batch16")
    S = len(w.scenes)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev).contiguous()  # noqa: E731

    def batch_of(scenes):
        means = t(np.concatenate([s.means for s in scenes]))
        prec = t(np.concatenate([s.prec for s in scenes]))
        weights = t(np.concatenate([s.weights for s in scenes]))
        betas = t(np.tile(w.betas, (S, 1)))
        cams = [fmb.Cameras.from_numpy(c.w2c, c.intr, c.hw, device=dev) for c in w.cameras]
        return fmb.Batch(means, prec, weights, betas, [w.eta] * S, [s.n for s in scenes], cams), \
            (means, prec, weights, betas)

    batch, params = batch_of(w.scenes)
    P = batch.n_rays
    pairs = w.n_pairs
    print(f"# workload batch16: S={S} rays={P} pairs/step={pairs}", file=sys.stderr, flush=True)

    # targets from the perturbed scenes (setup, untimed)
    tb, _ = batch_of(w.targets)
    tgt = tb.forward(tb.alloc_outputs(normals=False))
    torch.cuda.synchronize()
    d_t, a_t = tgt["depth"].clone(), tgt["alpha"].clone()
    del tb, tgt

    outs = batch.alloc_outputs(normals=True)
    grads = batch.alloc_grads()
    cot = {"depth": torch.empty(P, device=dev), "alpha": torch.empty(P, device=dev),
           "normal": None, "flow": None}

    def cotangents(o):
        # L = mean(alpha_t |depth - depth_t|) + mean(BCE(clamp(alpha), alpha_t)); one HIP kernel
        fmb.loss_grad(o, d_t, a_t, cot=cot)

    # eager warm-up builds the item lists; then tune the tile variants on this batch
    batch.forward(outs)
    cotangents(outs)
    batch.backward(outs, cot, grads)
    torch.cuda.synchronize()
    if not args.no_autotune:
        batch.autotune(outs, cot, grads)
        torch.cuda.synchronize()

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    # same steps, eager persistent launches, with HIP-event kernel timing
    def step_eager():
        # the forward writes the loss's depth and alpha cotangents in its per-ray epilogue (the
        # values the loss kernel would write), then the backward
        batch.forward_loss(outs, d_t, a_t, cot)
        batch.backward(outs, cot, grads)

    for _ in range(args.warmup):
        step_eager()
    fmb.timing_enable(True)
    fmb.kernel_times(reset=True)
    ms_eager = timed(step_eager, args.steps) * 1e3
    kt = fmb.kernel_times(reset=True)
    fmb.timing_enable(False)
    fwd_ms = kt["fwd_ms"] / max(kt["n_fwd"], 1)
    bwd_ms = kt["bwd_ms"] / max(kt["n_bwd"], 1)
    fin_ms = kt["fin_ms"] / max(kt["n_fin"], 1)
    print(f"# eager step {ms_eager:.3f} ms; kernels fwd {fwd_ms:.3f} bwd {bwd_ms:.3f} fin {fin_ms:.3f} ms",
          file=sys.stderr, flush=True)

    # the same steps replayed from graphs (after the eager leg, so that they run on a GPU that
    # has been busy for a while): the batch's own captured forward and backward graphs, then
    # one graph of the whole step
    ms_graph = ms_graph_api = None
    if not args.no_graph:
        st = torch.cuda.Stream(dev)
        torch.cuda.synchronize()
        batch.capture(outs, cot, grads, st)

        def step_graph():
            batch.graph_launch(0, st)
            with torch.cuda.stream(st):
                cotangents(outs)
            batch.graph_launch(1, st)

        for _ in range(args.warmup):
            step_graph()
        ms_graph_api = timed(step_graph, args.steps) * 1e3
        print(f"# library graphs (forward, backward; loss kernel between) {ms_graph_api:.3f} ms",
              file=sys.stderr, flush=True)

        # the timed value: the whole step (forward, loss cotangents, backward, finalize) as ONE
        # graph captured from the stream the library calls run on, replayed as one launch
        s2 = torch.cuda.Stream(dev)
        s2.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s2):
            step_eager()
        torch.cuda.current_stream().wait_stream(s2)
        torch.cuda.synchronize()
        g_step = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g_step):
            step_eager()
        for _ in range(args.warmup):
            g_step.replay()
        ms_graph = timed(g_step.replay, args.steps) * 1e3
        print(f"# graph step {ms_graph:.3f} ms", file=sys.stderr, flush=True)

    # plain: one launch sequence per scene
    plain_ms = plain_eager_ms = None
    if not args.no_plain:
        scenes = []
        for i, (sc, cams) in enumerate(zip(w.scenes, w.cameras)):
            g0, g1 = batch.gauss_off[i], batch.gauss_off[i + 1]
            r0, r1 = batch.ray_off[i], batch.ray_off[i + 1]
            s = fmb.Scene(params[0][g0:g1], params[1][g0:g1], params[2][g0:g1], params[3][i], w.eta,
                          fmb.Cameras.from_numpy(cams.w2c, cams.intr, cams.hw, device=dev))
            o = {"depth": outs["depth"][r0:r1], "alpha": outs["alpha"][r0:r1], "normal": outs["normal"][r0:r1],
                 "stash": outs["stash"][r0:r1]}
            gr = {"means": grads["means"][g0:g1], "prec": grads["prec"][g0:g1],
                  "weights": grads["weights"][g0:g1], "betas": grads["betas"][i]}
            scenes.append((s, o, gr, r0, r1))

        def step_plain():
            for s, o, gr, r0, r1 in scenes:
                s.render(normals=True, out=o)
            cotangents(outs)
            for s, o, gr, r0, r1 in scenes:
                s.backward(o, cot["depth"][r0:r1], cot["alpha"][r0:r1], None, None, grads=gr)

        for _ in range(args.warmup):
            step_plain()
        plain_eager_ms = timed(step_plain, args.steps) * 1e3
        print(f"# plain step (eager) {plain_eager_ms:.3f} ms", file=sys.stderr, flush=True)
        plain_ms = plain_eager_ms
        if not args.no_graph:
            # like for like with the batched value: the 16 per-scene launch sequences (forward, loss
            # kernel, backward + finalize of every scene) replayed as one graph
            s2p = torch.cuda.Stream(dev)
            s2p.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s2p):
                step_plain()
            torch.cuda.current_stream().wait_stream(s2p)
            torch.cuda.synchronize()
            g_plain = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g_plain):
                step_plain()
            for _ in range(args.warmup):
                g_plain.replay()
            plain_ms = timed(g_plain.replay, args.steps) * 1e3
            del g_plain
            print(f"# plain step (one graph) {plain_ms:.3f} ms", file=sys.stderr, flush=True)

    launch = fmb.launch_config(batch=batch)
    # the zero-parameter renderer on the same batch: eager step, HIP-event kernel times
    comp = None
    if not args.no_composite:
        batch.set_model("composite")
        for _ in range(args.warmup):
            step_eager()
        fmb.timing_enable(True)
        fmb.kernel_times(reset=True)
        ms_comp = timed(step_eager, args.steps) * 1e3
        kc = fmb.kernel_times(reset=True)
        fmb.timing_enable(False)
        batch.set_model("blend")
        cf = kc["fwd_ms"] / max(kc["n_fwd"], 1)
        cb = kc["bwd_ms"] / max(kc["n_bwd"], 1)
        cfin = kc["fin_ms"] / max(kc["n_fin"], 1)
        # the per-ray sort and prefix sum: sum over rays of N (ceil(log2 N) + 1)
        sort_ops = sum(c.n_rays * s.n * (int(np.ceil(np.log2(max(s.n, 2)))) + 1)
                       for s, c in zip(w.scenes, w.cameras))
        fl_f = pairs * FLOPS_COMP_FWD_NORMALS + sort_ops
        fl_b = pairs * (FLOPS_COMP_ADJ_PLAIN + 1)
        comp = {"value": pairs / (ms_comp * 1e-3), "unit": "pairs/s", "ms_per_step": ms_comp,
                "timed": "eager launches",
                "kernel_ms": {"forward": cf, "backward": cb, "finalize": cfin},
                "forward_tflops": fl_f / (cf * 1e-3) / 1e12, "backward_tflops": fl_b / (cb * 1e-3) / 1e12,
                "forward_frac": fl_f / (cf * 1e-3) / PEAK_FP32, "backward_frac": fl_b / (cb * 1e-3) / PEAK_FP32,
                "flops_per_pair": {"forward": f"{FLOPS_COMP_FWD_NORMALS} + ceil(log2 N) + 1 (sort-based)",
                                   "backward": f"{FLOPS_COMP_ADJ_PLAIN} + 1 (sort-based)"},
                "over_blend": ms_comp / ms_eager, "paper_over_blend": PAPER_COMP_OVER_BLEND}
        print(f"# composite step {ms_comp:.3f} ms; kernels fwd {cf:.3f} bwd {cb:.3f} fin {cfin:.3f} ms",
              file=sys.stderr, flush=True)

    # the other rows of the path, each timed as eager launches with HIP-event kernel times:
    # colour on the same batch, two-way flow on the 480x640 flow workload, split statistic
    extras = None
    if not args.no_extras:
        extras = {}
        g = np.random.Generator(np.random.PCG64(7))

        def leg(step, k, pairs_per_step):
            for _ in range(max(args.warmup, 3)):
                step()
            fmb.timing_enable(True)
            fmb.kernel_times(reset=True)
            ms = timed(step, k) * 1e3
            kt = fmb.kernel_times(reset=True)
            fmb.timing_enable(False)
            per = {n: kt[n + "_ms"] / kt["n_" + n] for n in ("fwd", "bwd", "fin") if kt["n_" + n]}
            return {"value": pairs_per_step / (ms * 1e-3), "unit": "pairs/s", "ms_per_step": ms,
                    "kernel_ms": per}

        # colour (sigmoid colours blended like depth; colour cotangent added to the loss's)
        q = t((1.5 * g.standard_normal((sum(s.n for s in w.scenes), 3))).astype(np.float32))
        batch.set_colors(q)
        outs_c = batch.alloc_outputs(normals=True, color=True)
        grads_c = batch.alloc_grads(colors=True)
        cot_c = dict(cot)
        cot_c["color"] = t((1e-6 * g.standard_normal((P, 3))).astype(np.float32))

        def step_colour():
            batch.forward(outs_c)
            cotangents(outs_c)
            batch.backward(outs_c, cot_c, grads_c)

        extras["colour"] = leg(step_colour, args.steps, pairs)
        batch.set_colors(None)

        # two-way flow: depth, alpha and flow to the poses before and after each view
        wf = W.make_config("flow480")
        sf, cf = wf.scenes[0], W.with_backward_flow(wf.cameras[0], seed=11)
        scene_f = fmb.Scene(t(sf.means), t(sf.prec), t(sf.weights), t(wf.betas), wf.eta,
                            fmb.Cameras.from_numpy(cf.w2c, cf.intr, cf.hw, w2c_b=cf.w2c_b, intr_b=cf.intr_b,
                                                   device=dev, w2c_c=cf.w2c_c, intr_c=cf.intr_c))
        pf = scene_f.n_rays
        gd, ga = (t((1e-6 * g.standard_normal(pf)).astype(np.float32)) for _ in range(2))
        gf = t((1e-6 * g.standard_normal((pf, 4))).astype(np.float32))
        outs_f = scene_f.render(normals=False, flow=True)
        grads_f = scene_f.backward(outs_f, gd, ga, None, gf)

        def step_flow():
            scene_f.render(normals=False, flow=True, out=outs_f)
            scene_f.backward(outs_f, gd, ga, None, gf, grads=grads_f)

        extras["two_way_flow"] = leg(step_flow, max(args.steps // 2, 5), pf * sf.n)
        extras["two_way_flow"]["workload"] = "flow480: N=100, 8 views 480x640, flow to both neighbouring poses"

        # the single-scene workloads: 40 Gaussians x 20 views of 128x128, and 10 000 Gaussians x
        # 1080x1920 (no culling); forward with normals, backward of depth and alpha cotangents
        for name, k in (("fwdbwd128", args.steps), ("large1080", 5)):
            wk = W.make_config(name)
            sk, ck = wk.scenes[0], wk.cameras[0]
            scene_k = fmb.Scene(t(sk.means), t(sk.prec), t(sk.weights), t(wk.betas), wk.eta,
                                fmb.Cameras.from_numpy(ck.w2c, ck.intr, ck.hw, device=dev))
            pk = scene_k.n_rays
            gdk, gak = (t((1e-6 * g.standard_normal(pk)).astype(np.float32)) for _ in range(2))
            outs_k = scene_k.render(normals=True)
            grads_k = scene_k.backward(outs_k, gdk, gak)
            scene_k.autotune(outs_k, {"depth": gdk, "alpha": gak, "normal": None, "flow": None}, grads_k)

            def step_k():
                scene_k.render(normals=True, out=outs_k)
                scene_k.backward(outs_k, gdk, gak, grads=grads_k)

            extras[name] = leg(step_k, k, pk * sk.n)
            # the same step as one graph, as the batch's step is timed (launch gaps left out)
            s2k = torch.cuda.Stream(dev)
            s2k.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s2k):
                step_k()
            torch.cuda.current_stream().wait_stream(s2k)
            torch.cuda.synchronize()
            g_k = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g_k):
                step_k()
            for _ in range(3):
                g_k.replay()
            ms_k = timed(g_k.replay, k) * 1e3
            extras[name]["eager_ms_per_step"] = extras[name]["ms_per_step"]
            extras[name]["ms_per_step"] = ms_k
            extras[name]["value"] = pk * sk.n / (ms_k * 1e-3)
            extras[name]["timed"] = "replays of one graph of the step"
            del g_k, scene_k, outs_k, grads_k

        # fwd64: the forward alone (depth, alpha, normals) of 40 Gaussians on one 64x64 view (a
        # single small launch: latency, not throughput)
        w64 = W.make_config("fwd64")
        s64, c64 = w64.scenes[0], w64.cameras[0]
        scene64 = fmb.Scene(t(s64.means), t(s64.prec), t(s64.weights), t(w64.betas), w64.eta,
                            fmb.Cameras.from_numpy(c64.w2c, c64.intr, c64.hw, device=dev))
        outs64 = scene64.render(normals=True)

        def step64():
            scene64.render(normals=True, out=outs64)

        for _ in range(3):
            step64()
        s264 = torch.cuda.Stream(dev)
        s264.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s264):
            step64()
        torch.cuda.current_stream().wait_stream(s264)
        torch.cuda.synchronize()
        g64 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g64):
            step64()
        for _ in range(3):
            g64.replay()
        ms64g = timed(g64.replay, args.steps) * 1e3
        ms64e = timed(step64, args.steps) * 1e3
        # one small launch: a graph replay costs more than the eager call, so both are given and
        # the value is the eager call's
        extras["fwd64"] = {"value": scene64.n_rays * s64.n / (ms64e * 1e-3), "unit": "pairs/s",
                           "ms_per_step": ms64e, "graph_ms_per_step": ms64g, "timed": "eager calls",
                           "workload": "fwd64: N=40, one 64x64 view, forward with normals"}
        del g64, scene64, outs64

        # split statistic: lbar_i = (1/M) sum_j L_j w_ji over the batch's rays
        lossr = t(g.random(P).astype(np.float32))
        lbar = torch.empty(sum(s.n for s in w.scenes), device=dev)
        batch.forward(outs)

        def step_split():
            batch.split_statistic(lossr, outs, lbar)

        for _ in range(max(args.warmup, 3)):
            step_split()
        ms_split = timed(step_split, args.steps) * 1e3
        extras["split_statistic"] = {"value": pairs / (ms_split * 1e-3), "unit": "pairs/s", "ms_per_call": ms_split}
        print("# extras: " + ", ".join(f"{k} {v.get('ms_per_step', v.get('ms_per_call')):.3f} ms"
                                       for k, v in extras.items()), file=sys.stderr, flush=True)

    if args.calibrate_copy:
        # Kernels of known HBM traffic for scaling FETCH_SIZE / WRITE_SIZE: a 1 GiB device copy
        # (the runtime's blit kernel) and a 1 GiB elementwise copy (dst = src + 1, plain
        # per-lane loads), each on a source evicted from the caches by writing 1 GiB first.
        src = torch.ones(256 << 20, device=dev)
        dst = torch.empty_like(src)
        evict = torch.zeros(256 << 20, device=dev)
        torch.cuda.synchronize()
        dst.copy_(src)
        evict.fill_(2.0)
        torch.cuda.synchronize()
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del evict
        print("# calibration: blit copy and elementwise add, each 1073741824 bytes read and written",
              file=sys.stderr, flush=True)

    ms_step = ms_graph if ms_graph is not None else ms_eager
    value = pairs / (ms_step * 1e-3)
    # dominant kernel: the persistent backward (adjoint with recompute) of the tuned variant
    flops_bwd_launch = pairs * FLOPS_ADJ_PLAIN
    achieved = flops_bwd_launch / (bwd_ms * 1e-3)
    step_flops = pairs * (FLOPS_FWD_NORMALS + FLOPS_ADJ_PLAIN)
    res = {
        "metric": "ray x Gaussian pairs/s fwd+bwd (batched vs plain), % FP32 VALU peak",
        "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch16: 16 uneven scenes, N~U{10..100}, V~U{4..32}, 64^2/128^2/256^2, "
                               "fwd (depth, alpha, normals) + bwd (L1 depth + BCE alpha), seed 3",
                   "scenes": S, "rays": P, "pairs_per_step": pairs, "global_batch": P,
                   "parallelism": "single GPU, persistent batched kernels in HIP graphs"},
        "plain_value": (pairs / (plain_ms * 1e-3)) if plain_ms else None,
        "plain_ms_per_step": plain_ms,
        "plain_timed": ("replays of one graph of the 16 per-scene launch sequences"
                        if plain_ms is not None and plain_ms != plain_eager_ms else "eager launches"),
        "plain_eager_ms_per_step": plain_eager_ms,
        "batched_over_plain": (plain_ms / ms_step) if plain_ms else None,
        "batched_over_plain_eager": (plain_eager_ms / ms_eager) if plain_eager_ms else None,
        "eager_ms_per_step": ms_eager,
        "timed": "replays of one graph of the whole step" if ms_graph is not None else "eager launches",
        "loss": "depth and alpha cotangents written by the forward's per-ray epilogue "
                "(library_graphs_ms_per_step and the plain leg run the separate loss kernel)",
        "library_graphs_ms_per_step": ms_graph_api,
        "fp32_peak_frac_step": step_flops / (ms_step * 1e-3) / PEAK_FP32,
        "kernel_ms": {"forward": fwd_ms, "backward": bwd_ms, "finalize": fin_ms},
        "launch": launch,
        "composite": comp,
        "other_rows": extras,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                     "traffic": measured_traffic(launch["bwd_variant"]),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "kernel": bwd_kernel_name(launch["bwd_variant"]), "flops_per_pair": FLOPS_ADJ_PLAIN,
                     "algorithmic_flops_per_pair": {"forward_normals": FLOPS_FWD_NORMALS,
                                                    "forward_plain": FLOPS_FWD_PLAIN,
                                                    "adjoint_normals": FLOPS_ADJ_NORMALS,
                                                    "adjoint_plain": FLOPS_ADJ_PLAIN},
                     **executed(pairs, bwd_ms, launch["bwd_variant"])},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
