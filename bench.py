"""Benchmark: Laplace S and D operator applies on the 512-spheroid suspension.

One step = one S apply and one D apply (nrhs = 1 each, fresh N(0,1) densities
already resident in HBM), i.e. one pass of the whole apply (transform, self,
near, far, assembly) per operator.  The headline line is the mixed-precision
path (FP32 sums and contractions with compensated tiles, FP64 geometry and
recurrences); the plain FP64 path is measured on the same inputs and reported
beside it.  Prints one JSON line with applies/s, pair-interactions/s, per-apply
p50/p99 latency, the far-field kernel's roofline figures (HIP events inside the
library, on the apply's stream) and the CPU oracle timed on a bounded sample.
Further sections of the same line: the FP64 path, S' and D', the Stokes single
layer (with and without its pressure) and double layer at 256 spheroids, the
GMRES study of the completion terms, the 512-spheroid Dirichlet and Neumann
solves, and the tree far field at 512 and 4096 spheroids beside the direct sum
(each can be skipped with its --no-* flag).

  python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--precision mixed|fp64]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# flop convention per far-field node pair (add/sub/mul = 1, FMA = 2, rsqrt = 1):
# S: 3 differences + 5 for r^2 + 1 rsqrt + 2 accumulate
# D: 3 differences + 5 for r^2 + 1 rsqrt + 2 for r^-3 + 5 for the dipole dot + 2 accumulate
FLOPS_PER_PAIR = {0: 11, 1: 18}
# MI355X vector peaks: FP64 78.6 TFLOP/s, FP32 157.3 TFLOP/s (256 CUs, 2.4 GHz)
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}


def cpu_baseline(geom, p, dens_s, dens_d, N, sample):
    """The FP64 oracle at `sample` evenly spaced nodes per operator (setup included)."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    tg = np.linspace(0, N - 1, sample).astype(np.int64)
    t0 = time.perf_counter()
    ref_s = oracle.apply_at(geom, p, 0, dens_s, tg)[0]
    ref_d = oracle.apply_at(geom, p, 1, dens_d, tg)[0]
    dt = time.perf_counter() - t0
    # one S and one D apply cost N/sample times the sampled work
    applies_per_s = 2.0 / (dt * N / sample)
    return ({"value": applies_per_s, "unit": "applies/s", "cores": oracle.num_threads(), "kind": "oracle",
             "sample": f"S and D at {sample} of {N} nodes (evenly spaced), geometry setup included, "
                       f"{dt:.1f} s, scaled to whole applies"}, tg, (ref_s, ref_d))


def error_vs_oracle(g, dens0, tg, refs):
    """Relative error of S and D against the FP64 oracle, per result (one apply of
    each operator in each precision, compared at the oracle's sampled nodes):
    relative l2 norm and max-norm relative to the oracle's largest value."""
    import numpy as np

    import paper_2506_20809_amd as sbie

    out = {"nodes_compared": int(len(tg))}
    for name, prec in (("mixed", sbie.SBIE_MIXED), ("fp64", sbie.SBIE_FP64)):
        out[name] = {}
        for op, ref in zip((sbie.SBIE_OP_S, sbie.SBIE_OP_D), refs):
            u = g.apply(op, dens0[op], precision=prec)
            g.sync()
            u = u.cpu().numpy()[tg]
            out[name]["SD"[op]] = {"rel_l2": float(np.linalg.norm(u - ref) / np.linalg.norm(ref)),
                                   "max_rel": float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))}
    return out


def counter_traffic(precision, workload):
    """HBM bytes per far-kernel launch from the committed counter summary, or None
    when that summary does not cover this workload and precision or the far
    kernel's source has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"far_pairs_{workload}_{precision}_hbm_counters.md")
    src = os.path.join(ROOT, "paper_2506_20809_amd", "csrc", "far_mfma.hip")
    if not os.path.exists(path):
        return None
    kv = dict(line.strip().split("=", 1) for line in open(path) if "=" in line and not line.startswith("|"))
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != kv.get("source_sha256"):
            return None
    return float(kv["traffic_bytes_per_launch"])


def run(g, dens, steps, warmup, precision):
    """Time `steps` steps (S then D) on the torch current stream."""
    import numpy as np
    import torch

    import paper_2506_20809_amd as sbie

    prec = sbie.SBIE_MIXED if precision == "mixed" else sbie.SBIE_FP64
    stream = torch.cuda.current_stream()
    out = torch.empty((2, g.N), dtype=torch.float64, device="cuda")
    ops = (sbie.SBIE_OP_S, sbie.SBIE_OP_D)
    for k in range(warmup):
        for o in range(2):
            g.apply(ops[o], dens[k % dens.shape[0], o], precision=prec, out=out[o], timing=True)
    g.sync()
    g.timing()  # discard warm-up timings
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(2 * steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        for o in range(2):
            e = ev[2 * k + o]
            e[0].record(stream)
            g.apply(ops[o], dens[(warmup + k) % dens.shape[0], o], precision=prec, out=out[o], timing=True)
            e[1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    g.sync()
    tim = g.timing()
    lat = np.array([e[0].elapsed_time(e[1]) for e in ev])
    # the far field of one apply runs as tim.far_launches launches over chunks of
    # partner offsets (balanced); far_kernel_ms covers all of them (and the
    # folds between them), so flops per launch over the mean launch time is
    # flops per apply over far_kernel_ms
    launches = max(1, tim.far_launches)
    flops_per_apply = 0.5 * (FLOPS_PER_PAIR[0] + FLOPS_PER_PAIR[1]) * tim.far_pairs
    flops_per_launch = flops_per_apply / launches
    achieved = flops_per_launch / (tim.far_kernel_ms / launches * 1e-3) / 1e12
    return {
        "applies_per_s": 2 * steps / elapsed,
        "elapsed_s": elapsed,
        "pair_interactions_per_s": tim.far_pairs / (tim.far_kernel_ms * 1e-3),
        "effective_all_pairs_per_s": float(g.N) * g.N / (np.mean(lat) * 1e-3),
        "near_evals_per_s": tim.near_evals / (tim.near_ms * 1e-3) if tim.near_ms > 0 else None,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(np.mean(lat))},
        "part_ms": {"prep": tim.prep_ms, "transform_self": tim.transform_ms, "near": tim.near_ms,
                    "far_kernel": tim.far_kernel_ms, "assemble": tim.assemble_ms, "apply_total": tim.total_ms},
        "far_pairs": tim.far_pairs,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[precision], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS[precision], "traffic": None,
                     "kernel": "k_far_pairs<float> (S and D alternating)" if precision == "mixed"
                     else "k_far_pairs<double> (S and D alternating)",
                     "flops_per_launch": flops_per_launch, "launches_per_apply": launches,
                     "flops_per_apply": flops_per_apply},
    }


def run_multi(g, steps, precision, nrhs=4):
    """S and D applied to nrhs densities per call (the shared far-field path),
    against nrhs one-density calls: densities per second each way."""
    import numpy as np
    import torch

    import paper_2506_20809_amd as sbie

    prec = sbie.SBIE_MIXED if precision == "mixed" else sbie.SBIE_FP64
    gen = torch.Generator(device="cuda")
    gen.manual_seed(17)
    dens = torch.randn((nrhs, g.N), dtype=torch.float64, device="cuda", generator=gen)
    out = torch.empty_like(dens)
    res = {"workload": f"{nrhs} densities per call, the headline suspension, precision={precision}"}
    for op, name in ((sbie.SBIE_OP_S, "S"), (sbie.SBIE_OP_D, "D")):
        rates = {}
        for mode in ("shared", "one_by_one"):
            def call():
                if mode == "shared":
                    g.apply(op, dens, precision=prec, out=out)
                else:
                    for k in range(nrhs):
                        g.apply(op, dens[k], precision=prec, out=out[k])
            call()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                call()
            torch.cuda.synchronize()
            rates[mode] = nrhs * steps / (time.perf_counter() - t0)
        res[name] = {"densities_per_s_shared": rates["shared"], "densities_per_s_one_by_one": rates["one_by_one"],
                     "speedup": rates["shared"] / rates["one_by_one"]}
    return res


# Stokeslet per far node pair: 3 differences + 5 for r^2 + 1 rsqrt + 2 for r^-3 + 5 for r.q
# + 1 for (r.q) r^-3 + 3 x (FMA for q/r + FMA for r (r.q) r^-3) = 29
FLOPS_PER_STOKES_PAIR = 29


# S' per far node pair: 3 differences + 5 for r^2 + 1 rsqrt + 2 for r^-3 + 5 for nu_x.d + 1 for q (nu_x.d)
# + 2 accumulate = 19.  D': 3 + 5 + 1 + 2 (r^-3) + 1 (r^-2) + 5 (nu_y.d) + 5 (nu_x.d) + 5 (nu_x.nu_y)
# + 2 (-3 (nu_y.d)(nu_x.d)) + 2 (FMA with r^-2 and nu_x.nu_y) + 1 (q r^-3) + 2 accumulate = 34
FLOPS_PER_NORMAL_PAIR = {3: 19, 4: 34}


def run_normal(g, dens, steps, precision):
    """S' and D' applies on the same geometry: applies/s per operator and the
    far kernel's share of the vector peak."""
    import numpy as np
    import torch

    import paper_2506_20809_amd as sbie

    prec = sbie.SBIE_MIXED if precision == "mixed" else sbie.SBIE_FP64
    out = torch.empty(g.N, dtype=torch.float64, device="cuda")
    res = {}
    for op, name in ((sbie.SBIE_OP_SP, "S'"), (sbie.SBIE_OP_DP, "D'")):
        g.apply(op, dens[0, 0], precision=prec, out=out, timing=True)
        g.sync()
        g.timing()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            g.apply(op, dens[k % dens.shape[0], 0], precision=prec, out=out, timing=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g.sync()
        tim = g.timing()
        achieved = FLOPS_PER_NORMAL_PAIR[op] * tim.far_pairs / (tim.far_kernel_ms * 1e-3) / 1e12
        res[name] = {"applies_per_s": steps / el, "ms_per_apply": 1e3 * el / steps,
                     "part_ms": {"prep": tim.prep_ms, "transform_self": tim.transform_ms, "near": tim.near_ms,
                                 "far_kernel": tim.far_kernel_ms, "assemble": tim.assemble_ms},
                     "far_roofline_frac": achieved / PEAK_TFLOPS[precision]}
    return res


# Stresslet per far node pair: 3 differences + 5 r^2 + 1 rsqrt + 1 r^-2 + 3 r^-5 + 5 d.(W mu) + 5 d.nu
# + 1 product + 3 x FMA (2) = 30
FLOPS_PER_STRESSLET_PAIR = 30


def run_stokes(ctx, steps, warmup, precision, op=2):
    """Stokes single layer (Eq. stokes; op 2), with its pressure (op 5), or the
    Stokes double layer (op 6) on the 256-spheroid suspension at p = 12."""
    import numpy as np
    import torch

    import paper_2506_20809_amd as sbie
    import workloads

    geom = workloads.geometry("c4")
    p = workloads.CONFIGS["c4"]["p"]
    g = sbie.Geometry(ctx, geom, p)
    prec = sbie.SBIE_MIXED if precision == "mixed" else sbie.SBIE_FP64
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    dens = torch.randn((steps + warmup, 3, g.N), dtype=torch.float64, device="cuda", generator=gen)
    out = torch.empty((4 if op == sbie.SBIE_OP_STOKES_SP else 3, g.N), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for k in range(warmup):
        g.apply(op, dens[k], precision=prec, out=out, timing=True)
    g.sync()
    g.timing()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        g.apply(op, dens[warmup + k], precision=prec, out=out, timing=True)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    g.sync()
    tim = g.timing()
    lat = np.array([e[0].elapsed_time(e[1]) for e in ev])
    per_pair = FLOPS_PER_STRESSLET_PAIR if op == sbie.SBIE_OP_STOKES_D else FLOPS_PER_STOKES_PAIR
    achieved = per_pair * tim.far_pairs / (tim.far_kernel_ms * 1e-3) / 1e12
    res = {
        "workload": f"256 polydisperse spheroids (volume fraction 0.20, gap 0.05), p={p}, N={g.N}, "
                    f"3-component density, op={op}, precision={precision}",
        "applies_per_s": steps / elapsed,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "part_ms": {"prep": tim.prep_ms, "transform_self": tim.transform_ms, "near": tim.near_ms,
                    "far_kernel": tim.far_kernel_ms, "assemble": tim.assemble_ms, "apply_total": tim.total_ms},
        "far_pairs": tim.far_pairs,
        "far_pair_interactions_per_s": tim.far_pairs / (tim.far_kernel_ms * 1e-3),
        "far_roofline_frac": achieved / PEAK_TFLOPS[precision],
    }
    g.close()
    return res


# Near-field work per (near pair, target) evaluation at order p, FP64 (add/mul = 1,
# FMA = 2): per (n, m) pair with n >= m, the Q column step (3), the Ferrers step (3),
# the spectral ratio (1) and the contraction with the cos and sin coefficients (4):
# 11 (p+1)(p+2)/2; per evaluation the frame map and coordinates (about 60).  The
# backward recurrences of orders 0 and 1 add 6 per step below the top degree; their
# depth depends on the target and is not counted.  The Stokes kernels evaluate four
# (single layer) or thirteen (double layer) coefficient sets with their gradients
# against each basis; their count is given per basis evaluation and set.
def near_flops(p):
    return 11 * (p + 1) * (p + 2) // 2 + 60


def target_points(geom, xyz, nrm, n, seed):
    """n points outside every particle: half 1e-2 outside random nodes along
    their normals (near their own particle and often a neighbour), half uniform
    in the suspension's bounding box with the points inside a particle redrawn."""
    import numpy as np

    from workloads import quat_rot

    rng = np.random.default_rng(seed)
    idx = rng.choice(len(xyz), n // 2, replace=False)
    near = xyz[idx] + 1e-2 * nrm[idx]
    c = geom["centers"]
    R = np.stack([quat_rot(q) for q in geom["quats"]])
    ax = np.stack([geom["A"], geom["A"], geom["C"]], axis=1)
    lo, hi = c.min(0) - 1.0, c.max(0) + 1.0
    box = np.zeros((0, 3))
    while len(box) < n - n // 2:
        cand = lo + (hi - lo) * rng.random((n, 3))
        inside = np.zeros(len(cand), dtype=bool)
        for i in range(len(c)):
            b = ((cand - c[i]) @ R[i]) / ax[i]
            inside |= np.einsum("ij,ij->i", b, b) <= 1.0
        box = np.concatenate([box, cand[~inside]])
    return np.concatenate([near, box[: n - n // 2]])


def run_targets(g, geom, dens, steps, n=65536):
    """Particle-to-target evaluation (S and D with gradients) at n points,
    mixed and FP64: points per second and, counting every (point, node) pair
    as far (an upper bound: near pairs go through the expansions), far-pair
    evaluations per second and the fraction of the vector peak by the direct
    sums' flop counts (value and gradient: S 17, D 30 per pair)."""
    import torch

    import paper_2506_20809_amd as sbie

    xyz, nrm, _ = g.nodes()
    pts = torch.tensor(target_points(geom, xyz, nrm, n, 23), dtype=torch.float64, device="cuda")
    out = {"workload": f"{n} points outside the headline suspension's particles, half 1e-2 off random nodes, "
                       "half uniform in its bounding box"}
    for prec, name, peak in ((sbie.SBIE_MIXED, "mixed", PEAK_TFLOPS["mixed"]), (sbie.SBIE_FP64, "fp64",
                                                                                 PEAK_TFLOPS["fp64"])):
        for op, on, fl in ((sbie.SBIE_OP_S, "S", 17), (sbie.SBIE_OP_D, "D", 30)):
            g.eval_targets(op, dens[op], pts, precision=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                g.eval_targets(op, dens[op], pts, precision=prec)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            pairs = n * g.N
            out[f"{name}_{on}"] = {"ms_per_call": dt * 1e3, "points_per_s": n / dt, "pair_evals_per_s": pairs / dt,
                                   "vector_frac_upper": fl * pairs / dt / 1e12 / peak}
    return out


def run_near(ctx, steps):
    """The near field alone (SBIE_PARTS_NEAR): S, D, S' and D' on the
    512-spheroid suspension (p = 16), the Stokes single layer (without and with
    the pressure) and double layer on the 256-spheroid one (p = 12), FP64 and
    mixed; evaluations per second and, for S and D, the FP64 vector-unit
    fraction by the flop count of near_flops."""
    import torch

    import paper_2506_20809_amd as sbie
    import workloads

    out = {}
    for wl, ops in (("c3", (sbie.SBIE_OP_S, sbie.SBIE_OP_D, sbie.SBIE_OP_SP, sbie.SBIE_OP_DP)),
                    ("c4", (sbie.SBIE_OP_STOKES_S, sbie.SBIE_OP_STOKES_SP, sbie.SBIE_OP_STOKES_D))):
        geom = workloads.geometry(wl)
        p = workloads.CONFIGS[wl]["p"]
        g = sbie.Geometry(ctx, geom, p)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(7)
        for op in ops:
            nrhs = 3 if op in (sbie.SBIE_OP_STOKES_S, sbie.SBIE_OP_STOKES_SP, sbie.SBIE_OP_STOKES_D) else 1
            d = torch.randn((nrhs, g.N) if nrhs > 1 else (g.N,), dtype=torch.float64, device="cuda", generator=gen)
            for prec, name in ((sbie.SBIE_FP64, "fp64"), (sbie.SBIE_MIXED, "mixed")):
                for k in range(steps + 1):
                    g.apply(op, d, precision=prec, parts=sbie.SBIE_PARTS_NEAR, timing=k > 0)
                g.sync()
                tim = g.timing()
                evals = tim.near_evals
                rate = evals / (tim.near_ms * 1e-3)
                rec = {"near_ms": tim.near_ms, "evaluations": int(evals), "evaluations_per_s": rate}
                if op in (sbie.SBIE_OP_S, sbie.SBIE_OP_D):
                    rec["fp64_frac"] = near_flops(p) * rate / 1e12 / PEAK_TFLOPS["fp64"]
                out[f"{wl}_op{op}_{name}"] = rec
        g.close()
    return out


# GMRES iteration counts printed in the paper's table of the lattice study
# (Section 5.2, four prolates at p = 16, tolerance 1e-10), for context:
# {R: {R*d: (C_I, eta C_I, S, eta S)}}
PAPER_GMRES = {
    1.1: {2.0: (14, 13, 10, 10), 1.0: (15, 14, 11, 12), 0.01: (36, 33, 33, 34)},
    2.0: {2.0: (19, 17, 12, 14), 1.0: (19, 17, 13, 16), 0.01: (39, 35, 35, 37)},
    4.0: {2.0: (27, 26, 16, 15), 1.0: (28, 27, 18, 17), 0.01: (49, 51, 39, 38)},
    8.0: {2.0: (44, 42, 23, 20), 1.0: (45, 45, 25, 21), 0.01: (65, 68, 51, 45)},
    16.0: {2.0: (69, 67, 31, 24), 1.0: (75, 72, 34, 26), 0.01: (107, 115, 68, 52)},
    32.0: {2.0: (103, 100, 40, 31), 1.0: (109, 107, 45, 32), 0.01: (170, 169, 91, 60)},
    64.0: {2.0: (131, 133, 47, 38), 1.0: (150, 154, 57, 40), 0.01: (223, 228, 124, 67)},
}


def run_tree(g, dens, steps, theta=0.6, order=10, leaf=2):
    """Mixed-precision S and D applies with the far field through the tree, and
    the tree far part's relative l2 distance from the direct FP64 far part on
    the same density, for the mixed and the FP64 tree sums."""
    import numpy as np
    import torch

    import paper_2506_20809_amd as sbie

    t0 = time.perf_counter()
    info = g.far_tree(theta, order, leaf)
    res = {"theta": theta, "order": order, "leaf": leaf, "plan_and_upload_s": time.perf_counter() - t0,
           "tree": info}
    for name, op in (("S", sbie.SBIE_OP_S), ("D", sbie.SBIE_OP_D)):
        g.apply(op, dens[0, op], precision=sbie.SBIE_MIXED, tree=True, timing=True)
        g.sync()
        g.timing()  # discard the warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            g.apply(op, dens[k % dens.shape[0], op], precision=sbie.SBIE_MIXED, tree=True, timing=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tim = g.timing()
        fd = g.apply(op, dens[0, op], parts=sbie.SBIE_PARTS_FAR, precision=sbie.SBIE_FP64)
        diff = {}
        for prec, pv in (("mixed", sbie.SBIE_MIXED), ("fp64", sbie.SBIE_FP64)):
            ft = g.apply(op, dens[0, op], parts=sbie.SBIE_PARTS_FAR, precision=pv, tree=True)
            diff[prec] = float(torch.linalg.norm(ft - fd) / torch.linalg.norm(fd))
        res[name] = {"applies_per_s": steps / el, "ms_per_apply": 1e3 * el / steps,
                     "tree_far_ms": tim.far_kernel_ms, "far_rel_l2_vs_direct_fp64": diff}
    evals = info["proxy_evals"] + info["direct_evals"]
    res["tree_evals_per_apply"] = evals
    return res


def tree_sweep(g, dens, settings=((0.5, 10), (0.5, 12), (0.4, 12), (0.3, 12), (0.2, 12))):
    """FP64 tree far field against the direct FP64 far sum for several (theta,
    order): relative l2 distance per operator and the FP64 tree apply time."""
    import torch

    import paper_2506_20809_amd as sbie

    out = []
    fd = {op: g.apply(op, dens[0, op], parts=sbie.SBIE_PARTS_FAR, precision=sbie.SBIE_FP64)
          for op in (sbie.SBIE_OP_S, sbie.SBIE_OP_D)}
    for theta, order in settings:
        info = g.far_tree(theta, order, 2)
        rec = {"theta": theta, "order": order, "proxy_evals": info["proxy_evals"],
               "direct_evals": info["direct_evals"]}
        for name, op in (("S", sbie.SBIE_OP_S), ("D", sbie.SBIE_OP_D)):
            ft = g.apply(op, dens[0, op], parts=sbie.SBIE_PARTS_FAR, precision=sbie.SBIE_FP64, tree=True)
            g.apply(op, dens[1, op], precision=sbie.SBIE_FP64, tree=True, timing=True)
            g.sync()
            tim = g.timing()
            rec[name] = {"far_rel_l2_vs_direct_fp64": float(torch.linalg.norm(ft - fd[op]) / torch.linalg.norm(fd[op])),
                         "tree_far_ms": tim.far_kernel_ms, "apply_ms": tim.total_ms}
        out.append(rec)
    return out


def tree_scaling(ctx, name, steps):
    """The tree far field at a larger suspension beside the direct paths."""
    import torch

    import paper_2506_20809_amd as sbie
    import workloads

    geom = workloads.geometry(name)
    p = workloads.CONFIGS[name]["p"]
    t0 = time.perf_counter()
    g = sbie.Geometry(ctx, geom, p)
    setup_s = time.perf_counter() - t0
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.CONFIGS[name]["seed"])
    dens = torch.randn((2, 2, g.N), dtype=torch.float64, device="cuda", generator=gen)
    res = {"workload": f"{len(geom['A'])} polydisperse prolate/oblate spheroids (RSA, volume fraction 0.25, "
                       f"min gap 0.02), p={p}, N={g.N} nodes",
           "setup_s": setup_s, "tree": run_tree(g, dens, steps)}
    direct = run(g, dens, 2, 1, "mixed")
    res["direct_mixed"] = {"applies_per_s": direct["applies_per_s"], "far_kernel_ms": direct["part_ms"]["far_kernel"],
                           "far_pairs": direct["far_pairs"]}
    g.close()
    return res


def charge_data(pos, q, xyz):
    """Potential of point charges at the nodes (the exterior Dirichlet data), on the GPU."""
    import torch

    x = torch.tensor(xyz, dtype=torch.float64, device="cuda")
    f = torch.zeros(len(xyz), dtype=torch.float64, device="cuda")
    P = torch.tensor(pos, dtype=torch.float64, device="cuda")
    Q = torch.tensor(q, dtype=torch.float64, device="cuda")
    for k in range(0, len(q), 64):
        r = torch.cdist(x, P[k:k + 64])
        f += (Q[k:k + 64] / (4.0 * math.pi * r)).sum(dim=1)
    return f


def charge_flux_data(pos, q, xyz, nrm):
    """Outward normal derivative of the charges' potential at the nodes (the
    exterior Neumann data), on the GPU."""
    import torch

    x = torch.tensor(xyz, dtype=torch.float64, device="cuda")
    n = torch.tensor(nrm, dtype=torch.float64, device="cuda")
    out = torch.zeros(len(xyz), dtype=torch.float64, device="cuda")
    P = torch.tensor(pos, dtype=torch.float64, device="cuda")
    Q = torch.tensor(q, dtype=torch.float64, device="cuda")
    for k in range(len(q)):
        d = x - P[k]
        r = torch.linalg.norm(d, dim=1)
        out -= Q[k] * (d * n).sum(dim=1) / (4.0 * math.pi * r ** 3)
    return out


def gmres_study(ctx, p=16, ratios=(1.1, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0), maxit=1000):
    """GMRES iterations of the completed double-layer Dirichlet solve on the
    four-prolate lattice (Section 5.2) for each completion, unscaled and scaled
    by the eta table; the data are the potential of three charges inside each
    prolate."""
    import numpy as np
    import torch

    import paper_2506_20809_amd as sbie
    import workloads

    rows = []
    t0 = time.perf_counter()
    for R in ratios:
        for Rd in (2.0, 1.0, 0.01):
            geom = workloads.lattice2x2(R, Rd)
            g = sbie.Geometry(ctx, geom, p)
            xyz, _, _ = g.nodes()
            pos, q = workloads.point_charges(geom, 3, 7, shrink=0.3)
            f = charge_data(pos, q, xyz)
            its, times = [], []
            for c, scaled in ((0, False), (0, True), (1, False), (1, True)):
                eta = None if scaled else np.ones(4)
                torch.cuda.synchronize()
                t = time.perf_counter()
                try:
                    _, it, res = g.solve_completed(c, f, eta=eta, tol=1e-10, maxit=maxit)
                    its.append(it if res <= 1e-10 else None)
                except sbie.SbieError as e:
                    its.append(f"error {e.status}")
                times.append(1e3 * (time.perf_counter() - t))
            rows.append({"R": R, "R_times_d": Rd, "iterations": its, "paper": list(PAPER_GMRES[R][Rd]),
                         "solve_ms": [round(x, 2) for x in times]})
            g.close()
    return {"order": ["C_I", "eta C_I", "S", "eta S"], "p": p, "tol": 1e-10, "rows": rows,
            "wall_s": time.perf_counter() - t0}


def solve_large(ctx, name, precision, maxit=300):
    """The completed Dirichlet solve with the scaled single-layer completion on a
    suspension workload: iterations, seconds per solve and per iteration."""
    import torch

    import paper_2506_20809_amd as sbie
    import workloads

    geom = workloads.geometry(name)
    p = workloads.CONFIGS[name]["p"]
    g = sbie.Geometry(ctx, geom, p)
    xyz, _, _ = g.nodes()
    pos, q = workloads.point_charges(geom, 3, 7, shrink=0.3)
    f = charge_data(pos, q, xyz)
    prec = sbie.SBIE_MIXED if precision == "mixed" else sbie.SBIE_FP64
    tol = 1e-6 if precision == "mixed" else 1e-10
    g.solve_completed(1, f, tol=tol, maxit=2, precision=prec)  # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, it, res = g.solve_completed(1, f, tol=tol, maxit=maxit, precision=prec)
    el = time.perf_counter() - t
    out = {"workload": f"{len(geom['A'])} spheroids, p={p}, N={g.N}, eta S completion, precision={precision}",
           "tol": tol, "iterations": it, "relres": res, "solve_s": el, "ms_per_iteration": 1e3 * el / max(it, 1)}
    # the single-layer Neumann problem with the charges' normal field as data
    xyz, nrm, _ = g.nodes()
    data = charge_flux_data(pos, q, xyz, nrm)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, it, res = g.solve_neumann(data, tol=tol, maxit=maxit, precision=prec)
    el = time.perf_counter() - t
    out["neumann"] = {"tol": tol, "iterations": it, "relres": res, "solve_s": el,
                      "ms_per_iteration": 1e3 * el / max(it, 1)}
    g.close()
    return out


def served(ctx, n_requests, rhos, precision, max_sessions, budgets=(64 << 30,), napply=20, workers=64, batch=False,
           tree=False):
    """Served mode on the request stream (Section 4 use as a Krylov inner loop):
    n_requests sessions of napply closed-loop applies each.

    1. Plain path, back to back: one request at a time (geometry build, napply
       applies, release) -> service times s_i and the capacity mu = n / sum s_i.
    2. Served, saturated: every request arrives at t = 0 -> served throughput.
    3. Served at Poisson arrivals of rate rho * mu, for each rho and each HBM
       budget -> request latency (arrival to last apply) and per-apply latency,
       p50/p99.  The plain path under the same arrivals is a single FIFO server;
       its latencies follow from the measured s_i (done_i = max(a_i, done_{i-1})
       + s_i).
    Clients are a pool of `workers` threads taking the requests in arrival
    order (a request waits for a free client like any other queue)."""
    import queue
    import threading

    import numpy as np
    import torch

    import paper_2506_20809_amd as sbie
    import workloads

    reqs = workloads.served_stream(n_requests)
    geoms = [workloads.served_request(r) for r in reqs]
    prec = sbie.SBIE_MIXED if precision == "mixed" else sbie.SBIE_FP64

    def density(r, k, N):
        gen = torch.Generator(device="cuda")
        gen.manual_seed(r["seed"] * 64 + k)
        return torch.randn(N, dtype=torch.float64, device="cuda", generator=gen)

    # 1. plain path
    service, far_pairs, plain_apply_ms = [], [], []
    for r, geom in zip(reqs, geoms):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = sbie.Geometry(ctx, geom, r["p"])
        out = torch.empty(g.N, dtype=torch.float64, device="cuda")
        for k in range(napply):
            d = density(r, k, g.N)
            ta = time.perf_counter()
            g.apply(r["op"], d, precision=prec, out=out, timing=(k == 0))
            g.sync()
            plain_apply_ms.append(1e3 * (time.perf_counter() - ta))
        far_pairs.append(g.timing().far_pairs)
        g.close()
        service.append(time.perf_counter() - t0)
    service = np.array(service)
    mu = n_requests / service.sum()
    total_pairs = float(np.sum(far_pairs)) * napply
    print(f"served: plain pass of {n_requests} requests in {service.sum():.1f} s", file=sys.stderr, flush=True)

    def run_served(arrivals, budget):
        srv = sbie.Server(ctx, max_sessions=max_sessions, budget_bytes=budget, graphs=True, batch=batch, tree=tree)
        done = [0.0] * n_requests
        apply_ms = []
        errors = []
        lock = threading.Lock()
        work = queue.Queue()
        t_start = time.perf_counter()

        def client():
            while True:
                i = work.get()
                if i is None:
                    return
                try:
                    r = reqs[i]
                    s = srv.open(geoms[i], r["p"], r["op"], prec)
                    out = torch.empty(s.N, dtype=torch.float64, device="cuda")
                    ms = []
                    for k in range(napply):
                        _, st = s.apply(density(r, k, s.N), out)
                        ms.append(1e-3 * (st.end_us - st.submit_us))
                    s.close()
                    done[i] = time.perf_counter() - t_start
                    with lock:
                        apply_ms.extend(ms)
                except Exception as e:  # reported by the caller
                    errors.append(repr(e))

        pool = [threading.Thread(target=client) for _ in range(workers)]
        for t in pool:
            t.start()
        for i in range(n_requests):
            wait = arrivals[i] - (time.perf_counter() - t_start)
            if wait > 0:
                time.sleep(wait)
            work.put(i)
        for _ in pool:
            work.put(None)
        for t in pool:
            t.join()
        info = srv.info()
        srv.close()
        if errors:
            raise RuntimeError(errors[0])
        lat = np.array(done) - np.array(arrivals)
        return {"makespan_s": max(done), "request_latency_s": lat, "apply_ms": np.array(apply_ms),
                "peak_bytes": info.peak_bytes, "passed": info.passed, "waited": info.waited,
                "batched": info.batched, "tree_sessions": info.tree_sessions}

    def pct(x):
        return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99))}

    # 2. saturated
    sat = run_served([0.0] * n_requests, budgets[0])
    print(f"served: saturated run in {sat['makespan_s']:.1f} s", file=sys.stderr, flush=True)
    Ms = np.array([r["M"] for r in reqs])
    res = {
        "workload": f"{n_requests} requests (particle count log-uniform in [8, 1024] cut from a 0.15 volume "
                    f"fraction packing, p in {{8, 12, 16}}, S or D), {napply} closed-loop applies each, "
                    f"precision={precision}, {max_sessions} lanes, HIP graph replay"
                    f"{', batching lanes' if batch else ''}"
                    f"{', tree far field for S/D sessions of 64+ particles' if tree else ''}, {workers} client threads",
        "mean_particles": float(Ms.mean()),
        "plain": {"capacity_requests_per_s": mu, "applies_per_s": mu * napply,
                  "pair_interactions_per_s": total_pairs / service.sum(),
                  "apply_latency_ms": pct(plain_apply_ms)},
        "served_saturated": {"requests_per_s": n_requests / sat["makespan_s"],
                             "applies_per_s": n_requests * napply / sat["makespan_s"],
                             "pair_interactions_per_s": total_pairs / sat["makespan_s"],
                             "speedup_vs_plain": (n_requests / sat["makespan_s"]) / mu,
                             "apply_latency_ms": pct(sat["apply_ms"]),
                             "batched_applies": int(sat["batched"]), "tree_sessions": int(sat["tree_sessions"])},
    }
    # 3. Poisson arrivals at rho * mu, per budget
    for budget in budgets:
        for rho in rhos:
            rng = np.random.default_rng(55)
            arrivals = np.cumsum(rng.exponential(1.0 / (rho * mu), size=n_requests))
            arrivals -= arrivals[0]
            run = run_served(list(arrivals), budget)
            print(f"served: rho {rho}, budget {budget >> 30} GiB in {run['makespan_s']:.1f} s", file=sys.stderr,
                  flush=True)
            plain_done, t = [], 0.0
            for a, s_ in zip(arrivals, service):
                t = max(a, t) + s_
                plain_done.append(t)
            plain_lat = np.array(plain_done) - arrivals
            res[f"poisson_rho_{rho}_budget_{budget >> 30}GiB"] = {
                "arrival_rate_per_s": rho * mu,
                "served_request_latency_s": pct(run["request_latency_s"]),
                "plain_fifo_request_latency_s": pct(plain_lat),
                "served_apply_latency_ms": pct(run["apply_ms"]),
                "served_applies_per_s": n_requests * napply / run["makespan_s"],
                "peak_arena_bytes": int(run["peak_bytes"]), "admissions_passed": int(run["passed"]),
                "admissions_waited": int(run["waited"]), "batched_applies": int(run["batched"]),
            }
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--cpu-sample", type=int, default=98304)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the other precision's measurement")
    ap.add_argument("--no-stokes", action="store_true", help="skip the Stokes single-layer measurement")
    ap.add_argument("--no-derivatives", action="store_true", help="skip the S' and D' measurement")
    ap.add_argument("--no-solve", action="store_true", help="skip the completed double-layer solves")
    ap.add_argument("--no-tree", action="store_true", help="skip the tree far-field measurement")
    ap.add_argument("--no-near", action="store_true", help="skip the near-field measurement")
    ap.add_argument("--no-targets", action="store_true", help="skip the particle-to-target measurement")
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-density (nrhs = 4) measurement")
    ap.add_argument("--tree-sweep", action="store_true",
                    help="add the FP64 tree's accuracy and time over several (theta, order)")
    ap.add_argument("--only-stokes", action="store_true",
                    help="only the Stokes single layer, with its pressure, and the double layer (both precisions), "
                         "for profiling")
    ap.add_argument("--only-near", action="store_true",
                    help="run only the near-field section (for counter runs); prints its JSON object")
    ap.add_argument("--only-targets", action="store_true",
                    help="run only the particle-to-target section on the headline suspension; prints its JSON object")
    ap.add_argument("--served-requests", type=int, default=96,
                    help="requests in the served-mode run (0: skip)")
    ap.add_argument("--served-rho", type=float, nargs="+", default=[0.8], help="loads of the Poisson arrivals")
    ap.add_argument("--served-budget-gib", type=int, nargs="+", default=[64], help="HBM budgets of the server")
    ap.add_argument("--served-precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--served-lanes", type=int, default=8)
    ap.add_argument("--served-tree", action="store_true",
                    help="S/D sessions of 64+ particles take the tree far field (theta 0.6, order 10)")
    ap.add_argument("--served-batch", action="store_true",
                    help="batching lanes: sessions of one kind share a lane and run in batched launches")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (a known-size reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the operator apply here is a one-GPU path (sharding across GPUs is designed, not built); --gpus must be 1"}))
        sys.exit(2)
    if args.served_requests > 0 and "GPU_MAX_HW_QUEUES" not in os.environ:
        # one hardware queue per served lane (HIP's default is four per process:
        # eight lanes would share them in pairs, each pair's kernels in order);
        # read when the HIP runtime starts, so set before torch is imported
        os.environ["GPU_MAX_HW_QUEUES"] = str(max(4, args.served_lanes))

    import torch

    import paper_2506_20809_amd as sbie
    import workloads

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.calibrate_copy:
        # an elementwise kernel that reads 256 MiB and writes 256 MiB
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.only_near:
        ctx = sbie.Context(0)
        print(json.dumps({"near_field": run_near(ctx, max(2, args.steps // 4))}), flush=True)
        ctx.close()
        return
    if args.only_targets:
        import torch

        ctx = sbie.Context(0)
        tgeom = workloads.geometry(args.workload)
        tg = sbie.Geometry(ctx, tgeom, workloads.CONFIGS[args.workload]["p"])
        gen = torch.Generator(device="cuda")
        gen.manual_seed(5)
        td = torch.randn((2, tg.N), dtype=torch.float64, device="cuda", generator=gen)
        print(json.dumps({"targets": run_targets(tg, tgeom, td, max(3, args.steps // 4))}), flush=True)
        tg.close()
        ctx.close()
        return
    if args.only_stokes:
        ctx = sbie.Context(0)
        print(json.dumps({f"stokes_op{op}": {pr: run_stokes(ctx, max(2, args.steps // 2), 1, pr, op=op)
                                              for pr in ("fp64", "mixed")} for op in (2, 5, 6)}), flush=True)
        ctx.close()
        return
    geom = workloads.geometry(args.workload)
    p = workloads.CONFIGS[args.workload]["p"]
    M = len(geom["A"])
    ctx = sbie.Context(0)
    t0 = time.perf_counter()
    g = sbie.Geometry(ctx, geom, p)
    setup_s = time.perf_counter() - t0
    N = g.N
    gen = torch.Generator(device="cuda")
    gen.manual_seed(workloads.CONFIGS[args.workload]["seed"])
    dens = torch.randn((args.steps + args.warmup, 2, N), dtype=torch.float64, device="cuda", generator=gen)

    main_run = run(g, dens, args.steps, args.warmup, args.precision)
    main_run["roofline"]["traffic"] = counter_traffic(args.precision, args.workload)
    res = {
        "metric": "S/D operator applies/sec and pair-interactions/sec at 512 spheroids; p50/p99",
        "value": main_run["applies_per_s"],
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * main_run["elapsed_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{M} polydisperse prolate/oblate spheroids (RSA, volume fraction 0.25, "
                               f"min gap 0.02), p={p}, N={N} nodes, S and D, nrhs=1, "
                               f"precision={args.precision}",
                   "spheroids": M, "p": p, "nodes": N, "near_pairs": g.num_near_pairs,
                   "far_pairs_per_apply": main_run["far_pairs"]},
        "pair_interactions_per_s": main_run["pair_interactions_per_s"],
        "effective_all_pairs_per_s": main_run["effective_all_pairs_per_s"],
        "near_evals_per_s": main_run["near_evals_per_s"],
        "latency_ms": main_run["latency_ms"],
        "part_ms": main_run["part_ms"],
        "setup_s": setup_s,
        "roofline": main_run["roofline"],
    }
    if not args.no_secondary:
        other = "fp64" if args.precision == "mixed" else "mixed"
        sec = run(g, dens, max(4, args.steps // 2), 1, other)
        res[f"{other}_path"] = {k: sec[k] for k in ("applies_per_s", "pair_interactions_per_s", "latency_ms",
                                                    "part_ms")}
        res[f"{other}_path"]["roofline"] = dict(sec["roofline"], traffic=counter_traffic(other, args.workload))
    if not args.no_near:
        res["near_field"] = run_near(ctx, max(3, args.steps // 4))
    if not args.no_targets:
        res["targets"] = run_targets(g, geom, dens[0], max(3, args.steps // 4))
    if not args.no_multi:
        res["multi_density"] = {pr: run_multi(g, max(2, args.steps // 4), pr) for pr in ("mixed", "fp64")}
    if not args.no_derivatives:
        res["derivatives"] = {pr: run_normal(g, dens, max(3, args.steps // 4), pr) for pr in ("mixed", "fp64")}
    if not args.no_stokes:
        res["stokes"] = {pr: run_stokes(ctx, max(4, args.steps // 2), 1, pr) for pr in ("fp64", "mixed")}
        res["stokes_with_pressure"] = {pr: run_stokes(ctx, max(3, args.steps // 4), 1, pr, op=5)
                                       for pr in ("fp64", "mixed")}
        res["stokes_double_layer"] = {pr: run_stokes(ctx, max(3, args.steps // 4), 1, pr, op=6)
                                      for pr in ("fp64", "mixed")}
    if not args.no_solve:
        res["solve"] = {"gmres_study": gmres_study(ctx),
                        **{f"{args.workload}_{pr}": solve_large(ctx, args.workload, pr) for pr in ("mixed", "fp64")}}
    if not args.no_tree:
        res["tree_far_field"] = {args.workload: run_tree(g, dens, max(4, args.steps // 4)),
                                 "c3x8": tree_scaling(ctx, "c3x8", 3)}
    if args.tree_sweep:
        res["tree_sweep_fp64"] = tree_sweep(g, dens)
    if args.served_requests > 0:
        res["served"] = served(ctx, args.served_requests, args.served_rho, args.served_precision,
                               args.served_lanes, budgets=tuple(b << 30 for b in args.served_budget_gib),
                               batch=args.served_batch, tree=args.served_tree)
    if not args.no_cpu_baseline:
        d = dens[0].cpu().numpy()
        res["cpu_baseline"], tg, refs = cpu_baseline(geom, p, d[0], d[1], N, args.cpu_sample)
        res["error_vs_oracle"] = error_vs_oracle(g, dens[0], tg, refs)
    g.close()
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
