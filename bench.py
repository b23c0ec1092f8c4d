#!/usr/bin/env python
"""Throughput of the batched alpha/beta bound pass + gradient on one MI355X.

Workload (the branch-and-bound batch): the 3x32x32 ReLU CNN (conv 16@3x3 s1, 32@4x4 s2,
32@3x3 s1, 64@4x4 s2, all padding 1; FC 4096-512-10; He-normal weights, seed 0), 64 root
inputs uniform in [0, 1] with an L-inf box of radius 2/255, 64 subdomains per root (4096)
with 1-12 random ReLU split constraints each (drawn from the root's unstable neurons),
9 margin rows per subdomain.  Root pre-activation bounds come from full CROWN on the GPU
(set-up, untimed).  An optimisation step = for all 4096 subdomains: the bound pass with
alpha, beta and the splits (SAVE_FOR_GRAD, best-so-far kept), the gradient with respect to
alpha and beta, and one projected Adam step on each.  The whole optimisation (10 such steps
and a final pass) is captured as one HIP graph; a bench step is one replay of it, timed
with HIP events (mean, median, p10, p90).  value = subdomain-steps per second (10 x 4096
per replay).

Also reported: the same work one subdomain per call ("plain"), eager optimisation steps
with per-launch HIP events (kernel breakdown; the dominant kernel's roofline fraction from
its average launch duration), the other workloads (plain CROWN on the small MLP, full CROWN
on the deep MLP and on the CNN, alpha-CROWN on the CNN), the planning loop, and the FP64
CPU oracle timed on a bounded sample of the same units with all host threads and with one.
"""
from __future__ import annotations

import argparse
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12
PEAK_HBM = 8.0e12
METRIC = "subdomains bounded/sec (alpha,beta pass + grad), batched vs plain, at 1e-4 rel vs FP64"


def connections(layer):
    """Number of weight applications (multiply-adds) of one layer per coefficient row."""
    import numpy as np
    if layer["kind"] == "linear":
        return int(np.prod(layer["W"].shape))
    co, ci, kh, kw = layer["W"].shape
    _, H, Wd = layer["in_shape"]
    _, OH, OW = layer["out_shape"]
    s, p = layer["stride"], layer["pad"]
    vy = sum(1 for oy in range(OH) for ky in range(kh) if 0 <= oy * s - p + ky < H)
    vx = sum(1 for ox in range(OW) for kx in range(kw) if 0 <= ox * s - p + kx < Wd)
    return vy * vx * ci * co


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


def _ev():
    import torch
    return torch.cuda.Event(enable_timing=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="graph replays timed (one replay = the whole alpha/beta optimisation "
                         "of the batch)")
    ap.add_argument("--warmup", type=int, default=3, help="untimed graph replays")
    ap.add_argument("--eager-steps", type=int, default=5,
                    help="optimisation steps run eagerly with per-kernel HIP events (kernel "
                         "breakdown and the dominant kernel's roofline)")
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--per-root", type=int, default=64)
    ap.add_argument("--plain", type=int, default=256, help="subdomains timed one per call")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="oracle sample budget per thread setting")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the kernel autotuner")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (plain CROWN MLP, deep MLP, CNN full CROWN, "
                         "alpha-CROWN)")
    ap.add_argument("--plans", default=None,
                    help="JSON line of an earlier run: reuse its tuned kernel plans (its "
                         "'autotune' field) instead of tuning, so that profiler runs time the "
                         "same kernels")
    ap.add_argument("--bab-iters", type=int, default=10,
                    help="iterations of the branch-and-bound planning loop timed after the "
                         "main measurement (0: skip)")
    ap.add_argument("--no-recompute", action="store_true",
                    help="skip the stored vs checkpointed and the atomic vs deterministic "
                         "comparisons (profiling runs: the timed replays are then the last "
                         "launches of every kernel)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (a known-size kernel "
                         "for scaling the HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the batch of subdomains is independent per GPU "
              "and this build has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2412_09584_amd import rocprof_summary
    from paper_2412_09584_amd import binding as B
    from paper_2412_09584_amd.batch import BetaBatch, chosen_plans

    dev = torch.device("cuda")
    if args.calibrate_copy:
        src = torch.ones(1 << 28, device=dev)          # 1 GiB of float32
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = W.beta_cnn(args.roots, args.per_root)
    net = w.net
    R = w.spec.shape[1]
    # ---- set-up (untimed): root bounds by full CROWN, splits, device state
    bb = BetaBatch(w, args.per_root, split_seed=W.SPLIT_SEED, max_rows=36864)
    n = bb.n
    opt_steps = int(w.extra["steps"])
    stream = torch.cuda.current_stream()

    tune_log = None
    pinned = None
    if args.plans:
        with open(args.plans) as f:
            pinned = json.loads(f.read().strip().splitlines()[-1])["autotune"]
        bb.set_plans(pinned)
    elif not args.no_tune:
        tune_log = bb.autotune(stream)
        print(tune_log, file=sys.stderr)
    plans = pinned if pinned is not None else chosen_plans(tune_log)

    # ---- eager steps with per-kernel HIP events on the library's stream
    bb.reset()
    t = 0
    for _ in range(3):
        t += 1
        bb.step(t, stream)
    torch.cuda.synchronize()
    B.bound_profile_read(bb.bn.handle)          # discard
    B.bound_profile(bb.bn.handle, True)
    e0, e1 = _ev(), _ev()
    e0.record(stream)
    for _ in range(args.eager_steps):
        t += 1
        bb.step(t, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    B.bound_profile(bb.bn.handle, False)
    prof = B.bound_profile_read(bb.bn.handle)
    eager_ms = e0.elapsed_time(e1) / max(args.eager_steps, 1)

    # ---- the headline: the whole optimisation (steps x (pass + gradient + Adam) for every
    # subdomain, then the final pass) captured as one HIP graph and replayed
    opt = bb.optimizer(opt_steps)
    opt.capture()
    for _ in range(args.warmup):
        opt.replay()
    torch.cuda.synchronize()
    evs = [_ev() for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(args.steps):
        opt.replay()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)]
    ms_replay = evs[0].elapsed_time(evs[-1]) / args.steps
    units = n * opt_steps
    value = units / (ms_replay / 1e3)

    # ---- algorithmic work
    conn = [connections(l) for l in net]
    flop_unit = 2.0 * R * (sum(conn) + sum(conn[:-1]))
    tflops = flop_unit * value / 1e12

    def launch_flops(label):
        if label.startswith("bwd_relax_L") or label.startswith("adj_L"):
            m = int(label.rsplit("L", 1)[1])
            return 2.0 * R * conn[m - 1] * n
        if label == "bwd_conc_L1":
            return 2.0 * R * conn[0] * n
        return None

    gemm = {k: v for k, v in prof.items() if launch_flops(k) is not None}
    dom = max(gemm, key=lambda k: gemm[k][0])
    dom_ms = gemm[dom][0] / gemm[dom][1]
    dom_flops = launch_flops(dom)
    achieved = dom_flops / (dom_ms / 1e3)
    # HBM bytes per launch of the dominant kernel from the committed FETCH_SIZE /
    # WRITE_SIZE summary, if it was taken from the current kernel sources
    traffic = None
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        rec_t = rocprof_summary.read_traffic(path, dom)
        if rec_t is not None:
            traffic = rec_t["bytes"]
            break
    roofline = {"kernel": dom, "bound": "mfma", "achieved": achieved / 1e12,
                "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_MFMA, "traffic": traffic,
                "avg_launch_ms": dom_ms, "flop_per_launch": dom_flops,
                "timed_over": f"{args.eager_steps} eager optimisation steps (HIP events per launch)"}
    breakdown = {k: round(v[0] / max(args.eager_steps, 1), 4)
                 for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}

    # ---- plain path: one subdomain per call
    plain = plain_path(bb, min(args.plain, n), stream) if args.plain > 0 else None
    if plain is not None:
        plain["batched_speedup"] = value / plain["value"]

    recompute = None if args.no_recompute else recompute_compare(bb, stream)
    determinism = None if args.no_recompute else deterministic_compare(bb, stream)

    others = None
    if not args.no_configs:
        del opt
        torch.cuda.synchronize()
        others = other_configs(w, bb, stream)

    # ---- branch-and-bound planning loop (pick-out, split, search, bound, prune)
    bab = None
    if args.bab_iters > 0:
        bab = {"crown": bab_loop(args.bab_iters),
               "early_stop": bab_loop(args.bab_iters, bounding="early_stop"),
               "cem_early_stop": bab_loop(args.bab_iters, bounding="early_stop", search="cem")}

    # ---- CPU oracle on a bounded sample (rank 0, N=1)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, args.cpu_seconds)

    rec = {"metric": METRIC, "value": value, "unit": "subdomains/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_replay,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"beta-crown BaB batch: CNN 3x32x32 c16k3s1-c32k4s2-c32k3s1-"
                                  f"c64k4s2-fc4096-512-10, {args.roots} roots x {args.per_root} "
                                  f"subdomains, 1-12 splits, {R} margin rows, eps 2/255, "
                                  f"{opt_steps} alpha/beta steps per graph replay",
                      "subdomains": n, "rows": R, "split_nnz": bb.nnz,
                      "units_per_step": units, "parallelism": "none"},
           "step": "one HIP-graph replay of the whole optimisation: per subdomain "
                   f"{opt_steps} x (bound pass + alpha/beta gradient + Adam) and a final pass",
           "replay_ms": {"mean": ms_replay, "median": _pct(per, 50), "p10": _pct(per, 10),
                         "p90": _pct(per, 90), "n": len(per)},
           "eager_ms_per_opt_step": eager_ms, "eager_value": n / (eager_ms / 1e3),
           "tflops_step": tflops, "flop_per_subdomain": flop_unit,
           "roofline_frac_step": tflops * 1e12 / PEAK_FP32_MFMA, "wall_s": wall,
           "plain": plain, "roofline": roofline, "kernel_ms_per_step": breakdown,
           "determinism": determinism,
           "autotune": plans, "checkpointed_recompute": recompute, "configs": others,
           "bab_loop": bab, "cpu_baseline": cpu}
    print(json.dumps(rec))


def _saved_floats_per_row(net, lo, hi, recompute):
    """Floats the gradient's saved state takes per coefficient row: the concretised layer's
    coefficients (dense), plus either every relaxed layer's pre-relaxation coefficients at
    its unstable neurons (mean over the bound rows lo / hi) or, checkpointed, the
    coefficient rows at every c-th product (c = ceil(sqrt(L - 1))) and the largest
    segment's layers."""
    import numpy as np
    L = len(net)
    d = [int(np.prod(net[0]["in_shape"]))] + [int(np.prod(l["out_shape"])) for l in net]
    if not recompute:
        unst = ((lo < 0) & (hi > 0)).sum(axis=1).mean()
        return float(d[0] + unst)
    c = 1
    while c * c < L - 1:
        c += 1
    f, seg = d[0], 0
    for t in range(L, 1, -c):
        f += d[t]
        seg = max(seg, sum(d[p - 1] for p in range(t, max(t - c, 1), -1)))
    return float(f + seg)


def recompute_compare(bb, stream, steps=5):
    """One optimisation step (pass + gradient + Adam) of the batch with the saved
    coefficients kept for every layer, and with checkpointed recomputation: time and the
    saved bytes per subdomain."""
    import torch
    lo, hi = bb.lo.double().cpu().numpy(), bb.hi.double().cpu().numpy()
    out = {}
    for mode in (False, True):
        bb.recompute = mode
        bb.reset()
        bb.step(1, stream)
        torch.cuda.synchronize()
        e0, e1 = _ev(), _ev()
        e0.record(stream)
        for t in range(2, steps + 2):
            bb.step(t, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out["checkpointed" if mode else "stored"] = {
            "ms_per_step": ms, "subdomains_per_s": bb.n / (ms / 1e3),
            "saved_bytes_per_subdomain": 4.0 * bb.R * _saved_floats_per_row(bb.w.net, lo, hi, mode)}
    bb.recompute = False
    bb.reset()
    return out


def deterministic_compare(bb, stream, steps=5):
    """One optimisation step of the batch with the row sums formed without float atomics
    (BOUND_OPT_DETERMINISTIC): time per step, and whether two passes from the same state
    give bitwise the same bounds (with and without the mode)."""
    import torch

    from paper_2412_09584_amd import binding as B
    out = {}
    for det in (False, True):
        B.bound_set_options(bb.bn.handle, B.BOUND_OPT_DETERMINISTIC if det else 0)
        lows = []
        for _ in range(2):
            bb.reset()
            bb.bound_and_grad(stream)
            torch.cuda.synchronize()
            lows.append(bb.lower.clone())
        bb.reset()
        bb.step(1, stream)
        torch.cuda.synchronize()
        e0, e1 = _ev(), _ev()
        e0.record(stream)
        for t in range(2, steps + 2):
            bb.step(t, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out["deterministic" if det else "atomic"] = {
            "ms_per_step": ms, "bitwise_repeat": bool(torch.equal(lows[0], lows[1])),
            "max_rel_diff_between_repeats": float(((lows[0] - lows[1]).abs() /
                                                    lows[1].abs().clamp_min(1.0)).max())}
    B.bound_set_options(bb.bn.handle, 0)
    bb.reset()
    return out


def plain_path(bb, m, stream):
    """The same units one subdomain per call (n_inst = 1, per-layer kernels, no graph)."""
    import torch

    from paper_2412_09584_amd import binding as B
    dev = bb.alpha.device
    R, L, n_relu = bb.R, bb.L, bb.bn.n_relu
    sp, spd = bb.splits, bb.spd
    per = []
    for i in range(m):
        q0, q1 = int(sp.off[i]), int(sp.off[i + 1])
        per.append(dict(
            C=bb.C[i:i + 1].contiguous(), x_lo=bb.x_lo[i:i + 1].contiguous(),
            x_hi=bb.x_hi[i:i + 1].contiguous(), bof=bb.bof[i:i + 1].contiguous(),
            alpha=torch.full((1, n_relu), bb.alpha0, device=dev),
            ma=torch.zeros(1, n_relu, device=dev), va=torch.zeros(1, n_relu, device=dev),
            off=torch.tensor([0, q1 - q0], dtype=torch.int32, device=dev),
            idx=spd["idx"][q0:q1].contiguous(), sign=spd["sign"][q0:q1].contiguous(),
            beta=torch.zeros(q1 - q0, R, device=dev), mb=torch.zeros(q1 - q0, R, device=dev),
            vb=torch.zeros(q1 - q0, R, device=dev), nnz=q1 - q0,
            lower=torch.empty(1, R, device=dev), best=torch.full((1, R), -float("inf"), device=dev),
            ga=torch.empty(1, n_relu, device=dev), gb=torch.empty(max(q1 - q0, 1), R, device=dev)))
    ones1 = torch.ones(1, R, device=dev)

    def unit(u, tt):
        B.bound_backward(bb.bn.handle, 1, R, L, spec=u["C"], lo=bb.lo, hi=bb.hi,
                         n_bounds=bb.n_roots, bound_of=u["bof"], alpha=u["alpha"],
                         split_off=u["off"], split_idx=u["idx"], split_sign=u["sign"], nnz=u["nnz"],
                         beta=u["beta"] if u["nnz"] else None, x_lo=u["x_lo"], x_hi=u["x_hi"],
                         flags=B.BOUND_SAVE_FOR_GRAD, lower=u["lower"], best=u["best"],
                         stream=stream)
        B.bound_grad(bb.bn.handle, ones1, u["ga"], u["gb"][:u["nnz"]] if u["nnz"] else None,
                     stream=stream)
        B.bound_adam(u["alpha"], u["ga"], u["ma"], u["va"], tt, bb.lr, grad_scale=-1.0,
                     clip_lo=0.0, clip_hi=1.0, stream=stream)
        if u["nnz"]:
            B.bound_adam(u["beta"], u["gb"][:u["nnz"]], u["mb"], u["vb"], tt, bb.lr,
                         grad_scale=-1.0, clip_lo=0.0, stream=stream)

    for u in per[:4]:
        unit(u, 1)
    torch.cuda.synchronize()
    e0, e1 = _ev(), _ev()
    e0.record(stream)
    for u in per:
        unit(u, 2)
    e1.record(stream)
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1)
    return {"value": m / (pms / 1e3), "unit": "subdomains/s", "sample": m,
            "ms_per_subdomain": pms / m,
            "path": "n_inst = 1 per call, per-layer kernels, no graph"}


def crown_flops(net, rows_final):
    """Algorithmic FLOP of full CROWN on one input: every pre-activation layer k bounded
    by a backward pass with rows [I; -I] through the products of layers k-1 .. 1 (the
    first step A W_k with A = I is a gather, not a product), then the spec rows [C; -C]
    through all layers; 2 FLOP per weight application, padding taps excluded."""
    import numpy as np
    conn = [connections(l) for l in net]
    dims = [int(np.prod(l["out_shape"])) for l in net]
    f = sum(2.0 * 2 * dims[k - 1] * sum(conn[:k - 1]) for k in range(2, len(net)))
    return f + 2.0 * 2 * rows_final * sum(conn)


def _time(fn, reps, warm=2):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _ev(), _ev()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def other_configs(w_cnn, bb, stream):
    """The smaller workloads, each with its own unit: plain CROWN on the small MLP (latency,
    eager and as one HIP graph), full CROWN on the deep MLP and on the CNN (inputs/s and
    the fraction of the FP32 MFMA peak), alpha-CROWN on the CNN (input-steps/s)."""
    import torch

    import workloads as W
    from paper_2412_09584_amd import net as N
    out = {}
    # plain CROWN, MLP 784-100-100-10, one input: lower and upper bounds of z_1, z_2 and the
    # margins
    w0 = W.mlp_small()
    bn0 = N.BoundNet(w0.net, 1, 4096)
    C0 = torch.as_tensor(w0.spec, device="cuda")
    xl0, xh0 = torch.as_tensor(w0.x_lo, device="cuda"), torch.as_tensor(w0.x_hi, device="cuda")

    def full0():
        lo, hi = bn0.crown_bounds(xl0, xh0)
        return bn0.spec_bounds(C0, lo, hi, xl0, xh0)

    us_eager = 1e3 * _time(full0, 50, 5)
    g0 = torch.cuda.CUDAGraph()
    full0()
    torch.cuda.synchronize()
    with torch.cuda.graph(g0):
        full0()
    us_graph = 1e3 * _time(g0.replay, 200, 5)
    out["plain_crown_mlp784-100-100-10_1_input"] = {
        "us_per_full_crown_eager": us_eager, "us_per_full_crown_graph": us_graph,
        "flop": crown_flops(w0.net, 9), "bound": "launch latency"}
    del g0, bn0
    # full CROWN, MLP 784-256x6-10, 256 inputs
    w1 = W.mlp_deep(256)
    bn1 = N.BoundNet(w1.net, 256, 256 * 512)
    C1 = torch.as_tensor(w1.spec, device="cuda")
    xl1, xh1 = torch.as_tensor(w1.x_lo, device="cuda"), torch.as_tensor(w1.x_hi, device="cuda")

    def full1():
        lo, hi = bn1.crown_bounds(xl1, xh1)
        return bn1.spec_bounds(C1, lo, hi, xl1, xh1)

    ms1 = _time(full1, 10, 2)
    f1 = crown_flops(w1.net, 9)
    out["full_crown_mlp784-256x6-10_256_inputs"] = {
        "inputs_per_s": 256 / (ms1 / 1e3), "ms_per_batch": ms1, "flop_per_input": f1,
        "tflops": f1 * 256 / (ms1 / 1e3) / 1e12,
        "frac_fp32_mfma": f1 * 256 / (ms1 / 1e3) / PEAK_FP32_MFMA}
    del bn1
    # full CROWN, the CNN, 64 inputs (the roots of the batch above)
    bn2 = bb.bn
    C2 = torch.as_tensor(w_cnn.spec, device="cuda")
    xl2, xh2 = torch.as_tensor(w_cnn.x_lo, device="cuda"), torch.as_tensor(w_cnn.x_hi, device="cuda")
    n2 = C2.shape[0]

    def full2():
        lo, hi = bn2.crown_bounds(xl2, xh2)
        return bn2.spec_bounds(C2, lo, hi, xl2, xh2)

    ms2 = _time(full2, 3, 1)
    f2 = crown_flops(w_cnn.net, 9)
    out[f"full_crown_cnn_{n2}_inputs"] = {
        "inputs_per_s": n2 / (ms2 / 1e3), "ms_per_batch": ms2, "flop_per_input": f2,
        "tflops": f2 * n2 / (ms2 / 1e3) / 1e12,
        "frac_fp32_mfma": f2 * n2 / (ms2 / 1e3) / PEAK_FP32_MFMA,
        "note": "padding taps excluded from the FLOP count"}
    # alpha-CROWN on the CNN: 64 inputs, 20 Adam steps, as one HIP graph
    lo, hi = bn2.crown_bounds(xl2, xh2)
    opt = N.AlphaBetaOptimizer(bn2, C2, lo, hi, xl2, xh2, steps=20, lr=0.1, alpha0=0.5,
                               use_beta=False)
    opt.capture()
    ms3 = _time(opt.replay, 5, 1)
    conn = [connections(l) for l in w_cnn.net]
    fu = 2.0 * 9 * (sum(conn) + sum(conn[:-1]))
    out[f"alpha_crown_cnn_{n2}_inputs_20_steps"] = {
        "input_steps_per_s": n2 * 20 / (ms3 / 1e3), "ms_per_replay": ms3, "flop_per_unit": fu,
        "frac_fp32_mfma": fu * n2 * 20 / (ms3 / 1e3) / PEAK_FP32_MFMA}
    del opt
    out["planning_unrolled_pushing_H20"] = planning_unrolled()
    out["standalone_concretize"] = standalone_concretize(stream)
    return out


def standalone_concretize(stream, n=4096, rows=9, d0=3072, reps=20):
    """Theorem 2 on its own (bound_concretize): coefficient rows G_1 [n, rows, d0] of the
    CNN's input width against per-instance boxes; HBM-bound, reported as GB/s of the
    algorithmic bytes (G_1, the boxes, offsets and bounds, each once) and as a fraction of
    the 8 TB/s HBM peak."""
    import torch

    from paper_2412_09584_amd import binding as B
    g = torch.Generator(device="cuda")
    g.manual_seed(17)
    coeff = torch.randn(n, rows, d0, device="cuda", generator=g)
    offset = torch.randn(n, rows, device="cuda", generator=g)
    mag = torch.rand(n, rows, device="cuda", generator=g)
    x = torch.rand(n, d0, device="cuda", generator=g)
    x_lo, x_hi = x - 0.01, x + 0.01
    lower = torch.empty(n, rows, device="cuda")

    def run():
        B.bound_concretize(n, rows, d0, coeff, offset, mag, x_lo, x_hi, 0, lower, stream=stream)

    ms = _time(run, reps, 3)
    nbytes = 4.0 * (n * rows * d0 + 2 * n * d0 + 3 * n * rows)
    gbs = nbytes / (ms / 1e3) / 1e9
    return {"shape": f"G_1 [{n}, {rows}, {d0}] + boxes [{n}, {d0}]", "ms": ms,
            "algorithmic_bytes": nbytes, "gb_per_s": gbs, "frac_hbm": gbs * 1e9 / PEAK_HBM}


def planning_unrolled(n=256, n_opt=64, samples=64, steps=2, stops=(77, 65, 41)):
    """The planning-shaped workload: the Pushing dynamics MLP unrolled over 20 steps (82
    layers, input = 40 action values), L1 objective, bounded over n action sub-boxes.
    Compared: full CROWN (every pre-activation layer bounded by a backward pass: 81
    passes), optimised intermediate bounds (each pass's slopes optimised, `steps` Adam
    steps per layer, on n_opt sub-boxes), and the paper's bounding -- pre-activation
    bounds from `samples` search samples per sub-box, then the objective's pass stopped
    early at a ReLU layer.  Reported per method: sub-boxes per second, the mean lower
    bound of the objective and the fraction that is finite, beside the mean best sample
    value (what the bound estimates from below)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2412_09584_amd import binding as B
    from paper_2412_09584_amd import net as N
    uw = W.pushing_unrolled(20)
    lo_b, hi_b = W.action_subboxes(uw, n, seed=61)
    xl, xh = torch.as_tensor(lo_b, device="cuda"), torch.as_tensor(hi_b, device="cuda")
    C = torch.ones(n, 1, 1, device="cuda")
    width = max(W.out_dim(l) for l in uw.net)
    bn = N.BoundNet(uw.net, n, max(n * 2 * width, n * samples), n)

    def stats(v):
        v = v.detach().double().cpu().numpy().ravel()
        fin = np.isfinite(v)
        return {"mean_lower": float(v[fin].mean()) if fin.any() else None,
                "finite": float(fin.mean())}

    out = {"layers": len(uw.net), "relu_layers": len(uw.net) - 1, "subdomains": n}

    def full():
        lo, hi = bn.crown_bounds(xl, xh)
        return bn.spec_bounds(C, lo, hi, xl, xh, both=False)[0]

    ms = _time(full, 2, 1)
    out["full_crown"] = {"subdomains_per_s": n / (ms / 1e3), "ms": ms, **stats(full())}
    # the objective's pass with its gradient (random slopes) on these bounds: every layer's
    # coefficients kept vs checkpointed recomputation
    lo, hi = bn.crown_bounds(xl, xh)
    alpha = torch.rand(n, bn.n_relu, device="cuda", generator=torch.Generator("cuda").manual_seed(63))
    low = torch.empty(n, 1, device="cuda")
    ones = torch.ones(n, 1, device="cuda")
    ga = torch.empty(n, bn.n_relu, device="cuda")
    lo_np, hi_np = lo.double().cpu().numpy(), hi.double().cpu().numpy()
    for mode in (0, B.BOUND_RECOMPUTE):
        def pg(mode=mode):
            B.bound_backward(bn.handle, n, 1, len(uw.net), spec=C, lo=lo, hi=hi, n_bounds=n,
                             alpha=alpha, x_lo=xl, x_hi=xh, flags=B.BOUND_SAVE_FOR_GRAD | mode,
                             lower=low)
            B.bound_grad(bn.handle, ones, ga)
        ms = _time(pg, 3, 1)
        out["pass_and_gradient_" + ("checkpointed" if mode else "stored")] = {
            "subdomains_per_s": n / (ms / 1e3), "ms": ms,
            "saved_bytes_per_subdomain": 4.0 * _saved_floats_per_row(uw.net, lo_np, hi_np, bool(mode))}
    # the paper's bounding: search samples -> empirical pre-activation bounds -> early stop
    rng = np.random.default_rng(62)
    U = torch.as_tensor(rng.uniform(0, 1, (n, samples, lo_b.shape[1])), dtype=torch.float32,
                        device="cuda")
    x = (xl[:, None, :] + (xh - xl)[:, None, :] * U).reshape(n * samples, -1).contiguous()
    slo = torch.empty(n, bn.n_relu, device="cuda")
    shi = torch.empty_like(slo)
    fval = torch.empty(n * samples, 1, device="cuda")
    B.bound_sample_bounds(bn.handle, n, samples, x, slo, shi, fval)
    out["best_sample_mean"] = float(fval.reshape(n, samples).min(dim=1).values.mean())
    for s in stops:
        def early(s=s):
            B.bound_sample_bounds(bn.handle, n, samples, x, slo, shi)
            return bn.spec_bounds(C, slo, shi, xl, xh, both=False, stop_layer=s,
                                  stop_mode=B.BOUND_STOP_RELU)[0]
        ms = _time(early, 5, 1)
        out[f"search_bounds_early_stop_at_relu_{s}"] = {"subdomains_per_s": n / (ms / 1e3),
                                                        "ms": ms, **stats(early())}
    del bn
    bo = N.BoundNet(uw.net, n_opt, n_opt * 2 * width, n_opt * 2 * width)

    def opt():
        lo, hi = bo.alpha_crown_bounds(xl[:n_opt], xh[:n_opt], steps=steps)
        return bo.spec_bounds(C[:n_opt], lo, hi, xl[:n_opt], xh[:n_opt], both=False)[0]

    ms = _time(opt, 1, 0)
    out["optimised_intermediate"] = {"subdomains_per_s": n_opt / (ms / 1e3), "ms": ms,
                                     "subdomains": n_opt, "adam_steps_per_layer": steps,
                                     **stats(opt())}
    del bo
    out["planning_loop"] = bab_loop_unrolled(uw)
    return out


def bab_loop_unrolled(uw, iters=10, n_pick=256, samples=64, rounds=3, n_elite=8, stop=77):
    """The paper's planning method on the unrolled chain: branch and bound over the action
    box with the CEM search, search-integrated bounds and the objective's pass stopped at
    ReLU layer `stop`; random numbers drawn on the device."""
    import torch

    import workloads as W
    from paper_2412_09584_amd.bab import BaBPlanner
    pl = BaBPlanner(uw.net, uw.u_lo, uw.u_hi, n_pick=n_pick, samples=samples,
                    bounding="early_stop", stop_layer=stop, search="cem", cem_rounds=rounds,
                    n_elite=n_elite)
    gu = torch.Generator(device="cuda").manual_seed(W.PLAN_SEED)
    gn = torch.Generator(device="cuda").manual_seed(W.PLAN_SEED + 1)
    uni = lambda tag, shape: torch.rand(shape, device="cuda", generator=gu)
    nrm = lambda tag, shape: torch.randn(shape, device="cuda", generator=gn)
    gum = lambda tag, shape: torch.empty(shape, device="cuda").exponential_(generator=gu).log_().neg_()
    root_best, _, _, _ = pl.run(0, uni, normals=nrm, gumbels=gum)
    pl.run(1, uni, normals=nrm, gumbels=gum)        # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best, _, P, log = pl.run(iters, uni, trace=True, normals=nrm, gumbels=gum)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bounded = sum(2 * len(e["picked"]) for e in log)
    return {"search": f"cem {rounds} rounds x {samples} samples, {n_elite} elites",
            "bounding": f"search-integrated bounds, early stop at ReLU {stop}",
            "n_pick": n_pick, "iters": len(log), "ms_per_iter": 1e3 * dt / max(len(log), 1),
            "subdomains_bounded_per_s": bounded / dt if log else None,
            "root_search_best": root_best, "best": best, "candidates": int(P["lo"].shape[0])}


def bab_loop(iters, d=16, hidden=(256, 256, 256), n_pick=1024, samples=64, bounding="crown",
             search="uniform", rounds=3, n_elite=8):
    """Throughput of the planning loop (Algorithm 2) on a seeded scalar ReLU objective over
    [-1, 1]^d: each iteration picks n_pick subdomains, splits them, searches the 2 n_pick
    children (uniform: `samples` each; CEM: `rounds` rounds of `samples`) and bounds them
    -- with full CROWN, or with the paper's search-integrated bounds and an early stop at
    the last ReLU layer -- then prunes.  The random numbers are drawn on the device."""
    import torch

    import workloads as W
    from paper_2412_09584_amd.bab import BaBPlanner
    net, lo, hi = W.plan_objective(d=d, hidden=hidden)
    pl = BaBPlanner(net, lo, hi, n_pick=n_pick, samples=samples, bounding=bounding, search=search,
                    cem_rounds=rounds, n_elite=n_elite)
    gu = torch.Generator(device="cuda").manual_seed(W.PLAN_SEED)
    gn = torch.Generator(device="cuda").manual_seed(W.PLAN_SEED + 1)
    uni = lambda tag, shape: torch.rand(shape, device="cuda", generator=gu)
    nrm = lambda tag, shape: torch.randn(shape, device="cuda", generator=gn)
    # standard Gumbel variates: -log of a standard exponential
    gum = lambda tag, shape: torch.empty(shape, device="cuda").exponential_(generator=gu).log_().neg_()
    pl.run(2, uni, normals=nrm, gumbels=gum)         # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best, _, P, log = pl.run(iters, uni, trace=True, normals=nrm, gumbels=gum)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bounded = sum(2 * len(e["picked"]) for e in log)          # children searched and bounded
    return {"objective": f"MLP {d}-{'-'.join(map(str, hidden))}-1 over [-1,1]^{d}", "bounding": bounding,
            "search": search if search == "uniform" else f"cem {rounds} rounds, {n_elite} elites",
            "n_pick": n_pick, "samples": samples, "iters": len(log),
            "ms_per_iter": 1e3 * dt / max(len(log), 1),
            "subdomains_bounded_per_s": bounded / dt if log else None,
            "best": best, "candidates": int(P["lo"].shape[0])}


def _cpu_model():
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return None


def _oracle_units(w, budget_s):
    """The FP64 oracle (as it stands) on subdomains of root 0 for about budget_s seconds:
    per subdomain the bound, its alpha/beta gradient and one Adam step."""
    import numpy as np

    from oracle import crown as O
    import workloads as W
    g = np.load(os.path.join(ROOT, "tests", "golden", "cnn_root0.npz"))
    net = w.net
    lo = g["lo"].astype(np.float32).astype(np.float64)
    hi = g["hi"].astype(np.float32).astype(np.float64)
    bounds = list(zip(O.per_layer(net, lo), O.per_layer(net, hi)))
    cand = np.nonzero((lo < 0) & (hi > 0))[0]
    sp = W.random_splits([cand], 256, 1, 12, seed=W.SPLIT_SEED)
    L = len(net)
    C = w.spec[0].astype(np.float64)
    done = 0
    t0 = time.perf_counter()
    while done < 256 and time.perf_counter() - t0 < budget_s:
        q0, q1 = sp.off[done], sp.off[done + 1]
        splits = O.split_list(net, sp.neuron[q0:q1], sp.sign[q0:q1])
        alpha = [np.full(len(l), 0.5) for (l, _) in bounds]
        beta = np.zeros((q1 - q0, C.shape[0]))
        O.spec_lower(net, L, C, bounds, w.x_lo[0], w.x_hi[0], alpha, splits, beta)
        _, ga, gb = O.spec_lower_grad(net, L, C, bounds, w.x_lo[0], w.x_hi[0], alpha, splits, beta)
        for i in range(len(alpha)):
            O.adam_step(alpha[i], -ga[i], np.zeros_like(ga[i]), np.zeros_like(ga[i]), 1, 0.1, lo=0.0, hi=1.0)
        O.adam_step(beta, -gb, np.zeros_like(gb), np.zeros_like(gb), 1, 0.1, lo=0.0)
        done += 1
    return done, time.perf_counter() - t0


def cpu_baseline(w, budget_s):
    """The oracle on a bounded sample of the same units, with every host thread as BLAS
    threads and with one thread."""
    threads = os.cpu_count()
    limits = None
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [threads])
        limits = threadpool_limits
    except Exception:
        pass
    done, el = _oracle_units(w, budget_s)
    one = None
    if limits is not None:
        with limits(limits=1):
            d1, e1 = _oracle_units(w, budget_s)
        one = {"value": d1 / e1, "unit": "subdomains/s", "cores": 1,
               "sample": f"{d1} subdomains of root 0, {e1:.1f} s"}
    return {"value": done / el, "unit": "subdomains/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} subdomains of root 0 (bound + alpha/beta gradient + Adam step), "
                      f"{el:.1f} s", "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(),
            "one_thread": one}


if __name__ == "__main__":
    main()
