#!/usr/bin/env python
"""Throughput of the batched alpha/beta bound pass + gradient on one MI355X.

Workload (the branch-and-bound batch): the 3x32x32 ReLU CNN (conv 16@3x3 s1, 32@4x4 s2,
32@3x3 s1, 64@4x4 s2, all padding 1; FC 4096-512-10; He-normal weights, seed 0), 64 root
inputs uniform in [0, 1] with an L-inf box of radius 2/255, 64 subdomains per root (4096)
with 1-12 random ReLU split constraints each (drawn from the root's unstable neurons),
9 margin rows per subdomain.  Root pre-activation bounds come from full CROWN on the GPU
(set-up, untimed).  One step = for all 4096 subdomains: the bound pass with alpha, beta
and the splits (SAVE_FOR_GRAD, best-so-far kept), the gradient with respect to alpha and
beta, and one projected Adam step on each.  value = subdomains per second.

Also reported: the same work one subdomain per call ("plain"), the dominant kernel's
roofline fraction (its average launch duration from HIP events on its own stream during
the timed steps), and the FP64 CPU oracle timed on a bounded sample of the same units.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--per-root", type=int, default=64)
    ap.add_argument("--plain", type=int, default=256, help="subdomains timed one per call")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample budget")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the kernel autotuner")
    ap.add_argument("--plans", default=None,
                    help="JSON line of an earlier run: reuse its tuned kernel plans (its "
                         "'autotune' field) instead of tuning, so that profiler runs time the "
                         "same kernels")
    ap.add_argument("--bab-iters", type=int, default=10,
                    help="iterations of the branch-and-bound planning loop timed after the "
                         "main measurement (0: skip)")
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
    from paper_2412_09584_amd import net as N

    dev = torch.device("cuda")
    if args.calibrate_copy:
        src = torch.ones(1 << 28, device=dev)          # 1 GiB of float32
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = W.beta_cnn(args.roots, args.per_root)
    net = w.net
    L = len(net)
    R = w.spec.shape[1]
    n = args.roots * args.per_root
    bn = N.BoundNet(net, max_inst=n, max_rows=max(n * R, 36864), max_save_rows=n * R)

    # ---- set-up (untimed): root bounds, splits, device state
    lo, hi = bn.crown_bounds(w.x_lo, w.x_hi)
    lo_np, hi_np = lo.cpu().numpy(), hi.cpu().numpy()
    root_of = np.repeat(np.arange(args.roots), args.per_root).astype(np.int32)
    cands = [np.nonzero((lo_np[r] < 0) & (hi_np[r] > 0))[0] for r in range(args.roots)]
    sp = W.random_splits(cands, n, w.extra["kmin"], w.extra["kmax"], seed=W.SPLIT_SEED,
                         root_of=root_of)
    spd = N.splits_to_device(sp)
    C = torch.as_tensor(w.spec[root_of], device=dev)
    x_lo = torch.as_tensor(w.x_lo[root_of], device=dev)
    x_hi = torch.as_tensor(w.x_hi[root_of], device=dev)
    bof = torch.as_tensor(root_of, device=dev)
    n_relu = bn.n_relu
    alpha = torch.full((n, n_relu), w.extra["alpha0"], device=dev)
    beta = torch.zeros(sp.nnz, R, device=dev)
    ma, va = torch.zeros_like(alpha), torch.zeros_like(alpha)
    mb, vb = torch.zeros_like(beta), torch.zeros_like(beta)
    ga = torch.empty_like(alpha)
    gb = torch.empty_like(beta)
    lower = torch.empty(n, R, device=dev)
    best = torch.full((n, R), -float("inf"), device=dev)
    ones = torch.ones(n, R, device=dev)
    lr = w.extra["lr"]
    stream = torch.cuda.current_stream()

    def step(t, h=bn.handle):
        B.bound_backward(h, n, R, L, spec=C, lo=lo, hi=hi, n_bounds=args.roots, bound_of=bof,
                         alpha=alpha, split_off=spd["off"], split_idx=spd["idx"],
                         split_sign=spd["sign"], nnz=sp.nnz, beta=beta, x_lo=x_lo, x_hi=x_hi,
                         flags=B.BOUND_SAVE_FOR_GRAD, lower=lower, best=best, stream=stream)
        B.bound_grad(h, ones, ga, gb, stream=stream)
        B.bound_adam(alpha, ga, ma, va, t, lr, grad_scale=-1.0, clip_lo=0.0, clip_hi=1.0,
                     stream=stream)
        B.bound_adam(beta, gb, mb, vb, t, lr, grad_scale=-1.0, clip_lo=0.0, stream=stream)

    tune_log = None
    pinned = None
    if args.plans:
        with open(args.plans) as f:
            pinned = json.loads(f.read().strip().splitlines()[-1])["autotune"]
        for key, plan in pinned.items():
            path, cfg, cc = plan.split()[:3]
            B.bound_set_plan(bn.handle, key[0], int(key[1:]), 1 if path == "direct" else 2,
                             int(cfg.split("=")[1]), int(cc.split("=")[1]))
    elif not args.no_tune:
        tune_log = B.bound_autotune(bn.handle, n, R, L, grad_lower=ones, spec=C, lo=lo, hi=hi,
                                    n_bounds=args.roots, bound_of=bof, alpha=alpha,
                                    split_off=spd["off"], split_idx=spd["idx"],
                                    split_sign=spd["sign"], nnz=sp.nnz, beta=beta, x_lo=x_lo,
                                    x_hi=x_hi, flags=B.BOUND_SAVE_FOR_GRAD, lower=lower,
                                    stream=stream)
        best.fill_(-float("inf"))
        print(tune_log, file=sys.stderr)
    t = 0
    for _ in range(args.warmup):
        t += 1
        step(t)
    torch.cuda.synchronize()
    B.bound_profile_read(bn.handle)          # discard
    B.bound_profile(bn.handle, True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        t += 1
        step(t)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    B.bound_profile(bn.handle, False)
    prof = B.bound_profile_read(bn.handle)
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = n / (ms_step / 1e3)

    # ---- algorithmic work
    conn = [connections(l) for l in net]
    flop_unit = 2.0 * R * (sum(conn) + sum(conn[:-1]))
    tflops = flop_unit * n / (ms_step / 1e3) / 1e12

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
                "avg_launch_ms": dom_ms, "flop_per_launch": dom_flops}
    breakdown = {k: round(v[0] / args.steps, 4) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}

    # ---- plain path: one subdomain per call
    plain = None
    if args.plain > 0:
        m = min(args.plain, n)
        per = []
        for i in range(m):
            q0, q1 = int(sp.off[i]), int(sp.off[i + 1])
            per.append(dict(
                C=C[i:i + 1].contiguous(), x_lo=x_lo[i:i + 1].contiguous(),
                x_hi=x_hi[i:i + 1].contiguous(), bof=bof[i:i + 1].contiguous(),
                alpha=alpha[i:i + 1].clone(), ma=torch.zeros(1, n_relu, device=dev),
                va=torch.zeros(1, n_relu, device=dev),
                off=torch.tensor([0, q1 - q0], dtype=torch.int32, device=dev),
                idx=spd["idx"][q0:q1].contiguous(), sign=spd["sign"][q0:q1].contiguous(),
                beta=beta[q0:q1].clone(), mb=torch.zeros(q1 - q0, R, device=dev),
                vb=torch.zeros(q1 - q0, R, device=dev), nnz=q1 - q0,
                lower=torch.empty(1, R, device=dev), best=torch.full((1, R), -float("inf"), device=dev),
                ga=torch.empty(1, n_relu, device=dev), gb=torch.empty(max(q1 - q0, 1), R, device=dev)))
        ones1 = torch.ones(1, R, device=dev)

        def plain_unit(u, tt):
            B.bound_backward(bn.handle, 1, R, L, spec=u["C"], lo=lo, hi=hi, n_bounds=args.roots,
                             bound_of=u["bof"], alpha=u["alpha"], split_off=u["off"],
                             split_idx=u["idx"], split_sign=u["sign"], nnz=u["nnz"],
                             beta=u["beta"] if u["nnz"] else None, x_lo=u["x_lo"], x_hi=u["x_hi"],
                             flags=B.BOUND_SAVE_FOR_GRAD, lower=u["lower"], best=u["best"],
                             stream=stream)
            B.bound_grad(bn.handle, ones1, u["ga"], u["gb"] if u["nnz"] else None, stream=stream)
            B.bound_adam(u["alpha"], u["ga"], u["ma"], u["va"], tt, lr, grad_scale=-1.0,
                         clip_lo=0.0, clip_hi=1.0, stream=stream)
            if u["nnz"]:
                B.bound_adam(u["beta"], u["gb"], u["mb"], u["vb"], tt, lr, grad_scale=-1.0,
                             clip_lo=0.0, stream=stream)

        for u in per[:4]:
            plain_unit(u, 1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for u in per:
            plain_unit(u, 2)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1)
        plain = {"value": m / (pms / 1e3), "unit": "subdomains/s", "sample": m,
                 "ms_per_subdomain": pms / m, "batched_speedup": value / (m / (pms / 1e3))}

    # ---- branch-and-bound planning loop (pick-out, split, search, bound, prune)
    bab = bab_loop(args.bab_iters) if args.bab_iters > 0 else None

    # ---- CPU oracle on a bounded sample (rank 0, N=1)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, args.cpu_seconds)

    rec = {"metric": METRIC, "value": value, "unit": "subdomains/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"beta-crown BaB batch: CNN 3x32x32 c16k3s1-c32k4s2-c32k3s1-"
                                  f"c64k4s2-fc4096-512-10, {args.roots} roots x {args.per_root} "
                                  f"subdomains, 1-12 splits, {R} margin rows, eps 2/255",
                      "subdomains": n, "rows": R, "split_nnz": sp.nnz, "parallelism": "none"},
           "tflops_step": tflops, "flop_per_subdomain": flop_unit, "wall_s": wall,
           "plain": plain, "roofline": roofline, "kernel_ms_per_step": breakdown,
           "autotune": _tuned(tune_log) if pinned is None else pinned, "bab_loop": bab,
           "cpu_baseline": cpu}
    print(json.dumps(rec))


def bab_loop(iters, d=16, hidden=(256, 256, 256), n_pick=1024, samples=64):
    """Throughput of the planning loop (Algorithm 2) on a seeded scalar ReLU objective over
    [-1, 1]^d: each iteration picks n_pick subdomains, splits them, searches the 2 n_pick
    children (samples each) and bounds them with full CROWN, then prunes."""
    import torch

    import workloads as W
    from paper_2412_09584_amd.bab import BaBPlanner
    net, lo, hi = W.plan_objective(d=d, hidden=hidden)
    pl = BaBPlanner(net, lo, hi, n_pick=n_pick, samples=samples)
    uni = W.plan_uniforms()
    pl.run(2, uni)                                   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best, _, P, log = pl.run(iters, uni, trace=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bounded = sum(2 * len(e["picked"]) for e in log)          # children searched and bounded
    return {"objective": f"MLP {d}-{'-'.join(map(str, hidden))}-1 over [-1,1]^{d}",
            "n_pick": n_pick, "samples": samples, "iters": len(log),
            "ms_per_iter": 1e3 * dt / max(len(log), 1),
            "subdomains_bounded_per_s": bounded / dt if log else None,
            "best": best, "candidates": int(P["lo"].shape[0])}


def _tuned(log):
    """Chosen plan per product from the autotuner's log (fastest line per product)."""
    if not log:
        return None
    best = {}
    for line in log.strip().splitlines():
        key, path, cfg, cc, ms, _ = line.split()
        t = float(ms)
        if key not in best or t < best[key][0]:
            best[key] = (t, f"{path} {cfg} {cc}")
    return {k: f"{v[1]} {v[0]:.3f}ms" for k, v in best.items()}


def cpu_baseline(w, budget_s):
    """The FP64 oracle (as it stands) on a bounded sample of the same units: for each
    sampled subdomain of root 0, the bound, its alpha/beta gradient and one Adam step."""
    import numpy as np

    from oracle import crown as O
    import workloads as W
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
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
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "subdomains/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} subdomains of root 0 (bound + alpha/beta gradient + Adam step), "
                      f"{el:.1f} s", "host_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()
