"""The branch-and-bound batch of subdomains as one object: the state that the bench times
and the full-size GPU tests check, built in one place so that both see the same
configuration.

A batch is n_roots root inputs with their boxes, per_root subdomains per root, each
subdomain carrying random ReLU split constraints drawn from its root's unstable neurons,
the margin spec of its root, and alpha / beta with their Adam moments.  Root
pre-activation bounds come from full CROWN on the GPU (library calls).  One step is: the
bound pass with alpha, beta and the splits (SAVE_FOR_GRAD, best-so-far kept), the
gradient with respect to alpha and beta, and one projected Adam step on each.  Only
library calls and tensor allocation happen here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from . import net as N


class BetaBatch:
    def __init__(self, workload, per_root, *, split_seed, kmin=1, kmax=12, max_rows=None,
                 device="cuda"):
        import workloads as W
        self.w = workload
        net = workload.net
        dev = torch.device(device)
        self.n_roots = workload.x_lo.shape[0]
        self.per_root = int(per_root)
        self.n = n = self.n_roots * self.per_root
        self.R = R = workload.spec.shape[1]
        self.L = len(net)
        self.bn = N.BoundNet(net, max_inst=n, max_rows=max(n * R, max_rows or 0),
                             max_save_rows=n * R)
        self.lo, self.hi = self.bn.crown_bounds(workload.x_lo, workload.x_hi)
        lo_np, hi_np = self.lo.cpu().numpy(), self.hi.cpu().numpy()
        self.root_of = np.repeat(np.arange(self.n_roots), self.per_root).astype(np.int32)
        cands = [np.nonzero((lo_np[r] < 0) & (hi_np[r] > 0))[0] for r in range(self.n_roots)]
        self.splits = W.random_splits(cands, n, kmin, kmax, seed=split_seed, root_of=self.root_of)
        self.spd = N.splits_to_device(self.splits, device)
        ro = torch.as_tensor(self.root_of, device=dev, dtype=torch.long)
        self.C = torch.as_tensor(workload.spec, device=dev)[ro].contiguous()
        self.x_lo = torch.as_tensor(workload.x_lo, device=dev)[ro].contiguous()
        self.x_hi = torch.as_tensor(workload.x_hi, device=dev)[ro].contiguous()
        self.bof = torch.as_tensor(self.root_of, device=dev)
        self.nnz = self.splits.nnz
        n_relu = self.bn.n_relu
        self.alpha = torch.empty(n, n_relu, device=dev)
        self.beta = torch.empty(self.nnz, R, device=dev)
        self.ma, self.va = torch.empty_like(self.alpha), torch.empty_like(self.alpha)
        self.mb, self.vb = torch.empty_like(self.beta), torch.empty_like(self.beta)
        self.ga = torch.empty_like(self.alpha)
        self.gb = torch.empty_like(self.beta)
        self.lower = torch.empty(n, R, device=dev)
        self.best = torch.empty(n, R, device=dev)
        self.ones = torch.ones(n, R, device=dev)
        self.alpha0 = float(workload.extra.get("alpha0", 0.5))
        self.lr = float(workload.extra.get("lr", 0.1))
        self.recompute = False       # checkpointed layer recomputation for the gradient
        self.fused = True            # step(): alpha-gradient fused into its Adam step
        self.reset()

    def reset(self):
        """alpha = alpha0, beta = 0, Adam moments 0, best = -inf."""
        self.alpha.fill_(self.alpha0)
        self.beta.zero_()
        for t in (self.ma, self.va, self.mb, self.vb):
            t.zero_()
        self.best.fill_(-float("inf"))

    def pass_args(self):
        return dict(spec=self.C, lo=self.lo, hi=self.hi, n_bounds=self.n_roots, bound_of=self.bof,
                    alpha=self.alpha, split_off=self.spd["off"], split_idx=self.spd["idx"],
                    split_sign=self.spd["sign"], nnz=self.nnz, beta=self.beta, x_lo=self.x_lo,
                    x_hi=self.x_hi,
                    flags=B.BOUND_SAVE_FOR_GRAD | (B.BOUND_RECOMPUTE if self.recompute else 0))

    def bound_and_grad(self, stream=None):
        """The bound pass (SAVE_FOR_GRAD, best kept) and its alpha / beta gradient."""
        B.bound_backward(self.bn.handle, self.n, self.R, self.L, lower=self.lower, best=self.best,
                         stream=stream, **self.pass_args())
        B.bound_grad(self.bn.handle, self.ones, self.ga, self.gb, stream=stream)

    def adam(self, t, stream=None):
        B.bound_adam(self.alpha, self.ga, self.ma, self.va, t, self.lr, grad_scale=-1.0,
                     clip_lo=0.0, clip_hi=1.0, stream=stream)
        B.bound_adam(self.beta, self.gb, self.mb, self.vb, t, self.lr, grad_scale=-1.0,
                     clip_lo=0.0, stream=stream)

    def step(self, t, stream=None):
        """One optimisation step: bound pass, gradient, Adam on alpha and beta (with
        `fused`, the alpha-gradient goes straight into alpha's Adam step inside the
        library, the moments ma / va then in slot order)."""
        if not self.fused:
            self.bound_and_grad(stream)
            self.adam(t, stream)
            return
        B.bound_backward(self.bn.handle, self.n, self.R, self.L, lower=self.lower, best=self.best,
                         stream=stream, **self.pass_args())
        B.bound_grad_adam(self.bn.handle, self.ones, self.alpha, self.ma, self.va, t, self.lr,
                          grad_scale=-1.0, clip_lo=0.0, clip_hi=1.0, grad_beta=self.gb,
                          stream=stream)
        B.bound_adam(self.beta, self.gb, self.mb, self.vb, t, self.lr, grad_scale=-1.0,
                     clip_lo=0.0, stream=stream)

    def autotune(self, stream=None):
        """Time every kernel variant of every product of one step on the live data and keep
        the fastest per product; returns the timing log."""
        log = B.bound_autotune(self.bn.handle, self.n, self.R, self.L, grad_lower=self.ones,
                               lower=self.lower, stream=stream, **self.pass_args())
        self.best.fill_(-float("inf"))
        return log

    def set_plans(self, plans):
        """plans: {'R2': 'direct cfg=1 cc=16 ...', ...} as chosen_plans() returns them."""
        for key, plan in plans.items():
            path, cfg, cc = plan.split()[:3]
            B.bound_set_plan(self.bn.handle, key[0], int(key[1:]), 1 if path == "direct" else 2,
                             int(cfg.split("=")[1]), int(cc.split("=")[1]))

    def optimizer(self, steps=None):
        """The whole alpha/beta optimisation of the batch as a capturable unit."""
        steps = int(self.w.extra.get("steps", 10)) if steps is None else int(steps)
        return N.AlphaBetaOptimizer(self.bn, self.C, self.lo, self.hi, self.x_lo, self.x_hi,
                                    bound_of=self.bof, splits=self.spd, steps=steps, lr=self.lr,
                                    alpha0=self.alpha0, use_beta=True, fused=self.fused)


def chosen_plans(log):
    """The fastest plan per product from an autotuning log."""
    if not log:
        return None
    best = {}
    for line in log.strip().splitlines():
        key, path, cfg, cc, ms, _ = line.split()
        t = float(ms)
        if key not in best or t < best[key][0]:
            best[key] = (t, f"{path} {cfg} {cc}")
    return {k: f"{v[1]} {v[0]:.3f}ms" for k, v in best.items()}
