"""Convenience layer over the C ABI: a network handle, full-CROWN intermediate bounds,
spec bounds, the alpha/beta gradient as a torch.autograd.Function, and the projected
Adam loop.  It only allocates output tensors and sequences library calls; every step of
the bound computation runs in libbound.so's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def _dev(x, device, dtype=torch.float32):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device)


class BoundNet:
    """A ReLU network (list of layer dicts as produced by ``workloads``) on the GPU."""

    def __init__(self, layers, max_inst, max_rows, max_save_rows=0, device="cuda"):
        self.device = torch.device(device)
        self.layers = []
        prev = None
        for L in layers:
            d = dict(L)
            d["W"] = _dev(L["W"], self.device)
            d["b"] = _dev(L["b"], self.device)
            if L["kind"] == "linear" and prev is not None and prev["kind"] == "conv":
                d["in_view"] = tuple(prev["out_shape"])
            self.layers.append(d)
            prev = L
        self.max_inst, self.max_rows, self.max_save_rows = max_inst, max_rows, max_save_rows
        self.handle = B.bound_init(self.layers, max_inst, max_rows, max_save_rows)
        self.d, self.n_relu = B.bound_dims(self.handle)
        self.L = len(self.layers)
        self.relu_off = [0]
        for w in self.d[1:-1]:
            self.relu_off.append(self.relu_off[-1] + w)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            B.bound_destroy(h)
            self.handle = None

    # ------------------------------------------------------------------ passes
    def crown_bounds(self, x_lo, x_hi, slack=True):
        """Full CROWN pre-activation bounds of z_1 .. z_{L-1}: (lo, hi) [n, n_relu]."""
        x_lo = _dev(x_lo, self.device)
        x_hi = _dev(x_hi, self.device)
        n = x_lo.shape[0]
        lo = torch.zeros(n, max(self.n_relu, 1), device=self.device)
        hi = torch.zeros_like(lo)
        flags = B.BOUND_BOTH_SIDES | (0 if slack else B.BOUND_NO_SLACK)
        for k in range(1, self.L):
            off = self.relu_off[k - 1]
            B.bound_backward(self.handle, n, self.d[k], k, lo=lo, hi=hi, n_bounds=n, x_lo=x_lo,
                             x_hi=x_hi, flags=flags, lower=lo[:, off:], upper=hi[:, off:],
                             ld=self.n_relu)
        return lo, hi

    def alpha_crown_bounds(self, x_lo, x_hi, steps=5, lr=0.1, alpha0=0.5, slack=True):
        """Pre-activation bounds of z_1 .. z_{L-1} with every intermediate pass's slopes
        optimised: bottom-up, for z_k the default-rule pass (rows [I; -I]), then `steps`
        projected Adam steps on the slopes of layers < k (one per neuron and instance,
        shared by the layer's lower- and upper-bound rows, starting at alpha0) maximising
        the rows' summed lower bounds, then one more pass; the library keeps the best
        lower / upper bound of every neuron over these passes (best / best_upper).
        Needs max_save_rows >= n * 2 * max width.  Returns (lo, hi) [n, n_relu]."""
        x_lo = _dev(x_lo, self.device)
        x_hi = _dev(x_hi, self.device)
        n = x_lo.shape[0]
        nr = max(self.n_relu, 1)
        lo = torch.zeros(n, nr, device=self.device)
        hi = torch.zeros_like(lo)
        tlo, thi = torch.empty_like(lo), torch.empty_like(lo)
        flags = B.BOUND_BOTH_SIDES | (0 if slack else B.BOUND_NO_SLACK)
        alpha = torch.empty(n, nr, device=self.device)
        ma, va, ga = torch.empty_like(alpha), torch.empty_like(alpha), torch.empty_like(alpha)
        for k in range(1, self.L):
            off, d = self.relu_off[k - 1], self.d[k]
            # the default slope rule on the bounds found so far: the starting best bounds
            B.bound_backward(self.handle, n, d, k, lo=lo, hi=hi, n_bounds=n, x_lo=x_lo, x_hi=x_hi,
                             flags=flags, lower=lo[:, off:], upper=hi[:, off:], ld=self.n_relu)
            if k == 1 or steps <= 0:
                continue
            spec = torch.eye(d, device=self.device).expand(n, d, d).contiguous()
            ones = torch.ones(n, 2 * d, device=self.device)
            alpha.fill_(float(alpha0))
            ma.zero_()
            va.zero_()
            kw = dict(spec=spec, lo=lo, hi=hi, n_bounds=n, alpha=alpha, x_lo=x_lo, x_hi=x_hi,
                      lower=tlo[:, off:], upper=thi[:, off:], ld=self.n_relu,
                      best=lo[:, off:], best_upper=hi[:, off:])
            for t in range(1, steps + 1):
                B.bound_backward(self.handle, n, d, k, flags=flags | B.BOUND_SAVE_FOR_GRAD, **kw)
                B.bound_grad(self.handle, ones, ga)
                B.bound_adam(alpha, ga, ma, va, t, lr, grad_scale=-1.0, clip_lo=0.0, clip_hi=1.0)
            B.bound_backward(self.handle, n, d, k, flags=flags, **kw)
        return lo, hi

    def spec_bounds(self, C, lo, hi, x_lo, x_hi, *, target=None, alpha=None, bound_of=None,
                    splits=None, beta=None, both=True, slack=True, save=False, best=None,
                    stop_layer=0, stop_mode=0):
        """Bounds of C z_target.  Returns (lower, upper or None)."""
        target = self.L if target is None else target
        C = _dev(C, self.device)
        n, rows = C.shape[0], C.shape[1]
        lower = torch.empty(n, rows, device=self.device)
        upper = torch.empty(n, rows, device=self.device) if both else None
        flags = (B.BOUND_BOTH_SIDES if both else 0) | (0 if slack else B.BOUND_NO_SLACK) | \
            (B.BOUND_SAVE_FOR_GRAD if save else 0)
        kw = {}
        if splits is not None:
            kw = dict(split_off=splits["off"], split_idx=splits["idx"], split_sign=splits["sign"],
                      nnz=int(splits["idx"].numel()))
        n_bounds = lo.shape[0] if lo is not None else 0
        self.last_pass_id = B.bound_backward(
            self.handle, n, rows, target, spec=C, lo=lo, hi=hi, n_bounds=n_bounds,
            bound_of=bound_of, alpha=alpha, beta=beta, x_lo=_dev(x_lo, self.device),
            x_hi=_dev(x_hi, self.device), flags=flags, lower=lower, upper=upper, best=best,
            stop_layer=stop_layer, stop_mode=stop_mode, **kw)
        return lower, upper

    def coefficients(self, C, lo, hi, *, target=None, alpha=None, both=False):
        """Coefficient form (W~(1), b~(1), sum |terms| of b~(1)) without concretisation."""
        target = self.L if target is None else target
        C = _dev(C, self.device)
        n, rows = C.shape[0], C.shape[1]
        tot = n * rows * (2 if both else 1)
        coeff = torch.empty(tot, self.d[0], device=self.device)
        offset = torch.empty(tot, device=self.device)
        mag = torch.empty(tot, device=self.device)
        B.bound_backward(self.handle, n, rows, target, spec=C, lo=lo, hi=hi,
                         n_bounds=lo.shape[0] if lo is not None else 0, alpha=alpha,
                         flags=B.BOUND_BOTH_SIDES if both else 0, coeff=coeff, offset=offset,
                         offset_mag=mag)
        return coeff, offset, mag

    def grad(self, grad_lower, nnz=0, pass_id=0):
        """d(sum grad_lower * lower_raw)/d(alpha, beta) of the last saved pass (or of the
        pass with this id: the library refuses if another pass has run since)."""
        n = grad_lower.shape[0]
        ga = torch.empty(n, self.n_relu, device=self.device)
        gb = torch.empty(nnz, grad_lower.shape[1], device=self.device) if nnz else None
        B.bound_grad(self.handle, grad_lower.contiguous(), ga, gb, pass_id=pass_id)
        return ga, gb


def splits_to_device(sp, device="cuda"):
    """workloads.Splits -> dict of device tensors for the C ABI."""
    return {"off": torch.as_tensor(sp.off, dtype=torch.int32, device=device),
            "idx": torch.as_tensor(sp.neuron, dtype=torch.int32, device=device),
            "sign": torch.as_tensor(sp.sign, dtype=torch.int8, device=device)}


class CrownBound(torch.autograd.Function):
    """lower = CROWN bound of C z_L as a function of (alpha, beta); backward = bound_grad.

    The library keeps the state of one SAVE_FOR_GRAD pass per handle; backward names the
    pass its forward made (by id), so a forward of another batch in between makes the
    backward raise instead of returning that batch's gradient."""

    @staticmethod
    def forward(ctx, alpha, beta, net, C, lo, hi, x_lo, x_hi, bound_of, splits, best):
        lower, _ = net.spec_bounds(C, lo, hi, x_lo, x_hi, alpha=alpha.detach(),
                                   beta=None if beta is None else beta.detach(),
                                   bound_of=bound_of, splits=splits, both=False, save=True,
                                   best=best)
        ctx.net = net
        ctx.pass_id = net.last_pass_id
        ctx.nnz = 0 if splits is None else int(splits["idx"].numel())
        ctx.has_beta = beta is not None
        return lower

    @staticmethod
    def backward(ctx, grad_lower):
        ga, gb = ctx.net.grad(grad_lower, ctx.nnz if ctx.has_beta else 0, pass_id=ctx.pass_id)
        return (ga, gb if ctx.has_beta else None) + (None,) * 9


def optimize_alpha_beta(net, C, lo, hi, x_lo, x_hi, *, steps=10, lr=0.1, alpha0=0.5,
                        bound_of=None, splits=None, use_beta=True, lower_of_step=None):
    """Projected Adam on (alpha, beta) maximising sum of lower bounds; returns best lower.

    Each step: bound pass with SAVE_FOR_GRAD (best-so-far fused), bound_grad with
    grad_lower = 1, then one Adam step each for alpha (clip [0, 1]) and beta (clip >= 0).
    """
    dev = net.device
    C = _dev(C, dev)
    n, rows = C.shape[0], C.shape[1]
    nnz = 0 if splits is None else int(splits["idx"].numel())
    alpha = torch.full((n, net.n_relu), float(alpha0), device=dev)
    ma, va = torch.zeros_like(alpha), torch.zeros_like(alpha)
    beta = torch.zeros(nnz, rows, device=dev) if (use_beta and nnz) else None
    if beta is not None:
        mb, vb = torch.zeros_like(beta), torch.zeros_like(beta)
    best = torch.full((n, rows), -float("inf"), device=dev)
    ones = torch.ones(n, rows, device=dev)
    ga = torch.empty(n, net.n_relu, device=dev)
    gb = torch.empty(nnz, rows, device=dev) if beta is not None else None
    for t in range(1, steps + 1):
        lower, _ = net.spec_bounds(C, lo, hi, x_lo, x_hi, alpha=alpha, beta=beta, bound_of=bound_of,
                                   splits=splits, both=False, save=True, best=best)
        if lower_of_step is not None:
            lower_of_step.append(lower.clone())
        B.bound_grad(net.handle, ones, ga, gb)
        B.bound_adam(alpha, ga, ma, va, t, lr, grad_scale=-1.0, clip_lo=0.0, clip_hi=1.0)
        if beta is not None:
            B.bound_adam(beta, gb, mb, vb, t, lr, grad_scale=-1.0, clip_lo=0.0)
    net.spec_bounds(C, lo, hi, x_lo, x_hi, alpha=alpha, beta=beta, bound_of=bound_of,
                    splits=splits, both=False, best=best)
    return best, alpha, beta


class AlphaBetaOptimizer:
    """The alpha/beta optimisation of one batch of subdomains as a replayable unit.

    run() issues, on the current stream: reset of alpha / beta / Adam state / best bound,
    then `steps` x (bound pass with SAVE_FOR_GRAD and best-so-far, gradient, Adam on
    alpha and on beta), then a last bound pass.  capture() records exactly that sequence
    into a HIP graph (through torch.cuda.CUDAGraph on a capture stream) after one eager
    warm-up run, so a whole optimisation is one graph launch; replay() launches it.
    The library allocates nothing inside a pass, and clears memory with kernels only, so
    the captured sequence is the eager one.  With `fused` (the default) the alpha-gradient
    goes straight into alpha's Adam step (bound_grad_adam; ma / va in slot order),
    otherwise through a dense gradient and bound_adam; alpha comes out the same.
    """

    def __init__(self, net, C, lo, hi, x_lo, x_hi, *, bound_of=None, splits=None, steps=10,
                 lr=0.1, alpha0=0.5, use_beta=True, fused=True):
        dev = net.device
        self.net, self.steps, self.lr, self.alpha0 = net, int(steps), float(lr), float(alpha0)
        self.C = _dev(C, dev)
        self.n, self.rows = self.C.shape[0], self.C.shape[1]
        self.lo, self.hi = lo, hi
        self.x_lo, self.x_hi = _dev(x_lo, dev), _dev(x_hi, dev)
        self.bound_of, self.splits = bound_of, splits
        self.nnz = 0 if splits is None else int(splits["idx"].numel())
        self.alpha = torch.empty(self.n, net.n_relu, device=dev)
        self.ma, self.va = torch.empty_like(self.alpha), torch.empty_like(self.alpha)
        self.fused = bool(fused)
        self.ga = None if self.fused else torch.empty_like(self.alpha)
        self.use_beta = bool(use_beta and self.nnz)
        if self.use_beta:
            self.beta = torch.empty(self.nnz, self.rows, device=dev)
            self.mb, self.vb = torch.empty_like(self.beta), torch.empty_like(self.beta)
            self.gb = torch.empty_like(self.beta)
        else:
            self.beta = self.gb = None
        self.best = torch.empty(self.n, self.rows, device=dev)
        self.lower = torch.empty(self.n, self.rows, device=dev)
        self.ones = torch.ones(self.n, self.rows, device=dev)
        self.graph = None

    def _pass(self, save):
        kw = {}
        if self.splits is not None:
            kw = dict(split_off=self.splits["off"], split_idx=self.splits["idx"],
                      split_sign=self.splits["sign"], nnz=self.nnz)
        B.bound_backward(self.net.handle, self.n, self.rows, self.net.L, spec=self.C, lo=self.lo,
                         hi=self.hi, n_bounds=self.lo.shape[0], bound_of=self.bound_of,
                         alpha=self.alpha, beta=self.beta, x_lo=self.x_lo, x_hi=self.x_hi,
                         flags=B.BOUND_SAVE_FOR_GRAD if save else 0, lower=self.lower,
                         best=self.best, **kw)

    def run(self):
        self.alpha.fill_(self.alpha0)
        self.ma.zero_()
        self.va.zero_()
        if self.use_beta:
            self.beta.zero_()
            self.mb.zero_()
            self.vb.zero_()
        self.best.fill_(-float("inf"))
        for t in range(1, self.steps + 1):
            self._pass(True)
            if self.fused:
                B.bound_grad_adam(self.net.handle, self.ones, self.alpha, self.ma, self.va, t,
                                  self.lr, grad_scale=-1.0, clip_lo=0.0, clip_hi=1.0,
                                  grad_beta=self.gb)
            else:
                B.bound_grad(self.net.handle, self.ones, self.ga, self.gb)
                B.bound_adam(self.alpha, self.ga, self.ma, self.va, t, self.lr, grad_scale=-1.0,
                             clip_lo=0.0, clip_hi=1.0)
            if self.use_beta:
                B.bound_adam(self.beta, self.gb, self.mb, self.vb, t, self.lr, grad_scale=-1.0,
                             clip_lo=0.0)
        self._pass(False)
        return self.best

    def capture(self):
        self.run()                       # warm-up: sizes scratch, sets kernel attributes
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.best
