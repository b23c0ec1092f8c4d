"""Branch and bound over input boxes for planning (Algorithm 2's order: search, then
bound, on the new subdomains), driven from Python over library calls: the pick-out,
split, sampling, search summary, best update and pruner run in libbound.so's kernels
(`bound_bab_*`), the objective's forward passes in its product kernels
(`bound_sample_bounds`), and each subdomain's lower bound is a full CROWN pass
(`bound_backward`).  This module keeps the candidate set as device tensors and gathers
rows by the index lists the kernels return.

The objective is the scalar output of a ReLU network over an action box.  Random
numbers are supplied by the caller: ``uniforms(tag, shape)`` for the uniform search
('search0', ('search', t)), ``gumbels(tag, shape)`` (standard Gumbel variates) for the
pick-out (('pick', t)) and ``normals(tag, shape)`` for the CEM search (('cem0', r),
('cem', t, r)) -- the stream layout of the test oracle.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binding as B
from .net import BoundNet


class BaBPlanner:
    """bounding: "crown" -- each box's lower bound by full CROWN (sound); "early_stop" --
    the paper's bounding for planning (Section 3.2): pre-activation bounds are the min /
    max of the box's search samples (search-integrated), and the objective's backward
    pass stops at the ReLU of layer stop_layer, concretised over that node's empirical box
    (a tight estimate, not a sound bound).

    search: "uniform" -- M uniform samples per box; "cem" -- cem_rounds rounds of the
    cross-entropy method (M samples each, n_elite elites, deviation jitter), started at
    the parent's best sample for the child that holds it (Section 3.3); all rounds'
    samples are the box's search samples."""

    def __init__(self, layers, box_lo, box_hi, *, n_pick=64, samples=64, eta=0.75,
                 temperature=0.05, w=1.0, max_dom=1 << 16, bounding="crown", stop_layer=None,
                 search="uniform", cem_rounds=3, n_elite=4, jitter=1e-3, device="cuda"):
        self.device = torch.device(device)
        self.lo0 = torch.as_tensor(np.asarray(box_lo, np.float32), device=self.device)[None]
        self.hi0 = torch.as_tensor(np.asarray(box_hi, np.float32), device=self.device)[None]
        self.d = self.lo0.shape[1]
        self.n_pick, self.M = int(n_pick), int(samples)
        self.eta, self.T, self.w = float(eta), float(temperature), float(w)
        if search not in ("uniform", "cem"):
            raise ValueError("search must be 'uniform' or 'cem'")
        self.cem = search == "cem"
        self.R = int(cem_rounds) if self.cem else 1
        self.n_elite, self.jitter = int(n_elite), float(jitter)
        if self.cem and not (self.R >= 1 and 1 <= self.n_elite <= self.M):
            raise ValueError("need cem_rounds >= 1 and 1 <= n_elite <= samples")
        ms = self.R * self.M                  # search samples per box
        self.k = max(1, min(ms, int(math.ceil(self.w / 100.0 * ms))))
        self.max_dom = int(max_dom)
        widths = [int(np.prod(L["out_shape"])) for L in layers]
        rows = 2 * max(widths[:-1] + [1]) * 2 * self.n_pick
        self.net = BoundNet(layers, max_inst=max(2 * self.n_pick, 1),
                            max_rows=max(rows, 2 * self.n_pick * self.M))
        if self.net.d[-1] != 1:
            raise ValueError("the objective network must have a scalar output")
        self.bab = B.bound_bab_init(self.max_dom, self.d, ms)
        if bounding not in ("crown", "early_stop"):
            raise ValueError("bounding must be 'crown' or 'early_stop'")
        self.bounding = bounding
        self.stop = int(stop_layer) if stop_layer is not None else len(layers) - 1
        if bounding == "early_stop" and not 1 <= self.stop < len(layers):
            raise ValueError("stop_layer must be in 1 .. n_layers - 1")
        self._sb = None        # empirical pre-activation bounds of the last searched boxes

    def __del__(self):
        h = getattr(self, "bab", None)
        if h:
            B.bound_bab_destroy(h)
            self.bab = None

    # ------------------------------------------------------------------ steps
    def bound(self, lo, hi):
        """Lower bound (or, with early stop, its estimate) of the objective over each box
        [n]; the early-stop bound uses the empirical bounds of the last search() of
        these boxes."""
        n = lo.shape[0]
        C = torch.ones(n, 1, 1, device=self.device)
        if self.bounding == "early_stop":
            slo, shi = self._sb
            lower, _ = self.net.spec_bounds(C, slo, shi, lo, hi, both=False, stop_layer=self.stop,
                                            stop_mode=B.BOUND_STOP_RELU)
            return lower[:, 0].contiguous()
        blo, bhi = self.net.crown_bounds(lo, hi)
        lower, _ = self.net.spec_bounds(C, blo, bhi, lo, hi, both=False)
        return lower[:, 0].contiguous()

    def search(self, lo, hi, rand, u_par=None):
        """The boxes' search: (f_hi [n], top [n, k, d]).  Uniform: rand is the uniforms
        U [n, M, d].  CEM: rand(r) gives round r's normals [n, M, d]; u_par [n / 2, d] are
        the parents' best samples (children 2i, 2i + 1 of parent i) or None."""
        if self.cem:
            return self._cem_search(lo, hi, rand, u_par)
        U = rand
        n = lo.shape[0]
        S = torch.empty(n, self.M, self.d, device=self.device)
        B.bound_bab_samples(self.bab, n, self.M, lo, hi, U, S)
        vals = torch.empty(n * self.M, 1, device=self.device)
        if self.bounding == "early_stop":
            # the same forward pass gives the empirical pre-activation bounds
            slo = torch.empty(n, self.net.n_relu, device=self.device)
            shi = torch.empty_like(slo)
            B.bound_sample_bounds(self.net.handle, n, self.M, S.view(n * self.M, self.d), slo, shi,
                                  out=vals)
            self._sb = (slo, shi)
        else:
            B.bound_sample_bounds(self.net.handle, n, self.M, S.view(n * self.M, self.d), out=vals)
        f_hi = torch.empty(n, device=self.device)
        top = torch.empty(n, self.k, self.d, device=self.device)
        B.bound_bab_search_summary(self.bab, n, self.M, vals, S, self.k, f_hi, top)
        return f_hi, top

    def _cem_search(self, lo, hi, normals_of, u_par):
        n, M, R, d, dev = lo.shape[0], self.M, self.R, self.d, self.device
        mu = torch.empty(n, d, device=dev)
        sg = torch.empty(n, d, device=dev)
        B.bound_bab_cem_start(self.bab, n, lo, hi, u_par, 2, mu, sg)
        S = torch.empty(n, M, d, device=dev)
        vals = torch.empty(n * M, 1, device=dev)
        S_all = torch.empty(n, R * M, d, device=dev)
        V_all = torch.empty(n, R * M, device=dev)
        es = self.bounding == "early_stop"
        if es:
            slo = torch.empty(n, self.net.n_relu, device=dev)
            shi = torch.empty_like(slo)
        for r in range(R):
            B.bound_bab_cem_samples(self.bab, n, M, lo, hi, mu, sg, normals_of(r), S, S_all, R * M, r * M)
            x = S.view(n * M, d)
            if es:
                (B.bound_sample_bounds if r == 0 else B.bound_sample_bounds_merge)(
                    self.net.handle, n, M, x, slo, shi, out=vals)
            else:
                B.bound_sample_bounds(self.net.handle, n, M, x, out=vals)
            B.bound_bab_cem_refit(self.bab, n, M, vals, S, self.n_elite, self.jitter, mu, sg,
                                  V_all, R * M, r * M)
        if es:
            self._sb = (slo, shi)
        f_hi = torch.empty(n, device=dev)
        top = torch.empty(n, self.k, d, device=dev)
        B.bound_bab_search_summary(self.bab, n, R * M, V_all, S_all, self.k, f_hi, top)
        return f_hi, top

    def _rand(self, uniforms, normals, tag, n):
        """The search's random numbers for n boxes under tag 'search0' or ('search', t)."""
        if not self.cem:
            return self._u(uniforms, tag, (n, self.M, self.d))
        if normals is None:
            raise ValueError("the CEM search needs normals(tag, shape)")
        zt = (lambda r: ("cem0", r)) if tag == "search0" else (lambda r: ("cem", tag[1], r))
        return lambda r: self._u(normals, zt(r), (n, self.M, self.d))

    def _u(self, draw, tag, shape):
        """draw(tag, shape): host arrays or device tensors of the random numbers."""
        x = draw(tag, shape)
        if isinstance(x, torch.Tensor):
            return x.to(device=self.device, dtype=torch.float32).contiguous()
        return torch.as_tensor(np.asarray(x, np.float32), device=self.device)

    # ------------------------------------------------------------------ the loop
    def run(self, iters, uniforms, trace=False, normals=None, gumbels=None):
        """Returns (best value, its sample [d], candidate set dict, per-iteration trace)."""
        dev = self.device
        f_hi, top = self.search(self.lo0, self.hi0, self._rand(uniforms, normals, "search0", 1))
        f_lo = self.bound(self.lo0, self.hi0)
        best = f_hi[:1].clone()
        ubest = top[0, 0].clone()
        P = dict(lo=self.lo0, hi=self.hi0, f_lo=f_lo, f_hi=f_hi, top=top)
        log = []
        n_keep = torch.zeros(1, dtype=torch.int32, device=dev)
        for t in range(iters):
            N = P["lo"].shape[0]
            if N == 0:
                break
            if N > self.max_dom:
                raise RuntimeError(f"candidate set ({N}) exceeds max_dom ({self.max_dom})")
            n = min(self.n_pick, N)
            picked = torch.empty(n, dtype=torch.int32, device=dev)
            rest = torch.empty(max(N - n, 1), dtype=torch.int32, device=dev)
            if gumbels is None:
                raise ValueError("the pick-out needs gumbels(tag, shape)")
            B.bound_bab_pick_out(self.bab, N, P["f_lo"], P["f_hi"], self._u(gumbels, ("pick", t), (N,)),
                                 self.n_pick, self.eta, self.T, picked, rest)
            rest = rest[: N - n]
            pl = P["lo"].index_select(0, picked).contiguous()
            ph = P["hi"].index_select(0, picked).contiguous()
            pt = P["top"].index_select(0, picked).contiguous()
            clo = torch.empty(2 * n, self.d, device=dev)
            chi = torch.empty(2 * n, self.d, device=dev)
            dims = torch.empty(n, dtype=torch.int32, device=dev)
            B.bound_bab_split(self.bab, n, pl, ph, pt, self.k, clo, chi, dims)
            c_fhi, c_top = self.search(clo, chi, self._rand(uniforms, normals, ("search", t), 2 * n),
                                       pt[:, 0].contiguous())
            c_flo = self.bound(clo, chi)
            B.bound_bab_update_best(self.bab, 2 * n, c_fhi, c_top, self.k, best, ubest)
            keep = torch.empty(2 * n, dtype=torch.int32, device=dev)
            B.bound_bab_prune(self.bab, 2 * n, c_flo, best, keep, n_keep)
            nk = int(n_keep.item())
            keep = keep[:nk]
            P = dict(lo=torch.cat([P["lo"].index_select(0, rest), clo.index_select(0, keep)]),
                     hi=torch.cat([P["hi"].index_select(0, rest), chi.index_select(0, keep)]),
                     f_lo=torch.cat([P["f_lo"].index_select(0, rest), c_flo.index_select(0, keep)]),
                     f_hi=torch.cat([P["f_hi"].index_select(0, rest), c_fhi.index_select(0, keep)]),
                     top=torch.cat([P["top"].index_select(0, rest), c_top.index_select(0, keep)]))
            if trace:
                log.append(dict(picked=picked.cpu().numpy(), dims=dims.cpu().numpy(),
                                kept=keep.cpu().numpy(), best=float(best.item()),
                                size=P["lo"].shape[0]))
        return float(best.item()), ubest, P, log
