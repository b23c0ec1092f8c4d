"""The configuration the bench times, at full size, against the oracle.

64 root inputs of the 3x32x32 CNN x 64 subdomains = 4096 subdomains with 1-12 random
splits each and 9 margin rows, the kernel plans chosen by the autotuner on this batch (as
the bench chooses them), one launch for all subdomains:

  * optimisation steps 1 and 2 (alpha = 0.5 and beta = 0, then after one Adam step) on a
    stratified sample of 16 subdomains from 8 roots -- per root the subdomain with the
    fewest and the one with the most split entries -- against the oracle at identical
    alpha / beta, stage-wise (the oracle takes the GPU's root bounds promoted to FP64):
    bounds at 1e-4 relative, gradients at 1e-4 of the infinity norm per subdomain;
  * the whole 10-step optimisation captured as one HIP graph and replayed three times,
    with eager work and synchronisations between the replays, against the eager run.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import crown as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_09584_amd.batch import BetaBatch
    w = W.beta_cnn(64, 64)
    bb = BetaBatch(w, 64, split_seed=W.SPLIT_SEED, max_rows=36864)
    bb.autotune()
    return bb


def _np(t):
    return t.detach().double().cpu().numpy()


def _sample(bb):
    counts = np.diff(bb.splits.off)
    out = []
    for r in range(0, bb.n_roots, bb.n_roots // 8):
        ids = np.arange(r * bb.per_root, (r + 1) * bb.per_root)
        out += [int(ids[np.argmin(counts[ids])]), int(ids[np.argmax(counts[ids])])]
    return out


def _check_step(bb, what):
    w = bb.w
    net = w.net
    L = len(net)
    lo, hi = _np(bb.lo), _np(bb.hi)
    lower, ga, gb = _np(bb.lower), _np(bb.ga), _np(bb.gb)
    alpha, beta = _np(bb.alpha), _np(bb.beta)
    sp = bb.splits
    for i in _sample(bb):
        r = int(bb.root_of[i])
        q0, q1 = sp.off[i], sp.off[i + 1]
        bounds = list(zip(O.per_layer(net, lo[r]), O.per_layer(net, hi[r])))
        splits = O.split_list(net, sp.neuron[q0:q1], sp.sign[q0:q1])
        al = O.per_layer(net, alpha[i])
        be = beta[q0:q1]
        low = O.spec_lower(net, L, w.spec[r], bounds, w.x_lo[r], w.x_hi[r], al, splits, be)
        _, oga, ogb = O.spec_lower_grad(net, L, w.spec[r], bounds, w.x_lo[r], w.x_hi[r], al,
                                        splits, be)
        err = np.abs(lower[i] - low)
        assert np.all(err <= 1e-4 * np.maximum(np.abs(low), 1.0)), f"{what}: lower of {i}"
        oga = np.concatenate(oga)
        sa = max(float(np.max(np.abs(oga))), 1e-30)
        assert np.max(np.abs(ga[i] - oga)) <= 1e-4 * sa, f"{what}: alpha gradient of {i}"
        sb = max(float(np.max(np.abs(ogb))), sa)
        assert np.max(np.abs(gb[q0:q1] - ogb)) <= 1e-4 * sb, f"{what}: beta gradient of {i}"


def test_bench_batch_steps_match_oracle(batch):
    bb = batch
    bb.reset()
    bb.bound_and_grad()
    torch.cuda.synchronize()
    _check_step(bb, "step 1")
    bb.adam(1)
    bb.bound_and_grad()
    torch.cuda.synchronize()
    assert float(bb.beta.max()) > 0 and float(bb.alpha.min()) < 0.5 < float(bb.alpha.max())
    _check_step(bb, "step 2")


def test_bench_batch_graph_replay_matches_eager(batch):
    bb = batch
    opt = bb.optimizer()
    best_e = opt.run().clone()
    alpha_e, beta_e = opt.alpha.clone(), opt.beta.clone()
    torch.cuda.synchronize()
    opt.capture()
    x = torch.randn(512, 512, device="cuda")
    for rep in range(3):
        y = (x @ x).sum()                       # eager work between the replays
        torch.cuda.synchronize()
        best_g = opt.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        # alpha and beta follow the gradients, which no atomic touches: exact
        assert torch.equal(opt.alpha, alpha_e), f"replay {rep}: alpha"
        assert torch.equal(opt.beta, beta_e), f"replay {rep}: beta"
        # the bound's row sums use float atomics: equal up to the order of the additions
        d = (best_g - best_e).abs()
        assert float((d / best_e.abs().clamp_min(1.0)).max()) <= 1e-5, f"replay {rep}: best"
    # the optimisation never loosens the bound of step 1 (best is a running maximum)
    bb.reset()
    bb.bound_and_grad()
    assert bool((best_e >= bb.lower - 1e-5 * bb.lower.abs().clamp_min(1.0)).all())
