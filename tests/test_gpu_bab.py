"""GPU parity of the branch-and-bound steps (libbound.so, through the C ABI) against the
oracle (oracle/bab.py) -- pick-out, uniform and CEM search, summary, split, best, pruner
-- and the planning loop on the GPU against brute force and the oracle's loop."""
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import bab as OB  # noqa: E402
from oracle import crown as O  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_09584_amd import binding
    return binding


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("N,n,eta,T", [(1, 4, 0.75, 0.05), (37, 10, 0.75, 0.05), (300, 64, 0.5, 0.05),
                                       (5000, 1024, 0.75, 0.05), (200, 200, 0.0, 1.0),
                                       (2000, 100, 1.0, 0.05)])
def test_pick_out_matches_oracle(B, N, n, eta, T):
    """Picked and rest index lists identical to the oracle's: both sides form the draw's
    keys from the same Gumbel variates with the same FP32 operations."""
    rng = np.random.default_rng(N + n)
    f_lo = rng.normal(size=N).astype(np.float32)
    f_hi = rng.normal(size=N).astype(np.float32)
    if N > 10:
        f_hi[5] = f_hi[2]                      # a tie in the upper bounds
        f_lo[7] = np.inf                       # an infeasible subdomain
        f_lo[9] = f_lo[8]                      # equal lower bounds ...
    g = (-np.log(-np.log(rng.random(N)))).astype(np.float32)
    if N > 10:
        g[9] = g[8]                            # ... and equal variates: a key tie
    bab = B.bound_bab_init(max(N, 1), 2, 8)
    m = min(n, N)
    picked = torch.empty(m, dtype=torch.int32, device="cuda")
    rest = torch.empty(max(N - m, 1), dtype=torch.int32, device="cuda")
    B.bound_bab_pick_out(bab, N, dev(f_lo), dev(f_hi), dev(g), n, eta, T, picked, rest)
    torch.cuda.synchronize()
    gp, gr = picked.cpu().numpy(), rest.cpu().numpy()[: N - m]
    op, orr = OB.pick_out(f_lo, f_hi, g, n, eta, T)
    assert list(gp) == list(op)
    assert list(gr) == list(orr)
    B.bound_bab_destroy(bab)


def test_samples_summary_split_best_prune_match_oracle(B):
    rng = np.random.default_rng(7)
    n, M, d, w = 300, 100, 6, 5.0
    k = OB.n_top(w, M)
    lo = rng.uniform(-2, 0, size=(n, d)).astype(np.float32)
    hi = (lo + rng.uniform(0.01, 2, size=(n, d))).astype(np.float32)
    U = rng.random((n, M, d)).astype(np.float32)
    bab = B.bound_bab_init(4 * n, d, M)
    S = torch.empty(n, M, d, device="cuda")
    B.bound_bab_samples(bab, n, M, dev(lo), dev(hi), dev(U), S)
    S_ref = lo[:, None, :] + (hi - lo)[:, None, :] * U          # float32 numpy, each op rounded
    assert np.array_equal(S.cpu().numpy(), S_ref)
    vals = rng.normal(size=(n, M)).astype(np.float32)
    vals[:, 3] = vals[:, 1]                                      # ties between samples
    f_hi = torch.empty(n, device="cuda")
    top = torch.empty(n, k, d, device="cuda")
    B.bound_bab_search_summary(bab, n, M, dev(vals), S, k, f_hi, top)
    of, ot = OB.search_summary(vals, S_ref, k)
    assert np.array_equal(f_hi.cpu().numpy(), of.astype(np.float32))
    assert np.array_equal(top.cpu().numpy(), ot)
    clo = torch.empty(2 * n, d, device="cuda")
    chi = torch.empty(2 * n, d, device="cuda")
    dims = torch.empty(n, dtype=torch.int32, device="cuda")
    B.bound_bab_split(bab, n, dev(lo), dev(hi), top, k, clo, chi, dims)
    rlo, rhi, rd = OB.split(lo, hi, ot)
    assert np.array_equal(dims.cpu().numpy(), rd)
    assert np.array_equal(clo.cpu().numpy(), rlo) and np.array_equal(chi.cpu().numpy(), rhi)
    best = dev(np.array([0.0], np.float32))
    ub = torch.zeros(d, device="cuda")
    B.bound_bab_update_best(bab, n, f_hi, top, k, best, ub)
    j = int(np.argmin(of))
    assert best.item() == np.float32(min(0.0, of[j]))
    assert np.array_equal(ub.cpu().numpy(), ot[j, 0] if of[j] < 0 else np.zeros(d, np.float32))
    f_lo = rng.normal(size=2 * n).astype(np.float32)
    keep = torch.empty(2 * n, dtype=torch.int32, device="cuda")
    nk = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.bound_bab_prune(bab, 2 * n, dev(f_lo), best, keep, nk)
    ref = OB.prune(f_lo, float(best.item()))
    assert int(nk.item()) == len(ref) and np.array_equal(keep.cpu().numpy()[: len(ref)], ref)
    B.bound_bab_destroy(bab)


def test_bad_arguments(B):
    bab = B.bound_bab_init(16, 2, 8)
    t = torch.zeros(16, device="cuda")
    i = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(B.BoundError):
        B.bound_bab_pick_out(bab, 16, t, t, t, 4, 0.75, 0.0, i, i)     # temperature 0
    with pytest.raises(B.BoundError):
        B.bound_bab_pick_out(bab, 17, t, t, t, 4, 0.75, 0.05, i, i)    # beyond max_dom
    with pytest.raises(B.BoundError):
        B.bound_bab_search_summary(bab, 1, 9, t, t, 1, t, t)            # M > max_samples
    B.bound_bab_destroy(bab)


def test_planning_loop_on_gpu_reaches_the_brute_force_minimum(B):
    from paper_2412_09584_amd.bab import BaBPlanner
    net, lo, hi = W.plan_objective(d=2, hidden=(16, 16))
    g = np.linspace(-1.0, 1.0, 401)
    G = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    true_min = O.forward(net, G)[-1][:, 0].min()
    pl = BaBPlanner(net, lo, hi, n_pick=8, samples=64, eta=0.75, temperature=0.05, w=5.0)
    best, ub, P, log = pl.run(12, W.plan_uniforms(), trace=True, gumbels=W.plan_gumbels())
    fu = O.forward(net, ub.cpu().numpy()[None].astype(np.float64))[-1][0, 0]
    assert abs(fu - best) <= 1e-5 * max(1.0, abs(best))          # the best value is attained
    assert best <= true_min + 2e-3 * max(1.0, abs(true_min))
    assert float(P["f_lo"].min()) <= true_min + 1e-5               # sound pruning
    # against the oracle's loop on the same random numbers
    ob, _, _, _ = OB.bab_plan(lambda U: O.forward(net, U)[-1][:, 0],
                              lambda a, b: np.array([O.crown(net, np.ones((1, 1)), a[i].astype(np.float64),
                                                             b[i].astype(np.float64))[1][0]
                                                     for i in range(a.shape[0])]),
                              lo, hi, 8, 64, 12, 0.75, 0.05, 5.0, W.plan_uniforms(), W.plan_gumbels())
    assert abs(best - ob) <= 2e-3 * max(1.0, abs(ob))


def test_planning_loop_larger_objective(B):
    from paper_2412_09584_amd.bab import BaBPlanner
    net, lo, hi = W.plan_objective(d=8, hidden=(64, 64))
    pl = BaBPlanner(net, lo, hi, n_pick=64, samples=64)
    best0, _, P0, _ = pl.run(0, W.plan_uniforms(), gumbels=W.plan_gumbels())
    best, ub, P, log = pl.run(8, W.plan_uniforms(), trace=True, gumbels=W.plan_gumbels())
    assert best <= best0
    assert all(a["best"] >= b["best"] for a, b in zip(log, log[1:]))  # monotone
    # every kept box's lower bound is below the value of a random point inside it
    rng = np.random.default_rng(0)
    lo_b, hi_b = P["lo"].cpu().numpy(), P["hi"].cpu().numpy()
    x = lo_b + (hi_b - lo_b) * rng.random(lo_b.shape)
    fx = O.forward(net, x.astype(np.float64))[-1][:, 0]
    assert np.all(P["f_lo"].cpu().numpy() <= fx + 1e-4)


def test_planning_loop_with_early_stop_bounding(B):
    """The loop with the paper's bounding (each box's pre-activation bounds from its own
    search samples, the objective's pass stopped at the last ReLU layer) on the GPU
    against the oracle's loop with the same bounding on the same random numbers."""
    from paper_2412_09584_amd.bab import BaBPlanner
    net, lo, hi = W.plan_objective(d=2, hidden=(16, 16))
    g = np.linspace(-1.0, 1.0, 401)
    G = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    true_min = O.forward(net, G)[-1][:, 0].min()
    pl = BaBPlanner(net, lo, hi, n_pick=8, samples=64, eta=0.75, temperature=0.05, w=5.0,
                    bounding="early_stop", stop_layer=2)
    best, ub, P, log = pl.run(12, W.plan_uniforms(), trace=True, gumbels=W.plan_gumbels())
    assert best <= true_min + 2e-3 * max(1.0, abs(true_min))
    f_lo, f_hi = P["f_lo"].cpu().numpy(), P["f_hi"].cpu().numpy()
    assert np.all(f_lo <= f_hi + 1e-4 * np.maximum(1.0, np.abs(f_hi)))

    def bound(a, b, S):
        out = []
        for i in range(a.shape[0]):
            sb = O.sample_bounds(net, S[i].astype(np.float64))
            out.append(O.spec_lower_early_stop(net, len(net), np.ones((1, 1)), sb, 2, "relu")[0])
        return np.array(out)

    ob, _, _, _ = OB.bab_plan(lambda U: O.forward(net, U)[-1][:, 0], bound, lo, hi, 8, 64, 12,
                              0.75, 0.05, 5.0, W.plan_uniforms(), W.plan_gumbels(),
                              bound_uses_samples=True)
    assert abs(best - ob) <= 2e-3 * max(1.0, abs(ob))


@pytest.mark.parametrize("n,M,d,R", [(64, 48, 5, 3), (512, 640, 16, 3), (6, 2048, 2, 1)])
def test_cem_steps_match_oracle(B, n, M, d, R):
    """CEM start and round samples bit-exact (FP32 steps), the refit's elites exact (one
    elite: the argmin sample itself, ties to the lower index) and its moments within FP32
    summation error of the FP64 oracle; the archives hold the round's slice.  Sizes up to
    the largest per-box sort (2048 samples)."""
    rng = np.random.default_rng(11 + n)
    lo = rng.uniform(-2, 0, size=(n, d)).astype(np.float32)
    hi = (lo + rng.uniform(0.01, 2, size=(n, d))).astype(np.float32)
    par = (lo[0::2] + (hi[0::2] - lo[0::2]) * rng.random((n // 2, d))).astype(np.float32)
    if n // 2 > 3:
        par[3] = hi[7] + 1.0                               # outside both children: centres
    bab = B.bound_bab_init(4 * n, d, R * M)
    mu, sg = torch.empty(n, d, device="cuda"), torch.empty(n, d, device="cuda")
    B.bound_bab_cem_start(bab, n, dev(lo), dev(hi), dev(par), 2, mu, sg)
    omu, osg = OB.cem_start(lo, hi, par, 2)
    assert np.array_equal(mu.cpu().numpy(), omu) and np.array_equal(sg.cpu().numpy(), osg)
    B.bound_bab_cem_start(bab, n, dev(lo), dev(hi), None, 1, mu, sg)
    assert np.array_equal(mu.cpu().numpy(), OB.cem_start(lo, hi)[0])
    Z = (3.0 * rng.standard_normal((n, M, d))).astype(np.float32)   # many clipped samples
    S = torch.empty(n, M, d, device="cuda")
    S_all = torch.full((n, R * M, d), float("nan"), device="cuda")
    sA, sV = min(1, R - 1), R - 1              # archive slices written by the calls below
    B.bound_bab_cem_samples(bab, n, M, dev(lo), dev(hi), dev(omu), dev(osg), dev(Z), S, S_all,
                            R * M, sA * M)
    oS = OB.cem_samples(lo, hi, omu, osg, Z)
    assert np.array_equal(S.cpu().numpy(), oS)
    assert np.array_equal(S_all[:, sA * M:(sA + 1) * M].cpu().numpy(), oS)
    assert torch.isnan(S_all[:, :sA * M]).all() and torch.isnan(S_all[:, (sA + 1) * M:]).all()
    vals = rng.integers(0, 6, size=(n, M)).astype(np.float32)       # many ties
    vals[n - 1, 0] = np.nan
    V_all = torch.full((n, R * M), float("nan"), device="cuda")
    for E, jit in ((1, 0.0), (min(7, M), 1e-3), (M, 0.0)):
        B.bound_bab_cem_refit(bab, n, M, dev(vals), S, E, jit, mu, sg, V_all, R * M, sV * M)
        rmu, rsg = OB.cem_refit(vals, oS, E, jit)
        gmu, gsg = mu.cpu().numpy(), sg.cpu().numpy()
        if E == 1:
            idx = OB.cem_elites(vals, 1)[:, 0]
            assert np.array_equal(gmu, oS[np.arange(n), idx]) and np.all(gsg == 0.0)
        scale = np.maximum(np.abs(lo), np.abs(hi))
        assert np.all(np.abs(gmu - rmu) <= 4 * E * 2.0 ** -24 * scale), f"mu, {E} elites"
        assert np.all(np.abs(gsg - rsg) <= 1e-5 * scale), f"sigma, {E} elites"
    assert np.array_equal(V_all[:, sV * M:].cpu().numpy(), vals, equal_nan=True)
    assert torch.isnan(V_all[:, :sV * M]).all()
    with pytest.raises(B.BoundError):
        B.bound_bab_cem_refit(bab, n, M, dev(vals), S, M + 1, 0.0, mu, sg)   # n_elite > M
    with pytest.raises(B.BoundError):
        B.bound_bab_cem_samples(bab, n, M, dev(lo), dev(hi), mu, sg, dev(Z), S, S_all, R * M,
                                (R - 1) * M + 1)
    B.bound_bab_destroy(bab)


def test_sample_bounds_merge_equals_one_pass_over_all_samples(B):
    from paper_2412_09584_amd.net import BoundNet
    net, lo, hi = W.plan_objective(d=4, hidden=(32, 32))
    bn = BoundNet(net, 8, 8 * 64)
    rng = np.random.default_rng(12)
    n, M = 6, 40
    X = rng.uniform(-1, 1, (n, 2 * M, 4)).astype(np.float32)
    a_lo = torch.empty(n, bn.n_relu, device="cuda")
    a_hi = torch.empty_like(a_lo)
    B.bound_sample_bounds(bn.handle, n, 2 * M, dev(X.reshape(-1, 4)), a_lo, a_hi)
    m_lo, m_hi = torch.empty_like(a_lo), torch.empty_like(a_lo)
    B.bound_sample_bounds(bn.handle, n, M, dev(X[:, :M].reshape(-1, 4)), m_lo, m_hi)
    out = torch.empty(n * M, 1, device="cuda")
    B.bound_sample_bounds_merge(bn.handle, n, M, dev(X[:, M:].reshape(-1, 4)), m_lo, m_hi, out=out)
    assert torch.equal(m_lo, a_lo) and torch.equal(m_hi, a_hi)
    ref = O.forward(net, X[:, M:].reshape(-1, 4).astype(np.float64))[-1]
    assert np.allclose(out.cpu().numpy(), ref, rtol=1e-4, atol=1e-5)


@pytest.mark.parametrize("bounding", ["crown", "early_stop"])
def test_planning_loop_with_cem_search(B, bounding):
    """The loop with the CEM search (3 rounds of 32 samples, 4 elites) reaches the
    brute-force minimum and agrees with the oracle's loop on the same random numbers."""
    from paper_2412_09584_amd.bab import BaBPlanner
    net, lo, hi = W.plan_objective(d=2, hidden=(16, 16))
    g = np.linspace(-1.0, 1.0, 401)
    G = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    true_min = O.forward(net, G)[-1][:, 0].min()
    cem = dict(rounds=3, n_elite=4, jitter=1e-3)
    pl = BaBPlanner(net, lo, hi, n_pick=8, samples=32, eta=0.75, temperature=0.05, w=5.0,
                    bounding=bounding, stop_layer=2, search="cem", cem_rounds=3, n_elite=4,
                    jitter=1e-3)
    best, ub, P, log = pl.run(12, W.plan_uniforms(), trace=True, normals=W.plan_normals(),
                                  gumbels=W.plan_gumbels())
    fu = O.forward(net, ub.cpu().numpy()[None].astype(np.float64))[-1][0, 0]
    assert abs(fu - best) <= 1e-5 * max(1.0, abs(best))
    assert best <= true_min + 2e-3 * max(1.0, abs(true_min))
    if bounding == "crown":
        assert float(P["f_lo"].min()) <= true_min + 1e-5
        bound = (lambda a, b: np.array([O.crown(net, np.ones((1, 1)), a[i].astype(np.float64),
                                                b[i].astype(np.float64))[1][0]
                                        for i in range(a.shape[0])]))
    else:
        def bound(a, b, S):
            return np.array([O.spec_lower_early_stop(net, len(net), np.ones((1, 1)),
                                                     O.sample_bounds(net, S[i].astype(np.float64)),
                                                     2, "relu")[0] for i in range(a.shape[0])])
    ob, _, _, _ = OB.bab_plan(lambda U: O.forward(net, U)[-1][:, 0], bound, lo, hi, 8, 32, 12,
                              0.75, 0.05, 5.0, W.plan_uniforms(), W.plan_gumbels(),
                              bound_uses_samples=bounding == "early_stop", cem=cem,
                              normals=W.plan_normals())
    assert abs(best - ob) <= 2e-3 * max(1.0, abs(ob))
