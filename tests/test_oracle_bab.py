"""Pins of the branch-and-bound planning oracle (oracle/bab.py) against what the paper and
elementary probability fix: the pruning example of the appendix, the softmax law of the
pick-out (Eq. lf_pick) checked by frequencies, its limits, the split heuristic on hand
cases, and the whole loop against brute force on a small objective."""
import itertools
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import bab as OB  # noqa: E402
from oracle import crown as O  # noqa: E402


def test_prune_paper_example():
    # appendix illustration: lower bound 4 on C1, best found objective 3 (in C2)
    f_lo = np.array([4.0, 1.0, 3.0])
    assert list(OB.prune(f_lo, 3.0)) == [1, 2]        # C1 pruned, equality kept


def _gumbel(u):
    """Standard Gumbel variates from uniforms (float64, then float32)."""
    return (-np.log(-np.log(np.asarray(u, np.float64)))).astype(np.float32)


def test_pick_eta_one_is_the_sort_by_upper_bound():
    rng = np.random.default_rng(0)
    f_hi = rng.normal(size=50)
    f_hi[7] = f_hi[3]                                   # a tie: lower index first
    picked, rest = OB.pick_out(rng.normal(size=50), f_hi, _gumbel(rng.random(50)), 10, 1.0, 0.05)
    ref = sorted(range(50), key=lambda i: (f_hi[i], i))[:10]
    assert list(picked) == ref
    assert list(rest) == [i for i in range(50) if i not in ref]


def _softmax_p(f_lo, T):
    s = (f_lo - f_lo.min()) / (f_lo.max() - f_lo.min())
    e = np.exp(-s / T)
    return e / e.sum()


def test_pick_single_draw_follows_the_softmax():
    f_lo = np.array([0.0, 0.5, 1.0, 0.2, 0.9])
    T = 0.5
    p = _softmax_p(f_lo, T)
    rng = np.random.default_rng(1)
    n_draw = 40000
    cnt = np.zeros(5)
    f_hi = np.zeros(5)
    for _ in range(n_draw):
        picked, _ = OB.pick_out(f_lo, f_hi, _gumbel(rng.random(5)), 1, 0.0, T)
        cnt[picked[0]] += 1
    sd = np.sqrt(n_draw * p * (1 - p))
    assert np.all(np.abs(cnt - n_draw * p) <= 4.5 * sd), (cnt / n_draw, p)


def test_pick_two_draws_without_replacement():
    f_lo = np.array([0.0, 0.3, 1.0, 0.6])
    T = 0.4
    p = _softmax_p(f_lo, T)
    law = {}
    for a, b in itertools.permutations(range(4), 2):
        law[frozenset((a, b))] = law.get(frozenset((a, b)), 0.0) + p[a] * p[b] / (1 - p[a])
    rng = np.random.default_rng(2)
    n_draw = 30000
    cnt = {k: 0 for k in law}
    for _ in range(n_draw):
        picked, _ = OB.pick_out(f_lo, np.zeros(4), _gumbel(rng.random(4)), 2, 0.0, T)
        assert picked[0] != picked[1]
        cnt[frozenset(picked)] += 1
    for k, q in law.items():
        sd = math.sqrt(n_draw * q * (1 - q))
        assert abs(cnt[k] - n_draw * q) <= 4.5 * sd, (k, cnt[k] / n_draw, q)


def test_pick_low_temperature_takes_the_smallest_lower_bounds():
    rng = np.random.default_rng(3)
    f_lo = rng.permutation(40).astype(float)            # distinct, spaced by 1
    f_hi = rng.normal(size=40)
    n, eta = 12, 0.5
    picked, _ = OB.pick_out(f_lo, f_hi, _gumbel(rng.random(40)), n, eta, 1e-4)
    first = sorted(range(40), key=lambda i: (f_hi[i], i))[:6]
    assert list(picked[:6]) == first
    rest = [i for i in range(40) if i not in first]
    assert list(picked[6:]) == sorted(rest, key=lambda i: f_lo[i])[:6]


def test_pick_is_invariant_to_affine_rescaling_of_lower_bounds():
    rng = np.random.default_rng(4)
    f_lo, f_hi, u = rng.normal(size=30), rng.normal(size=30), _gumbel(rng.random(30))
    a, _ = OB.pick_out(f_lo, f_hi, u, 10, 0.3, 0.05)
    b, _ = OB.pick_out(3.0 * f_lo + 7.0, f_hi, u, 10, 0.3, 0.05)
    assert list(a) == list(b)


def test_pick_puts_nonfinite_lower_bounds_last():
    f_lo = np.array([np.inf, 0.2, np.inf, 0.1, 0.3])
    picked, rest = OB.pick_out(f_lo, np.zeros(5), np.zeros(5, np.float32), 4, 0.0, 0.05)
    assert set(picked[:3]) == {1, 3, 4} and picked[3] == 0 and list(rest) == [2]


def test_split_hand_cases():
    lo = np.array([[0.0, 0.0, 0.0]], np.float32)
    hi = np.array([[1.0, 1.0, 2.0]], np.float32)
    # 4 top samples: all in the lower half of dim 0 (|4-0|*1 = 4), 3:1 in dim 1
    # (|3-1|*1 = 2), 2:2 in dim 2 (0)
    top = np.array([[[0.1, 0.2, 0.1], [0.2, 0.3, 1.9], [0.3, 0.4, 0.2], [0.4, 0.9, 1.5]]],
                   np.float32)
    clo, chi, dims = OB.split(lo, hi, top)
    assert dims[0] == 0
    assert np.array_equal(chi[0], [0.5, 1.0, 2.0]) and np.array_equal(clo[0], [0.0, 0.0, 0.0])
    assert np.array_equal(clo[1], [0.5, 0.0, 0.0]) and np.array_equal(chi[1], [1.0, 1.0, 2.0])
    # the midpoint itself counts on the lower side
    top2 = np.array([[[0.5, 0.5, 1.0], [0.5, 0.5, 1.0]]], np.float32)
    _, _, d2 = OB.split(lo, hi, top2)
    assert d2[0] == 2                                   # |2-0| * 2 beats |2-0| * 1
    # balanced everywhere: the widest dimension
    top3 = np.array([[[0.1, 0.1, 0.1], [0.9, 0.9, 1.9]]], np.float32)
    _, _, d3 = OB.split(lo, hi, top3)
    assert d3[0] == 2


def test_search_summary_min_and_ties():
    vals = np.array([[3.0, 1.0, 1.0, 2.0]])
    S = np.arange(8, dtype=np.float32).reshape(1, 4, 2)
    f_hi, top = OB.search_summary(vals, S, 3)
    assert f_hi[0] == 1.0
    assert np.array_equal(top[0], S[0, [1, 2, 3]])
    assert OB.n_top(1.0, 64) == 1 and OB.n_top(10.0, 64) == 7 and OB.n_top(100.0, 5) == 5


def _objective_and_bound(net):
    C = np.ones((1, 1))

    def objective(U):
        return O.forward(net, U)[-1][:, 0]

    def bound(lo, hi):
        return np.array([O.crown(net, C, lo[i].astype(np.float64), hi[i].astype(np.float64))[1][0]
                         for i in range(lo.shape[0])])
    return objective, bound


def test_bab_loop_reaches_the_brute_force_minimum():
    net, lo, hi = W.plan_objective(d=2, hidden=(16, 16))
    objective, bound = _objective_and_bound(net)
    g = np.linspace(-1.0, 1.0, 401)
    G = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    true_min = objective(G).min()
    best, ubest, trace, P = OB.bab_plan(objective, bound, lo, hi, n_pick=8, M=64, iters=12,
                                        eta=0.75, T=0.05, w=5.0, uniforms=W.plan_uniforms(),
                                        gumbels=W.plan_gumbels())
    assert abs(objective(ubest[None])[0] - best) < 1e-9        # the best value is attained
    assert best <= true_min + 2e-3 * max(1.0, abs(true_min))
    # sound pruning: the surviving boxes still bound the minimum from below
    assert P["f_lo"].min() <= true_min + 1e-9
    # the loop shrinks the search space: boxes are smaller than the root
    assert trace[-1]["size"] > 0 and np.all(P["hi"] - P["lo"] <= 2.0)


def _early_stop_bound(net, stop):
    """The paper's bounding of a box from its search samples: empirical pre-activation
    bounds, then the objective's pass stopped at the ReLU of layer `stop`."""
    def bound(lo, hi, S):
        out = []
        for b in range(lo.shape[0]):
            sb = O.sample_bounds(net, S[b].astype(np.float64))
            out.append(O.spec_lower_early_stop(net, len(net), np.ones((1, 1)), sb, stop, "relu")[0])
        return np.array(out)
    return bound


def test_bab_loop_with_search_integrated_early_stop_bounding():
    """The loop with the paper's bounding (empirical bounds from each box's own search
    samples, early stop at the last ReLU layer) still reaches the brute-force minimum of
    a small 2-D objective, and its estimates sit at or below the box's best sample."""
    net, lo, hi = W.plan_objective(d=2, hidden=(16, 16))
    g = np.linspace(-1.0, 1.0, 401)
    G = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    true_min = O.forward(net, G)[-1][:, 0].min()
    best, ub, trace, P = OB.bab_plan(lambda U: O.forward(net, U)[-1][:, 0], _early_stop_bound(net, 2),
                                     lo, hi, 8, 64, 12, 0.75, 0.05, 5.0, W.plan_uniforms(), W.plan_gumbels(),
                                     bound_uses_samples=True)
    assert best <= true_min + 2e-3 * max(1.0, abs(true_min))
    assert np.all(P["f_lo"] <= P["f_hi"] + 1e-9)


# ------------------------------------------------------------------ CEM search (Section 3.3)
def test_cem_start_uses_the_parent_sample_only_inside_the_child():
    lo = np.array([[0.0, 0.0], [0.5, 0.0]], np.float32)
    hi = np.array([[0.5, 1.0], [1.0, 1.0]], np.float32)
    u = np.array([[0.25, 0.75]], np.float32)          # lies in child 0, not in child 1
    mu, sigma = OB.cem_start(lo, hi, u, 2)
    assert np.array_equal(mu[0], u[0])
    assert np.array_equal(mu[1], np.array([0.75, 0.5], np.float32))
    assert np.array_equal(sigma, np.array([[0.25, 0.5], [0.25, 0.5]], np.float32))
    mu0, _ = OB.cem_start(lo, hi)
    assert np.array_equal(mu0, (lo + hi) / 2)


def test_cem_samples_follow_the_clipped_normal_law():
    """Mean and deviation of unclipped samples match mu and sigma; in a tight box the
    mass at each face is the normal tail beyond it, Phi((lo - mu) / sigma)."""
    from scipy.stats import norm
    rng = np.random.default_rng(3)
    n, M, d = 1, 200000, 2
    Z = rng.standard_normal((n, M, d)).astype(np.float32)
    mu = np.array([[0.3, -0.2]], np.float32)
    sg = np.array([[0.05, 0.1]], np.float32)
    S = OB.cem_samples(np.full((1, d), -10, np.float32), np.full((1, d), 10, np.float32), mu, sg, Z)
    assert np.all(np.abs(S[0].mean(0) - mu[0]) < 4 * sg[0] / np.sqrt(M))
    assert np.all(np.abs(S[0].std(0) / sg[0] - 1) < 0.01)
    lo, hi = np.array([[0.25, -0.3]], np.float32), np.array([[0.4, -0.05]], np.float32)
    S = OB.cem_samples(lo, hi, mu, sg, Z)
    assert np.all((S >= lo[:, None]) & (S <= hi[:, None]))
    p_lo = norm.cdf((lo[0] - mu[0]) / sg[0])
    p_hi = norm.sf((hi[0] - mu[0]) / sg[0])
    assert np.all(np.abs((S[0] == lo[0]).mean(0) - p_lo) < 5 * np.sqrt(p_lo * (1 - p_lo) / M) + 1e-4)
    assert np.all(np.abs((S[0] == hi[0]).mean(0) - p_hi) < 5 * np.sqrt(p_hi * (1 - p_hi) / M) + 1e-4)


def test_cem_refit_with_every_sample_an_elite_is_the_sample_mean_and_std():
    rng = np.random.default_rng(4)
    S = rng.normal(size=(3, 50, 4)).astype(np.float32)
    V = rng.normal(size=(3, 50))
    mu, sigma = OB.cem_refit(V, S, 50, 0.0)
    assert np.allclose(mu, S.astype(np.float64).mean(1), rtol=0, atol=1e-12)
    assert np.allclose(sigma, S.astype(np.float64).std(1), rtol=0, atol=1e-12)
    mu, sigma = OB.cem_refit(V, S, 50, 0.25)
    assert np.allclose(sigma, S.astype(np.float64).std(1) + 0.25, rtol=0, atol=1e-12)


def test_cem_refit_single_elite_ties_and_nan():
    S = np.arange(10, dtype=np.float32).reshape(1, 5, 2)
    V = np.array([[2.0, 1.0, np.nan, 1.0, np.inf]])
    mu, sigma = OB.cem_refit(V, S, 1, 0.001)
    assert np.array_equal(mu[0], S[0, 1]) and np.all(sigma == 0.001)   # tie: lower index
    assert list(OB.cem_elites(V, 5)[0]) == [1, 3, 0, 2, 4]              # NaN as +inf, by index


def test_cem_elites_by_brute_force():
    rng = np.random.default_rng(5)
    for trial in range(50):
        M = int(rng.integers(1, 12))
        E = int(rng.integers(1, M + 1))
        V = rng.integers(0, 4, size=(1, M)).astype(np.float64)     # many ties
        best = min(itertools.combinations(range(M), E), key=lambda c: (sorted(V[0, list(c)]), c))
        assert set(OB.cem_elites(V, E)[0]) == set(best)


def test_cem_concentrates_on_the_minimiser_of_a_convex_quadratic():
    """On f(u) = |u - c|^2 the refitted mean approaches c, and the best of R rounds beats
    R * M uniform samples."""
    c = np.array([0.31, -0.52, 0.77], np.float32)
    lo, hi = -np.ones((1, 3), np.float32), np.ones((1, 3), np.float32)
    f = lambda U: np.sum((np.asarray(U, np.float64) - c) ** 2, axis=1)
    rng = np.random.default_rng(6)
    S, V, mu, sigma = OB.cem_search(f, lo, hi, lambda r, shape: rng.standard_normal(shape).astype(np.float32),
                                    10, 200, 20, 1e-4)
    assert np.max(np.abs(mu[0] - c)) < 5e-3
    assert np.max(sigma) < 5e-3
    U = np.random.default_rng(7).uniform(-1, 1, (2000, 3))
    assert V.min() < f(U).min()
    assert S.shape == (1, 2000, 3) and V.shape == (1, 2000)


def test_bab_loop_with_cem_search_reaches_the_brute_force_minimum():
    net, lo, hi = W.plan_objective(d=2, hidden=(16, 16))
    objective, bound = _objective_and_bound(net)
    g = np.linspace(-1.0, 1.0, 401)
    G = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    true_min = objective(G).min()
    best, ubest, trace, P = OB.bab_plan(objective, bound, lo, hi, n_pick=8, M=32, iters=12,
                                        eta=0.75, T=0.05, w=5.0, uniforms=W.plan_uniforms(),
                                        gumbels=W.plan_gumbels(), cem=dict(rounds=3, n_elite=4, jitter=1e-3),
                                        normals=W.plan_normals())
    assert abs(objective(ubest[None])[0] - best) < 1e-9
    assert best <= true_min + 2e-3 * max(1.0, abs(true_min))
    assert P["f_lo"].min() <= true_min + 1e-9


def test_pick_fp32_keys_agree_with_fp64_softmax_draws_up_to_rounding():
    """The FP32 keys of the pick-out give a valid Gumbel-top-k under keys formed in FP64:
    every pick's FP64 score is within rounding of the best score left out."""
    rng = np.random.default_rng(9)
    N, n = 3000, 500
    f_lo = rng.normal(size=N).astype(np.float32)
    g = _gumbel(rng.random(N))
    T = 0.05
    picked, _ = OB.pick_out(f_lo, np.zeros(N, np.float32), g, n, 0.0, T)
    f = f_lo.astype(np.float64)
    score = -(f - f.min()) / (f.max() - f.min()) / T + g.astype(np.float64)
    out = np.setdiff1d(np.arange(N), picked)
    tol = 1e-5 * (1.0 + np.abs(score).max())
    assert score[picked].min() >= score[out].max() - tol
    assert np.all(np.diff(score[picked]) <= tol)          # in descending order of score
