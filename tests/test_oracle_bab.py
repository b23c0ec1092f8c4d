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


def test_pick_eta_one_is_the_sort_by_upper_bound():
    rng = np.random.default_rng(0)
    f_hi = rng.normal(size=50)
    f_hi[7] = f_hi[3]                                   # a tie: lower index first
    picked, rest = OB.pick_out(rng.normal(size=50), f_hi, rng.random(50), 10, 1.0, 0.05)
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
        picked, _ = OB.pick_out(f_lo, f_hi, rng.random(5), 1, 0.0, T)
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
        picked, _ = OB.pick_out(f_lo, np.zeros(4), rng.random(4), 2, 0.0, T)
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
    picked, _ = OB.pick_out(f_lo, f_hi, rng.random(40), n, eta, 1e-4)
    first = sorted(range(40), key=lambda i: (f_hi[i], i))[:6]
    assert list(picked[:6]) == first
    rest = [i for i in range(40) if i not in first]
    assert list(picked[6:]) == sorted(rest, key=lambda i: f_lo[i])[:6]


def test_pick_is_invariant_to_affine_rescaling_of_lower_bounds():
    rng = np.random.default_rng(4)
    f_lo, f_hi, u = rng.normal(size=30), rng.normal(size=30), rng.random(30)
    a, _ = OB.pick_out(f_lo, f_hi, u, 10, 0.3, 0.05)
    b, _ = OB.pick_out(3.0 * f_lo + 7.0, f_hi, u, 10, 0.3, 0.05)
    assert list(a) == list(b)


def test_pick_puts_nonfinite_lower_bounds_last():
    f_lo = np.array([np.inf, 0.2, np.inf, 0.1, 0.3])
    picked, rest = OB.pick_out(f_lo, np.zeros(5), np.full(5, 0.5), 4, 0.0, 0.05)
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
                                        eta=0.75, T=0.05, w=5.0, uniforms=W.plan_uniforms())
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
                                     lo, hi, 8, 64, 12, 0.75, 0.05, 5.0, W.plan_uniforms(),
                                     bound_uses_samples=True)
    assert best <= true_min + 2e-3 * max(1.0, abs(true_min))
    assert np.all(P["f_lo"] <= P["f_hi"] + 1e-9)
