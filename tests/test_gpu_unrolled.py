"""GPU parity on the unrolled dynamics model (the planning-shaped workload): the Pushing
dynamics MLP 10-128-256-256-128-8 unrolled over H steps as one ReLU layer chain (4 H + 2
layers) with an L1 objective, bounded over action sub-boxes (planning subdomains).

  * H = 2: full CROWN end to end against the oracle (every pre-activation bound and the
    objective's lower bound).
  * H = 20 (82 layers, 81 ReLU layers): full CROWN on the GPU; stage-wise, the oracle
    recomputes the bounds of several layers from the GPU's own bounds of the layers below
    (the widths pass 1e30 near the top: relative parity still holds), and the objective's
    bound is checked for soundness against the oracle's (vacuous at this depth).
  * The pass of an optimised intermediate bound (rows [I; -I], both sides saved for the
    gradient, best and best_upper kept) at random slopes: bounds, best / best_upper and
    the slope gradient against the oracle.
  * Optimised intermediate bounds (H = 2): sound on sampled action sequences and tighter
    in total than the GPU's plain CROWN.
  * Early stop over search-integrated bounds on the H = 20 chain against the oracle.
  * The planning loop (CEM search, search-integrated bounds, early stop) on the H = 20
    chain.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import crown as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_09584_amd import net as N
    from paper_2412_09584_amd import binding as B
    return N, B


def np_(t):
    return t.detach().double().cpu().numpy()


def close(g, o, rel=1e-4, what=""):
    g, o = np.asarray(g, np.float64), np.asarray(o, np.float64)
    err = np.abs(g - o)
    lim = rel * np.maximum(np.abs(o), 1.0)
    assert np.all(err <= lim), f"{what}: worst {float(np.max(err / lim))} x tol"


def test_unrolled_h2_full_crown_end_to_end(mod):
    N, B = mod
    uw = W.pushing_unrolled(2)
    lo_b, hi_b = W.action_subboxes(uw, 4, seed=51)
    bn = N.BoundNet(uw.net, 4, 4 * 600)
    glo, ghi = bn.crown_bounds(lo_b, hi_b)
    C = np.ones((4, 1, 1), np.float32)
    gl, gu = bn.spec_bounds(C, glo, ghi, lo_b, hi_b)
    for i in range(4):
        bounds, ol, ou = O.crown(uw.net, C[i], lo_b[i], hi_b[i])
        close(np_(glo)[i], np.concatenate([b[0] for b in bounds]), what=f"lo {i}")
        close(np_(ghi)[i], np.concatenate([b[1] for b in bounds]), what=f"hi {i}")
        close(np_(gl)[i], ol, what=f"objective lower {i}")
        close(np_(gu)[i], ou, what=f"objective upper {i}")


def test_unrolled_h20_deep_chain_stagewise(mod):
    N, B = mod
    uw = W.pushing_unrolled(20)
    assert len(uw.net) == 82
    lo_b, hi_b = W.action_subboxes(uw, 2, seed=52, width=(0.01, 0.03))
    bn = N.BoundNet(uw.net, 2, 2 * 600)
    glo, ghi = bn.crown_bounds(lo_b, hi_b)
    C = np.ones((2, 1, 1), np.float32)
    gl, _ = bn.spec_bounds(C, glo, ghi, lo_b, hi_b)
    lo, hi = np_(glo), np_(ghi)
    off = O.relu_offsets(uw.net)
    for i in range(2):
        bounds = list(zip(O.per_layer(uw.net, lo[i]), O.per_layer(uw.net, hi[i])))
        for k in (2, 5, 21, 42, 63, 80, 81):
            d = W.out_dim(uw.net[k - 1])
            A = np.concatenate([np.eye(d), -np.eye(d)])
            ref = O.spec_lower(uw.net, k, A, bounds[:k - 1], lo_b[i], hi_b[i])
            close(lo[i, off[k - 1]:off[k]], ref[:d], what=f"lo z{k} of {i}")
            close(hi[i, off[k - 1]:off[k]], -ref[d:], what=f"hi z{k} of {i}")
        # past about 30 layers every neuron is unstable and the widths grow ~500x per
        # step: the objective's bound is vacuous (about -1e34 in FP64), and in FP32 its
        # rounding allowance overflows, so the GPU reports -inf -- still a lower bound
        ref = O.spec_lower(uw.net, 82, C[i], bounds, lo_b[i], hi_b[i])
        g = np_(gl)[i]
        assert np.all(g <= ref + 1e-4 * np.maximum(1.0, np.abs(ref)))
        if np.all(np.abs(ref) < 1e30):
            close(g, ref, what=f"objective {i}")


def test_optimised_intermediate_pass_and_gradient(mod):
    N, B = mod
    uw = W.pushing_unrolled(2)
    n = 3
    lo_b, hi_b = W.action_subboxes(uw, n, seed=53, width=(0.3, 0.6))
    k = 6
    d = W.out_dim(uw.net[k - 1])
    bn = N.BoundNet(uw.net, n, n * 600, n * 2 * 300)
    glo, ghi = bn.crown_bounds(lo_b, hi_b)
    lo, hi = np_(glo), np_(ghi)
    rng = np.random.default_rng(54)
    alpha = rng.uniform(0.0, 1.0, (n, bn.n_relu)).astype(np.float32)
    spec = torch.eye(d, device="cuda").expand(n, d, d).contiguous()
    off = bn.relu_off[k - 1]
    low = torch.empty(n, bn.n_relu, device="cuda")
    upp = torch.empty_like(low)
    best = torch.full_like(low, -float("inf"))
    best_u = torch.full_like(low, float("inf"))
    B.bound_backward(bn.handle, n, d, k, spec=spec, lo=glo, hi=ghi, n_bounds=n,
                     alpha=torch.as_tensor(alpha, device="cuda"), x_lo=torch.as_tensor(lo_b, device="cuda"),
                     x_hi=torch.as_tensor(hi_b, device="cuda"),
                     flags=B.BOUND_BOTH_SIDES | B.BOUND_SAVE_FOR_GRAD, lower=low[:, off:],
                     upper=upp[:, off:], ld=bn.n_relu, best=best[:, off:], best_upper=best_u[:, off:])
    wts = torch.as_tensor(rng.normal(size=(n, 2 * d)), dtype=torch.float32, device="cuda")
    ga = torch.empty(n, bn.n_relu, device="cuda")
    B.bound_grad(bn.handle, wts, ga)
    A = np.concatenate([np.eye(d), -np.eye(d)])
    for i in range(n):
        bounds = list(zip(O.per_layer(uw.net, lo[i]), O.per_layer(uw.net, hi[i])))[:k - 1]
        al = O.per_layer(uw.net, alpha[i])[:k - 1]
        ref = O.spec_lower(uw.net, k, A, bounds, lo_b[i], hi_b[i], al)
        close(np_(low)[i, off:off + d], ref[:d], what=f"lower {i}")
        close(np_(upp)[i, off:off + d], -ref[d:], what=f"upper {i}")
        assert np.array_equal(np_(best)[i, off:off + d], np_(low)[i, off:off + d])
        assert np.array_equal(np_(best_u)[i, off:off + d], np_(upp)[i, off:off + d])
        _, oga, _ = O.spec_lower_grad(uw.net, k, A, bounds, lo_b[i], hi_b[i], al,
                                      gbar=np_(wts)[i])
        oga = np.concatenate(oga)
        g = np_(ga)[i, :len(oga)]
        assert np.max(np.abs(g - oga)) <= 1e-4 * max(np.max(np.abs(oga)), 1e-30), f"grad {i}"
        assert np.all(np_(ga)[i, len(oga):] == 0)          # layers >= k have no slope here


def test_optimised_intermediate_bounds_sound_and_not_looser(mod):
    N, B = mod
    uw = W.pushing_unrolled(2)
    n = 4
    lo_b, hi_b = W.action_subboxes(uw, n, seed=55, width=(0.3, 0.6))
    bn = N.BoundNet(uw.net, n, n * 600, n * 2 * 300)
    plo, phi = bn.crown_bounds(lo_b, hi_b)
    alo, ahi = bn.alpha_crown_bounds(lo_b, hi_b, steps=5)
    plo, phi, alo, ahi = np_(plo), np_(phi), np_(alo), np_(ahi)
    assert (ahi - alo).sum() < (phi - plo).sum()
    for i in range(n):
        u = np.random.default_rng(56 + i).uniform(lo_b[i], hi_b[i], (20000, lo_b.shape[1]))
        z = np.concatenate(O.forward(uw.net, u)[:-1], axis=1)
        assert np.all(z.min(axis=0) >= alo[i]), f"lower bound violated on {i}"
        assert np.all(z.max(axis=0) <= ahi[i]), f"upper bound violated on {i}"


@pytest.mark.parametrize("mode", ["relu", "linear"])
def test_early_stop_over_search_bounds_h20(mod, mode):
    """The paper's bounding for planning on the 82-layer chain: empirical pre-activation
    bounds from 64 samples per subdomain, then the objective's backward pass stopped at
    the ReLU layer of the last step boundary, concretised over that node's box."""
    N, B = mod
    uw = W.pushing_unrolled(20)
    n, M = 3, 64
    lo_b, hi_b = W.action_subboxes(uw, n, seed=57)
    rng = np.random.default_rng(58)
    samp = (lo_b[:, None, :] + (hi_b - lo_b)[:, None, :] *
            rng.uniform(0, 1, (n, M, lo_b.shape[1]))).astype(np.float32)
    bn = N.BoundNet(uw.net, n, max(n * M, n * 600), n)
    slo = torch.empty(n, bn.n_relu, device="cuda")
    shi = torch.empty_like(slo)
    B.bound_sample_bounds(bn.handle, n, M, torch.as_tensor(samp.reshape(n * M, -1), device="cuda"),
                          slo, shi)
    stop = 77                                     # the first ReLU layer of the last step
    C = np.ones((n, 1, 1), np.float32)
    gl, _ = bn.spec_bounds(C, slo, shi, lo_b, hi_b, both=False,
                           stop_layer=stop, stop_mode=B.BOUND_STOP_RELU if mode == "relu"
                           else B.BOUND_STOP_LINEAR)
    lo, hi = np_(slo), np_(shi)
    for i in range(n):
        zs = O.forward(uw.net, samp[i].astype(np.float64))
        ref_lo = np.concatenate([z.min(axis=0) for z in zs[:-1]])
        ref_hi = np.concatenate([z.max(axis=0) for z in zs[:-1]])
        close(lo[i], ref_lo, what=f"sample min {i}")
        close(hi[i], ref_hi, what=f"sample max {i}")
        bounds = list(zip(O.per_layer(uw.net, lo[i]), O.per_layer(uw.net, hi[i])))
        ref = O.spec_lower_early_stop(uw.net, 82, C[i], bounds, stop, mode)
        close(np_(gl)[i], ref, what=f"early-stop bound {i}")


def test_planning_loop_on_the_h20_chain_with_cem_and_early_stop(mod):
    """The paper's planning method end to end on the 82-layer chain: branch and bound over
    the 40-dimensional action box with the CEM search, search-integrated pre-activation
    bounds and the objective's pass stopped at the last step's first ReLU layer.  The best
    value improves on the root's search and is attained by its action sequence; every
    candidate's estimate lies at or below its best sample."""
    N, B = mod
    from paper_2412_09584_amd.bab import BaBPlanner
    uw = W.pushing_unrolled(20)
    pl = BaBPlanner(uw.net, uw.u_lo, uw.u_hi, n_pick=32, samples=64, bounding="early_stop",
                    stop_layer=77, search="cem", cem_rounds=3, n_elite=8)
    best0, _, _, _ = pl.run(0, W.plan_uniforms(), normals=W.plan_normals(), gumbels=W.plan_gumbels())
    best, ub, P, log = pl.run(6, W.plan_uniforms(), trace=True, normals=W.plan_normals(),
                              gumbels=W.plan_gumbels())
    assert best <= best0 and len(log) == 6
    fu = O.forward(uw.net, ub.cpu().numpy()[None].astype(np.float64))[-1][0, 0]
    assert abs(fu - best) <= 1e-4 * max(1.0, abs(best))
    f_lo, f_hi = P["f_lo"].cpu().numpy(), P["f_hi"].cpu().numpy()
    assert np.all(np.isfinite(f_hi))
    assert np.all(f_lo <= f_hi + 1e-4 * np.maximum(1.0, np.abs(f_hi)))
