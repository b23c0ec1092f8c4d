"""bound_grad_adam: the alpha-gradient fused into alpha's Adam step inside the library.

With zero moments at the start it must give, step after step, the alpha of bound_grad
followed by bound_adam on the dense gradient (whose parity with the oracle the other
tests pin), the same beta gradient, and so the same bounds -- bitwise, since the row sums
of the gradient are added in the same order and both Adam kernels share one update
routine.  Covered: splits (with repeated entries), full propagation, early stop at a
linear node, checkpointed recomputation, both bound sides, one bounds row per instance,
and the bench's subdomain batch through AlphaBetaOptimizer.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_09584_amd import net as N
    from paper_2412_09584_amd import binding as B
    return N, B


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


@pytest.mark.parametrize("case", ["full", "stop_linear", "recompute", "both_sides", "per_instance"])
def test_fused_alpha_step_equals_gradient_then_adam(mod, case):
    N, B = mod
    net = W.cnn(seed=191, in_shape=(3, 8, 8), spec=[(16, 3, 1), (16, 4, 2), (32, 3, 1)], fc=(16, 5))
    n_roots, per_root = 2, 5
    n = n_roots * per_root
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), 192)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    bn = N.BoundNet(net, n, 4096, 4096)
    B.bound_set_options(bn.handle, B.BOUND_OPT_DETERMINISTIC)
    lo, hi = bn.crown_bounds(x_lo, x_hi)
    lo_np, hi_np = lo.double().cpu().numpy(), hi.double().cpu().numpy()
    cands = [np.nonzero((lo_np[r] < 0) & (hi_np[r] > 0))[0] for r in range(n_roots)]
    sp = W.random_splits(cands, n, 1, 6, seed=193, root_of=root_of)
    # a repeated entry of opposite sign on one subdomain's first split neuron
    off, neu, sgn = list(sp.off), list(sp.neuron), list(sp.sign)
    k0 = off[0]
    neu.insert(k0 + 1, neu[k0])
    sgn.insert(k0 + 1, -sgn[k0])
    off = [off[0]] + [o + 1 for o in off[1:]]
    spd = {"off": dev(off, torch.int32), "idx": dev(neu, torch.int32), "sign": dev(sgn, torch.int8)}
    nnz, rows, L = len(neu), C.shape[1], len(net)
    Cd, xl, xh, bof = dev(C[root_of]), dev(x_lo[root_of]), dev(x_hi[root_of]), dev(root_of, torch.int32)
    flags = B.BOUND_SAVE_FOR_GRAD | (B.BOUND_RECOMPUTE if case == "recompute" else 0) | \
        (B.BOUND_BOTH_SIDES if case == "both_sides" else 0)
    stop = dict(stop_layer=L - 1, stop_mode=B.BOUND_STOP_LINEAR) if case == "stop_linear" else {}
    nb = n_roots
    if case == "per_instance":        # one bounds row per instance instead of per root
        ridx = dev(root_of, torch.long)
        lo, hi, nb, bof = lo[ridx].contiguous(), hi[ridx].contiguous(), n, None
    # with both sides the gradient weights the lower bounds and the negated upper bounds
    wrows = 2 * rows if case == "both_sides" else rows
    ones = torch.ones(n, wrows, device="cuda")

    use_beta = case != "both_sides"     # both sides: splits clamp, no multipliers

    def run(fused, steps=4):
        alpha = torch.full((n, bn.n_relu), 0.5, device="cuda")
        beta = torch.zeros(nnz, rows, device="cuda")
        ma, va = torch.zeros_like(alpha), torch.zeros_like(alpha)
        mb, vb = torch.zeros_like(beta), torch.zeros_like(beta)
        ga, gb = torch.empty_like(alpha), torch.zeros_like(beta)
        lower = torch.empty(n, rows, device="cuda")
        upper = torch.empty(n, rows, device="cuda") if case == "both_sides" else None
        out = []
        for t in range(1, steps + 1):
            B.bound_backward(bn.handle, n, rows, L, spec=Cd, lo=lo, hi=hi, n_bounds=nb,
                             bound_of=bof, alpha=alpha, split_off=spd["off"], split_idx=spd["idx"],
                             split_sign=spd["sign"], nnz=nnz, beta=beta if use_beta else None,
                             x_lo=xl, x_hi=xh, flags=flags, lower=lower, upper=upper, **stop)
            g_b = gb if use_beta else None
            if fused:
                B.bound_grad_adam(bn.handle, ones, alpha, ma, va, t, 0.1, grad_scale=-1.0,
                                  clip_lo=0.0, clip_hi=1.0, grad_beta=g_b)
            else:
                B.bound_grad(bn.handle, ones, ga, g_b)
                B.bound_adam(alpha, ga, ma, va, t, 0.1, grad_scale=-1.0, clip_lo=0.0, clip_hi=1.0)
            if use_beta:
                B.bound_adam(beta, gb, mb, vb, t, 0.1, grad_scale=-1.0, clip_lo=0.0)
            torch.cuda.synchronize()
            out.append((torch.cat([lower] + ([upper] if upper is not None else []), 1).clone(),
                        alpha.clone(), beta.clone(), gb.clone()))
        return out

    ref, got = run(False), run(True)
    moved = False
    for t, ((l0, a0, b0, g0), (l1, a1, b1, g1)) in enumerate(zip(ref, got), 1):
        assert torch.equal(l0, l1), f"step {t}: lower"
        assert torch.equal(a0, a1), f"step {t}: alpha ({(a0 != a1).sum().item()} entries differ)"
        assert torch.equal(g0, g1), f"step {t}: beta gradient"
        assert torch.equal(b0, b1), f"step {t}: beta"
        moved |= bool((a1 != 0.5).any())
    assert moved, "alpha never moved: the test exercises nothing"
    # a later pass without SAVE_FOR_GRAD leaves nothing to differentiate
    lower = torch.empty(n, rows, device="cuda")
    B.bound_backward(bn.handle, n, rows, L, spec=Cd, lo=lo, hi=hi, n_bounds=nb, bound_of=bof,
                     alpha=torch.full((n, bn.n_relu), 0.5, device="cuda"), x_lo=xl, x_hi=xh,
                     flags=0, lower=lower)
    z = [torch.zeros(n, bn.n_relu, device="cuda") for _ in range(3)]
    with pytest.raises(B.BoundError, match="no SAVE_FOR_GRAD pass"):
        B.bound_grad_adam(bn.handle, ones, z[0], z[1], z[2], 1, 0.1)


def test_fused_optimizer_on_the_bench_slice(mod):
    """AlphaBetaOptimizer on a 512-subdomain slice of the bench's batch (autotuned plans):
    the fused optimisation ends with the same alpha, beta and best bounds as the unfused
    one, and its graph replay with the eager run's."""
    N, B = mod
    from paper_2412_09584_amd.batch import BetaBatch
    w = W.beta_cnn(8, 64)
    bb = BetaBatch(w, 64, split_seed=W.SPLIT_SEED)
    bb.autotune()
    B.bound_set_options(bb.bn.handle, B.BOUND_OPT_DETERMINISTIC)
    res = {}
    for fused in (False, True):
        bb.fused = fused
        opt = bb.optimizer(4)
        best = opt.run().clone()
        torch.cuda.synchronize()
        res[fused] = (best, opt.alpha.clone(), opt.beta.clone())
        if fused:
            opt.capture()
            torch.randn(128, 128, device="cuda").sum()
            torch.cuda.synchronize()
            rb = opt.replay()
            torch.cuda.synchronize()
            assert torch.equal(rb, best), "graph replay: best"
            assert torch.equal(opt.alpha, res[True][1]), "graph replay: alpha"
    for a, b, what in zip(res[False], res[True], ("best", "alpha", "beta")):
        assert torch.equal(a, b), what
