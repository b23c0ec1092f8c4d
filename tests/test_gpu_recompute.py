"""Checkpointed layer recomputation for the gradient (BOUND_RECOMPUTE) against the mode
that keeps every layer's pre-relaxation coefficients: same bound, same alpha- and
beta-gradients, bit for bit (the recomputed products run the same kernels on the same
inputs; only the bound's row sums use atomics) -- on a CNN with splits and beta, on a
deep MLP, and on the unrolled dynamics chain (H = 5, 22 layers) -- and against the oracle.
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


def _case(kind):
    if kind == "cnn":
        net = W.cnn(seed=171, in_shape=(3, 12, 12), spec=[(8, 3, 1), (8, 4, 2), (16, 3, 1), (16, 4, 2)],
                    fc=(32, 5))
        x0 = W.uniform_inputs(2, W.in_dim(net), 172)
        x_lo, x_hi = W.linf_box(x0, 0.05)
        C = W.margin_spec(W.clean_logits(net, x0))
    elif kind == "mlp":
        net = W.mlp([40] + [64] * 7 + [6], seed=173)
        x0 = W.uniform_inputs(2, 40, 174)
        x_lo, x_hi = W.linf_box(x0, 0.02)
        C = W.margin_spec(W.clean_logits(net, x0))
    else:
        uw = W.pushing_unrolled(5)
        net = uw.net
        x_lo, x_hi = W.action_subboxes(uw, 2, seed=175, width=(0.05, 0.2))
        C = np.ones((2, 1, 1), np.float32)
    return net, x_lo, x_hi, C


@pytest.mark.parametrize("kind", ["cnn", "mlp", "unrolled"])
def test_recompute_gradient_equals_stored(mod, kind):
    N, B = mod
    net, x_lo, x_hi, C = _case(kind)
    n_roots, per_root = 2, 4
    n = n_roots * per_root
    R = C.shape[1]
    bn = N.BoundNet(net, n, max(n * 2 * 1200, 4096), n * R)
    lo, hi = bn.crown_bounds(x_lo, x_hi)
    lo_np, hi_np = np_(lo), np_(hi)
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    cands = [np.nonzero((l < 0) & (u > 0))[0] for l, u in zip(lo_np, hi_np)]
    sp = W.random_splits(cands, n, 1, 6, seed=176, root_of=root_of)
    spd = N.splits_to_device(sp)
    alpha = torch.as_tensor(W.random_alpha(n, bn.n_relu, 177), device="cuda")
    beta = torch.as_tensor(W.random_beta(sp.nnz, R, 178), device="cuda")
    bof = torch.as_tensor(root_of, device="cuda")
    Cs = torch.as_tensor(C[root_of], device="cuda")
    xl = torch.as_tensor(x_lo[root_of], device="cuda")
    xh = torch.as_tensor(x_hi[root_of], device="cuda")
    wts = torch.as_tensor(np.random.default_rng(179).normal(size=(n, R)), dtype=torch.float32,
                          device="cuda")
    out = {}
    for mode in ("store", "recompute"):
        lower = torch.empty(n, R, device="cuda")
        flags = B.BOUND_SAVE_FOR_GRAD | (B.BOUND_RECOMPUTE if mode == "recompute" else 0)
        B.bound_backward(bn.handle, n, R, len(net), spec=Cs, lo=lo, hi=hi, n_bounds=n_roots,
                         bound_of=bof, alpha=alpha, split_off=spd["off"], split_idx=spd["idx"],
                         split_sign=spd["sign"], nnz=sp.nnz, beta=beta, x_lo=xl, x_hi=xh,
                         flags=flags, lower=lower)
        ga = torch.empty(n, bn.n_relu, device="cuda")
        gb = torch.empty(sp.nnz, R, device="cuda")
        B.bound_grad(bn.handle, wts, ga, gb)
        torch.cuda.synchronize()
        out[mode] = (np_(lower), np_(ga), np_(gb))
    s, r = out["store"], out["recompute"]
    assert np.allclose(s[0], r[0], rtol=1e-6, atol=1e-6)
    assert np.array_equal(s[1], r[1]), "alpha gradient"
    assert np.array_equal(s[2], r[2]), "beta gradient"
    # and against the oracle on two subdomains
    L = len(net)
    for i in (0, n - 1):
        q0, q1 = sp.off[i], sp.off[i + 1]
        rr = root_of[i]
        bounds = list(zip(O.per_layer(net, lo_np[rr]), O.per_layer(net, hi_np[rr])))
        splits = O.split_list(net, sp.neuron[q0:q1], sp.sign[q0:q1])
        al = O.per_layer(net, np_(alpha)[i])
        be = np_(beta)[q0:q1]
        _, oga, ogb = O.spec_lower_grad(net, L, C[rr], bounds, x_lo[rr], x_hi[rr], al, splits, be,
                                        gbar=np_(wts)[i])
        oga = np.concatenate(oga)
        sa = max(float(np.max(np.abs(oga))), 1e-30)
        assert np.max(np.abs(r[1][i] - oga)) <= 1e-4 * sa
        assert np.max(np.abs(r[2][q0:q1] - ogb)) <= 1e-4 * max(float(np.max(np.abs(ogb))), sa)


def test_recompute_rejects_early_stop_and_needs_save(mod):
    N, B = mod
    net = W.mlp([10, 12, 12, 3], seed=180)
    x0 = W.uniform_inputs(1, 10, 181)
    x_lo, x_hi = W.linf_box(x0, 0.1)
    bn = N.BoundNet(net, 1, 256, 256)
    lo, hi = bn.crown_bounds(x_lo, x_hi)
    C = torch.eye(3, device="cuda")[None]
    low = torch.empty(1, 3, device="cuda")
    with pytest.raises(B.BoundError):
        B.bound_backward(bn.handle, 1, 3, 3, spec=C, lo=lo, hi=hi, n_bounds=1,
                         x_lo=torch.as_tensor(x_lo, device="cuda"), x_hi=torch.as_tensor(x_hi, device="cuda"),
                         flags=B.BOUND_RECOMPUTE, lower=low)
    with pytest.raises(B.BoundError):
        B.bound_backward(bn.handle, 1, 3, 3, spec=C, lo=lo, hi=hi, n_bounds=1,
                         x_lo=torch.as_tensor(x_lo, device="cuda"), x_hi=torch.as_tensor(x_hi, device="cuda"),
                         flags=B.BOUND_RECOMPUTE | B.BOUND_SAVE_FOR_GRAD, lower=low, stop_layer=1,
                         stop_mode=B.BOUND_STOP_RELU)


def test_debug_check_reports_non_finite(mod):
    """BOUND_OPT_CHECK: a clean pass and gradient pass the checks; a NaN in the input box
    reaches the concretising product's sums and is reported as BOUND_E_NUMERIC."""
    N, B = mod
    net = W.mlp([10, 12, 12, 3], seed=182)
    x0 = W.uniform_inputs(1, 10, 183)
    x_lo, x_hi = W.linf_box(x0, 0.1)
    bn = N.BoundNet(net, 1, 256, 256)
    lo, hi = bn.crown_bounds(x_lo, x_hi)
    B.bound_set_options(bn.handle, B.BOUND_OPT_CHECK)
    C = torch.eye(3, device="cuda")[None]
    low = torch.empty(1, 3, device="cuda")
    xl, xh = torch.as_tensor(x_lo, device="cuda"), torch.as_tensor(x_hi, device="cuda")
    B.bound_backward(bn.handle, 1, 3, 3, spec=C, lo=lo, hi=hi, n_bounds=1, x_lo=xl, x_hi=xh,
                     flags=B.BOUND_SAVE_FOR_GRAD, lower=low)
    ga = torch.empty(1, bn.n_relu, device="cuda")
    B.bound_grad(bn.handle, torch.ones(1, 3, device="cuda"), ga)
    xl_bad = xl.clone()
    xl_bad[0, 3] = float("nan")
    with pytest.raises(B.BoundError) as e:
        B.bound_backward(bn.handle, 1, 3, 3, spec=C, lo=lo, hi=hi, n_bounds=1, x_lo=xl_bad, x_hi=xh,
                         lower=low)
    assert e.value.status == B.BOUND_E_NUMERIC and "NaN" in str(e.value)
