"""GPU parity of the split multipliers' gradient where the relaxation slope does not tell
the split's sign, and of the torch.autograd.Function over the bound pass.

  * A split sign -1 on a neuron whose lower bound is exactly 0 clamps the box to
    [0, 0]: the record is the active one (slope 1), yet d lower / d beta = +Lambda_bar
    (the derivative is -sign times the coefficient's adjoint).
  * Opposite-sign entries on one unstable neuron (either order): the clamped box is
    [0, 0] again, each entry gets -sign times the same adjoint.
  * CrownBound through torch.autograd on the 3x32x32 CNN (64 inputs, random alpha) and
    on an MLP with splits and beta: alpha.grad / beta.grad against the oracle's adjoint
    at the same weights of the rows; a backward after another forward is refused.
Bar as in the other parity tests: 1e-4 relative (bounds per element, gradients in the
infinity norm per instance), at identical alpha and beta.
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


def f32(x):
    return np.asarray(x, np.float32)


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def np_(t):
    return t.detach().double().cpu().numpy()


def close(g, o, rel=1e-4, what=""):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    err = np.abs(g - o)
    lim = rel * np.maximum(np.abs(o), 1.0)
    assert np.all(err <= lim), f"{what}: worst {float(np.max(err / lim))} x tol"


def grad_close(g, o, what):
    scale = max(float(np.max(np.abs(o))), 1e-30)
    assert np.max(np.abs(np.asarray(g) - o)) <= 1e-4 * scale, what


def _net(kind):
    if kind == "mlp":
        return W.mlp([30, 24, 24, 24, 6], seed=161)
    return W.cnn(seed=162, in_shape=(3, 12, 12), spec=[(8, 3, 1), (8, 4, 2), (16, 3, 1), (16, 4, 2)],
                 fc=(32, 5))


@pytest.mark.parametrize("kind", ["mlp", "cnn"])
def test_split_sign_where_the_clamped_box_is_zero(mod, kind):
    N, B = mod
    net = _net(kind)
    x0 = W.uniform_inputs(1, W.in_dim(net), 163)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))[0]
    ob = O.crown_bounds(net, x_lo[0], x_hi[0])
    lo = f32(np.concatenate([b[0] for b in ob])).astype(np.float64)
    hi = f32(np.concatenate([b[1] for b in ob])).astype(np.float64)
    unst = np.nonzero((lo < 0) & (hi > 0))[0]
    # spread the chosen neurons over the ReLU layers
    off = O.relu_offsets(net)
    pick = []
    for m in range(len(off) - 1):
        cand = unst[(unst >= off[m]) & (unst < off[m + 1])]
        pick += list(cand[:3])
    assert len(pick) >= 6
    j0, j1, j2 = pick[0], pick[len(pick) // 2], pick[-1]
    lo[j0] = 0.0                      # root box of j0 starts at exactly 0
    # subdomain 0: sign -1 on j0 (clamped to [0, 0]); 1: j1 with -1 then +1;
    # 2: j2 with +1 then -1; 3: the three of them together, with other unstable neurons
    entries = [[(j0, -1)], [(j1, -1), (j1, 1)], [(j2, 1), (j2, -1)],
               [(pick[1], 1), (j0, -1), (j1, 1), (j1, -1), (pick[-2], -1)]]
    n = len(entries)
    offs, neu, sg = [0], [], []
    for e in entries:
        neu += [a for a, _ in e]
        sg += [b for _, b in e]
        offs.append(len(neu))
    sp = W.Splits(np.array(offs, np.int32), np.array(neu, np.int32), np.array(sg, np.int8))
    n_relu = lo.size
    alpha = W.random_alpha(n, n_relu, 164)
    beta = W.random_beta(sp.nnz, C.shape[0], 165)
    bn = N.BoundNet(net, n, 4096, 4096)
    zero = np.zeros(n, np.int32)
    gl, _ = bn.spec_bounds(np.repeat(C[None], n, 0), dev(f32(lo)[None]), dev(f32(hi)[None]),
                           np.repeat(x_lo, n, 0), np.repeat(x_hi, n, 0), alpha=dev(alpha),
                           bound_of=dev(zero, torch.int32), splits=N.splits_to_device(sp),
                           beta=dev(beta), both=False, save=True)
    ga, gb = bn.grad(torch.ones(n, C.shape[0], device="cuda"), sp.nnz)
    ga, gb = np_(ga), np_(gb)
    bounds = list(zip(O.per_layer(net, lo), O.per_layer(net, hi)))
    L = len(net)
    for i in range(n):
        q0, q1 = sp.off[i], sp.off[i + 1]
        splits = O.split_list(net, sp.neuron[q0:q1], sp.sign[q0:q1])
        al = O.per_layer(net, alpha[i])
        be = beta[q0:q1].astype(np.float64)
        low = O.spec_lower(net, L, C, bounds, x_lo[0], x_hi[0], al, splits, be)
        _, oga, ogb = O.spec_lower_grad(net, L, C, bounds, x_lo[0], x_hi[0], al, splits, be)
        close(np_(gl)[i], low, what=f"lower {i}")
        grad_close(ga[i], np.concatenate(oga), f"grad alpha {i}")
        grad_close(gb[q0:q1], ogb, f"grad beta {i}")
        # the sign matters: opposite-sign entries of one neuron get opposite gradients
        for a in range(q1 - q0):
            for b in range(a + 1, q1 - q0):
                if sp.neuron[q0 + a] == sp.neuron[q0 + b] and sp.sign[q0 + a] != sp.sign[q0 + b]:
                    assert np.allclose(ogb[a], -ogb[b])
                    assert np.max(np.abs(ogb[a])) > 0


def _cnn_batch(N, n):
    w = W.cnn_cifar(n)
    bn = N.BoundNet(w.net, n, max(n * 9, 16384), n * 9)
    lo, hi = bn.crown_bounds(w.x_lo, w.x_hi)
    return w, bn, lo, hi


def test_crown_bound_autograd_cnn_64_inputs(mod):
    """alpha-CROWN shapes (the CNN, 64 inputs, alpha free): torch.autograd through the
    bound Function against the oracle adjoint with the same row weights, on 8 of the 64
    inputs (stage-wise: the oracle takes the GPU's intermediate bounds)."""
    N, B = mod
    n = 64
    w, bn, lo, hi = _cnn_batch(N, n)
    rng = np.random.default_rng(166)
    alpha = torch.tensor(rng.uniform(0.0, 1.0, (n, bn.n_relu)), dtype=torch.float32,
                         device="cuda", requires_grad=True)
    wts = rng.normal(size=(n, 9))
    C = dev(w.spec)
    lower = N.CrownBound.apply(alpha, None, bn, C, lo, hi, dev(w.x_lo), dev(w.x_hi), None, None,
                               None)
    (lower * dev(wts)).sum().backward()
    g = np_(alpha.grad)
    lo_np, hi_np = np_(lo), np_(hi)
    L = len(w.net)
    for i in range(0, n, 8):
        bounds = list(zip(O.per_layer(w.net, lo_np[i]), O.per_layer(w.net, hi_np[i])))
        al = O.per_layer(w.net, np_(alpha)[i])
        low = O.spec_lower(w.net, L, w.spec[i], bounds, w.x_lo[i], w.x_hi[i], al)
        _, oga, _ = O.spec_lower_grad(w.net, L, w.spec[i], bounds, w.x_lo[i], w.x_hi[i], al,
                                      gbar=wts[i])
        close(np_(lower)[i], low, what=f"lower {i}")
        grad_close(g[i], np.concatenate(oga), f"alpha.grad {i}")


def test_crown_bound_autograd_with_beta_and_refusals(mod):
    N, B = mod
    net = W.mlp([30, 24, 24, 24, 6], seed=167)
    n = 6
    x0 = W.uniform_inputs(n, 30, 168)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    bn = N.BoundNet(net, n, 4096, 4096)
    lo, hi = bn.crown_bounds(x_lo, x_hi)
    lo_np, hi_np = np_(lo), np_(hi)
    cands = [np.nonzero((l < 0) & (u > 0))[0] for l, u in zip(lo_np, hi_np)]
    sp = W.random_splits(cands, n, 1, 6, seed=169, root_of=np.arange(n))
    spd = N.splits_to_device(sp)
    rng = np.random.default_rng(170)
    alpha = torch.tensor(rng.uniform(0, 1, (n, bn.n_relu)), dtype=torch.float32, device="cuda",
                         requires_grad=True)
    beta = torch.tensor(rng.uniform(0, 0.5, (sp.nnz, 5)), dtype=torch.float32, device="cuda",
                        requires_grad=True)
    wts = rng.normal(size=(n, 5))
    args = (bn, dev(C), lo, hi, dev(x_lo), dev(x_hi), None, spd, None)
    lower = N.CrownBound.apply(alpha, beta, *args)
    (lower * dev(wts)).sum().backward()
    ga, gb = np_(alpha.grad), np_(beta.grad)
    L = len(net)
    for i in range(n):
        q0, q1 = sp.off[i], sp.off[i + 1]
        bounds = list(zip(O.per_layer(net, lo_np[i]), O.per_layer(net, hi_np[i])))
        splits = O.split_list(net, sp.neuron[q0:q1], sp.sign[q0:q1])
        al = O.per_layer(net, np_(alpha)[i])
        be = np_(beta)[q0:q1]
        _, oga, ogb = O.spec_lower_grad(net, L, C[i], bounds, x_lo[i], x_hi[i], al, splits, be,
                                        gbar=wts[i])
        grad_close(ga[i], np.concatenate(oga), f"alpha.grad {i}")
        grad_close(gb[q0:q1], ogb, f"beta.grad {i}")
    # a second forward before the first backward: the first backward is refused
    alpha.grad = None
    first = N.CrownBound.apply(alpha, beta, *args)
    second = N.CrownBound.apply(alpha, beta, *args)
    with pytest.raises(B.BoundError) as e:
        first.sum().backward()
    assert e.value.status == B.BOUND_E_STATE
    second.sum().backward()            # the latest pass is still differentiable
    assert alpha.grad is not None
    # buffer shapes that are not the saved pass's are refused
    with pytest.raises(B.BoundError) as e:
        B.bound_grad(bn.handle, torch.ones(n - 1, 5, device="cuda"),
                     torch.empty(n - 1, bn.n_relu, device="cuda"))
    assert e.value.status == B.BOUND_E_SHAPE
    with pytest.raises(B.BoundError) as e:
        B.bound_grad(bn.handle, torch.ones(n, 5, device="cuda"),
                     torch.empty(n, bn.n_relu, device="cuda"),
                     torch.empty(sp.nnz + 1, 5, device="cuda"))
    assert e.value.status == B.BOUND_E_SHAPE
