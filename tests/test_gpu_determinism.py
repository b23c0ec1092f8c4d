"""Deterministic row sums (BOUND_OPT_DETERMINISTIC): the products store every tile's
partial row sums in a slot of their own and a fixed-order reduction adds them, instead of
float atomics.

  * On every kernel family (dense GEMMs, direct convolutions staged through registers or
    by LDS DMA, the narrow VALU convolution, implicit GEMMs): full CROWN and an alpha /
    beta pass with splits give bitwise the same bounds on repeated runs, agree with the
    atomic mode up to the order of the additions (1e-5 relative) and with the oracle
    stage-wise (1e-4 relative); the gradient equals the atomic mode's.
  * On a 512-subdomain slice of the bench's batch with autotuned plans: two bound and
    gradient steps give bitwise the same lower bounds and gradients.
  * Under HIP-graph capture: every replay of the whole optimisation equals the eager run
    bit for bit.
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


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def close(g, o, rel, what):
    g, o = np.asarray(g, np.float64), np.asarray(o, np.float64)
    lim = rel * np.maximum(np.abs(o), 1.0)
    assert np.all(np.abs(g - o) <= lim), f"{what}: worst {float(np.max(np.abs(g - o) / lim))} x tol"


NETS = {
    "mlp": lambda: W.mlp([30, 24, 24, 24, 6], seed=161),
    "cnn_direct": lambda: W.cnn(seed=162, in_shape=(3, 8, 8), spec=[(16, 3, 1), (16, 4, 2), (32, 3, 1)],
                                fc=(16, 5)),
    "cnn_gemm": lambda: W.cnn(seed=163, in_shape=(3, 12, 12), spec=[(8, 3, 1), (8, 4, 2), (16, 3, 1),
                                                                    (16, 4, 2)], fc=(32, 5)),
    "cnn_odd": lambda: W.cnn(seed=164, in_shape=(4, 6, 6), spec=[(33, 3, 1), (17, 3, 1)], fc=(9, 4)),
}


@pytest.mark.parametrize("kind,opt", [("mlp", 0), ("cnn_direct", 0), ("cnn_direct", "dma"),
                                      ("cnn_direct", "gemm"), ("cnn_gemm", 0), ("cnn_odd", 0)])
def test_deterministic_sums_repeat_bitwise(mod, kind, opt):
    N, B = mod
    net = NETS[kind]()
    n_roots, per_root = 2, 5
    n = n_roots * per_root
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), 165)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    extra = {0: 0, "dma": B.BOUND_OPT_DIRECT_DMA, "gemm": B.BOUND_OPT_GEMM_ONLY}[opt]

    def run(det, fixed=None):
        bn = N.BoundNet(net, n, 4096, 4096)
        B.bound_set_options(bn.handle, extra | (B.BOUND_OPT_DETERMINISTIC if det else 0))
        glo, ghi = bn.crown_bounds(x_lo[root_of], x_hi[root_of])
        if fixed is None:
            lo_np, hi_np = np_(glo), np_(ghi)
            cands = [np.nonzero((lo_np[i] < 0) & (hi_np[i] > 0))[0] for i in range(n)]
            sp = W.random_splits(cands, n, 1, 8, seed=166, root_of=np.arange(n, dtype=np.int32))
            fixed = (glo, ghi, sp, dev(W.random_alpha(n, lo_np.shape[1], 167)),
                     dev(W.random_beta(sp.nnz, C.shape[1], 168)))
        flo, fhi, sp, alpha, beta = fixed
        gl, _ = bn.spec_bounds(C[root_of], flo, fhi, x_lo[root_of], x_hi[root_of], alpha=alpha,
                               splits=N.splits_to_device(sp), beta=beta, both=False, save=True)
        ga, gb = bn.grad(torch.ones(n, C.shape[1], device="cuda"), sp.nnz)
        return [np_(glo), np_(ghi), np_(gl), np_(ga), np_(gb)], fixed

    d1, fixed = run(True)
    d2, _ = run(True, fixed)
    for a, b, what in zip(d1, d2, ("lo", "hi", "lower", "grad alpha", "grad beta")):
        assert np.array_equal(a, b), f"{what} not bitwise reproducible"
    at, _ = run(False, fixed)
    for a, b, what in zip(d1[:3], at[:3], ("lo", "hi", "lower")):
        close(a, b, 1e-5, f"{what}: deterministic vs atomic")
    for a, b, what in zip(d1[3:], at[3:], ("grad alpha", "grad beta")):
        sc = max(float(np.max(np.abs(b))), 1e-30)
        assert np.max(np.abs(a - b)) <= 1e-5 * sc, f"{what}: deterministic vs atomic"
    # stage-wise against the oracle: the pass at the GPU's own intermediate bounds
    flo, fhi, sp, alpha, beta = fixed
    lo64, hi64, al, be = np_(flo), np_(fhi), np_(alpha), np_(beta)
    L = len(net)
    for i in (0, n - 1):
        r = root_of[i]
        q0, q1 = sp.off[i], sp.off[i + 1]
        bounds = list(zip(O.per_layer(net, lo64[i]), O.per_layer(net, hi64[i])))
        splits = O.split_list(net, sp.neuron[q0:q1], sp.sign[q0:q1])
        ref = O.spec_lower(net, L, C[r], bounds, x_lo[r], x_hi[r], O.per_layer(net, al[i]), splits,
                           be[q0:q1])
        close(d1[2][i], ref, 1e-4, f"lower {i} vs oracle")


def test_deterministic_bench_slice_repeats_bitwise(mod):
    N, B = mod
    from paper_2412_09584_amd.batch import BetaBatch
    w = W.beta_cnn(8, 64)
    bb = BetaBatch(w, 64, split_seed=W.SPLIT_SEED)
    bb.autotune()
    B.bound_set_options(bb.bn.handle, B.BOUND_OPT_DETERMINISTIC)
    out = []
    for _ in range(2):
        bb.reset()
        bb.bound_and_grad()
        torch.cuda.synchronize()
        out.append((bb.lower.clone(), bb.ga.clone(), bb.gb.clone()))
    for a, b, what in zip(out[0], out[1], ("lower", "grad alpha", "grad beta")):
        assert torch.equal(a, b), f"{what} not bitwise reproducible"
    B.bound_set_options(bb.bn.handle, 0)
    bb.reset()
    bb.bound_and_grad()
    close(np_(out[0][0]), np_(bb.lower), 1e-5, "lower: deterministic vs atomic")


def test_deterministic_graph_replays_equal_the_eager_run_bitwise(mod):
    """The whole alpha / beta optimisation captured as one HIP graph with deterministic
    row sums: every replay's best bounds and final alpha / beta equal the eager run's
    bit for bit (with float atomics only the bounds' rounding could differ)."""
    N, B = mod
    net = NETS["cnn_direct"]()
    n_roots, per_root = 2, 6
    n = n_roots * per_root
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), 181)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    bn = N.BoundNet(net, n, 4096, 4096)
    B.bound_set_options(bn.handle, B.BOUND_OPT_DETERMINISTIC)
    lo, hi = bn.crown_bounds(x_lo, x_hi)
    lo_np, hi_np = np_(lo), np_(hi)
    cands = [np.nonzero((lo_np[r] < 0) & (hi_np[r] > 0))[0] for r in range(n_roots)]
    sp = W.random_splits(cands, n, 1, 6, seed=182, root_of=root_of)
    opt = N.AlphaBetaOptimizer(bn, C[root_of], lo, hi, x_lo[root_of], x_hi[root_of],
                               bound_of=dev(root_of, torch.int32), splits=N.splits_to_device(sp),
                               steps=5)
    best_e = opt.run().clone()
    alpha_e, beta_e = opt.alpha.clone(), opt.beta.clone()
    opt.capture()
    for rep in range(2):
        torch.randn(256, 256, device="cuda").sum()          # eager work between replays
        torch.cuda.synchronize()
        best_g = opt.replay()
        torch.cuda.synchronize()
        assert torch.equal(best_g, best_e), f"replay {rep}: best"
        assert torch.equal(opt.alpha, alpha_e) and torch.equal(opt.beta, beta_e), f"replay {rep}"
