"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Bar: |gpu - oracle| <= 1e-4 * max(|oracle|, 1) for every bound; gradients
||g - o||_inf <= 1e-4 * ||o||_inf per instance, at identical alpha / beta.
Stage-wise checks hand both sides the same (oracle-computed, FP32-rounded)
intermediate bounds, so the stable / unstable classes agree; end-to-end checks let each
side compute its own intermediate bounds.
"""
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import crown as O

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def mod():
    _need_gpu()
    from paper_2412_09584_amd import net as N
    from paper_2412_09584_amd import binding as B
    return N, B


def close(g, o, rel=1e-4, what=""):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    both_inf = np.isinf(g) & np.isinf(o) & (np.sign(g) == np.sign(o))
    err = np.where(both_inf, 0.0, np.abs(g - o))
    lim = rel * np.maximum(np.abs(np.where(both_inf, 0.0, o)), 1.0)
    bad = err > lim
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} beyond tolerance; worst "
                           f"{float(np.max(err / lim))} x tol, e.g. gpu {g[bad][:3]} oracle {o[bad][:3]}")


def np_(t):
    return t.detach().double().cpu().numpy()


def oracle_bounds(net, x_lo, x_hi, slack=True):
    return [O.crown_bounds(net, x_lo[i], x_hi[i], use_slack=slack) for i in range(len(x_lo))]


def flat(bounds_list):
    lo = np.stack([np.concatenate([b[0] for b in bl]) for bl in bounds_list])
    hi = np.stack([np.concatenate([b[1] for b in bl]) for bl in bounds_list])
    return lo, hi


def split_layers(net, flat_row):
    return O.per_layer(net, flat_row)


def f32(x):
    return np.asarray(x, np.float32)


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def tiny_cnn(seed=5, H=12, convs=((8, 3, 1), (8, 4, 2), (16, 3, 1), (16, 4, 2)), fc=(32, 5), cin=3):
    return W.cnn(seed=seed, in_shape=(cin, H, H), spec=list(convs), fc=fc)


# ---------------------------------------------------------------------------- passes
def test_single_linear_layer(mod):
    N, B = mod
    net = W.mlp([20, 6], seed=3)
    x0 = W.uniform_inputs(4, 20, 4)
    lo_x, hi_x = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    bn = N.BoundNet(net, 8, 256)
    low, up = bn.spec_bounds(C, None, None, lo_x, hi_x, slack=False)
    for i in range(4):
        close(np_(low)[i], O.spec_lower(net, 1, C[i], [], lo_x[i], hi_x[i], use_slack=False), what="lower")
        close(np_(up)[i], -O.spec_lower(net, 1, -C[i].astype(np.float64), [], lo_x[i], hi_x[i],
                                       use_slack=False), what="upper")


@pytest.mark.parametrize("slack", [True, False])
def test_mlp_small_stagewise_and_end_to_end(mod, slack):
    N, B = mod
    w = W.mlp_small()
    ob = oracle_bounds(w.net, w.x_lo, w.x_hi, slack)
    lo, hi = flat(ob)
    bn = N.BoundNet(w.net, 4, 4096)
    # stage-wise: every target k with the oracle's bounds of the layers below (FP32)
    lo32, hi32 = dev(f32(lo)), dev(f32(hi))
    below = [(l.astype(np.float32).astype(np.float64), u.astype(np.float32).astype(np.float64))
             for (l, u) in ob[0]]
    flags = B.BOUND_BOTH_SIDES | (0 if slack else B.BOUND_NO_SLACK)
    for k in range(1, len(w.net)):
        d = bn.d[k]
        glo = torch.empty(1, d, device="cuda")
        ghi = torch.empty(1, d, device="cuda")
        B.bound_backward(bn.handle, 1, d, k, lo=lo32, hi=hi32, n_bounds=1, x_lo=dev(w.x_lo),
                         x_hi=dev(w.x_hi), flags=flags, lower=glo, upper=ghi)
        I = np.eye(d)
        olo = O.spec_lower(w.net, k, I, below[:k - 1], w.x_lo[0], w.x_hi[0], use_slack=slack)
        ohi = -O.spec_lower(w.net, k, -I, below[:k - 1], w.x_lo[0], w.x_hi[0], use_slack=slack)
        close(np_(glo)[0], olo, what=f"stage lo z{k}")
        close(np_(ghi)[0], ohi, what=f"stage hi z{k}")
    gl, gu = bn.spec_bounds(w.spec, lo32, hi32, w.x_lo, w.x_hi, slack=slack)
    L = len(w.net)
    close(np_(gl)[0], O.spec_lower(w.net, L, w.spec[0], below, w.x_lo[0], w.x_hi[0], use_slack=slack),
          what="stage final lower")
    # end to end
    glo_all, ghi_all = bn.crown_bounds(w.x_lo, w.x_hi, slack=slack)
    close(np_(glo_all), lo, what="e2e lo")
    close(np_(ghi_all), hi, what="e2e hi")
    el, eu = bn.spec_bounds(w.spec, glo_all, ghi_all, w.x_lo, w.x_hi, slack=slack)
    ol = O.spec_lower(w.net, L, w.spec[0], ob[0], w.x_lo[0], w.x_hi[0], use_slack=slack)
    close(np_(el)[0], ol, what="e2e final")


def test_mlp_deep_full_batch_sampled(mod):
    """784-256x6-10, all 256 inputs in one launch; 6 inputs checked against the oracle."""
    N, B = mod
    w = W.mlp_deep(256)
    bn = N.BoundNet(w.net, 256, 256 * 512)
    glo, ghi = bn.crown_bounds(w.x_lo, w.x_hi)
    gl, gu = bn.spec_bounds(w.spec, glo, ghi, w.x_lo, w.x_hi)
    L = len(w.net)
    for i in (0, 1, 77, 128, 200, 255):
        ob = O.crown_bounds(w.net, w.x_lo[i], w.x_hi[i])
        lo, hi = flat([ob])
        close(np_(glo)[i], lo[0], what=f"lo inst {i}")
        close(np_(ghi)[i], hi[0], what=f"hi inst {i}")
        close(np_(gl)[i], O.spec_lower(w.net, L, w.spec[i], ob, w.x_lo[i], w.x_hi[i]), what="final lo")
        close(np_(gu)[i], -O.spec_lower(w.net, L, -w.spec[i].astype(np.float64), ob, w.x_lo[i],
                                        w.x_hi[i]), what="final hi")


CNN_GEOMS = [
    # channel counts 3 / 16 / 32 and power-of-two image sizes take the direct-convolution
    # kernels (LDS-tiled MFMA, VALU for the 3-channel input); the others the implicit GEMM
    dict(H=8, convs=((16, 3, 1), (16, 4, 2), (32, 3, 1)), fc=(16, 5), cin=3),
    dict(H=8, convs=((32, 3, 1), (16, 4, 2), (64, 3, 1)), fc=(10, 4), cin=16),
    dict(H=12, convs=((8, 3, 1), (8, 4, 2), (16, 3, 1), (16, 4, 2)), fc=(32, 5), cin=3),
    dict(H=7, convs=((4, 3, 2), (6, 3, 1)), fc=(10, 3), cin=2),     # odd size, k3 s2
    dict(H=9, convs=((5, 4, 2), (3, 2, 2)), fc=(7,), cin=1),        # k4 s2 on odd, k2 s2
    dict(H=6, convs=((33, 3, 1), (17, 3, 1)), fc=(9, 4), cin=4),    # N not a tile multiple
]


_ORACLE_CACHE = {}


def _cached_crown(key, net, x_lo, x_hi):
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = O.crown_bounds(net, x_lo, x_hi)
    return _ORACLE_CACHE[key]


@pytest.mark.parametrize("path", ["auto", "gemm", "dma"])
@pytest.mark.parametrize("gi", range(len(CNN_GEOMS)))
def test_cnn_small_end_to_end(mod, gi, path):
    N, B = mod
    net = tiny_cnn(seed=10 + gi, **CNN_GEOMS[gi])
    n = 3
    x0 = W.uniform_inputs(n, W.in_dim(net), 20 + gi)
    x_lo, x_hi = W.linf_box(x0, 0.03)
    C = W.margin_spec(W.clean_logits(net, x0))
    bn = N.BoundNet(net, n, 1 << 16)
    if path == "gemm":
        B.bound_set_options(bn.handle, B.BOUND_OPT_GEMM_ONLY)
    elif path == "dma":
        B.bound_set_options(bn.handle, B.BOUND_OPT_DIRECT_DMA)
    glo, ghi = bn.crown_bounds(x_lo, x_hi)
    gl, gu = bn.spec_bounds(C, glo, ghi, x_lo, x_hi)
    L = len(net)
    for i in range(n):
        ob = _cached_crown(("geom", gi, i), net, x_lo[i], x_hi[i])
        lo, hi = flat([ob])
        close(np_(glo)[i], lo[0], what=f"lo {i}")
        close(np_(ghi)[i], hi[0], what=f"hi {i}")
        close(np_(gl)[i], O.spec_lower(net, L, C[i], ob, x_lo[i], x_hi[i]), what="final lo")
        close(np_(gu)[i], -O.spec_lower(net, L, -C[i].astype(np.float64), ob, x_lo[i], x_hi[i]),
              what="final hi")


def test_chunked_passes_match_unchunked(mod):
    N, B = mod
    net = tiny_cnn(seed=31)
    x0 = W.uniform_inputs(5, W.in_dim(net), 32)
    x_lo, x_hi = W.linf_box(x0, 0.02)
    big = N.BoundNet(net, 5, 1 << 16)
    small = N.BoundNet(net, 5, 97)          # forces ragged chunks inside instances
    a = big.crown_bounds(x_lo, x_hi)
    b = small.crown_bounds(x_lo, x_hi)
    # Both runs are FP32 with atomic row sums whose order follows the tile schedule, so
    # they may differ by a few ulps of the summed magnitudes (which exceed the results
    # several-fold); a chunking mistake shows up as an O(1) difference.
    close(np_(b[0]), np_(a[0]), rel=1e-5, what="chunked lo")
    close(np_(b[1]), np_(a[1]), rel=1e-5, what="chunked hi")


def test_coefficients_and_standalone_concretize(mod):
    N, B = mod
    w = W.mlp_small()
    ob = oracle_bounds(w.net, w.x_lo, w.x_hi)
    lo, hi = flat(ob)
    lo32, hi32 = dev(f32(lo)), dev(f32(hi))
    bn = N.BoundNet(w.net, 2, 4096)
    coeff, offset, mag = bn.coefficients(w.spec, lo32, hi32)
    below = [(l.astype(np.float32).astype(np.float64), u.astype(np.float32).astype(np.float64))
             for (l, u) in ob[0]]
    Wt, bt, omag = O.backward(w.net, len(w.net), w.spec[0], below)
    close(np_(coeff), Wt, what="coeff")
    close(np_(offset), bt, what="offset")
    lower = torch.empty(1, 9, device="cuda")
    B.bound_concretize(1, 9, bn.d[0], coeff, offset, mag, dev(w.x_lo), dev(w.x_hi), 0, lower)
    gl, _ = bn.spec_bounds(w.spec, lo32, hi32, w.x_lo, w.x_hi, both=False)
    close(np_(lower), np_(gl), rel=1e-5, what="standalone vs fused")
    ol = O.concretize(Wt, bt, w.x_lo[0], w.x_hi[0]) - O.slack(Wt, omag, w.x_lo[0], w.x_hi[0])
    close(np_(lower)[0], ol, what="standalone vs oracle")


@pytest.mark.parametrize("d0,rows,shift", [(3072, 9, 0), (1001, 13, 0), (1000, 24, 1), (7, 3, 0)])
def test_standalone_concretize_row_groups_and_widths(mod, d0, rows, shift):
    """bound_concretize (one block per instance, rows in groups of twelve) against Theorem 2
    and the allowance in FP64, per row: widths below, at and above the block width, row
    counts with and without a partial last group, buffers shifted by one float."""
    N, B = mod
    rng = np.random.default_rng(301 + d0 + shift)
    n = 3
    G = rng.standard_normal((n, rows, d0)).astype(np.float32)
    off = rng.standard_normal((n, rows)).astype(np.float32)
    mag = rng.random((n, rows)).astype(np.float32)
    x = rng.random((n, d0)).astype(np.float32)
    xl, xh = (x - np.float32(0.02)).astype(np.float32), (x + np.float32(0.02)).astype(np.float32)

    def placed(a):   # the array's data starting `shift` floats into a device buffer
        flat_ = torch.zeros(a.size + shift, device="cuda")
        flat_[shift:] = torch.as_tensor(a.ravel(), device="cuda")
        return flat_[shift:]

    lower = torch.empty(n, rows, device="cuda")
    B.bound_concretize(n, rows, d0, placed(G), dev(off), dev(mag), placed(xl), placed(xh), 0, lower)
    got = np_(lower)
    for i in range(n):
        for r in range(rows):
            g64 = G[i, r].astype(np.float64)
            ref = O.concretize(g64, float(off[i, r]), xl[i], xh[i]) - \
                O.slack(g64, float(mag[i, r]), xl[i], xh[i])
            close(got[i, r], ref, rel=1e-5, what=f"row {i},{r}")


def test_eps_zero_and_first_layer(mod):
    N, B = mod
    net = tiny_cnn(seed=41)
    x0 = W.uniform_inputs(2, W.in_dim(net), 42)
    bn = N.BoundNet(net, 2, 1 << 16)
    glo, ghi = bn.crown_bounds(x0, x0, slack=False)
    zs = O.forward(net, x0)
    off = 0
    for m in range(len(net) - 1):
        d = zs[m].shape[1]
        close(np_(glo)[:, off:off + d], zs[m], what=f"eps0 lo z{m + 1}")
        close(np_(ghi)[:, off:off + d], zs[m], what=f"eps0 hi z{m + 1}")
        off += d


# ------------------------------------------------------------------ alpha / beta
def _random_splits(net, bounds_flat_lo, bounds_flat_hi, n_sub, seed, root_of=None):
    cands = [np.nonzero((l < 0) & (u > 0))[0] for l, u in zip(bounds_flat_lo, bounds_flat_hi)]
    return W.random_splits(cands, n_sub, 1, 12, seed=seed, root_of=root_of)


def _oracle_unit(net, C, lo_row, hi_row, x_lo, x_hi, alpha_row, sp, q0, q1, beta, slack=True):
    """Oracle lower bound (with slack) and raw gradients for one subdomain."""
    bounds = list(zip(O.per_layer(net, lo_row), O.per_layer(net, hi_row)))
    splits = O.split_list(net, sp.neuron[q0:q1], sp.sign[q0:q1])
    al = O.per_layer(net, alpha_row)
    be = None if beta is None else beta[q0:q1]
    L = len(net)
    low = O.spec_lower(net, L, C, bounds, x_lo, x_hi, al, splits, be, use_slack=slack)
    _, ga, gb = O.spec_lower_grad(net, L, C, bounds, x_lo, x_hi, al, splits,
                                  np.zeros((q1 - q0, C.shape[0])) if be is None else be)
    return low, np.concatenate(ga), gb


@pytest.mark.parametrize("kind", ["mlp", "mlp_wide", "cnn", "cnn_direct", "cnn_direct_gemm",
                                  "cnn_direct_dma"])
def test_alpha_beta_pass_and_grad(mod, kind):
    N, B = mod
    if kind == "mlp":
        net = W.mlp([30, 24, 24, 24, 6], seed=51)
    elif kind == "mlp_wide":
        # a ReLU layer wider than 256 x 64 neurons: each thread of the slot numbering
        # walks more than one 64-neuron flag mask
        net = W.mlp([10, 17000, 6], seed=58)
    elif kind == "cnn":
        net = tiny_cnn(seed=52)
    else:
        net = tiny_cnn(seed=57, **CNN_GEOMS[0])
    n_roots, per_root = 2, 6
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), 53)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    ob = oracle_bounds(net, x_lo, x_hi)
    lo, hi = flat(ob)
    lo, hi = f32(lo).astype(np.float64), f32(hi).astype(np.float64)
    n = n_roots * per_root
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    sp = _random_splits(net, lo, hi, n, 54, root_of)
    n_relu = lo.shape[1]
    alpha = W.random_alpha(n, n_relu, 55)
    beta = W.random_beta(sp.nnz, C.shape[1], 56)
    Cs = C[root_of]
    bn = N.BoundNet(net, n, 4096, 4096)
    if kind.endswith("_gemm"):
        B.bound_set_options(bn.handle, B.BOUND_OPT_GEMM_ONLY)
    elif kind.endswith("_dma"):
        B.bound_set_options(bn.handle, B.BOUND_OPT_DIRECT_DMA)
    spd = N.splits_to_device(sp)
    gl, _ = bn.spec_bounds(Cs, dev(f32(lo)), dev(f32(hi)), x_lo[root_of], x_hi[root_of],
                           alpha=dev(alpha), bound_of=dev(root_of, torch.int32), splits=spd,
                           beta=dev(beta), both=False, save=True)
    ga, gb = bn.grad(torch.ones(n, C.shape[1], device="cuda"), sp.nnz)
    ga, gb = np_(ga), np_(gb)
    for i in range(n):
        r = root_of[i]
        q0, q1 = sp.off[i], sp.off[i + 1]
        low, oga, ogb = _oracle_unit(net, C[r], lo[r], hi[r], x_lo[r], x_hi[r], alpha[i], sp, q0, q1,
                                     beta.astype(np.float64))
        close(np_(gl)[i], low, what=f"lower {i}")
        scale = max(np.max(np.abs(oga)), 1e-30)
        assert np.max(np.abs(ga[i] - oga)) <= 1e-4 * scale, f"grad alpha {i}"
        if q1 > q0:
            sb = max(np.max(np.abs(ogb)), 1e-30)
            assert np.max(np.abs(gb[q0:q1] - ogb)) <= 1e-4 * max(sb, scale), f"grad beta {i}"


@pytest.mark.parametrize("kind", ["mlp", "cnn"])
def test_repeated_split_entries_bound_and_grad(mod, kind):
    """A neuron split twice with the same sign: each entry has its own beta; the bound and
    both entries' beta-gradients match the oracle (the later entry's gradient is the one
    the separate beta-gradient kernel computes)."""
    N, B = mod
    net = W.mlp([30, 24, 24, 24, 6], seed=141) if kind == "mlp" else tiny_cnn(seed=142)
    n_roots, per_root = 2, 3
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), 143)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    ob = oracle_bounds(net, x_lo, x_hi)
    lo, hi = flat(ob)
    lo, hi = f32(lo).astype(np.float64), f32(hi).astype(np.float64)
    n = n_roots * per_root
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    base = _random_splits(net, lo, hi, n, 144, root_of)
    off, neu, sg = [0], [], []
    for i in range(n):          # every subdomain repeats its first entry at the end
        q0, q1 = base.off[i], base.off[i + 1]
        neu += list(base.neuron[q0:q1]) + [base.neuron[q0]]
        sg += list(base.sign[q0:q1]) + [base.sign[q0]]
        off.append(len(neu))
    sp = W.Splits(np.array(off, np.int32), np.array(neu, np.int32), np.array(sg, np.int8))
    n_relu = lo.shape[1]
    alpha = W.random_alpha(n, n_relu, 145)
    beta = W.random_beta(sp.nnz, C.shape[1], 146)
    bn = N.BoundNet(net, n, 4096, 4096)
    gl, _ = bn.spec_bounds(C[root_of], dev(f32(lo)), dev(f32(hi)), x_lo[root_of], x_hi[root_of],
                           alpha=dev(alpha), bound_of=dev(root_of, torch.int32),
                           splits=N.splits_to_device(sp), beta=dev(beta), both=False, save=True)
    ga, gb = bn.grad(torch.ones(n, C.shape[1], device="cuda"), sp.nnz)
    ga, gb = np_(ga), np_(gb)
    for i in range(n):
        r = root_of[i]
        q0, q1 = sp.off[i], sp.off[i + 1]
        low, oga, ogb = _oracle_unit(net, C[r], lo[r], hi[r], x_lo[r], x_hi[r], alpha[i], sp, q0,
                                     q1, beta.astype(np.float64))
        close(np_(gl)[i], low, what=f"lower {i}")
        scale = max(np.max(np.abs(oga)), 1e-30)
        assert np.max(np.abs(ga[i] - oga)) <= 1e-4 * scale, f"grad alpha {i}"
        sb = max(np.max(np.abs(ogb)), scale, 1e-30)
        assert np.max(np.abs(gb[q0:q1] - ogb)) <= 1e-4 * sb, f"grad beta {i}"
        assert np.array_equal(ogb[0], ogb[-1])      # the oracle gives both entries one gradient


def test_infeasible_split_gives_inf(mod):
    N, B = mod
    net = W.mlp([10, 12, 12, 3], seed=61)
    x0 = W.uniform_inputs(1, 10, 62)
    x_lo, x_hi = W.linf_box(x0, 0.1)
    ob = oracle_bounds(net, x_lo, x_hi)
    lo, hi = flat(ob)
    j = int(np.argmin(hi[0]))
    assert hi[0, j] < 0
    sp = W.Splits(np.array([0, 1, 2], np.int32), np.array([j, j], np.int32),
                  np.array([1, -1], np.int8))   # instance 0: infeasible; instance 1: consistent
    bn = N.BoundNet(net, 2, 256, 256)
    C = np.eye(3)[None].repeat(2, 0)
    gl, _ = bn.spec_bounds(C, dev(f32(lo)), dev(f32(hi)), np.repeat(x_lo, 2, 0), np.repeat(x_hi, 2, 0),
                           bound_of=dev(np.zeros(2), torch.int32), splits=N.splits_to_device(sp),
                           both=False, save=True)
    g = np_(gl)
    assert np.all(np.isinf(g[0])) and np.all(g[0] > 0)
    assert np.all(np.isfinite(g[1]))
    ga, _ = bn.grad(torch.ones(2, 3, device="cuda"), 2)
    assert np.all(np_(ga)[0] == 0)


@pytest.mark.parametrize("n", [1000, 1001])  # and a length that is not a multiple of four
def test_adam_kernel(mod, n):
    N, B = mod
    rng = np.random.default_rng(71)
    p0 = rng.uniform(0, 1, n)
    p, m, v = dev(p0), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    op, om, ov = p0.astype(np.float32).astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = rng.normal(size=n)
        B.bound_adam(p, dev(g), m, v, t, 0.1, grad_scale=-1.0, clip_lo=0.0, clip_hi=1.0)
        op, om, ov = O.adam_step(op, -g.astype(np.float32).astype(np.float64), om, ov, t, 0.1,
                                 lo=0.0, hi=1.0)
    close(np_(p), op, rel=1e-5, what="adam")


def test_optimisation_loop_improves_and_first_step_matches(mod):
    N, B = mod
    net = tiny_cnn(seed=81)
    n_roots, per_root = 2, 4
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), 82)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    ob = oracle_bounds(net, x_lo, x_hi)
    lo, hi = flat(ob)
    lo, hi = f32(lo).astype(np.float64), f32(hi).astype(np.float64)
    n = n_roots * per_root
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    sp = _random_splits(net, lo, hi, n, 83, root_of)
    bn = N.BoundNet(net, n, 4096, 4096)
    steps = []
    best, alpha, beta = N.optimize_alpha_beta(bn, C[root_of], dev(f32(lo)), dev(f32(hi)), x_lo[root_of],
                                              x_hi[root_of], steps=10, lr=0.1,
                                              bound_of=dev(root_of, torch.int32),
                                              splits=N.splits_to_device(sp), lower_of_step=steps)
    first = np_(steps[0])
    for i in range(n):
        r = root_of[i]
        q0, q1 = sp.off[i], sp.off[i + 1]
        a0 = np.full(lo.shape[1], 0.5)
        low, _, _ = _oracle_unit(net, C[r], lo[r], hi[r], x_lo[r], x_hi[r], a0, sp, q0, q1,
                                 np.zeros((sp.nnz, C.shape[1])))
        close(first[i], low, what=f"step-1 bound {i}")
    b = np_(best)
    assert np.all(b >= first - 1e-6)
    assert np.mean(b - first) > 0
    al = np_(alpha)
    assert al.min() >= 0 and al.max() <= 1
    if beta is not None:
        assert np_(beta).min() >= 0


@pytest.mark.parametrize("dims,seed", [([12, 32, 32, 4], 221), ([8, 24, 24, 24, 3], 223)])
def test_optimiser_trajectory_three_steps_matches_oracle(mod, dims, seed):
    """Three projected-Adam steps on alpha and beta (GPU: bound pass, gradient, Adam) from
    the same start and the same intermediate bounds as the oracle's optimisation: the
    best bound after the steps agrees to 1e-4.  (Entries whose gradient is zero up to
    rounding may step in different directions on the two sides, which moves the bound by
    no more than that gradient; the bound is what is compared.)"""
    N, B = mod
    net = W.mlp(dims, seed=seed)
    n_roots, per_root = 2, 3
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), seed + 1)
    x_lo, x_hi = W.linf_box(x0, 0.1)
    C = W.margin_spec(W.clean_logits(net, x0))
    ob = oracle_bounds(net, x_lo, x_hi)
    lo, hi = flat(ob)
    lo, hi = f32(lo).astype(np.float64), f32(hi).astype(np.float64)
    n = n_roots * per_root
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    sp = _random_splits(net, lo, hi, n, seed + 2, root_of)
    bn = N.BoundNet(net, n, 4096, 4096)
    best, _, _ = N.optimize_alpha_beta(bn, C[root_of], dev(f32(lo)), dev(f32(hi)), x_lo[root_of],
                                       x_hi[root_of], steps=3, lr=0.1,
                                       bound_of=dev(root_of, torch.int32),
                                       splits=N.splits_to_device(sp))
    got = np_(best)
    for i in range(n):
        r = root_of[i]
        q0, q1 = sp.off[i], sp.off[i + 1]
        bounds = list(zip(O.per_layer(net, lo[r]), O.per_layer(net, hi[r])))
        splits = O.split_list(net, sp.neuron[q0:q1], sp.sign[q0:q1])
        ref, _, _ = O.optimize_alpha_beta(net, C[r], bounds, x_lo[r], x_hi[r], splits, steps=3,
                                          lr=0.1)
        close(got[i], ref, rel=1e-4, what=f"best bound after 3 steps, subdomain {i}")


# -------------------------------------------------------------------------- soundness
@pytest.mark.parametrize("dims,seed", [([2, 8, 8, 3], 91), ([2, 16, 16, 16, 2], 92), ([2, 12, 3], 93)])
def test_soundness_tiny_2d(mod, dims, seed):
    N, B = mod
    net = W.mlp(dims, seed=seed)
    x_lo = np.array([[-1.0, -0.5]], np.float32)
    x_hi = np.array([[0.5, 1.0]], np.float32)
    rng = np.random.default_rng(seed)
    pts = np.concatenate([x_lo + (x_hi - x_lo) * rng.uniform(0, 1, (100_000, 2)),
                          np.stack(np.meshgrid(np.linspace(-1, 0.5, 317), np.linspace(-0.5, 1, 317),
                                               indexing="ij"), -1).reshape(-1, 2)])
    zs = O.forward(net, pts)
    bn = N.BoundNet(net, 64, 4096, 4096)
    glo, ghi = bn.crown_bounds(x_lo, x_hi)
    lo_np, hi_np = np_(glo)[0], np_(ghi)[0]
    off = 0
    for m in range(len(net) - 1):
        d = zs[m].shape[1]
        assert np.all(zs[m] >= lo_np[off:off + d]) and np.all(zs[m] <= hi_np[off:off + d])
        off += d
    k = dims[-1]
    C = np.concatenate([np.eye(k), -np.eye(k)])[None]
    f = zs[-1] @ C[0].T
    # random alpha, beta and splits over many subdomains at once
    n = 48
    unst = np.nonzero((lo_np < 0) & (hi_np > 0))[0]
    sp = W.random_splits([unst], n, 1, min(4, len(unst)), seed=seed)
    alpha = W.random_alpha(n, lo_np.size, seed + 1)
    beta = W.random_beta(sp.nnz, C.shape[1], seed + 2, scale=2.0)
    gl, _ = bn.spec_bounds(np.repeat(C, n, 0), glo, ghi, np.repeat(x_lo, n, 0), np.repeat(x_hi, n, 0),
                           alpha=dev(alpha), bound_of=dev(np.zeros(n), torch.int32),
                           splits=N.splits_to_device(sp), beta=dev(beta), both=False)
    g = np_(gl)
    checked = 0
    for i in range(n):
        feas = np.ones(len(pts), bool)
        for q in range(sp.off[i], sp.off[i + 1]):
            gidx, sg = int(sp.neuron[q]), int(sp.sign[q])
            m = int(np.searchsorted(np.cumsum([zz.shape[1] for zz in zs[:-1]]), gidx, side="right"))
            j = gidx - int(np.sum([zz.shape[1] for zz in zs[:m]]))
            feas &= sg * zs[m][:, j] >= 0
        if feas.sum() == 0:
            continue
        assert np.all(f[feas].min(axis=0) >= g[i]), f"unsound subdomain {i}"
        checked += 1
    assert checked >= 10


# ------------------------------------------------------------- full-size workloads
@pytest.fixture(scope="module")
def golden_cnn():
    path = os.path.join(GOLDEN, "cnn_root0.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/cnn_root0.npz missing (run tests/golden/make_cnn_root.py)")
    return dict(np.load(path))


def test_cnn_full_batch_against_golden(mod, golden_cnn):
    """3x32x32 CNN, 64 inputs in one full-CROWN launch; input 0 against the stored oracle."""
    N, B = mod
    w = W.cnn_cifar(64)
    bn = N.BoundNet(w.net, 64, 36864)
    glo, ghi = bn.crown_bounds(w.x_lo, w.x_hi)
    gl, gu = bn.spec_bounds(w.spec, glo, ghi, w.x_lo, w.x_hi)
    lo0, hi0 = np_(glo)[0], np_(ghi)[0]
    flips = int(np.sum(((lo0 < 0) & (hi0 > 0)) != ((golden_cnn["lo"] < 0) & (golden_cnn["hi"] > 0))))
    print(f"stability flips vs oracle: {flips}")
    close(lo0, golden_cnn["lo"], what="e2e lo")
    close(hi0, golden_cnn["hi"], what="e2e hi")
    close(np_(gl)[0], golden_cnn["lower"], what="e2e final lower")
    close(np_(gu)[0], golden_cnn["upper"], what="e2e final upper")
    # stage-wise final pass from the oracle's bounds
    lo32 = dev(f32(golden_cnn["lo"])[None])
    hi32 = dev(f32(golden_cnn["hi"])[None])
    sl, su = bn.spec_bounds(w.spec[:1], lo32, hi32, w.x_lo[:1], w.x_hi[:1])
    b64 = list(zip(O.per_layer(w.net, f32(golden_cnn["lo"]).astype(np.float64)),
                   O.per_layer(w.net, f32(golden_cnn["hi"]).astype(np.float64))))
    close(np_(sl)[0], O.spec_lower(w.net, len(w.net), w.spec[0], b64, w.x_lo[0], w.x_hi[0]),
          what="stage final")


def test_beta_crown_batch_full_size(mod, golden_cnn):
    """4096 subdomains x 9 rows with 1-12 splits, random alpha / beta, one pass + gradient
    (the bench's launch); 6 subdomains against the oracle."""
    N, B = mod
    w = W.cnn_cifar(1)
    lo = f32(golden_cnn["lo"]).astype(np.float64)
    hi = f32(golden_cnn["hi"]).astype(np.float64)
    n = 4096
    root_of = np.zeros(n, np.int32)
    sp = W.random_splits([np.nonzero((lo < 0) & (hi > 0))[0]], n, 1, 12, seed=2, root_of=root_of)
    n_relu = lo.size
    alpha = W.random_alpha(n, n_relu, 3)
    beta = W.random_beta(sp.nnz, 9, 4)
    bn = N.BoundNet(w.net, n, n * 9, n * 9)
    Cs = np.repeat(w.spec, n, 0)
    gl, _ = bn.spec_bounds(Cs, dev(f32(lo)[None]), dev(f32(hi)[None]), np.repeat(w.x_lo, n, 0),
                           np.repeat(w.x_hi, n, 0), alpha=dev(alpha), bound_of=dev(root_of, torch.int32),
                           splits=N.splits_to_device(sp), beta=dev(beta), both=False, save=True)
    ga, gb = bn.grad(torch.ones(n, 9, device="cuda"), sp.nnz)
    gl, ga, gb = np_(gl), np_(ga), np_(gb)
    for i in (0, 1, 1000, 2047, 3001, 4095):
        q0, q1 = sp.off[i], sp.off[i + 1]
        low, oga, ogb = _oracle_unit(w.net, w.spec[0], lo, hi, w.x_lo[0], w.x_hi[0], alpha[i], sp,
                                     q0, q1, beta.astype(np.float64))
        close(gl[i], low, what=f"lower {i}")
        scale = np.max(np.abs(oga))
        assert np.max(np.abs(ga[i] - oga)) <= 1e-4 * scale, f"grad alpha {i}"
        sb = max(np.max(np.abs(ogb)), scale)
        assert np.max(np.abs(gb[q0:q1] - ogb)) <= 1e-4 * sb, f"grad beta {i}"


def test_ragged_batch_one_launch_vs_chunked(mod, golden_cnn):
    """1023 subdomains (9207 imgs, so image groups of the direct kernels and GEMM row
    tiles end part-way): one launch per layer against the same pass cut into launches
    of 1500 imgs (cutting instances); pass and gradient of three subdomains against the
    oracle."""
    N, B = mod
    w = W.cnn_cifar(1)
    lo = f32(golden_cnn["lo"]).astype(np.float64)
    hi = f32(golden_cnn["hi"]).astype(np.float64)
    n = 1023
    root_of = np.zeros(n, np.int32)
    sp = W.random_splits([np.nonzero((lo < 0) & (hi > 0))[0]], n, 1, 12, seed=8, root_of=root_of)
    alpha = W.random_alpha(n, lo.size, 9)
    beta = W.random_beta(sp.nnz, 9, 10)
    res = []
    for rows, save in ((n * 9, n * 9), (1500, 0)):
        bn = N.BoundNet(w.net, n, rows, save)
        gl, _ = bn.spec_bounds(np.repeat(w.spec, n, 0), dev(f32(lo)[None]), dev(f32(hi)[None]),
                               np.repeat(w.x_lo, n, 0), np.repeat(w.x_hi, n, 0), alpha=dev(alpha),
                               bound_of=dev(root_of, torch.int32), splits=N.splits_to_device(sp),
                               beta=dev(beta), both=False, save=save > 0)
        if save:
            ga, gb = bn.grad(torch.ones(n, 9, device="cuda"), sp.nnz)
            ga, gb = np_(ga), np_(gb)
        res.append(np_(gl))
        del bn
    # same tiles and k order; only the order of the atomic row sums differs
    close(res[0], res[1], rel=1e-5, what="lower grouped vs chunked")
    gl = res[0]
    for i in (0, 511, n - 1):
        q0, q1 = sp.off[i], sp.off[i + 1]
        low, oga, ogb = _oracle_unit(w.net, w.spec[0], lo, hi, w.x_lo[0], w.x_hi[0], alpha[i], sp,
                                     q0, q1, beta.astype(np.float64))
        close(gl[i], low, what=f"lower {i}")
        scale = np.max(np.abs(oga))
        assert np.max(np.abs(ga[i] - oga)) <= 1e-4 * scale, f"grad alpha {i}"
        sb = max(np.max(np.abs(ogb)), scale)
        assert np.max(np.abs(gb[q0:q1] - ogb)) <= 1e-4 * sb, f"grad beta {i}"


def test_direct_and_gemm_paths_agree_full_size(mod, golden_cnn):
    """The 4096-subdomain pass + gradient through the kernel paths (direct convolution with
    register or LDS DMA staging, implicit GEMM) on the same inputs."""
    N, B = mod
    w = W.cnn_cifar(1)
    lo = f32(golden_cnn["lo"])[None]
    hi = f32(golden_cnn["hi"])[None]
    n = 4096
    root_of = np.zeros(n, np.int32)
    sp = W.random_splits([np.nonzero((lo[0] < 0) & (hi[0] > 0))[0]], n, 1, 12, seed=5,
                         root_of=root_of)
    alpha = dev(W.random_alpha(n, lo.shape[1], 6))
    beta = dev(W.random_beta(sp.nnz, 9, 7))
    bn = N.BoundNet(w.net, n, n * 9, n * 9)
    out = []
    for opt in (0, B.BOUND_OPT_GEMM_ONLY, B.BOUND_OPT_DIRECT_DMA):
        B.bound_set_options(bn.handle, opt)
        gl, _ = bn.spec_bounds(np.repeat(w.spec, n, 0), dev(lo), dev(hi), np.repeat(w.x_lo, n, 0),
                               np.repeat(w.x_hi, n, 0), alpha=alpha, bound_of=dev(root_of, torch.int32),
                               splits=N.splits_to_device(sp), beta=beta, both=False, save=True)
        ga, gb = bn.grad(torch.ones(n, 9, device="cuda"), sp.nnz)
        out.append((np_(gl), np_(ga), np_(gb)))
    # Both paths round differently; where a coefficient lies within rounding of zero the
    # relaxation branch (and its adjoint mask) can flip, so a few gradient entries may
    # differ by more than rounding.  Bounds: rounding only; gradients: almost all
    # entries to 1e-5, none beyond 1e-3 of the instance's largest entry.
    close(out[0][0], out[1][0], rel=1e-5, what="lower direct vs gemm")
    da = np.abs(out[0][1] - out[1][1])
    sa = np.maximum(np.max(np.abs(out[1][1]), axis=1, keepdims=True), 1e-30)
    db = np.abs(out[0][2] - out[1][2])
    sb = max(np.max(np.abs(out[1][2])), 1e-30)
    print(f"alpha-grad entries off by >1e-5: {np.mean(da > 1e-5 * sa):.2e}; "
          f"beta-grad: {np.mean(db > 1e-5 * sb):.2e}; worst {np.max(da / sa):.2e} / {np.max(db) / sb:.2e}")
    assert np.mean(da > 1e-5 * sa) <= 1e-4 and np.max(da / sa) <= 1e-3
    assert np.mean(db > 1e-5 * sb) <= 1e-3 and np.max(db) / sb <= 1e-3
    # tiles staged by LDS DMA: the same products (the channel chunking, and with it the
    # summation order, may differ), same criteria against the register-staged kernels
    close(out[2][0], out[0][0], rel=1e-5, what="lower dma vs registers")
    da = np.abs(out[2][1] - out[0][1])
    db = np.abs(out[2][2] - out[0][2])
    assert np.mean(da > 1e-5 * sa) <= 1e-4 and np.max(da / sa) <= 1e-3
    assert np.mean(db > 1e-5 * sb) <= 1e-3 and np.max(db) / sb <= 1e-3


def test_graph_captured_optimisation_matches_eager(mod):
    """The whole 10-step alpha/beta optimisation captured as one HIP graph: every replay,
    with eager work and synchronisations in between, equals the eager run."""
    N, B = mod
    net = tiny_cnn(seed=91, **CNN_GEOMS[0])
    n_roots, per_root = 2, 24
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), 92)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    bn = N.BoundNet(net, n_roots * per_root, 1 << 14, 1 << 12)
    glo, ghi = bn.crown_bounds(x_lo, x_hi)
    lo_np, hi_np = np_(glo), np_(ghi)
    n = n_roots * per_root
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    sp = _random_splits(net, lo_np, hi_np, n, 93, root_of)
    opt = N.AlphaBetaOptimizer(bn, C[root_of], glo, ghi, x_lo[root_of], x_hi[root_of],
                               bound_of=dev(root_of, torch.int32), splits=N.splits_to_device(sp),
                               steps=10)
    eager = np_(opt.run()).copy()
    ea, eb = np_(opt.alpha).copy(), np_(opt.beta).copy()
    # float atomics make two eager runs differ in the last bits; replays are held to the
    # parity tolerance (a wrong replay is off by far more)
    eager2 = np_(opt.run()).copy()
    close(eager2, eager, rel=1e-4, what="eager vs eager")
    opt.capture()
    for rep in range(3):
        opt.alpha.fill_(0.123)           # eager work between replays
        opt.best.fill_(7.0)
        torch.cuda.synchronize()
        got = np_(opt.replay()).copy()
        torch.cuda.synchronize()
        close(got, eager, rel=1e-4, what=f"replay {rep} best bound")
        np.testing.assert_allclose(np_(opt.alpha), ea, atol=2e-3)
        np.testing.assert_allclose(np_(opt.beta), eb, atol=2e-3, rtol=1e-3)
        bn.crown_bounds(x_lo, x_hi)      # an unrelated eager pass on the same handle


def test_autotuned_plans_keep_the_bound(mod):
    """After bound_autotune picks a kernel per product, pass and gradient are unchanged
    (to rounding) and the timing log covers every product."""
    N, B = mod
    net = tiny_cnn(seed=95, **CNN_GEOMS[0])
    n = 64
    x0 = W.uniform_inputs(1, W.in_dim(net), 96)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    bn = N.BoundNet(net, n, 1 << 14, 1 << 14)
    glo, ghi = bn.crown_bounds(x_lo, x_hi)
    lo_np, hi_np = np_(glo), np_(ghi)
    sp = _random_splits(net, lo_np, hi_np, n, 97, np.zeros(n, np.int32))
    spd = N.splits_to_device(sp)
    alpha = dev(W.random_alpha(n, bn.n_relu, 98))
    beta = dev(W.random_beta(sp.nnz, C.shape[1], 99))
    args = (np.repeat(C, n, 0), glo, ghi, np.repeat(x_lo, n, 0), np.repeat(x_hi, n, 0))
    kw = dict(alpha=alpha, bound_of=dev(np.zeros(n), torch.int32), splits=spd, beta=beta,
              both=False, save=True)
    l0, _ = bn.spec_bounds(*args, **kw)
    g0 = bn.grad(torch.ones(n, C.shape[1], device="cuda"), sp.nnz)
    ref = (np_(l0), np_(g0[0]), np_(g0[1]))
    lower = torch.empty(n, C.shape[1], device="cuda")
    log = B.bound_autotune(bn.handle, n, C.shape[1], len(net), grad_lower=torch.ones(n, C.shape[1], device="cuda"),
                           spec=dev(np.repeat(C, n, 0)), lo=glo, hi=ghi, n_bounds=1,
                           bound_of=dev(np.zeros(n), torch.int32), alpha=alpha,
                           split_off=spd["off"], split_idx=spd["idx"], split_sign=spd["sign"],
                           nnz=sp.nnz, beta=beta, x_lo=dev(np.repeat(x_lo, n, 0)),
                           x_hi=dev(np.repeat(x_hi, n, 0)), flags=B.BOUND_SAVE_FOR_GRAD, lower=lower)
    keys = {line.split()[0] for line in log.strip().splitlines()}
    assert {f"R{m}" for m in range(2, len(net) + 1)} <= keys and "C1" in keys
    assert {f"A{m}" for m in range(1, len(net))} <= keys
    close(np_(lower), ref[0], rel=1e-5, what="autotune call output")
    l1, _ = bn.spec_bounds(*args, **kw)
    g1 = bn.grad(torch.ones(n, C.shape[1], device="cuda"), sp.nnz)
    close(np_(l1), ref[0], rel=1e-5, what="tuned lower")
    s = np.max(np.abs(ref[1]), axis=1, keepdims=True) + 1e-30
    assert np.mean(np.abs(np_(g1[0]) - ref[1]) > 1e-5 * s) <= 1e-3
    # the chosen plans pinned on a fresh handle run the same kernels: the same results up
    # to the order of the atomic row sums
    best = {}
    for line in log.strip().splitlines():
        key, path, cfg, cc, ms, _ = line.split()
        if key not in best or float(ms) < best[key][0]:
            best[key] = (float(ms), path, int(cfg.split("=")[1]), int(cc.split("=")[1]))
    bn2 = N.BoundNet(net, n, 1 << 14, 1 << 14)
    for key, (_, path, cfg, cc) in best.items():
        B.bound_set_plan(bn2.handle, key[0], int(key[1:]), 1 if path == "direct" else 2, cfg, cc)
    l2, _ = bn2.spec_bounds(*args, **kw)
    g2 = bn2.grad(torch.ones(n, C.shape[1], device="cuda"), sp.nnz)
    close(np_(l2), np_(l1), rel=1e-6, what="pinned lower")
    np.testing.assert_allclose(np_(g2[0]), np_(g1[0]), rtol=1e-5, atol=1e-6 * float(np.max(s)))
    np.testing.assert_allclose(np_(g2[1]), np_(g1[1]), rtol=1e-5, atol=1e-6)


def test_alpha_crown_cnn_64_instances(mod, golden_cnn):
    """alpha-CROWN on the CNN (64 instances, random alpha in [0, 1]): the bound and its
    alpha-gradient at identical alpha, 4 instances against the oracle; then 20 Adam steps
    (lr 0.1, alpha0 = 0.5) never lower the best bound."""
    N, B = mod
    w = W.cnn_cifar(1)
    lo = f32(golden_cnn["lo"]).astype(np.float64)
    hi = f32(golden_cnn["hi"]).astype(np.float64)
    n = 64
    alpha = W.random_alpha(n, lo.size, 11)
    bn = N.BoundNet(w.net, n, n * 9, n * 9)
    args = (np.repeat(w.spec, n, 0), dev(f32(lo)[None]), dev(f32(hi)[None]), np.repeat(w.x_lo, n, 0),
            np.repeat(w.x_hi, n, 0))
    gl, _ = bn.spec_bounds(*args, alpha=dev(alpha), bound_of=dev(np.zeros(n), torch.int32),
                           both=False, save=True)
    ga, _ = bn.grad(torch.ones(n, 9, device="cuda"))
    gl, ga = np_(gl), np_(ga)
    bounds = list(zip(O.per_layer(w.net, lo), O.per_layer(w.net, hi)))
    for i in (0, 21, 42, 63):
        al = O.per_layer(w.net, alpha[i])
        ol = O.spec_lower(w.net, len(w.net), w.spec[0], bounds, w.x_lo[0], w.x_hi[0], al)
        _, oga, _ = O.spec_lower_grad(w.net, len(w.net), w.spec[0], bounds, w.x_lo[0], w.x_hi[0], al)
        oga = np.concatenate(oga)
        close(gl[i], ol, what=f"alpha-CROWN lower {i}")
        assert np.max(np.abs(ga[i] - oga)) <= 1e-4 * np.max(np.abs(oga)), f"alpha grad {i}"
    steps = []
    best, a, _ = N.optimize_alpha_beta(bn, *args[:1], args[1], args[2], args[3], args[4], steps=20,
                                       lr=0.1, bound_of=dev(np.zeros(n), torch.int32),
                                       lower_of_step=steps)
    b, first = np_(best), np_(steps[0])
    assert np.all(b >= first - 1e-6) and np.mean(b - first) > 0
    assert 0.0 <= np_(a).min() and np_(a).max() <= 1.0


@pytest.mark.parametrize("mode", ["relu", "linear"])
@pytest.mark.parametrize("kind", ["mlp", "cnn"])
def test_early_stop_pass_and_grad(mod, mode, kind):
    """Propagation early stop at every layer: bound and alpha/beta gradients at identical
    alpha / beta against the oracle (splits clamp the stop node's box too)."""
    N, B = mod
    net = W.mlp([30, 24, 24, 24, 6], seed=131) if kind == "mlp" else tiny_cnn(seed=132, **CNN_GEOMS[0])
    n_roots, per_root = 2, 5
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), 133)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    ob = oracle_bounds(net, x_lo, x_hi)
    lo, hi = flat(ob)
    lo, hi = f32(lo).astype(np.float64), f32(hi).astype(np.float64)
    n = n_roots * per_root
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    sp = _random_splits(net, lo, hi, n, 134, root_of)
    alpha = W.random_alpha(n, lo.shape[1], 135)
    beta = W.random_beta(sp.nnz, C.shape[1], 136)
    bn = N.BoundNet(net, n, 4096, 4096)
    sm = B.BOUND_STOP_RELU if mode == "relu" else B.BOUND_STOP_LINEAR
    L = len(net)
    for stop in range(1, L):
        gl, _ = bn.spec_bounds(C[root_of], dev(f32(lo)), dev(f32(hi)), x_lo[root_of], x_hi[root_of],
                               alpha=dev(alpha), bound_of=dev(root_of, torch.int32),
                               splits=N.splits_to_device(sp), beta=dev(beta), both=False, save=True,
                               stop_layer=stop, stop_mode=sm)
        ga, gb = bn.grad(torch.ones(n, C.shape[1], device="cuda"), sp.nnz)
        gl, ga, gb = np_(gl), np_(ga), np_(gb)
        for i in range(n):
            r = root_of[i]
            q0, q1 = sp.off[i], sp.off[i + 1]
            bounds = list(zip(O.per_layer(net, lo[r]), O.per_layer(net, hi[r])))
            splits = O.split_list(net, sp.neuron[q0:q1], sp.sign[q0:q1])
            al = O.per_layer(net, alpha[i])
            be = beta[q0:q1].astype(np.float64)
            ol = O.spec_lower_early_stop(net, L, C[r], bounds, stop, mode, al, splits, be)
            close(gl[i], ol, what=f"stop {stop} lower {i}")
            if np.all(np.isinf(ol)):
                continue
            _, oga, ogb = O.spec_lower_grad(net, L, C[r], bounds, x_lo[r], x_hi[r], al, splits, be,
                                            stop=stop, mode=mode)
            oga = np.concatenate(oga)
            sa = max(np.max(np.abs(oga)), 1e-30)
            assert np.max(np.abs(ga[i] - oga)) <= 1e-4 * sa, f"stop {stop} alpha grad {i}"
            if q1 > q0:
                sb = max(np.max(np.abs(ogb)), sa)
                assert np.max(np.abs(gb[q0:q1] - ogb)) <= 1e-4 * sb, f"stop {stop} beta grad {i}"


@pytest.mark.parametrize("kind", ["mlp", "cnn"])
def test_sample_bounds_and_early_stop_over_them(mod, kind):
    """Search-integrated bounds (min / max over each subdomain's samples) against the
    oracle's forward pass; then an early-stop pass over (oracle) empirical bounds."""
    N, B = mod
    net = W.mlp([30, 24, 24, 24, 6], seed=151) if kind == "mlp" else tiny_cnn(seed=152, **CNN_GEOMS[0])
    n_sub, per = 6, 40
    x0 = W.uniform_inputs(n_sub, W.in_dim(net), 153)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    rng = np.random.default_rng(154)
    samples = (x_lo[:, None, :] + (x_hi - x_lo)[:, None, :] *
               rng.uniform(0, 1, (n_sub, per, x_lo.shape[1]))).astype(np.float32)
    bn = N.BoundNet(net, n_sub, 4096, 1024)
    lo = torch.empty(n_sub, bn.n_relu, device="cuda")
    hi = torch.empty_like(lo)
    out = torch.empty(n_sub * per, bn.d[-1], device="cuda")
    B.bound_sample_bounds(bn.handle, n_sub, per, dev(samples.reshape(n_sub * per, -1)), lo, hi, out)
    emp = []
    for i in range(n_sub):
        eb = O.sample_bounds(net, samples[i].astype(np.float64))
        e_lo = np.concatenate([b[0] for b in eb])
        e_hi = np.concatenate([b[1] for b in eb])
        close(np_(lo)[i], e_lo, what=f"sample lo {i}")
        close(np_(hi)[i], e_hi, what=f"sample hi {i}")
        close(np_(out)[i * per:(i + 1) * per], O.forward(net, samples[i])[-1], what="outputs")
        emp.append((e_lo, e_hi))
    e_lo = f32(np.stack([e[0] for e in emp])).astype(np.float64)
    e_hi = f32(np.stack([e[1] for e in emp])).astype(np.float64)
    C = W.margin_spec(W.clean_logits(net, x0))
    L = len(net)
    for mode, sm in (("relu", B.BOUND_STOP_RELU), ("linear", B.BOUND_STOP_LINEAR)):
        gl, _ = bn.spec_bounds(C, dev(f32(e_lo)), dev(f32(e_hi)), x_lo, x_hi, both=False,
                               stop_layer=L - 1, stop_mode=sm)
        for i in range(n_sub):
            b = list(zip(O.per_layer(net, e_lo[i]), O.per_layer(net, e_hi[i])))
            close(np_(gl)[i], O.spec_lower_early_stop(net, L, C[i], b, L - 1, mode), what=f"{mode} {i}")


@pytest.mark.parametrize("cfg", [9, 10])
@pytest.mark.parametrize("kind", ["mlp", "cnn"])
def test_gemm_dma_chunks_keep_the_bound(mod, cfg, kind):
    """The dense GEMM with its k chunks by LDS DMA (tile configurations 9 and 10) pinned on
    every product gives the bound and gradient of the default plans; a width that is not
    a multiple of 16 (the MLP's 30 inputs, 5 outputs) takes the staged path."""
    N, B = mod
    net = (W.mlp([30, 64, 48, 32, 5], seed=211) if kind == "mlp" else
           W.cnn(seed=212, in_shape=(3, 8, 8), spec=[(16, 3, 1), (16, 4, 2)], fc=(64, 32, 5)))
    n_roots, per_root = 2, 6
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), 213)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    n = n_roots * per_root
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    L = len(net)

    def run(pin, fixed=None):
        bn = N.BoundNet(net, n, 4096, 4096)
        if pin is not None:
            for m in range(1, L + 1):
                for prod in "RCA":
                    B.bound_set_plan(bn.handle, prod, m, 2, pin, 0)
        glo, ghi = bn.crown_bounds(x_lo[root_of], x_hi[root_of])
        out = [np_(glo)]
        if fixed is None:
            lo_np, hi_np = np_(glo), np_(ghi)
            sp = _random_splits(net, lo_np.astype(np.float64), hi_np.astype(np.float64), n, 214,
                                np.arange(n, dtype=np.int32))
            fixed = (glo, ghi, sp, dev(W.random_alpha(n, lo_np.shape[1], 215)),
                     dev(W.random_beta(sp.nnz, C.shape[1], 216)))
        flo, fhi, sp, alpha, beta = fixed
        gl, _ = bn.spec_bounds(C[root_of], flo, fhi, x_lo[root_of], x_hi[root_of], alpha=alpha,
                               splits=N.splits_to_device(sp), beta=beta, both=False, save=True)
        ga, gb = bn.grad(torch.ones(n, C.shape[1], device="cuda"), sp.nnz)
        return out + [np_(gl), np_(ga), np_(gb)], fixed

    ref, fixed = run(None)
    got, _ = run(cfg, fixed)
    close(got[0], ref[0], rel=1e-5, what="intermediate bounds")
    close(got[1], ref[1], rel=1e-5, what="lower")
    sa = np.max(np.abs(ref[2]), axis=1, keepdims=True) + 1e-30
    assert np.max(np.abs(got[2] - ref[2]) / sa) <= 1e-3, "grad alpha"
    sb = np.max(np.abs(ref[3])) + 1e-30
    assert np.max(np.abs(got[3] - ref[3])) <= 1e-3 * sb, "grad beta"


# the first two small geometries, and 32x32 images whose tiles are bands of rows
VARIANT_GEOMS = [CNN_GEOMS[0], CNN_GEOMS[1],
                 dict(H=32, convs=((16, 3, 1), (32, 4, 2), (16, 3, 1)), fc=(10,), cin=3)]


@pytest.mark.parametrize("gi", [0, 1, 2])
def test_every_direct_variant_keeps_the_bound(mod, gi):
    """Every direct-convolution variant pinned on every product (staging through
    registers or by LDS DMA, 32x32 or 16x16 MFMA tiles, largest or 4-channel chunks)
    gives the bound and gradient of the default plans (which the oracle tests pin)."""
    N, B = mod
    geom = VARIANT_GEOMS[gi]
    net = tiny_cnn(seed=170 + gi, **geom)
    n_roots, per_root = (2, 5) if geom["H"] <= 8 else (2, 2)
    x0 = W.uniform_inputs(n_roots, W.in_dim(net), 171)
    x_lo, x_hi = W.linf_box(x0, 0.05)
    C = W.margin_spec(W.clean_logits(net, x0))
    n = n_roots * per_root
    root_of = np.repeat(np.arange(n_roots), per_root).astype(np.int32)
    L = len(net)

    def run(pin, fixed=None):
        bn = N.BoundNet(net, n, 4096, 4096)
        if pin is not None:
            for m in range(1, L + 1):
                for prod in "RCA":
                    B.bound_set_plan(bn.handle, prod, m, 1, pin[0], pin[1])
        glo, ghi = bn.crown_bounds(x_lo[root_of], x_hi[root_of])
        out = [np_(glo)]
        if fixed is None:          # the reference run fixes bounds, splits, alpha, beta
            lo_np, hi_np = np_(glo), np_(ghi)
            sp = _random_splits(net, lo_np.astype(np.float64), hi_np.astype(np.float64), n, 172,
                                np.arange(n, dtype=np.int32))
            fixed = (glo, ghi, sp, dev(W.random_alpha(n, lo_np.shape[1], 173)),
                     dev(W.random_beta(sp.nnz, C.shape[1], 174)))
        flo, fhi, sp, alpha, beta = fixed
        gl, _ = bn.spec_bounds(C[root_of], flo, fhi, x_lo[root_of], x_hi[root_of], alpha=alpha,
                               splits=N.splits_to_device(sp), beta=beta, both=False, save=True)
        ga, gb = bn.grad(torch.ones(n, C.shape[1], device="cuda"), sp.nnz)
        return out + [np_(gl), np_(ga), np_(gb)], fixed

    ref, fixed = run(None)
    for pin in [(-1, 0), (1, 0), (2, 0), (3, 0), (2, 4), (3, 4)]:
        got, _ = run(pin, fixed)
        close(got[0], ref[0], rel=1e-5, what=f"intermediate bounds {pin}")
        close(got[1], ref[1], rel=1e-5, what=f"lower {pin}")
        sa = np.max(np.abs(ref[2]), axis=1, keepdims=True) + 1e-30
        assert np.max(np.abs(got[2] - ref[2]) / sa) <= 1e-3, f"grad alpha {pin}"
        assert np.mean(np.abs(got[2] - ref[2]) > 1e-5 * sa) <= 1e-2, f"grad alpha {pin}"
        sb = np.max(np.abs(ref[3])) + 1e-30
        assert np.max(np.abs(got[3] - ref[3])) <= 1e-3 * sb, f"grad beta {pin}"
