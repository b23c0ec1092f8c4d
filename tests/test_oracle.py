"""Pins for the FP64 oracle: each check is fixed by the paper or by mathematics,
not by re-typing the oracle's own formula.

  * Lemma 1: the relaxation sandwiches ReLU on a dense grid; the paper's boundary
    cases; a hand-computed unstable neuron.
  * The layer operators against PyTorch's own conv2d / conv_transpose2d (float64)
    and the adjoint identity <W x, y> = <x, W^T y>.
  * Theorem 2: for a box the closed form is exact -> equals brute-force vertex
    enumeration.
  * Theorem 1 with no unstable neuron is exact -> equals the true minimum found by
    enumerating the vertices of a 2-D box.
  * eps = 0 gives lower = upper = C f(x0).
  * Soundness on tiny 2-D-input nets: 1e5 uniform samples plus a 317x317 grid
    (corners included) for random alpha, and for random beta >= 0 on the split-feasible
    points.
  * Linear programming (scipy HiGHS) on the triangle relaxation: any alpha gives a
    bound <= the LP value <= the sampled minimum; for one hidden layer and one row the
    optimised alpha (and beta with split constraints) reaches the LP value.
  * The adjoint against central finite differences (h = 1e-6).
  * Adam against torch.optim.Adam.
  * CROWN with alpha = 0 is never looser than interval bounds on one hidden layer.
  * The default slope rule picks, of alpha in {0, 1}, the one with the smaller relaxed
    area (numerical integration over [l, u]).
  * The FP32 rounding allowance: an FP32 evaluation of the same bound stays within
    KAPPA / 4 units of 2^-24 M of the FP64 raw bound (CNN and random MLPs).
"""
import itertools

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import crown as O
import workloads as W


def tiny_mlp(dims, seed):
    return W.mlp(dims, seed=seed)


def sample_box(x_lo, x_hi, n, seed):
    rng = np.random.default_rng(seed)
    lo = np.asarray(x_lo, np.float64)
    hi = np.asarray(x_hi, np.float64)
    return lo + (hi - lo) * rng.uniform(0, 1, size=(n, lo.size))


def grid_2d(x_lo, x_hi, k=317):
    a = np.linspace(float(x_lo[0]), float(x_hi[0]), k)
    b = np.linspace(float(x_lo[1]), float(x_hi[1]), k)
    A, B = np.meshgrid(a, b, indexing="ij")
    return np.stack([A.ravel(), B.ravel()], axis=1)


# ---------------------------------------------------------------------------- Lemma 1
def test_relax_hand_example():
    D_lo, D_up, b_lo, b_up, unst = O.relax(np.array([-1.0]), np.array([3.0]), np.array([0.3]))
    assert unst[0]
    assert D_up[0] == pytest.approx(0.75) and b_up[0] == pytest.approx(0.75)
    assert D_lo[0] == pytest.approx(0.3) and b_lo[0] == 0.0


def test_relax_cases():
    l = np.array([0.0, 0.5, -1.0, -2.0, 0.0, -1.0])
    u = np.array([0.0, 1.0, 0.0, -1.0, 2.0, 1.0])
    D_lo, D_up, b_lo, b_up, unst = O.relax(l, u, np.full(6, 0.25))
    # active (l >= 0), inactive (u <= 0), unstable (l < 0 < u)
    assert list(unst) == [False, False, False, False, False, True]
    assert list(D_lo[:5]) == [1, 1, 0, 0, 1] and list(D_up[:5]) == [1, 1, 0, 0, 1]
    assert np.all(b_up[:5] == 0)


def test_relax_sandwich_grid():
    rng = np.random.default_rng(0)
    for _ in range(200):
        l = -rng.uniform(0.01, 3)
        u = rng.uniform(0.01, 3)
        a = rng.uniform(0, 1)
        D_lo, D_up, b_lo, b_up, _ = O.relax(np.array([l]), np.array([u]), np.array([a]))
        z = np.linspace(l, u, 1001)
        r = np.maximum(z, 0)
        assert np.all(D_lo[0] * z + b_lo[0] <= r + 1e-12)
        assert np.all(r <= D_up[0] * z + b_up[0] + 1e-12)
        # the upper line passes through (l, 0) and (u, u)
        assert D_up[0] * l + b_up[0] == pytest.approx(0.0, abs=1e-12)
        assert D_up[0] * u + b_up[0] == pytest.approx(u, abs=1e-12)


# -------------------------------------------------------------------- layer operators
@pytest.mark.parametrize("cin,cout,k,s,p,H", [(3, 4, 3, 1, 1, 7), (2, 5, 4, 2, 1, 8),
                                              (4, 3, 3, 2, 0, 9), (1, 2, 4, 2, 1, 6)])
def test_conv_operators_vs_torch(cin, cout, k, s, p, H):
    rng = np.random.default_rng(1)
    Wt = rng.normal(size=(cout, cin, k, k))
    b = rng.normal(size=cout)
    OH = (H + 2 * p - k) // s + 1
    layer = {"kind": "conv", "W": Wt, "b": b, "in_shape": (cin, H, H),
             "out_shape": (cout, OH, OH), "stride": s, "pad": p}
    x = rng.normal(size=(3, cin * H * H))
    ref = F.conv2d(torch.from_numpy(x.reshape(3, cin, H, H)), torch.from_numpy(Wt),
                   torch.from_numpy(b), stride=s, padding=p).numpy().reshape(3, -1)
    np.testing.assert_allclose(O.affine(layer, x), ref, rtol=1e-12, atol=1e-12)
    lam = rng.normal(size=(4, cout * OH * OH))
    opad = H - ((OH - 1) * s - 2 * p + k)
    refT = F.conv_transpose2d(torch.from_numpy(lam.reshape(4, cout, OH, OH)),
                              torch.from_numpy(Wt), stride=s, padding=p,
                              output_padding=opad).numpy().reshape(4, -1)
    np.testing.assert_allclose(O.linear_T(layer, lam), refT, rtol=1e-12, atol=1e-12)
    # adjoint identity
    lhs = np.sum(O.linear_fwd(layer, x[:1]) * lam[:1])
    rhs = np.sum(x[:1] * O.linear_T(layer, lam[:1]))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_linear_operators_vs_numpy_definition():
    rng = np.random.default_rng(2)
    layer = W.mlp([5, 4])[0]
    x = rng.normal(size=(3, 5))
    ref = torch.nn.functional.linear(torch.from_numpy(x),
                                     torch.from_numpy(layer["W"].astype(np.float64)),
                                     torch.from_numpy(layer["b"].astype(np.float64))).numpy()
    np.testing.assert_allclose(O.affine(layer, x), ref, rtol=1e-13)


# -------------------------------------------------------------------------- Theorem 2
def test_concretize_equals_vertex_enumeration():
    rng = np.random.default_rng(3)
    for d in (1, 3, 6, 9):
        Wt = rng.normal(size=(5, d))
        bt = rng.normal(size=5)
        lo = rng.uniform(-1, 0, d)
        hi = lo + rng.uniform(0, 2, d)
        verts = np.array(list(itertools.product(*[(lo[j], hi[j]) for j in range(d)])))
        brute = (verts @ Wt.T + bt).min(axis=0)
        np.testing.assert_allclose(O.concretize(Wt, bt, lo, hi), brute, rtol=1e-12, atol=1e-12)


def test_single_linear_layer_closed_form():
    net = W.mlp([6, 4], seed=5)
    x0 = W.uniform_inputs(1, 6, seed=6)[0]
    eps = 0.1
    lo, hi = W.linf_box(x0, eps)
    C = np.eye(4)[[0, 1, 2]] - np.eye(4)[[3, 3, 3]]
    got = O.spec_lower(net, 1, C, [], lo, hi, use_slack=False)
    # lower_i = (C W c + C b)_i - sum_j |(CW)_ij| r_j, with the fp32 box (exact in fp64)
    Wm = net[0]["W"].astype(np.float64)
    c = (lo.astype(np.float64) + hi) / 2
    r = (hi.astype(np.float64) - lo) / 2
    verts = np.array(list(itertools.product(*[(lo[j], hi[j]) for j in range(6)])),
                     dtype=np.float64)
    vals = (verts @ Wm.T + net[0]["b"].astype(np.float64)) @ C.T
    np.testing.assert_allclose(got, vals.min(axis=0), rtol=1e-12, atol=1e-12)
    # with an eps-ball of radius exactly eps: minus eps * ||(CW)_i||_1
    cw = C @ Wm
    closed = C @ (Wm @ c + net[0]["b"]) - np.abs(cw) @ r
    np.testing.assert_allclose(got, closed, rtol=1e-12)


# -------------------------------------------------------------------------- Theorem 1
def _planted_stable_net(seed, active_only):
    net = W.mlp([2, 6, 5, 3], seed=seed)
    for layer in net[:-1]:
        if active_only:
            layer["b"] = (np.abs(layer["b"]) + 20.0).astype(np.float32)
        else:
            sgn = np.where(np.arange(len(layer["b"])) % 2 == 0, 1.0, -1.0)
            layer["b"] = (sgn * 20.0).astype(np.float32)
    return net


@pytest.mark.parametrize("active_only", [True, False])
def test_no_unstable_neuron_is_exact(active_only):
    net = _planted_stable_net(7, active_only)
    lo = np.array([-0.5, 0.25], np.float32)
    hi = np.array([0.5, 0.75], np.float32)
    C = np.array([[1.0, -1.0, 0.0], [0.0, 1.0, -1.0], [1.0, 0.0, 0.0]])
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    for (l, u) in bounds:
        assert np.all((l >= 0) | (u <= 0))
    low = O.spec_lower(net, 3, C, bounds, lo, hi, use_slack=False)
    up = -O.spec_lower(net, 3, -C, bounds, lo, hi, use_slack=False)
    verts = np.array(list(itertools.product((lo[0], hi[0]), (lo[1], hi[1]))), np.float64)
    f = O.forward(net, verts)[-1] @ C.T
    np.testing.assert_allclose(low, f.min(axis=0), rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(up, f.max(axis=0), rtol=1e-12, atol=1e-10)


def test_eps_zero():
    net = W.mlp([4, 7, 6, 3], seed=8)
    x0 = W.uniform_inputs(1, 4, seed=9)[0]
    C = np.array([[1.0, -1.0, 0.0], [1.0, 0.0, -1.0]])
    bounds, low, up = O.crown(net, C, x0, x0, use_slack=False)
    f = O.forward(net, x0[None])[-1][0] @ C.T
    np.testing.assert_allclose(low, f, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(up, f, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------- soundness
SOUND_NETS = [([2, 8, 8, 3], 11), ([2, 16, 16, 16, 2], 12), ([2, 12, 3], 13)]


@pytest.mark.parametrize("dims,seed", SOUND_NETS)
def test_soundness_random_alpha(dims, seed):
    net = tiny_mlp(dims, seed)
    lo = np.array([-1.0, -0.5], np.float32)
    hi = np.array([0.5, 1.0], np.float32)
    pts = np.concatenate([sample_box(lo, hi, 100_000, seed), grid_2d(lo, hi)])
    zs = O.forward(net, pts)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    for m, (l, u) in enumerate(bounds):
        assert np.all(zs[m] >= l - 1e-9) and np.all(zs[m] <= u + 1e-9)
    L = len(net)
    C = np.eye(dims[-1])
    C = np.concatenate([C, -C])
    rng = np.random.default_rng(seed)
    f = zs[-1] @ C.T
    for trial in range(4):
        alpha = [rng.uniform(0, 1, len(l)) for (l, _) in bounds]
        low = O.spec_lower(net, L, C, bounds, lo, hi, alpha, use_slack=False)
        assert np.all(f.min(axis=0) >= low - 1e-9)


@pytest.mark.parametrize("dims,seed", SOUND_NETS)
def test_soundness_beta_splits(dims, seed):
    net = tiny_mlp(dims, seed)
    lo = np.array([-1.0, -0.5], np.float32)
    hi = np.array([0.5, 1.0], np.float32)
    pts = np.concatenate([sample_box(lo, hi, 100_000, seed + 1), grid_2d(lo, hi)])
    zs = O.forward(net, pts)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    unst = [(m + 1, j) for m, (l, u) in enumerate(bounds) for j in range(len(l))
            if l[j] < 0 < u[j]]
    assert len(unst) >= 3
    rng = np.random.default_rng(seed)
    L = len(net)
    C = np.concatenate([np.eye(dims[-1]), -np.eye(dims[-1])])
    checked = 0
    for trial in range(12):
        k = int(rng.integers(1, min(4, len(unst)) + 1))
        pick = rng.choice(len(unst), size=k, replace=False)
        splits = [(unst[i][0], unst[i][1], int(rng.choice([-1, 1]))) for i in pick]
        feas = np.ones(len(pts), bool)
        for (m, j, sg) in splits:
            feas &= sg * zs[m - 1][:, j] >= 0
        if feas.sum() < 10:
            continue
        beta = rng.uniform(0, 2, size=(len(splits), C.shape[0]))
        alpha = [rng.uniform(0, 1, len(l)) for (l, _) in bounds]
        low = O.spec_lower(net, L, C, bounds, lo, hi, alpha, splits, beta, use_slack=False)
        f = zs[-1][feas] @ C.T
        assert np.all(f.min(axis=0) >= low - 1e-9)
        low0 = O.spec_lower(net, L, C, bounds, lo, hi, alpha, splits, None, use_slack=False)
        assert np.all(f.min(axis=0) >= low0 - 1e-9)
        checked += 1
    assert checked >= 4


def test_beta_zero_equals_clamped_plain_crown():
    net = tiny_mlp([3, 10, 10, 4], 21)
    lo = np.array([-1.0, -1.0, -1.0], np.float32)
    hi = np.array([1.0, 1.0, 1.0], np.float32)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    unst = [(m + 1, j) for m, (l, u) in enumerate(bounds) for j in range(len(l))
            if l[j] < 0 < u[j]]
    splits = [(unst[0][0], unst[0][1], 1), (unst[-1][0], unst[-1][1], -1)]
    C = np.eye(4)
    a = O.spec_lower(net, 3, C, bounds, lo, hi, None, splits, np.zeros((2, 4)),
                     use_slack=False)
    # the same constraints written directly into the pre-activation box
    manual = [(l.copy(), u.copy()) for (l, u) in bounds]
    manual[unst[0][0] - 1][0][unst[0][1]] = 0.0
    manual[unst[-1][0] - 1][1][unst[-1][1]] = 0.0
    b = O.spec_lower(net, 3, C, manual, lo, hi, use_slack=False)
    np.testing.assert_allclose(a, b, rtol=1e-13)


def test_infeasible_split_gives_plus_inf():
    net = tiny_mlp([2, 6, 2], 22)
    lo = np.array([-1.0, -1.0], np.float32)
    hi = np.array([1.0, 1.0], np.float32)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    l, u = bounds[0]
    j = int(np.argmin(u))
    bounds[0][1][j] = -abs(bounds[0][1][j]) - 1.0   # make it strictly inactive
    bounds[0][0][j] = min(bounds[0][0][j], bounds[0][1][j] - 1.0)
    low = O.spec_lower(net, 2, np.eye(2), bounds, lo, hi, None, [(1, j, 1)], None)
    assert np.all(np.isinf(low)) and np.all(low > 0)


# -------------------------------------------------------------------------------- LP
def _lp_one_hidden(net, c_row, lo, hi, bounds, splits=()):
    """min c^T (W2 h + b2) over the triangle relaxation of one hidden layer (HiGHS)."""
    from scipy.optimize import linprog
    W1 = net[0]["W"].astype(np.float64)
    b1 = net[0]["b"].astype(np.float64)
    W2 = net[1]["W"].astype(np.float64)
    b2 = net[1]["b"].astype(np.float64)
    d0, d1 = W1.shape[1], W1.shape[0]
    l, u = [np.array(v, np.float64) for v in bounds[0]]
    for (m, j, sg) in splits:
        if sg > 0:
            l[j] = max(l[j], 0.0)
        else:
            u[j] = min(u[j], 0.0)
    nv = d0 + 2 * d1          # x, z, h
    cost = np.zeros(nv)
    cost[d0 + d1:] = c_row @ W2
    A_eq, b_eq, A_ub, b_ub = [], [], [], []
    for j in range(d1):      # z = W1 x + b1
        row = np.zeros(nv)
        row[:d0] = -W1[j]
        row[d0 + j] = 1.0
        A_eq.append(row)
        b_eq.append(b1[j])
    for j in range(d1):
        zi, hi_ = d0 + j, d0 + d1 + j
        if l[j] >= 0:
            row = np.zeros(nv); row[hi_] = 1; row[zi] = -1
            A_eq.append(row); b_eq.append(0.0)
        elif u[j] <= 0:
            row = np.zeros(nv); row[hi_] = 1
            A_eq.append(row); b_eq.append(0.0)
        else:
            row = np.zeros(nv); row[hi_] = -1; row[zi] = 1          # z - h <= 0
            A_ub.append(row); b_ub.append(0.0)
            s = u[j] / (u[j] - l[j])                                 # h <= s (z - l)
            row = np.zeros(nv); row[hi_] = 1; row[zi] = -s
            A_ub.append(row); b_ub.append(-s * l[j])
        for (m, jj, sg) in splits:                                   # sigma z >= 0
            if jj == j:
                row = np.zeros(nv); row[zi] = -sg
                A_ub.append(row); b_ub.append(0.0)
    bnds = [(float(lo[i]), float(hi[i])) for i in range(d0)] + \
        [(float(l[j]), float(u[j])) for j in range(d1)] + [(0.0, None)] * d1
    res = linprog(cost, A_ub=np.array(A_ub) if A_ub else None,
                  b_ub=np.array(b_ub) if b_ub else None, A_eq=np.array(A_eq),
                  b_eq=np.array(b_eq), bounds=bnds, method="highs")
    assert res.status == 0
    return res.fun + c_row @ b2


def _maximise(net, C, bounds, lo, hi, splits, use_beta, steps=1500):
    best, _, _ = O.optimize_alpha_beta(net, C, bounds, lo, hi, splits, steps=steps, lr=0.02,
                                       alpha0=0.5, use_beta=use_beta)
    return best


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_lp_one_hidden_layer(seed):
    net = tiny_mlp([3, 8, 2], seed)
    lo = np.array([-1.0, -1.0, -1.0], np.float32)
    hi = np.array([1.0, 1.0, 1.0], np.float32)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    C = np.array([[1.0, -1.0]])
    lp = _lp_one_hidden(net, C[0], lo, hi, bounds)
    pts = sample_box(lo, hi, 100_000, seed)
    true_min = (O.forward(net, pts)[-1] @ C.T).min()
    rng = np.random.default_rng(seed)
    for _ in range(5):
        alpha = [rng.uniform(0, 1, 8)]
        assert O.spec_lower(net, 2, C, bounds, lo, hi, alpha, use_slack=False)[0] <= lp + 1e-9
    assert lp <= true_min + 1e-9
    best = _maximise(net, C, bounds, lo, hi, (), False)
    assert best[0] <= lp + 1e-7
    assert best[0] >= lp - 2e-3 * max(1.0, abs(lp))


@pytest.mark.parametrize("seed", [41, 42])
def test_lp_one_hidden_layer_with_splits(seed):
    net = tiny_mlp([3, 8, 2], seed)
    lo = np.array([-1.0, -1.0, -1.0], np.float32)
    hi = np.array([1.0, 1.0, 1.0], np.float32)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    l, u = bounds[0]
    unst = [j for j in range(8) if l[j] < 0 < u[j]]
    splits = [(1, unst[0], 1), (1, unst[1], -1)]
    C = np.array([[1.0, -1.0]])
    lp = _lp_one_hidden(net, C[0], lo, hi, bounds, splits)
    best = _maximise(net, C, bounds, lo, hi, splits, True)
    assert best[0] <= lp + 1e-7
    assert best[0] >= lp - 2e-3 * max(1.0, abs(lp))


# ---------------------------------------------------------------------------- adjoint
def _fd_check(net, C, bounds, lo, hi, splits, n_coord=32, seed=0):
    rng = np.random.default_rng(seed)
    L = len(net)
    alpha = [rng.uniform(0.05, 0.95, len(l)) for (l, _) in bounds]
    beta = rng.uniform(0.05, 1.0, size=(len(splits), C.shape[0])) if splits else None
    gbar = rng.uniform(0.5, 1.5, C.shape[0])
    _, ga, gb = O.spec_lower_grad(net, L, C, bounds, lo, hi, alpha, splits, beta, gbar)

    def val(al, be):
        return float(gbar @ O.spec_lower(net, L, C, bounds, lo, hi, al, splits, be,
                                         use_slack=False))

    coords = []
    cb, _ = O.clamp_splits(bounds, splits)
    for m, (l, u) in enumerate(cb):
        for j in np.nonzero((l < 0) & (u > 0))[0]:
            coords.append(("a", m, int(j)))
    if splits:
        for q in range(len(splits)):
            for r in range(C.shape[0]):
                coords.append(("b", q, r))
    pick = rng.choice(len(coords), size=min(n_coord, len(coords)), replace=False)
    h = 1e-6
    n_alpha_nonzero = 0
    for i in pick:
        kind, a, b = coords[i]
        if kind == "a":
            ap = [x.copy() for x in alpha]; am = [x.copy() for x in alpha]
            ap[a][b] += h; am[a][b] -= h
            fd = (val(ap, beta) - val(am, beta)) / (2 * h)
            an = ga[a][b]
            n_alpha_nonzero += an != 0
        else:
            bp = beta.copy(); bm = beta.copy()
            bp[a, b] += h; bm[a, b] -= h
            fd = (val(alpha, bp) - val(alpha, bm)) / (2 * h)
            an = gb[a, b]
        assert an == pytest.approx(fd, rel=1e-5, abs=1e-6 * (1 + abs(fd))), (kind, a, b)
    return n_alpha_nonzero


def test_adjoint_fd_mlp():
    net = tiny_mlp([5, 12, 12, 12, 4], 51)
    lo, hi = W.linf_box(W.uniform_inputs(1, 5, 52)[0], 0.3)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    C = np.array([[1.0, -1.0, 0, 0], [1.0, 0, -1.0, 0], [1.0, 0, 0, -1.0]])
    assert _fd_check(net, C, bounds, lo, hi, ()) > 0


def test_adjoint_fd_mlp_splits():
    net = tiny_mlp([5, 12, 12, 12, 4], 53)
    lo, hi = W.linf_box(W.uniform_inputs(1, 5, 54)[0], 0.3)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    unst = [(m + 1, j) for m, (l, u) in enumerate(bounds) for j in range(len(l))
            if l[j] < 0 < u[j]]
    splits = [(unst[0][0], unst[0][1], 1), (unst[3][0], unst[3][1], -1),
              (unst[-1][0], unst[-1][1], 1)]
    C = np.array([[1.0, -1.0, 0, 0], [1.0, 0, -1.0, 0], [1.0, 0, 0, -1.0]])
    _fd_check(net, C, bounds, lo, hi, splits, n_coord=32, seed=1)


def test_adjoint_fd_cnn():
    net = W.cnn(seed=55, in_shape=(2, 8, 8), spec=[(3, 3, 1), (4, 4, 2)], fc=(16, 3))
    lo, hi = W.linf_box(W.uniform_inputs(1, 128, 56)[0], 0.1)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    unst = [(m + 1, j) for m, (l, u) in enumerate(bounds) for j in range(len(l))
            if l[j] < 0 < u[j]]
    splits = [(unst[1][0], unst[1][1], -1), (unst[-2][0], unst[-2][1], 1)]
    C = np.array([[1.0, -1.0, 0], [0, 1.0, -1.0]])
    assert _fd_check(net, C, bounds, lo, hi, splits, n_coord=32, seed=2) > 0


# ------------------------------------------------------------------------------- Adam
def test_adam_matches_torch():
    rng = np.random.default_rng(61)
    p0 = rng.uniform(0, 1, 20)
    grads = [rng.normal(size=20) for _ in range(5)]
    tp = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=0.1)
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = O.adam_step(p, g, m, v, t, 0.1)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------------ IBP relation
@pytest.mark.parametrize("seed", [71, 72, 73])
def test_crown_alpha0_not_looser_than_ibp_one_hidden(seed):
    net = tiny_mlp([6, 20, 5], seed)
    lo, hi = W.linf_box(W.uniform_inputs(1, 6, seed)[0], 0.2)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    ib = O.ibp(net, lo, hi)
    np.testing.assert_allclose(bounds[0][0], ib[0][0], rtol=1e-12, atol=1e-12)
    alpha = [np.zeros(20)]
    C = np.eye(5)
    low = O.spec_lower(net, 2, C, bounds, lo, hi, alpha, use_slack=False)
    up = -O.spec_lower(net, 2, -C, bounds, lo, hi, alpha, use_slack=False)
    assert np.all(low >= ib[1][0] - 1e-12)
    assert np.all(up <= ib[1][1] + 1e-12)


def test_adaptive_alpha_minimises_the_relaxed_area():
    """The default lower slope (alpha = 1 if u >= -l, else 0) picks, of the two slopes in
    {0, 1}, the one whose lower line leaves the smaller area between the two relaxation
    lines over [l, u] (the choice plain CROWN makes when no alpha is given).  Areas are
    integrated numerically on a dense z-grid, not taken from a closed form; at u = -l
    both areas are equal and the rule takes 1."""
    ls = -np.geomspace(1e-3, 10.0, 61)
    us = np.geomspace(1e-3, 10.0, 61)
    for l in ls:
        for u in us:
            z = np.linspace(l, u, 2001)
            D_lo, D_up, b_lo, b_up, unst = O.relax(np.array([l]), np.array([u]), np.array([0.0]))
            assert unst[0]
            upper = D_up[0] * z + b_up[0]
            area = [np.trapezoid(upper - a * z, z) for a in (0.0, 1.0)]
            a = float(O.adaptive_alpha(np.array([l]), np.array([u]))[0])
            other = 1.0 - a
            assert area[int(a)] <= area[int(other)] + 1e-9 * abs(area[int(other)])
    # exact tie and the two sides of it
    assert O.adaptive_alpha(np.array([-2.0]), np.array([2.0]))[0] == 1.0
    assert O.adaptive_alpha(np.array([-2.0]), np.array([1.999]))[0] == 0.0
    assert O.adaptive_alpha(np.array([-1.999]), np.array([2.0]))[0] == 1.0


# ---------------------------------------------------- FP32 rounding allowance (kappa)
def _t32(a):
    return torch.as_tensor(np.asarray(a, np.float32))


def _lin_T32(layer, lam):
    Wt = _t32(layer["W"])
    if layer["kind"] == "linear":
        return lam @ Wt
    R = lam.shape[0]
    ci, H, Wd = layer["in_shape"]
    co, OH, OW = layer["out_shape"]
    s, p = layer["stride"], layer["pad"]
    k = Wt.shape[2]
    op = H - ((OH - 1) * s - 2 * p + k)
    return F.conv_transpose2d(lam.reshape(R, co, OH, OW), Wt, stride=s, padding=p,
                              output_padding=op).reshape(R, -1)


def _bias32(layer):
    b = _t32(layer["b"])
    if layer["kind"] == "conv":
        b = b.repeat_interleave(layer["out_shape"][1] * layer["out_shape"][2])
    return b


def _bound_fp32(net, k, C, bounds, x_lo, x_hi, alpha, splits, beta):
    """The bound of Theorem 1 + Theorem 2 with every operation in float32 (PyTorch CPU
    products): what an FP32 implementation of the same steps returns."""
    A = _t32(C)
    Wt = _lin_T32(net[k - 1], A)
    bt = A @ _bias32(net[k - 1])
    for m in range(k - 1, 0, -1):
        l, u = _t32(bounds[m - 1][0]).clone(), _t32(bounds[m - 1][1]).clone()
        for (ms, j, sg) in splits:
            if ms == m:
                if sg > 0:
                    l[j] = max(float(l[j]), 0.0)
                else:
                    u[j] = min(float(u[j]), 0.0)
        a = _t32(alpha[m - 1]) if alpha is not None else torch.where(u >= -l, 1.0, 0.0)
        act = l >= 0
        ina = (~act) & (u <= 0)
        un = ~(act | ina)
        su = torch.where(un, u / torch.where(un, u - l, torch.ones_like(u)), torch.zeros_like(u))
        D_lo = torch.where(act, 1.0, torch.where(ina, 0.0, a))
        D_up = torch.where(act, 1.0, torch.where(ina, 0.0, su))
        b_up = torch.where(un, -l * su, torch.zeros_like(u))
        pos = Wt >= 0
        Am = torch.where(pos, Wt * D_lo, Wt * D_up)
        bt = bt + torch.where(pos, torch.zeros_like(Wt), Wt * b_up).sum(1)
        for q, (ms, j, sg) in enumerate(splits):
            if ms == m and beta is not None:
                Am[:, j] -= _t32(beta[q]) * float(sg)
        Wt = _lin_T32(net[m - 1], Am)
        bt = bt + Am @ _bias32(net[m - 1])
    xl, xh = _t32(x_lo), _t32(x_hi)
    c, r = 0.5 * (xl + xh), 0.5 * (xh - xl)
    return (Wt @ c - Wt.abs() @ r + bt).double().numpy()


def _allowance_ratio(net, k, C, bounds, x_lo, x_hi, alpha, splits, beta):
    """|FP32 bound - FP64 raw bound| in units of 2^-24 M, M the oracle's magnitude sum."""
    cb, feasible = O.clamp_splits(bounds, splits)
    assert feasible
    Wt, bt, mag = O.backward(net, k, C, cb, alpha, splits, beta)
    exact = O.concretize(Wt, bt, x_lo, x_hi)
    allowance = O.slack(Wt, mag, x_lo, x_hi, kappa=1.0)       # 2^-24 M
    got = _bound_fp32(net, k, C, bounds, x_lo, x_hi, alpha, splits, beta)
    return np.abs(got - exact) / allowance


def test_fp32_error_stays_well_inside_the_rounding_allowance():
    """kappa = 64 is a margin, not a guess: on the 3x32x32 CNN (root 0, random splits,
    alpha, beta) and on 20 random MLPs (random widths, depths, boxes, splits, alpha,
    beta) the FP32 evaluation of the bound differs from the FP64 raw bound by at most
    KAPPA / 4 units of 2^-24 M, so the outward allowance covers the FP32 arithmetic with
    a factor of at least 4 to spare."""
    import os
    torch.set_num_threads(max(1, min(8, os.cpu_count() or 1)))
    worst = 0.0
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cnn_root0.npz"))
    w = W.cnn_cifar(1)
    net = w.net
    lo = g["lo"].astype(np.float32).astype(np.float64)
    hi = g["hi"].astype(np.float32).astype(np.float64)
    bounds = list(zip(O.per_layer(net, lo), O.per_layer(net, hi)))
    cand = np.nonzero((lo < 0) & (hi > 0))[0]
    rng = np.random.default_rng(0)
    for trial in range(4):
        sp = W.random_splits([cand], 1, 1, 12, seed=100 + trial)
        splits = O.split_list(net, sp.neuron, sp.sign)
        alpha = [rng.uniform(0, 1, len(l)) for (l, _) in bounds] if trial % 2 else None
        beta = rng.uniform(0, 0.5, (len(splits), 9)) if trial > 1 else None
        worst = max(worst, _allowance_ratio(net, len(net), w.spec[0].astype(np.float64), bounds,
                                            w.x_lo[0], w.x_hi[0], alpha, splits, beta).max())
    for seed in range(20):
        dims = ([int(rng.choice([16, 64, 256, 784]))] +
                [int(x) for x in rng.choice([32, 128, 256, 512], rng.integers(2, 6))] + [10])
        net = W.mlp(dims, seed=200 + seed)
        x0 = W.uniform_inputs(1, dims[0], 300 + seed)[0]
        xl, xh = W.linf_box(x0, float(rng.choice([0.005, 0.02, 0.1])))
        b32 = [(l.astype(np.float32).astype(np.float64), u.astype(np.float32).astype(np.float64))
               for (l, u) in O.crown_bounds(net, xl, xh)]
        C = W.margin_spec(W.clean_logits(net, x0[None]))[0].astype(np.float64)
        flo = np.concatenate([b[0] for b in b32])
        fhi = np.concatenate([b[1] for b in b32])
        cand = np.nonzero((flo < 0) & (fhi > 0))[0]
        splits, beta = [], None
        if len(cand):
            sp = W.random_splits([cand], 1, 1, 8, seed=400 + seed)
            splits = O.split_list(net, sp.neuron, sp.sign)
            beta = rng.uniform(0, 0.5, (len(splits), C.shape[0]))
        alpha = [rng.uniform(0, 1, len(l)) for (l, _) in b32]
        worst = max(worst, _allowance_ratio(net, len(net), C, b32, xl, xh, alpha, splits, beta).max())
        # an intermediate-bound pass (identity rows on a middle layer, adaptive alpha)
        k = len(net) // 2 + 1
        I = np.eye(len(b32[k - 1][0]))[:64]
        worst = max(worst, _allowance_ratio(net, k, np.concatenate([I, -I]), b32[:k - 1], xl, xh,
                                            None, (), None).max())
    assert worst <= O.KAPPA / 4, worst


def test_slack_is_outward_and_small():
    net = tiny_mlp([4, 9, 9, 3], 81)
    lo, hi = W.linf_box(W.uniform_inputs(1, 4, 82)[0], 0.1)
    b_raw = O.crown_bounds(net, lo, hi, use_slack=False)
    b_sl = O.crown_bounds(net, lo, hi, use_slack=True)
    for (l0, u0), (l1, u1) in zip(b_raw, b_sl):
        assert np.all(l1 <= l0) and np.all(u1 >= u0)
        assert np.all(l0 - l1 <= 1e-4 * (1 + np.abs(l0)))


# ----------------------------------------------------------- full-size alpha-CROWN
def test_adjoint_fd_full_cnn_32_coordinates():
    """The 3x32x32 CNN with its full-CROWN root bounds (stored oracle output): the adjoint
    of the final margin bound against central differences (h = 1e-6) at 32 random alpha
    coordinates of unstable neurons, FP64."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cnn_root0.npz")
    g = np.load(path)
    w = W.cnn_cifar(1)
    net = w.net
    lo = g["lo"].astype(np.float32).astype(np.float64)
    hi = g["hi"].astype(np.float32).astype(np.float64)
    bounds = list(zip(O.per_layer(net, lo), O.per_layer(net, hi)))
    rng = np.random.default_rng(7)
    alpha = [rng.uniform(0.05, 0.95, len(l)) for (l, _) in bounds]
    C = w.spec[0].astype(np.float64)
    L = len(net)
    _, ga, _ = O.spec_lower_grad(net, L, C, bounds, w.x_lo[0], w.x_hi[0], alpha)
    unst = [(m, j) for m, (l, u) in enumerate(bounds) for j in np.nonzero((l < 0) & (u > 0))[0]]
    pick = rng.choice(len(unst), size=32, replace=False)
    h = 1e-6
    for i in pick:
        m, j = unst[i]
        ap = [a.copy() for a in alpha]
        am = [a.copy() for a in alpha]
        ap[m][j] += h
        am[m][j] -= h
        fp = O.spec_lower(net, L, C, bounds, w.x_lo[0], w.x_hi[0], ap, use_slack=False).sum()
        fm = O.spec_lower(net, L, C, bounds, w.x_lo[0], w.x_hi[0], am, use_slack=False).sum()
        fd = (fp - fm) / (2 * h)
        assert ga[m][j] == pytest.approx(fd, rel=1e-5, abs=1e-7 * (1 + abs(fd)))


# ------------------------------------------------------------------ early stop (B.2)
def test_early_stop_relu_node_is_interval_arithmetic_of_the_layers_above():
    """Stopping at the last ReLU node of a 2-layer net leaves C W2 h + C b2 over the box of
    h = ReLU(z_1): exactly the interval bound of the last layer (the oracle's IBP)."""
    net = tiny_mlp([5, 9, 4], 101)
    lo, hi = W.linf_box(W.uniform_inputs(1, 5, 102)[0], 0.3)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    C = np.eye(4)
    got = O.spec_lower_early_stop(net, 2, C, bounds, 1, "relu", use_slack=False)
    l1, u1 = bounds[0]
    last = dict(net[1])
    ib = O.ibp([last], np.maximum(l1, 0), np.maximum(u1, 0))
    np.testing.assert_allclose(got, ib[0][0], rtol=1e-12, atol=1e-12)


def test_early_stop_linear_node_is_vertex_minimum_of_relaxed_function():
    """Stopping at the linear node below the ReLU (relax, then concretise over [l, u]) equals
    the brute-force minimum, over the vertices of the pre-activation box, of the relaxed
    linear function (Theorem 2 is exact for a box)."""
    net = tiny_mlp([4, 6, 3], 103)
    lo, hi = W.linf_box(W.uniform_inputs(1, 4, 104)[0], 0.4)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    l1, u1 = bounds[0]
    rng = np.random.default_rng(105)
    alpha = [rng.uniform(0, 1, 6)]
    C = np.array([[1.0, -1.0, 0.0], [0.0, 1.0, -1.0]])
    got = O.spec_lower_early_stop(net, 2, C, bounds, 1, "linear", alpha, use_slack=False)
    W2 = net[1]["W"].astype(np.float64)
    b2 = net[1]["b"].astype(np.float64)
    D_lo, D_up, _, b_up, _ = O.relax(l1, u1, alpha[0])
    verts = np.array(list(itertools.product(*[(l1[j], u1[j]) for j in range(6)])))
    for r in range(2):
        g = C[r] @ W2
        # per-neuron relaxed value: lower line where the coefficient is >= 0, upper otherwise
        vals = np.where(g >= 0, g * D_lo * verts, g * (D_up * verts + b_up)).sum(1) + C[r] @ b2
        assert got[r] == pytest.approx(vals.min(), rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("dims,seed", [([2, 8, 8, 3], 111), ([2, 16, 16, 16, 2], 112)])
def test_early_stop_is_sound_and_ordered(dims, seed):
    """With exact intermediate bounds every early-stop bound is sound; stopping at the
    ReLU node is never looser than relaxing it first (per neuron, the interval of
    ReLU(z) is the tightest), and full propagation is a separate valid bound."""
    net = tiny_mlp(dims, seed)
    lo = np.array([-1.0, -0.5], np.float32)
    hi = np.array([0.5, 1.0], np.float32)
    pts = np.concatenate([sample_box(lo, hi, 100_000, seed), grid_2d(lo, hi)])
    f = O.forward(net, pts)[-1]
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    L = len(net)
    C = np.concatenate([np.eye(dims[-1]), -np.eye(dims[-1])])
    fmin = (f @ C.T).min(axis=0)
    rng = np.random.default_rng(seed)
    alpha = [rng.uniform(0, 1, len(l)) for (l, _) in bounds]
    for s in range(1, L):
        a = O.spec_lower_early_stop(net, L, C, bounds, s, "relu", alpha, use_slack=False)
        b = O.spec_lower_early_stop(net, L, C, bounds, s, "linear", alpha, use_slack=False)
        assert np.all(fmin >= a - 1e-9) and np.all(fmin >= b - 1e-9)
        assert np.all(a >= b - 1e-9)


@pytest.mark.parametrize("mode", ["relu", "linear"])
def test_early_stop_adjoint_fd(mode):
    net = tiny_mlp([5, 12, 12, 12, 4], 121)
    lo, hi = W.linf_box(W.uniform_inputs(1, 5, 122)[0], 0.3)
    bounds = O.crown_bounds(net, lo, hi, use_slack=False)
    unst = [(m + 1, j) for m, (l, u) in enumerate(bounds) for j in range(len(l)) if l[j] < 0 < u[j]]
    C = np.array([[1.0, -1.0, 0, 0], [1.0, 0, -1.0, 0], [1.0, 0, 0, -1.0]])
    rng = np.random.default_rng(123)
    L = len(net)
    for stop in (1, 2):
        splits = [u_ for u_ in unst if u_[0] >= stop][:3]
        splits = [(m, j, int(rng.choice([-1, 1]))) for (m, j) in splits]
        alpha = [rng.uniform(0.05, 0.95, len(l)) for (l, _) in bounds]
        beta = rng.uniform(0.05, 1.0, size=(len(splits), 3))
        gbar = rng.uniform(0.5, 1.5, 3)
        low, ga, gb = O.spec_lower_grad(net, L, C, bounds, lo, hi, alpha, splits, beta, gbar,
                                        stop=stop, mode=mode)
        np.testing.assert_allclose(low, O.spec_lower_early_stop(net, L, C, bounds, stop, mode, alpha,
                                                                splits, beta, use_slack=False), rtol=1e-12)

        def val(al, be):
            return float(gbar @ O.spec_lower_early_stop(net, L, C, bounds, stop, mode, al, splits, be,
                                                        use_slack=False))
        h = 1e-6
        cb, _ = O.clamp_splits(bounds, splits)
        lowest = stop + 1 if mode == "relu" else stop
        coords = [(m, j) for m, (l, u) in enumerate(cb) for j in np.nonzero((l < 0) & (u > 0))[0]
                  if m + 1 >= lowest]
        for i in rng.choice(len(coords), size=min(16, len(coords)), replace=False):
            m, j = coords[i]
            ap = [x.copy() for x in alpha]; am = [x.copy() for x in alpha]
            ap[m][j] += h; am[m][j] -= h
            fd = (val(ap, beta) - val(am, beta)) / (2 * h)
            assert ga[m][j] == pytest.approx(fd, rel=1e-5, abs=1e-7)
        for q in range(len(splits)):
            for r in range(3):
                bp = beta.copy(); bm = beta.copy()
                bp[q, r] += h; bm[q, r] -= h
                fd = (val(alpha, bp) - val(alpha, bm)) / (2 * h)
                assert gb[q, r] == pytest.approx(fd, rel=1e-5, abs=1e-7)


# ------------------------------------------------------- search-integrated bounds
def test_sample_bounds_inside_sound_bounds_and_exact_on_vertices():
    net = tiny_mlp([3, 10, 10, 2], 141)
    lo, hi = W.linf_box(W.uniform_inputs(1, 3, 142)[0], 0.2)
    crown_b = O.crown_bounds(net, lo, hi, use_slack=False)
    pts = sample_box(lo, hi, 20_000, 143)
    emp = O.sample_bounds(net, pts)
    for (el, eu), (cl, cu) in zip(emp, crown_b):
        assert np.all(el >= cl - 1e-12) and np.all(eu <= cu + 1e-12)
    # first layer: z_1 is affine in x, so its extremes over the box sit at vertices
    verts = np.array(list(itertools.product(*[(lo[j], hi[j]) for j in range(3)])), np.float64)
    ev = O.sample_bounds(net, verts)
    np.testing.assert_allclose(ev[0][0], crown_b[0][0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ev[0][1], crown_b[0][1], rtol=1e-12, atol=1e-12)


# -------------------------------------------- unrolled dynamics and optimised bounds
def test_unrolled_chain_equals_stepwise_rollout():
    """The layer chain of the unrolled dynamics model (composed step boundaries, carried
    actions) computes the same objective as stepping the dynamics MLP H times."""
    for H in (1, 2, 3, 20):
        uw = W.pushing_unrolled(H)
        assert len(uw.net) == 4 * H + 2 and W.in_dim(uw.net) == 2 * H
        rng = np.random.default_rng(H)
        u = rng.uniform(uw.u_lo, uw.u_hi, (64, 2 * H))
        f = O.forward(uw.net, u)[-1][:, 0]
        ref = W.rollout_cost(u, uw)
        assert np.max(np.abs(f - ref) / np.maximum(1.0, np.abs(ref))) < 1e-5
    assert sum(l["W"].size + l["b"].size for l in W.pushing_mlp()) == 134152


def test_carried_actions_are_stable_active_neurons():
    """Carried actions stay >= the pass-through offset on the action box, so CROWN keeps
    them exact (active neurons, no relaxation)."""
    uw = W.pushing_unrolled(3)
    lo, hi = W.action_subboxes(uw, 1, seed=31)
    b = O.crown_bounds(uw.net, lo[0], hi[0])
    for m, (l, u) in enumerate(b[:-1]):
        width = W.out_dim(uw.net[m])
        hidden = {0: 128, 1: 256, 2: 256, 3: 128}[m % 4]
        assert width >= hidden
        assert np.all(l[hidden:] >= 0.5 * W.PUSH_PASS)


@pytest.mark.parametrize("H,seed", [(1, 41), (2, 42)])
def test_alpha_crown_bounds_sound_and_tighter(H, seed):
    """Optimised intermediate bounds of the unrolled model on an action sub-box: sound on
    10^5 sampled action sequences (every pre-activation inside [l, u]), and in total
    tighter than plain CROWN's (each layer's bound includes the default-rule pass on the
    same lower-layer bounds, and the slopes are optimised from there)."""
    uw = W.pushing_unrolled(H)
    lo, hi = W.action_subboxes(uw, 1, seed=seed, width=(0.3, 0.6))
    lo, hi = lo[0], hi[0]
    plain = O.crown_bounds(uw.net, lo, hi)
    opt = O.alpha_crown_bounds(uw.net, lo, hi, steps=5)
    u = sample_box(lo, hi, 100000, seed)
    zs = O.forward(uw.net, u)
    for m, (l, h) in enumerate(opt):
        assert np.all(zs[m].min(axis=0) >= l - 1e-9), m
        assert np.all(zs[m].max(axis=0) <= h + 1e-9), m
    w_plain = sum(float(np.sum(h - l)) for (l, h) in plain)
    w_opt = sum(float(np.sum(h - l)) for (l, h) in opt)
    assert w_opt < w_plain
    # layer by layer: never looser than the default-rule pass on the same lower-layer bounds
    for k in range(2, len(uw.net)):
        d = W.out_dim(uw.net[k - 1])
        A = np.concatenate([np.eye(d), -np.eye(d)])
        ref = O.spec_lower(uw.net, k, A, opt[:k - 1], lo, hi, None)
        assert np.all(opt[k - 1][0] >= ref[:d]) and np.all(opt[k - 1][1] <= -ref[d:])


def test_both_sided_rows_adjoint_fd():
    """The adjoint of a pass whose rows are [I; -I] (the optimised intermediate bounds'
    objective) against central differences, on the unrolled model."""
    uw = W.pushing_unrolled(2)
    lo, hi = W.action_subboxes(uw, 1, seed=43, width=(0.3, 0.6))
    bounds = O.crown_bounds(uw.net, lo[0], hi[0])
    k = 6
    d = W.out_dim(uw.net[k - 1])
    A = np.concatenate([np.eye(d), -np.eye(d)])
    rng = np.random.default_rng(44)
    alpha = [rng.uniform(0.05, 0.95, len(l)) for (l, _) in bounds[:k - 1]]
    gbar = rng.normal(size=2 * d)
    _, ga, _ = O.spec_lower_grad(uw.net, k, A, bounds[:k - 1], lo[0], hi[0], alpha, gbar=gbar)
    unst = [(m, j) for m, (l, u) in enumerate(bounds[:k - 1]) for j in np.nonzero((l < 0) & (u > 0))[0]]
    assert len(unst) >= 16
    h = 1e-6
    for i in rng.choice(len(unst), size=16, replace=False):
        m, j = unst[i]
        ap = [a.copy() for a in alpha]
        am = [a.copy() for a in alpha]
        ap[m][j] += h
        am[m][j] -= h
        fp = gbar @ O.spec_lower(uw.net, k, A, bounds[:k - 1], lo[0], hi[0], ap, use_slack=False)
        fm = gbar @ O.spec_lower(uw.net, k, A, bounds[:k - 1], lo[0], hi[0], am, use_slack=False)
        fd = (fp - fm) / (2 * h)
        assert ga[m][j] == pytest.approx(fd, rel=1e-5, abs=1e-7 * (1 + abs(fd)))
