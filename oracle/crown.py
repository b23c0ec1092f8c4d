"""Plain FP64 CPU oracle for CROWN backward linear bound propagation with alpha and beta.

TEST INFRASTRUCTURE. Only tests/, the smoke check of the package entry file and the
cpu_baseline leg of the bench may import this module.  The HIP library never calls it,
and it shares no code with the HIP library: only the seeded input generators in
``workloads`` serve both.

Everything is computed in float64 (inputs are the float32 weights, boxes, bounds,
alpha and beta, promoted exactly).  Each function follows the paper's Appendix B:

  * the network and the verification problem: the equation defining min f(x) with
    z_i = W_i h_{i-1} + b_i, h_i = ReLU(z_i), x in C                 -> affine()
  * Lemma 1 (ReLU relaxation by the active / inactive / unstable case) -> relax()
  * Theorem 1 (backward recursion for W~ and b~)                       -> backward()
  * Theorem 2 (concretisation; for a box it is exact)                  -> concretize()
  * the intermediate (pre-activation) bound recursion of original CROWN
    described with the early-stop algorithm in Appendix B.2           -> crown_bounds()
Readings where the text is silent or garbled (each is listed in the design notes):
  * Lemma 1 prints both intercept columns under the lower-intercept name; the first is
    the lower intercept (always 0), the second the upper one, -u l / (u - l).
  * Boundary cases: active iff l >= 0, else inactive iff u <= 0, else unstable.
  * Theorem 1's start value "b~(L) = 0" is the accumulator d(L) = 0, b~(L) = A(L) b(L);
    d(l) adds b~(l+1) (as the proof does), not b~(l).
  * A(L) = I generalises to a spec matrix C (rows = specifications).
  * Zero coefficients take the lower relaxation line (either gives the same value).
  * beta: a split sigma*z_j >= 0 clamps l or u, and its Lagrange multiplier beta >= 0
    adds -beta*sigma to the coefficient of z_j (weak duality keeps the bound sound).
  * Intermediate bounds use the adaptive slope alpha_j = 1 if u_j >= -l_j else 0 and
    stay frozen while alpha / beta are optimised.  The paper allows any slope in [0, 1];
    the rule is pinned as the choice in {0, 1} with the smaller relaxed area.
  * FP32 soundness slack: every bound moves outward by KAPPA * 2^-24 * M, where M sums
    the magnitudes of every term of the final dot products; at a split neuron the
    coefficient that multiplies the bias is the relaxed one with the beta term already
    added, |(Lambda - beta sigma) b|.  KAPPA = 64 is a convention, pinned as a margin:
    an FP32 evaluation of the same bound stays within KAPPA / 4 units of 2^-24 M of
    the FP64 raw bound on the test networks.  The raw bound is pinned exactly.
  * Gradient (adjoint) of the raw lower bound w.r.t. alpha and beta: reverse mode of
    backward() + concretize(), with intermediate bounds held fixed.
  * Adam with PyTorch's default moments, followed by projection of alpha to [0, 1] and
    beta to [0, inf).  Optimiser trajectories are compared over three steps on small
    networks (the best bound); longer runs one step at a time at identical alpha / beta,
    since an entry whose gradient is zero up to rounding may step either way.
  * Optimised intermediate bounds (alpha_crown_bounds): every pass that bounds a
    pre-activation layer gets its own slopes, optimised like the final pass's (one slope
    per neuron shared by the lower- and upper-bound rows of that layer), bottom-up; each
    bound is the best over the evaluated passes, which include the default-rule pass.
  * Propagation early stop (Appendix B.2, the early-stop algorithm): the backward
    search ends at an early-stop node and the bound is concretised against that node's
    box.  On a layer chain the node is either the ReLU of layer s (its propagation step
    is skipped, so the bound is linear in h_s and is concretised over
    [ReLU(l_s), ReLU(u_s)]) or the linear node producing z_s (the ReLU of layer s is
    relaxed first, then the bound is concretised over [l_s, u_s]).  The text's worked
    example describes both; both are provided (stop_mode "relu" / "linear").
"""
from __future__ import annotations

import numpy as np

F64 = np.float64
KAPPA = 64.0
U32 = 2.0 ** -24


# --------------------------------------------------------------------------------------
# The network's layers: z = W h + b (Appendix B, the verification problem).
# --------------------------------------------------------------------------------------
def _W(layer):
    return np.asarray(layer["W"], dtype=F64)


def _b(layer):
    return np.asarray(layer["b"], dtype=F64)


def out_dim(layer):
    return int(np.prod(layer["out_shape"]))


def in_dim(layer):
    return int(np.prod(layer["in_shape"]))


def linear_fwd(layer, h):
    """W h for a batch of flat inputs h [n, d_in] -> [n, d_out] (no bias)."""
    h = np.asarray(h, dtype=F64)
    W = _W(layer)
    if layer["kind"] == "linear":
        return h @ W.T
    n = h.shape[0]
    c_in, H, Wd = layer["in_shape"]
    c_out, OH, OW = layer["out_shape"]
    s, p = layer["stride"], layer["pad"]
    kh, kw = W.shape[2], W.shape[3]
    x = np.zeros((n, c_in, H + 2 * p, Wd + 2 * p))
    x[:, :, p:p + H, p:p + Wd] = h.reshape(n, c_in, H, Wd)
    out = np.zeros((n, OH, OW, c_out))
    for ky in range(kh):
        for kx in range(kw):
            patch = x[:, :, ky:ky + s * (OH - 1) + 1:s, kx:kx + s * (OW - 1) + 1:s]
            out += np.tensordot(patch, W[:, :, ky, kx], axes=([1], [1]))
    return out.transpose(0, 3, 1, 2).reshape(n, -1)


def affine(layer, h):
    """z = W h + b."""
    z = linear_fwd(layer, h)
    b = _b(layer)
    if layer["kind"] == "conv":
        b = np.repeat(b, layer["out_shape"][1] * layer["out_shape"][2])
    return z + b


def bias_full(layer):
    """b as a vector over all output neurons (a conv bias repeats over H x W)."""
    b = _b(layer)
    if layer["kind"] == "conv":
        b = np.repeat(b, layer["out_shape"][1] * layer["out_shape"][2])
    return b


def linear_T(layer, lam):
    """lam [R, d_out] -> lam W as [R, d_in]: the product A W of Theorem 1.

    For a convolution this is the transposed convolution with the same stride and
    padding: output pixel (oy, ox) of channel co sends lam * W[co, ci, ky, kx] to input
    pixel (oy*s - p + ky, ox*s - p + kx) of channel ci.
    """
    lam = np.asarray(lam, dtype=F64)
    W = _W(layer)
    if layer["kind"] == "linear":
        return lam @ W
    R = lam.shape[0]
    c_in, H, Wd = layer["in_shape"]
    c_out, OH, OW = layer["out_shape"]
    s, p = layer["stride"], layer["pad"]
    kh, kw = W.shape[2], W.shape[3]
    lam4 = lam.reshape(R, c_out, OH, OW)
    g = np.zeros((R, c_in, H + 2 * p + s, Wd + 2 * p + s))
    for ky in range(kh):
        for kx in range(kw):
            contrib = np.tensordot(lam4, W[:, :, ky, kx], axes=([1], [0]))  # [R,OH,OW,c_in]
            g[:, :, ky:ky + s * (OH - 1) + 1:s, kx:kx + s * (OW - 1) + 1:s] += \
                contrib.transpose(0, 3, 1, 2)
    return g[:, :, p:p + H, p:p + Wd].reshape(R, -1)


def forward(net, x):
    """All pre-activations z_1 .. z_L for a batch of flat inputs x [n, d_0]."""
    zs = []
    h = np.asarray(x, dtype=F64)
    for i, layer in enumerate(net):
        z = affine(layer, h)
        zs.append(z)
        h = np.maximum(z, 0.0)
    return zs


def ibp(net, x_lo, x_hi):
    """Interval arithmetic bounds on z_1 .. z_L for one box (diagnostic only)."""
    lo, hi = np.asarray(x_lo, F64), np.asarray(x_hi, F64)
    out = []
    for i, layer in enumerate(net):
        c, r = (lo + hi) / 2, (hi - lo) / 2
        zc = affine(layer, c[None])[0]
        zr = np.abs(linear_fwd(_abs_layer(layer), r[None])[0])
        out.append((zc - zr, zc + zr))
        lo, hi = np.maximum(zc - zr, 0), np.maximum(zc + zr, 0)
    return out


def _abs_layer(layer):
    d = dict(layer)
    d["W"] = np.abs(_W(layer))
    return d


# --------------------------------------------------------------------------------------
# Lemma 1: linear relaxation of ReLU given l <= z <= u.
# --------------------------------------------------------------------------------------
def relax(l, u, alpha):
    """Return (D_lo, D_up, b_lo, b_up, unstable) as per-neuron vectors."""
    l = np.asarray(l, F64)
    u = np.asarray(u, F64)
    alpha = np.asarray(alpha, F64)
    active = l >= 0
    inactive = (~active) & (u <= 0)
    unstable = (~active) & (~inactive)
    den = np.where(unstable, u - l, 1.0)
    D_lo = np.where(active, 1.0, np.where(inactive, 0.0, alpha))
    D_up = np.where(active, 1.0, np.where(inactive, 0.0, u / den))
    b_lo = np.zeros_like(l)
    b_up = np.where(unstable, -u * l / den, 0.0)
    return D_lo, D_up, b_lo, b_up, unstable


def adaptive_alpha(l, u):
    """Default lower slope for plain CROWN: 1 where u >= -l, else 0."""
    return np.where(np.asarray(u, F64) >= -np.asarray(l, F64), 1.0, 0.0)


def clamp_splits(bounds, splits):
    """Apply split constraints sigma*z_j >= 0 to the (l, u) of their layer.

    bounds: list of (l_m, u_m) for ReLU layers m = 1..; splits: list of (m, j, sigma)
    with m 1-based.  Returns new bounds and whether every box is still non-empty.
    """
    out = [(np.array(l, F64), np.array(u, F64)) for (l, u) in bounds]
    for (m, j, sg) in splits:
        l, u = out[m - 1]
        if sg > 0:
            l[j] = max(l[j], 0.0)
        else:
            u[j] = min(u[j], 0.0)
    feasible = all(bool(np.all(l <= u)) for (l, u) in out)
    return out, feasible


# --------------------------------------------------------------------------------------
# Theorem 1: backward propagation of the linear lower bound.
# --------------------------------------------------------------------------------------
def backward(net, k, A, bounds, alpha=None, splits=(), beta=None, tape=None):
    """Propagate coefficient rows A [R, d_k] on z_k back to the input.

    bounds: (l_m, u_m) for m = 1..k-1 (already clamped by the splits);
    alpha:  list of per-layer vectors for m = 1..k-1, or None for the adaptive rule;
    splits: (m, j, sigma) triples; beta: [len(splits), R] multipliers (None -> 0).
    Returns (Wt1 [R, d_0], bt1 [R], mag [R]) with z_k-coefficients satisfying
    A z_k >= Wt1 x + bt1 on the box, and mag = sum of |offset terms| (for the slack).
    If tape is a list, per-layer values needed by the adjoint are appended to it.
    """
    A = np.asarray(A, F64)
    layer = net[k - 1]
    Wt = linear_T(layer, A)
    bfull = bias_full(layer)
    bt = A @ bfull
    mag = np.abs(A) @ np.abs(bfull)
    for m in range(k - 1, 0, -1):
        l, u = bounds[m - 1]
        a_m = adaptive_alpha(l, u) if alpha is None else alpha[m - 1]
        D_lo, D_up, b_lo, b_up, unstable = relax(l, u, a_m)
        pos = Wt >= 0
        Am = np.where(pos, Wt * D_lo, Wt * D_up)
        off = np.where(pos, Wt * b_lo, Wt * b_up)
        d = off.sum(axis=1) + bt
        mag = mag + np.abs(off).sum(axis=1)
        for q, (ms, j, sg) in enumerate(splits):
            if ms == m and beta is not None:
                Am[:, j] -= np.asarray(beta[q], F64) * sg
        if tape is not None:
            tape.append(dict(m=m, Wt=Wt, D_lo=D_lo, D_up=D_up, b_up=b_up,
                             unstable=unstable))
        layer = net[m - 1]
        bfull = bias_full(layer)
        Wt = linear_T(layer, Am)
        bt = Am @ bfull + d
        mag = mag + np.abs(Am) @ np.abs(bfull)
    return Wt, bt, mag


# --------------------------------------------------------------------------------------
# Theorem 2: concretisation over the input box (exact for a box).
# --------------------------------------------------------------------------------------
def concretize(Wt, bt, x_lo, x_hi):
    x_lo = np.asarray(x_lo, F64)
    x_hi = np.asarray(x_hi, F64)
    c = (x_lo + x_hi) / 2
    r = (x_hi - x_lo) / 2
    return Wt @ c - np.abs(Wt) @ r + bt


def slack(Wt, mag, x_lo, x_hi, kappa=KAPPA):
    """Outward FP32 rounding allowance kappa * 2^-24 * M for each bound."""
    x_lo = np.asarray(x_lo, F64)
    x_hi = np.asarray(x_hi, F64)
    c = (x_lo + x_hi) / 2
    r = (x_hi - x_lo) / 2
    M = np.abs(Wt) @ (np.abs(c) + r) + mag
    return kappa * U32 * M


def spec_lower(net, k, A, bounds, x_lo, x_hi, alpha=None, splits=(), beta=None,
               use_slack=True):
    """Lower bound of each row of A z_k over the box (one instance)."""
    cb, feasible = clamp_splits(bounds, splits)
    if not feasible:
        return np.full(np.asarray(A).shape[0], np.inf)
    Wt, bt, mag = backward(net, k, A, cb, alpha, splits, beta)
    lower = concretize(Wt, bt, x_lo, x_hi)
    if use_slack:
        lower = lower - slack(Wt, mag, x_lo, x_hi)
    return lower


def crown_bounds(net, x_lo, x_hi, use_slack=True, chunk=4096):
    """Full CROWN pre-activation bounds (l_m, u_m), m = 1..L-1, for one box.

    Each z_k is bounded by a backward pass with rows [I; -I] down to the input, using
    the bounds of the layers below (so the total work is quadratic in depth).
    Rows are independent; they are processed in chunks only to bound memory.
    """
    bounds = []
    for k in range(1, len(net)):
        d = out_dim(net[k - 1])
        lo = np.empty(d)
        hi = np.empty(d)
        for a in range(0, d, chunk):
            b = min(d, a + chunk)
            I = np.zeros((b - a, d))
            I[np.arange(b - a), np.arange(a, b)] = 1.0
            lo[a:b] = spec_lower(net, k, I, bounds, x_lo, x_hi, use_slack=use_slack)
            hi[a:b] = -spec_lower(net, k, -I, bounds, x_lo, x_hi, use_slack=use_slack)
        bounds.append((lo, hi))
    return bounds


def alpha_crown_bounds(net, x_lo, x_hi, steps=5, lr=0.1, alpha0=0.5, use_slack=True):
    """Pre-activation bounds (l_m, u_m), m = 1..L-1, for one box, with the slopes of every
    intermediate pass optimised (the relaxation's alpha is free for any bound, Lemma 1).

    Layers are bounded bottom-up.  For z_k the rows are [I; -I] (lower bounds of z_k and
    of -z_k).  First the pass with the default slope rule and the bounds found so far;
    then `steps` projected Adam steps (lr, PyTorch's default moments) on the slopes of
    layers 1..k-1, one slope per neuron shared by all rows of this target layer, starting
    at alpha0 and maximising the sum of the rows' lower bounds; then one more pass.  Each
    neuron keeps the best of the steps + 2 passes.  Layer 1 is exact (no ReLU below)."""
    bounds = []
    for k in range(1, len(net)):
        d = out_dim(net[k - 1])
        A = np.concatenate([np.eye(d), -np.eye(d)])
        best = spec_lower(net, k, A, bounds, x_lo, x_hi, None, use_slack=use_slack)
        if k > 1 and steps > 0:
            alpha = [np.full(len(l), float(alpha0)) for (l, _) in bounds]
            ma = [np.zeros(len(l)) for (l, _) in bounds]
            va = [np.zeros(len(l)) for (l, _) in bounds]
            for t in range(1, steps + 1):
                best = np.maximum(best, spec_lower(net, k, A, bounds, x_lo, x_hi, alpha,
                                                   use_slack=use_slack))
                _, ga, _ = spec_lower_grad(net, k, A, bounds, x_lo, x_hi, alpha)
                for i in range(len(alpha)):
                    alpha[i], ma[i], va[i] = adam_step(alpha[i], -ga[i], ma[i], va[i], t, lr,
                                                       lo=0.0, hi=1.0)
            best = np.maximum(best, spec_lower(net, k, A, bounds, x_lo, x_hi, alpha,
                                               use_slack=use_slack))
        bounds.append((best[:d], -best[d:]))
    return bounds


def crown(net, C, x_lo, x_hi, use_slack=True):
    """Full CROWN: intermediate bounds, then lower and upper bounds of C f(x)."""
    bounds = crown_bounds(net, x_lo, x_hi, use_slack)
    L = len(net)
    lower = spec_lower(net, L, C, bounds, x_lo, x_hi, use_slack=use_slack)
    upper = -spec_lower(net, L, -np.asarray(C, F64), bounds, x_lo, x_hi,
                        use_slack=use_slack)
    return bounds, lower, upper


# --------------------------------------------------------------------------------------
# Propagation early stop (Appendix B.2).
# --------------------------------------------------------------------------------------
def backward_to(net, k, A, bounds, stop, mode, alpha=None, splits=(), beta=None):
    """Theorem 1's recursion from z_k down to the early-stop node of layer `stop`.

    mode "relu":   stop before relaxing z_stop; returns (coefficients on h_stop, offset,
                   mag).
    mode "linear": relax z_stop (Lemma 1, alpha, beta) and stop; returns (coefficients on
                   z_stop, offset, mag).
    """
    A = np.asarray(A, F64)
    layer = net[k - 1]
    Wt = linear_T(layer, A)
    bfull = bias_full(layer)
    bt = A @ bfull
    mag = np.abs(A) @ np.abs(bfull)
    for m in range(k - 1, stop - 1, -1):
        if mode == "relu" and m == stop:
            return Wt, bt, mag
        l, u = bounds[m - 1]
        a_m = adaptive_alpha(l, u) if alpha is None else alpha[m - 1]
        D_lo, D_up, b_lo, b_up, _ = relax(l, u, a_m)
        pos = Wt >= 0
        Am = np.where(pos, Wt * D_lo, Wt * D_up)
        off = np.where(pos, Wt * b_lo, Wt * b_up)
        bt = off.sum(axis=1) + bt
        mag = mag + np.abs(off).sum(axis=1)
        for q, (ms, j, sg) in enumerate(splits):
            if ms == m and beta is not None:
                Am[:, j] -= np.asarray(beta[q], F64) * sg
        if m == stop:
            return Am, bt, mag
        layer = net[m - 1]
        bfull = bias_full(layer)
        Wt = linear_T(layer, Am)
        bt = Am @ bfull + bt
        mag = mag + np.abs(Am) @ np.abs(bfull)
    raise ValueError("stop layer must be in 1..k-1")


def spec_lower_early_stop(net, k, A, bounds, stop, mode, alpha=None, splits=(), beta=None,
                          use_slack=True):
    """Lower bound of A z_k with the backward pass stopped at layer `stop`, concretised
    over that node's box (Theorem 2 with the node in place of the input)."""
    cb, feasible = clamp_splits(bounds, splits)
    if not feasible:
        return np.full(np.asarray(A).shape[0], np.inf)
    Wt, bt, mag = backward_to(net, k, A, cb, stop, mode, alpha, splits, beta)
    l, u = cb[stop - 1]
    if mode == "relu":
        l, u = np.maximum(l, 0.0), np.maximum(u, 0.0)
    lower = concretize(Wt, bt, l, u)
    if use_slack:
        lower = lower - slack(Wt, mag, l, u)
    return lower


def sample_bounds(net, samples):
    """Search-integrated (empirical) pre-activation bounds of one subdomain (Section 3.2,
    approach 2): per neuron of z_1 .. z_{L-1}, the min and max over the sample inputs."""
    zs = forward(net, samples)
    return [(z.min(axis=0), z.max(axis=0)) for z in zs[:-1]]


# --------------------------------------------------------------------------------------
# Adjoint: gradient of the raw lower bound w.r.t. alpha and beta.
# --------------------------------------------------------------------------------------
def spec_lower_grad(net, k, A, bounds, x_lo, x_hi, alpha, splits=(), beta=None,
                    gbar=None, stop=0, mode=None):
    """Return (lower_raw [R], d(sum_r gbar_r lower_r)/d alpha (list per layer),
    d(...)/d beta [nnz, R]).  gbar defaults to ones.  With stop > 0 the bound is the
    early-stop bound of spec_lower_early_stop(stop, mode)."""
    A = np.asarray(A, F64)
    R = A.shape[0]
    cb, feasible = clamp_splits(bounds, splits)
    nnz = len(splits)
    if not feasible:
        return (np.full(R, np.inf), [np.zeros(len(l)) for (l, _) in bounds[:k - 1]],
                np.zeros((nnz, R)))
    tape = []
    if stop > 0:
        Wt1, bt1 = _backward_taped(net, k, A, cb, alpha, splits, beta, tape, stop, mode)
        l, u = cb[stop - 1]
        if mode == "relu":
            l, u = np.maximum(l, 0.0), np.maximum(u, 0.0)
        x_lo, x_hi = l, u
    else:
        Wt1, bt1, _ = backward(net, k, A, cb, alpha, splits, beta, tape=tape)
    lower = concretize(Wt1, bt1, x_lo, x_hi)
    gbar = np.ones(R) if gbar is None else np.asarray(gbar, F64)
    x_lo = np.asarray(x_lo, F64)
    x_hi = np.asarray(x_hi, F64)
    c, r = (x_lo + x_hi) / 2, (x_hi - x_lo) / 2
    # d lower_r / d Wt1[r, j] = c_j - sign(Wt1[r, j]) r_j ; d lower / d bt1 = 1.
    Wbar = gbar[:, None] * (c[None, :] - np.sign(Wt1) * r[None, :])
    bbar = gbar.copy()
    g_alpha = [np.zeros(len(l)) for (l, _) in cb[:k - 1]]
    g_beta = np.zeros((nnz, R))
    first = True
    for rec in reversed(tape):           # m = lowest, ..., k-1
        m = rec["m"]
        if first and stop > 0 and mode == "linear":
            Abar = Wbar                  # the concretised coefficients are A_stop itself
        else:
            layer = net[m - 1]
            # Wt_m = A_m W_m and bt_m = A_m b_m + d_m  ->  A_m bar:
            Abar = linear_fwd(layer, Wbar) + bbar[:, None] * bias_full(layer)[None, :]
        first = False
        for q, (ms, j, sg) in enumerate(splits):
            if ms == m and beta is not None:
                g_beta[q] += -sg * Abar[:, j]
        Wt = rec["Wt"]
        pos = Wt >= 0
        # A_m = where(pos, Wt D_lo, Wt D_up); alpha enters D_lo at unstable neurons.
        g_alpha[m - 1] += np.sum(np.where(pos & rec["unstable"][None, :], Wt * Abar, 0.0),
                                 axis=0)
        # d_m = sum_j where(pos, 0, Wt b_up) + bt_{m+1}
        Wbar = Abar * np.where(pos, rec["D_lo"][None, :], rec["D_up"][None, :]) + \
            bbar[:, None] * np.where(pos, 0.0, rec["b_up"][None, :])
    return lower, g_alpha, g_beta


def _backward_taped(net, k, A, bounds, alpha, splits, beta, tape, stop, mode):
    """backward_to with the per-layer values the adjoint needs appended to tape."""
    A = np.asarray(A, F64)
    layer = net[k - 1]
    Wt = linear_T(layer, A)
    bt = A @ bias_full(layer)
    for m in range(k - 1, stop - 1, -1):
        if mode == "relu" and m == stop:
            return Wt, bt
        l, u = bounds[m - 1]
        a_m = adaptive_alpha(l, u) if alpha is None else alpha[m - 1]
        D_lo, D_up, b_lo, b_up, unstable = relax(l, u, a_m)
        pos = Wt >= 0
        Am = np.where(pos, Wt * D_lo, Wt * D_up)
        bt = np.where(pos, Wt * b_lo, Wt * b_up).sum(axis=1) + bt
        for q, (ms, j, sg) in enumerate(splits):
            if ms == m and beta is not None:
                Am[:, j] -= np.asarray(beta[q], F64) * sg
        tape.append(dict(m=m, Wt=Wt, D_lo=D_lo, D_up=D_up, b_up=b_up, unstable=unstable))
        if m == stop:
            return Am, bt
        layer = net[m - 1]
        Wt = linear_T(layer, Am)
        bt = Am @ bias_full(layer) + bt
    raise ValueError("stop layer must be in 1..k-1")


# --------------------------------------------------------------------------------------
# Optimiser step (Adam, PyTorch default moments) and projection.
# --------------------------------------------------------------------------------------
def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, lo=None, hi=None):
    """One Adam step minimising a loss with gradient g; returns (p, m, v)."""
    p, g, m, v = (np.asarray(a, F64) for a in (p, g, m, v))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    if lo is not None or hi is not None:
        p = np.clip(p, lo, hi)
    return p, m, v


def optimize_alpha_beta(net, A, bounds, x_lo, x_hi, splits=(), steps=10, lr=0.1,
                        alpha0=0.5, use_beta=True):
    """alpha / beta optimisation of the final spec bound (loss = -sum of lower bounds).

    Returns (best lower per row over steps 0..T, with slack; final alpha; final beta).
    """
    k = len(net)
    R = np.asarray(A).shape[0]
    dims = [len(l) for (l, _) in bounds]
    alpha = [np.full(d, alpha0) for d in dims]
    beta = np.zeros((len(splits), R)) if use_beta else None
    ma = [np.zeros(d) for d in dims]
    va = [np.zeros(d) for d in dims]
    mb = np.zeros((len(splits), R))
    vb = np.zeros((len(splits), R))
    best = np.full(R, -np.inf)
    for t in range(1, steps + 1):
        low = spec_lower(net, k, A, bounds, x_lo, x_hi, alpha, splits, beta)
        best = np.maximum(best, low)
        _, ga, gb = spec_lower_grad(net, k, A, bounds, x_lo, x_hi, alpha, splits, beta)
        for i in range(len(dims)):
            alpha[i], ma[i], va[i] = adam_step(alpha[i], -ga[i], ma[i], va[i], t, lr,
                                               lo=0.0, hi=1.0)
        if use_beta and len(splits):
            beta, mb, vb = adam_step(beta, -gb, mb, vb, t, lr, lo=0.0, hi=None)
    low = spec_lower(net, k, A, bounds, x_lo, x_hi, alpha, splits, beta)
    best = np.maximum(best, low)
    return best, alpha, beta


# --------------------------------------------------------------------------------------
# Helpers for the flat (all-ReLU-layers) layouts used at the library boundary.
# --------------------------------------------------------------------------------------
def relu_offsets(net):
    off = [0]
    for layer in net[:-1]:
        off.append(off[-1] + out_dim(layer))
    return off


def split_list(net, neuron, sign):
    """Global ReLU indices + signs -> (m, j, sigma) triples (m 1-based)."""
    off = relu_offsets(net)
    out = []
    for g, s in zip(np.asarray(neuron).tolist(), np.asarray(sign).tolist()):
        m = int(np.searchsorted(off, g, side="right"))
        out.append((m, int(g - off[m - 1]), int(s)))
    return out


def per_layer(net, flat):
    off = relu_offsets(net)
    flat = np.asarray(flat, F64)
    return [flat[off[i]:off[i + 1]] for i in range(len(off) - 1)]
