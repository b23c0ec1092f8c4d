"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the bench.

This module only draws inputs: network weights, input points, perturbation boxes,
margin specifications and random ReLU split constraints.  It contains none of the
bound-propagation arithmetic; the FP64 oracle and the HIP library each implement that
on their own.

Networks follow the layer definition of the paper's verification problem (Appendix B,
the equation defining min f(x) subject to z_i = W_i h_{i-1} + b_i, h_i = ReLU(z_i)):
a chain of Linear / Conv2d layers with a ReLU after every layer but the last.
Everything is generated in float64 by ``numpy.random.default_rng`` and cast to float32.

Layer dicts (the one network description every consumer reads):
    kind     'linear' or 'conv'
    W        float32, linear: [d_out, d_in]; conv: [C_out, C_in, kh, kw]
    b        float32, linear: [d_out];        conv: [C_out]
    in_shape (C, H, W) for conv, (d_in,) for linear
    out_shape(C, H, W) for conv, (d_out,) for linear
    stride, pad  (conv only)
Flattening between a conv layer and a following linear layer is C-major (NCHW).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

WEIGHT_SEED = 0
INPUT_SEED = 1
SPLIT_SEED = 2
BIAS_STD = 0.1


def _linear(rng, d_in, d_out, bias=True):
    W = rng.normal(0.0, math.sqrt(2.0 / d_in), size=(d_out, d_in))
    b = rng.normal(0.0, BIAS_STD, size=(d_out,)) if bias else np.zeros(d_out)
    return {"kind": "linear", "W": W.astype(np.float32), "b": b.astype(np.float32),
            "in_shape": (d_in,), "out_shape": (d_out,)}


def _conv(rng, in_shape, c_out, k, stride, pad, bias=True):
    c_in, h, w = in_shape
    fan_in = c_in * k * k
    W = rng.normal(0.0, math.sqrt(2.0 / fan_in), size=(c_out, c_in, k, k))
    b = rng.normal(0.0, BIAS_STD, size=(c_out,)) if bias else np.zeros(c_out)
    oh = (h + 2 * pad - k) // stride + 1
    ow = (w + 2 * pad - k) // stride + 1
    return {"kind": "conv", "W": W.astype(np.float32), "b": b.astype(np.float32),
            "in_shape": (c_in, h, w), "out_shape": (c_out, oh, ow),
            "stride": stride, "pad": pad}


def mlp(dims, seed=WEIGHT_SEED, bias=True):
    """ReLU MLP with He-normal weights; dims = [d_0, d_1, ..., d_L]."""
    rng = np.random.default_rng(seed)
    return [_linear(rng, dims[i], dims[i + 1], bias) for i in range(len(dims) - 1)]


def cnn(seed=WEIGHT_SEED, bias=True, spec=None, in_shape=(3, 32, 32), fc=(512, 10)):
    """ReLU CNN; spec is a list of (C_out, k, stride) conv layers, padding 1 each."""
    if spec is None:
        spec = [(16, 3, 1), (32, 4, 2), (32, 3, 1), (64, 4, 2)]
    rng = np.random.default_rng(seed)
    layers = []
    shape = tuple(in_shape)
    for c_out, k, s in spec:
        layers.append(_conv(rng, shape, c_out, k, s, 1, bias))
        shape = layers[-1]["out_shape"]
    d = int(np.prod(shape))
    for width in fc:
        layers.append(_linear(rng, d, width, bias))
        d = width
    return layers


def in_dim(net):
    return int(np.prod(net[0]["in_shape"]))


def out_dim(layer):
    return int(np.prod(layer["out_shape"]))


def relu_dims(net):
    """Widths of the ReLU layers z_1 .. z_{L-1}."""
    return [out_dim(l) for l in net[:-1]]


def uniform_inputs(n, d, seed=INPUT_SEED):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n, d)).astype(np.float32)


def linf_box(x0, eps):
    """Per-dimension box fl32(x0 - eps), fl32(x0 + eps); not clipped to [0, 1]."""
    x = x0.astype(np.float64)
    return (x - eps).astype(np.float32), (x + eps).astype(np.float32)


def clean_logits(net, x):
    """Plain float64 forward pass of the network (used only to pick the margin label)."""
    import torch
    import torch.nn.functional as F
    h = torch.from_numpy(np.asarray(x, dtype=np.float64))
    n = h.shape[0]
    for i, layer in enumerate(net):
        W = torch.from_numpy(layer["W"].astype(np.float64))
        b = torch.from_numpy(layer["b"].astype(np.float64))
        if layer["kind"] == "conv":
            h = F.conv2d(h.reshape(n, *layer["in_shape"]), W, b,
                         stride=layer["stride"], padding=layer["pad"]).reshape(n, -1)
        else:
            h = h.reshape(n, -1) @ W.T + b
        if i + 1 < len(net):
            h = torch.clamp(h, min=0.0)
    return h.numpy()


def margin_spec(logits):
    """Rows e_y - e_j for every j != y (ascending), y = argmax (lowest index on ties)."""
    n, k = logits.shape
    C = np.zeros((n, k - 1, k), dtype=np.float32)
    y = np.argmax(logits, axis=1)
    for i in range(n):
        others = [j for j in range(k) if j != y[i]]
        for r, j in enumerate(others):
            C[i, r, y[i]] = 1.0
            C[i, r, j] = -1.0
    return C


@dataclass
class Splits:
    """CSR list of ReLU split constraints sigma * z_j >= 0 per subdomain.

    off    int32 [n+1]
    neuron int32 [nnz]  global ReLU index (layer offset + C-major neuron index)
    sign   int8  [nnz]  +1 (z >= 0) or -1 (z <= 0)
    """
    off: np.ndarray
    neuron: np.ndarray
    sign: np.ndarray
    root: np.ndarray = field(default=None)

    @property
    def n(self):
        return len(self.off) - 1

    @property
    def nnz(self):
        return int(self.off[-1])


def random_splits(candidates, n_sub, kmin=1, kmax=12, seed=SPLIT_SEED, root_of=None):
    """Per subdomain: k ~ U{kmin..kmax} distinct neurons from its candidate set, sign ~ U{+-1}.

    candidates: list (one per root) of int arrays of global ReLU indices eligible for a split.
    root_of:    int array [n_sub] selecting each subdomain's root (default: round robin).
    """
    rng = np.random.default_rng(seed)
    if root_of is None:
        root_of = np.arange(n_sub) % len(candidates)
    off = [0]
    neuron, sign = [], []
    for s in range(n_sub):
        cand = np.asarray(candidates[root_of[s]])
        k = int(rng.integers(kmin, kmax + 1))
        k = min(k, len(cand))
        pick = rng.choice(cand, size=k, replace=False) if k > 0 else np.zeros(0, np.int64)
        sg = rng.choice(np.array([-1, 1]), size=k)
        order = np.argsort(pick, kind="stable")
        neuron.extend(pick[order].tolist())
        sign.extend(sg[order].tolist())
        off.append(len(neuron))
    return Splits(np.asarray(off, np.int32), np.asarray(neuron, np.int32),
                  np.asarray(sign, np.int8), np.asarray(root_of, np.int32))


def random_alpha(n, n_relu, seed=3):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n, n_relu)).astype(np.float32)


def random_beta(nnz, rows, seed=4, scale=0.5):
    rng = np.random.default_rng(seed)
    return (scale * rng.uniform(0.0, 1.0, size=(nnz, rows))).astype(np.float32)


# --------------------------------------------------------------------------------------
# The five workloads, by what they are.
# --------------------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    net: list
    x0: np.ndarray
    x_lo: np.ndarray
    x_hi: np.ndarray
    spec: np.ndarray
    eps: float
    extra: dict = field(default_factory=dict)


def _make(name, net, n, eps, seed_in=INPUT_SEED, **extra):
    x0 = uniform_inputs(n, in_dim(net), seed_in)
    x_lo, x_hi = linf_box(x0, eps)
    spec = margin_spec(clean_logits(net, x0))
    return Workload(name, net, x0, x_lo, x_hi, spec, eps, dict(extra))


def mlp_small():
    """MLP 784-100-100-10, 1 input, eps 0.02, plain CROWN."""
    return _make("mlp784-100-100-10_n1_eps0.02", mlp([784, 100, 100, 10]), 1, 0.02)


def mlp_deep(n=256):
    """MLP 784-256x6-10, batch 256, eps 0.015, full CROWN."""
    return _make(f"mlp784-256x6-10_n{n}_eps0.015", mlp([784] + [256] * 6 + [10]), n, 0.015)


def cnn_cifar(n=64):
    """CNN 3x32x32: c16k3s1, c32k4s2, c32k3s1, c64k4s2, FC 4096-512-10; eps 2/255."""
    return _make(f"cnn4c2f_n{n}_eps2/255", cnn(), n, 2.0 / 255.0)


def alpha_cnn(n=64):
    """alpha-CROWN on the CNN: alpha = 0.5, 20 Adam steps at lr 0.1."""
    w = cnn_cifar(n)
    w.name = f"alpha-crown_cnn_n{n}_steps20"
    w.extra.update(steps=20, lr=0.1, alpha0=0.5)
    return w


def beta_cnn(n_roots=64, per_root=64):
    """beta-CROWN BaB batch on the CNN: n_roots*per_root subdomains, 1-12 splits each."""
    w = cnn_cifar(n_roots)
    w.name = f"beta-crown_cnn_{n_roots}x{per_root}_steps10"
    w.extra.update(steps=10, lr=0.1, alpha0=0.5, per_root=per_root, kmin=1, kmax=12)
    return w


# ----------------------------------------------------------------- planning (BaB) inputs
PLAN_SEED = 3


def plan_objective(d=8, hidden=(64, 64), seed=WEIGHT_SEED):
    """A scalar ReLU objective f(u) over an action box (stands in for the paper's cost of
    unrolled learned dynamics, which is not available): MLP d -> hidden -> 1, He-normal
    weights.  Returns the net and the box [-1, 1]^d."""
    net = mlp([d, *hidden, 1], seed=seed)
    return net, -np.ones(d, np.float32), np.ones(d, np.float32)


def plan_uniforms(seed=PLAN_SEED):
    """uniforms(tag, shape): float32 uniforms in [0, 1) for the planning loop's random
    draws, one independent stream per tag ('search0', ('search', t), ('pick', t))."""
    def code(tag):
        if tag == "search0":
            return 0
        kind, t = tag
        return 1 + 2 * int(t) + (0 if kind == "search" else 1)

    def draw(tag, shape):
        rng = np.random.default_rng([seed, code(tag)])
        return rng.random(shape, dtype=np.float64).astype(np.float32)

    return draw


def plan_gumbels(seed=PLAN_SEED):
    """gumbels(tag, shape): float32 standard Gumbel variates -log(-log U) for the
    planning loop's pick-out, from the uniform streams of plan_uniforms (tag ('pick', t)),
    formed in float64 before the cast."""
    def draw(tag, shape):
        kind, t = tag
        if kind != "pick":
            raise ValueError("Gumbel variates are drawn for the pick-out only")
        rng = np.random.default_rng([seed, 1 + 2 * int(t) + 1])
        u = np.clip(rng.random(shape, dtype=np.float64), 1e-300, 1.0)
        return (-np.log(-np.log(u))).astype(np.float32)

    return draw


def plan_normals(seed=PLAN_SEED):
    """normals(tag, shape): float32 standard normals for the CEM rounds of the planning
    loop's search, one independent stream per tag (('cem0', r) for the root's round r,
    ('cem', t, r) for round r of iteration t's children)."""
    def code(tag):
        if tag[0] == "cem0":
            return (1 << 20) + int(tag[1])
        _, t, r = tag
        return (2 << 20) + (int(t) << 8) + int(r)

    def draw(tag, shape):
        rng = np.random.default_rng([seed, code(tag)])
        return rng.standard_normal(shape, dtype=np.float64).astype(np.float32)

    return draw


# ----------------------------------------------------------------- unrolled dynamics model
PUSH_DIMS = (10, 128, 256, 256, 128, 8)   # state 8 (four keypoints, 2-D) + action 2 -> state 8
PUSH_PASS = 1.0                           # pass-through offset (see pushing_unrolled)


@dataclass
class Unrolled:
    """A dynamics MLP unrolled over a planning horizon as one ReLU layer chain.

    net      layer dicts of the chain (input: the H actions, 2H values)
    mlp      layer dicts of the dynamics MLP itself
    x0       initial state [8]; target [8]
    u_lo, u_hi  the action box [2H] (the root domain of the planner)
    H        horizon
    """
    net: list
    mlp: list
    x0: np.ndarray
    target: np.ndarray
    u_lo: np.ndarray
    u_hi: np.ndarray
    H: int


def pushing_mlp(seed=WEIGHT_SEED):
    """The Pushing-with-Obstacles dynamics model's shape: MLP 10-128-256-256-128-8 (134,152
    parameters), He-normal weights from seed (trained weights are not available)."""
    return mlp(list(PUSH_DIMS), seed=seed)


def pushing_unrolled(H=20, seed=WEIGHT_SEED, state_seed=5, u_bound=1.0):
    """f(u) = sum_j |x_H - target|_j with x_{t+1} = MLP(x_t, u_t), as a ReLU layer chain.

    The objective is the L1 step cost at the horizon, written with ReLUs
    (|y| = ReLU(y) + ReLU(-y)), so the whole objective is a chain of Linear layers with a
    ReLU after every layer but the last:

      * step t's first layer reads x_t and u_t.  For t > 0, x_t = W5 h + b5 is the
        previous step's last (linear) layer, so that layer and this one are composed
        into one linear layer (no ReLU lies between them);
      * actions not yet used are carried through the ReLU layers as pass-through neurons
        v = u - u_lo + PUSH_PASS >= PUSH_PASS > 0 (identity rows; ReLU(v) = v on the
        box), and read back as u = v + u_lo - PUSH_PASS where they enter;
      * after the last step, the layer [W5; -W5] h + [b5 - target; target - b5] gives the
        16 values +-(x_H - target), a ReLU, and a final layer of ones sums them.

    Layers: 4 H + 2 (4 H + 1 ReLU layers); input 2 H.  Composed weights are formed in
    float64 and rounded to float32 once.
    """
    m = pushing_mlp(seed)
    W = [l["W"].astype(np.float64) for l in m]
    b = [l["b"].astype(np.float64) for l in m]
    rng = np.random.default_rng(state_seed)
    x0 = rng.uniform(-1.0, 1.0, 8)
    target = rng.uniform(-1.0, 1.0, 8)
    nu = 2 * H
    u_lo = -u_bound * np.ones(nu)
    u_hi = u_bound * np.ones(nu)
    W1x, W1u = W[0][:, :8], W[0][:, 8:]
    layers = []

    def add(Wm, bm):
        Wm = np.asarray(Wm)
        layers.append({"kind": "linear", "W": Wm.astype(np.float32), "b": np.asarray(bm).astype(np.float32),
                       "in_shape": (Wm.shape[1],), "out_shape": (Wm.shape[0],)})

    def pass_rows(first_action, n_in, col_of):
        """Identity rows carrying actions first_action .. H-1 (2 values each)."""
        rows = []
        for a in range(first_action, H):
            for c in range(2):
                r = np.zeros(n_in)
                r[col_of(a, c)] = 1.0
                rows.append(r)
        return np.array(rows).reshape(-1, n_in)

    # step 0, first layer: input u (2H)
    P = 2 * (H - 1)
    top = np.zeros((128, nu))
    top[:, 0:2] = W1u
    rows = pass_rows(1, nu, lambda a, c: 2 * a + c)
    Wm = np.vstack([top, rows])
    bm = np.concatenate([W1x @ x0 + b[0], (PUSH_PASS - u_lo[2:])])
    add(Wm, bm)
    for t in range(H):
        P = 2 * (H - 1 - t)                      # actions carried after step t's first layer
        # layers 2..4 of step t: hidden plus the carried actions
        for k in (1, 2, 3):
            d_in, d_out = W[k].shape[1], W[k].shape[0]
            Wm = np.zeros((d_out + P, d_in + P))
            Wm[:d_out, :d_in] = W[k]
            Wm[d_out:, d_in:] = np.eye(P)
            add(Wm, np.concatenate([b[k], np.zeros(P)]))
        if t + 1 < H:
            # W5 of step t composed with W1 of step t + 1; u_{t+1} from its carried values
            Pn = P - 2
            Wm = np.zeros((128 + Pn, 128 + P))
            Wm[:128, :128] = W1x @ W[4]
            Wm[:128, 128:130] = W1u
            if Pn:
                Wm[128:, 130:] = np.eye(Pn)
            ua = u_lo[2 * (t + 1):2 * (t + 1) + 2]
            bm = np.concatenate([W1x @ b[4] + b[0] + W1u @ (ua - PUSH_PASS), np.zeros(Pn)])
            add(Wm, bm)
    add(np.vstack([W[4], -W[4]]), np.concatenate([b[4] - target, target - b[4]]))
    add(np.ones((1, 16)), np.zeros(1))
    return Unrolled(layers, m, x0, target, u_lo, u_hi, H)


def rollout_cost(u_seq, uw):
    """The same objective by stepping the dynamics MLP in float64: u_seq [n, 2H]."""
    u = np.asarray(u_seq, np.float64)
    n = u.shape[0]
    x = np.repeat(uw.x0[None], n, 0)
    for t in range(uw.H):
        h = np.concatenate([x, u[:, 2 * t:2 * t + 2]], axis=1)
        for i, l in enumerate(uw.mlp):
            h = h @ l["W"].astype(np.float64).T + l["b"].astype(np.float64)
            if i + 1 < len(uw.mlp):
                h = np.maximum(h, 0.0)
        x = h
    return np.abs(x - uw.target).sum(axis=1)


def action_subboxes(uw, n, seed=6, width=(0.05, 0.4)):
    """n random sub-boxes of the action box (planning subdomains): per coordinate a
    width drawn uniformly from `width` (fractions of the box) at a uniform position."""
    rng = np.random.default_rng(seed)
    span = uw.u_hi - uw.u_lo
    w = rng.uniform(width[0], width[1], (n, span.size)) * span
    lo = uw.u_lo + rng.uniform(0.0, 1.0, (n, span.size)) * (span - w)
    return lo.astype(np.float32), (lo + w).astype(np.float32)
