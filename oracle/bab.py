"""Plain CPU oracle for the branch-and-bound planning loop over input boxes: the loop of
Algorithms 1-2, the subdomain pick-out and split heuristics of Section 3.1 (Eq. lf_pick),
the search summary (Section 3.3) and the pruner (Section 3).

TEST INFRASTRUCTURE. Only tests/, the smoke check of the package entry file and the
cpu_baseline leg of the bench may import this module.  The HIP library never calls it,
and it shares no code with the HIP library: only the seeded input generators in
``workloads`` serve both.  Random numbers the method draws (Gumbel variates for the
pick-out, uniforms or normals for the search samples) are inputs.

Readings where the text leaves a choice (each is listed in the design notes):
  * batch_pick_out: n = min(n, |P|) and n1 = floor(eta * n) (in double precision).
    The first n1 picks are the subdomains with the smallest upper bound f_hi (ties:
    lower index).  The other n - n1 are drawn without replacement from the rest with
    p_i proportional to exp(-s_i / T), s_i = (f_lo_i - min) / (max - min) over the rest
    (min-max scaling; s = 0 when max = min).  Drawing without replacement uses the
    Gumbel-top-k construction -- the n - n1 largest of -s_i / T + G_i with G_i supplied
    standard Gumbel variates (ties: lower index) -- which yields the ordered sample of
    successive softmax draws.  The keys decide integers, so they are formed in the
    kernel's precision (FP32, each operation rounded: s_i * fl(1 / T) - G_i, smallest
    first).  A subdomain with a non-finite f_lo comes after every finite one.
  * batch_split: the box coordinates are FP32 and so is the midpoint (lo + hi) * 0.5.
    The top samples are the k = max(1, ceil(w / 100 * M)) samples of the box's search
    with the smallest objective (ties: lower index); a sample counts on the lower side
    of dimension j iff u_j <= mid_j.  score_j = (hi_j - lo_j) * |n_lo_j - n_up_j| in
    FP32; j* = argmax (ties: lower j); if every score is 0, the widest dimension.
  * batch_search, uniform: M samples per box, u = lo + (hi - lo) * U with supplied
    uniforms U; f_hi = the smallest objective among them and u~ its sample (ties: lower
    index).
  * batch_search, CEM (the paper's choice of sampler; it gives no details, so this is
    the textbook cross-entropy method per box): a Gaussian with per-coordinate mean mu
    and deviation sigma, started at mu = the parent's best sample u~ for the child that
    contains it (the paper: the recorded u~ initialises the search of a split
    subdomain), else the box centre, and sigma = half the box width; each of R rounds
    draws M samples u = min(max(mu + sigma * Z, lo), hi) from supplied standard normals
    Z (product and sum rounded to FP32), evaluates them and refits mu and sigma to the
    n_elite samples of smallest objective (ties: lower index; NaN as +inf): their mean
    and their deviation about it (divided by n_elite) plus a jitter.  All R * M samples
    are the box's search samples (summary, top samples, search-integrated bounds).
  * Pruner: a subdomain is kept iff f_lo <= f_hi_best (pruned iff f_lo > f_hi_best).
  * Bounding: any lower-bound function of a box; with search-integrated bounding it also
    receives the box's search samples (the paper's bounding takes pre-activation bounds
    from them and stops the backward propagation early).
  * Loop: Algorithm 2's order (search, then bound, on the new subdomains); the best
    (f_hi, u~) is updated from the children; the pruner tests only the children, which
    join the rest of P.  It stops after a given number of iterations or when P is empty.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32


def pick_out(f_lo, f_hi, g, n, eta, T):
    """Indices picked (in pick order) and the rest (in original order).  g: the supplied
    standard Gumbel variates.  The draw's keys decide integers, so they are formed in the
    kernel's precision: FP32 throughout, each operation rounded (s = (f_lo - min) /
    (max - min), key = s * fl(1 / T) - g, ascending; -0 equals +0, NaN counts as +inf)."""
    f_lo = np.asarray(f_lo, F32)
    f_hi = np.asarray(f_hi, F32)
    f_hi = np.where(np.isnan(f_hi), F32(np.inf), f_hi)
    g = np.asarray(g, F32)
    N = f_lo.size
    n = min(int(n), N)
    n1 = int(math.floor(float(eta) * n))
    first = list(np.argsort(f_hi, kind="stable")[:n1])
    taken = np.zeros(N, bool)
    taken[first] = True
    rest = np.nonzero(~taken)[0]
    fin = rest[np.isfinite(f_lo[rest])]
    picks = []
    if n - n1 > 0 and rest.size:
        lo = f_lo[fin].min() if fin.size else F32(0)
        hi = f_lo[fin].max() if fin.size else F32(0)
        inv_t = F32(1) / F32(T)
        s = (f_lo[fin] - lo) / (hi - lo) if hi > lo else np.zeros(fin.size, F32)
        key = np.full(N, np.inf, F32)
        key[fin] = s * inv_t - g[fin]
        order = sorted(rest, key=lambda i: (0, float(key[i]), i) if np.isfinite(f_lo[i]) else (1, 0.0, i))
        picks = list(order[: n - n1])
    picked = [int(i) for i in first] + [int(i) for i in picks]
    mark = np.zeros(N, bool)
    mark[picked] = True
    return np.array(picked, np.int64), np.nonzero(~mark)[0]


def search_summary(values, samples, k):
    """Per box: f_hi = smallest objective, u~ and the k best samples (ascending objective,
    ties: lower index).  values [n, M], samples [n, M, d]."""
    values = np.asarray(values)
    n, M = values.shape
    order = np.argsort(values, axis=1, kind="stable")
    f_hi = values[np.arange(n), order[:, 0]]
    top = np.stack([samples[i, order[i, :k]] for i in range(n)])
    return f_hi, top


def cem_start(lo, hi, u=None, u_div=1):
    """Start of each box's search distribution: mu = u[i // u_div] when that point lies
    in box i (lo <= u <= hi in every coordinate), else the box centre (lo + hi) * 0.5;
    sigma = (hi - lo) * 0.5.  FP32, as the boxes."""
    lo = np.asarray(lo, F32)
    hi = np.asarray(hi, F32)
    mu = (lo + hi) * F32(0.5)
    if u is not None:
        for i in range(lo.shape[0]):
            p = np.asarray(u[i // u_div], F32)
            if np.all((p >= lo[i]) & (p <= hi[i])):
                mu[i] = p
    return mu, (hi - lo) * F32(0.5)


def cem_samples(lo, hi, mu, sigma, Z):
    """One round's samples u = min(max(mu + sigma * Z, lo), hi) of each box; Z [n, M, d]
    standard normals; the product and the sum are each rounded to FP32."""
    lo, hi = np.asarray(lo, F32), np.asarray(hi, F32)
    mu, sigma = np.asarray(mu, F32), np.asarray(sigma, F32)
    step = sigma[:, None, :] * np.asarray(Z, F32)
    u = mu[:, None, :] + step
    return np.minimum(np.maximum(u, lo[:, None, :]), hi[:, None, :])


def cem_elites(values, n_elite):
    """Indices of the n_elite smallest values of each row (ascending; ties: lower index;
    NaN counts as +inf)."""
    v = np.asarray(values, np.float64)
    v = np.where(np.isnan(v), np.inf, v)
    return np.argsort(v, axis=1, kind="stable")[:, :n_elite]


def cem_refit(values, samples, n_elite, jitter):
    """Mean and deviation (about that mean, divided by n_elite) of each box's elites, the
    deviation plus jitter (FP64).  values [n, M], samples [n, M, d]."""
    idx = cem_elites(values, n_elite)
    E = np.stack([np.asarray(samples[i], np.float64)[idx[i]] for i in range(idx.shape[0])])
    mu = E.mean(axis=1)
    sigma = np.sqrt(((E - mu[:, None, :]) ** 2).mean(axis=1)) + float(jitter)
    return mu, sigma


def cem_search(objective, lo, hi, normals, rounds, M, n_elite, jitter, u=None, u_div=1):
    """R = rounds of CEM on each box; normals(r, shape) gives round r's Z.  Returns all
    samples [n, R * M, d] (round by round per box), their values [n, R * M] and the final
    mu, sigma."""
    lo, hi = np.asarray(lo, F32), np.asarray(hi, F32)
    n, d = lo.shape
    mu, sigma = cem_start(lo, hi, u, u_div)
    S_all, V_all = [], []
    for r in range(rounds):
        S = cem_samples(lo, hi, mu, sigma, normals(r, (n, M, d)))
        V = np.asarray(objective(S.reshape(-1, d)), np.float64).reshape(n, M)
        m64, s64 = cem_refit(V, S, n_elite, jitter)
        mu, sigma = m64.astype(F32), s64.astype(F32)
        S_all.append(S)
        V_all.append(V)
    return np.concatenate(S_all, axis=1), np.concatenate(V_all, axis=1), mu, sigma


def n_top(w, M):
    return max(1, min(M, int(math.ceil(float(w) / 100.0 * M))))


def split(lo, hi, top):
    """Bisect each box [lo, hi] (FP32, [n, d]) along the dimension chosen from its top
    samples top [n, k, d]; returns (child_lo, child_hi) [2n, d] (lower child 2i, upper
    child 2i + 1) and the chosen dimensions."""
    lo = np.asarray(lo, F32)
    hi = np.asarray(hi, F32)
    n, d = lo.shape
    mid = (lo + hi) * F32(0.5)
    clo = np.repeat(lo, 2, axis=0)
    chi = np.repeat(hi, 2, axis=0)
    dims = np.zeros(n, np.int64)
    for i in range(n):
        t = np.asarray(top[i], F32)
        nlo = np.sum(t <= mid[i][None, :], axis=0)
        nup = t.shape[0] - nlo
        width = hi[i] - lo[i]
        score = width * np.abs(nlo - nup).astype(F32)
        j = int(np.argmax(score)) if np.max(score) > 0 else int(np.argmax(width))
        dims[i] = j
        chi[2 * i, j] = mid[i, j]
        clo[2 * i + 1, j] = mid[i, j]
    return clo, chi, dims


def prune(f_lo, best):
    """Indices kept (in order): f_lo <= best."""
    f_lo = np.asarray(f_lo, np.float64)
    return np.nonzero(f_lo <= best)[0]


def bab_plan(objective, bound, lo0, hi0, n_pick, M, iters, eta, T, w, uniforms, gumbels,
             bound_uses_samples=False, cem=None, normals=None):
    """Algorithm 2 with the heuristics above.  objective(u [m, d]) -> [m] values;
    bound(lo [b, d], hi [b, d]) -> [b] lower bounds of the objective over each box, or
    with bound_uses_samples bound(lo, hi, S [b, R * M, d]) taking each box's search
    samples too (search-integrated bounding, Section 3.2); uniforms(tag, shape) -> the
    supplied uniforms of the search (tag 'search0', ('search', t)); gumbels(tag, shape) ->
    the supplied Gumbel variates of the pick-out (tag ('pick', t)).  With cem =
    dict(rounds, n_elite, jitter) the search is CEM (normals(tag, shape), tags ('cem0',
    r) and ('cem', t, r)) started from the parents' best samples; else M uniform
    samples.  Returns the best value, its sample and the per-iteration trace."""
    lo0 = np.asarray(lo0, F32)[None]
    hi0 = np.asarray(hi0, F32)[None]
    d = lo0.shape[1]
    R = int(cem["rounds"]) if cem else 1
    k = n_top(w, R * M)

    def search(lo, hi, tag, u_par=None):
        if cem:
            ztag = (lambda r: ("cem0", r)) if tag == "search0" else (lambda r: ("cem", tag[1], r))
            S, vals, _, _ = cem_search(objective, lo, hi, lambda r, shape: normals(ztag(r), shape),
                                       R, M, cem["n_elite"], cem["jitter"], u_par, 2)
            return search_summary(vals, S, k) + (S,)
        U = np.asarray(uniforms(tag, (lo.shape[0], M, d)), F32)
        S = lo[:, None, :] + (hi - lo)[:, None, :] * U
        vals = np.asarray(objective(S.reshape(-1, d)), np.float64).reshape(lo.shape[0], M)
        return search_summary(vals, S, k) + (S,)

    def bound_of(lo, hi, S):
        return np.asarray(bound(lo, hi, S) if bound_uses_samples else bound(lo, hi), np.float64)

    f_hi, top, S0 = search(lo0, hi0, "search0")
    f_lo = bound_of(lo0, hi0, S0)
    best, ubest = float(f_hi[0]), top[0, 0]
    P = dict(lo=lo0, hi=hi0, f_lo=f_lo, f_hi=f_hi, top=top)
    trace = []
    for t in range(iters):
        N = P["lo"].shape[0]
        if N == 0:
            break
        picked, rest = pick_out(P["f_lo"], P["f_hi"], gumbels(("pick", t), (N,)), n_pick, eta, T)
        clo, chi, dims = split(P["lo"][picked], P["hi"][picked], P["top"][picked])
        c_fhi, c_top, cS = search(clo, chi, ("search", t), P["top"][picked][:, 0])
        c_flo = bound_of(clo, chi, cS)
        j = int(np.argmin(c_fhi))
        if c_fhi[j] < best:
            best, ubest = float(c_fhi[j]), c_top[j, 0]
        keep = prune(c_flo, best)
        P = dict(lo=np.concatenate([P["lo"][rest], clo[keep]]),
                 hi=np.concatenate([P["hi"][rest], chi[keep]]),
                 f_lo=np.concatenate([P["f_lo"][rest], c_flo[keep]]),
                 f_hi=np.concatenate([P["f_hi"][rest], c_fhi[keep]]),
                 top=np.concatenate([P["top"][rest], c_top[keep]]))
        trace.append(dict(picked=picked, dims=dims, kept=keep, best=best, size=P["lo"].shape[0]))
    return best, ubest, trace, P
