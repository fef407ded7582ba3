"""FP64 reference of the learned global proposal (test infrastructure only).

Not part of the paper, which is silent on learned moves; this is the plain
definition of the construction the library implements, so that its kernels
can be checked value by value:

coordinates on the constraint surface sum |a_k|^4 = N (eq. SmoothedCubic):
  w_k = |a_k|^4 / N (a point of the simplex), y = alr(w) = log(w_k / w_{N-1}),
  k < N-1, and the phases psi_k = arg a_k.  The flat reference measure of
  eq. ProbDistr gives w ~ Dirichlet(1/2, ..., 1/2) (squares of a uniform
  point of the sphere), so its density in (y, psi) is proportional to
  prod_k w_k^(1/2) (Dirichlet density prod w^(-1/2) times the alr Jacobian
  prod w).
network: features = Re/Im of a rotated so that a_0 is real and positive;
  h1 = SiLU(x W1 + b1), h2 = SiLU(h1 W2 + b2), o = h2 W3 + b3; weights rounded
  to bfloat16 (round to nearest even); the precision policy (bfloat16 network,
  FP32 accumulation) is read as bfloat16 operands of every matrix product, so
  the inputs of each product (activations, and output gradients in training)
  are rounded to bfloat16 too; everything else is FP64 here.
proposal: a K-component diagonal Gaussian mixture over the displacement
  delta = (dy, dpsi) in R^(2N-1): weights softmax(o[:K]), means o[K:K+KD],
  widths sigma = smax * sigmoid(o[K+KD:]) with smax = 2 for y and pi/2 for
  psi; a step scale s multiplies means and widths.  Phase displacements are
  wrapped: their density is the sum over n of N(dpsi + 2 pi n).
acceptance: min(1, exp(-beta dH) rho(y')/rho(y) q(y,psi|y',psi')/q(y',psi'|y,psi)).
training loss: the mean negative log-likelihood of observed displacements
  under the unwrapped mixture (any parameters give an exact proposal).
the boundary of the chart: y is defined on the interior of the simplex only
  (every w_k > 0).  A configuration with some a_k = 0 lies on its boundary, a
  set of measure zero under the reference law that the pair move can still
  reach in finite precision (a drawn angle of exactly 0 or pi/2).  Rule: a
  learned move from such a configuration, or one whose proposal has some
  w'_k = 0, has log acceptance ratio -inf (rejected; both directions of every
  move touching the set are rejected, so detailed balance holds); a training
  pair with a zero or non-finite amplitude in either configuration is left out
  of the loss, which is the mean over the remaining pairs of the minibatch.
Pins (tests/test_oracle_mlp.py): finite differences of the loss (exact
arithmetic, gemm_bf16=False; the rounding is an elementwise map), the
single-Gaussian closed form, torch's bfloat16 rounding, the proposal density
integrating to one, and the infinite-temperature closed forms of the chain.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O

LOG2PI = math.log(2.0 * math.pi)
SMAX_Y = 2.0
SMAX_PSI = math.pi / 2.0
TAG_LEARN = 0x4C4541524E  # "LEARN"
TAG_TRAIN = 0x545241494E  # "TRAIN"


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) and return as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def sizes(N: int, K: int) -> tuple:
    D = 2 * N - 1
    return 2 * N, D, K * (2 * D + 1)


def features(a: np.ndarray) -> np.ndarray:
    """[..., N] complex -> [..., 2N]: rotate so that a_0 is real positive."""
    a = np.asarray(a)
    rot = np.exp(-1j * np.angle(a[..., :1]))
    b = a * rot
    return np.concatenate([b.real, b.imag], axis=-1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def forward(params, X, gemm_bf16=True):
    """params: dict W1 [2N,H], b1, W2 [H,H], b2, W3 [H,Out], b3 (weights used as given).
    gemm_bf16: round every matrix-product input to bfloat16 as the library's
    matrix cores take it (products and sums stay exact here); False gives the
    network in exact arithmetic."""
    r = bf16_round if gemm_bf16 else (lambda v: v)
    p1 = r(X) @ params["W1"] + params["b1"]
    h1 = silu(p1)
    p2 = r(h1) @ params["W2"] + params["b2"]
    h2 = silu(p2)
    o = r(h2) @ params["W3"] + params["b3"]
    return o, (X, p1, h1, p2, h2, gemm_bf16)


def mixture(o: np.ndarray, N: int, K: int):
    """Split outputs [..., Out] into log-weights [..., K], means and widths [..., K, D]."""
    D = 2 * N - 1
    logits = o[..., :K]
    mu = o[..., K:K + K * D].reshape(o.shape[:-1] + (K, D))
    s = o[..., K + K * D:].reshape(o.shape[:-1] + (K, D))
    smax = np.concatenate([np.full(N - 1, SMAX_Y), np.full(N, SMAX_PSI)])
    sigma = smax / (1.0 + np.exp(-s))
    lw = logits - np.logaddexp.reduce(logits, axis=-1, keepdims=True)
    return lw, mu, sigma, smax


def nll_and_grad(o: np.ndarray, delta: np.ndarray, N: int, K: int):
    """Mean negative log-likelihood of delta [B, D] under the unwrapped
    mixture of o [B, Out], and its gradient with respect to o."""
    lw, mu, sigma, smax = mixture(o, N, K)
    z = (delta[:, None, :] - mu) / sigma
    ell = lw - np.sum(np.log(sigma) + 0.5 * LOG2PI + 0.5 * z * z, axis=-1)
    logp = np.logaddexp.reduce(ell, axis=-1)
    r = np.exp(ell - logp[:, None])
    B = o.shape[0]
    pi = np.exp(lw)
    d_logits = (pi - r) / B
    d_mu = -(r[:, :, None] * z / sigma) / B
    d_s = -(r[:, :, None] * (z * z - 1.0) * (1.0 - sigma / smax)) / B
    g = np.concatenate([d_logits, d_mu.reshape(B, -1), d_s.reshape(B, -1)], axis=1)
    return float(-np.mean(logp)), g


def backward(params, cache, dO):
    """Parameter gradients of the network for output gradients dO, with the
    matrix-product inputs rounded as in forward (bias gradients are plain sums)."""
    X, p1, h1, p2, h2, gemm_bf16 = cache
    r = bf16_round if gemm_bf16 else (lambda v: v)
    grads = {"W3": r(h2).T @ r(dO), "b3": dO.sum(0)}
    dh2 = r(dO) @ params["W3"].T
    s2 = 1.0 / (1.0 + np.exp(-p2))
    dp2 = dh2 * s2 * (1.0 + p2 * (1.0 - s2))
    grads["W2"] = r(h1).T @ r(dp2)
    grads["b2"] = dp2.sum(0)
    dh1 = r(dp2) @ params["W2"].T
    s1 = 1.0 / (1.0 + np.exp(-p1))
    dp1 = dh1 * s1 * (1.0 + p1 * (1.0 - s1))
    grads["W1"] = r(X).T @ r(dp1)
    grads["b1"] = dp1.sum(0)
    return grads


def interior(a) -> np.ndarray:
    """True for configurations inside the chart: every amplitude finite and nonzero."""
    a = np.asarray(a)
    return np.all(np.isfinite(a) & (np.abs(a) > 0.0), axis=-1)


def loss_and_grads(params, a_before, a_after, N, K, gemm_bf16=True):
    """Training loss on pairs of configurations and its parameter gradients:
    the mean over the pairs whose two configurations are both inside the chart
    (the others are left out).  Raises ValueError when no pair is."""
    keep = interior(a_before) & interior(a_after)
    if not np.any(keep):
        raise ValueError("no training pair inside the chart")
    a_before, a_after = np.asarray(a_before)[keep], np.asarray(a_after)[keep]
    X = features(a_before)
    o, cache = forward(params, X, gemm_bf16)
    delta = displacement(a_before, a_after)
    L, dO = nll_and_grad(o, delta, N, K)
    return L, backward(params, cache, dO)


# ----------------------------------------------------------------- coordinates
def coords(a: np.ndarray):
    """(y [N-1], psi [N], w [N]) of a configuration on sum |a|^4 = N."""
    N = a.shape[-1]
    w = np.abs(a) ** 4 / N
    y = np.log(w[..., :-1]) - np.log(w[..., -1:])
    return y, np.angle(a), w


def from_coords(y: np.ndarray, psi: np.ndarray) -> np.ndarray:
    N = psi.shape[-1]
    e = np.concatenate([np.exp(y), np.ones(y.shape[:-1] + (1,))], axis=-1)
    w = e / e.sum(axis=-1, keepdims=True)
    return (N * w) ** 0.25 * np.exp(1j * psi)


def wrap(x):
    """Representative in (-pi, pi]."""
    return x - 2.0 * math.pi * np.ceil((x - math.pi) / (2.0 * math.pi))


def displacement(a, b):
    """delta = (y(b) - y(a), wrap(psi(b) - psi(a)))."""
    ya, pa, _ = coords(a)
    yb, pb, _ = coords(b)
    return np.concatenate([yb - ya, wrap(pb - pa)], axis=-1)


def log_ref(w):
    """log of the reference density in (y, psi) up to a constant: 1/2 sum log w."""
    return 0.5 * np.sum(np.log(w), axis=-1)


def log_q(o, dy, dpsi, N, K, scale):
    """log density [B] of proposal displacements (dy [B, N-1], dpsi [B, N])
    under the mixtures of outputs o [B, Out] with step scale s: unwrapped in
    y, wrapped (|n| <= 3 images) in psi."""
    lw, mu, sigma, _ = mixture(o, N, K)
    mu, sigma = scale * mu, scale * sigma
    dy, dpsi = dy[:, None, :], dpsi[:, None, :]
    ly = -np.sum(np.log(sigma[..., :N - 1]) + 0.5 * LOG2PI + 0.5 * ((dy - mu[..., :N - 1]) / sigma[..., :N - 1]) ** 2,
                 axis=-1)
    d = wrap(dpsi - mu[..., N - 1:])
    n = np.arange(-3, 4).reshape(7, 1, 1, 1)
    t = (d[None] + 2.0 * math.pi * n) / sigma[None, ..., N - 1:]
    lp = np.log(np.sum(np.exp(-0.5 * t * t), axis=0)) - np.log(sigma[..., N - 1:]) - 0.5 * LOG2PI
    return np.logaddexp.reduce(lw + ly + np.sum(lp, axis=-1), axis=-1)


# ----------------------------------------------------------------- draws and the move
def draws(run_seed: int, move: int, copy: int, D: int):
    """Gaussians g[D] and the component and acceptance uniforms of one move:
    Philox block i (i < ceil(D/2)) gives g[2i] = BM(w0, w1), g[2i+1] = BM(w2, w3);
    block ceil(D/2) gives the component uniform (w0) and the acceptance uniform (w1)."""
    nb = (D + 1) // 2
    g = np.zeros(2 * nb)
    for i in range(nb):
        w = O.philox([i, move, copy, 0], [run_seed, TAG_LEARN])
        for h in range(2):
            u1 = 1.0 - (int(w[2 * h]) >> 11) * 2.0 ** -53
            u2 = (int(w[2 * h + 1]) >> 11) * 2.0 ** -53
            g[2 * i + h] = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
    w = O.philox([nb, move, copy, 0], [run_seed, TAG_LEARN])
    return g[:D], (int(w[0]) >> 11) * 2.0 ** -53, (int(w[1]) >> 11) * 2.0 ** -53


def propose(params, a, N, K, scale, g, u_comp):
    """Batched proposal: a [B, N], g [B, D], u_comp [B] -> (a_new, delta, o_fwd, component)."""
    o, _ = forward(params, features(a))
    lw, mu, sigma, _ = mixture(o, N, K)
    cw = np.cumsum(np.exp(lw), axis=-1)
    m = np.minimum(np.sum(cw <= u_comp[:, None], axis=-1), K - 1)
    rows = np.arange(a.shape[0])
    delta = scale * mu[rows, m] + scale * sigma[rows, m] * g
    y, psi, _ = coords(a)
    a_new = from_coords(y + delta[:, :N - 1], psi + delta[:, N - 1:])
    return a_new, delta, o, m


def move_log_alpha(params, a, dH, beta, N, K, scale, g, u_comp, energy=None):
    """Batched learned move.  Returns (a_new, log acceptance ratio, parts).
    dH: callable a_new -> energy change per row, or None for infinite temperature.
    Rows whose current configuration or proposal is not inside the chart get
    a log acceptance ratio of -inf (their a_new is then meaningless)."""
    a = np.asarray(a)
    inside = interior(a)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        a_new, delta, o_fwd, m = propose(params, a, N, K, scale, g, u_comp)
    inside &= interior(a_new)
    a_new = np.where(inside[:, None], a_new, a)
    o_rev, _ = forward(params, features(a_new))
    lq_f = log_q(o_fwd, delta[:, :N - 1], delta[:, N - 1:], N, K, scale)
    lq_r = log_q(o_rev, -delta[:, :N - 1], -delta[:, N - 1:], N, K, scale)
    with np.errstate(divide="ignore", invalid="ignore"):
        _, _, w = coords(a)
        _, _, w2 = coords(a_new)
        dref = log_ref(w2) - log_ref(w)
    de = np.zeros(a.shape[0]) if dH is None else dH(a_new)
    la = np.where(inside, -beta * de + dref + lq_r - lq_f, -np.inf)
    return a_new, la, {"dH": de, "lq_f": lq_f, "lq_r": lq_r, "dlogref": dref, "component": m, "inside": inside}


def init_params(N, H, K, rng, out_scale=0.01):
    In, D, Out = sizes(N, K)
    return {"W1": rng.standard_normal((In, H)) / math.sqrt(In), "b1": np.zeros(H),
            "W2": rng.standard_normal((H, H)) / math.sqrt(H), "b2": np.zeros(H),
            "W3": out_scale * rng.standard_normal((H, Out)) / math.sqrt(H), "b3": np.zeros(Out)}


def rounded(params):
    """Weights as the GPU uses them: bfloat16 matrices, FP32 biases."""
    return {k: (bf16_round(v) if k.startswith("W") else np.asarray(v, np.float32).astype(np.float64))
            for k, v in params.items()}


# ----------------------------------------------------------------- the subset move
# A structured variant of the learned move (also not in the paper): each move
# redraws a random subset S of m modes and leaves the others where they are.
#   S: m distinct modes drawn uniformly (a partial Fisher-Yates shuffle), in
#     ascending order s_1 < ... < s_m; the draw does not depend on the state,
#     so its probability cancels in the acceptance ratio.
#   chart of the subset: with w = |a|^4 / N and W_S = sum_{i in S} w_i fixed,
#     u_i = log(w_{s_i} / w_{s_m}) (i < m) and the phases psi_{s_i}.  Under
#     the flat law of eq. ProbDistr the other modes fixed leave w_S / W_S
#     Dirichlet(1/2, ..., 1/2), whose density in u is prod_{i in S} w_i^(1/2)
#     up to a constant: the reference ratio only involves S.
#   proposal: the network's mixture at a (same outputs as the all-mode move):
#     component c from its weights, du_i = s (mu_c[s_i] + sigma_c[s_i] g_i) from
#     the y channel of mode s_i (i < m), dpsi_i = s (mu_c[N-1+s_i] +
#     sigma_c[N-1+s_i] g_{m-1+i}) from its phase channel; wrapped phases.
#   acceptance: min(1, exp(-beta dH) prod_S (w'/w)^(1/2) q(-d | a') / q(d | a)),
#     q the subset mixture density at the network's outputs; a move touching a
#     zero amplitude of S is rejected as for the all-mode move.
#   training: the negative log-likelihood of a harvested pair's displacement
#     in the chart of a random subset drawn for each training item.
def index_below(w: int, n: int) -> int:
    """index in [0, n) from the top 32 bits of a 64-bit word"""
    return ((int(w) >> 32) * n) >> 32


def subset_draw(words, N: int, m: int) -> np.ndarray:
    """m distinct modes, ascending: a partial Fisher-Yates shuffle of 0..N-1
    whose step t swaps position t with t + index_below(word_t, N - t)."""
    perm = list(range(N))
    for t in range(m):
        j = t + index_below(words[t], N - t)
        perm[t], perm[j] = perm[j], perm[t]
    return np.array(sorted(perm[:m]), dtype=np.int64)


def subset_draws(run_seed: int, move: int, copy: int, N: int, m: int):
    """Draws of one subset move: Philox (run_seed, LEARN) at counter
    (i, move, copy, 1): blocks i < nb = ceil((2m-1)/2) give the Gaussians
    (Box-Muller on word pairs, as draws()), block nb the component and
    acceptance uniforms (words 0, 1), blocks nb+1+t//4 word t%4 the shuffle
    words.  Returns (S, g [2m-1], u_comp, u_acc)."""
    D = 2 * m - 1
    nb = (D + 1) // 2
    g = np.zeros(2 * nb)
    for i in range(nb):
        w = O.philox([i, move, copy, 1], [run_seed, TAG_LEARN])
        for h in range(2):
            u1 = 1.0 - (int(w[2 * h]) >> 11) * 2.0 ** -53
            u2 = (int(w[2 * h + 1]) >> 11) * 2.0 ** -53
            g[2 * i + h] = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
    w = O.philox([nb, move, copy, 1], [run_seed, TAG_LEARN])
    uc, ua = (int(w[0]) >> 11) * 2.0 ** -53, (int(w[1]) >> 11) * 2.0 ** -53
    words = []
    for b in range((m + 3) // 4):
        words.extend(int(x) for x in O.philox([nb + 1 + b, move, copy, 1], [run_seed, TAG_LEARN]))
    return subset_draw(words[:m], N, m), g[:D], uc, ua


def train_subset(seed: int, step: int, net: int, item: int, N: int, m: int) -> np.ndarray:
    """The subset of training item `item` of network `net` at training step
    `step`: Philox (seed, TRAIN) at counter (step, net, item, 1 + t//4), word t%4."""
    words = []
    for b in range((m + 3) // 4):
        words.extend(int(x) for x in O.philox([step, net, item, 1 + b], [seed, TAG_TRAIN]))
    return subset_draw(words[:m], N, m)


def subset_coords(a: np.ndarray, S: np.ndarray):
    """(u [m-1], psi_S [m], w_S [m]) of one configuration in the chart of S"""
    N = a.shape[-1]
    w = np.abs(a[S]) ** 4 / N
    return np.log(w[:-1]) - np.log(w[-1]), np.angle(a[S]), w


def subset_channels(N: int, S: np.ndarray):
    """output indices (within a component's D values) of the subset's
    coordinates: y channel of s_1..s_{m-1}, then phase channel of s_1..s_m"""
    return np.concatenate([S[:-1], N - 1 + S])


def subset_log_q(o: np.ndarray, S: np.ndarray, du: np.ndarray, dpsi: np.ndarray, N: int, K: int,
                 scale: float):
    """log density of the subset displacement (du [..., m-1], dpsi [..., m])
    under the scaled mixture of one output row o: unwrapped in u, wrapped
    (|n| <= 3) in psi.  A float for one displacement, an array for a batch."""
    lw, mu, sigma, _ = mixture(o[None], N, K)
    ch = subset_channels(N, S)
    m = len(S)
    mu, sigma = scale * mu[0][:, ch], scale * sigma[0][:, ch]  # [K][2m-1]
    du = np.asarray(du, dtype=np.float64)[..., None, :]        # [..., 1, m-1]
    dpsi = np.asarray(dpsi, dtype=np.float64)[..., None, :]    # [..., 1, m]
    ly = -np.sum(np.log(sigma[:, :m - 1]) + 0.5 * LOG2PI + 0.5 * ((du - mu[:, :m - 1]) / sigma[:, :m - 1]) ** 2,
                 axis=-1)
    d = wrap(dpsi - mu[:, m - 1:])
    t = [(d + 2.0 * math.pi * n) / sigma[:, m - 1:] for n in range(-3, 4)]
    lp = np.log(sum(np.exp(-0.5 * x * x) for x in t)) - np.log(sigma[:, m - 1:]) - 0.5 * LOG2PI
    r = np.logaddexp.reduce(lw[0] + ly + np.sum(lp, axis=-1), axis=-1)
    return float(r) if np.ndim(r) == 0 else r


def subset_move_log_alpha(params, a: np.ndarray, S: np.ndarray, dH, beta: float, N: int, K: int, scale: float,
                          g: np.ndarray, u_comp: float):
    """One subset move of one configuration a [N].  Returns (a_new, log
    acceptance ratio, parts).  dH: callable a_new -> energy change, or None
    for infinite temperature."""
    m = len(S)
    inside = bool(np.all(np.isfinite(a[S]) & (np.abs(a[S]) > 0.0)))
    o_f, _ = forward(params, features(a[None]))
    lw, mu, sigma, _ = mixture(o_f, N, K)
    c = min(int(np.sum(np.cumsum(np.exp(lw[0])) <= u_comp)), K - 1)
    ch = subset_channels(N, S)
    d = scale * mu[0, c, ch] + scale * sigma[0, c, ch] * g
    du, dpsi = d[:m - 1], d[m - 1:]
    a_new = a.copy()
    if inside:
        u, psi, w = subset_coords(a, S)
        e = np.concatenate([np.exp(u + du), [1.0]])
        wn = w.sum() * e / e.sum()
        a_new[S] = (N * wn) ** 0.25 * np.exp(1j * (psi + dpsi))
        inside = bool(np.all(np.abs(a_new[S]) > 0.0))
    if not inside:
        return a.copy(), -np.inf, {"inside": False, "component": c, "du": du, "dpsi": dpsi}
    o_r, _ = forward(params, features(a_new[None]))
    lq_f = subset_log_q(o_f[0], S, du, dpsi, N, K, scale)
    lq_r = subset_log_q(o_r[0], S, -du, -dpsi, N, K, scale)
    w0 = np.abs(a[S]) ** 4 / N
    w1 = np.abs(a_new[S]) ** 4 / N
    dref = 0.5 * float(np.sum(np.log(w1) - np.log(w0)))
    de = 0.0 if dH is None else float(dH(a_new))
    la = -beta * de + dref + lq_r - lq_f
    return a_new, la, {"inside": True, "component": c, "du": du, "dpsi": dpsi, "dH": de, "lq_f": lq_f,
                       "lq_r": lq_r, "dlogref": dref}


def subset_displacement(a: np.ndarray, b: np.ndarray, S: np.ndarray):
    """(du, dpsi) from a to b in the chart of S (b's subset intensity need
    not equal a's: only the ratios enter u)"""
    ua, pa, _ = subset_coords(a, S)
    ub, pb, _ = subset_coords(b, S)
    return ub - ua, wrap(pb - pa)


def subset_nll_and_grad(o: np.ndarray, subsets, deltas, N: int, K: int):
    """Mean negative log-likelihood of the subset displacements (one subset
    and one displacement [2m-1] per row of o [B, Out]) under the unwrapped
    mixture restricted to the subset's channels, and its gradient with
    respect to o (zero outside the logits and those channels)."""
    B, Out = o.shape
    D = 2 * N - 1
    lw, mu, sigma, smax = mixture(o, N, K)
    g = np.zeros_like(o)
    L = 0.0
    for b in range(B):
        ch = subset_channels(N, subsets[b])
        z = (deltas[b][None, :] - mu[b][:, ch]) / sigma[b][:, ch]
        ell = lw[b] - np.sum(np.log(sigma[b][:, ch]) + 0.5 * LOG2PI + 0.5 * z * z, axis=-1)
        logp = np.logaddexp.reduce(ell)
        r = np.exp(ell - logp)
        L -= logp
        g[b, :K] = (np.exp(lw[b]) - r) / B
        for k in range(K):
            g[b, K + k * D + ch] = -(r[k] * z[k] / sigma[b][k, ch]) / B
            g[b, K + K * D + k * D + ch] = -(r[k] * (z[k] ** 2 - 1.0) * (1.0 - sigma[b][k, ch] / smax[ch])) / B
    return L / B, g


def subset_loss_and_grads(params, a_before, a_after, subsets, N, K, gemm_bf16=True):
    """Training loss of the subset move on pairs of configurations (one subset
    per pair) and its parameter gradients; pairs with a zero or non-finite
    amplitude in their subset are left out (ValueError when none is left)."""
    keep = np.array([bool(np.all(np.isfinite(x[S]) & (np.abs(x[S]) > 0)) and np.all(np.isfinite(y[S]) &
                                                                                      (np.abs(y[S]) > 0)))
                     for x, y, S in zip(a_before, a_after, subsets)])
    if not np.any(keep):
        raise ValueError("no training pair inside the chart")
    a_before = np.asarray(a_before)[keep]
    a_after = np.asarray(a_after)[keep]
    subsets = [S for S, k in zip(subsets, keep) if k]
    X = features(a_before)
    o, cache = forward(params, X, gemm_bf16)
    deltas = [np.concatenate(subset_displacement(x, y, S)) for x, y, S in zip(a_before, a_after, subsets)]
    L, dO = subset_nll_and_grad(o, subsets, deltas, N, K)
    return L, backward(params, cache, dO)
