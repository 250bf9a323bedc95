"""FP64 oracle of the preconditioner network (test infrastructure only).

The network is an MLP 5 -> 64 -> 64 -> 64 -> 1 with ReLU, packed as
W1[64][5] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4[1]
(W[out][in]).  The GPU multiplies bf16-rounded weights and layer inputs with
float accumulation; ``forward(..., bf16=True)`` rounds the same operands
(round to nearest even) and otherwise computes in float64.  ``loss_grad``
back-propagates the weighted mean squared error
L = (1/R) sum_i w_i (o_i - t_i)^2 in float64, treating the rounding as the
identity (straight-through), which is what the GPU's backward products do.

Pin: with bf16=False the function is smooth and ``loss_grad`` is checked
against central differences of ``loss`` (parity of the backprop algebra).
"""
import numpy as np

H, F = 64, 5
SIZES = [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)),
         ("b3", (H,)), ("W4", (H,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16_round(a):
    """Round to bfloat16 (nearest, ties to even) via the float32 bit pattern."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, X, bf16=True):
    q = unpack(p)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    z1 = r(X) @ r(q["W1"]).T + q["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = r(h1) @ r(q["W2"]).T + q["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = r(h2) @ r(q["W3"]).T + q["b3"]
    h3 = np.maximum(z3, 0.0)
    o = h3 @ q["W4"] + q["b4"][0]
    return o, (X, h1, h2, h3)


def loss(p, X, t, w=None, bf16=True):
    o, _ = forward(p, X, bf16)
    w = np.ones_like(o) if w is None else np.asarray(w, dtype=np.float64)
    return float(np.mean(w * (o - t) ** 2))


def loss_grad(p, X, t, w=None, bf16=True):
    q = unpack(p)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    o, (X, h1, h2, h3) = forward(p, X, bf16)
    R = len(o)
    w = np.ones(R) if w is None else np.asarray(w, dtype=np.float64)
    g = 2.0 * w * (o - np.asarray(t, dtype=np.float64)) / R
    d = {}
    d["W4"] = h3.T @ g
    d["b4"] = np.array([g.sum()])
    dz3 = np.outer(g, q["W4"]) * (h3 > 0)
    d["W3"] = dz3.T @ r(h2)
    d["b3"] = dz3.sum(0)
    dz2 = (dz3 @ r(q["W3"])) * (h2 > 0)
    d["W2"] = dz2.T @ r(h1)
    d["b2"] = dz2.sum(0)
    dz1 = (dz2 @ r(q["W2"])) * (h1 > 0)
    d["W1"] = dz1.T @ r(X)
    d["b1"] = dz1.sum(0)
    return float(np.mean(w * (o - t) ** 2)), pack(d)


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) in float64; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0, scale=1.0):
    """He-style random initialisation (used by tests)."""
    rng = np.random.default_rng(seed)
    d = {"W1": rng.normal(0, scale * np.sqrt(2.0 / F), (H, F)), "b1": rng.normal(0, 0.1, H),
         "W2": rng.normal(0, scale * np.sqrt(2.0 / H), (H, H)), "b2": rng.normal(0, 0.1, H),
         "W3": rng.normal(0, scale * np.sqrt(2.0 / H), (H, H)), "b3": rng.normal(0, 0.1, H),
         "W4": rng.normal(0, scale * np.sqrt(1.0 / H), H), "b4": np.array([0.05])}
    return pack(d)


def preconditioner_features(v, D, m, dim, h, ell, n, s2):
    """Per-frequency inputs of the network, as the library's interface
    defines them (efgp_features), for j in J_m (C order): h |j| ell,
    0.1 log(N D_j^2 / sigma^2), 0.2 log sigma^2, 0.5 log ell, and
    0.1 log(mean |v_k| / N + 1e-12) over the box |k_l - j_l| <= 2 clipped to
    J_2m.  v: Toeplitz vector on J_2m (C order), D: weights on J_m.
    Parity unpinned against the paper (the features are this library's
    design, not the paper's); pinned by special cases: a single point or
    coincident points give |v_k| = N, hence a zero last feature."""
    from .efgp import freq_grid
    W2 = 4 * m + 1
    J = freq_grid(m, dim)
    av = np.abs(np.asarray(v)).reshape((W2,) * dim)
    tot = np.zeros(len(J))
    cnt = np.zeros(len(J))
    offs = np.stack(np.meshgrid(*([np.arange(-2, 3)] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    for off in offs:
        K = J + off
        ok = np.all(np.abs(K) <= 2 * m, axis=1)
        idx = tuple((K[ok] + 2 * m).T)
        tot[ok] += av[idx]
        cnt[ok] += 1
    jn = np.sqrt(np.sum(J.astype(np.float64) ** 2, axis=1))
    D = np.asarray(D, dtype=np.float64)
    f = np.empty((len(J), 5))
    f[:, 0] = h * jn * ell
    f[:, 1] = 0.1 * np.log(n * D * D / s2 + 1e-300)
    f[:, 2] = 0.2 * np.log(s2)
    f[:, 3] = 0.5 * np.log(ell)
    f[:, 4] = 0.1 * np.log(tot / cnt / n + 1e-12)
    return f
