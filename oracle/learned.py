"""FP64 NumPy oracle of the learned coarse-mesh correction.

TEST INFRASTRUCTURE ONLY: used by tests and the smoke check, never by the GPU
product path, and it shares no code with it.

The learned form runs PPPM on a mesh twice as coarse and adds a per-particle
correction predicted by a small network from the particle's local charge
neighbourhood, trained on force residuals between fine- and coarse-mesh PPPM.
The paper motivates the descriptor-plus-fitting-network structure with the
Deep Potential / Deep Wannier models (DPLR background section: an embedding
net producing atomic descriptors D_i from the neighbour list, then a
three-layer fitting net); the Deep Wannier model predicts a vector per atom,
which is the form used here for the force correction.

Definitions (the reading taken here; the paper gives no formulas):
  neighbours:  j != i with r_ij = |r_j - r_i| < r_c (minimum image), r_c = 4 A;
  radial basis g_k(r) = T_k(2 r / r_c - 1), Chebyshev of the first kind,
               k = 0..31, with the switch s(r) = (1 + cos(pi r / r_c)) / 2;
  T_i[k, a] = sum_j q_j g_k(r_ij) s(r_ij) u_a,  u = (1, x, y, z) of the unit
               vector from i to j;
  D_i[k, l] = sum_a T_i[k, a] T_i[l, a], l = 0..3 (128 invariant features,
               index 4 k + l);
  x_i = (D_i - mu) * inv_sigma (fixed normalisation from training data);
  h1 = silu(x W1 + b1), h2 = silu(h1 W2 + b2), h3 = silu(h2 W3 + b3),
  c = h3 W4 + b4 (128 -> 64 -> 64 -> 64 -> 32), silu(z) = z / (1 + exp(-z));
  dF_i = s_out * q_i * sum_k c_ik T_i[k, 1:4]   (rotation equivariant);
  loss = mean over particles and components of (dF - dF_target)^2.

With emulate_bf16 the layer inputs (x, h1, h2, h3) and the weights are
rounded to bfloat16 (round to nearest even) where the GPU kernels round
them; everything else stays FP64.
"""
from __future__ import annotations

import math

import numpy as np

RC = 4.0
NK = 32
NL = 4
SIZES = [(128, 64), (64, 64), (64, 64), (64, 32)]


def bf16(a):
    """Round float64/float32 values to bfloat16 (nearest even), as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def neighbours(pos, box, rc=RC):
    """All ordered pairs (i, j), i != j, with minimum-image distance < rc, by
    brute force over all pairs (small systems only).  Returns i, j, d (r_j - r_i)."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = pos.shape[0]
    ii, jj, dd = [], [], []
    for i in range(n):
        d = pos - pos[i]
        d -= box * np.round(d / box)
        r2 = (d * d).sum(1)
        m = (r2 < rc * rc)
        m[i] = False
        js = np.nonzero(m)[0]
        ii.append(np.full(js.size, i))
        jj.append(js)
        dd.append(d[js])
    return np.concatenate(ii), np.concatenate(jj), np.concatenate(dd)


def chebyshev(x, nk=NK):
    """T_k(x), k = 0..nk-1, by the three-term recurrence."""
    t = np.zeros(x.shape + (nk,))
    t[..., 0] = 1.0
    if nk > 1:
        t[..., 1] = x
    for k in range(2, nk):
        t[..., k] = 2 * x * t[..., k - 1] - t[..., k - 2]
    return t


def descriptor(pos, q, box, rc=RC, pairs=None):
    """T [n, 32, 4] and D [n, 128]."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    i, j, d = pairs if pairs is not None else neighbours(pos, box, rc)
    r = np.linalg.norm(d, axis=1)
    u = np.concatenate([np.ones((r.size, 1)), d / r[:, None]], axis=1)   # [m, 4]
    g = chebyshev(2 * r / rc - 1) * (0.5 * (1 + np.cos(math.pi * r / rc)))[:, None]
    T = np.zeros((pos.shape[0], NK, NL))
    np.add.at(T, i, q[j][:, None, None] * g[:, :, None] * u[:, None, :])
    D = np.einsum("nka,nla->nkl", T, T[:, :NL, :]).reshape(pos.shape[0], -1)
    return T, D


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed=0):
    """Deterministic initial weights (scaled normal) and zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for l, (a, b) in enumerate(SIZES, start=1):
        p[f"W{l}"] = rng.normal(0.0, 1.0 / math.sqrt(a), (a, b))
        p[f"b{l}"] = np.zeros(b)
    p["W4"] *= 0.1
    return p


def forward(params, T, D, q, mu, inv_sigma, s_out, emulate_bf16=False):
    """Returns dF [n, 3] and the cache needed by backward."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    x = r((D - mu) * inv_sigma)
    W = [r(params[f"W{l}"]) for l in range(1, 5)]
    b = [np.asarray(params[f"b{l}"], dtype=np.float64) for l in range(1, 5)]
    z1 = x @ W[0] + b[0]
    h1 = r(silu(z1))
    z2 = h1 @ W[1] + b[1]
    h2 = r(silu(z2))
    z3 = h2 @ W[2] + b[2]
    h3 = r(silu(z3))
    c = h3 @ W[3] + b[3]
    dF = s_out * q[:, None] * np.einsum("nk,nka->na", c, T[:, :, 1:])
    cache = dict(x=x, W=W, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3, c=c, T=T, q=q, s_out=s_out)
    return dF, cache


def loss_and_grad(params, cache, dF, target, emulate_bf16=False):
    """Mean-squared loss and its gradients with respect to every parameter,
    by the chain rule written out layer by layer.  With emulate_bf16 the
    gradient at each layer output (dL/dc, then dL/dz3, dL/dz2, dL/dz1) is
    rounded to bfloat16 before it is used, where the GPU backward rounds it
    for its matrix products; pass the cache of forward(..., emulate_bf16=True)
    so that activations and weights carry the forward's rounding too."""
    r = bf16 if emulate_bf16 else (lambda a: a)
    n = dF.shape[0]
    diff = dF - target
    loss = float((diff * diff).mean())
    g = 2.0 * diff / (3 * n)                                   # dL/d dF
    dc = r(cache["s_out"] * cache["q"][:, None] * np.einsum("na,nka->nk", g, cache["T"][:, :, 1:]))
    W = cache["W"]
    grads = {}
    grads["W4"] = cache["h3"].T @ dc
    grads["b4"] = dc.sum(0)
    dz3 = r((dc @ W[3].T) * dsilu(cache["z3"]))
    grads["W3"] = cache["h2"].T @ dz3
    grads["b3"] = dz3.sum(0)
    dz2 = r((dz3 @ W[2].T) * dsilu(cache["z2"]))
    grads["W2"] = cache["h1"].T @ dz2
    grads["b2"] = dz2.sum(0)
    dz1 = r((dz2 @ W[1].T) * dsilu(cache["z1"]))
    grads["W1"] = cache["x"].T @ dz1
    grads["b1"] = dz1.sum(0)
    return loss, grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of every parameter; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = beta1 * m + (1 - beta1) * grads[k]
        v[...] = beta2 * v + (1 - beta2) * grads[k] * grads[k]
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params
