"""Pins of the learned-correction oracle: the radial basis against the
Chebyshev closed form and NumPy's Chebyshev routine, exact invariances of the
descriptor (translation; rotation of an isolated cluster), rotation
equivariance of the predicted force, the switch at the cutoff, the manual
backward against finite differences of the loss in every parameter tensor,
Adam's first step, and bfloat16 rounding on representable edge values."""
import math

import numpy as np
import pytest

from oracle import learned as L


def test_chebyshev_matches_closed_form_and_numpy():
    x = np.linspace(-1, 1, 41)
    t = L.chebyshev(x)
    for k in (0, 1, 2, 7, 31):
        assert np.allclose(t[:, k], np.cos(k * np.arccos(x)), atol=1e-12)
        c = np.zeros(k + 1)
        c[k] = 1.0
        assert np.allclose(t[:, k], np.polynomial.chebyshev.chebval(x, c), atol=1e-12)


def _cluster(seed=0, n=30):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-3.0, 3.0, (n, 3)) + 50.0          # far from the box faces
    q = rng.choice([6.0, 1.0, -8.0, 1.0], n)
    return pos, q, np.array([100.0, 100.0, 100.0])


def test_descriptor_matches_double_loop():
    pos, q, box = _cluster(1, 12)
    T, D = L.descriptor(pos, q, box)
    T2 = np.zeros_like(T)
    for i in range(len(q)):
        for j in range(len(q)):
            if i == j:
                continue
            d = pos[j] - pos[i]
            r = math.sqrt(d @ d)
            if r >= L.RC:
                continue
            s = 0.5 * (1 + math.cos(math.pi * r / L.RC))
            x = 2 * r / L.RC - 1
            for k in range(L.NK):
                g = math.cos(k * math.acos(max(-1.0, min(1.0, x)))) * s
                T2[i, k] += q[j] * g * np.array([1.0, *(d / r)])
    assert np.allclose(T, T2, atol=1e-10)
    assert np.allclose(D[:, 4 * 3 + 2], (T[:, 3, :] * T[:, 2, :]).sum(1))


def test_descriptor_translation_and_rotation():
    pos, q, box = _cluster(2)
    T, D = L.descriptor(pos, q, box)
    T2, D2 = L.descriptor(pos + np.array([1.3, -0.7, 2.2]), q, box)
    assert np.allclose(T, T2, atol=1e-12) and np.allclose(D, D2, atol=1e-10)
    a = 0.7
    R = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1.0]])
    c = pos.mean(0)
    T3, D3 = L.descriptor((pos - c) @ R.T + c, q, box)
    assert np.allclose(D3, D, atol=1e-9 * np.abs(D).max())
    assert np.allclose(T3[:, :, 1:], T[:, :, 1:] @ R.T, atol=1e-10)


def test_force_head_is_rotation_equivariant():
    pos, q, box = _cluster(3)
    p = L.init_params(1)
    T, D = L.descriptor(pos, q, box)
    mu, isd = D.mean(0), 1.0 / (D.std(0) + 1e-3)
    dF, _ = L.forward(p, T, D, q, mu, isd, 0.1)
    a = 1.1
    R = np.array([[1, 0, 0], [0, math.cos(a), -math.sin(a)], [0, math.sin(a), math.cos(a)]])
    c = pos.mean(0)
    T3, D3 = L.descriptor((pos - c) @ R.T + c, q, box)
    dF3, _ = L.forward(p, T3, D3, q, mu, isd, 0.1)
    assert np.allclose(dF3, dF @ R.T, atol=1e-8 * np.abs(dF).max())


def test_switch_vanishes_at_cutoff():
    box = np.array([50.0, 50.0, 50.0])
    q = np.array([1.0, 2.0])
    for r, expect_zero in ((L.RC - 1e-9, True), (L.RC + 1e-9, True), (L.RC / 2, False)):
        pos = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
        T, _ = L.descriptor(pos, q, box)
        assert (np.abs(T).max() < 1e-15) == expect_zero


def test_backward_matches_finite_differences():
    pos, q, box = _cluster(4, 20)
    T, D = L.descriptor(pos, q, box)
    mu, isd = D.mean(0), 1.0 / (D.std(0) + 1e-3)
    p = L.init_params(2)
    for k in p:
        if k.startswith("b"):
            p[k] = np.random.default_rng(5).normal(0, 0.1, p[k].shape)
    target = np.random.default_rng(6).normal(size=(len(q), 3))
    dF, cache = L.forward(p, T, D, q, mu, isd, 0.05)
    loss, g = L.loss_and_grad(p, cache, dF, target)
    rng = np.random.default_rng(7)
    h = 1e-6
    for k in p:
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p[k].shape)
            pp, pm = {a: b.copy() for a, b in p.items()}, {a: b.copy() for a, b in p.items()}
            pp[k][idx] += h
            pm[k][idx] -= h
            lp = L.loss_and_grad(pp, L.forward(pp, T, D, q, mu, isd, 0.05)[1], L.forward(pp, T, D, q, mu, isd, 0.05)[0], target)[0]
            lm = L.loss_and_grad(pm, L.forward(pm, T, D, q, mu, isd, 0.05)[1], L.forward(pm, T, D, q, mu, isd, 0.05)[0], target)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1e-3, abs(fd)), (k, idx, fd, g[k][idx])


def test_adam_first_step_is_signed_lr():
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -4.0, 1e-3])}
    st = {}
    L.adam_step(p, g, st, lr=0.01)
    # after one step m_hat = g, v_hat = g^2: update = lr * g / (|g| + eps)
    assert np.allclose(p["w"], [1.0 - 0.01, -2.0 + 0.01, 0.5 - 0.01 * 1e-3 / (1e-3 + 1e-8)], atol=1e-12)


def test_bf16_rounding_edges():
    v = L.bf16(np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -3.0, 1e-40, np.inf]))
    assert v[0] == 1.0 and v[1] == 1.0 and v[2] == 1 + 2 ** -7 and v[3] == -3.0 and v[5] == np.inf
    assert abs(v[4]) < 1e-38


def test_bf16_emulated_backward_is_a_small_rounding_of_the_exact_one():
    # the emulation only rounds the layer-output gradients: every parameter
    # gradient moves by bf16-level amounts (not zero, not O(1)), and with the
    # flag off the function is the exact chain rule pinned above
    rng = np.random.default_rng(4)
    n = 40
    T = rng.normal(0, 1, (n, L.NK, L.NL))
    D = np.einsum("nka,nla->nkl", T, T[:, :L.NL, :]).reshape(n, -1)
    q = rng.choice([6.0, 1.0, -8.0], n)
    p = L.init_params(2)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    mu, isd = D.mean(0), 1.0 / (D.std(0) + 1e-3)
    dF, cache = L.forward(p, T, D, q, mu, isd, 0.01, emulate_bf16=True)
    target = rng.normal(0, 0.05, dF.shape)
    _, g_exact = L.loss_and_grad(p, cache, dF, target)
    _, g_emul = L.loss_and_grad(p, cache, dF, target, emulate_bf16=True)
    for k in g_exact:
        d = np.linalg.norm(g_emul[k] - g_exact[k]) / np.linalg.norm(g_exact[k])
        assert 1e-6 < d < 2e-2, (k, d)
