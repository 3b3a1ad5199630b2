"""Plain FP64 NumPy PPPM with ik-differentiation: the ORACLE of the mesh method.

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
CPU baseline, never by the GPU product path, and it shares no code with it.

The paper computes the Gaussian-charge energy E_Gt (DPLR background section,
the reciprocal sum over m != 0 with S(m) over ions and Wannier centroids) by
PPPM with the Poisson-IK scheme of Hockney and Eastwood (Optimization section,
hardware-offloaded 3D FFT: one forward and three inverse 3D FFTs).  The paper
does not print the scheme's formulas; this module follows the standard
particle-mesh method in its order:

 1. mesh coordinates u = r / h (h = L/K per axis), wrapped into [0, K);
 2. charge assignment with the cardinal B-spline M_p of order p, centred:
        Q(g) = sum_j q_j prod_a M_p(u_ja - g_a + p/2)   (periodic in g);
 3. forward DFT  Q^(n) = sum_g Q(g) exp(-2 pi i n.g/K);
 4. the optimal influence function for ik-differentiation,
        G(k) = sum_m (k . k_m) U^2(k_m) phi(k_m) / ( |k|^2 [sum_m U^2(k_m)]^2 ),
    k = 2 pi n / L, k_m = k + 2 pi m / h, U(k) = prod_a sinc(k_a h_a/2)^p,
    phi(k) = 4 pi exp(-k^2/(4 beta^2)) / k^2 (the Fourier transform of the
    Gaussian-screened Coulomb kernel), alias sum |m_a| <= alias, G(0) = 0;
 5. energy  E = k_e/(2V) sum_{n != 0} G(n) |Q^(n)|^2;
 6. field spectra  E^_a(n) = -i k'_a G(n) Q^(n), with k'_a = 0 on the Nyquist
    index n_a = -K_a/2 (its derivative has no real representation);
 7. three inverse DFTs without normalisation  E_a(g) = sum_n E^_a(n) exp(+2 pi i n.g/K);
 8. force interpolation with the same assignment function
        F_ja = (k_e q_j / V) sum_g prod_b M_p(u_jb - g_b + p/2) E_a(g);
 9. virial  W_ab = k_e/(2V) sum_{n != 0} G |Q^|^2 [delta_ab - 2 (1 + k^2/(4 beta^2)) k_a k_b / k^2].

With k = 2 pi m the factor phi/(2V) equals the paper's exp(-pi^2 m^2/beta^2) /
(2 pi V m^2), so as h -> 0 this converges to the direct Ewald sum.
Everything here uses full (not half) spectra and numpy.fft.

pppm_int32() takes the transforms as the paper's Mixed-Int32 configuration
does: partial sums over node blocks of each axis, quantised to int32 at a
scale of 1e7 and summed as integers.

pppm_ad() is the analytic-differentiation variant of the same energy (not in
the paper, which uses ik; it is the adjacent textbook scheme).  Steps 1-5 and
9 are shared; the forces are the exact gradient of the step-5 energy:
 6'. potential phi(g) = sum_n G(n) Q^(n) exp(+2 pi i n.g/K) (one inverse DFT);
 7'. since dE/dQ(g) = (k_e/V) phi(g) and dQ(g)/dr_ja = q_j dW/du_a / h_a,
        F_ja = -(k_e q_j / (V h_a)) sum_g phi(g) M'_p(u_ja - g_a + p/2)
                                        prod_{b != a} M_p(u_jb - g_b + p/2),
     with the B-spline derivative M'_p(x) = M_{p-1}(x) - M_{p-1}(x - 1).
"""
from __future__ import annotations

import math

import numpy as np


def bspline(p: int, x):
    """Cardinal B-spline M_p(x) on [0, p] by the textbook recursion
    M_1 = 1 on [0, 1), M_p(x) = [x M_{p-1}(x) + (p - x) M_{p-1}(x - 1)] / (p - 1)."""
    x = np.asarray(x, dtype=np.float64)
    if p == 1:
        return ((x >= 0.0) & (x < 1.0)).astype(np.float64)
    return (x * bspline(p - 1, x) + (p - x) * bspline(p - 1, x - 1.0)) / (p - 1)


def stencil(u, p: int):
    """Assignment stencil along one axis: the p mesh points g = s..s+p-1 with
    s = floor(u - p/2) + 1 (those with |u - g| < p/2) and their weights
    M_p(u - g + p/2).  Returns (g [n, p] int (unwrapped), w [n, p])."""
    u = np.asarray(u, dtype=np.float64)
    s = np.floor(u - p / 2.0).astype(np.int64) + 1
    g = s[:, None] + np.arange(p)[None, :]
    w = bspline(p, u[:, None] - g + p / 2.0)
    return g, w


def dbspline(p: int, x):
    """Derivative of the cardinal B-spline: M'_p(x) = M_{p-1}(x) - M_{p-1}(x - 1)."""
    x = np.asarray(x, dtype=np.float64)
    return bspline(p - 1, x) - bspline(p - 1, x - 1.0)


def mesh_coords(pos, box, K):
    """u = r / h wrapped into [0, K) per axis."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    K = np.asarray(K)
    u = pos / (box / K)
    u = np.mod(u, K)
    return np.where(u >= K, 0.0, u)


def spread(pos, q, box, K, p: int):
    """Charge mesh Q[Kx, Ky, Kz] (index order x, y, z)."""
    K = tuple(int(k) for k in K)
    u = mesh_coords(pos, box, K)
    q = np.asarray(q, dtype=np.float64)
    st = [stencil(u[:, a], p) for a in range(3)]
    Q = np.zeros(K[0] * K[1] * K[2])
    for tx in range(p):
        gx = np.mod(st[0][0][:, tx], K[0])
        wx = q * st[0][1][:, tx]
        for ty in range(p):
            gy = np.mod(st[1][0][:, ty], K[1])
            wxy = wx * st[1][1][:, ty]
            for tz in range(p):
                gz = np.mod(st[2][0][:, tz], K[2])
                idx = (gx * K[1] + gy) * K[2] + gz
                Q += np.bincount(idx, weights=wxy * st[2][1][:, tz], minlength=Q.size)
    return Q.reshape(K)


def interpolate(pos, box, K, p: int, field):
    """sum_g W(u_j - g) field(g) for every particle j (same W as spread)."""
    K = tuple(int(k) for k in K)
    u = mesh_coords(pos, box, K)
    st = [stencil(u[:, a], p) for a in range(3)]
    out = np.zeros(u.shape[0])
    flat = field.reshape(-1)
    for tx in range(p):
        gx = np.mod(st[0][0][:, tx], K[0])
        wx = st[0][1][:, tx]
        for ty in range(p):
            gy = np.mod(st[1][0][:, ty], K[1])
            wxy = wx * st[1][1][:, ty]
            for tz in range(p):
                gz = np.mod(st[2][0][:, tz], K[2])
                out += wxy * st[2][1][:, tz] * flat[(gx * K[1] + gy) * K[2] + gz]
    return out


def interpolate_grad(pos, box, K, p: int, field):
    """[n, 3]: sum_g field(g) dW(u_j - g)/du_a for a = x, y, z, where
    W(d) = prod_b M_p(d_b + p/2) is the assignment function of spread()."""
    K = tuple(int(k) for k in K)
    u = mesh_coords(pos, box, K)
    st = [stencil(u[:, a], p) for a in range(3)]
    dw = [dbspline(p, u[:, a][:, None] - st[a][0] + p / 2.0) for a in range(3)]
    out = np.zeros((u.shape[0], 3))
    flat = field.reshape(-1)
    for tx in range(p):
        gx = np.mod(st[0][0][:, tx], K[0])
        for ty in range(p):
            gy = np.mod(st[1][0][:, ty], K[1])
            for tz in range(p):
                gz = np.mod(st[2][0][:, tz], K[2])
                f = flat[(gx * K[1] + gy) * K[2] + gz]
                wx, wy, wz = st[0][1][:, tx], st[1][1][:, ty], st[2][1][:, tz]
                out[:, 0] += f * dw[0][:, tx] * wy * wz
                out[:, 1] += f * wx * dw[1][:, ty] * wz
                out[:, 2] += f * wx * wy * dw[2][:, tz]
    return out


def wavevectors(box, K):
    """Signed integer indices n (numpy.fft order; the Nyquist index is -K/2)
    and k = 2 pi n / L per axis."""
    n = [np.fft.fftfreq(int(K[a]), 1.0 / int(K[a])) for a in range(3)]
    k = [2.0 * math.pi * n[a] / float(box[a]) for a in range(3)]
    return n, k


def influence(box, K, beta: float, p: int, alias: int = 2):
    """Optimal ik influence function G on the full signed grid [Kx, Ky, Kz]."""
    box = np.asarray(box, dtype=np.float64)
    K = [int(k) for k in K]
    h = box / np.asarray(K)
    n, k = wavevectors(box, K)
    kx, ky, kz = np.meshgrid(k[0], k[1], k[2], indexing="ij")
    num = np.zeros(kx.shape)
    den = np.zeros(kx.shape)
    for mx in range(-alias, alias + 1):
        kmx = kx + 2 * math.pi * mx / h[0]
        ux = np.sinc(n[0] / K[0] + mx) ** (2 * p)
        for my in range(-alias, alias + 1):
            kmy = ky + 2 * math.pi * my / h[1]
            uy = np.sinc(n[1] / K[1] + my) ** (2 * p)
            for mz in range(-alias, alias + 1):
                kmz = kz + 2 * math.pi * mz / h[2]
                uz = np.sinc(n[2] / K[2] + mz) ** (2 * p)
                u2 = ux[:, None, None] * uy[None, :, None] * uz[None, None, :]
                km2 = kmx * kmx + kmy * kmy + kmz * kmz
                with np.errstate(divide="ignore", invalid="ignore"):
                    phi = np.where(km2 > 0, 4 * math.pi * np.exp(-km2 / (4 * beta * beta)) / km2, 0.0)
                num += (kx * kmx + ky * kmy + kz * kmz) * u2 * phi
                den += u2
    k2 = kx * kx + ky * ky + kz * kz
    with np.errstate(divide="ignore", invalid="ignore"):
        G = np.where(k2 > 0, num / (k2 * den * den), 0.0)
    return G


def pppm(pos, q, box, K, p: int, beta: float, ke: float, alias: int = 2, G=None,
         return_parts: bool = False):
    """PPPM-ik energy, forces [n,3] and virial [6] (xx,yy,zz,xy,xz,yz)."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    box = np.asarray(box, dtype=np.float64).reshape(3)
    K = [int(k) for k in K]
    V = float(np.prod(box))
    Q = spread(pos, q, box, K, p)
    Qh = np.fft.fftn(Q)
    if G is None:
        G = influence(box, K, beta, p, alias)
    n, k = wavevectors(box, K)
    kg = np.meshgrid(k[0], k[1], k[2], indexing="ij")
    s2 = (Qh.conj() * Qh).real
    E = ke / (2 * V) * float((G * s2).sum())
    k2 = kg[0] ** 2 + kg[1] ** 2 + kg[2] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        c = np.where(k2 > 0, 2 * (1 + k2 / (4 * beta * beta)) / k2, 0.0)
    W = np.empty(6)
    for i, (a, b) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        W[i] = ke / (2 * V) * float((G * s2 * ((1.0 if a == b else 0.0) - c * kg[a] * kg[b])).sum())
    ntot = K[0] * K[1] * K[2]
    F = np.zeros_like(pos)
    fields = []
    for a in range(3):
        kd = np.where(n[a] == -K[a] // 2, 0.0, k[a]) if K[a] % 2 == 0 else k[a]
        shape = [1, 1, 1]
        shape[a] = K[a]
        Eh = -1j * kd.reshape(shape) * G * Qh
        Ea = np.fft.ifftn(Eh) * ntot
        fields.append(Ea.real)
        F[:, a] = ke * q / V * interpolate(pos, box, K, p, Ea.real)
    if return_parts:
        return E, F, W, dict(Q=Q, Qhat=Qh, G=G, fields=fields)
    return E, F, W


def pppm_ad(pos, q, box, K, p: int, beta: float, ke: float, alias: int = 2, G=None,
            return_parts: bool = False):
    """PPPM energy and virial as pppm(), with forces by analytic
    differentiation of the assignment weights: F = -dE/dr of the returned E."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    box = np.asarray(box, dtype=np.float64).reshape(3)
    K = [int(k) for k in K]
    V = float(np.prod(box))
    h = box / np.asarray(K)
    Q = spread(pos, q, box, K, p)
    Qh = np.fft.fftn(Q)
    if G is None:
        G = influence(box, K, beta, p, alias)
    n, k = wavevectors(box, K)
    kg = np.meshgrid(k[0], k[1], k[2], indexing="ij")
    s2 = (Qh.conj() * Qh).real
    E = ke / (2 * V) * float((G * s2).sum())
    k2 = kg[0] ** 2 + kg[1] ** 2 + kg[2] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        c = np.where(k2 > 0, 2 * (1 + k2 / (4 * beta * beta)) / k2, 0.0)
    W = np.empty(6)
    for i, (a, b) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        W[i] = ke / (2 * V) * float((G * s2 * ((1.0 if a == b else 0.0) - c * kg[a] * kg[b])).sum())
    ntot = K[0] * K[1] * K[2]
    phi = (np.fft.ifftn(G * Qh) * ntot).real
    F = -(ke / V) * q[:, None] * interpolate_grad(pos, box, K, p, phi) / h[None, :]
    if return_parts:
        return E, F, W, dict(Q=Q, Qhat=Qh, G=G, phi=phi)
    return E, F, W


def dft_axis_int32(x, axis: int, nodes: int, scale: float, sign: int, return_partials: bool = False):
    """Unnormalised DFT along one axis as the paper's hardware-offloaded FFT
    forms it (Optimization section, reduction chains and int32 quantisation):
    the K points of the axis belong to `nodes` consecutive blocks of K/nodes
    points; every block forms its partial sum
        P_b[k] = sum_{n in block b} x[n] exp(sign 2 pi i n k / K),
    whose real and imaginary parts are scaled by `scale`, rounded to the
    nearest integer and clamped to the int32 range; the integers are summed
    over the blocks (exactly) and the sum is divided by `scale`.
    With return_partials the unrounded scaled partial values P_b * scale are
    returned too, as an array [nodes, ...] in the axis-last layout of x with
    the axis moved to the end."""
    x = np.asarray(x, dtype=np.complex128)
    K = x.shape[axis]
    if nodes < 1 or K % nodes:
        raise ValueError("the node count must divide the axis length")
    seg = K // nodes
    xm = np.moveaxis(x, axis, -1)
    k = np.arange(K)
    lo, hi = -2.0 ** 31, 2.0 ** 31 - 1
    acc_re = np.zeros(xm.shape, dtype=np.int64)
    acc_im = np.zeros(xm.shape, dtype=np.int64)
    parts = []
    for b in range(nodes):
        n = np.arange(b * seg, (b + 1) * seg)
        w = np.exp(sign * 2j * math.pi * (np.outer(n, k) % K) / K)
        P = xm[..., n] @ w
        acc_re += np.clip(np.rint(P.real * scale), lo, hi).astype(np.int64)
        acc_im += np.clip(np.rint(P.imag * scale), lo, hi).astype(np.int64)
        if return_partials:
            parts.append(P * scale)
    out = np.moveaxis((acc_re.astype(np.float64) + 1j * acc_im.astype(np.float64)) / scale, -1, axis)
    if return_partials:
        return out, np.stack(parts)
    return out


def pppm_int32(pos, q, box, K, p: int, beta: float, ke: float, nodes, scale: float = 1e7,
               alias: int = 2, G=None, return_parts: bool = False):
    """pppm() with the paper's Mixed-Int32 transforms (Evaluation, precision
    configurations): every 3D transform is taken axis by axis (x, y, z) with
    dft_axis_int32 and nodes[a] node blocks along axis a.  The charge mesh is
    transformed in charge units; the field spectra carry k_e / V, so the
    inverse transforms produce the field itself (eV/A per unit charge), the
    O(1) values the scaling by `scale` is meant for.  Energy and virial follow
    from the quantised charge spectrum with the formulas of pppm()."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    box = np.asarray(box, dtype=np.float64).reshape(3)
    K = [int(k) for k in K]
    V = float(np.prod(box))
    Q = spread(pos, q, box, K, p)
    Qh = Q.astype(np.complex128)
    for a in range(3):
        Qh = dft_axis_int32(Qh, a, int(nodes[a]), scale, -1)
    if G is None:
        G = influence(box, K, beta, p, alias)
    n, k = wavevectors(box, K)
    kg = np.meshgrid(k[0], k[1], k[2], indexing="ij")
    s2 = (Qh.conj() * Qh).real
    E = ke / (2 * V) * float((G * s2).sum())
    k2 = kg[0] ** 2 + kg[1] ** 2 + kg[2] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        c = np.where(k2 > 0, 2 * (1 + k2 / (4 * beta * beta)) / k2, 0.0)
    W = np.empty(6)
    for i, (a, b) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        W[i] = ke / (2 * V) * float((G * s2 * ((1.0 if a == b else 0.0) - c * kg[a] * kg[b])).sum())
    F = np.zeros_like(pos)
    for a in range(3):
        kd = np.where(n[a] == -K[a] // 2, 0.0, k[a]) if K[a] % 2 == 0 else k[a]
        shape = [1, 1, 1]
        shape[a] = K[a]
        Ea = (ke / V) * (-1j * kd.reshape(shape) * G * Qh)
        for b in range(3):
            Ea = dft_axis_int32(Ea, b, int(nodes[b]), scale, +1)
        F[:, a] = q * interpolate(pos, box, K, p, Ea.real)
    if return_parts:
        return E, F, W, dict(Q=Q, Qhat=Qh, G=G)
    return E, F, W


def system_pppm(sys, K, p: int, beta: float, ke: float, alias: int = 2, G=None):
    """pppm() on a systems.System; returns (E, F_ion, F_wc, W)."""
    if np.isscalar(K):
        K = (int(K),) * 3
    E, F, W = pppm(sys.all_pos(), sys.all_q(), sys.box, K, p, beta, ke, alias, G)
    return E, F[: sys.n_ion], F[sys.n_ion:], W


def rel_rmse(F, Fref) -> float:
    """||F - Fref||_2 / ||Fref||_2 over all components."""
    F = np.asarray(F, dtype=np.float64)
    Fref = np.asarray(Fref, dtype=np.float64)
    return float(np.linalg.norm(F - Fref) / np.linalg.norm(Fref))
