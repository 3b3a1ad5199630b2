"""GPU parity of the mixed-radix path (meshes whose sizes are not all powers
of two from 16 to 512) against the oracles, through the C ABI.

The paper's precision study uses per-node grids of 4 to 6 points per axis
over a 2 x 3 x 2 node layout: meshes 8x12x8, 10x15x10 and 12x18x12 for 128
waters in a box of about 16 Angstrom (Results, accuracy of the precision
variants).  The oracle's NumPy transforms take any size, so the bars are those
of the power-of-two path: FP64 to 1e-9 relative, FP32 (against the oracle at
the FP32-rounded inputs) to 1e-5 in the forces and 2e-6 in energy and virial.
"""
import numpy as np
import pytest

import systems
from oracle import ewald, pppm

from test_gpu_parity import BETA, KE, check_vs_pppm, rel, run_gpu, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu

FP32_TOL_F, FP32_TOL_E = 1e-5, 2e-6
PAPER_GRIDS = [(8, 12, 8), (10, 15, 10), (12, 18, 12)]


def small_water():
    return systems.water_box(128, 16.0, seed=20261128, name="water128_16A")


@pytest.mark.parametrize("mesh", PAPER_GRIDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_paper_grids(torch_dev, mesh, precision):
    s = small_water()
    if precision == "fp64":
        check_vs_pppm(torch_dev, s, mesh, 5, "fp64", 1e-9, 1e-9, 1e-9)
    else:
        check_vs_pppm(torch_dev, s, mesh, 5, "fp32", FP32_TOL_F, FP32_TOL_E, FP32_TOL_E)


# (160, 135, 8) and (240, 90, 10): xy planes too large for LDS, so the
# spread takes the global-atomic kernel instead of the plane kernel;
# (120, 100, 12): the plane of 64-bit accumulators fits in LDS but the FP64
# complex plane of the fused transforms does not (per-axis transforms)
@pytest.mark.parametrize("mesh,order", [((15, 25, 27), 3), ((45, 30, 20), 7), ((8, 8, 8), 5), ((9, 10, 6), 6),
                                        ((6, 5, 4), 4), ((96, 80, 75), 5), ((160, 135, 8), 5), ((240, 90, 10), 4),
                                        ((480, 18, 20), 5), ((12, 500, 9), 3), ((120, 100, 12), 5)])
def test_mixed_sizes_fp64(torch_dev, mesh, order):
    s = systems.water_box(512, 25.0, seed=20261129, name="water512_25A")
    s.box = np.array([25.0, 27.5, 23.0])
    check_vs_pppm(torch_dev, s, mesh, order, "fp64", 1e-9, 1e-9, 1e-9)


# (120, 135, 10): an FP32 complex plane of 16,200 points, just under the fused
# kernels' 16,384; (144, 120, 8): 17,280 points, just over (per-axis transforms
# after the plane spread)
@pytest.mark.parametrize("mesh", [(48, 60, 40), (72, 72, 72), (100, 64, 90), (120, 135, 10), (144, 120, 8)])
def test_mixed_sizes_fp32(torch_dev, mesh):
    s = systems.workload(2).system()
    check_vs_pppm(torch_dev, s, mesh, 5, "fp32", FP32_TOL_F, FP32_TOL_E, FP32_TOL_E)


@pytest.mark.parametrize("precision,order", [("fp64", 5), ("fp32", 5), ("fp32", 8)])
def test_split_plane_spectra(torch_dev, precision, order):
    # 68,000 charges: enough for the plane spread to split every plane's
    # particles over several blocks (Kz = 36: four splits), whose partial
    # spectra the z pass adds; odd-length y rows (45 = 3^2 5) and C = 8
    # columns per z block (Kx Ky = 1800)
    s = systems.water_box(17000, 82.0, seed=20261203, name="water17000_82A")
    if precision == "fp64":
        check_vs_pppm(torch_dev, s, (40, 45, 36), order, "fp64", 1e-9, 1e-9, 1e-9)
    else:
        check_vs_pppm(torch_dev, s, (40, 45, 36), order, "fp32", FP32_TOL_F, FP32_TOL_E, FP32_TOL_E)


def test_refined_mixed_mesh_meets_ewald(torch_dev):
    # 128 waters, 16 A: at 60^3 and order 7 the method error is far below 1e-6
    s = small_water()
    E, fi, fw, W, _ = run_gpu(torch_dev, s, (60, 60, 60), 7, "fp64")
    E0, _, fi0, fw0 = ewald.system_recip(s, BETA, KE)
    F, F0 = np.concatenate([fi, fw]), np.concatenate([fi0, fw0])
    print(f"60^3 p7 vs Ewald: dE={abs(E - E0) / abs(E0):.2e} dF={rel(F, F0):.2e}", flush=True)
    assert abs(E - E0) <= 1e-8 * abs(E0)
    assert rel(F, F0) <= 1e-6


def test_paper_grid_error_vs_ewald_is_reported(torch_dev):
    # the method error of each paper grid against the exact sum (FP64 kernels)
    s = small_water()
    E0, _, fi0, fw0 = ewald.system_recip(s, BETA, KE)
    F0 = np.concatenate([fi0, fw0])
    errs = []
    for mesh in PAPER_GRIDS + [(32, 32, 32)]:
        E, fi, fw, _, _ = run_gpu(torch_dev, s, mesh, 5, "fp64")
        errs.append(rel(np.concatenate([fi, fw]), F0))
        print(f"{mesh}: force error vs Ewald {errs[-1]:.2e}, energy {abs(E - E0) / abs(E0):.2e}", flush=True)
    # finer meshes are more accurate; the 32^3 baseline of the paper is the best
    assert errs[0] > errs[1] > errs[2] > errs[3]


@pytest.mark.parametrize("mesh", [(10, 15, 10), (160, 135, 8)])
def test_empty_accumulate_no_virial_and_repeatability(torch_dev, mesh):
    import paper_2504_15508_amd as dl
    torch = torch_dev
    s = small_water()
    r = s.rounded(np.float32)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    plan = dl.Plan(mesh, order=5, beta=BETA, coulomb_k=KE, precision="fp32", capacity=s.n)
    plan.set_box(s.box)
    E1, fi1, fw1, W1 = plan.compute(t(r.ion_pos), t(r.ion_q), t(r.wc_pos), t(r.wc_q))
    E2, fi2, fw2, W2 = plan.compute(t(r.ion_pos), t(r.ion_q), t(r.wc_pos), t(r.wc_q))
    torch.cuda.synchronize()
    # integer mesh sums and fixed reduction trees: bitwise repeatable
    assert torch.equal(fi1, fi2) and torch.equal(fw1, fw2) and float(E1) == float(E2)
    assert torch.equal(W1, W2)
    # empty input: zero energy and virial
    z = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    zq = torch.zeros((0,), dtype=torch.float32, device="cuda")
    E0, fi0, fw0, W0 = plan.compute(z, zq, z, zq)
    torch.cuda.synchronize()
    assert float(E0) == 0.0 and float(W0.abs().max()) == 0.0 and fi0.numel() == 0
    # the next call after the empty one is unchanged (the mesh was cleared)
    E3, fi3, _, _ = plan.compute(t(r.ion_pos), t(r.ion_q), t(r.wc_pos), t(r.wc_q))
    torch.cuda.synchronize()
    assert torch.equal(fi1, fi3) and float(E1) == float(E3)
    # accumulate into given outputs; no virial
    pa = dl.Plan(mesh, order=5, beta=BETA, coulomb_k=KE, precision="fp32", capacity=s.n,
                 flags=dl._lib.ACCUMULATE | dl._lib.NO_VIRIAL)
    pa.set_box(s.box)
    base_i = torch.full_like(fi1, 0.5)
    base_w = torch.full_like(fw1, -0.25)
    Ea, fia, fwa, Wa = pa.compute(t(r.ion_pos), t(r.ion_q), t(r.wc_pos), t(r.wc_q),
                                  ion_force=base_i.clone(), wc_force=base_w.clone())
    torch.cuda.synchronize()
    assert float(Ea) == float(E1)
    assert torch.equal(fia, base_i + fi1) and torch.equal(fwa, base_w + fw1)


def test_mixed_mesh_rejects_ad_and_bad_sizes(torch_dev):
    import paper_2504_15508_amd as dl
    with pytest.raises(Exception, match="power-of-two"):
        dl.Plan((12, 18, 12), order=5, precision="fp64", capacity=10, diff="ad")
    with pytest.raises(Exception, match="2, 3 and 5"):
        dl.Plan((14, 18, 12), order=5, precision="fp64", capacity=10)
    with pytest.raises(Exception, match="order"):
        dl.Plan((4, 18, 12), order=5, precision="fp64", capacity=10)


# ---------------------------------------------------------------------------
# The paper's Mixed-Int32 transforms (node-block partial DFTs quantised to
# int32 at 1e7) against the oracle's pppm_int32.  Exact ties are frequent:
# after the first quantised axis every value is a multiple of the quantum,
# and twiddles such as cos(60 deg) = 1/2 put partial sums on half-quanta,
# where the last bit of a twiddle (sincospi on the GPU, exp in NumPy) decides
# the rounding.  Both roundings are valid, and each moves one partial value by
# one quantum (1e-7), so the FP64 bars are one quantum's scale: 1e-7 in the
# forces and 1e-8 in energy and virial, and a quarter of the int32 effect
# itself (int32 against exact transforms).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mesh", PAPER_GRIDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_int32_transforms_match_oracle(torch_dev, mesh, precision):
    import paper_2504_15508_amd as dl
    torch = torch_dev
    s = small_water()
    ref = s.rounded(np.float32) if precision == "fp32" else s
    dt = torch.float64 if precision == "fp64" else torch.float32
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    plan = dl.Plan(mesh, order=5, beta=BETA, coulomb_k=KE, precision=precision, capacity=s.n)
    plan.set_box(s.box)
    plan.set_fft_int32((2, 3, 2), 1e7)
    E, fi, fw, W = plan.compute(t(ref.ion_pos), t(ref.ion_q), t(ref.wc_pos), t(ref.wc_q))
    torch.cuda.synchronize()
    F = np.concatenate([fi.double().cpu().numpy(), fw.double().cpu().numpy()])
    E0, F0, W0 = pppm.pppm_int32(ref.all_pos(), ref.all_q(), ref.box, mesh, 5, BETA, KE, (2, 3, 2), 1e7)
    E1, F1, _ = pppm.pppm(ref.all_pos(), ref.all_q(), ref.box, mesh, 5, BETA, KE)
    dE, dF = abs(float(E) - E0) / abs(E0), rel(F, F0)
    dW = np.abs(W.cpu().numpy() - W0).max() / abs(E0)
    print(f"int32 {mesh} {precision}: dE={dE:.2e} dF={dF:.2e} dW={dW:.2e}  "
          f"(int32 vs exact transforms: {rel(F0, F1):.2e})", flush=True)
    assert plan.q32_clamped() == 0
    if precision == "fp64":
        assert dF <= 1e-7 and dE <= 1e-8 and dW <= 1e-8
        assert dF <= 0.25 * rel(F0, F1)
    else:
        # FP32 partial sums carry ~1e-7 relative rounding, several quanta at
        # scale 1e7, so FP32 int32 transforms cannot match the oracle's
        # quantised values; their parity is that of any FP32 plan (the int32
        # arithmetic itself is pinned by the FP64 tests above and below)
        assert dF <= FP32_TOL_F and dE <= FP32_TOL_E and dW <= FP32_TOL_E


# ---------------------------------------------------------------------------
# The int32-quantised transform element by element, one axis at a time on
# identical inputs: the kernel (through dplr_lr_debug_dft_q32) and the
# oracle's dft_axis_int32 transform the same data, the input of each axis
# being the oracle's output of the previous one (the charge mesh forward along
# x, y, z; the three field spectra back along x, y, z).  Every output is an
# integer multiple of the quantum 1/scale on both sides.  The two may differ
# only where a node's partial value lies on a half-quantum, where the last
# bit of a twiddle decides the rounding: a partial counts as tied when its
# scaled value is within 1e-6 of k + 1/2 (about 30 FP64 ulp at the largest
# values here).  So every output must satisfy
#   |GPU - oracle| in quanta <= number of its tied partials,
# which fails for any difference that a tie does not explain (a dropped or
# doubled partial, a wrong twiddle, rounding in the wrong precision).
# ---------------------------------------------------------------------------
def _ties(parts, axis):
    """Tied partials per output (real, imaginary) from the oracle's unrounded
    scaled partials [nodes, ..., K] (axis last)."""
    def count(v):
        return (np.abs(v - (np.floor(v) + 0.5)) <= 1e-6).sum(axis=0)
    return np.moveaxis(count(parts.real), -1, axis), np.moveaxis(count(parts.imag), -1, axis)


@pytest.mark.parametrize("mesh", [(10, 15, 10), (12, 18, 12)])
def test_int32_axis_transforms_elementwise(torch_dev, mesh):
    import paper_2504_15508_amd as dl
    torch = torch_dev
    nodes, scale = (2, 3, 2), 1e7
    s = small_water()
    V = float(np.prod(s.box))
    plan = dl.Plan(mesh, order=5, beta=BETA, coulomb_k=KE, precision="fp64", capacity=s.n)
    plan.set_box(s.box)
    plan.set_fft_int32(nodes, scale)

    def gpu_axis(x, axis, sign):
        t = torch.tensor(np.ascontiguousarray(np.moveaxis(x, (0, 1, 2), (2, 1, 0))), dtype=torch.complex128,
                         device="cuda")
        plan.debug_dft_q32(axis, sign, t)
        torch.cuda.synchronize()
        return np.moveaxis(t.cpu().numpy(), (0, 1, 2), (2, 1, 0))

    stats = dict(outputs=0, mismatched=0, ties=0)

    def check(x, axis, sign):
        out_o, parts = pppm.dft_axis_int32(x, axis, nodes[axis], scale, sign, return_partials=True)
        out_g = gpu_axis(x, axis, sign)
        tr, ti = _ties(parts, axis)
        for g, o, t in ((out_g.real, out_o.real, tr), (out_g.imag, out_o.imag, ti)):
            q = (g - o) * scale
            dq = np.rint(q)
            assert np.abs(q - dq).max() <= 1e-5          # both sides on the quantum grid
            bad = np.abs(dq) > t
            assert not bad.any(), (axis, sign, int(bad.sum()), float(np.abs(dq).max()))
            stats["outputs"] += dq.size
            stats["mismatched"] += int((dq != 0).sum())
            stats["ties"] += int(t.sum())
        return out_o

    Q = pppm.spread(s.all_pos(), s.all_q(), s.box, mesh, 5).astype(np.complex128)
    Qh = Q
    for a in range(3):
        Qh = check(Qh, a, -1)
    G = pppm.influence(s.box, mesh, BETA, 5)
    n, k = pppm.wavevectors(s.box, mesh)
    for a in range(3):
        kd = np.where(n[a] == -mesh[a] // 2, 0.0, k[a]) if mesh[a] % 2 == 0 else k[a]
        shape = [1, 1, 1]
        shape[a] = mesh[a]
        Ea = (KE / V) * (-1j * kd.reshape(shape) * G * Qh)
        for b in range(3):
            Ea = check(Ea, b, +1)
    print(f"int32 axis transforms {mesh}: {stats['mismatched']} of {stats['outputs']} outputs differ by one "
          f"quantum per tied partial; {stats['ties']} tied partials", flush=True)
    plan.close()


def test_int32_mode_switches_and_rejections(torch_dev):
    import paper_2504_15508_amd as dl
    torch = torch_dev
    s = small_water()
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    plan = dl.Plan((10, 15, 10), order=5, beta=BETA, coulomb_k=KE, precision="fp64", capacity=s.n)
    plan.set_box(s.box)
    args = (t(s.ion_pos), t(s.ion_q), t(s.wc_pos), t(s.wc_q))
    _, fa, _, _ = plan.compute(*args)
    fa = fa.clone()
    plan.set_fft_int32((2, 3, 2))
    _, fb, _, _ = plan.compute(*args)
    fb = fb.clone()
    plan.set_fft_int32(None)
    _, fc, _, _ = plan.compute(*args)
    torch.cuda.synchronize()
    assert torch.equal(fa, fc) and not torch.equal(fa, fb)
    with pytest.raises(Exception, match="divide"):
        plan.set_fft_int32((3, 3, 2))
    with pytest.raises(Exception, match="scale"):
        plan.set_fft_int32((2, 3, 2), 0.0)
    p2 = dl.Plan(32, order=5, precision="fp64", capacity=10)
    with pytest.raises(Exception, match="mixed-radix"):
        p2.set_fft_int32((2, 2, 2))


def test_full_size_split_plane_spread(torch_dev):
    # 288,768 charges on a mesh with 30 z planes: the plane spread splits the
    # particles over 8 blocks per plane and adds the integer partial planes
    w = systems.workload(3)
    s = w.system()
    check_vs_pppm(torch_dev, s, (60, 48, 30), 5, "fp32", FP32_TOL_F, FP32_TOL_E, FP32_TOL_E)


def test_full_size_mixed_mesh_fp32(torch_dev):
    # the benchmark's 216,576 atoms + 72,192 WCs on a 120^3 mesh (the bench
    # leg's launch), element-wise against the oracle at the same mesh
    w = systems.workload(3)
    s = w.system()
    check_vs_pppm(torch_dev, s, (120, 120, 120), 5, "fp32", FP32_TOL_F, FP32_TOL_E, FP32_TOL_E)


def test_mixed_plan_debug_buffers(torch_dev):
    import paper_2504_15508_amd as dl
    box = np.array([16.0, 16.0, 16.0])
    plan = dl.Plan((12, 18, 12), order=5, beta=BETA, coulomb_k=KE, precision="fp64", capacity=4)
    plan.set_box(box)
    torch_dev.cuda.synchronize()
    G = plan.debug_buffer(dl._lib.BUF_INFLUENCE).cpu().numpy()
    G0 = pppm.influence(box, (12, 18, 12), BETA, 5)
    assert np.abs(G - G0[:7, :10, :7]).max() <= 1e-13 * np.abs(G0).max()
    with pytest.raises(ValueError, match="not available"):
        plan.debug_buffer(dl._lib.BUF_SPECTRUM)


def test_int32_saturation_matches_oracle(torch_dev):
    # at a scale of 2e9 every partial value above ~1.07 overflows int32 and
    # clamps; the kernels must clamp exactly as the oracle does (a scale that
    # is not a power of two, so that no exact half-quantum ties arise)
    import paper_2504_15508_amd as dl
    torch = torch_dev
    s = small_water()
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    plan = dl.Plan((10, 15, 10), order=5, beta=BETA, coulomb_k=KE, precision="fp64", capacity=s.n)
    plan.set_box(s.box)
    plan.set_fft_int32((2, 3, 2), 2e9)
    E, fi, fw, W = plan.compute(t(s.ion_pos), t(s.ion_q), t(s.wc_pos), t(s.wc_q))
    torch.cuda.synchronize()
    F = np.concatenate([fi.cpu().numpy(), fw.cpu().numpy()])
    E0, F0, W0 = pppm.pppm_int32(s.all_pos(), s.all_q(), s.box, (10, 15, 10), 5, BETA, KE, (2, 3, 2), 2e9)
    E1, F1, _ = pppm.pppm(s.all_pos(), s.all_q(), s.box, (10, 15, 10), 5, BETA, KE)
    print(f"saturated int32: dE={abs(float(E) - E0) / abs(E0):.2e} dF={rel(F, F0):.2e} "
          f"(vs exact transforms {rel(F0, F1):.2e})", flush=True)
    assert rel(F0, F1) > 1e-3            # the clamp really changes the result
    assert plan.q32_clamped() > 0        # and the library reports it
    # agreement to the quantum's scale (5e-10: a value whose FP64 rounding in
    # the two summation orders straddles a half-quantum moves by one quantum)
    assert rel(F, F0) <= 1e-8 and abs(float(E) - E0) <= 1e-9 * abs(E0)


def test_int32_longest_rows(torch_dev):
    # int32 transforms take rows up to 256 points: 240 points on 8 nodes
    import paper_2504_15508_amd as dl
    torch = torch_dev
    s = small_water()
    mesh, nodes = (240, 12, 10), (8, 2, 2)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    plan = dl.Plan(mesh, order=5, beta=BETA, coulomb_k=KE, precision="fp64", capacity=s.n)
    plan.set_box(s.box)
    plan.set_fft_int32(nodes, 1e7)
    E, fi, fw, W = plan.compute(t(s.ion_pos), t(s.ion_q), t(s.wc_pos), t(s.wc_q))
    torch.cuda.synchronize()
    F = np.concatenate([fi.cpu().numpy(), fw.cpu().numpy()])
    E0, F0, W0 = pppm.pppm_int32(s.all_pos(), s.all_q(), s.box, mesh, 5, BETA, KE, nodes, 1e7)
    print(f"int32 {mesh} nodes {nodes}: dE={abs(float(E) - E0) / abs(E0):.2e} dF={rel(F, F0):.2e}", flush=True)
    assert rel(F, F0) <= 1e-7 and abs(float(E) - E0) <= 1e-8 * abs(E0)
