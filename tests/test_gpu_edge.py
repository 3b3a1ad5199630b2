"""GPU edge cases of the C ABI: empty and one-sided inputs, wrapping of
coordinates outside the box, flags, capacity/box errors, repeated calls with
shrinking inputs and non-neutral charge sets.  Every numeric result is checked
against the oracle.  FP64 plans accumulate the charge mesh in 64-bit fixed
point (quantum 2^-40), which bounds their agreement with the FP64 oracle at
~1e-11 relative; the bar used here is 1e-10."""
import numpy as np
import pytest

import systems
from oracle import pppm

pytestmark = pytest.mark.gpu

KE = systems.COULOMB_K
BETA = systems.BETA


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return t


@pytest.fixture(scope="module")
def dl():
    import paper_2504_15508_amd as m
    return m


def _t(torch, a, dt):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(np.shape(a)), dtype=dt, device="cuda")


def _plan(dl, mesh=32, order=5, precision="fp64", capacity=1000, flags=0, box=(12.42,) * 3):
    p = dl.Plan(mesh, order=order, beta=BETA, coulomb_k=KE, precision=precision,
                capacity=capacity, flags=flags)
    p.set_box(box)
    return p


def _ref(pos, q, box, mesh=32, order=5):
    return pppm.pppm(np.asarray(pos, float).reshape(-1, 3), np.asarray(q, float), np.asarray(box, float),
                     (mesh,) * 3, order, BETA, KE)


@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_empty_input(torch, dl, diff):
    p = _plan(dl, flags=dl._lib.DIFF_AD if diff == "ad" else 0)
    E, fi, fw, W = p.compute(None, None, None, None)
    torch.cuda.synchronize()
    assert float(E) == 0.0 and np.all(W.cpu().numpy() == 0.0)
    assert fi.shape == (0, 3) and fw.shape == (0, 3)


@pytest.mark.parametrize("side", ["ions_only", "wcs_only"])
def test_one_sided_sets(torch, dl, side):
    s = systems.workload(1).system()
    p = _plan(dl)
    dt = torch.float64
    if side == "ions_only":
        E, fi, fw, W = p.compute(_t(torch, s.ion_pos, dt), _t(torch, s.ion_q, dt))
        pos, q = s.ion_pos, s.ion_q
        F = fi.cpu().numpy()
    else:
        E, fi, fw, W = p.compute(None, None, _t(torch, s.wc_pos, dt), _t(torch, s.wc_q, dt))
        pos, q = s.wc_pos, s.wc_q
        F = fw.cpu().numpy()
    E0, F0, W0 = _ref(pos, q, s.box)      # non-neutral: computed as given
    assert abs(float(E) - E0) <= 1e-10 * abs(E0)
    assert np.abs(F - F0).max() <= 1e-10 * np.abs(F0).max()


def test_single_particle(torch, dl):
    p = _plan(dl)
    pos = np.array([[3.3, 7.1, 0.2]])
    q = np.array([1.5])
    E, fi, _, W = p.compute(_t(torch, pos, torch.float64), _t(torch, q, torch.float64))
    E0, F0, W0 = _ref(pos, q, [12.42] * 3)
    assert abs(float(E) - E0) <= 1e-10 * abs(E0)
    # one charge feels only the mesh's aliasing self-force, which is tiny
    assert np.abs(fi.cpu().numpy() - F0).max() <= 1e-9


def test_coordinates_outside_box_are_wrapped(torch, dl):
    s = systems.workload(1).system()
    L = s.box[0]
    rng = np.random.default_rng(1)
    shift = rng.integers(-3, 4, size=s.ion_pos.shape) * L
    ion = s.ion_pos + shift
    ion[0] = [0.0, 0.0, 0.0]
    ion[1] = [L, L, L]                   # exactly on the far face: same as 0
    ion[2] = [-1e-13, L - 1e-13, 2 * L]
    p = _plan(dl)
    dt = torch.float64
    E, fi, fw, W = p.compute(_t(torch, ion, dt), _t(torch, s.ion_q, dt), _t(torch, s.wc_pos, dt),
                             _t(torch, s.wc_q, dt))
    E0, F0, W0 = _ref(np.concatenate([ion, s.wc_pos]), s.all_q(), s.box)
    F = np.concatenate([fi.cpu().numpy(), fw.cpu().numpy()])
    assert abs(float(E) - E0) <= 1e-10 * abs(E0)
    assert np.linalg.norm(F - F0) <= 1e-10 * np.linalg.norm(F0)


@pytest.mark.parametrize("diff", ["ik", "ad"])
def test_accumulate_and_no_virial_flags(torch, dl, diff):
    s = systems.workload(1).system()
    dt = torch.float64
    args = [_t(torch, s.ion_pos, dt), _t(torch, s.ion_q, dt), _t(torch, s.wc_pos, dt), _t(torch, s.wc_q, dt)]
    extra = dl._lib.DIFF_AD if diff == "ad" else 0
    p0 = _plan(dl, flags=extra)
    E0, fi0, fw0, W0 = p0.compute(*args)
    p1 = _plan(dl, flags=dl._lib.ACCUMULATE | dl._lib.NO_VIRIAL | extra)
    fi = torch.ones_like(fi0)
    fw = torch.full_like(fw0, 2.0)
    vir = torch.full((6,), 7.0, dtype=torch.float64, device="cuda")
    E1, _, _, _ = p1.compute(*args, ion_force=fi, wc_force=fw, virial=vir)
    torch.cuda.synchronize()
    assert torch.allclose(fi, fi0 + 1.0, rtol=0, atol=1e-12)
    assert torch.allclose(fw, fw0 + 2.0, rtol=0, atol=1e-12)
    assert torch.all(vir == 7.0)
    assert abs(float(E1) - float(E0)) <= 1e-12 * abs(float(E0))


def test_errors_are_reported(torch, dl):
    p = dl.Plan(32, order=5, beta=BETA, coulomb_k=KE, precision="fp32", capacity=10)
    x = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    q = torch.zeros(4, dtype=torch.float32, device="cuda")
    with pytest.raises(dl.DplrError) as e:
        p.compute(x, q)
    assert e.value.status == dl._lib.E_NO_BOX
    p.set_box([10.0, 10.0, 10.0])
    big = torch.zeros((11, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(dl.DplrError) as e:
        p.compute(big, torch.zeros(11, dtype=torch.float32, device="cuda"))
    assert e.value.status == dl._lib.E_CAPACITY
    with pytest.raises(ValueError):
        p.compute(x.double(), q.double())
    with pytest.raises(dl.DplrError):
        p.set_box([10.0, -1.0, 10.0])


def test_repeated_calls_with_shrinking_input(torch, dl):
    s = systems.workload(2).system()
    p = _plan(dl, mesh=64, precision="fp64", capacity=s.n, box=tuple(s.box))
    dt = torch.float64
    for n_w in (4096, 1000, 17):
        ni, nw = 3 * n_w, n_w
        E, fi, fw, W = p.compute(_t(torch, s.ion_pos[:ni], dt), _t(torch, s.ion_q[:ni], dt),
                                 _t(torch, s.wc_pos[:nw], dt), _t(torch, s.wc_q[:nw], dt))
        E0, F0, W0 = pppm.pppm(np.concatenate([s.ion_pos[:ni], s.wc_pos[:nw]]),
                               np.concatenate([s.ion_q[:ni], s.wc_q[:nw]]), s.box, (64,) * 3, 5, BETA, KE)
        F = np.concatenate([fi.cpu().numpy(), fw.cpu().numpy()])
        assert abs(float(E) - E0) <= 1e-10 * abs(E0)
        assert np.linalg.norm(F - F0) <= 1e-10 * np.linalg.norm(F0)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("mesh", [32, (12, 18, 12)])
def test_non_finite_coordinates_count_as_zero(torch, dl, precision, mesh):
    """A NaN or infinite coordinate is taken as 0 on its axis (documented in
    the header): the step runs, and its results are those of the same input
    with 0 in place of each non-finite coordinate, bit for bit."""
    s = systems.workload(1).system()
    K = (mesh,) * 3 if isinstance(mesh, int) else mesh
    p = _plan(dl, mesh=K, precision=precision, capacity=s.n, box=tuple(s.box))
    dt = torch.float32 if precision == "fp32" else torch.float64
    bad_i, bad_w = s.ion_pos.copy(), s.wc_pos.copy()
    bad_i[3] = [np.nan, bad_i[3, 1], bad_i[3, 2]]
    bad_i[7] = [np.inf, -np.inf, np.nan]
    bad_w[2] = [bad_w[2, 0], -np.inf, bad_w[2, 2]]
    fix_i, fix_w = np.where(np.isfinite(bad_i), bad_i, 0.0), np.where(np.isfinite(bad_w), bad_w, 0.0)
    iq, wq = _t(torch, s.ion_q, dt), _t(torch, s.wc_q, dt)
    E1, fi1, fw1, W1 = [x.clone() for x in p.compute(_t(torch, bad_i, dt), iq, _t(torch, bad_w, dt), wq)]
    E2, fi2, fw2, W2 = p.compute(_t(torch, fix_i, dt), iq, _t(torch, fix_w, dt), wq)
    torch.cuda.synchronize()
    assert torch.isfinite(fi1).all() and torch.isfinite(fw1).all() and bool(torch.isfinite(E1))
    assert torch.equal(fi1, fi2) and torch.equal(fw1, fw2)
    assert torch.equal(E1, E2) and torch.equal(W1, W2)


def test_fp32_is_bitwise_repeatable(torch, dl):
    """The charge mesh is summed in integers (order-independent), every force
    is accumulated by one thread in a fixed order and the FP64 reductions use
    fixed trees, so two calls give identical bits even though the order of
    particles inside a bin varies between calls (the race check)."""
    s = systems.workload(2).system()
    p = _plan(dl, mesh=64, precision="fp32", capacity=s.n, box=tuple(s.box))
    dt = torch.float32
    args = [_t(torch, s.ion_pos, dt), _t(torch, s.ion_q, dt), _t(torch, s.wc_pos, dt), _t(torch, s.wc_q, dt)]
    E1, fi1, fw1, W1 = [x.clone() for x in p.compute(*args)]
    E2, fi2, fw2, W2 = p.compute(*args)
    F1 = torch.cat([fi1, fw1]).double()
    F2 = torch.cat([fi2, fw2]).double()
    assert torch.equal(F1, F2)
    assert torch.equal(E1, E2) and torch.equal(W1, W2)
