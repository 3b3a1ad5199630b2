"""Pins of the oracle's int32-quantised transforms (the paper's Mixed-Int32
configuration: partial DFT sums of node blocks, scaled by 1e7, rounded to
int32 and summed as integers).

Pinned by: numpy.fft at a fine dyadic scale (2^26, every output within
nodes/2 quanta of it for every node count, which fixes the block
decomposition, the twiddle indices and the sign), the rounding bound
(round to nearest: each output part is within nodes/2 quanta of the exact
DFT, a bound that truncation or a missing block breaks), saturation at the
int32 limits, and end to end the fine-scale limit of pppm_int32 against
pppm() together with the paper's finding that int32 transforms leave the
energy and force errors of the small grids unchanged.
"""
import numpy as np
import pytest

import systems
from oracle import pppm

KE, BETA = systems.COULOMB_K, systems.BETA


@pytest.mark.parametrize("K,nodes", [(12, 1), (12, 2), (12, 3), (15, 3), (10, 5), (18, 3), (8, 2), (16, 4)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fine_scale_reproduces_numpy_fft(K, nodes, sign):
    # |partial| <= K sqrt(2) < 32: a scale of 2^26 stays inside int32
    rng = np.random.default_rng(K * 10 + nodes)
    x = rng.uniform(-1, 1, (3, K, 4)) + 1j * rng.uniform(-1, 1, (3, K, 4))
    y = pppm.dft_axis_int32(x, 1, nodes, 2.0 ** 26, sign)
    ref = np.fft.fft(x, axis=1) if sign < 0 else np.fft.ifft(x, axis=1) * K
    err = y - ref
    bound = nodes * 2.0 ** -27 + 1e-13
    assert np.abs(err.real).max() <= bound and np.abs(err.imag).max() <= bound


@pytest.mark.parametrize("K,nodes", [(12, 2), (15, 3), (18, 3), (10, 2)])
def test_rounding_bound_at_the_paper_scale(K, nodes):
    rng = np.random.default_rng(7 + K)
    x = rng.uniform(-1, 1, (64, K)) + 1j * rng.uniform(-1, 1, (64, K))
    y = pppm.dft_axis_int32(x, 1, nodes, 1e7, -1)
    ref = np.fft.fft(x, axis=1)
    bound = nodes * 0.5e-7 + 1e-14
    err_re, err_im = np.abs((y - ref).real), np.abs((y - ref).imag)
    assert err_re.max() <= bound and err_im.max() <= bound
    # the quanta are really spent: errors reach a good part of the bound
    assert max(err_re.max(), err_im.max()) > 0.25 * bound


def test_saturation_at_int32_limits():
    # one block, constant 300: X[0] = 300 K exceeds (2^31 - 1) / 1e7 and clamps
    x = np.full(6, 300.0 + 0j)
    y = pppm.dft_axis_int32(x, 0, 1, 1e7, -1)
    assert y[0].real == (2 ** 31 - 1) / 1e7
    assert np.abs(y[1:]).max() <= 0.5e-7
    y = pppm.dft_axis_int32(-x, 0, 1, 1e7, -1)
    assert y[0].real == -(2 ** 31) / 1e7


def test_pppm_int32_fine_scale_equals_pppm():
    s = systems.water_box(128, 16.0, seed=20261128)
    K = (10, 15, 10)
    E0, F0, W0 = pppm.pppm(s.all_pos(), s.all_q(), s.box, K, 5, BETA, KE)
    errs = []
    for scale in (2.0 ** 20, 2.0 ** 24):
        E, F, W = pppm.pppm_int32(s.all_pos(), s.all_q(), s.box, K, 5, BETA, KE, (2, 3, 2), scale=scale)
        errs.append(pppm.rel_rmse(F, F0))
        assert abs(E - E0) <= 1e-6 * abs(E0) and np.abs(W - W0).max() <= 1e-5 * abs(E0)
    # the difference is the quantisation alone: 16x finer quanta, ~16x smaller error
    assert errs[1] < 1e-6 and 8 < errs[0] / errs[1] < 32


@pytest.mark.parametrize("K", [(8, 12, 8), (10, 15, 10), (12, 18, 12)])
def test_paper_grids_int32_error_is_negligible(ewald, K):
    # Mixed-Int32 on 2 x 3 x 2 nodes: its change to energy and forces is far
    # below the method error of these grids against the exact sum
    s = systems.water_box(128, 16.0, seed=20261128)
    e0, _, fi, fw = ewald.system_recip(s, BETA, KE)
    f0 = np.concatenate([fi, fw])
    E, F, W = pppm.pppm(s.all_pos(), s.all_q(), s.box, K, 5, BETA, KE)
    Eq, Fq, Wq = pppm.pppm_int32(s.all_pos(), s.all_q(), s.box, K, 5, BETA, KE, (2, 3, 2))
    method = pppm.rel_rmse(F, f0)
    quant = pppm.rel_rmse(Fq, F)
    assert quant < 1e-3 * method
    assert abs(Eq - E) < 1e-3 * abs(E - e0)
