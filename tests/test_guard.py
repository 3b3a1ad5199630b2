"""The learned form's fallback decision is a host function: every trigger is
exercised on the CPU without a GPU."""
import pytest

from paper_2504_15508_amd import _lib


def decide(cfg, st):
    from paper_2504_15508_amd.learned import guard_decide
    return guard_decide(cfg, st)


CFG = dict(max_audit_rel_rmse=1e-3, max_correction_ratio=0.5, audit_interval=10, min_neighbours=5.0,
           max_neighbours=80.0)
OK = dict(audit_valid=1, audit_rel_rmse=5e-4, steps_since_audit=2, max_correction=0.1, max_force=10.0,
          min_neighbours=20.0, max_neighbours=50.0, unseen_charges=0)


def test_learned_when_everything_in_range():
    assert decide(CFG, OK) == _lib.GUARD_LEARNED


@pytest.mark.parametrize("change,expect", [
    (dict(audit_valid=0), _lib.GUARD_AUDIT),
    (dict(steps_since_audit=10), _lib.GUARD_AUDIT),
    (dict(audit_rel_rmse=2e-3), _lib.GUARD_FINE),
    (dict(unseen_charges=3), _lib.GUARD_FINE),
    (dict(min_neighbours=2.0), _lib.GUARD_FINE),
    (dict(max_neighbours=120.0), _lib.GUARD_FINE),
    (dict(max_correction=6.0), _lib.GUARD_FINE),
])
def test_each_trigger(change, expect):
    assert decide(CFG, {**OK, **change}) == expect


def test_disabled_checks():
    cfg = dict(CFG, max_correction_ratio=0.0, min_neighbours=0.0, max_neighbours=0.0)
    assert decide(cfg, {**OK, "max_correction": 1e9, "min_neighbours": 0.0, "max_neighbours": 1e9}) == _lib.GUARD_LEARNED


def test_null_arguments_rejected():
    import ctypes
    d = ctypes.c_int32()
    assert _lib.load().dplr_lr_guard_decide(None, None, ctypes.byref(d)) == _lib.E_INVALID
