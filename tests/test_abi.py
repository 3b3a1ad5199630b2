"""The C ABI on the CPU: the shared library loads without a GPU, exports every
function include/dplr_lr.h declares, and validates configurations on the host
(no device call is made by these checks)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2504_15508_amd import _lib
    return _lib


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dplr_lr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dplr_lr_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    handle = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(handle, n)]
    assert not missing, missing
    assert sorted(lib.EXPORTS) == names


def test_abi_version(lib):
    assert lib.load().dplr_lr_abi_version() == 1


def _cfg(lib, **kw):
    c = lib.Config()
    lib.load().dplr_lr_config_default(ctypes.byref(c))
    for k, v in kw.items():
        if k == "mesh":
            c.mesh[:] = v
        else:
            setattr(c, k, v)
    return c


def _validate(lib, c):
    buf = ctypes.create_string_buffer(256)
    st = lib.load().dplr_lr_config_validate(ctypes.byref(c), buf, 256)
    return st, buf.value.decode()


def test_default_config_is_valid(lib):
    c = _cfg(lib)
    assert list(c.mesh) == [32, 32, 32] and c.order == 5 and c.beta == 0.4
    assert abs(c.coulomb_k - 14.399645) < 1e-12
    assert _validate(lib, c) == (lib.OK, "")


@pytest.mark.parametrize("kw,status", [
    (dict(mesh=[14, 32, 32]), "E_UNSUPPORTED"),
    (dict(mesh=[4, 32, 32]), "E_UNSUPPORTED"),
    (dict(mesh=[48, 32, 32], flags=0x4), "E_UNSUPPORTED"),
    (dict(mesh=[1024, 32, 32]), "E_UNSUPPORTED"),
    (dict(mesh=[960, 32, 32]), "E_UNSUPPORTED"),
    (dict(mesh=[0, 32, 32]), "E_INVALID"),
    (dict(order=9), "E_UNSUPPORTED"),
    (dict(order=1), "E_UNSUPPORTED"),
    (dict(order=0), "E_INVALID"),
    (dict(beta=0.0), "E_INVALID"),
    (dict(beta=float("nan")), "E_INVALID"),
    (dict(coulomb_k=float("inf")), "E_INVALID"),
    (dict(precision=2), "E_INVALID"),
    (dict(alias_range=5), "E_INVALID"),
    (dict(capacity=-1), "E_INVALID"),
    (dict(capacity=2 ** 31), "E_INVALID"),
    (dict(flags=0x10), "E_INVALID"),
])
def test_invalid_configs_rejected(lib, kw, status):
    st, msg = _validate(lib, _cfg(lib, **kw))
    assert lib.STATUS_NAMES[st] == status and msg


@pytest.mark.parametrize("mesh", [[48, 32, 32], [8, 12, 8], [10, 15, 10], [12, 18, 12], [5, 5, 5], [8, 8, 8],
                                  [512, 375, 500]])
def test_mixed_radix_meshes_accepted(lib, mesh):
    # sizes with prime factors 2, 3 and 5 only, each at least the order
    assert _validate(lib, _cfg(lib, mesh=mesh)) == (lib.OK, "")


def test_plan_create_rejects_before_device_work(lib):
    h = ctypes.c_void_p(123)
    st = lib.load().dplr_lr_plan_create(ctypes.byref(_cfg(lib, order=0)), None, ctypes.byref(h))
    assert st == lib.E_INVALID and h.value is None
    assert b"order" in lib.load().dplr_lr_last_error(None)


def test_null_plan_calls_fail_cleanly(lib):
    L = lib.load()
    box = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    assert L.dplr_lr_set_box(None, box) == lib.E_INVALID
    assert L.dplr_lr_compute_energy_forces_virial(None, 0, None, None, 0, None, None, None, None, None,
                                                  None) == lib.E_INVALID
    assert L.dplr_lr_plan_destroy(None) == lib.OK
    nodes = (ctypes.c_int32 * 3)(2, 3, 2)
    assert L.dplr_lr_set_fft_int32(None, nodes, 1e7) == lib.E_INVALID
    assert L.dplr_lr_workspace_bytes(None) == 0
    assert L.dplr_lr_profile_stage_name(3) == b"spread_fftx"
    assert L.dplr_lr_profile_stage_name(99) == b""


def test_product_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2504_15508_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.replace("oracle-free", ""), f
