"""The C-ABI library loads, exports every function that include/vplbm.h declares,
and rejects invalid arguments before touching a device (runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_1905_05110_amd import build, vplbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "vplbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(lbm_[a-z_0-9]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    build.build(force=False)
    return vplbm.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(vplbm.EXPORTS)


def test_struct_sizes_match_header(lib):
    assert C.sizeof(vplbm.Body) == 8 * 7 + 4 + 4 + 8 * 2 + 8 * 12 + 8 * 4 + 8
    assert vplbm.RECORD_DTYPE.itemsize == 128


def _create(lib, nx=10, ny=8, rates=(1.6, 1.5, 1.9, 1.2), eta=1e-3, **kw):
    spec = dict(nx=nx, ny=ny, rates=rates, eta=eta)
    spec.update(kw)
    o = vplbm.make_opts(spec)
    h = C.c_void_p()
    rc = lib.lbm_create(nx, ny, vplbm.Rates(*rates), eta, C.byref(o), C.byref(h))
    return rc, h, lib.lbm_last_error(None).decode()


@pytest.mark.parametrize("kw,frag", [
    (dict(nx=2), "nx and ny"),
    (dict(ny=1), "nx and ny"),
    (dict(rates=(0.0, 1.5, 1.9, 1.2)), "rates"),
    (dict(rates=(1.6, 1.5, 2.0, 1.2)), "rates"),
    (dict(eta=0.0), "eta"),
    (dict(eta=-1.0), "eta"),
    (dict(bc=("periodic", "wall", "wall", "wall")), "pairs"),
    (dict(bc=("outflow", "wall", "wall", "wall")), "OUTFLOW"),
    (dict(bc=("wall", "wall", "outflow", "wall")), "OUTFLOW"),
    (dict(storage=7), "storage"),
    (dict(storage="fp16", fp16_scale_log2=20), "fp16_scale"),
])
def test_invalid_arguments_are_rejected(lib, kw, frag):
    rc, h, msg = _create(lib, **kw)
    assert rc == vplbm.LBM_ERR_ARG
    assert frag in msg
    assert not h.value


def test_null_handles_are_rejected(lib):
    assert lib.lbm_step(None, 1) == vplbm.LBM_ERR_ARG
    assert lib.lbm_sync(None) == vplbm.LBM_ERR_ARG
    assert lib.lbm_destroy(None) == vplbm.LBM_ERR_ARG
    assert lib.lbm_step_index(None) == -1
    assert lib.lbm_pop_bytes(0, 5, 1) == 0
    assert lib.lbm_pop_bytes(10, 5, 1) > 9 * 10 * 5 * 4


def test_create_without_device_reports_hip_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h, msg = _create(lib)
    assert rc == vplbm.LBM_ERR_HIP
    assert msg
