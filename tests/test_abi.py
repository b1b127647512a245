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
    assert C.sizeof(vplbm.Body) == 8 * 7 + 4 + 4 + 8 * 2 + 8 * 12 + 8 * 4 + 8 + 8 + 8
    assert vplbm.RECORD_DTYPE.itemsize == 128 + 24


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
    (dict(tile_width=384), "tile_width"),
    (dict(tile_width=128), "tile_width"),
    (dict(storage="fp16", fp16_scale_log2=20), "fp16_scale"),
    # the step's lane offsets are 32-bit from bases at the tile's rows: the 18 rows a tile
    # reaches must span less than 4 GiB (9 directions of 3.4 M FP64 columns for the ROWS
    # layout, one direction of 30 M FP64 or 60 M FP32 columns for either)
    (dict(nx=3400000, ny=3, storage="fp64", layout="rows"), "4 GiB"),
    (dict(nx=30000000, ny=3, storage="fp64"), "4 GiB"),
    (dict(nx=60000000, ny=3, storage="fp32"), "4 GiB"),
])
def test_invalid_arguments_are_rejected(lib, kw, frag):
    rc, h, msg = _create(lib, **kw)
    assert rc == vplbm.LBM_ERR_ARG
    assert frag in msg
    assert not h.value


def test_invalid_layout_and_offset_reference_are_rejected(lib):
    spec = dict(nx=10, ny=8, rates=(1.6, 1.5, 1.9, 1.2), eta=1e-3)
    for field, value, frag in (("layout", 3, "layout"), ("offset_ref", 3, "offset reference")):
        o = vplbm.make_opts(spec)
        setattr(o, field, value)
        h = C.c_void_p()
        rc = lib.lbm_create(10, 8, vplbm.Rates(1.6, 1.5, 1.9, 1.2), 1e-3, C.byref(o), C.byref(h))
        assert rc == vplbm.LBM_ERR_ARG and frag in lib.lbm_last_error(None).decode()


def test_null_handles_are_rejected(lib):
    assert lib.lbm_step(None, 1) == vplbm.LBM_ERR_ARG
    assert lib.lbm_sync(None) == vplbm.LBM_ERR_ARG
    assert lib.lbm_destroy(None) == vplbm.LBM_ERR_ARG
    assert lib.lbm_step_index(None) == -1
    assert lib.lbm_pop_bytes(0, 5, 1) == 0
    assert lib.lbm_pop_bytes(10, 5, 1) > 9 * 10 * 5 * 4


@pytest.mark.parametrize("nx,rp", [(3, 64), (64, 64), (65, 192), (128, 192), (500, 576),
                                   (512, 576), (576, 576), (640, 704), (1024, 1088),
                                   (8192, 8256)])
def test_population_rows_are_padded_to_an_odd_multiple_of_64(lib, nx, rp):
    # lbm_pop_bytes = 9 (rp ny + 320) elements, rp the row pitch: nx rounded up to an odd
    # multiple of 64 elements, in every storage
    ny = 7
    for storage, e in ((0, 8), (1, 4), (2, 2), (3, 2)):
        assert lib.lbm_pop_bytes(nx, ny, storage) == 9 * (rp * ny + 320) * e


def test_create_without_device_reports_hip_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h, msg = _create(lib)
    assert rc == vplbm.LBM_ERR_HIP
    assert msg


def _batch_desc(nx=10, ny=8, rates=(1.6, 1.5, 1.9, 1.2), eta=1e-3):
    d = vplbm.BatchDesc()
    d.nx, d.ny = nx, ny
    d.rates = vplbm.Rates(*rates)
    d.eta = eta
    return d


@pytest.mark.parametrize("field,value,frag", [
    ("order", 3, "order"),
    ("store_mode", 5, "store mode"),
    ("storage", 9, "storage"),
    ("rows_per_tile", 3, "rows_per_tile"),
    ("tile_width", 384, "tile_width"),
    ("tile_width", 128, "tile_width"),
])
def test_invalid_batch_options_are_rejected(lib, field, value, frag):
    descs = (vplbm.BatchDesc * 2)(_batch_desc(), _batch_desc(12, 9))
    bo = vplbm.BatchOpts()
    lib.lbm_default_batch_opts(C.byref(bo))
    setattr(bo, field, value)
    h = C.c_void_p()
    assert lib.lbm_batch_create(2, descs, C.byref(bo), C.byref(h)) == vplbm.LBM_ERR_ARG
    assert frag in lib.lbm_batch_last_error(None).decode()
    assert not h.value


def test_batch_null_arguments_are_rejected(lib):
    h = C.c_void_p()
    descs = (vplbm.BatchDesc * 1)(_batch_desc())
    assert lib.lbm_batch_create(0, descs, None, C.byref(h)) == vplbm.LBM_ERR_ARG
    assert lib.lbm_batch_create(1, None, None, C.byref(h)) == vplbm.LBM_ERR_ARG
    assert lib.lbm_batch_step(None, 1) == vplbm.LBM_ERR_ARG
    assert lib.lbm_batch_sync(None) == vplbm.LBM_ERR_ARG
    assert lib.lbm_batch_destroy(None) == vplbm.LBM_ERR_ARG
    assert lib.lbm_batch_size(None) == -1
    assert lib.lbm_batch_sim(None, 0, C.byref(h)) == vplbm.LBM_ERR_ARG


def test_structs_match_the_header(tmp_path):
    """Sizes and field offsets of the binding's ctypes structures against the C compiler's
    reading of include/vplbm.h."""
    import subprocess
    structs = {"lbm_opts": vplbm.Opts, "lbm_batch_opts": vplbm.BatchOpts,
               "lbm_batch_desc": vplbm.BatchDesc, "lbm_body": vplbm.Body,
               "lbm_rates": vplbm.Rates, "lbm_adjoint_opts": vplbm.AdjointOpts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "vplbm.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append('return 0; }')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", inc, "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_batch_create_without_device_reports_hip_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    descs = (vplbm.BatchDesc * 2)(_batch_desc(), _batch_desc(12, 9))
    h = C.c_void_p()
    assert lib.lbm_batch_create(2, descs, None, C.byref(h)) == vplbm.LBM_ERR_HIP
    assert lib.lbm_batch_last_error(None).decode()
    assert not h.value


def _adj_create(lib, storage="fp64", mode="fixed", steps=8, every=4):
    spec = dict(nx=10, ny=8, rates=(1.6, 1.5, 1.9, 1.2), eta=1e-3, storage=storage)
    o = vplbm.make_opts(spec)
    b = vplbm.make_body(dict(radius=2.0, x=4.0, y=4.0, mode=mode, mass=1.0, inertia=1.0))
    ao = vplbm.AdjointOpts()
    lib.lbm_default_adjoint_opts(C.byref(ao))
    ao.steps, ao.checkpoint_every = steps, every
    h = C.c_void_p()
    rc = lib.lbm_adjoint_create(10, 8, vplbm.Rates(1.6, 1.5, 1.9, 1.2), 1e-3, C.byref(o),
                                C.byref(b), C.byref(ao), C.byref(h))
    return rc, h, lib.lbm_adjoint_last_error(None).decode()


@pytest.mark.parametrize("kw,frag", [
    (dict(steps=10, every=4), "multiple"),
    (dict(steps=9, every=3), "even"),
    (dict(steps=0, every=4), "steps"),
    (dict(mode="free"), "FIXED"),
    (dict(storage="fp16"), "FP64 or FP32"),
])
def test_invalid_adjoint_arguments_are_rejected(lib, kw, frag):
    rc, h, msg = _adj_create(lib, **kw)
    assert rc == vplbm.LBM_ERR_ARG
    assert frag in msg
    assert not h.value


def test_adjoint_null_handles_and_layout(lib):
    assert C.sizeof(vplbm.AdjointOpts) == 8 + 8 + 8 + 8 + 8
    J = C.c_double()
    assert lib.lbm_adjoint_forward(None, C.byref(J)) == vplbm.LBM_ERR_ARG
    assert lib.lbm_adjoint_backward(None) == vplbm.LBM_ERR_ARG
    assert lib.lbm_adjoint_gradient(None, None, None, None) == vplbm.LBM_ERR_ARG
    assert lib.lbm_adjoint_destroy(None) == vplbm.LBM_ERR_ARG
