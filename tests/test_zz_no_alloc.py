"""The entry point that allocates nothing (lbm_step_static), through the C ABI: the same
steps as lbm_step with graphs off, the partial force sums in the library's static
array instead of the simulation's own."""
import numpy as np
import pytest

from paper_1905_05110_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_05110_amd import vplbm
    vplbm.load_library()
    return vplbm


def _pair(gpu, spec, body, steps):
    a = gpu.Sim(spec, body)
    b = gpu.Sim(spec, body)
    a.step(steps)
    b.step_static(steps)
    fa, fb = a.get_populations(), b.get_populations()
    ra, rb = a.forces(), b.forces()
    a.close()
    b.close()
    assert np.array_equal(fa, fb)
    assert len(ra) == len(rb) == steps
    for key in ("step", "fvp", "tvp", "pin", "fh", "th", "q", "v", "fmem", "tmem"):
        assert np.array_equal(ra[key], rb[key]), key


@pytest.mark.parametrize("tile", [256, 64])
def test_static_steps_match_lbm_step_two_calls(gpu, tile):
    """Two calls in a row, the second on a smaller grid with a smaller body: each is
    bitwise the plain stepping of the same simulation (the array keeps the first call's
    contents, which the second must not read); 256- or 64-column tiles."""
    wl = W.imposed_oscillation(storage="fp32", nx=600, ny=90, D=24.0)
    wl["body"].update(mode="free", free_mask=7, mass=400.0, inertia=4000.0, k=(0.01, 0.01, 0.0),
                      force_model="vp+mem")
    _pair(gpu, dict(wl["spec"], tile_width=tile), wl["body"], 30)
    small = W.imposed_oscillation(storage="fp64", nx=120, ny=48, D=12.0)
    _pair(gpu, dict(small["spec"], tile_width=tile), small["body"], 17)


def test_static_and_plain_steps_interleave(gpu):
    """Plain and static steps in any order continue one run bitwise (each kind finds the
    state final and reads only its own slots); graphs replayed in between."""
    wl = W.imposed_oscillation(storage="fp32", nx=600, ny=90, D=24.0)
    a = gpu.Sim(wl["spec"], wl["body"])
    b = gpu.Sim(wl["spec"], wl["body"], graph_steps=8)
    a.step(40)
    b.step(5)
    b.step_static(7)
    b.step(16)
    b.step_static(12)
    assert np.array_equal(a.get_populations(), b.get_populations())
    assert np.array_equal(a.forces()["fvp"], b.forces()["fvp"])
    a.close()
    b.close()


def test_static_steps_refuse_a_body_beyond_the_array(gpu):
    """A disc spanning more tiles than the static array's slots: refused, nothing run."""
    spec = W.channel_spec(1024, 12000, 0.05, 0.6)
    body = W.fixed_disc(11000.0, 512.0, 6000.0)
    g = gpu.Sim(dict(spec, rows_per_tile=1, tile_width=256), body)
    with pytest.raises(gpu.LbmError) as e:
        g.step_static(1)
    assert e.value.code == gpu.LBM_ERR_ARG and "static" in str(e.value)
    assert g.step_index() == 0
    g.close()
