"""GPU (HIP, through the C ABI) against the FP64 CPU oracle, element by element.

Tolerances (relative, as defined for this project): populations and densities
max|a - b| <= tol * max|b|; velocities max|a - b| <= tol * U; forces
max_n |F_gpu(n) - F_orc(n)| <= tol * max_n |F_orc(n)|.  FP64 storage: tol = 1e-12.
"""
import sys

import numpy as np
import pytest

from paper_1905_05110_amd import workloads as W

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_05110_amd import vplbm
    vplbm.load_library()
    return vplbm


def spec_of(nx, ny, bc, tau=0.7, storage="fp64", g=(0.0, 0.0), u_wall=None, u_conv=0.0,
            u0=(0.0, 0.0), rates=None):
    return dict(nx=nx, ny=ny, rates=rates or (1.64, 1.54, 1.9, 1.0 / tau), eta=1e-3, bc=bc,
                u_wall=u_wall or [[0.0, 0.0]] * 4, u_conv=u_conv, g_fluid=g, rho0=1.0, u0=u0,
                storage=storage)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def force_err(ra, rb, radius=None):
    """Relative force errors.  Torques (and the angular part of the internal momentum)
    are summed from terms r x dF that cancel; their round-off scales with
    R * max|F|, which is added to their scale."""
    out = {}
    R = radius if radius is not None else 0.0
    fscale = max(np.abs(rb["fvp"]).max(), np.abs(rb["fh"]).max(), np.abs(rb["fmem"]).max())
    pscale = np.abs(rb["pin"][:, :2]).max() if len(rb) else 0.0
    for key in ("fvp", "fh", "fmem"):
        out[key] = rel(ra[key], rb[key])
    out["pin"] = max(np.abs(ra["pin"][:, :2] - rb["pin"][:, :2]).max() / max(pscale, 1e-300),
                     np.abs(ra["pin"][:, 2] - rb["pin"][:, 2]).max()
                     / max(np.abs(rb["pin"][:, 2]).max() + R * pscale, 1e-300))
    for key in ("tvp", "th", "tmem"):
        out[key] = np.abs(ra[key] - rb[key]).max() / max(np.abs(rb[key]).max() + R * fscale,
                                                          1e-300)
    out["q"] = np.abs(ra["q"] - rb["q"]).max()
    out["v"] = np.abs(ra["v"] - rb["v"]).max()
    return out


BCS = {
    "periodic": ("periodic",) * 4,
    "channel": ("velocity", "outflow", "symmetry", "symmetry"),
    "wallbox": ("wall",) * 4,
    "symbox": ("symmetry",) * 4,
    "mixed": ("velocity", "outflow", "wall", "velocity"),
    "pipe": ("periodic", "periodic", "wall", "symmetry"),
}
UWALL = [[0.04, 0.01], [0.0, 0.0], [0.0, 0.0], [0.03, -0.005]]


def body_of(kind, nx, ny, smooth):
    D = min(nx, ny) * 0.45
    b = W.fixed_disc(D, nx * 0.42 + 0.17, ny * 0.5 - 0.23, smooth_delta=1.0 if smooth else 0.0)
    b["force_model"] = "vp+mem"  # record the momentum-exchange load alongside
    if kind == "fixed":
        b.update(vx=0.002, omega=0.001)
    elif kind == "imposed":
        b.update(mode="imposed_sin", imp_amp=0.8, imp_freq=0.05, imp_y0=ny * 0.5 - 0.23,
                 imp_phase=0.7)
    elif kind == "free":
        b.update(mode="free", free_mask=7, mass=400.0, inertia=3000.0, k=(0.01, 0.02, 0.0),
                 c=(0.001, 0.0, 0.0), q0=(b["x"], b["y"], 0.0), f_ext=(1e-4, -2e-4, 0.0))
    elif kind == "free_mem":  # driven by the momentum-exchange load
        b.update(mode="free", free_mask=7, mass=400.0, inertia=3000.0, k=(0.01, 0.02, 0.0),
                 c=(0.001, 0.0, 0.0), q0=(b["x"], b["y"], 0.0), f_ext=(1e-4, -2e-4, 0.0),
                 force_model="mem")
    elif kind == "const_vel":
        b.update(mode="const_vel", vx=0.03, vy=-0.02, omega=0.004)
    return b


def run_pair(gpu, spec, body, steps, seed, check_every=1, tol=1e-12, init_random=True):
    from oracle import oracle as orc
    nx, ny = spec["nx"], spec["ny"]
    o = orc.OracleSim(spec, body)
    g = gpu.Sim(spec, body)
    if init_random:
        f0 = W.random_populations(nx, ny, seed=seed, amp=0.05)
        o.set_populations(f0)
        g.set_populations(f0)
    worst = 0.0
    for s in range(0, steps, check_every):
        n = min(check_every, steps - s)
        ro = o.step(n)
        g.step(n)
        rg = g.forces()
        fo, fg = o.get_populations(), g.get_populations()
        e = rel(fg, fo)
        worst = max(worst, e)
        assert e <= tol, (s, e)
        if body is None:
            assert len(rg) == 0  # steps without a body have no record
            continue
        fe = force_err(rg, ro, body["radius"])
        keys = ["fvp", "tvp", "pin", "fh", "th"]
        if body.get("force_model", "vp") in ("mem", "vp+mem"):
            keys += ["fmem", "tmem"]
        else:
            assert not rg["fmem"].any() and not rg["tmem"].any()
        for key in keys:
            # the hydrodynamic load and the exchange sums are differences of larger terms
            # (internal momentum, link pairs): their round-off is held to 10 tol
            ktol = tol * 10 if key in ("fh", "th", "fmem", "tmem") else tol
            if np.abs(ro[key]).max() > 1e-14:
                assert fe[key] <= ktol, (s, key, fe)
        assert fe["q"] <= 1e-12 * max(nx, ny) and fe["v"] <= 1e-12, (s, fe)
    g.close()
    return worst


# (body kind, smoothed indicator): a run without a body has no indicator to smooth
BODY_CASES = [(k, sm) for k in ("none", "fixed", "imposed", "free", "free_mem", "const_vel")
              for sm in (False, True) if not (k == "none" and sm)]


@pytest.mark.parametrize("bcname", list(BCS))
@pytest.mark.parametrize("bodykind,smooth", BODY_CASES)
@pytest.mark.parametrize("tile", [256, 64])
def test_tiny_grids_step_by_step_fp64(gpu, bcname, bodykind, smooth, tile):
    nx, ny = 13, 11
    _flush("tiny %s %s smooth=%s tile %d" % (bcname, bodykind, smooth, tile))
    spec = spec_of(nx, ny, BCS[bcname], u_wall=UWALL, u_conv=0.04,
                   g=(2e-5, -1e-5) if bcname in ("periodic", "pipe") else (0.0, 0.0))
    spec["tile_width"] = tile
    body = None if bodykind == "none" else body_of(bodykind, nx, ny, smooth)
    run_pair(gpu, spec, body, steps=6, seed=1234)


@pytest.mark.parametrize("bcname", list(BCS))
@pytest.mark.parametrize("nx,ny", [(3, 3), (3, 17), (17, 3), (65, 3), (4, 4), (66, 5)])
@pytest.mark.parametrize("tile,rows", [(256, 1), (64, 1), (64, 4), (512, 2)])
def test_smallest_grids_step_by_step_fp64(gpu, bcname, nx, ny, tile, rows):
    """Grids of the smallest allowed sizes (three nodes a side), with rows or columns of
    three and a partly filled wave: every node is an edge node, or every wave holds both
    x edges; a free disc of radius 1.1 near the centre.  4 steps against the oracle."""
    _flush("smallest %s %dx%d tile %d rows %d" % (bcname, nx, ny, tile, rows))
    spec = spec_of(nx, ny, BCS[bcname], u_wall=UWALL, u_conv=0.04,
                   g=(2e-5, -1e-5) if bcname in ("periodic", "pipe") else (0.0, 0.0))
    spec.update(tile_width=tile, rows_per_tile=rows)
    b = W.fixed_disc(2.2, nx / 2.0 - 0.3, ny / 2.0 + 0.2)
    b.update(mode="free", free_mask=7, mass=50.0, inertia=30.0, k=(0.01, 0.01, 0.0),
             q0=(b["x"], b["y"], 0.0), force_model="vp+mem")
    run_pair(gpu, spec, b, steps=4, seed=17)


@pytest.mark.parametrize("tile", [256, 64])
def test_largest_rows_layout_grid_is_periodic_after_a_step(gpu, tile):
    """The largest FP32 grid the row-interleaved layout takes (11200 x 10624, rows of an
    odd multiple of 64 elements: a population buffer of 4.28 GB, 99.7 % of the 4 GiB that
    32-bit byte offsets address), periodic on every side and started from a seeded 64 x 64
    pattern repeated over it: after one step every 64 x 64 block is bitwise the step of
    that pattern on its own periodic 64 x 64 grid, so no node far into the buffer reads or
    writes a wrong address."""
    nx, ny, n = 11200, 10624, 64
    spec = spec_of(nx, ny, BCS["periodic"], storage="fp32", g=(2e-5, -1e-5))
    spec.update(tile_width=tile, rows_per_tile=1, layout="rows")
    assert gpu.load_library().lbm_pop_bytes(nx, ny, gpu.STORAGE["fp32"]) < (1 << 32)
    pat = W.random_populations(n, n, seed=91, amp=0.05)
    small = gpu.Sim(dict(spec, nx=n, ny=n), None)
    small.set_populations(pat)
    small.step(1)
    ref = small.get_populations()
    small.close()
    _flush("largest rows-layout grid %dx%d tile %d" % (nx, ny, tile))
    big = gpu.Sim(spec, None)
    assert big.layout_name() == "rows"
    big.set_populations(np.tile(pat, (1, ny // n, nx // n)))
    big.step(1)
    f = big.get_populations()
    big.close()
    blocks = f.reshape(9, ny // n, n, nx // n, n)
    assert np.array_equal(blocks, np.broadcast_to(ref[:, None, :, None, :], blocks.shape))


@pytest.mark.parametrize("tile", [256, 64])
def test_rows_layout_beyond_4_gib_is_periodic_after_a_step(gpu, tile):
    """A population buffer beyond what 32-bit offsets from its base address: FP64 8192 x
    8192 in the row-interleaved layout (4.87 GB per buffer), periodic on every side and
    started from a seeded 64 x 64 pattern repeated over it.  The step addresses each tile
    from a base at its own rows and the edge and export paths with 64-bit offsets: after
    one step every 64 x 64 block is bitwise the step of that pattern on its own periodic
    64 x 64 grid."""
    nx = ny = 8192
    n = 64
    spec = spec_of(nx, ny, BCS["periodic"], storage="fp64", g=(2e-5, -1e-5))
    spec.update(tile_width=tile, rows_per_tile=1, layout="rows")
    assert gpu.load_library().lbm_pop_bytes(nx, ny, gpu.STORAGE["fp64"]) > (1 << 32)
    pat = W.random_populations(n, n, seed=92, amp=0.05)
    small = gpu.Sim(dict(spec, nx=n, ny=n), None)
    small.set_populations(pat)
    small.step(1)
    ref = small.get_populations()
    small.close()
    _flush("rows layout beyond 4 GiB %dx%d fp64 tile %d" % (nx, ny, tile))
    big = gpu.Sim(spec, None)
    assert big.layout_name() == "rows"
    big.set_populations(np.tile(pat, (1, ny // n, nx // n)))
    big.step(1)
    f = big.get_populations()
    big.close()
    blocks = f.reshape(9, ny // n, n, nx // n, n)
    assert np.array_equal(blocks, np.broadcast_to(ref[:, None, :, None, :], blocks.shape))


def test_zero_steps_and_empty_records(gpu):
    """Stepping zero steps does nothing (no record, the populations unchanged); forces
    with nothing pending returns no record."""
    wl = W.imposed_oscillation(storage="fp64", nx=40, ny=20, D=6.0)
    g = gpu.Sim(wl["spec"], wl["body"])
    f0 = g.get_populations()
    g.step(0)
    assert len(g.forces()) == 0 and g.step_index() == 0
    assert np.array_equal(g.get_populations(), f0)
    g.step(3)
    assert len(g.forces()) == 3 and len(g.forces()) == 0
    g.step(0)
    assert g.step_index() == 3 and len(g.forces()) == 0
    g.close()


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("bcname", ["channel", "wallbox", "mixed", "pipe"])
@pytest.mark.parametrize("bodykind", ["fixed", "free"])
def test_tiny_grids_step_by_step_reduced(gpu, storage, bcname, bodykind):
    """FP32 arithmetic with FP32 / FP16 / BF16 storage: one step at a time from the
    same state, so only one step's rounding separates the two."""
    from oracle import oracle as orc
    nx, ny = 13, 11
    spec = spec_of(nx, ny, BCS[bcname], u_wall=UWALL, u_conv=0.04, storage=storage,
                   g=(2e-5, -1e-5) if bcname == "pipe" else (0.0, 0.0))
    body = body_of(bodykind, nx, ny, False)
    # one step's storage rounding of offsets |g| < 0.032, relative to max f ~ 0.47:
    # fp32 half-ulp 2^-30, fp16 half-ulp of g * 2^10 (< 32) is 2^-17, bf16 half-ulp 2^-14
    tol = {"fp32": 2e-7, "fp16": 5e-5, "bf16": 5e-4}[storage]
    g = gpu.Sim(spec, body)
    o = orc.OracleSim(spec, body)
    f0 = W.random_populations(nx, ny, seed=77, amp=0.05)
    g.set_populations(f0)
    for s in range(4):
        fs = g.get_populations()  # the stored (rounded) state both sides start from
        o.set_populations(fs)
        g.step(1)
        o.step(1)
        e = rel(g.get_populations(), o.get_populations())
        assert e <= tol, (s, e)
    g.close()


@pytest.mark.parametrize("storage", ["fp16", "bf16", "fp32"])
@pytest.mark.parametrize("bcname", ["channel", "periodic", "wallbox"])
@pytest.mark.parametrize("rows,tile", [(1, 256), (2, 256), (1, 512), (2, 512), (4, 256), (4, 512),
                                       (1, 64), (2, 64), (4, 64)])
def test_reduced_storage_several_tiles_step_by_step(gpu, storage, bcname, rows, tile):
    """601 x 40 (three 256-column tiles, two 512-column ones or ten 64-column ones, the last
    ragged and of odd width; 64-column tiles 4, 8 or 16 rows high, the last tile row
    ragged), free body across the first 256-column border: one step at a time from the
    stored state, against the oracle."""
    from oracle import oracle as orc
    nx, ny = 601, 40
    spec = spec_of(nx, ny, BCS[bcname], u_wall=UWALL, u_conv=0.04, storage=storage,
                   g=(2e-5, -1e-5) if bcname == "periodic" else (0.0, 0.0))
    spec["rows_per_tile"] = rows
    spec["tile_width"] = tile
    b = W.fixed_disc(14.0, 255.6, 19.3)
    b.update(mode="free", free_mask=7, mass=300.0, inertia=2000.0, k=(0.01, 0.01, 0.0),
             q0=(255.6, 19.3, 0.0))
    tol = {"fp32": 2e-7, "fp16": 5e-5, "bf16": 5e-4}[storage]
    g = gpu.Sim(spec, b)
    o = orc.OracleSim(spec, b)
    g.set_populations(W.random_populations(nx, ny, seed=21, amp=0.05))
    for s in range(3):
        fs = g.get_populations()
        o.set_populations(fs)
        g.step(1)
        o.step(1)
        e = rel(g.get_populations(), o.get_populations())
        assert e <= tol, (s, e)
    g.close()


@pytest.mark.parametrize("bcname", list(BCS))
@pytest.mark.parametrize("nx,ny,rows,tile,layout", [
    (130, 12, 1, 256, "rows"), (130, 12, 2, 256, "rows"), (600, 9, 2, 256, "rows"),
    (600, 9, 1, 512, "rows"), (1100, 7, 2, 512, "rows"), (130, 12, 4, 256, "rows"),
    (600, 9, 4, 512, "rows"), (1100, 7, 4, 256, "rows"),
    (130, 12, 1, 256, "planes"), (600, 9, 4, 512, "planes"),
    (130, 12, 1, 64, "rows"), (600, 9, 2, 64, "rows"), (131, 13, 1, 64, "planes"),
    (66, 10, 4, 64, "rows")])
def test_x_edge_waves_every_boundary_set_fp64(gpu, bcname, nx, ny, rows, tile, layout):
    """Grids wider than a wave: the waves holding the west or the east node of an
    interior row take the x-edge pull (the east node at 129 sits in a partly filled
    wave), the first and last rows the general one; every boundary set, rows per tile 1,
    2 and 4 (the later rows' pulls come after the earlier rows' stores; 9 and 7 rows
    leave a partly filled last tile row), both population layouts, a body near the
    west edge."""
    _flush("x-edge %s %dx%d rows %d tile %d %s" % (bcname, nx, ny, rows, tile, layout))
    spec = spec_of(nx, ny, BCS[bcname], u_wall=UWALL, u_conv=0.04,
                   g=(2e-5, -1e-5) if bcname in ("periodic", "pipe") else (0.0, 0.0))
    spec["rows_per_tile"] = rows
    spec["tile_width"] = tile
    spec["layout"] = layout
    b = W.fixed_disc(5.0, 4.3, ny / 2.0 - 0.3)
    b.update(vx=0.002, omega=0.001, force_model="vp+mem")
    run_pair(gpu, spec, b, steps=6, seed=7)


@pytest.mark.parametrize("bcname", ["channel", "wallbox", "periodic"])
@pytest.mark.parametrize("tile,xb,rows", [(256, 256.3, 1), (512, 511.7, 1), (256, 256.3, 4),
                                          (512, 511.7, 4), (64, 256.3, 1), (64, 319.7, 2)])
def test_several_tiles_and_ragged_tail_fp64(gpu, bcname, tile, xb, rows):
    """nx = 600 spans three 256-wide tiles or two 512-wide ones, the last one ragged;
    the body straddles a tile border; one or four rows per tile."""
    nx, ny = 600, 24
    _flush("ragged %s tile %d rows %d" % (bcname, tile, rows))
    spec = spec_of(nx, ny, BCS[bcname], u_wall=UWALL, u_conv=0.04)
    spec["tile_width"] = tile
    spec["rows_per_tile"] = rows
    b = W.fixed_disc(14.0, xb, 11.6)
    b.update(mode="free", free_mask=7, mass=300.0, inertia=2000.0, k=(0.01, 0.01, 0.0),
             q0=(xb, 11.6, 0.0))
    run_pair(gpu, spec, b, steps=8, seed=99, check_every=2)


@pytest.mark.parametrize("tile", [256, 512, 64])
@pytest.mark.parametrize("fin", ["tiles", "kernel"])
def test_body_over_more_tiles_than_a_workgroup_has_threads_fp64(gpu, tile, fin):
    """A disc of diameter 260 on a 300x300 grid: with one row per tile its participation
    box holds about 540 (256-column tiles) or 270 (512-column) tiles, more than the 256
    threads that add the slots, so each of them adds several.  Three steps between
    synchronising calls: the derivation inside the step (or in the launch after it) and
    the flush both run."""
    nx, ny = 300, 300
    _flush("large body tile %d finalize %s" % (tile, fin))
    spec = spec_of(nx, ny, BCS["channel"], u_wall=UWALL, u_conv=0.04)
    spec["tile_width"] = tile
    spec["finalize"] = fin
    b = W.fixed_disc(260.0, 150.3, 149.6)
    b.update(mode="free", free_mask=7, mass=5e6, inertia=5e9, k=(0.01, 0.01, 0.0),
             q0=(150.3, 149.6, 0.0))
    run_pair(gpu, spec, b, steps=9, seed=5, check_every=3)


def test_circle_ties_are_classified_like_the_oracle(gpu):
    """Disc of radius 10 centred on a node: the 12 nodes lying exactly on the circle
    (d^2 == R^2) count as inside on both sides (317 nodes in all)."""
    from oracle import oracle as orc
    wl = W.imposed_oscillation()
    spec = dict(wl["spec"], storage="fp64")
    body = dict(wl["body"], mode="fixed")
    o = orc.OracleSim(spec, body)
    assert (o.chi_field()[0] > 0).sum() == 317
    g = gpu.Sim(spec, body)
    ro = o.step(3)
    g.step(3)
    rg = g.forces()
    # chi * rho * u summed over the inside nodes: one misclassified node changes it
    # by ~1/300 of its value
    assert rel(rg["pin"], ro["pin"]) <= 1e-12
    assert rel(rg["fvp"], ro["fvp"]) <= 1e-12
    g.close()


def test_imposed_oscillation_full_run_fp64(gpu):
    """200x80 channel, imposed transverse oscillation, 2000 steps: every step's force
    record and the final fields against the oracle."""
    from oracle import oracle as orc
    wl = W.imposed_oscillation(storage="fp64")
    wl["body"]["force_model"] = "vp+mem"
    _flush("imposed oscillation fp64 2000 steps")
    o = orc.OracleSim(wl["spec"], wl["body"])
    g = gpu.Sim(wl["spec"], wl["body"])
    ro = o.step(wl["steps"])
    g.step(wl["steps"])
    rg = g.forces()
    assert len(rg) == wl["steps"]
    assert (rg["step"] == np.arange(wl["steps"])).all()
    fe = force_err(rg, ro, wl["body"]["radius"])
    _flush("fp64 2000 steps: %s" % fe)
    assert fe["fvp"] <= 1e-12 and fe["tvp"] <= 1e-12 and fe["pin"] <= 1e-12, fe
    assert fe["fh"] <= 1e-11 and fe["fmem"] <= 1e-11 and fe["tmem"] <= 1e-11, fe
    assert fe["q"] <= 1e-12, fe
    rho_o, ux_o, uy_o = o.fields()
    rho_g, ux_g, uy_g = g.fields()
    U0 = wl["U0"]
    assert rel(rho_g, rho_o) <= 1e-12
    assert np.abs(ux_g - ux_o).max() <= 1e-12 * U0
    assert np.abs(uy_g - uy_o).max() <= 1e-12 * U0
    g.close()


def test_imposed_oscillation_fp32_velocity(gpu):
    """FP32 storage and arithmetic against the FP64 oracle: velocity within 1e-5 U0 after
    200 steps and after the full 2000 steps.  Unbiased rounding at FP32's unit roundoff
    stays well inside that bound over the run (independent relative noise of 2^-24 on
    the stored populations departs by about 2.5e-6 U0), while a coherent bias of that
    size does not (about 1.2e-4 U0): the CPU pin test_fp32_rounding_model_of_the_
    imposed_oscillation holds both numbers."""
    from oracle import oracle as orc
    wl = W.imposed_oscillation(storage="fp32")
    _flush("imposed oscillation fp32")
    o = orc.OracleSim(wl["spec"], wl["body"])
    g = gpu.Sim(wl["spec"], wl["body"])
    U0 = wl["U0"]
    for steps, tol in ((200, 1e-5), (1800, 1e-5)):
        ro = o.step(steps)
        g.step(steps)
        rg = g.forces()
        rho_o, ux_o, uy_o = o.fields()
        rho_g, ux_g, uy_g = g.fields()
        eu = max(np.abs(ux_g - ux_o).max(), np.abs(uy_g - uy_o).max()) / U0
        ef = rel(rg["fvp"], ro["fvp"])
        _flush("fp32 after %d more steps: velocity err %.3e U0, force err %.3e" % (steps, eu, ef))
        assert eu <= tol
        assert ef <= 1e-4
    g.close()


def test_same_configuration_is_deterministic(gpu):
    wl = W.imposed_oscillation(storage="fp32", nx=600, ny=90, D=24.0)
    runs = []
    for _ in range(2):
        g = gpu.Sim(wl["spec"], wl["body"])
        g.step(25)
        runs.append((g.get_populations(), g.forces()))
        g.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1]["fvp"], runs[1][1]["fvp"])


def test_timed_steps_match_plain_steps(gpu):
    """lbm_step_timed runs the same eager launches as lbm_step, bracketed by events: the
    state is bitwise the plain run's, the step index advances, and the kernel time is
    positive and within the region's."""
    _flush("timed steps")
    wl = W.imposed_oscillation(storage="fp32", nx=600, ny=90, D=24.0)
    a = gpu.Sim(wl["spec"], wl["body"])
    b = gpu.Sim(wl["spec"], wl["body"])
    a.step(7)
    kms, rms = b.step_timed(7)
    assert b.step_index() == a.step_index() == 7
    assert 0.0 < kms <= rms * 1.001
    assert np.array_equal(a.get_populations(), b.get_populations())
    assert np.array_equal(a.forces()["fvp"], b.forces()["fvp"])
    a.close()
    b.close()


@pytest.mark.parametrize("tile", [256, 512])
def test_flushes_do_not_change_results(gpu, tile):
    """A synchronising call makes the pending body state final with a one-workgroup
    kernel of 256 threads; the step's own tiles (256 or 512 threads) derive the same
    state: a run synchronised after every step is bitwise the run that never is."""
    wl = W.imposed_oscillation(storage="fp32", nx=600, ny=90, D=24.0)
    wl["body"].update(mode="free", free_mask=7, mass=400.0, inertia=4000.0, k=(0.01, 0.01, 0.0))
    spec = dict(wl["spec"], tile_width=tile)
    a = gpu.Sim(spec, wl["body"])
    b = gpu.Sim(spec, wl["body"])
    for _ in range(25):
        a.step(1)
        a.sync()
    b.step(25)
    b.sync()
    assert np.array_equal(a.get_populations(), b.get_populations())
    ra, rb = a.forces(), b.forces()
    for key in ("fvp", "pin", "fh", "q", "v"):
        assert np.array_equal(ra[key], rb[key]), key
    a.close()
    b.close()


def test_graph_replay_is_bitwise_equal_to_eager(gpu):
    wl = W.imposed_oscillation(storage="fp32")
    a = gpu.Sim(wl["spec"], wl["body"])
    b = gpu.Sim(wl["spec"], wl["body"], graph_steps=8)
    a.step(3)
    b.step(3)  # odd start: one eager step, then graphs
    a.step(37)
    b.step(37)
    assert np.array_equal(a.get_populations(), b.get_populations())
    ra, rb = a.forces(), b.forces()
    assert np.array_equal(ra["fvp"], rb["fvp"]) and np.array_equal(ra["q"], rb["q"])
    a.close()
    b.close()


def test_save_and_load_resume_bitwise(gpu):
    wl = W.imposed_oscillation(storage="fp32")
    a = gpu.Sim(wl["spec"], wl["body"])
    a.step(50)
    blob = a.save()
    a.step(30)
    ref = a.get_populations()
    rref = a.forces()[-30:]
    b = gpu.Sim(wl["spec"], wl["body"])
    b.load(blob)
    b.step(30)
    assert np.array_equal(b.get_populations(), ref)
    rb = b.forces()
    assert np.array_equal(rb["fvp"][-30:], rref["fvp"])
    a.close()
    b.close()


@pytest.mark.parametrize("saver,loader", [(256, 512), (64, 256), (512, 64)])
def test_save_and_load_across_tile_widths(gpu, saver, loader):
    """A state saved by a simulation with one tile width resumes in one with another (the
    body's participation box is re-expressed in the loader's tiles): the continuation
    agrees with the saver's own to rounding."""
    wl = W.imposed_oscillation(storage="fp32", nx=600, ny=90, D=24.0)
    wl["body"].update(x=300.4, q0=(300.4, 45.0, 0.0), imp_y0=45.0)
    a = gpu.Sim(dict(wl["spec"], tile_width=saver), wl["body"])
    a.step(40)
    blob = a.save()
    a.step(30)
    b = gpu.Sim(dict(wl["spec"], tile_width=loader), wl["body"])
    b.load(blob)
    b.step(30)
    assert rel(b.get_populations(), a.get_populations()) <= 1e-6
    ra, rb = a.forces()[-30:], b.forces()[-30:]
    assert rel(rb["fvp"], ra["fvp"]) <= 1e-4
    a.close()
    b.close()


def test_torch_memory_and_stream(gpu):
    import torch
    wl = W.imposed_oscillation(storage="fp32")
    a = gpu.Sim(wl["spec"], wl["body"])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = gpu.Sim(wl["spec"], wl["body"], torch_memory=True)
        b.step(40)
    a.step(40)
    assert np.array_equal(a.get_populations(), b.get_populations())
    a.close()
    b.close()


def test_instability_is_reported(gpu):
    spec = spec_of(16, 12, BCS["periodic"], tau=0.7)
    g = gpu.Sim(spec, None)
    f = W.random_populations(16, 12, seed=3)
    f[:, 5, 5] = np.nan
    g.set_populations(f)
    g.step(2)
    with pytest.raises(gpu.LbmError) as e:
        g.sync()
    assert e.value.code == gpu.LBM_ERR_UNSTABLE
    g.close()


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_full_size_free_viv_first_steps(gpu, storage):
    """The 2048x1024 free-VIV grid in the launch configuration of the benchmark:
    20 full steps against the oracle.  The disc is moved off the lattice node it is
    centred on in the workload: a node-centred disc has nodes exactly on its rim,
    whose classification then hinges on round-off-level drift of the free pose."""
    from oracle import oracle as orc
    wl = W.free_viv(storage=storage)
    wl["body"].update(x=512.31, y=511.83, q0=(512.31, 511.83, 0.0))
    _flush("full size free viv %s" % storage)
    o = orc.OracleSim(wl["spec"], wl["body"])
    g = gpu.Sim(wl["spec"], wl["body"])
    ro = o.step(20)
    g.step(20)
    rg = g.forces()
    rho_o, ux_o, uy_o = o.fields()
    rho_g, ux_g, uy_g = g.fields()
    tol = 1e-12 if storage == "fp64" else 1e-5
    U0 = wl["U0"]
    assert max(np.abs(ux_g - ux_o).max(), np.abs(uy_g - uy_o).max()) <= tol * U0
    assert rel(rho_g, rho_o) <= tol
    assert rel(rg["fvp"], ro["fvp"]) <= (1e-12 if storage == "fp64" else 1e-4)
    g.close()


def test_full_size_sedimentation_first_steps(gpu):
    """The 1024x4096 closed box with its free falling disc (FP32 storage), in the launch
    configuration the benchmark picks for it (one row and 512 columns per tile, plain
    stores, body state finalized in the tiles): 10 steps from a seeded near-rest state
    against the FP64 oracle."""
    from oracle import oracle as orc
    wl = W.sedimentation(storage="fp32")
    spec = dict(wl["spec"], rows_per_tile=1, store_mode="plain", tile_width=512,
                finalize="tiles")
    _flush("full size sedimentation fp32")
    f0 = W.random_populations(spec["nx"], spec["ny"], seed=2024, amp=0.02)
    o = orc.OracleSim(wl["spec"], wl["body"])
    g = gpu.Sim(spec, wl["body"], graph_steps=2)
    o.set_populations(f0)
    g.set_populations(f0)
    ro = o.step(10)
    g.step(10)
    rg = g.forces()
    e = rel(g.get_populations(), o.get_populations())
    ef = rel(rg["fvp"], ro["fvp"])
    eq = np.abs(rg["q"] - ro["q"]).max()
    _flush("sedimentation: population err %.2e, force err %.2e, pose err %.2e (moved %.2e)"
           % (e, ef, eq, np.abs(ro["q"][-1] - ro["q"][0]).max()))
    moved = np.abs(ro["q"][-1] - ro["q"][0]).max()
    assert e <= 1e-6 and ef <= 1e-4 and eq <= 1e-4 * moved + 1e-12
    g.close()


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16"])
def test_launch_configurations_agree(gpu, storage):
    """Rows and columns per tile and store instructions change the schedule, not the method: the
    compiler may contract multiply-adds differently in each kernel instantiation, so
    populations agree to rounding (each configuration itself is deterministic)."""
    wl = W.imposed_oscillation(storage=storage, nx=600, ny=90, D=24.0)
    ref = None
    configs = [(r, s, t) for t in (256, 512, 64) for r in (1, 2, 4) for s in ("plain", "nontemporal")]
    for rows, store, tile in configs:
        g = gpu.Sim(dict(wl["spec"], rows_per_tile=rows, store_mode=store, tile_width=tile),
                    wl["body"])
        g.step(30)
        f, r = g.get_populations(), g.forces()
        g.close()
        if ref is None:
            ref = (f, r)
            continue
        tol = {"fp64": 1e-14, "fp32": 1e-6, "fp16": 1e-4}[storage]
        assert rel(f, ref[0]) <= tol, (rows, store, tile)
        assert rel(r["fvp"], ref[1]["fvp"]) <= 100 * tol


def test_autotune_applies_a_configuration(gpu, tmp_path):
    wl = W.imposed_oscillation(storage="fp32", nx=600, ny=90, D=24.0)
    a = gpu.Sim(wl["spec"], wl["body"])
    cache = str(tmp_path / "tune.jsonl")
    rows, nt, us = a.autotune(trial_steps=5, cache=cache)
    assert rows in (1, 2, 4) and nt in (0, 1) and us > 0
    assert a.launch_config()[:2] == (rows, nt) and a.launch_config()[2] in (64, 256, 512)
    b = gpu.Sim(wl["spec"], wl["body"])
    rows2, nt2, us2 = b.autotune(trial_steps=5, cache=cache)  # from the cache
    assert (rows2, nt2, us2) == (rows, nt, -1.0)
    assert b.launch_config() == a.launch_config()
    a.step(20)
    b.step(20)
    assert np.array_equal(a.get_populations(), b.get_populations())
    a.close()
    b.close()


def test_records_exist_only_for_steps_with_a_body(gpu):
    wl = W.imposed_oscillation(storage="fp32", nx=120, ny=48, D=12.0)
    g = gpu.Sim(wl["spec"], wl["body"])
    g.step(3)
    g.clear_body()
    g.step(4)
    r = g.forces()
    assert list(r["step"]) == [0, 1, 2]
    g.step(2)
    assert len(g.forces()) == 0
    g.set_body(wl["body"])
    g.step(2)
    r = g.forces()
    assert list(r["step"]) == [9, 10] and np.isfinite(r["fvp"]).all()
    g.close()


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_momentum_exchange_reduced_storage_one_step(gpu, storage):
    """Momentum-exchange load of one step from a common stored state, FP32 arithmetic:
    every link term (e - u_G) f carries at most the one-step storage error of f
    (the populations test's bound, relative to max f) times |e - u_G| <= 1.5, so the
    force error is bounded by that times the number of link terms."""
    from oracle import oracle as orc
    nx, ny = 40, 36
    spec = spec_of(nx, ny, BCS["periodic"], storage=storage)
    body = W.fixed_disc(17.3, 19.4, 17.8)
    body.update(vx=0.004, vy=-0.003, omega=0.0015, force_model="vp+mem")
    tol = {"fp32": 2e-7, "fp16": 5e-5, "bf16": 5e-4}[storage]
    g = gpu.Sim(spec, body)
    g.set_populations(W.random_populations(nx, ny, seed=91, amp=0.05))
    o = orc.OracleSim(spec, body)
    o.set_populations(g.get_populations())
    cx, cy, _, _, _, _ = orc.lattice()
    R2 = body["radius"] ** 2
    solid = lambda i, j: (i - body["x"]) ** 2 + (j - body["y"]) ** 2 <= R2
    terms = sum(1 for j in range(ny) for i in range(nx) for a in range(1, 9)
                if solid(i, j) != solid(i + cx[a], j + cy[a]))
    g.step(1)
    ro, rg = o.step(1), g.forces()
    fmax = o.get_populations().max()
    bound = terms * 1.5 * tol * fmax
    _flush("%s: %d link terms, fmem err %.3e (bound %.3e)" % (
        storage, terms, np.abs(rg["fmem"] - ro["fmem"]).max(), bound))
    assert np.abs(rg["fmem"] - ro["fmem"]).max() <= bound
    assert abs(rg["tmem"][0] - ro["tmem"][0]) <= bound * (body["radius"] + 1.0)
    g.close()


@pytest.mark.parametrize("bcname", ["channel", "periodic", "wallbox", "mixed"])
@pytest.mark.parametrize("bodykind", ["none", "fixed", "free"])
def test_bgk_collision_step_by_step_fp64(gpu, bcname, bodykind):
    """The BGK operator (Sec. 2.2, Eqs. (11)-(12) with Guo's source): relaxation of every
    population at 1/tau = s_nu, the other rates given but ignored."""
    nx, ny = 13, 11
    spec = spec_of(nx, ny, BCS[bcname], u_wall=UWALL, u_conv=0.04)
    spec.update(collision="bgk", rates=(1.1, 1.25, 1.8, 1.0 / 0.62))
    body = None if bodykind == "none" else body_of(bodykind, nx, ny, False)
    run_pair(gpu, spec, body, steps=6, seed=4321)


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("bcname", ["channel", "wallbox", "periodic"])
@pytest.mark.parametrize("rows,tile", [(1, 256), (4, 512), (2, 64)])
def test_layouts_are_bitwise_equal(gpu, storage, bcname, rows, tile):
    """The row-interleaved and the planar population layouts change addresses only:
    populations and every record field agree bitwise (a free body, a ragged last tile
    column and tile row)."""
    nx, ny = 601, 43
    spec = spec_of(nx, ny, BCS[bcname], u_wall=UWALL, u_conv=0.04, storage=storage,
                   g=(2e-5, -1e-5) if bcname == "periodic" else (0.0, 0.0))
    spec.update(rows_per_tile=rows, tile_width=tile)
    b = W.fixed_disc(14.0, 255.6, 19.3)
    b.update(mode="free", free_mask=7, mass=300.0, inertia=2000.0, k=(0.01, 0.01, 0.0),
             q0=(255.6, 19.3, 0.0), force_model="vp+mem")
    f0 = W.random_populations(nx, ny, seed=31, amp=0.05)
    out = []
    for layout in ("rows", "planes"):
        g = gpu.Sim(dict(spec, layout=layout), b)
        assert g.layout_name() == layout
        g.set_populations(f0)
        g.step(12)
        out.append((g.get_populations(), g.forces()))
        g.close()
    assert np.array_equal(out[0][0], out[1][0])
    for key in ("fvp", "tvp", "pin", "fh", "th", "q", "v", "fmem", "tmem"):
        assert np.array_equal(out[0][1][key], out[1][1][key]), key


@pytest.mark.parametrize("tile", [64, 256])
def test_finalize_modes_are_bitwise_equal_large_body(gpu, tile):
    """A disc of diameter 560 on 600x600 (about 1 400 tiles of 64 columns x 4 rows, or
    1 700 of 256 x 1): the finalize launch sums several slots per thread, several of
    them per round of loads, the tiles one per round; the sums, hence populations and
    records, are bitwise the same."""
    spec = spec_of(600, 600, BCS["channel"], u_wall=UWALL, u_conv=0.04, storage="fp64")
    spec.update(tile_width=tile, rows_per_tile=1)
    b = W.fixed_disc(560.0, 300.3, 299.6)
    b.update(mode="free", free_mask=7, mass=5e7, inertia=5e11, k=(0.01, 0.01, 0.0),
             q0=(300.3, 299.6, 0.0))
    res = []
    for fin in ("tiles", "kernel"):
        g = gpu.Sim(dict(spec, finalize=fin), b)
        g.step(7)
        res.append((g.get_populations(), g.forces()))
        g.close()
    assert np.array_equal(res[0][0], res[1][0])
    for key in ("fvp", "tvp", "pin", "fh", "th", "q", "v", "step"):
        assert np.array_equal(res[0][1][key], res[1][1][key]), key


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("tile", [256, 512, 64])
def test_finalize_modes_are_bitwise_equal(gpu, storage, tile):
    """The body state made final by the next step's tiles or by a one-workgroup launch
    after each step (eager and replayed from graphs): the same fixed-order sums, so
    populations and every record field agree bitwise."""
    wl = W.imposed_oscillation(storage=storage, nx=600, ny=90, D=24.0)
    wl["body"].update(mode="free", free_mask=7, mass=400.0, inertia=4000.0, k=(0.01, 0.01, 0.0),
                      force_model="vp+mem")
    res = []
    for fin, graphs in (("tiles", 0), ("kernel", 0), ("kernel", 8), ("auto", 8)):
        g = gpu.Sim(dict(wl["spec"], tile_width=tile, finalize=fin), wl["body"],
                    graph_steps=graphs)
        assert g.finalize_by_kernel() == (fin == "kernel")  # auto: a small box, in the tiles
        g.step(3)
        g.step(37)
        res.append((g.get_populations(), g.forces()))
        g.close()
    for f, r in res[1:]:
        assert np.array_equal(f, res[0][0])
        for key in ("fvp", "tvp", "pin", "fh", "th", "q", "v", "fmem", "tmem", "step"):
            assert np.array_equal(r[key], res[0][1][key]), key
