"""The paper's own configurations on the GPU path (Sec. 3.1 and Sec. 3.2.1), checked
against the values the paper prints or the closed form it compares with.

* Imposed transverse oscillation (Sec. 3.1, Table 1): 1230 x 410, D = 41, Re = 100,
  omega* = 1.55, B* = 1/4.  The paper prints a mean drag coefficient of 1.653 from the
  momentum-exchange force.  Reading: the flow past the fixed disc is first run to
  periodic shedding (100 000 steps, t* = 119), then the motion starts; the mean is
  taken over the whole periods up to t* = 64 (the time of the paper's field snapshots).
* Centred settling (Sec. 3.2.1, Eqs. (33)-(35)): H/D = 5, D = 24, tau = 0.8, six density
  ratios; the terminal velocity against the confined Stokes settling velocity.  The
  paper finds agreement for rho_r in {0.98, 0.99, 1.01, 1.02} and a visible gap for
  0.95 and 1.05 (Re = 3.2, beyond the Stokes regime of the closed form).
"""
import math
import sys

import numpy as np
import pytest

from paper_1905_05110_amd import workloads as W
from golden import value as printed

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


def _run(sim, n, chunk=20000):
    out = []
    done = 0
    while done < n:
        k = min(chunk, n - done)
        sim.step(k)
        out.append(sim.forces())
        done += k
    return np.concatenate(out)


def test_paper_imposed_oscillation_mean_drag(gpu):
    wl = W.paper_imposed_oscillation(storage="fp64")
    U0, D, T = wl["U0"], wl["D"], wl["period"]
    s = 0.5 * U0 ** 2 * D
    _flush("paper imposed oscillation 1230x410 fp64: fixed-cylinder run")
    g = gpu.Sim(wl["spec"], wl["fixed"])
    g.set_graph_steps(64)
    pre = _run(g, 100000)
    cl = pre["fmem"][50000:, 1] / s
    zc = np.where(np.diff(np.sign(cl - cl.mean())) > 0)[0]
    st = D / (np.diff(zc).mean() * U0)
    _flush("fixed cylinder: CD %.4f, St %.4f" % (pre["fmem"][-10000:, 0].mean() / s, st))
    assert 0.15 <= st <= 0.19  # periodic shedding at Re = 100 before the motion starts
    g.set_body(wl["body"])
    k = int(64.0 * D / U0 // T)  # whole periods up to t* = 64
    n = int(round(k * T))
    r = _run(g, n)
    g.close()
    cd_mem = r["fmem"][:, 0].mean() / s
    cd_h = r["fh"][:, 0].mean() / s
    _flush("moving, %d periods: mean CD %.4f (momentum exchange), %.4f (penalization); "
           "paper %.3f" % (k, cd_mem, cd_h, printed("mean_cd_imposed_oscillation")))
    y = r["q"][:, 1]
    assert abs(y.max() - wl["fixed"]["y"]) < 1e-9 and abs(y.min() - (wl["fixed"]["y"] - 2 * wl["body"]["imp_amp"])) < 1e-3
    assert abs(cd_mem / printed("mean_cd_imposed_oscillation") - 1.0) <= 0.02
    assert abs(cd_h / cd_mem - 1.0) <= 0.01


def test_paper_centred_settling_velocities(gpu):
    wls = [W.paper_sedimentation_centered(r, storage="fp64") for r in W.PAPER_DENSITY_RATIOS]
    _flush("paper centred settling: 6 runs of 1200x120 in one batch, 30000 steps")
    b = gpu.Batch([(w["spec"], w["body"]) for w in wls], storage="fp64", graph_steps=64)
    recs = [[] for _ in wls]
    for _ in range(6):
        b.step(5000)
        for i, sm in enumerate(b.sims):
            recs[i].append(sm.forces())
    b.close()
    ratio = {}
    for w, rl in zip(wls, recs):
        r = np.concatenate(rl)
        rr = W.PAPER_DENSITY_RATIOS[wls.index(w)]
        ratio[rr] = r["v"][-5000:, 0].mean() / w["vs"]
        _flush("rho_r %.2f: terminal / closed form %.4f" % (rr, ratio[rr]))
        # the centred disc stays on the mirror line and does not turn
        assert np.abs(r["q"][:, 1] - w["body"]["y"]).max() <= 1e-12
        assert np.abs(r["v"][:, 2]).max() <= 1e-12
    for rr in (0.98, 0.99, 1.01, 1.02):
        assert 0.95 <= ratio[rr] <= 1.02, (rr, ratio[rr])
    for rr in (0.95, 1.05):
        assert 0.85 <= ratio[rr] < min(ratio[0.98], ratio[1.02])
    # Stokes regime: a lighter and a heavier disc of the same |1 - rho_r| mirror each other
    for a, c in ((0.99, 1.01), (0.98, 1.02), (0.95, 1.05)):
        assert abs(ratio[a] / ratio[c] - 1.0) <= 2e-3


def _response(y, y0, D, U0):
    """Largest |y - y0| / D and the dominant angular frequency omega* = omega D / U0
    of the displacement over the second half of a run (FFT peak of the Hann-windowed
    signal, refined by a parabola through the peak and its neighbours)."""
    a = (y - y0) / D
    tail = a[len(a) // 2:]
    x = (tail - tail.mean()) * np.hanning(len(tail))
    F = np.abs(np.fft.rfft(x))
    k = int(np.argmax(F[1:])) + 1
    al, be, ga = F[k - 1], F[k], F[k + 1]
    f = (k + 0.5 * (al - ga) / (al - 2 * be + ga)) / len(tail)
    return np.abs(tail).max(), 2 * np.pi * f * D / U0


def test_paper_viv_effective_stiffness(gpu):
    """Sec. 3.3: the paper prints k*_eff = k* - m* omega*^2 for k* = 9, 19, 28 (0.058,
    3.20, 16.37) and finds lock-in displacements above half a diameter.  m* is not
    stated.  The k* = 28 case (response at the wake's shedding frequency) is the
    calibration point: m* = 9 was chosen so that it reproduces 16.37, so its bound below
    only confirms that calibration and is not a check of the method.  The checks are
    the other two cases, predicted with that m*: the lock-in case k* = 9, and k* = 19 on
    the edge of lock-in, where k*_eff moves by 1 for a 3 % change of the response
    frequency (bound 1.5 there)."""
    wls = [W.paper_viv(k, storage="fp32") for k in (9.0, 19.0, 28.0)]
    _flush("paper VIV 1230x410, k* = 9, 19, 28 in one batch, 240000 steps")
    b = gpu.Batch([(w["spec"], w["body"]) for w in wls], storage="fp32", graph_steps=64)
    ys = [[] for _ in wls]
    for _ in range(12):
        b.step(20000)
        for i, sm in enumerate(b.sims):
            ys[i].append(sm.forces()["q"][:, 1].copy())
    b.close()
    res = {}
    for w, yl in zip(wls, ys):
        amp, om = _response(np.concatenate(yl), w["body"]["y"], w["D"], w["U0"])
        keff = w["k_star"] - w["m_star"] * om ** 2
        res[w["k_star"]] = (amp, keff)
        _flush("k* %g: amplitude %.3f D, omega* %.4f, k*_eff %.3f" % (w["k_star"], amp, om, keff))
    assert abs(res[9.0][1] - printed("keff_vortex_induced_k9")) <= 0.15
    assert abs(res[19.0][1] - printed("keff_vortex_induced_k19")) <= 1.5
    # the calibration point of m* (not a check)
    assert abs(res[28.0][1] - printed("keff_vortex_induced_k28")) <= 0.3
    assert max(res[9.0][0], res[19.0][0]) > 0.5  # lock-in: more than half a diameter
    assert res[28.0][0] < 0.1  # far from lock-in the displacement stays small


def test_paper_offcentre_settling(gpu):
    """Sec. 3.2.2: a disc released 0.75 D from a wall moves towards the centre line while
    turning in the positive sense, oscillates briefly about it, and settles there at a
    final particle Reynolds number of 8.33 (paper).  Channel along x, gravity along +x
    (a quarter turn of the paper's axes, which keeps the sense of rotation)."""
    w = W.paper_sedimentation_offcentre(storage="fp32")
    _flush("paper off-centre settling 1550x125, 100000 steps")
    g = gpu.Sim(w["spec"], w["body"])
    g.set_graph_steps(64)
    r = _run(g, 100000)
    g.close()
    yc = (w["spec"]["ny"] - 1) / 2.0
    D, nu = w["D"], w["nu"]
    y = r["q"][:, 1] - yc
    re = r["v"][-5000:, 0].mean() * D / nu
    re_paper = printed("reynolds_offcentre_settling")
    _flush("final Re %.3f (paper %.2f); max overshoot %.3f D; final offset %.4f D; first "
           "rotation %.2e" % (re, re_paper, y.max() / D, y[-1] / D, r["v"][2000, 2]))
    assert abs(re / re_paper - 1.0) <= 0.03
    assert y[0] < -D  # released near the wall ...
    assert r["v"][2000, 1] > 0.0 and r["v"][2000, 2] > 0.0  # ... moving off it, turning positively
    assert y.max() > 0.05 * D  # crosses the centre line once (brief oscillation)
    assert abs(y[-1]) <= 0.01 * D and abs(r["v"][-1, 2]) <= 1e-6  # settled on the centre line
