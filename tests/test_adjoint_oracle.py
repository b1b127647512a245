"""Pins of the reverse-mode oracle (torch-CPU FP64 mirror of the step).

The mirror's forward step is compared with the C oracle (itself pinned against closed
forms and conservation laws), and its gradients with central finite differences of the
objective computed by the C oracle:
  * pose and rigid velocity: h = 1e-4 (lattice units);
  * indicator field, node by node: h = 1e-4 * eta.  The objective depends on chi through
    chi / eta (Eq. (22)), so a step of 1e-4 in chi is a step of 0.1 in the penalization
    factor, far outside the linear range; scaled to eta, the truncation error is of
    relative order 1e-8.
The bound on |FD - gradient| is 1e-6 of the largest gradient entry.
"""
import numpy as np
import pytest
from conftest import torch_threads

from oracle import adjoint_oracle as ado
from oracle import oracle as orc
from paper_1905_05110_amd import workloads as W

BCS = {
    "channel": ("velocity", "outflow", "symmetry", "symmetry"),
    "wallbox": ("wall",) * 4,
    "periodic": ("periodic",) * 4,
    "symbox": ("symmetry",) * 4,
    "mixed": ("velocity", "outflow", "wall", "velocity"),
    "pipe": ("periodic", "periodic", "wall", "symmetry"),
}
UWALL = [[0.04, 0.01], [0.0, 0.0], [0.0, 0.0], [0.03, -0.005]]


def tiny(bcname, smooth=True, nx=13, ny=11):
    spec = dict(nx=nx, ny=ny, rates=(1.64, 1.54, 1.9, 1.25), eta=1e-3, bc=BCS[bcname],
                u_wall=UWALL, u_conv=0.04, rho0=1.0, u0=(0.04, 0.0),
                g_fluid=(2e-5, -1e-5) if bcname in ("periodic", "pipe") else (0.0, 0.0))
    body = W.fixed_disc(5.0, 5.4, 4.8, smooth_delta=1.0 if smooth else 0.0)
    body.update(vx=0.003, vy=-0.002, omega=0.001)
    return spec, body


def c_objective(spec, body, f0, out0, steps, weights, chi_add=None):
    o = orc.OracleSim(spec, body)
    o.set_populations(f0)
    o.set_outlet(out0)
    if chi_add is not None:
        o.set_chi_perturbation(chi_add)
    r = o.step(steps)
    return float((weights[0] * r["fvp"][:, 0] + weights[1] * r["fvp"][:, 1]).sum())


@pytest.mark.parametrize("bcname", list(BCS))
@pytest.mark.parametrize("smooth", [True, False])
def test_mirror_step_equals_the_c_oracle(bcname, smooth):
    spec, body = tiny(bcname, smooth)
    f0 = W.random_populations(13, 11, seed=5, amp=0.05)
    _, out0 = ado.initial_state(spec)
    o = orc.OracleSim(spec, body)
    o.set_populations(f0)
    o.set_outlet(out0)
    rec = o.step(8)
    f, _, F = ado.Mirror(spec, body).run(f0, out0, 8)
    fo = o.get_populations()
    assert np.abs(f - fo).max() <= 1e-13 * np.abs(fo).max()
    assert np.abs(F - rec["fvp"]).max() <= 1e-12 * np.abs(rec["fvp"]).max()


def fd_check(spec, body, f0, out0, steps, every, weights, nodes, hq=1e-4, hchi=None):
    with torch_threads(1):
        g = ado.Mirror(spec, body).gradient(steps, every, weights, f0, out0)
    J = c_objective(spec, body, f0, out0, steps, weights)
    assert abs(g["J"] - J) <= 1e-12 * abs(J)
    fd = {}
    for name, key in (("x", ("pos", 0)), ("y", ("pos", 1)), ("vx", ("vel", 0)),
                      ("vy", ("vel", 1)), ("omega", ("vel", 2))):
        bp, bm = dict(body), dict(body)
        bp[name] += hq
        bm[name] -= hq
        fd[key] = (c_objective(spec, bp, f0, out0, steps, weights)
                   - c_objective(spec, bm, f0, out0, steps, weights)) / (2 * hq)
    hchi = hchi if hchi is not None else 1e-4 * float(spec["eta"])
    ny, nx = int(spec["ny"]), int(spec["nx"])
    for (i, j) in nodes:
        ca = np.zeros((ny, nx))
        ca[j, i] = hchi
        jp = c_objective(spec, body, f0, out0, steps, weights, ca)
        ca[j, i] = -hchi
        jm = c_objective(spec, body, f0, out0, steps, weights, ca)
        fd[("chi", (j, i))] = (jp - jm) / (2 * hchi)
    scale_q = max(np.abs(g["pos"]).max(), np.abs(g["vel"]).max())
    scale_chi = np.abs(g["chi"]).max()
    for key, v in fd.items():
        got = g[key[0]][key[1]]
        scale = scale_chi if key[0] == "chi" else scale_q
        assert abs(got - v) <= 1e-6 * scale, (key, got, v)
    return g


@pytest.mark.parametrize("bcname", list(BCS))
def test_gradients_match_finite_differences_tiny(bcname):
    spec, body = tiny(bcname)
    f0 = W.random_populations(13, 11, seed=5, amp=0.05)
    _, out0 = ado.initial_state(spec)
    # the body's interface band, its inside, the corners and the east column
    nodes = [(5, 5), (8, 4), (7, 8), (0, 0), (12, 10), (12, 3), (0, 10), (1, 10)]
    fd_check(spec, body, f0, out0, steps=8, every=4, weights=(1.0, 0.5), nodes=nodes)


def test_binary_indicator_has_no_pose_gradient_through_chi():
    spec, body = tiny("channel", smooth=False)
    body.update(vx=0.0, vy=0.0, omega=0.0)
    f0 = W.random_populations(13, 11, seed=6, amp=0.05)
    _, out0 = ado.initial_state(spec)
    g = ado.Mirror(spec, body).gradient(6, 3, (1.0, 0.0), f0, out0)
    assert g["pos"][0] == 0.0 and g["pos"][1] == 0.0
    assert np.abs(g["chi"]).max() > 0


def test_reduced_copy_of_the_drag_workload():
    """128x64 channel, D = 8, Re = 100, tanh indicator with delta = 1: time-averaged
    drag over 400 steps (checkpoints every 50: the interval changes only how much the
    reverse sweep recomputes), from the uniform inflow state."""
    wl = W.adjoint_drag(storage="fp64", nx=128, ny=64, D=8.0)
    spec, body = wl["spec"], wl["body"]
    steps = 400
    wx = 1.0 / (steps * 0.5 * wl["U0"] ** 2 * wl["D"])
    f0, out0 = ado.initial_state(spec)
    R = body["radius"]
    X, Y = body["x"], body["y"]
    nodes = [(int(X + R), int(Y)), (int(X), int(Y - R)), (int(X), int(Y)), (int(X - R - 2), int(Y))]
    g = fd_check(spec, body, f0, out0, steps=steps, every=50, weights=(wx, 0.0), nodes=nodes)
    assert g["J"] > 0.5  # a drag coefficient of order one
