"""Adjoint (reverse-mode) path on the GPU, through the C ABI, against the reverse-mode
oracle (torch-CPU FP64 mirror of the step differentiated by autograd) and against
central finite differences of the C oracle's objective.

Bounds (FP64): J to 1e-12 relative; dJ/dchi to 1e-10 of its largest entry; dJ/d(X, Y)
and dJ/d(V, Omega) to 1e-10 of the largest of them.  Finite differences: 1e-6 (their
truncation error, measured 1e-9 to 1e-10).
"""
import sys

import numpy as np
import pytest
from conftest import torch_threads

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


BCS = {
    "channel": ("velocity", "outflow", "symmetry", "symmetry"),
    "wallbox": ("wall",) * 4,
    "periodic": ("periodic",) * 4,
    "symbox": ("symmetry",) * 4,
    "mixed": ("velocity", "outflow", "wall", "velocity"),
    "pipe": ("periodic", "periodic", "wall", "symmetry"),
}
UWALL = [[0.04, 0.01], [0.0, 0.0], [0.0, 0.0], [0.03, -0.005]]


def tiny(bcname, smooth=True, storage="fp64"):
    spec = dict(nx=13, ny=11, rates=(1.64, 1.54, 1.9, 1.25), eta=1e-3, bc=BCS[bcname],
                u_wall=UWALL, u_conv=0.04, rho0=1.0, u0=(0.04, 0.0), storage=storage,
                g_fluid=(2e-5, -1e-5) if bcname in ("periodic", "pipe") else (0.0, 0.0))
    body = W.fixed_disc(5.0, 5.4, 4.8, smooth_delta=1.0 if smooth else 0.0)
    body.update(vx=0.003, vy=-0.002, omega=0.001)
    return spec, body


def compare(g, ref, tol=1e-10):
    assert abs(g["J"] - ref["J"]) <= 1e-12 * abs(ref["J"]), (g["J"], ref["J"])
    ec = np.abs(g["chi"] - ref["chi"]).max() / np.abs(ref["chi"]).max()
    sq = max(np.abs(ref["pos"]).max(), np.abs(ref["vel"]).max())
    ep = np.abs(g["pos"] - ref["pos"]).max() / sq
    ev = np.abs(g["vel"] - ref["vel"]).max() / sq
    assert ec <= tol and ep <= tol and ev <= tol, (ec, ep, ev)
    return ec, ep, ev


def run_gpu(gpu, spec, body, steps, every, weights, f0=None, out0=None):
    adj = gpu.Adjoint(spec, body, steps, every, weights)
    if f0 is not None:
        adj.set_initial(f0, out0)
    J = adj.forward()
    adj.backward()
    g = adj.gradient()
    g["J"] = J
    return adj, g


@pytest.mark.parametrize("bcname", list(BCS))
@pytest.mark.parametrize("smooth", [True, False])
@pytest.mark.parametrize("tile", [256, 64])
def test_tiny_grids_against_the_reverse_mode_oracle(gpu, bcname, smooth, tile):
    """The forward and recomputing steps in 256- or 64-column tiles."""
    from oracle import adjoint_oracle as ado
    _flush("adjoint tiny %s smooth=%s tile %d" % (bcname, smooth, tile))
    spec, body = tiny(bcname, smooth)
    spec = dict(spec, tile_width=tile)
    f0 = W.random_populations(13, 11, seed=5, amp=0.05)
    _, out0 = ado.initial_state(spec)
    out0 = out0 * (1.0 + 0.01 * np.arange(11)[None, :] / 11.0)  # a non-uniform memory
    ref = ado.Mirror(spec, body).gradient(8, 4, (1.0, 0.5), f0, out0)
    adj, g = run_gpu(gpu, spec, body, 8, 4, (1.0, 0.5), f0, out0)
    compare(g, ref)
    adj.close()


def test_reduced_drag_copy_against_the_oracle(gpu):
    """128 x 64, D = 8, Re = 100, tanh indicator (delta = 1), drag weights, 400 steps
    with a checkpoint every 100, from the uniform inflow state."""
    from oracle import adjoint_oracle as ado
    wl = W.adjoint_drag(storage="fp64", nx=128, ny=64, D=8.0)
    steps = 400
    w = (1.0 / (steps * 0.5 * wl["U0"] ** 2 * wl["D"]), 0.0)
    _flush("adjoint 128x64 vs oracle")
    with torch_threads(1):
        ref = ado.Mirror(wl["spec"], wl["body"]).gradient(steps, 100, w)
    adj, g = run_gpu(gpu, wl["spec"], wl["body"], steps, 100, w)
    _flush("errors %s" % (compare(g, ref),))
    adj.close()


def test_reduced_drag_copy_finite_differences_full_length(gpu):
    """The 128 x 64 copy over the full 4000 steps (checkpoint every 100): dJ/d(X, Y)
    and dJ/dchi at two interface nodes against central differences of the C oracle
    (h = 1e-4 for the centre, 1e-4 eta for chi)."""
    from oracle import oracle as orc
    wl = W.adjoint_drag(storage="fp64", nx=128, ny=64, D=8.0)
    spec, body = wl["spec"], wl["body"]
    steps = wl["steps"]
    w = (1.0 / (steps * 0.5 * wl["U0"] ** 2 * wl["D"]), 0.0)
    adj, g = run_gpu(gpu, spec, body, steps, wl["checkpoint_every"], w)
    orc.set_threads(16)

    def J(bd, chi_add=None):
        o = orc.OracleSim(spec, bd)
        if chi_add is not None:
            o.set_chi_perturbation(chi_add)
        r = o.step(steps)
        return float((w[0] * r["fvp"][:, 0]).sum())

    J0 = J(body)
    _flush("J gpu %.15g oracle %.15g" % (g["J"], J0))
    assert abs(g["J"] - J0) <= 1e-11 * abs(J0)
    h = 1e-4
    fd = []
    for k in ("x", "y"):
        bp, bm = dict(body), dict(body)
        bp[k] += h
        bm[k] -= h
        fd.append((J(bp) - J(bm)) / (2 * h))
    scale = np.abs(g["pos"]).max()
    _flush("dJ/dX gpu %s fd %s" % (g["pos"], fd))
    assert np.abs(np.array(fd) - g["pos"]).max() <= 1e-6 * scale
    hc = 1e-4 * spec["eta"]
    R = body["radius"]
    for (i, j) in [(int(body["x"] + R), int(body["y"])), (int(body["x"]), int(body["y"] - R))]:
        ca = np.zeros((spec["ny"], spec["nx"]))
        ca[j, i] = hc
        jp = J(body, ca)
        ca[j, i] = -hc
        jm = J(body, ca)
        fdc = (jp - jm) / (2 * hc)
        assert abs(fdc - g["chi"][j, i]) <= 1e-6 * np.abs(g["chi"]).max(), (i, j, fdc, g["chi"][j, i])
    adj.close()


def test_adjoint_refuses_direction_arrays_of_4_gib(gpu):
    """The reverse step addresses a direction's populations with 32-bit offsets from its
    base: an FP64 8192 x 8192 grid (a direction spans 4.87 GB in the row-interleaved
    layout, which the forward step itself runs) is refused with LBM_ERR_ARG."""
    wl = W.adjoint_drag(storage="fp64", nx=8192, ny=8192, D=32.0)
    with pytest.raises(gpu.LbmError) as e:
        gpu.Adjoint(wl["spec"], wl["body"], 4, 2, (1.0, 0.0))
    assert e.value.code == gpu.LBM_ERR_ARG and "4 GiB" in str(e.value)


def test_repeated_backward_is_deterministic(gpu):
    spec, body = tiny("channel")
    adj = gpu.Adjoint(spec, body, 8, 4, (1.0, 0.0))
    adj.forward()
    adj.backward()
    g1 = adj.gradient()
    adj.backward()
    g2 = adj.gradient()
    assert np.array_equal(g1["chi"], g2["chi"]) and np.array_equal(g1["pos"], g2["pos"])
    adj.close()


def test_autograd_function(gpu):
    import torch
    wl = W.adjoint_drag(storage="fp64", nx=128, ny=64, D=8.0)
    steps = 200
    w = (1.0 / (steps * 0.5 * wl["U0"] ** 2 * wl["D"]), 0.0)
    adj = gpu.Adjoint(wl["spec"], wl["body"], steps, 100, w)
    Obj = gpu.body_position_objective()
    c = torch.tensor([wl["body"]["x"] + 0.3, wl["body"]["y"] - 0.2], dtype=torch.float64,
                     requires_grad=True)
    J = Obj.apply(c, adj, wl["body"])
    J.backward()
    ref = adj.gradient(chi=False)["pos"]
    assert np.array_equal(c.grad.numpy(), ref)
    adj.close()


def chi_window_field(spec, body, amp, seed):
    """A random additive indicator over the nodes within the disc's reach plus one of its
    centre (the window the library accepts), zero elsewhere."""
    nx, ny = spec["nx"], spec["ny"]
    reach = body["radius"] + (20.0 * body["smooth_delta"] if body["smooth_delta"] > 0 else 0.0)
    i0 = max(0, int(np.floor(body["x"] - reach)) - 1)
    i1 = min(nx - 1, int(np.ceil(body["x"] + reach)) + 1)
    j0 = max(0, int(np.floor(body["y"] - reach)) - 1)
    j1 = min(ny - 1, int(np.ceil(body["y"] + reach)) + 1)
    f = np.zeros((ny, nx))
    rng = np.random.default_rng(seed)
    f[j0:j1 + 1, i0:i1 + 1] = amp * rng.uniform(-1.0, 1.0, (j1 - j0 + 1, i1 - i0 + 1))
    return f, (i0, i1, j0, j1)


@pytest.mark.parametrize("bcname", ["channel", "mixed", "pipe"])
def test_additive_indicator_forward_matches_the_oracle(gpu, bcname):
    """The forward run with an additive indicator field (the oracle's chi_add) against
    the C oracle: every record to 1e-12, J to 1e-12; a field non-zero outside the box is
    refused."""
    from oracle import oracle as orc
    spec, body = tiny(bcname, smooth=True)
    field, (i0, i1, j0, j1) = chi_window_field(spec, body, 1e-3, 3)
    adj = gpu.Adjoint(spec, body, 8, 4, (1.0, 0.5))
    adj.set_chi_add(field)
    J = adj.forward()
    rg = adj.forces()
    o = orc.OracleSim(spec, body)
    o.set_chi_perturbation(field)
    ro = o.step(8)
    Jo = float((ro["fvp"][:, 0] + 0.5 * ro["fvp"][:, 1]).sum())
    assert abs(J - Jo) <= 1e-12 * abs(Jo), (J, Jo)
    for key in ("fvp", "tvp", "pin"):
        assert np.abs(rg[key] - ro[key]).max() <= 1e-12 * max(np.abs(ro[key]).max(), 1e-300), key
    if i1 < spec["nx"] - 1:
        bad = field.copy()
        bad[j0, i1 + 1] = 1e-3
        with pytest.raises(gpu.LbmError) as e:
            adj.set_chi_add(bad)
        assert e.value.code == gpu.LBM_ERR_ARG
    adj.close()


def test_autograd_over_the_additive_indicator(gpu):
    """The torch.autograd.Function over (centre, additive indicator): its gradients are
    the adjoint's dJ/d(X, Y) and dJ/dchi; dJ/dchi at interface nodes against central
    differences of the GPU objective through the same input (h = 1e-4 eta) and of the C
    oracle; two applications before one backward give each its own gradient."""
    import torch
    from oracle import oracle as orc
    wl = W.adjoint_drag(storage="fp64", nx=128, ny=64, D=8.0)
    spec, body = wl["spec"], wl["body"]
    steps = 200
    w = (1.0 / (steps * 0.5 * wl["U0"] ** 2 * wl["D"]), 0.0)
    adj = gpu.Adjoint(spec, body, steps, 100, w)
    F = gpu.adjoint_objective()
    field, _ = chi_window_field(spec, body, 1e-4, 8)
    c = torch.tensor([body["x"], body["y"]], dtype=torch.float64, requires_grad=True)
    chi = torch.tensor(field, requires_grad=True)
    J = F.apply(c, chi, adj, body)
    J.backward()
    adj.set_body(body)
    adj.set_chi_add(field)
    J_ref = adj.forward()
    adj.backward()
    ref = adj.gradient()
    assert float(J) == J_ref
    assert np.array_equal(c.grad.numpy(), ref["pos"])
    assert np.array_equal(chi.grad.numpy(), ref["chi"])
    # central differences through the same input, at two interface nodes
    hc = 1e-4 * spec["eta"]
    R = body["radius"]
    orc.set_threads(16)
    for (i, j) in [(int(body["x"] + R), int(body["y"])), (int(body["x"]), int(body["y"] - R))]:
        Js, Jo = [], []
        for sgn in (1.0, -1.0):
            f = field.copy()
            f[j, i] += sgn * hc
            adj.set_body(body)
            adj.set_chi_add(f)
            Js.append(adj.forward())
            o = orc.OracleSim(spec, body)
            o.set_chi_perturbation(f)
            r = o.step(steps)
            Jo.append(float((w[0] * r["fvp"][:, 0]).sum()))
        fd, fdo = (Js[0] - Js[1]) / (2 * hc), (Jo[0] - Jo[1]) / (2 * hc)
        _flush("dJ/dchi(%d, %d): autograd %.12g, fd gpu %.12g, fd oracle %.12g"
               % (i, j, chi.grad[j, i], fd, fdo))
        scale = np.abs(ref["chi"]).max()
        assert abs(fd - float(chi.grad[j, i])) <= 1e-6 * scale
        assert abs(fdo - float(chi.grad[j, i])) <= 1e-6 * scale
    # two applications, then the first one's backward: its own gradient, not the second's
    c1 = torch.tensor([body["x"], body["y"]], dtype=torch.float64, requires_grad=True)
    c2 = torch.tensor([body["x"] + 0.4, body["y"] - 0.3], dtype=torch.float64,
                      requires_grad=True)
    J1 = F.apply(c1, None, adj, body)
    J2 = F.apply(c2, None, adj, body)
    J1.backward()
    J2.backward()
    adj.set_body(body)
    adj.forward()
    adj.backward()
    g1 = adj.gradient(chi=False)["pos"]
    adj.set_body(dict(body, x=body["x"] + 0.4, y=body["y"] - 0.3))
    adj.forward()
    adj.backward()
    g2 = adj.gradient(chi=False)["pos"]
    assert np.array_equal(c1.grad.numpy(), g1) and np.array_equal(c2.grad.numpy(), g2)
    assert not np.array_equal(g1, g2)
    adj.close()


def test_full_size_fp32_against_fp64(gpu):
    """The 1024 x 512 drag workload (D = 32, Re = 100, tanh indicator, 4000 steps, a
    checkpoint every 100): FP32 storage and arithmetic against FP64, and the FP64
    dJ/dX against central differences of the FP64 forward run (h = 1e-4).  dJ/dX is
    small here (2.5e-5 against J = 2.9: the disc sits in a long channel), so the
    rounding of the two objectives enters the FD bound."""
    wl = W.adjoint_drag(storage="fp64")
    steps = wl["steps"]
    w = (1.0 / (steps * 0.5 * wl["U0"] ** 2 * wl["D"]), 0.0)
    _flush("adjoint 1024x512 fp64")
    a64, g64 = run_gpu(gpu, wl["spec"], wl["body"], steps, wl["checkpoint_every"], w)
    _flush("adjoint 1024x512 fp32")
    s32 = dict(wl["spec"], storage="fp32")
    a32, g32 = run_gpu(gpu, s32, wl["body"], steps, wl["checkpoint_every"], w)
    eJ = abs(g32["J"] - g64["J"]) / abs(g64["J"])
    ep = np.abs(g32["pos"] - g64["pos"]).max() / np.abs(g64["pos"]).max()
    ec = np.abs(g32["chi"] - g64["chi"]).max() / np.abs(g64["chi"]).max()
    _flush("fp32 vs fp64: J %.3e pos %.3e chi %.3e; J %.6f dJ/dX %s" % (eJ, ep, ec, g64["J"],
                                                                         g64["pos"]))
    # FP32 bounds: J and dJ/dchi at about ten times their measured errors (1.1e-6 each).
    # dJ/dX = sum_i dJ/dchi_i d(chi_i)/dX (reading 22 of the design notes) cancels between
    # the front and the back of the disc: 2.5e-5 against 0.09 for the sum of the terms'
    # magnitudes, so the field's small error is a large part of it (measured 2.9e-3 of
    # |dJ/dX|).  It is held to what the FP32 field's own error carries into that sum,
    # sum_i |dJ/dchi_i(FP32) - dJ/dchi_i(FP64)| |d(chi_i)/dX|, plus FP64 rounding.
    assert eJ <= 1e-5 and ec <= 1e-5
    X, Y = wl["body"]["x"], wl["body"]["y"]
    R, delta = wl["body"]["radius"], wl["body"]["smooth_delta"]
    jj, ii = np.mgrid[0:wl["spec"]["ny"], 0:wl["spec"]["nx"]]
    d = np.hypot(ii - X, jj - Y)
    z = (d - R) / delta
    chi = np.where(z > 20, 0.0, np.where(z < -20, 1.0, 1.0 / (1.0 + np.exp(2.0 * np.clip(z, -20, 20)))))
    dchi = np.where(np.abs(z) > 20, 0.0, 2.0 * chi * (1.0 - chi) / (delta * np.maximum(d, 1e-300)))
    dfield = np.abs(g32["chi"] - g64["chi"])
    prop = np.array([(dfield * dchi * np.abs(ii - X)).sum(), (dfield * dchi * np.abs(jj - Y)).sum()])
    prop += 1e-12 * np.abs(g64["pos"]).max()
    _flush("pose gradient error %s, propagated bound %s (cancellation: |dJ/dX| %s against "
           "sum |dJ/dchi d(chi)/dX| %s)" % (np.abs(g32["pos"] - g64["pos"]), prop,
                                           np.abs(g64["pos"]),
                                           [(np.abs(g64["chi"]) * dchi * np.abs(ii - X)).sum(),
                                            (np.abs(g64["chi"]) * dchi * np.abs(jj - Y)).sum()]))
    assert (np.abs(g32["pos"] - g64["pos"]) <= prop).all()
    h = 1e-4
    fd = []
    for k in ("x", "y"):
        Js = []
        for sgn in (1, -1):
            b = dict(wl["body"])
            b[k] += sgn * h
            a64.set_body(b)
            Js.append(a64.forward())
        fd.append((Js[0] - Js[1]) / (2 * h))
    _flush("fd %s" % (fd,))
    # truncation (relative 1e-6) plus the rounding of the two objectives divided by 2h:
    # J sums ~4000 x 10^5 node forces, whose rounding is taken as 1e-12 |J|
    bound = 1e-6 * np.abs(g64["pos"]) + 1e-12 * abs(g64["J"]) / (2 * h)
    assert (np.abs(np.array(fd) - g64["pos"]) <= bound).all(), (fd, g64["pos"], bound)
    a64.close()
    a32.close()


def test_eager_and_graph_runs_agree(gpu):
    spec, body = tiny("mixed")
    f0 = W.random_populations(13, 11, seed=9, amp=0.05)
    out = []
    for graphs in (True, False):
        adj = gpu.Adjoint(spec, body, 8, 4, (1.0, 0.3), graphs=graphs)
        adj.set_initial(f0)
        J = adj.forward()
        adj.backward()
        out.append((J, adj.gradient()))
        adj.close()
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1]["chi"], out[1][1]["chi"])
    assert np.array_equal(out[0][1]["pos"], out[1][1]["pos"])
