"""ctypes front end of the FP64 CPU oracle (``vplbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and the
benchmark's CPU-baseline leg; never by the GPU product path.

A simulation is described by two plain dicts shared with the GPU binding (their
keys only; no code is shared):

* ``spec``: ``nx, ny, rates=(s_e, s_eps, s_q, s_nu), eta, bc=(west, east, south,
  north), u_wall (4x2), u_conv, g_fluid (2), rho0, u0 (2)``, and ``collision``
  (``"mrt"``, or ``"bgk"``: every rate 1/tau = s_nu, which the BGK pin equates with
  the single-relaxation-time collision and Guo's source);
* ``body``: ``radius, x, y, theta, vx, vy, omega, mode, free_mask, mass, inertia,
  k, c, q0, f_ext (3 each), imp_amp, imp_freq, imp_y0, imp_phase, smooth_delta,
  internal_mass_correction, force_model`` (``"vp"``, ``"mem"`` or ``"vp+mem"``: the load
  that drives a free body is the momentum exchange for ``"mem"`` only).

The relaxation matrix follows the paper's choice for the conserved moments
(Sec. 3, Eq. (28): s_0 = s_3 = s_5 = 1/tau = s_nu); the other rates come from the
spec (Sec. 2.2, Eq. (16)).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

BC = {"periodic": 0, "wall": 1, "velocity": 2, "symmetry": 3, "outflow": 4}
MODE = {"fixed": 0, "imposed_sin": 1, "free": 2, "const_vel": 3}
FORCE = {"vp": 0, "mem": 1, "vp+mem": 2}  # the oracle evaluates both loads always


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int),
        ("s", C.c_double * 9),
        ("eta", C.c_double),
        ("bc", C.c_int * 4),
        ("u_wall", (C.c_double * 2) * 4),
        ("u_conv", C.c_double),
        ("g_fluid", C.c_double * 2),
        ("has_body", C.c_int),
        ("radius", C.c_double),
        ("smooth_delta", C.c_double),
        ("mode", C.c_int),
        ("free_mask", C.c_uint),
        ("mass", C.c_double), ("inertia", C.c_double),
        ("k", C.c_double * 3), ("c", C.c_double * 3), ("q0", C.c_double * 3),
        ("f_ext", C.c_double * 3),
        ("imp_amp", C.c_double), ("imp_freq", C.c_double), ("imp_y0", C.c_double),
        ("imp_phase", C.c_double),
        ("internal_mass_correction", C.c_int),
        ("force_model", C.c_int),
        ("chi_add", C.c_void_p),
    ]


class Body(C.Structure):
    _fields_ = [("q", C.c_double * 3), ("v", C.c_double * 3), ("t_body", C.c_int64),
                ("pin_prev", C.c_double * 3), ("pin_valid", C.c_int)]


RECORD_DTYPE = np.dtype([("step", "<i8"), ("fvp", "<f8", (2,)), ("tvp", "<f8"),
                         ("pin", "<f8", (3,)), ("fh", "<f8", (2,)), ("th", "<f8"),
                         ("q", "<f8", (3,)), ("v", "<f8", (3,)),
                         ("fmem", "<f8", (2,)), ("tmem", "<f8")])

_LIB = None
_DP = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    """Load (building first if missing or stale) the oracle shared library."""
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        assert L.orc_sizeof_params() == C.sizeof(Params)
        assert L.orc_sizeof_body() == C.sizeof(Body)
        assert L.orc_sizeof_record() == RECORD_DTYPE.itemsize
        P, B = C.POINTER(Params), C.POINTER(Body)
        L.orc_lattice.argtypes = [C.POINTER(C.c_int)] * 3 + [_DP] * 3
        L.orc_feq.argtypes = [C.c_double] * 3 + [_DP]
        L.orc_guo.argtypes = [C.c_double] * 4 + [_DP]
        L.orc_chi.argtypes = [P, B, C.c_int, C.c_int] + [C.POINTER(C.c_double)] * 3
        L.orc_node.argtypes = [P, _DP, C.c_double, C.c_double, C.c_double, _DP] + \
            [C.POINTER(C.c_double)] * 3 + [_DP, _DP]
        L.orc_rk4.argtypes = [C.c_double] * 5 + [C.POINTER(C.c_double)] * 2
        L.orc_body_init.argtypes = [P, B, _DP, _DP]
        L.orc_body_advance.argtypes = [P, B, _DP]
        L.orc_step.argtypes = [P, _DP, _DP, _DP, B, C.c_void_p, C.c_int64]
        L.orc_step.restype = C.c_int
        L.orc_run.argtypes = [P, _DP, _DP, B, C.c_void_p, C.c_int64, C.c_int64]
        L.orc_run.restype = C.c_int
        L.orc_init.argtypes = [P, _DP, _DP, C.c_double, C.c_double, C.c_double]
        L.orc_fields.argtypes = [P, _DP, _DP, B, _DP, _DP, _DP]
        L.orc_pull_node.argtypes = [P, _DP, _DP, C.c_int, C.c_int, _DP]
        L.orc_mem_node.argtypes = [P, B, C.c_int, C.c_int, _DP, _DP]
        L.orc_link_point.argtypes = [P, B, C.c_int, C.c_int, C.c_int] + \
            [C.POINTER(C.c_double)] * 2
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_max_threads.restype = C.c_int
        _LIB = L
    return _LIB


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def lattice():
    """(cx, cy, opp, w, M, Minv) as the oracle holds them."""
    cx, cy, opp = (C.c_int * 9)(), (C.c_int * 9)(), (C.c_int * 9)()
    w, M, Mi = np.zeros(9), np.zeros(81), np.zeros(81)
    lib().orc_lattice(cx, cy, opp, w, M, Mi)
    return (np.array(cx[:]), np.array(cy[:]), np.array(opp[:]), w, M.reshape(9, 9),
            Mi.reshape(9, 9))


def feq(rho, ux, uy):
    out = np.zeros(9)
    lib().orc_feq(rho, ux, uy, out)
    return out


def guo(ux, uy, gx, gy):
    out = np.zeros(9)
    lib().orc_guo(ux, uy, gx, gy, out)
    return out


def rk4(Mq, cq, kq, q0, F, q, v):
    a, b = C.c_double(q), C.c_double(v)
    lib().orc_rk4(Mq, cq, kq, q0, F, C.byref(a), C.byref(b))
    return a.value, b.value


def relaxation_vector(rates, conserved=None):
    """Diagonal of S in moment order (rho, e, eps, jx, qx, jy, qy, pxx, pxy)."""
    s_e, s_eps, s_q, s_nu = rates
    sc = s_nu if conserved is None else conserved
    if np.ndim(sc) == 0:
        sc = (sc, sc, sc)
    return [sc[0], s_e, s_eps, sc[1], s_q, sc[2], s_q, s_nu, s_nu]


def make_params(spec, body=None, conserved=None) -> Params:
    p = Params()
    p.nx, p.ny = int(spec["nx"]), int(spec["ny"])
    rates = spec["rates"]
    if spec.get("collision", "mrt") == "bgk":  # single relaxation time 1/tau = s_nu
        rates = (rates[3],) * 4
    for k, v in enumerate(relaxation_vector(rates, conserved)):
        p.s[k] = float(v)
    p.eta = float(spec["eta"])
    bc = spec.get("bc", ("periodic",) * 4)
    for k in range(4):
        p.bc[k] = BC[bc[k]] if isinstance(bc[k], str) else int(bc[k])
    uw = spec.get("u_wall", [[0.0, 0.0]] * 4)
    for k in range(4):
        p.u_wall[k][0], p.u_wall[k][1] = float(uw[k][0]), float(uw[k][1])
    p.u_conv = float(spec.get("u_conv", 0.0))
    g = spec.get("g_fluid", (0.0, 0.0))
    p.g_fluid[0], p.g_fluid[1] = float(g[0]), float(g[1])
    if body is not None:
        p.has_body = 1
        p.radius = float(body["radius"])
        p.smooth_delta = float(body.get("smooth_delta", 0.0))
        m = body.get("mode", "fixed")
        p.mode = MODE[m] if isinstance(m, str) else int(m)
        p.free_mask = int(body.get("free_mask", 0))
        p.mass = float(body.get("mass", 1.0))
        p.inertia = float(body.get("inertia", 1.0))
        for name in ("k", "c", "q0", "f_ext"):
            vals = body.get(name, (0.0, 0.0, 0.0))
            arr = getattr(p, name)
            for d in range(3):
                arr[d] = float(vals[d])
        p.imp_amp = float(body.get("imp_amp", 0.0))
        p.imp_freq = float(body.get("imp_freq", 0.0))
        p.imp_y0 = float(body.get("imp_y0", body.get("y", 0.0)))
        p.imp_phase = float(body.get("imp_phase", 0.0))
        p.internal_mass_correction = int(body.get("internal_mass_correction", 1))
        fm = body.get("force_model", "vp")
        p.force_model = FORCE[fm] if isinstance(fm, str) else int(fm)
    return p


class OracleSim:
    """One simulation held on the host in FP64: populations ``f[9, ny, nx]`` (post-
    collision state), the convective-outflow memory ``outlet[3, ny]`` and the body."""

    def __init__(self, spec, body=None, conserved=None):
        self.spec = dict(spec)
        self.conserved = conserved
        self.nx, self.ny = int(spec["nx"]), int(spec["ny"])
        self.p = make_params(spec, body, conserved)
        self.f = np.zeros((9, self.ny, self.nx))
        self.outlet = np.zeros((3, self.ny))
        u0 = spec.get("u0", (0.0, 0.0))
        lib().orc_init(C.byref(self.p), self.f, self.outlet, float(spec.get("rho0", 1.0)),
                       float(u0[0]), float(u0[1]))
        self.b = Body()
        self.step_index = 0
        if body is not None:
            self.set_body(body)

    def set_body(self, body):
        self.p = make_params(self.spec, body, self.conserved)
        self._apply_chi_add()
        q = np.array([body["x"], body["y"], body.get("theta", 0.0)], dtype=np.float64)
        v = np.array([body.get("vx", 0.0), body.get("vy", 0.0), body.get("omega", 0.0)],
                     dtype=np.float64)
        lib().orc_body_init(C.byref(self.p), C.byref(self.b), q, v)

    def set_chi_perturbation(self, field):
        """Field [ny, nx] added to the indicator of the body at every step (None: off)."""
        self._chi_add = None if field is None else np.ascontiguousarray(field, dtype=np.float64)
        if self._chi_add is not None:
            assert self._chi_add.shape == (self.ny, self.nx)
        self._apply_chi_add()

    def _apply_chi_add(self):
        ca = getattr(self, "_chi_add", None)
        self.p.chi_add = None if ca is None else ca.ctypes.data

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        self.f[...] = f

    def get_populations(self):
        return self.f.copy()

    def set_outlet(self, outlet):
        self.outlet[...] = np.asarray(outlet, dtype=np.float64).reshape(3, self.ny)

    def step(self, n=1):
        """Advance n steps; returns the n per-step records (structured array)."""
        recs = np.zeros(n, dtype=RECORD_DTYPE)
        bad = lib().orc_run(C.byref(self.p), self.f, self.outlet, C.byref(self.b),
                            recs.ctypes.data, self.step_index, n)
        self.step_index += n
        self.unstable = bool(bad)
        return recs

    def fields(self):
        rho = np.zeros((self.ny, self.nx))
        ux = np.zeros_like(rho)
        uy = np.zeros_like(rho)
        lib().orc_fields(C.byref(self.p), self.f, self.outlet, C.byref(self.b), rho, ux, uy)
        return rho, ux, uy

    def pull_node(self, i, j):
        P = np.zeros(9)
        lib().orc_pull_node(C.byref(self.p), self.f, self.outlet, i, j, P)
        return P

    def body_state(self):
        return np.array(self.b.q[:]), np.array(self.b.v[:])

    def mem_node(self, i, j, out):
        """Momentum-exchange contribution (Fx, Fy, T) of node (i, j) whose post-collision
        populations are ``out`` (9 values), at the current pose."""
        F = np.zeros(3)
        lib().orc_mem_node(C.byref(self.p), C.byref(self.b), int(i), int(j),
                           np.ascontiguousarray(out, dtype=np.float64), F)
        return F

    def link_point(self, i, j, a):
        """Crossing of the circle by the link from fluid node (i, j) along c_a."""
        x, y = C.c_double(), C.c_double()
        lib().orc_link_point(C.byref(self.p), C.byref(self.b), int(i), int(j), int(a),
                             C.byref(x), C.byref(y))
        return x.value, y.value

    def chi_field(self):
        """Characteristic function and solid velocity at the current pose."""
        chi = np.zeros((self.ny, self.nx))
        usx, usy = np.zeros_like(chi), np.zeros_like(chi)
        c, a, b = C.c_double(), C.c_double(), C.c_double()
        for j in range(self.ny):
            for i in range(self.nx):
                lib().orc_chi(C.byref(self.p), C.byref(self.b), i, j, C.byref(c), C.byref(a),
                              C.byref(b))
                chi[j, i], usx[j, i], usy[j, i] = c.value, a.value, b.value
        return chi, usx, usy


def node(spec, P, chi=0.0, us=(0.0, 0.0), conserved=None):
    """Single-node collision: returns (post-collision populations, rho, u, G, dF)."""
    p = make_params(spec, None, conserved)
    out, G, dF = np.zeros(9), np.zeros(2), np.zeros(2)
    rho, ux, uy = C.c_double(), C.c_double(), C.c_double()
    lib().orc_node(C.byref(p), np.ascontiguousarray(P, dtype=np.float64), float(chi),
                   float(us[0]), float(us[1]), out, C.byref(rho), C.byref(ux), C.byref(uy), G, dF)
    return out, rho.value, np.array([ux.value, uy.value]), G, dF


os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")
