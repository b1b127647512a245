"""Python binding of the HIP library ``libvplbm.so`` (C ABI of ``include/vplbm.h``).

Argument marshalling only: every step of the method runs in the library's kernels.
PyTorch, when given, supplies the device memory of the two population buffers and
the HIP stream; there is no CPU fallback -- a missing library raises at import of
the first simulation.

A simulation is described by two dicts (``spec`` and ``body``, see ``workloads``).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvplbm.so")

LBM_OK, LBM_ERR_ARG, LBM_ERR_ALLOC, LBM_ERR_HIP, LBM_ERR_UNSTABLE, LBM_ERR_STATE = 0, -1, -2, -3, -4, -5
STORAGE = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
BC = {"periodic": 0, "wall": 1, "velocity": 2, "symmetry": 3, "outflow": 4}
MODE = {"fixed": 0, "imposed_sin": 1, "free": 2, "const_vel": 3}
FORCE = {"vp": 0, "mem": 1, "vp+mem": 2}  # driving load; "mem"/"vp+mem" evaluate the exchange sum
STORE = {"auto": 0, "plain": 1, "nontemporal": 2}
ORDER = {"given": 0, "largest_first": 1, "interleaved": 2}
OFFSET_REF = {"auto": 0, "initial": 1, "rest": 2}  # auto: rest for 16-bit storage, else initial
LAYOUT = {"auto": 0, "rows": 1, "planes": 2}
FINALIZE = {"auto": 0, "tiles": 1, "kernel": 2}

EXPORTS = ["lbm_default_opts", "lbm_pop_bytes", "lbm_create", "lbm_set_body", "lbm_clear_body",
           "lbm_step", "lbm_step_static", "lbm_set_graph_steps", "lbm_sync", "lbm_forces",
           "lbm_fields",
           "lbm_set_populations", "lbm_get_populations", "lbm_get_body_state",
           "lbm_step_index", "lbm_step_timed", "lbm_autotune", "lbm_launch_config", "lbm_layout",
           "lbm_finalize_by_kernel",
           "lbm_save", "lbm_load",
           "lbm_destroy", "lbm_last_error",
           "lbm_default_batch_opts", "lbm_batch_create", "lbm_batch_step",
           "lbm_batch_set_graph_steps", "lbm_batch_sync", "lbm_batch_sim", "lbm_batch_size",
           "lbm_batch_configure", "lbm_batch_autotune", "lbm_batch_order", "lbm_batch_destroy",
           "lbm_batch_last_error",
           "lbm_default_adjoint_opts", "lbm_adjoint_create", "lbm_adjoint_set_body",
           "lbm_adjoint_set_initial", "lbm_adjoint_set_chi_add", "lbm_adjoint_forward", "lbm_adjoint_forces",
           "lbm_adjoint_backward", "lbm_adjoint_gradient", "lbm_adjoint_time_kernels",
           "lbm_adjoint_destroy", "lbm_adjoint_last_error"]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("vplbm error %d: %s" % (code, msg))
        self.code = code


class Rates(C.Structure):
    _fields_ = [("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
                ("s_nu", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("bc", C.c_int * 4), ("u_wall", (C.c_double * 2) * 4), ("u_conv", C.c_double),
                ("g_fluid", C.c_double * 2), ("rho0", C.c_double), ("u0", C.c_double * 2),
                ("storage", C.c_int), ("fp16_scale_log2", C.c_int), ("history_cap", C.c_int),
                ("offset_ref", C.c_int), ("rows_per_tile", C.c_int), ("store_mode", C.c_int),
                ("hip_stream", C.c_void_p),
                ("pop_buffers", C.c_void_p * 2), ("collision", C.c_int), ("tile_width", C.c_int),
                ("layout", C.c_int), ("finalize", C.c_int)]


class Body(C.Structure):
    _fields_ = [("radius", C.c_double), ("x", C.c_double), ("y", C.c_double),
                ("theta", C.c_double), ("vx", C.c_double), ("vy", C.c_double),
                ("omega", C.c_double), ("mode", C.c_int), ("free_mask", C.c_uint),
                ("mass", C.c_double), ("inertia", C.c_double), ("k", C.c_double * 3),
                ("c", C.c_double * 3), ("q0", C.c_double * 3), ("f_ext", C.c_double * 3),
                ("imp_amp", C.c_double), ("imp_freq", C.c_double), ("imp_y0", C.c_double),
                ("smooth_delta", C.c_double), ("internal_mass_correction", C.c_int),
                ("imp_phase", C.c_double), ("force_model", C.c_int)]


class BatchDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("rates", Rates), ("eta", C.c_double),
                ("opts", C.POINTER(Opts)), ("body", C.POINTER(Body))]


class BatchOpts(C.Structure):
    _fields_ = [("storage", C.c_int), ("rows_per_tile", C.c_int), ("store_mode", C.c_int),
                ("order", C.c_int), ("hip_stream", C.c_void_p), ("tile_width", C.c_int),
                ("layout", C.c_int), ("finalize", C.c_int)]


class AdjointOpts(C.Structure):
    _fields_ = [("steps", C.c_int64), ("checkpoint_every", C.c_int), ("weight_fx", C.c_double),
                ("weight_fy", C.c_double), ("use_graphs", C.c_int)]


RECORD_DTYPE = np.dtype([("step", "<i8"), ("fvp", "<f8", (2,)), ("tvp", "<f8"),
                         ("pin", "<f8", (3,)), ("fh", "<f8", (2,)), ("th", "<f8"),
                         ("q", "<f8", (3,)), ("v", "<f8", (3,)),
                         ("fmem", "<f8", (2,)), ("tmem", "<f8")])

_LIB = None
_DP = C.POINTER(C.c_double)


def load_library(path=LIB_PATH):
    """Load ``libvplbm.so``; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError("libvplbm.so is not built (run paper_1905_05110_amd.build)")
    L = C.CDLL(path)
    P = C.c_void_p
    L.lbm_default_opts.argtypes = [C.POINTER(Opts)]
    L.lbm_default_opts.restype = None
    L.lbm_pop_bytes.argtypes = [C.c_int, C.c_int, C.c_int]
    L.lbm_pop_bytes.restype = C.c_size_t
    L.lbm_create.argtypes = [C.c_int, C.c_int, Rates, C.c_double, C.POINTER(Opts), C.POINTER(P)]
    L.lbm_set_body.argtypes = [P, C.POINTER(Body)]
    L.lbm_clear_body.argtypes = [P]
    L.lbm_step.argtypes = [P, C.c_int64]
    L.lbm_step_static.argtypes = [P, C.c_int64]
    L.lbm_set_graph_steps.argtypes = [P, C.c_int]
    L.lbm_sync.argtypes = [P]
    L.lbm_forces.argtypes = [P, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]
    L.lbm_fields.argtypes = [P, _DP, _DP, _DP]
    L.lbm_set_populations.argtypes = [P, _DP]
    L.lbm_get_populations.argtypes = [P, _DP]
    L.lbm_get_body_state.argtypes = [P, _DP, _DP]
    L.lbm_step_index.argtypes = [P]
    L.lbm_step_index.restype = C.c_int64
    L.lbm_step_timed.argtypes = [P, C.c_int64, _DP, _DP]
    L.lbm_autotune.argtypes = [P, C.c_int, C.c_char_p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_double)]
    L.lbm_launch_config.argtypes = [P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.lbm_layout.argtypes = [P, C.POINTER(C.c_int)]
    L.lbm_finalize_by_kernel.argtypes = [P, C.POINTER(C.c_int)]
    L.lbm_save.argtypes = [P, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]
    L.lbm_load.argtypes = [P, C.c_void_p, C.c_size_t]
    L.lbm_destroy.argtypes = [P]
    L.lbm_last_error.argtypes = [P]
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_default_batch_opts.argtypes = [C.POINTER(BatchOpts)]
    L.lbm_default_batch_opts.restype = None
    L.lbm_batch_create.argtypes = [C.c_int, C.POINTER(BatchDesc), C.POINTER(BatchOpts),
                                   C.POINTER(P)]
    L.lbm_batch_step.argtypes = [P, C.c_int64]
    L.lbm_batch_set_graph_steps.argtypes = [P, C.c_int]
    L.lbm_batch_sync.argtypes = [P]
    L.lbm_batch_sim.argtypes = [P, C.c_int, C.POINTER(P)]
    L.lbm_batch_size.argtypes = [P]
    L.lbm_batch_configure.argtypes = [P, C.c_int, C.c_int, C.c_int]
    L.lbm_batch_autotune.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.lbm_batch_order.argtypes = [P, C.POINTER(C.c_int)]
    L.lbm_batch_destroy.argtypes = [P]
    L.lbm_batch_last_error.argtypes = [P]
    L.lbm_batch_last_error.restype = C.c_char_p
    L.lbm_default_adjoint_opts.argtypes = [C.POINTER(AdjointOpts)]
    L.lbm_default_adjoint_opts.restype = None
    L.lbm_adjoint_create.argtypes = [C.c_int, C.c_int, Rates, C.c_double, C.POINTER(Opts),
                                     C.POINTER(Body), C.POINTER(AdjointOpts), C.POINTER(P)]
    L.lbm_adjoint_set_body.argtypes = [P, C.POINTER(Body)]
    L.lbm_adjoint_set_initial.argtypes = [P, _DP, _DP]
    L.lbm_adjoint_set_chi_add.argtypes = [P, _DP]
    L.lbm_adjoint_forward.argtypes = [P, _DP]
    L.lbm_adjoint_forces.argtypes = [P, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]
    L.lbm_adjoint_backward.argtypes = [P]
    L.lbm_adjoint_gradient.argtypes = [P, _DP, _DP, _DP]
    L.lbm_adjoint_time_kernels.argtypes = [P, C.c_int, _DP, _DP]
    L.lbm_adjoint_destroy.argtypes = [P]
    L.lbm_adjoint_last_error.argtypes = [P]
    L.lbm_adjoint_last_error.restype = C.c_char_p
    _LIB = L
    return L


def _ptr(a):
    return a.ctypes.data_as(_DP)


def make_opts(spec, stream=None, buffers=None, history_cap=65536):
    L = load_library()
    o = Opts()
    L.lbm_default_opts(C.byref(o))
    bc = spec.get("bc", ("periodic",) * 4)
    for k in range(4):
        o.bc[k] = BC[bc[k]] if isinstance(bc[k], str) else int(bc[k])
    uw = spec.get("u_wall", [[0.0, 0.0]] * 4)
    for k in range(4):
        o.u_wall[k][0], o.u_wall[k][1] = float(uw[k][0]), float(uw[k][1])
    o.u_conv = float(spec.get("u_conv", 0.0))
    g = spec.get("g_fluid", (0.0, 0.0))
    o.g_fluid[0], o.g_fluid[1] = float(g[0]), float(g[1])
    o.rho0 = float(spec.get("rho0", 1.0))
    u0 = spec.get("u0", (0.0, 0.0))
    o.u0[0], o.u0[1] = float(u0[0]), float(u0[1])
    st = spec.get("storage", "fp32")
    o.storage = STORAGE[st] if isinstance(st, str) else int(st)
    o.fp16_scale_log2 = int(spec.get("fp16_scale_log2", 10))
    o.history_cap = int(history_cap)
    o.offset_ref = OFFSET_REF[spec.get("offset_ref", "auto")]
    o.rows_per_tile = int(spec.get("rows_per_tile", 0))
    o.store_mode = {"auto": 0, "plain": 1, "nontemporal": 2}[spec.get("store_mode", "auto")]
    o.collision = {"mrt": 0, "bgk": 1}[spec.get("collision", "mrt")]
    o.tile_width = int(spec.get("tile_width", 0))
    o.layout = LAYOUT[spec.get("layout", "auto")]
    o.finalize = FINALIZE[spec.get("finalize", "auto")]
    o.hip_stream = stream
    if buffers is not None:
        o.pop_buffers[0], o.pop_buffers[1] = buffers
    return o


def make_body(body):
    b = Body()
    b.radius = float(body["radius"])
    for name in ("x", "y", "theta", "vx", "vy", "omega"):
        setattr(b, name, float(body.get(name, 0.0)))
    m = body.get("mode", "fixed")
    b.mode = MODE[m] if isinstance(m, str) else int(m)
    b.free_mask = int(body.get("free_mask", 0))
    b.mass = float(body.get("mass", 1.0))
    b.inertia = float(body.get("inertia", 1.0))
    for name in ("k", "c", "q0", "f_ext"):
        vals = body.get(name, (0.0, 0.0, 0.0))
        arr = getattr(b, name)
        for d in range(3):
            arr[d] = float(vals[d])
    b.imp_amp = float(body.get("imp_amp", 0.0))
    b.imp_freq = float(body.get("imp_freq", 0.0))
    b.imp_y0 = float(body.get("imp_y0", body.get("y", 0.0)))
    b.smooth_delta = float(body.get("smooth_delta", 0.0))
    b.internal_mass_correction = int(body.get("internal_mass_correction", 1))
    b.imp_phase = float(body.get("imp_phase", 0.0))
    fm = body.get("force_model", "vp")
    b.force_model = FORCE[fm] if isinstance(fm, str) else int(fm)
    return b


class Sim:
    """One simulation on the current GPU.

    ``torch_memory=True`` allocates the two population buffers as torch tensors and
    runs on torch's current stream (the library then borrows them); otherwise the
    library allocates its own buffers and stream.
    """

    @classmethod
    def _member(cls, L, h, spec):
        """Borrowed handle of a batch member (the batch owns and frees it)."""
        self = cls.__new__(cls)
        self.L, self.h, self.spec = L, h, dict(spec)
        self.nx, self.ny = int(spec["nx"]), int(spec["ny"])
        self._tensors = None
        self._borrowed = True
        return self

    def __init__(self, spec, body=None, torch_memory=False, history_cap=65536, graph_steps=0):
        L = load_library()
        self._borrowed = False
        self.L = L
        self.spec = dict(spec)
        self.nx, self.ny = int(spec["nx"]), int(spec["ny"])
        self._tensors = None
        stream, buffers = None, None
        if torch_memory:
            import torch
            st = spec.get("storage", "fp32")
            nbytes = L.lbm_pop_bytes(self.nx, self.ny, STORAGE[st] if isinstance(st, str) else st)
            self._tensors = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
            buffers = (self._tensors[0].data_ptr(), self._tensors[1].data_ptr())
            stream = torch.cuda.current_stream().cuda_stream
        o = make_opts(spec, stream, buffers, history_cap)
        r = spec["rates"]
        h = C.c_void_p()
        rc = L.lbm_create(self.nx, self.ny, Rates(*[float(x) for x in r]), float(spec["eta"]),
                          C.byref(o), C.byref(h))
        if rc != LBM_OK:
            raise LbmError(rc, L.lbm_last_error(None).decode())
        self.h = h
        if graph_steps:
            self._check(L.lbm_set_graph_steps(self.h, int(graph_steps)))
        if body is not None:
            self.set_body(body)

    def _check(self, rc):
        if rc != LBM_OK:
            raise LbmError(rc, self.L.lbm_last_error(self.h).decode())
        return rc

    def set_body(self, body):
        self._body = make_body(body)
        self._check(self.L.lbm_set_body(self.h, C.byref(self._body)))

    def clear_body(self):
        self._check(self.L.lbm_clear_body(self.h))

    def step(self, n=1):
        self._check(self.L.lbm_step(self.h, int(n)))

    def step_static(self, n=1):
        """n steps that allocate nothing (eager launches, the partial force sums in the
        library's static array); see lbm_step_static."""
        self._check(self.L.lbm_step_static(self.h, int(n)))

    def sync(self):
        self._check(self.L.lbm_sync(self.h))

    def set_graph_steps(self, k):
        self._check(self.L.lbm_set_graph_steps(self.h, int(k)))

    def forces(self, cap=None):
        """Records of the steps not yet drained (structured array, oldest first)."""
        if cap is None:
            cap = max(self.step_index(), 1)
        out = np.zeros(int(cap), dtype=RECORD_DTYPE)
        n = C.c_int64()
        self._check(self.L.lbm_forces(self.h, out.ctypes.data, int(cap), C.byref(n)))
        return out[: n.value]

    def fields(self):
        rho = np.zeros((self.ny, self.nx))
        ux, uy = np.zeros_like(rho), np.zeros_like(rho)
        self._check(self.L.lbm_fields(self.h, _ptr(rho), _ptr(ux), _ptr(uy)))
        return rho, ux, uy

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        self._check(self.L.lbm_set_populations(self.h, _ptr(f)))

    def get_populations(self):
        f = np.zeros((9, self.ny, self.nx))
        self._check(self.L.lbm_get_populations(self.h, _ptr(f)))
        return f

    def body_state(self):
        q, v = np.zeros(3), np.zeros(3)
        self._check(self.L.lbm_get_body_state(self.h, _ptr(q), _ptr(v)))
        return q, v

    def step_index(self):
        return int(self.L.lbm_step_index(self.h))

    def step_timed(self, n):
        k, r = C.c_double(), C.c_double()
        self._check(self.L.lbm_step_timed(self.h, int(n), C.byref(k), C.byref(r)))
        return k.value, r.value

    def autotune(self, trial_steps=20, cache=None):
        """Pick rows per tile, store mode and columns per tile by timing; returns (rows, nt,
        us/step); launch_config() also gives the columns per tile."""
        r, n, us = C.c_int(), C.c_int(), C.c_double()
        path = cache.encode() if cache else None
        self._check(self.L.lbm_autotune(self.h, int(trial_steps), path, C.byref(r), C.byref(n),
                                        C.byref(us)))
        return r.value, n.value, us.value

    def launch_config(self):
        """The launch configuration in use: (rows per tile, nt flag, columns per tile)."""
        r, n, w = C.c_int(), C.c_int(), C.c_int()
        self._check(self.L.lbm_launch_config(self.h, C.byref(r), C.byref(n), C.byref(w)))
        return r.value, n.value, w.value

    def layout_name(self):
        """The population layout in use: "rows" or "planes"."""
        v = C.c_int()
        self._check(self.L.lbm_layout(self.h, C.byref(v)))
        return {LAYOUT["rows"]: "rows", LAYOUT["planes"]: "planes"}[v.value]

    def finalize_by_kernel(self):
        """True if the body state is made final by a launch after each step."""
        v = C.c_int()
        self._check(self.L.lbm_finalize_by_kernel(self.h, C.byref(v)))
        return bool(v.value)

    def save(self):
        size = C.c_size_t()
        self._check(self.L.lbm_save(self.h, None, 0, C.byref(size)))
        buf = np.zeros(size.value, dtype=np.uint8)
        self._check(self.L.lbm_save(self.h, buf.ctypes.data, size.value, C.byref(size)))
        return buf

    def load(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.L.lbm_load(self.h, buf.ctypes.data, buf.size))

    def close(self):
        if getattr(self, "h", None):
            if not getattr(self, "_borrowed", False):
                self.L.lbm_destroy(self.h)
            self.h = None
        self._tensors = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many independent simulations advanced by one kernel launch per step.

    ``members`` is a list of (spec, body-or-None); all share ``storage`` and the launch
    configuration.  ``batch.sims[i]`` is a borrowed :class:`Sim` for reading member i
    (forces, fields, body state, populations); stepping goes through the batch.
    """

    def __init__(self, members, storage="fp32", order="largest_first", rows=0, store="auto",
                 history_cap=65536, graph_steps=0, stream=None, tile_width=0, layout="auto",
                 finalize="auto"):
        L = load_library()
        self.L = L
        self.h = None
        n = len(members)
        self._opts = (Opts * n)()
        self._bodies = (Body * n)()
        descs = (BatchDesc * n)()
        for i, (spec, body) in enumerate(members):
            self._opts[i] = make_opts(dict(spec, storage=storage), None, None, history_cap)
            descs[i].nx, descs[i].ny = int(spec["nx"]), int(spec["ny"])
            descs[i].rates = Rates(*[float(x) for x in spec["rates"]])
            descs[i].eta = float(spec["eta"])
            descs[i].opts = C.pointer(self._opts[i])
            if body is not None:
                self._bodies[i] = make_body(body)
                descs[i].body = C.pointer(self._bodies[i])
        bo = BatchOpts()
        L.lbm_default_batch_opts(C.byref(bo))
        bo.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        bo.order = ORDER[order] if isinstance(order, str) else int(order)
        bo.rows_per_tile = int(rows)
        bo.store_mode = STORE[store] if isinstance(store, str) else int(store)
        bo.hip_stream = stream
        bo.tile_width = int(tile_width)
        bo.layout = LAYOUT[layout] if isinstance(layout, str) else int(layout)
        bo.finalize = FINALIZE[finalize] if isinstance(finalize, str) else int(finalize)
        h = C.c_void_p()
        rc = L.lbm_batch_create(n, descs, C.byref(bo), C.byref(h))
        if rc != LBM_OK:
            raise LbmError(rc, L.lbm_batch_last_error(None).decode())
        self.h = h
        self.sims = []
        for i, (spec, _) in enumerate(members):
            sh = C.c_void_p()
            self._check(L.lbm_batch_sim(self.h, i, C.byref(sh)))
            self.sims.append(Sim._member(L, sh, dict(spec, storage=storage)))
        if graph_steps:
            self.set_graph_steps(graph_steps)

    def _check(self, rc):
        if rc != LBM_OK:
            raise LbmError(rc, self.L.lbm_batch_last_error(self.h).decode())
        return rc

    def __len__(self):
        return len(self.sims)

    def step(self, n=1):
        self._check(self.L.lbm_batch_step(self.h, int(n)))

    def sync(self):
        self._check(self.L.lbm_batch_sync(self.h))

    def set_graph_steps(self, k):
        self._check(self.L.lbm_batch_set_graph_steps(self.h, int(k)))

    def configure(self, rows, store, order):
        self._check(self.L.lbm_batch_configure(
            self.h, int(rows), STORE[store] if isinstance(store, str) else int(store),
            ORDER[order] if isinstance(order, str) else int(order)))

    def autotune(self, trial_steps=20):
        """Pick rows, store mode, columns per tile and order by timing; returns (rows, nt,
        order, us/step); a member's launch_config() gives the columns per tile."""
        r, n, o, us = C.c_int(), C.c_int(), C.c_int(), C.c_double()
        self._check(self.L.lbm_batch_autotune(self.h, int(trial_steps), C.byref(r), C.byref(n),
                                              C.byref(o), C.byref(us)))
        return r.value, n.value, o.value, us.value

    def order_name(self):
        """The schedule order in use."""
        v = C.c_int()
        self._check(self.L.lbm_batch_order(self.h, C.byref(v)))
        return {k: n for n, k in ORDER.items()}[v.value]

    def close(self):
        if getattr(self, "h", None):
            for s in self.sims:
                s.h = None
            self.L.lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Adjoint:
    """Reverse-mode gradients of J = sum_{n<N} (w_x F_x(n) + w_y F_y(n)) for a body held
    at a fixed pose: ``forward()`` runs N steps keeping checkpoints and returns J,
    ``backward()`` sweeps them in reverse, ``gradient()`` returns dJ/dchi [ny, nx],
    dJ/d(X, Y) and dJ/d(V_x, V_y, Omega)."""

    def __init__(self, spec, body, steps, checkpoint_every=100, weights=(1.0, 0.0),
                 graphs=True):
        L = load_library()
        self.L, self.h = L, None
        self.nx, self.ny = int(spec["nx"]), int(spec["ny"])
        self.spec = dict(spec)
        self._opts = make_opts(spec)
        self._body = make_body(body)
        ao = AdjointOpts()
        L.lbm_default_adjoint_opts(C.byref(ao))
        ao.steps, ao.checkpoint_every = int(steps), int(checkpoint_every)
        ao.weight_fx, ao.weight_fy = float(weights[0]), float(weights[1])
        ao.use_graphs = 1 if graphs else 0
        self.steps = int(steps)
        self.generation = 0  # forward runs so far; the autograd Function checks it
        self._inputs = None  # (centre, additive indicator) of the last forward run
        h = C.c_void_p()
        rc = L.lbm_adjoint_create(self.nx, self.ny, Rates(*[float(x) for x in spec["rates"]]),
                                  float(spec["eta"]), C.byref(self._opts), C.byref(self._body),
                                  C.byref(ao), C.byref(h))
        if rc != LBM_OK:
            raise LbmError(rc, L.lbm_adjoint_last_error(None).decode())
        self.h = h

    def _check(self, rc):
        if rc != LBM_OK:
            raise LbmError(rc, self.L.lbm_adjoint_last_error(self.h).decode())
        return rc

    def set_body(self, body):
        """Moves the (fixed) body; removes an additive indicator set before."""
        self._body = make_body(body)
        self._check(self.L.lbm_adjoint_set_body(self.h, C.byref(self._body)))

    def set_chi_add(self, field=None):
        """Additive indicator [ny, nx] (zero outside the body's box), or None."""
        if field is None:
            self._check(self.L.lbm_adjoint_set_chi_add(self.h, None))
            return
        field = np.ascontiguousarray(field, dtype=np.float64)
        assert field.shape == (self.ny, self.nx)
        self._check(self.L.lbm_adjoint_set_chi_add(self.h, _ptr(field)))

    def set_initial(self, f=None, outlet=None):
        fp = op = None
        if f is not None:
            f = np.ascontiguousarray(f, dtype=np.float64)
            assert f.shape == (9, self.ny, self.nx)
            fp = _ptr(f)
        if outlet is not None:
            outlet = np.ascontiguousarray(outlet, dtype=np.float64)
            assert outlet.shape == (3, self.ny)
            op = _ptr(outlet)
        self._check(self.L.lbm_adjoint_set_initial(self.h, fp, op))

    def forward(self):
        J = C.c_double()
        self.generation += 1
        self._check(self.L.lbm_adjoint_forward(self.h, C.byref(J)))
        return J.value

    def forces(self):
        out = np.zeros(self.steps, dtype=RECORD_DTYPE)
        n = C.c_int64()
        self._check(self.L.lbm_adjoint_forces(self.h, out.ctypes.data, self.steps, C.byref(n)))
        return out[: n.value]

    def backward(self):
        self._check(self.L.lbm_adjoint_backward(self.h))

    def gradient(self, chi=True):
        g = np.zeros((self.ny, self.nx)) if chi else None
        pos, vel = np.zeros(2), np.zeros(3)
        self._check(self.L.lbm_adjoint_gradient(self.h, _ptr(g) if chi else None, _ptr(pos),
                                                _ptr(vel)))
        return dict(chi=g, pos=pos, vel=vel)

    def time_kernels(self, reps=50):
        a, s = C.c_double(), C.c_double()
        self._check(self.L.lbm_adjoint_time_kernels(self.h, int(reps), C.byref(a), C.byref(s)))
        return a.value, s.value

    def close(self):
        if getattr(self, "h", None):
            self.L.lbm_adjoint_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def adjoint_objective():
    """A ``torch.autograd.Function`` for J of an :class:`Adjoint`:
    ``J = F.apply(center, chi_add, adjoint, body)`` with ``center`` a tensor of 2 (the
    disc's X, Y) and ``chi_add`` a tensor [ny, nx] added to the disc's indicator (zero
    outside the body's box; may be None).  Backward runs the adjoint sweep and returns
    dJ/d(X, Y) and dJ/dchi.  The Function keeps no state of its own between forward and
    backward: it saves its inputs, and when the adjoint has run another forward pass
    since (another apply), backward first runs this one's forward again."""
    import torch

    def run_forward(adj, body, c, chi):
        adj.set_body(dict(body, x=float(c[0]), y=float(c[1])))
        if chi is not None:
            adj.set_chi_add(chi)
        return adj.forward()

    class Objective(torch.autograd.Function):
        @staticmethod
        def forward(ctx, center, chi_add, adj, body):
            c = center.detach().double().cpu().numpy().copy()
            chi = None if chi_add is None else chi_add.detach().double().cpu().numpy().copy()
            J = run_forward(adj, body, c, chi)
            ctx.adj, ctx.body, ctx.c, ctx.chi = adj, dict(body), c, chi
            ctx.generation = adj.generation
            ctx.has_chi = chi_add is not None
            ctx.like = center
            ctx.chi_like = chi_add
            return center.new_tensor(J)

        @staticmethod
        def backward(ctx, grad):
            adj = ctx.adj
            if adj.generation != ctx.generation:  # another forward ran since: redo this one
                run_forward(adj, ctx.body, ctx.c, ctx.chi)
            adj.backward()
            g = adj.gradient(chi=ctx.has_chi)
            gc = grad * ctx.like.new_tensor(g["pos"])
            gchi = grad * ctx.chi_like.new_tensor(g["chi"]) if ctx.has_chi else None
            return gc, gchi, None, None

    return Objective


def body_position_objective():
    """The centre-only form of :func:`adjoint_objective`:
    ``J = Objective.apply(center, adjoint, body)``."""
    import torch
    F = adjoint_objective()

    class Objective(torch.autograd.Function):
        @staticmethod
        def forward(ctx, center, adj, body):
            return F.forward(ctx, center, None, adj, body)

        @staticmethod
        def backward(ctx, grad):
            gc, _, _, _ = F.backward(ctx, grad)
            return gc, None, None

    return Objective
