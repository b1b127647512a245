"""FP64 torch-CPU mirror of the VP-LBM time step, differentiated in reverse mode.

TEST INFRASTRUCTURE ONLY: imported by the tests; never by the GPU product path.  It
shares no code with the GPU path (nor with the C oracle: the lattice, the boundary
rules and the collision are written out here again, from the paper).

What it computes.  A body held at a fixed pose (X, Y) with a rigid velocity field
u_s = V + Omega e_z x (x - X) (Sec. 2.1) in a flow advanced by the step of Sec. 2.2:
pull streaming with the boundary rules (Eq. (18)), the implicit penalized velocity and
force density (Eqs. (19)-(22)), and the MRT collision with the Guo source in moment
space (Eqs. (8), (12)-(17)).  The objective is a weighted sum of the penalization force
on the body over the first N steps,

    J = sum_{n < N} ( w_x F_x(n) + w_y F_y(n) ),   F(n) = sum_nodes rho (chi/eta)(u - u_s),

and torch autograd gives dJ/d(chi perturbation field), dJ/d(X, Y) (through the smoothed
indicator chi = 1 / (1 + exp(2 (d - R)/delta)), Eq. (2) smoothed, and through u_s) and
dJ/d(V_x, V_y, Omega).  The time loop is cut into segments of K steps whose internals
are recomputed during the reverse sweep (checkpointing), so memory stays bounded.

Readings shared with the C oracle: nodes at integer (i, j); walls half-way; the x rule
takes precedence at corners; the VELOCITY rule adds 6 w_a (c_a . u_w) with rho_w = 1;
the convective outflow P = (O + U_c Q) / (1 + U_c) with Q the value pulled one node in
and O the previous step's east-column value; the indicator is clamped to 0 / 1 where
|d - R| / delta > 20; the conserved moments relax with s_nu (the result does not depend
on their rates).
"""
import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

BC = {"periodic": 0, "wall": 1, "velocity": 2, "symmetry": 3, "outflow": 4}
PERIODIC, WALL, VELOCITY, SYMMETRY, OUTFLOW = range(5)

# D2Q9 velocities in the order of Sec. 2.2 (rest, E, N, W, S, NE, NW, SW, SE)
CX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
CY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
W = (4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36)
CS2 = 1.0 / 3.0
# moment basis of Eq. (15): rho, e, eps, jx, qx, jy, qy, pxx, pxy
M = np.array([[1, 1, 1, 1, 1, 1, 1, 1, 1],
              [-4, -1, -1, -1, -1, 2, 2, 2, 2],
              [4, -2, -2, -2, -2, 1, 1, 1, 1],
              [0, 1, 0, -1, 0, 1, -1, -1, 1],
              [0, -2, 0, 2, 0, 1, -1, -1, 1],
              [0, 0, 1, 0, -1, 1, 1, -1, -1],
              [0, 0, -2, 0, 2, 1, 1, -1, -1],
              [0, 1, -1, 1, -1, 0, 0, 0, 0],
              [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=np.float64)


def _find(cx, cy):
    for b in range(9):
        if CX[b] == cx and CY[b] == cy:
            return b
    raise ValueError


def opposite(a):
    return _find(-CX[a], -CY[a])


def flip_x(a):
    return _find(-CX[a], CY[a])


def flip_y(a):
    return _find(CX[a], -CY[a])


def _bc_kinds(spec):
    bc = spec.get("bc", ("periodic",) * 4)
    return [BC[b] if isinstance(b, str) else int(b) for b in bc]


class PullMap:
    """Where each pulled value P_a(i, j) comes from: a flat index into f[9, ny, nx] plus
    a constant, or the convective outflow rule (east side only)."""

    def __init__(self, spec):
        self.nx, self.ny = nx, ny = int(spec["nx"]), int(spec["ny"])
        self.bc = _bc_kinds(spec)
        self.uw = np.asarray(spec.get("u_wall", [[0.0, 0.0]] * 4), dtype=np.float64)
        self.uc = float(spec.get("u_conv", 0.0))
        src = np.zeros((9, ny, nx), dtype=np.int64)
        cst = np.zeros((9, ny, nx))
        outs = []  # (a, j, q_src, q_cst)
        for a in range(9):
            for j in range(ny):
                for i in range(nx):
                    r = self.resolve(a, i, j)
                    if r is None:
                        q = self.resolve(a, nx - 2, j)
                        outs.append((a, j, self._flat(*q[0]), q[1]))
                    else:
                        src[a, j, i] = self._flat(*r[0])
                        cst[a, j, i] = r[1]
        self.src = torch.from_numpy(src)
        self.cst = torch.from_numpy(cst)
        self.n_out = len(outs)
        if outs:
            a_idx = np.array([o[0] for o in outs])
            self.out_a = torch.from_numpy(a_idx)
            self.out_j = torch.from_numpy(np.array([o[1] for o in outs]))
            self.out_i = torch.full((len(outs),), nx - 1, dtype=torch.int64)
            self.out_slot = torch.from_numpy(np.array([{3: 0, 6: 1, 7: 2}[a] for a in a_idx]))
            self.out_qsrc = torch.from_numpy(np.array([o[2] for o in outs]))
            self.out_qcst = torch.from_numpy(np.array([o[3] for o in outs], dtype=np.float64))

    def _flat(self, a, i, j):
        return (a * self.ny + j) * self.nx + i

    def _wall_const(self, a, side):
        if self.bc[side] != VELOCITY:
            return 0.0
        cu = CX[a] * self.uw[side][0] + CY[a] * self.uw[side][1]
        return 2.0 * W[a] * cu / CS2

    def resolve(self, a, i, j):
        """((direction, i, j), constant) of the population read, or None (outflow)."""
        nx, ny = self.nx, self.ny
        si, sj, d = i - CX[a], j - CY[a], a
        if not 0 <= si < nx:
            side = 0 if si < 0 else 1
            kind = self.bc[side]
            if kind == PERIODIC:
                si %= nx
            elif kind == SYMMETRY:
                d, si = flip_x(a), i
            elif kind == OUTFLOW:
                return None
            else:
                return (opposite(a), i, j), self._wall_const(a, side)
        if not 0 <= sj < ny:
            side = 2 if sj < 0 else 3
            kind = self.bc[side]
            if kind == PERIODIC:
                sj %= ny
            elif kind == SYMMETRY:
                d, sj = flip_y(d), j
            else:
                return (opposite(a), i, j), self._wall_const(a, side)
        return (d, si, sj), 0.0

    def pull(self, f, outlet):
        """P[9, ny, nx] from the post-collision field f and the outflow memory."""
        flat = f.reshape(-1)
        P = flat[self.src] + self.cst
        if self.n_out:
            q = flat[self.out_qsrc] + self.out_qcst
            v = (outlet[self.out_slot, self.out_j] + self.uc * q) / (1.0 + self.uc)
            P = P.index_put((self.out_a, self.out_j, self.out_i), v)
        return P


class Collision:
    """Node-wise penalized MRT collision (vectorised over the grid)."""

    def __init__(self, spec):
        s_e, s_eps, s_q, s_nu = [float(x) for x in spec["rates"]]
        self.s = torch.tensor([s_nu, s_e, s_eps, s_nu, s_q, s_nu, s_q, s_nu, s_nu],
                              dtype=torch.float64).view(9, 1, 1)
        self.M = torch.from_numpy(M)
        self.Minv = torch.from_numpy(M.T / (M * M).sum(axis=1))
        self.eta = float(spec["eta"])
        g = spec.get("g_fluid", (0.0, 0.0))
        self.gx, self.gy = float(g[0]), float(g[1])
        self.cx = torch.tensor(CX, dtype=torch.float64).view(9, 1, 1)
        self.cy = torch.tensor(CY, dtype=torch.float64).view(9, 1, 1)
        self.w = torch.tensor(W, dtype=torch.float64).view(9, 1, 1)

    def __call__(self, P, chi, usx, usy):
        rho = P.sum(0)
        jx = (self.cx * P).sum(0)
        jy = (self.cy * P).sum(0)
        lam = chi / self.eta
        den = rho * (1.0 + 0.5 * lam)
        rx = (jx + 0.5 * rho * self.gx - rho * usx) / den
        ry = (jy + 0.5 * rho * self.gy - rho * usy) / den
        ux, uy = usx + rx, usy + ry
        Gx = rho * self.gx - rho * lam * rx
        Gy = rho * self.gy - rho * lam * ry
        m = torch.einsum("kb,bji->kji", self.M, P)
        usq = ux * ux + uy * uy
        meq = torch.stack([rho, rho * (-2.0 + 3.0 * usq), rho * (1.0 - 3.0 * usq), rho * ux,
                           -rho * ux, rho * uy, -rho * uy, rho * (ux * ux - uy * uy),
                           rho * ux * uy])
        cu = self.cx * ux + self.cy * uy
        ex = (self.cx - ux) / CS2 + cu * self.cx / (CS2 * CS2)
        ey = (self.cy - uy) / CS2 + cu * self.cy / (CS2 * CS2)
        fhat = self.w * (ex * Gx + ey * Gy)
        mF = torch.einsum("kb,bji->kji", self.M, fhat)
        ms = m - self.s * (m - meq) + (1.0 - 0.5 * self.s) * mF
        out = torch.einsum("ak,kji->aji", self.Minv, ms)
        return out, (rho * lam * rx).sum(), (rho * lam * ry).sum()


def indicator(spec, body, X, Y, Vx, Vy, Om, chi_add=None):
    """chi and u_s on the grid for the pose (X, Y) and rigid velocity (V, Omega)."""
    nx, ny = int(spec["nx"]), int(spec["ny"])
    jj, ii = torch.meshgrid(torch.arange(ny, dtype=torch.float64),
                            torch.arange(nx, dtype=torch.float64), indexing="ij")
    dx, dy = ii - X, jj - Y
    d2 = dx * dx + dy * dy
    R = float(body["radius"])
    delta = float(body.get("smooth_delta", 0.0))
    if delta > 0.0:
        pos = d2 > 0.0
        d = torch.where(pos, torch.sqrt(torch.where(pos, d2, torch.ones_like(d2))),
                        torch.zeros_like(d2))
        z = (d - R) / delta
        zc = z.clamp(-20.0, 20.0)
        chi = torch.where(z > 20.0, torch.zeros_like(z),
                          torch.where(z < -20.0, torch.ones_like(z), 1.0 / (1.0 + torch.exp(2.0 * zc))))
    else:
        chi = (d2 <= R * R).to(torch.float64)
    if chi_add is not None:
        chi = chi + chi_add
    return chi, Vx - Om * dy, Vy + Om * dx


def initial_state(spec):
    """f = f_eq(rho0, u0) everywhere and the outflow memory likewise (Eq. (11))."""
    nx, ny = int(spec["nx"]), int(spec["ny"])
    rho0 = float(spec.get("rho0", 1.0))
    u0 = spec.get("u0", (0.0, 0.0))
    feq = np.zeros(9)
    for a in range(9):
        cu = CX[a] * u0[0] + CY[a] * u0[1]
        uu = cu * cu - CS2 * (u0[0] ** 2 + u0[1] ** 2)
        feq[a] = W[a] * rho0 * (1.0 + cu / CS2 + uu / (2.0 * CS2 * CS2))
    f = np.broadcast_to(feq.reshape(9, 1, 1), (9, ny, nx)).copy()
    outlet = np.broadcast_to(feq[[3, 6, 7]].reshape(3, 1), (3, ny)).copy()
    return f, outlet


class Mirror:
    """The step and the objective of one configuration."""

    def __init__(self, spec, body):
        self.spec, self.body = dict(spec), dict(body)
        self.pull_map = PullMap(spec)
        self.collide = Collision(spec)

    def step(self, f, outlet, chi, usx, usy):
        P = self.pull_map.pull(f, outlet)
        if self.pull_map.bc[1] == OUTFLOW:
            outlet = P[[3, 6, 7], :, -1]
        out, Fx, Fy = self.collide(P, chi, usx, usy)
        return out, outlet, Fx, Fy

    def run(self, f, outlet, n, pose=None):
        """n plain steps (no gradient); returns f, outlet and the forces per step."""
        X, Y, Vx, Vy, Om = pose if pose is not None else self._pose()
        with torch.no_grad():
            chi, usx, usy = indicator(self.spec, self.body, X, Y, Vx, Vy, Om)
            f, outlet = torch.as_tensor(f), torch.as_tensor(outlet)
            F = []
            for _ in range(n):
                f, outlet, Fx, Fy = self.step(f, outlet, chi, usx, usy)
                F.append((Fx.item(), Fy.item()))
        return f.numpy(), outlet.numpy(), np.array(F)

    def _pose(self):
        b = self.body
        return tuple(torch.tensor(float(b.get(k, 0.0)), dtype=torch.float64)
                     for k in ("x", "y", "vx", "vy", "omega"))

    def gradient(self, steps, every, weights, f0=None, outlet0=None):
        """J and its gradients: dict(J, chi (field [ny, nx]), pos (X, Y), vel (Vx, Vy, Omega))."""
        if steps % every:
            raise ValueError("steps must be a multiple of the checkpoint interval")
        wx, wy = float(weights[0]), float(weights[1])
        f_init, o_init = initial_state(self.spec)
        f0 = f_init if f0 is None else f0
        outlet0 = o_init if outlet0 is None else outlet0
        f = torch.as_tensor(np.ascontiguousarray(f0, dtype=np.float64))
        outlet = torch.as_tensor(np.ascontiguousarray(outlet0, dtype=np.float64))
        pose = [t.clone().requires_grad_(True) for t in self._pose()]
        chi_add = torch.zeros((int(self.spec["ny"]), int(self.spec["nx"])), dtype=torch.float64,
                              requires_grad=True)
        chi, usx, usy = indicator(self.spec, self.body, *pose, chi_add=chi_add)

        def segment(f, outlet, chi, usx, usy):
            J = torch.zeros((), dtype=torch.float64)
            for _ in range(every):
                f, outlet, Fx, Fy = self.step(f, outlet, chi, usx, usy)
                J = J + (wx * Fx + wy * Fy)
            return f, outlet, J

        J = torch.zeros((), dtype=torch.float64)
        for _ in range(steps // every):
            f, outlet, Js = checkpoint(segment, f, outlet, chi, usx, usy, use_reentrant=False)
            J = J + Js
        J.backward()
        g = [t.grad.item() if t.grad is not None else 0.0 for t in pose]
        return dict(J=J.item(), chi=chi_add.grad.numpy().copy(), pos=np.array(g[:2]),
                    vel=np.array(g[2:]))
