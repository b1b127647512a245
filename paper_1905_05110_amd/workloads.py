"""Synthetic workloads and seeded input generators for the VP-LBM time step.

This module holds configuration only: grid sizes, boundary kinds, body parameters
and seeded random states.  It contains none of the stream/collide/penalization
arithmetic, imports nothing else from this package, and serves both the GPU path
and the CPU oracle (through the tests and the benchmark).

Parameter readings (the paper leaves these open; each reading is documented once in
the design notes of the repository):

* viscosity from the Reynolds number, nu = U0 D / Re, and the relaxation time from
  nu = c_s^2 (tau - 1/2)  (Sec. 2.2, Eq. (6)); s_nu = 1/tau;
* the remaining MRT rates (s_e, s_eps, s_q) = (1.64, 1.54, 1.9) with eta = 1e-3;
* channel flows: west inlet by moving-wall half-way bounce-back at (U0, 0), east
  convective outflow at U_c = U0, south/north free-slip symmetry (Sec. 3.1);
* imposed oscillation y = y0 + A sin(2 pi f t) with A = 0.2 D and f = 0.2 U0 / D;
* free VIV: mass = 10 x displaced fluid mass, stiffness from the reduced velocity
  U_r = U0 / (f_n D), f_n = sqrt(k/m) / (2 pi), no damping;
* sedimentation: closed box, density ratio 1.5, gravity from the confined-drag
  settling law of Sec. 3.2 (Eqs. (33)-(35)) so that the particle Reynolds number is 1.
"""
import math

import numpy as np

RATES_BASE = (1.64, 1.54, 1.9)  # s_e, s_eps, s_q
ETA = 1e-3


def tau_from(U0: float, D: float, Re: float) -> float:
    nu = U0 * D / Re
    return 3.0 * nu + 0.5


def rates_for_tau(tau: float, base=RATES_BASE):
    return (base[0], base[1], base[2], 1.0 / tau)


def channel_spec(nx, ny, U0, tau, eta=ETA, storage="fp32"):
    return dict(nx=int(nx), ny=int(ny), rates=rates_for_tau(tau), eta=float(eta),
                bc=("velocity", "outflow", "symmetry", "symmetry"),
                u_wall=[[U0, 0.0], [0.0, 0.0], [0.0, 0.0], [0.0, 0.0]],
                u_conv=float(U0), g_fluid=(0.0, 0.0), rho0=1.0, u0=(float(U0), 0.0),
                storage=storage)


def fixed_disc(D, x, y, smooth_delta=0.0):
    return dict(radius=D / 2.0, x=float(x), y=float(y), theta=0.0, vx=0.0, vy=0.0, omega=0.0,
                mode="fixed", free_mask=0, mass=1.0, inertia=1.0, k=(0.0,) * 3, c=(0.0,) * 3,
                q0=(float(x), float(y), 0.0), f_ext=(0.0,) * 3, imp_amp=0.0, imp_freq=0.0,
                imp_y0=float(y), smooth_delta=float(smooth_delta), internal_mass_correction=1)


# ---- the five workloads -------------------------------------------------------------

def imposed_oscillation(storage="fp64", nx=200, ny=80, D=20.0, U0=0.05, Re=100.0):
    """200x80 channel, disc D=20 at (50, 40) in imposed transverse oscillation."""
    tau = tau_from(U0, D, Re)
    spec = channel_spec(nx, ny, U0, tau, storage=storage)
    body = fixed_disc(D, nx / 4.0, ny / 2.0)
    body.update(mode="imposed_sin", imp_amp=0.2 * D, imp_freq=0.2 * U0 / D, imp_y0=ny / 2.0)
    return dict(name="imposed_oscillation_%dx%d" % (nx, ny), spec=spec, body=body, steps=2000,
                U0=U0, D=D)


def paper_imposed_oscillation(storage="fp64", nx=1230, ny=410, D=41.0, U0=0.04878,
                              tau=0.56, omega_star=1.55, B_star=0.25, eta=1e-6):
    """The paper's imposed-displacement case (Sec. 3.1): channel 1230 x 410, D = 41,
    tau = 0.56 (Re = 100), U0 = 0.04878, rates (1.1, 1.25, 1.8) for (e, eps, q) with
    the others 1/tau (Eq. (28)), eta = 1e-6, and after a fixed-cylinder run the law
    y_G(t) = (y_G(0) - B) + B cos(omega t) of Eq. (29) with omega* = omega D / U0 = 1.55
    and B* = B / D = 1/4.  The disc sits at (nx/4, ny/2).  Returns the fixed body of the
    preliminary run and the moving one (cosine law: phase pi/2)."""
    spec = channel_spec(nx, ny, U0, tau, eta=eta, storage=storage)
    spec["rates"] = (1.1, 1.25, 1.8, 1.0 / tau)
    x, y = nx / 4.0, ny / 2.0
    fixed = fixed_disc(D, x, y)
    fixed["force_model"] = "mem"
    B = B_star * D
    omega = omega_star * U0 / D
    moving = dict(fixed, mode="imposed_sin", imp_amp=B, imp_freq=omega / (2.0 * math.pi),
                  imp_y0=y - B, imp_phase=0.5 * math.pi)
    return dict(name="paper_imposed_%dx%d" % (nx, ny), spec=spec, fixed=fixed, body=moving,
                U0=U0, D=D, period=2.0 * math.pi / omega)


def paper_viv(k_star, m_star=9.0, storage="fp32", nx=1230, ny=410, D=41.0, U0=0.04878,
              tau=0.56, eta=1e-6):
    """The paper's vortex-induced vibration case (Sec. 3.3): the channel and parameters of
    Sec. 3.1 (1230 x 410, D = 41, tau = 0.56, U0 = 0.04878, Re = 100), the disc free in
    y on an undamped spring, m* y*'' + k* (y* - y0*) = C_L with m* = m / (rho D^2 / 2) and
    k* = k / (rho U0^2 / 2); released at rest with the spring relaxed, in the uniform
    inflow state.  The momentum-exchange load drives it.  m* is not stated in the paper;
    9 is the value for which the printed k*_eff of the case far from lock-in (k* = 28,
    response at the wake's shedding frequency) is reproduced."""
    spec = channel_spec(nx, ny, U0, tau, eta=eta, storage=storage)
    spec["rates"] = (1.1, 1.25, 1.8, 1.0 / tau)
    x, y = nx / 4.0, ny / 2.0
    m = m_star * 0.5 * D * D
    k = k_star * 0.5 * U0 * U0
    b = fixed_disc(D, x, y)
    b.update(mode="free", free_mask=0b010, mass=m, inertia=0.5 * m * (D / 2.0) ** 2,
             k=(0.0, k, 0.0), c=(0.0, 0.0, 0.0), q0=(x, y, 0.0), force_model="mem")
    return dict(name="paper_viv_k%g" % k_star, spec=spec, body=b, U0=U0, D=D, m_star=m_star,
                k_star=k_star)


def viv_body(D, x, y, U0, Ur, mass_ratio=10.0, damping=0.0):
    m = mass_ratio * math.pi * D * D / 4.0  # mass ratio x displaced fluid mass (rho0 = 1)
    fn = U0 / (Ur * D)
    k = m * (2.0 * math.pi * fn) ** 2
    b = fixed_disc(D, x, y)
    b.update(mode="free", free_mask=0b010, mass=m, inertia=0.5 * m * (D / 2.0) ** 2,
             k=(0.0, k, 0.0), c=(0.0, damping, 0.0), q0=(float(x), float(y), 0.0))
    return b


def free_viv(storage="fp32", nx=2048, ny=1024, D=40.0, U0=0.05, Re=150.0, Ur=5.0):
    """2048x1024 channel, disc D=40 on a transverse spring (mass ratio 10, U_r = 5)."""
    tau = tau_from(U0, D, Re)
    spec = channel_spec(nx, ny, U0, tau, storage=storage)
    body = viv_body(D, nx / 4.0, ny / 2.0, U0, Ur)
    return dict(name="free_viv_%dx%d" % (nx, ny), spec=spec, body=body, steps=100000, U0=U0, D=D)


def confinement_kappa(Ht: float) -> float:
    """Wall-correction factor of the confined settling law (Sec. 3.2, Eq. (34))."""
    return 1.0 / (math.log(Ht) - 0.9157 + 1.7244 * Ht ** -2 - 1.7302 * Ht ** -4
                  + 2.4056 * Ht ** -6 - 4.5913 * Ht ** -8)


PAPER_DENSITY_RATIOS = (0.95, 0.98, 0.99, 1.01, 1.02, 1.05)


def paper_sedimentation_centered(rho_ratio, storage="fp64", D=24.0, Ht=5.0, L=1200,
                                 tau=0.8, D_cm=0.24, mu=0.1, g_cm=980.0,
                                 force_model="mem"):
    """The paper's centred settling case (Sec. 3.2.1): a disc of D = 0.24 cm (24 nodes)
    in a channel of width H = 5 D and length L = 1200 nodes, fluid rho = 1 g/cm^3,
    mu = 0.1 g/(cm s), |g| = 980 cm/s^2, tau = 0.8, released at rest on the centre
    line half-way along the channel.  Lattice units follow from dx = D_cm / D and
    nu_lattice = (tau - 1/2)/3 = nu dt / dx^2.  The channel axis is x here (the D2Q9
    lattice is symmetric under a quarter turn) with gravity along +x; both ends are
    closed (the net flux through every section is zero, as with the zero-velocity top
    and far outlet of the paper).  The disc is free in x, y and theta with
    m = rho_s pi D^2 / 4, I = m R^2 / 2 and the load of Eq. (31): m (1 - rho/rho_s) g.
    Returns also the confined settling velocity of Eqs. (33)-(35) in lattice units."""
    H = int(round(Ht * D))
    nu_l = (tau - 0.5) / 3.0
    dx = D_cm / D
    dt = nu_l * dx * dx / (mu / 1.0)
    g = g_cm * dt * dt / dx
    spec = dict(nx=int(L), ny=H, rates=rates_for_tau(tau), eta=ETA, bc=("wall",) * 4,
                u_wall=[[0.0, 0.0]] * 4, u_conv=0.0, g_fluid=(0.0, 0.0), rho0=1.0,
                u0=(0.0, 0.0), storage=storage)
    m = rho_ratio * math.pi * D * D / 4.0
    body = fixed_disc(D, L / 2.0, (H - 1) / 2.0)
    body.update(mode="free", free_mask=0b111, mass=m, inertia=0.5 * m * (D / 2.0) ** 2,
                f_ext=(m * (1.0 - 1.0 / rho_ratio) * g, 0.0, 0.0), force_model=force_model)
    kappa = confinement_kappa(Ht)
    vs = D * D * (rho_ratio - 1.0) * g / (16.0 * kappa * nu_l)  # along +x (mu = nu, rho = 1)
    return dict(name="paper_sedimentation_%g" % rho_ratio, spec=spec, body=body, vs=vs,
                g=g, dt=dt, dx=dx, kappa=kappa, D=D)


def paper_sedimentation_offcentre(storage="fp32", D=31.0, H=125, L=1550, tau=0.6,
                                  rho_ratio=1.03, D_cm=0.1, mu=0.01, g_cm=980.0,
                                  x0_D=0.75, y0_D=12.5, force_model="mem"):
    """The paper's non-centred settling case (Sec. 3.2.2): D = 0.1 cm (31 nodes) in a
    channel 125 nodes wide and 1550 long, rho_s / rho = 1.03, |g| = 980 cm/s^2, tau = 0.6,
    released at rest 0.75 D from a side wall and 12.5 D below the top.  The viscosity is
    taken as 0.01 g/(cm s): with the printed 0.1 the confined Stokes settling velocity
    gives a particle Reynolds number of 0.1, against the final 8.33 the paper states.  Axes as in paper_sedimentation_centered (channel along x, gravity
    along +x, closed ends).  The paper gives the particle Reynolds number of the final
    velocity, 8.33; re_final converts it to a lattice velocity."""
    nu_l = (tau - 0.5) / 3.0
    dx = D_cm / D
    dt = nu_l * dx * dx / mu
    g = g_cm * dt * dt / dx
    spec = dict(nx=int(L), ny=int(H), rates=rates_for_tau(tau), eta=ETA, bc=("wall",) * 4,
                u_wall=[[0.0, 0.0]] * 4, u_conv=0.0, g_fluid=(0.0, 0.0), rho0=1.0,
                u0=(0.0, 0.0), storage=storage)
    m = rho_ratio * math.pi * D * D / 4.0
    y0 = -0.5 + x0_D * D  # from the wall half-way below node 0
    x0 = -0.5 + y0_D * D
    body = fixed_disc(D, x0, y0)
    body.update(mode="free", free_mask=0b111, mass=m, inertia=0.5 * m * (D / 2.0) ** 2,
                f_ext=(m * (1.0 - 1.0 / rho_ratio) * g, 0.0, 0.0), force_model=force_model)
    return dict(name="paper_sedimentation_offcentre", spec=spec, body=body, g=g, dt=dt,
                dx=dx, D=D, nu=nu_l, re_final=8.33)


def sedimentation(storage="fp32", nx=1024, ny=4096, D=32.0, x=512.0, y=3800.0, rho_ratio=1.5,
                  tau=0.8, Re_p=1.0):
    """Closed box, disc released from rest, free in x, y and theta under gravity."""
    nu = (tau - 0.5) / 3.0
    vs = Re_p * nu / D
    kappa = confinement_kappa(nx / D)
    g = 16.0 * kappa * nu * vs / (D * D * (rho_ratio - 1.0))  # mu = rho nu, rho = 1
    R = D / 2.0
    m = rho_ratio * math.pi * R * R
    spec = dict(nx=int(nx), ny=int(ny), rates=rates_for_tau(tau), eta=ETA,
                bc=("wall", "wall", "wall", "wall"), u_wall=[[0.0, 0.0]] * 4, u_conv=0.0,
                g_fluid=(0.0, 0.0), rho0=1.0, u0=(0.0, 0.0), storage=storage)
    body = fixed_disc(D, x, y)
    body.update(mode="free", free_mask=0b111, mass=m, inertia=0.5 * m * R * R,
                f_ext=(0.0, -m * (1.0 - 1.0 / rho_ratio) * g, 0.0))
    return dict(name="sedimentation_%dx%d" % (nx, ny), spec=spec, body=body, steps=200000,
                g=g, vs=vs, kappa=kappa, D=D, U0=vs)


def batch_sweep(storage="fp32", n=64, seed=0, U0=0.05, Re=150.0):
    """64 VIV runs of uneven size: ny ~ U{128..512}, nx = 2 ny, D = ny/12, U_r 2..12."""
    rng = np.random.default_rng(seed)
    nys = rng.integers(128, 513, n)
    sims = []
    for i, ny in enumerate(nys):
        ny = int(ny)
        nx = 2 * ny
        D = ny / 12.0
        Ur = 2.0 + 10.0 * i / max(n - 1, 1)
        tau = tau_from(U0, D, Re)
        spec = channel_spec(nx, ny, U0, tau, storage=storage)
        body = viv_body(D, nx / 4.0, ny / 2.0, U0, Ur)
        sims.append(dict(name="viv_%d_%dx%d" % (i, nx, ny), spec=spec, body=body, U0=U0, D=D))
    return sims


def adjoint_drag(storage="fp32", nx=1024, ny=512, D=32.0, U0=0.05, Re=100.0, delta=1.0):
    """Fixed disc with a tanh-smoothed indicator (interface width 2 delta)."""
    tau = tau_from(U0, D, Re)
    spec = channel_spec(nx, ny, U0, tau, storage=storage)
    body = fixed_disc(D, nx / 4.0, ny / 2.0, smooth_delta=delta)
    return dict(name="adjoint_drag_%dx%d" % (nx, ny), spec=spec, body=body, steps=4000,
                checkpoint_every=100, U0=U0, D=D)


def roofline_grid(storage="fp32", n=8192, D=512.0, U0=0.05, Re=100.0):
    tau = tau_from(U0, D, Re)
    spec = channel_spec(n, n, U0, tau, storage=storage)
    body = fixed_disc(D, n / 4.0, n / 2.0)
    return dict(name="roofline_%dx%d" % (n, n), spec=spec, body=body, steps=200, U0=U0, D=D)


# ---- seeded random states -------------------------------------------------------------

LATTICE_WEIGHTS = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def random_populations(nx, ny, seed=1234, amp=0.1):
    """Post-collision populations w_a (1 + amp * xi), xi ~ U(-1, 1): a random,
    positive, near-rest state used to drive the step-by-step comparisons."""
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=(9, ny, nx))
    return LATTICE_WEIGHTS[:, None, None] * (1.0 + amp * xi)
