/*
 * vplbm_oracle.c -- plain, slow FP64 CPU reference of one time step of the
 * volume-penalization lattice-Boltzmann method (VP-LBM) of Liberge & Beghein,
 * "Fluid Structure Interaction modelling using Lattice Boltzmann and Volume
 * Penalization method" (arXiv 1905.05110).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The GPU product path never
 * links, loads or calls it, and it shares no code, header or table with that path.
 *
 * It is written to be checked against the paper by eye:
 *   - lattice, weights, equilibrium, Guo forcing ........ Sec. 2.2, Eqs. (10)-(13)
 *   - moment matrix M and its inverse ................... Sec. 2.2, Eqs. (9), (15)
 *   - MRT collision with source (sign of Eq. (8)) ....... Sec. 2.2, Eqs. (8), (14), (16), (17)
 *   - streaming (applied as a pull) ..................... Sec. 2.2, Eq. (18)
 *   - implicit penalized velocity ....................... Sec. 2.2, Eqs. (19)-(22)
 *   - rigid-body equations, 4th-order Runge-Kutta ....... Sec. 2.3, Eqs. (23), (24), Algorithm 1
 *   - imposed transverse motion, y0 + A sin(2 pi f t + phi) .. Sec. 3.1, Eq. (29)
 *   - momentum-exchange force and torque ................ Sec. 2.3, Eqs. (25)-(27)
 * The body is driven either by the volume integral of the penalization force
 * (rho*chi/eta*(u - u_s), with the internal-fluid momentum term) or by the
 * momentum-exchange sum of Eqs. (25)-(27); both are recorded at every step.
 *
 * Every 9x9 product is a plain double loop; there is no blocking, fusion or
 * reordering.  Compile with -O2 -ffp-contract=off (no -ffast-math).
 *
 * Parity status of each function (what pins it) is listed in the test suite
 * (tests/test_oracle_pins.py); every function here is pinned.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

/* ---- Lattice (Sec. 2.2, Eqs. (10), (13)) -------------------------------------- */
/* c_0 = 0; c_1..c_4 = (cos((a-1)pi/2), sin((a-1)pi/2)); c_5..c_8 = sqrt2 (cos((2a-9)pi/4), sin(...)) */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WGT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* speed of sound squared, c_s = c/sqrt(3) */

/* Transformation matrix M as printed in Eq. (15). */
static const double MM[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},          {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},      {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},       {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},       {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* Boundary kinds (one per domain side), body motion modes. */
enum { BC_PERIODIC = 0, BC_WALL = 1, BC_VELOCITY = 2, BC_SYMMETRY = 3, BC_OUTFLOW = 4 };
enum { SIDE_W = 0, SIDE_E = 1, SIDE_S = 2, SIDE_N = 3 };
enum { MODE_FIXED = 0, MODE_IMPOSED_SIN = 1, MODE_FREE = 2, MODE_CONST_VEL = 3 };
enum { FORCE_VP = 0, FORCE_MEM = 1, FORCE_VP_WITH_MEM = 2 };

typedef struct {
    int nx, ny;
    double s[Q];          /* diagonal of S, Eq. (16); s[0], s[3], s[5] act on conserved moments */
    double eta;           /* penalization factor, Eq. (2) */
    int bc[4];            /* west, east, south, north */
    double u_wall[4][2];  /* wall velocity of each side (VELOCITY sides) */
    double u_conv;        /* convective velocity of the outflow condition */
    double g_fluid[2];    /* uniform body-force acceleration on the fluid */
    /* rigid body (one disc) */
    int has_body;
    double radius;
    double smooth_delta;  /* 0: sharp indicator of Eq. (2); >0: 1/(1+exp(2(d-R)/delta)) */
    int mode;
    unsigned free_mask;   /* bit 0: x, bit 1: y, bit 2: theta */
    double mass, inertia;
    double k[3], c[3], q0[3], f_ext[3];
    double imp_amp, imp_freq, imp_y0, imp_phase;
    int internal_mass_correction;
    int force_model;      /* FORCE_MEM: the exchange load drives a FREE body; else the
                             penalization load (both are always recorded here) */
    /* optional [ny][nx] field added to the indicator (NULL: none); the design variable
     * of the sensitivity checks, perturbed node by node for finite differences */
    const double* chi_add;
} orc_params;

typedef struct {
    double q[3];     /* X, Y, theta */
    double v[3];     /* Vx, Vy, Omega */
    int64_t t_body;  /* steps since the body was set (phase of the imposed motion) */
    double pin_prev[3];
    int pin_valid;
} orc_body;

typedef struct {
    int64_t step;
    double fvp[2], tvp;   /* penalization force and torque on the body */
    double pin[3];        /* post-collision momentum and angular momentum of the fluid
                             inside the body: sum of chi * (j + G) and chi * r x (j + G) */
    double fh[2], th;     /* hydrodynamic force/torque (with the internal-fluid term when enabled) */
    double q[3], v[3];    /* pose and velocities used during this step */
    double fmem[2], tmem; /* momentum-exchange force and torque, Eqs. (25)-(27) */
} orc_record;

/* ---- small helpers ------------------------------------------------------------- */
static double MINV[Q][Q]; /* filled once when the library is loaded */

static void inverse_of_M(double Minv[Q][Q]) {
    /* Rows of M are mutually orthogonal, so M^-1 = M^T diag(1/|row_k|^2). */
    for (int k = 0; k < Q; ++k) {
        double n2 = 0.0;
        for (int a = 0; a < Q; ++a) n2 += MM[k][a] * MM[k][a];
        for (int a = 0; a < Q; ++a) Minv[a][k] = MM[k][a] / n2;
    }
}

__attribute__((constructor)) static void orc_load(void) { inverse_of_M(MINV); }

void orc_lattice(int* cx, int* cy, int* opp, double* w, double* M, double* Minv) {
    double mi[Q][Q];
    inverse_of_M(mi);
    for (int a = 0; a < Q; ++a) {
        cx[a] = CX[a];
        cy[a] = CY[a];
        w[a] = WGT[a];
        int o = 0;
        for (int b = 0; b < Q; ++b)
            if (CX[b] == -CX[a] && CY[b] == -CY[a]) o = b;
        opp[a] = o;
        for (int b = 0; b < Q; ++b) {
            M[a * Q + b] = MM[a][b];
            Minv[a * Q + b] = mi[a][b];
        }
    }
}

/* Second-order equilibrium, Eq. (11). */
void orc_feq(double rho, double ux, double uy, double* feq) {
    for (int a = 0; a < Q; ++a) {
        double cu = CX[a] * ux + CY[a] * uy;
        /* u u : (c c - cs2 I) = (c.u)^2 - cs2 |u|^2 */
        double uu = cu * cu - CS2 * (ux * ux + uy * uy);
        feq[a] = WGT[a] * rho * (1.0 + cu / CS2 + uu / (2.0 * CS2 * CS2));
    }
}

/* Guo forcing vector without its (1 - 1/2tau) prefactor (that role is taken by
 * (I - S/2) in Eq. (8)):  Fhat_a = w_a [ (c_a - u)/cs2 + (c_a.u) c_a / cs2^2 ] . G,
 * G being the force density rho*F (Eq. (12)). */
void orc_guo(double ux, double uy, double Gx, double Gy, double* fhat) {
    for (int a = 0; a < Q; ++a) {
        double cu = CX[a] * ux + CY[a] * uy;
        double ex = (CX[a] - ux) / CS2 + cu * CX[a] / (CS2 * CS2);
        double ey = (CY[a] - uy) / CS2 + cu * CY[a] / (CS2 * CS2);
        fhat[a] = WGT[a] * (ex * Gx + ey * Gy);
    }
}

/* Characteristic function of the disc (Eq. (2)) and the solid velocity at node (i, j). */
void orc_chi(const orc_params* p, const orc_body* b, int i, int j, double* chi, double* usx,
             double* usy) {
    *chi = 0.0;
    *usx = 0.0;
    *usy = 0.0;
    if (!p->has_body) return;
    double dx = (double)i - b->q[0];
    double dy = (double)j - b->q[1];
    double d2 = dx * dx + dy * dy;
    double R = p->radius;
    if (p->smooth_delta <= 0.0) {
        *chi = (d2 <= R * R) ? 1.0 : 0.0;
    } else {
        double z = (sqrt(d2) - R) / p->smooth_delta;
        if (z > 20.0)
            *chi = 0.0;
        else if (z < -20.0)
            *chi = 1.0;
        else
            *chi = 1.0 / (1.0 + exp(2.0 * z));
    }
    if (p->chi_add) *chi += p->chi_add[(size_t)j * (size_t)p->nx + (size_t)i];
    /* rigid motion: u_s = V + Omega e_z x (x - x_G) */
    *usx = b->v[0] - b->v[2] * dy;
    *usy = b->v[1] + b->v[2] * dx;
}

/* One node: macroscopic quantities with the implicit penalized velocity, then the
 * MRT collision with the forcing source.  P = populations after streaming.
 * Outputs the post-collision populations, rho, u, the force density G on the fluid
 * and the penalization force on the body (rho chi/eta (u - u_s)).               */
void orc_node(const orc_params* p, const double* P, double chi, double usx, double usy,
              double* out, double* rho_o, double* ux_o, double* uy_o, double* G_o, double* dF_o) {
    /* Eq. (19): density and lattice momentum */
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < Q; ++a) {
        rho += P[a];
        jx += CX[a] * P[a];
        jy += CY[a] * P[a];
    }
    /* Eq. (22), with the half-step fluid body force of Eq. (19) kept alongside:
     * rho (1 + lam/2) u = j + rho g_f/2 + rho lam u_s / 2.  Solved for r = u - u_s. */
    double lam = chi / p->eta;
    double gx = p->g_fluid[0], gy = p->g_fluid[1];
    double rx = (jx + 0.5 * rho * gx - rho * usx) / (rho * (1.0 + 0.5 * lam));
    double ry = (jy + 0.5 * rho * gy - rho * usy) / (rho * (1.0 + 0.5 * lam));
    double ux = usx + rx, uy = usy + ry;
    /* force density on the fluid: rho (g_f - chi/eta (u - u_s)), Eq. (1) */
    double Gx = rho * gx - rho * lam * rx;
    double Gy = rho * gy - rho * lam * ry;

    /* Eq. (9): moments */
    double m[Q];
    for (int k = 0; k < Q; ++k) {
        m[k] = 0.0;
        for (int a = 0; a < Q; ++a) m[k] += MM[k][a] * P[a];
    }
    /* Eq. (14): equilibrium moments */
    double usq = ux * ux + uy * uy;
    double meq[Q] = {rho,       rho * (-2.0 + 3.0 * usq), rho * (1.0 - 3.0 * usq),
                     rho * ux,  -rho * ux,                rho * uy,
                     -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy};
    /* forcing in moment space: M Fhat */
    double fhat[Q], mF[Q];
    orc_guo(ux, uy, Gx, Gy, fhat);
    for (int k = 0; k < Q; ++k) {
        mF[k] = 0.0;
        for (int a = 0; a < Q; ++a) mF[k] += MM[k][a] * fhat[a];
    }
    /* Eqs. (8)/(17): m* = m - S (m - meq) + (I - S/2) M F  (source sign of Eq. (8)) */
    double ms[Q];
    for (int k = 0; k < Q; ++k)
        ms[k] = m[k] - p->s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * p->s[k]) * mF[k];
    /* back to populations */
    for (int a = 0; a < Q; ++a) {
        out[a] = 0.0;
        for (int k = 0; k < Q; ++k) out[a] += MINV[a][k] * ms[k];
    }
    if (rho_o) *rho_o = rho;
    if (ux_o) *ux_o = ux;
    if (uy_o) *uy_o = uy;
    if (G_o) {
        G_o[0] = Gx;
        G_o[1] = Gy;
    }
    if (dF_o) {
        dF_o[0] = rho * lam * rx;
        dF_o[1] = rho * lam * ry;
    }
}

/* ---- momentum-exchange force (Sec. 2.3, Eqs. (25)-(27)) ------------------------ */
static int opposite(int a);

/* A node is solid when it lies in the closed disc, d^2 <= R^2 (the sharp indicator of
 * Eq. (2); the same classification is used when chi is smoothed). */
static int solid_node(const orc_params* p, const orc_body* b, int i, int j) {
    double dx = (double)i - b->q[0];
    double dy = (double)j - b->q[1];
    return dx * dx + dy * dy <= p->radius * p->radius;
}

/* Point x_Gamma where the link from fluid node (fi, fj) along c_a (towards a solid
 * node) crosses the circle: x_f + q c_a with |x_f + q c_a - x_G| = R, the root of
 * |c_a|^2 q^2 + 2 (c_a . d) q + |d|^2 - R^2 = 0 (d = x_f - x_G) nearest x_f. */
void orc_link_point(const orc_params* p, const orc_body* b, int fi, int fj, int a, double* xg,
                    double* yg) {
    double dx = (double)fi - b->q[0];
    double dy = (double)fj - b->q[1];
    double A = (double)(CX[a] * CX[a] + CY[a] * CY[a]);
    double Bh = CX[a] * dx + CY[a] * dy;
    double Cc = dx * dx + dy * dy - p->radius * p->radius;
    double q = (-Bh - sqrt(Bh * Bh - A * Cc)) / A;
    *xg = (double)fi + q * CX[a];
    *yg = (double)fj + q * CY[a];
}

/* Contribution of node (i, j), with post-collision populations out[], to the
 * momentum-exchange force F[0..1] and torque F[2] on the body.  A link joins a fluid
 * node x_f to the solid node x_s = x_f + e_alpha; on it the force of Eq. (25) is
 * (e_alpha - u_Gamma) f~_alpha(x_f) - (e_alphabar - u_Gamma) f~_alphabar(x_s), with
 * u_Gamma the rigid-body velocity at x_Gamma; Eq. (27) takes its moment about x_G.
 * Each end of a link adds its own term: the fluid node the first, the solid node the
 * second (its population along the link, back towards x_f). */
void orc_mem_node(const orc_params* p, const orc_body* b, int i, int j, const double* out,
                  double* F) {
    F[0] = F[1] = F[2] = 0.0;
    if (!p->has_body) return;
    int self_solid = solid_node(p, b, i, j);
    for (int a = 1; a < Q; ++a) {
        int ni = i + CX[a], nj = j + CY[a];
        if (solid_node(p, b, ni, nj) == self_solid) continue;
        double xg, yg, sgn;
        if (!self_solid) { /* this node is x_f, e_alpha = c_a */
            orc_link_point(p, b, i, j, a, &xg, &yg);
            sgn = 1.0;
        } else { /* this node is x_s; x_f = (ni, nj), e_alpha = -c_a, alphabar = a */
            orc_link_point(p, b, ni, nj, opposite(a), &xg, &yg);
            sgn = -1.0;
        }
        double rgx = xg - b->q[0], rgy = yg - b->q[1];
        double ugx = b->v[0] - b->v[2] * rgy;
        double ugy = b->v[1] + b->v[2] * rgx;
        double fx = sgn * (CX[a] - ugx) * out[a];
        double fy = sgn * (CY[a] - ugy) * out[a];
        F[0] += fx;
        F[1] += fy;
        F[2] += rgx * fy - rgy * fx;
    }
}

/* ---- streaming with boundary rules (Eq. (18) as a pull; Sec. 3.1 boundaries) ---- */
static int flip_x(int a) {
    for (int b = 0; b < Q; ++b)
        if (CX[b] == -CX[a] && CY[b] == CY[a]) return b;
    return a;
}
static int flip_y(int a) {
    for (int b = 0; b < Q; ++b)
        if (CX[b] == CX[a] && CY[b] == -CY[a]) return b;
    return a;
}
static int opposite(int a) {
    for (int b = 0; b < Q; ++b)
        if (CX[b] == -CX[a] && CY[b] == -CY[a]) return b;
    return a;
}

#define FAT(f, a, i, j) (f)[((size_t)(a) * ny + (size_t)(j)) * nx + (size_t)(i)]

/* Value pulled by node (i, j) for direction a from the post-collision field f.
 * outlet: convective-outflow memory (3 x ny, directions 3, 6, 7), may be NULL
 * when no side is OUTFLOW. */
static double pull(const orc_params* p, const double* f, const double* outlet, int a, int i,
                   int j) {
    const int nx = p->nx, ny = p->ny;
    int si = i - CX[a];
    int sj = j - CY[a];
    int dir = a; /* direction of the population that is read */
    if (si < 0 || si >= nx) {
        int side = (si < 0) ? SIDE_W : SIDE_E;
        switch (p->bc[side]) {
            case BC_PERIODIC:
                si = (si + nx) % nx;
                break;
            case BC_WALL:
                return FAT(f, opposite(a), i, j);
            case BC_VELOCITY: {
                double cu = CX[a] * p->u_wall[side][0] + CY[a] * p->u_wall[side][1];
                return FAT(f, opposite(a), i, j) + 2.0 * WGT[a] * 1.0 * cu / CS2;
            }
            case BC_SYMMETRY:
                dir = flip_x(a);
                si = i;
                break;
            case BC_OUTFLOW: {
                /* implicit first-order discretisation of df/dt + U_c df/dx = 0 */
                int k = (a == 3) ? 0 : (a == 6) ? 1 : 2;
                double qv = pull(p, f, outlet, a, nx - 2, j);
                double uc = p->u_conv;
                return (outlet[(size_t)k * ny + j] + uc * qv) / (1.0 + uc);
            }
        }
    }
    if (sj < 0 || sj >= ny) {
        int side = (sj < 0) ? SIDE_S : SIDE_N;
        switch (p->bc[side]) {
            case BC_PERIODIC:
                sj = (sj + ny) % ny;
                break;
            case BC_WALL:
                return FAT(f, opposite(a), i, j);
            case BC_VELOCITY: {
                double cu = CX[a] * p->u_wall[side][0] + CY[a] * p->u_wall[side][1];
                return FAT(f, opposite(a), i, j) + 2.0 * WGT[a] * 1.0 * cu / CS2;
            }
            case BC_SYMMETRY:
                dir = flip_y(dir);
                sj = j;
                break;
            default: /* OUTFLOW is only accepted on the east side */
                return NAN;
        }
    }
    return FAT(f, dir, si, sj);
}

/* ---- rigid body (Sec. 2.3) ---------------------------------------------------- */
/* Classical RK4 with unit step for  M q'' + c q' + k (q - q0) = F  (F frozen). */
void orc_rk4(double Mq, double cq, double kq, double q0, double F, double* q, double* v) {
    double x = *q, u = *v;
#define ACC(X, U) ((F - cq * (U) - kq * ((X) - q0)) / Mq)
    double k1x = u, k1v = ACC(x, u);
    double k2x = u + 0.5 * k1v, k2v = ACC(x + 0.5 * k1x, u + 0.5 * k1v);
    double k3x = u + 0.5 * k2v, k3v = ACC(x + 0.5 * k2x, u + 0.5 * k2v);
    double k4x = u + k3v, k4v = ACC(x + k3x, u + k3v);
#undef ACC
    *q = x + (k1x + 2.0 * k2x + 2.0 * k3x + k4x) / 6.0;
    *v = u + (k1v + 2.0 * k2v + 2.0 * k3v + k4v) / 6.0;
}

static const double TWO_PI = 6.283185307179586476925286766559;

/* Pose for the imposed motion y = y0 + A sin(2 pi f t + phi); phi = pi/2 gives the
 * cosine law of Eq. (29) with y0 = y_G(0) - A. */
static void imposed_pose(const orc_params* p, orc_body* b) {
    double ph = TWO_PI * p->imp_freq * (double)b->t_body + p->imp_phase;
    b->q[1] = p->imp_y0 + p->imp_amp * sin(ph);
    b->v[1] = TWO_PI * p->imp_freq * p->imp_amp * cos(ph);
}

void orc_body_init(const orc_params* p, orc_body* b, const double* q, const double* v) {
    for (int d = 0; d < 3; ++d) {
        b->q[d] = q[d];
        b->v[d] = v[d];
        b->pin_prev[d] = 0.0;
    }
    b->t_body = 0;
    b->pin_valid = 0;
    if (p->mode == MODE_IMPOSED_SIN) imposed_pose(p, b);
}

/* Advance the body by one step given the hydrodynamic force/torque of this step. */
void orc_body_advance(const orc_params* p, orc_body* b, const double* F) {
    b->t_body += 1;
    switch (p->mode) {
        case MODE_FIXED:
            break;
        case MODE_IMPOSED_SIN:
            imposed_pose(p, b);
            break;
        case MODE_CONST_VEL:
            for (int d = 0; d < 3; ++d) b->q[d] += b->v[d];
            break;
        case MODE_FREE:
            for (int d = 0; d < 3; ++d) {
                if (!(p->free_mask & (1u << d))) continue;
                double Mq = (d < 2) ? p->mass : p->inertia;
                orc_rk4(Mq, p->c[d], p->k[d], p->q0[d], F[d] + p->f_ext[d], &b->q[d], &b->v[d]);
            }
            break;
    }
}

/* ---- one full time step --------------------------------------------------------- */
/* fin: post-collision populations of the previous step, [9][ny][nx].
 * fout: post-collision populations of this step.  outlet: 3 x ny memory of the
 * convective outflow (updated in place).  b: body state (advanced in place).
 * rec: record of this step.  step: step index written into the record.
 * Returns 0, or 1 when a non-positive or non-finite density was met.             */
int orc_step(const orc_params* p, const double* fin, double* fout, double* outlet, orc_body* b,
             orc_record* rec, int64_t step) {
    const int nx = p->nx, ny = p->ny;
    double* rows = (double*)calloc((size_t)ny * 12, sizeof(double));
    double* new_out = (double*)calloc((size_t)3 * ny, sizeof(double));
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int j = 0; j < ny; ++j) {
        double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int i = 0; i < nx; ++i) {
            double P[Q], out[Q], rho, ux, uy, G[2], dF[2], chi, usx, usy, Fm[3];
            double jx = 0.0, jy = 0.0;
            for (int a = 0; a < Q; ++a) P[a] = pull(p, fin, outlet, a, i, j);
            for (int a = 0; a < Q; ++a) {
                jx += CX[a] * P[a];
                jy += CY[a] * P[a];
            }
            if (i == nx - 1 && p->bc[SIDE_E] == BC_OUTFLOW) {
                new_out[0 * (size_t)ny + j] = P[3];
                new_out[1 * (size_t)ny + j] = P[6];
                new_out[2 * (size_t)ny + j] = P[7];
            }
            orc_chi(p, b, i, j, &chi, &usx, &usy);
            orc_node(p, P, chi, usx, usy, out, &rho, &ux, &uy, G, dF);
            if (!(rho > 0.0) || !isfinite(rho) || !isfinite(ux) || !isfinite(uy)) bad = 1;
            for (int a = 0; a < Q; ++a) FAT(fout, a, i, j) = out[a];
            double rx = (double)i - b->q[0], ry = (double)j - b->q[1];
            acc[0] += dF[0];
            acc[1] += dF[1];
            acc[2] += rx * dF[1] - ry * dF[0];
            /* momentum inside the body after collision (j + G) and before it (j) */
            double px = jx + G[0], py = jy + G[1];
            acc[3] += chi * px;
            acc[4] += chi * py;
            acc[5] += chi * (rx * py - ry * px);
            acc[6] += chi * jx;
            acc[7] += chi * jy;
            acc[8] += chi * (rx * jy - ry * jx);
            orc_mem_node(p, b, i, j, out, Fm);
            acc[9] += Fm[0];
            acc[10] += Fm[1];
            acc[11] += Fm[2];
            (void)ux;
            (void)uy;
        }
        for (int k = 0; k < 12; ++k) rows[(size_t)j * 12 + k] = acc[k];
    }
    double tot[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = 0; j < ny; ++j)
        for (int k = 0; k < 12; ++k) tot[k] += rows[(size_t)j * 12 + k];
    if (p->bc[SIDE_E] == BC_OUTFLOW) memcpy(outlet, new_out, sizeof(double) * 3 * (size_t)ny);
    free(rows);
    free(new_out);

    orc_record r;
    r.step = step;
    r.fvp[0] = tot[0];
    r.fvp[1] = tot[1];
    r.tvp = tot[2];
    r.pin[0] = tot[3];
    r.pin[1] = tot[4];
    r.pin[2] = tot[5];
    /* Internal-fluid correction: F_h = F_vp + (P_in(n) - P_in(n-1)) with P_in the
     * post-collision momentum inside the body.  For a sharp indicator this equals the
     * momentum carried across the interface by streaming, i.e. the momentum-exchange
     * force (Sec. 2.3, Eqs. (25)-(27)).  On the first step after the body is set,
     * P_in(n-1) is taken as the momentum that streamed into the body (sum chi j). */
    double dp[3] = {0, 0, 0};
    if (p->internal_mass_correction)
        for (int d = 0; d < 3; ++d)
            dp[d] = r.pin[d] - (b->pin_valid ? b->pin_prev[d] : tot[6 + d]);
    r.fh[0] = r.fvp[0] + dp[0];
    r.fh[1] = r.fvp[1] + dp[1];
    r.th = r.tvp + dp[2];
    for (int d = 0; d < 3; ++d) {
        r.q[d] = b->q[d];
        r.v[d] = b->v[d];
        b->pin_prev[d] = r.pin[d];
    }
    r.fmem[0] = tot[9];
    r.fmem[1] = tot[10];
    r.tmem = tot[11];
    b->pin_valid = 1;
    if (rec) *rec = r;
    double F[3] = {r.fh[0], r.fh[1], r.th};
    if (p->force_model == FORCE_MEM) {
        F[0] = r.fmem[0];
        F[1] = r.fmem[1];
        F[2] = r.tmem;
    }
    if (p->has_body) orc_body_advance(p, b, F);
    return bad;
}

/* Run n steps, ping-ponging between fa (holds the state on entry and on exit) and a
 * scratch buffer.  recs (may be NULL) receives n records. */
int orc_run(const orc_params* p, double* fa, double* outlet, orc_body* b, orc_record* recs,
            int64_t step0, int64_t n) {
    size_t cnt = (size_t)Q * p->nx * p->ny;
    double* fb = (double*)malloc(cnt * sizeof(double));
    int bad = 0;
    for (int64_t s = 0; s < n; ++s) {
        bad |= orc_step(p, fa, fb, outlet, b, recs ? &recs[s] : NULL, step0 + s);
        memcpy(fa, fb, cnt * sizeof(double));
    }
    free(fb);
    return bad;
}

/* Initial state: f = f^eq(rho, u) everywhere; outlet memory likewise. */
void orc_init(const orc_params* p, double* f, double* outlet, double rho, double ux, double uy) {
    const int nx = p->nx, ny = p->ny;
    double feq[Q];
    orc_feq(rho, ux, uy, feq);
    for (int a = 0; a < Q; ++a)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) FAT(f, a, i, j) = feq[a];
    if (outlet) {
        for (int j = 0; j < ny; ++j) {
            outlet[0 * (size_t)ny + j] = feq[3];
            outlet[1 * (size_t)ny + j] = feq[6];
            outlet[2 * (size_t)ny + j] = feq[7];
        }
    }
}

/* Density and penalized velocity (Eq. (22)) of the state held in f, with the body
 * at its current pose: stream (pull) and evaluate, without colliding. */
void orc_fields(const orc_params* p, const double* f, const double* outlet, const orc_body* b,
                double* rho_o, double* ux_o, double* uy_o) {
    const int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double P[Q], out[Q], rho, ux, uy, chi, usx, usy;
            for (int a = 0; a < Q; ++a) P[a] = pull(p, f, outlet, a, i, j);
            orc_chi(p, b, i, j, &chi, &usx, &usy);
            orc_node(p, P, chi, usx, usy, out, &rho, &ux, &uy, NULL, NULL);
            size_t o = (size_t)j * nx + i;
            rho_o[o] = rho;
            ux_o[o] = ux;
            uy_o[o] = uy;
        }
}

/* Populations after streaming at one node (exposed for boundary-rule tests). */
void orc_pull_node(const orc_params* p, const double* f, const double* outlet, int i, int j,
                   double* P) {
    for (int a = 0; a < Q; ++a) P[a] = pull(p, f, outlet, a, i, j);
}

void orc_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}
int orc_max_threads(void) { return omp_get_max_threads(); }

int orc_sizeof_params(void) { return (int)sizeof(orc_params); }
int orc_sizeof_body(void) { return (int)sizeof(orc_body); }
int orc_sizeof_record(void) { return (int)sizeof(orc_record); }
