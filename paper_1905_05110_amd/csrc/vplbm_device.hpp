// vplbm_device.hpp -- device-side data structures and per-node arithmetic of the
// VP-LBM time step for gfx950 (MI355X).
//
// Populations are held as offsets g = f - w_a from the rest-state weights in every
// storage precision; the moment transform below works on the offsets directly,
// using M w = (1, -2, 1, 0, ..., 0) (the equilibrium moments of rho = 1, u = 0).
// Method: Liberge & Beghein (arXiv 1905.05110), Sec. 2.1-2.3 and Algorithm 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vplbm {

constexpr int NQ = 9;
constexpr int TILE_X = 256;  // nodes of one row handled by a workgroup (one per lane)
constexpr int NWAVE = TILE_X / 64;

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_VELOCITY = 2, BC_SYMMETRY = 3, BC_OUTFLOW = 4 };
enum { MODE_FIXED = 0, MODE_IMPOSED_SIN = 1, MODE_FREE = 2, MODE_CONST_VEL = 3 };

// ---- D2Q9 directions (Sec. 2.2, Eq. (10)): 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW,
// 7 SW, 8 SE.  Written as arithmetic so that run-time indices need no table.
__host__ __device__ __forceinline__ int dir_cx(int a) {
    return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0);
}
__host__ __device__ __forceinline__ int dir_cy(int a) {
    return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0);
}
__host__ __device__ __forceinline__ int dir_opp(int a) {
    return a == 0 ? 0 : (a <= 4 ? ((a + 1) & 3) + 1 : ((a - 3) & 3) + 5);
}
// reflection that flips the x component (specular plane x = const)
__host__ __device__ __forceinline__ int dir_flip_x(int a) {
    switch (a) {
        case 1: return 3;
        case 3: return 1;
        case 5: return 6;
        case 6: return 5;
        case 7: return 8;
        case 8: return 7;
        default: return a;
    }
}
// reflection that flips the y component (specular plane y = const)
__host__ __device__ __forceinline__ int dir_flip_y(int a) {
    switch (a) {
        case 2: return 4;
        case 4: return 2;
        case 5: return 8;
        case 8: return 5;
        case 6: return 7;
        case 7: return 6;
        default: return a;
    }
}

// ---- device-resident state --------------------------------------------------------
struct BodyDev {
    // constants of the disc and its motion law
    int active, mode;
    unsigned free_mask;
    int imc;  // internal-fluid momentum correction for FREE bodies
    int smooth, pad0;
    double R, R2, delta, reach;
    double mass, inertia;
    double k[3], c[3], q0[3], fext[3];
    double amp, freq, y0;
    // state, double-buffered by step parity: step n reads [n & 1], writes [(n + 1) & 1]
    double q[2][3], v[2][3];
    long long t_body;  // steps since the body was set
    long long step;    // index of the next step
    double pin_prev[3];
    int pin_valid, pad1;
};

struct Record {  // same layout as lbm_force_rec
    long long step;
    double fvp[2], tvp, pin[3], fh[2], th, q[3], v[3];
};

struct SimDesc {
    void* pop[2];        // two population buffers, 9 planes of ps elements each
    void* outlet;        // 3 x ny offsets (directions 3, 6, 7) of the outflow memory
    BodyDev* body;
    double* partials;    // 6 FP64 sums per participating workgroup
    unsigned* counter;   // arrival counter of the participating workgroups
    Record* hist;        // ring of per-step records
    int* flag;           // set to 1 when an unstable node is met
    long long ps;        // plane stride (elements)
    int nx, ny, pitch, tiles_x, tiles_y, hist_cap;
    int bc[4];
    double s_e, s_eps, s_q, s_nu;
    double inv_eta;
    double gx, gy;
    double u_conv;
    double bbc[4][NQ];   // moving-wall increments 6 w_a (c_a . u_wall) per side
    float scale, inv_scale;  // storage scale of 16-bit offsets
};

// ---- storage codecs -----------------------------------------------------------------
struct bf16s {
    uint16_t bits;
};

template <class S>
struct Codec;

template <>
struct Codec<double> {
    using T = double;
    static __device__ __forceinline__ T load(const double* p, long long i, float) { return p[i]; }
    static __device__ __forceinline__ void store(double* p, long long i, T v, float) {
        __builtin_nontemporal_store(v, p + i);
    }
};

template <>
struct Codec<float> {
    using T = float;
    static __device__ __forceinline__ T load(const float* p, long long i, float) { return p[i]; }
    static __device__ __forceinline__ void store(float* p, long long i, T v, float) {
        __builtin_nontemporal_store(v, p + i);
    }
};

template <>
struct Codec<_Float16> {
    using T = float;
    // stored value: round-to-nearest-even of g * 2^k
    static __device__ __forceinline__ T load(const _Float16* p, long long i, float inv_scale) {
        return (float)p[i] * inv_scale;
    }
    static __device__ __forceinline__ void store(_Float16* p, long long i, T v, float scale) {
        __builtin_nontemporal_store((_Float16)(v * scale), p + i);
    }
};

__host__ __device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <>
struct Codec<bf16s> {
    using T = float;
    static __device__ __forceinline__ T load(const bf16s* p, long long i, float inv_scale) {
        const uint16_t b = reinterpret_cast<const uint16_t*>(p)[i];
        return __builtin_bit_cast(float, (uint32_t)b << 16) * inv_scale;
    }
    static __device__ __forceinline__ void store(bf16s* p, long long i, T v, float scale) {
        __builtin_nontemporal_store(f32_to_bf16_rne(v * scale), reinterpret_cast<uint16_t*>(p) + i);
    }
};

// ---- streaming with boundary rules (Eq. (18) applied as a pull) -----------------------
// Value pulled by node (i, j) for direction a.  Returns false when the source crosses
// an OUTFLOW side (the caller then applies the convective rule).
template <class S>
__device__ bool pull_rules(const SimDesc& d, const S* __restrict__ fin, int a, int i, int j,
                           typename Codec<S>::T& out) {
    using T = typename Codec<S>::T;
    int dir = a;
    int si = i - dir_cx(a);
    int sj = j - dir_cy(a);
    if (si < 0 || si >= d.nx) {
        const int side = si < 0 ? 0 : 1;
        const int kind = d.bc[side];
        if (kind == BC_PERIODIC) {
            si += (si < 0) ? d.nx : -d.nx;
        } else if (kind == BC_SYMMETRY) {
            dir = dir_flip_x(a);
            si = i;
        } else if (kind == BC_OUTFLOW) {
            return false;
        } else {  // WALL or VELOCITY: half-way bounce-back of the population leaving (i, j)
            T v = Codec<S>::load(fin, (long long)dir_opp(a) * d.ps + (long long)j * d.pitch + i,
                                 d.inv_scale);
            if (kind == BC_VELOCITY) v += (T)d.bbc[side][a];
            out = v;
            return true;
        }
    }
    if (sj < 0 || sj >= d.ny) {
        const int side = sj < 0 ? 2 : 3;
        const int kind = d.bc[side];
        if (kind == BC_PERIODIC) {
            sj += (sj < 0) ? d.ny : -d.ny;
        } else if (kind == BC_SYMMETRY) {
            dir = dir_flip_y(dir);
            sj = j;
        } else {
            T v = Codec<S>::load(fin, (long long)dir_opp(a) * d.ps + (long long)j * d.pitch + i,
                                 d.inv_scale);
            if (kind == BC_VELOCITY) v += (T)d.bbc[side][a];
            out = v;
            return true;
        }
    }
    out = Codec<S>::load(fin, (long long)dir * d.ps + (long long)sj * d.pitch + si, d.inv_scale);
    return true;
}

// Index of a direction in the 3-slot outflow memory (directions 3, 6, 7).
__device__ __forceinline__ int outflow_slot(int a) { return a == 3 ? 0 : (a == 6 ? 1 : 2); }

// All nine pulled offsets of node (i, j).  The interior fast path reads the nine
// shifted planes directly; nodes on the domain edge go through the boundary rules.
// When update_outlet is set, the east column stores its pulled values 3, 6, 7 as the
// outflow memory of the next step.
template <class S>
__device__ __forceinline__ void pull_node(const SimDesc& d, const S* __restrict__ fin, int i, int j,
                                          typename Codec<S>::T g[NQ], bool update_outlet) {
    using T = typename Codec<S>::T;
    const long long ps = d.ps;
    const int pitch = d.pitch;
    if (i >= 1 && i <= d.nx - 2 && j >= 1 && j <= d.ny - 2) {
        const S* b = fin + (long long)j * pitch + i;
        const float is = d.inv_scale;
        g[0] = Codec<S>::load(b, 0, is);
        g[1] = Codec<S>::load(b, 1 * ps - 1, is);
        g[2] = Codec<S>::load(b, 2 * ps - pitch, is);
        g[3] = Codec<S>::load(b, 3 * ps + 1, is);
        g[4] = Codec<S>::load(b, 4 * ps + pitch, is);
        g[5] = Codec<S>::load(b, 5 * ps - pitch - 1, is);
        g[6] = Codec<S>::load(b, 6 * ps - pitch + 1, is);
        g[7] = Codec<S>::load(b, 7 * ps + pitch + 1, is);
        g[8] = Codec<S>::load(b, 8 * ps + pitch - 1, is);
        return;
    }
    T* outlet = reinterpret_cast<T*>(d.outlet);
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
        T v;
        if (!pull_rules<S>(d, fin, a, i, j, v)) {
            // convective outflow: implicit upwind step of df/dt + U_c df/dx = 0 using
            // last step's value at the east column and this step's value one node in
            T qv;
            pull_rules<S>(d, fin, a, d.nx - 2, j, qv);
            const T uc = (T)d.u_conv;
            v = (outlet[outflow_slot(a) * d.ny + j] + uc * qv) / (T(1) + uc);
        }
        g[a] = v;
    }
    if (update_outlet && i == d.nx - 1 && d.bc[1] == BC_OUTFLOW) {
        outlet[0 * d.ny + j] = g[3];
        outlet[1 * d.ny + j] = g[6];
        outlet[2 * d.ny + j] = g[7];
    }
}

// ---- indicator function of the disc (Sec. 2.1, Eq. (2)) and rigid velocity ---------
// The sharp test d^2 <= R^2 is evaluated without contraction so that nodes lying on
// the circle are classified identically on every platform.
__device__ __forceinline__ double disc_d2(double dx, double dy) {
#pragma clang fp contract(off)
    const double a = dx * dx;
    const double b = dy * dy;
    return a + b;
}

__device__ __forceinline__ double disc_chi(const BodyDev& B, double d2) {
    if (!B.smooth) return d2 <= B.R2 ? 1.0 : 0.0;
    const double z = (sqrt(d2) - B.R) / B.delta;
    if (z > 20.0) return 0.0;
    if (z < -20.0) return 1.0;
    return 1.0 / (1.0 + exp(2.0 * z));
}

// Tile range (inclusive) of the workgroups whose rows/columns meet the support of the
// body; all its nodes with chi > 0 lie inside.  An absent or out-of-domain body maps
// to tile (0, 0) alone, so that exactly one workgroup finalises every step.
__device__ __forceinline__ void body_tiles(const SimDesc& d, const BodyDev& B, double X, double Y,
                                           int& tx0, int& tx1, int& ty0, int& ty1) {
    tx0 = tx1 = ty0 = ty1 = 0;
    if (!B.active) return;
    const double xl = fmax(floor(X - B.reach) - 1.0, 0.0);
    const double xh = fmin(ceil(X + B.reach) + 1.0, (double)(d.nx - 1));
    const double yl = fmax(floor(Y - B.reach) - 1.0, 0.0);
    const double yh = fmin(ceil(Y + B.reach) + 1.0, (double)(d.ny - 1));
    if (!(xl <= xh) || !(yl <= yh)) return;
    tx0 = (int)xl / TILE_X;
    tx1 = (int)xh / TILE_X;
    ty0 = (int)yl;
    ty1 = (int)yh;
}

// ---- macroscopic quantities, penalized velocity and MRT collision ------------------
template <class T>
struct NodeOut {
    T rho, ux, uy, dFx, dFy;
};

// Density, momentum and the implicit penalized velocity (Sec. 2.2, Eqs. (19)-(22)):
//   rho (1 + lam/2) u = j + rho g/2 + rho lam u_s / 2,   lam = chi / eta,
// solved for r = u - u_s; the fluid receives G = rho g - rho lam r and the body
// rho lam r.
template <class T>
__device__ __forceinline__ void macros(const SimDesc& d, const T g[NQ], T chi, T usx, T usy,
                                       T& drho, T& jx, T& jy, NodeOut<T>& o, T& Gx, T& Gy) {
    const T s1234 = (g[1] + g[2]) + (g[3] + g[4]);
    const T s5678 = (g[5] + g[6]) + (g[7] + g[8]);
    drho = g[0] + s1234 + s5678;
    jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    jy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const T rho = T(1) + drho;
    const T lam = chi * (T)d.inv_eta;
    const T gx = (T)d.gx, gy = (T)d.gy;
    const T inv = T(1) / (rho * (T(1) + T(0.5) * lam));
    const T rx = (jx + T(0.5) * rho * gx - rho * usx) * inv;
    const T ry = (jy + T(0.5) * rho * gy - rho * usy) * inv;
    o.rho = rho;
    o.ux = usx + rx;
    o.uy = usy + ry;
    o.dFx = rho * lam * rx;
    o.dFy = rho * lam * ry;
    Gx = rho * gx - o.dFx;
    Gy = rho * gy - o.dFy;
}

// Collision in moment space with the forcing source (Eqs. (8), (14), (16), (17); the
// source enters with the sign of Eq. (8)):  m* = m - S (m - m_eq) + (I - S/2) M F,
// F the Guo forcing vector of Eq. (12) without its (1 - 1/2tau) factor, whose moments
// are (0, 6 u.G, -6 u.G, Gx, -Gx, Gy, -Gy, 2(ux Gx - uy Gy), ux Gy + uy Gx).
// The conserved moments come out as rho, j + G whatever their rates.
template <class T>
__device__ __forceinline__ void collide(const SimDesc& d, const T g[NQ], T chi, T usx, T usy,
                                        T out[NQ], NodeOut<T>& o) {
    T drho, jx, jy, Gx, Gy;
    macros<T>(d, g, chi, usx, usy, drho, jx, jy, o, Gx, Gy);
    const T s1234 = (g[1] + g[2]) + (g[3] + g[4]);
    const T s5678 = (g[5] + g[6]) + (g[7] + g[8]);
    // non-conserved moments of the offsets (M g)
    const T e = T(2) * s5678 - T(4) * g[0] - s1234;
    const T ep = T(4) * g[0] - T(2) * s1234 + s5678;
    const T dxs = (g[5] - g[6]) + (g[8] - g[7]);
    const T dys = (g[5] + g[6]) - (g[7] + g[8]);
    const T qx = dxs - T(2) * (g[1] - g[3]);
    const T qy = dys - T(2) * (g[2] - g[4]);
    const T pxx = (g[1] + g[3]) - (g[2] + g[4]);
    const T pxy = (g[5] + g[7]) - (g[6] + g[8]);

    const T rho = o.rho, ux = o.ux, uy = o.uy;
    const T usq = ux * ux + uy * uy;
    // equilibria of the offsets (m_eq - M w)
    const T e_eq = T(3) * rho * usq - T(2) * drho;
    const T ep_eq = drho - T(3) * rho * usq;
    const T qx_eq = -rho * ux;
    const T qy_eq = -rho * uy;
    const T pxx_eq = rho * (ux * ux - uy * uy);
    const T pxy_eq = rho * ux * uy;
    const T uG = ux * Gx + uy * Gy;

    const T se = (T)d.s_e, sp = (T)d.s_eps, sq = (T)d.s_q, sn = (T)d.s_nu;
    const T e_s = e - se * (e - e_eq) + (T(1) - T(0.5) * se) * (T(6) * uG);
    const T ep_s = ep - sp * (ep - ep_eq) - (T(1) - T(0.5) * sp) * (T(6) * uG);
    const T qx_s = qx - sq * (qx - qx_eq) - (T(1) - T(0.5) * sq) * Gx;
    const T qy_s = qy - sq * (qy - qy_eq) - (T(1) - T(0.5) * sq) * Gy;
    const T pxx_s = pxx - sn * (pxx - pxx_eq) + (T(1) - T(0.5) * sn) * (T(2) * (ux * Gx - uy * Gy));
    const T pxy_s = pxy - sn * (pxy - pxy_eq) + (T(1) - T(0.5) * sn) * (ux * Gy + uy * Gx);
    const T jx_s = jx + Gx;
    const T jy_s = jy + Gy;

    // f = M^-1 m*, M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    const T a0 = drho * T(1.0 / 9.0);
    const T a1 = e_s * T(1.0 / 36.0);
    const T a2 = ep_s * T(1.0 / 36.0);
    const T a3 = jx_s * T(1.0 / 6.0);
    const T a4 = qx_s * T(1.0 / 12.0);
    const T a5 = jy_s * T(1.0 / 6.0);
    const T a6 = qy_s * T(1.0 / 12.0);
    const T a7 = pxx_s * T(0.25);
    const T a8 = pxy_s * T(0.25);
    const T b = a0 - a1 - T(2) * a2;
    const T c = a0 + T(2) * a1 + a2;
    const T x1 = a3 - T(2) * a4, y1 = a5 - T(2) * a6;
    const T x2 = a3 + a4, y2 = a5 + a6;
    out[0] = a0 - T(4) * a1 + T(4) * a2;
    out[1] = b + x1 + a7;
    out[2] = b + y1 - a7;
    out[3] = b - x1 + a7;
    out[4] = b - y1 - a7;
    out[5] = c + x2 + y2 + a8;
    out[6] = c - x2 + y2 - a8;
    out[7] = c - x2 - y2 + a8;
    out[8] = c + x2 - y2 - a8;
}

// ---- rigid body (Sec. 2.3, Eqs. (23)-(24); RK4 of Algorithm 1) -----------------------
// One classical RK4 step of unit length for M q'' + c q' + k (q - q0) = F, F frozen.
__device__ __forceinline__ void rk4_dof(double Mq, double cq, double kq, double q0, double F,
                                        double& q, double& v) {
    auto acc = [&](double x, double u) { return (F - cq * u - kq * (x - q0)) / Mq; };
    const double x = q, u = v;
    const double k1x = u, k1v = acc(x, u);
    const double k2x = u + 0.5 * k1v, k2v = acc(x + 0.5 * k1x, u + 0.5 * k1v);
    const double k3x = u + 0.5 * k2v, k3v = acc(x + 0.5 * k2x, u + 0.5 * k2v);
    const double k4x = u + k3v, k4v = acc(x + k3x, u + k3v);
    q = x + (k1x + 2.0 * k2x + 2.0 * k3x + k4x) / 6.0;
    v = u + (k1v + 2.0 * k2v + 2.0 * k3v + k4v) / 6.0;
}

// Finalise one step: record it and advance the body (reads [p], writes [p ^ 1]).
// tot = (F_vp x, y, T_vp, P_in x, y, theta).
__device__ inline void body_advance(const SimDesc& d, int p, const double tot[6]) {
    BodyDev& B = *d.body;
    Record r;
    r.step = B.step;
    r.fvp[0] = tot[0];
    r.fvp[1] = tot[1];
    r.tvp = tot[2];
    r.pin[0] = tot[3];
    r.pin[1] = tot[4];
    r.pin[2] = tot[5];
    double dp[3] = {0.0, 0.0, 0.0};
    if (B.imc && B.pin_valid)
        for (int k = 0; k < 3; ++k) dp[k] = tot[3 + k] - B.pin_prev[k];
    r.fh[0] = tot[0] + dp[0];
    r.fh[1] = tot[1] + dp[1];
    r.th = tot[2] + dp[2];
    double q[3], v[3];
    for (int k = 0; k < 3; ++k) {
        q[k] = B.q[p][k];
        v[k] = B.v[p][k];
        r.q[k] = q[k];
        r.v[k] = v[k];
    }
    d.hist[B.step % d.hist_cap] = r;
    B.t_body += 1;
    if (B.active) {
        if (B.mode == MODE_IMPOSED_SIN) {
            const double w = 6.283185307179586476925286766559 * B.freq;
            const double ph = w * (double)B.t_body;
            q[1] = B.y0 + B.amp * sin(ph);
            v[1] = w * B.amp * cos(ph);
        } else if (B.mode == MODE_CONST_VEL) {
            for (int k = 0; k < 3; ++k) q[k] += v[k];
        } else if (B.mode == MODE_FREE) {
            const double F[3] = {r.fh[0], r.fh[1], r.th};
            for (int k = 0; k < 3; ++k) {
                if (!(B.free_mask & (1u << k))) continue;
                rk4_dof(k < 2 ? B.mass : B.inertia, B.c[k], B.k[k], B.q0[k], F[k] + B.fext[k],
                        q[k], v[k]);
            }
        }
    }
    for (int k = 0; k < 3; ++k) {
        B.q[p ^ 1][k] = q[k];
        B.v[p ^ 1][k] = v[k];
        B.pin_prev[k] = tot[3 + k];
    }
    B.pin_valid = 1;
    B.step += 1;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// XCD-aware placement: the hardware hands workgroup b to XCD b mod 8; renumber so
// that each XCD receives one contiguous band of tiles (rows), keeping neighbouring
// rows in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int xcd = b & 7, local = b >> 3;
    const int base = n >> 3, rem = n & 7;
    return xcd < rem ? xcd * (base + 1) + local : rem * (base + 1) + (xcd - rem) * base + local;
}

// ---- one tile of one step ------------------------------------------------------------
// Pull, penalize, collide and store a row segment of TILE_X nodes; workgroups that
// meet the body reduce force, torque and internal momentum in FP64 into their slot;
// the last of them to arrive sums the slots in fixed order and advances the body.
template <class S>
__device__ __forceinline__ void step_tile(const SimDesc& d, int tile, int p) {
    using T = typename Codec<S>::T;
    __shared__ double red[NWAVE][6];
    __shared__ int last;
    const S* __restrict__ fin = reinterpret_cast<const S*>(d.pop[p]);
    S* __restrict__ fout = reinterpret_cast<S*>(d.pop[p ^ 1]);
    const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
    const int i = tx * TILE_X + (int)threadIdx.x;
    const int j = ty;
    const bool valid = i < d.nx;
    const BodyDev& B = *d.body;
    const double X = B.q[p][0], Y = B.q[p][1];
    int bx0, bx1, by0, by1;
    body_tiles(d, B, X, Y, bx0, bx1, by0, by1);
    const bool part = tx >= bx0 && tx <= bx1 && ty >= by0 && ty <= by1;

    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (valid) {
        T g[NQ], out[NQ];
        pull_node<S>(d, fin, i, j, g, true);
        double chi = 0.0, usx = 0.0, usy = 0.0, rx = 0.0, ry = 0.0;
        if (part && B.active) {
            rx = (double)i - X;
            ry = (double)j - Y;
            chi = disc_chi(B, disc_d2(rx, ry));
            const double om = B.v[p][2];
            usx = B.v[p][0] - om * ry;
            usy = B.v[p][1] + om * rx;
        }
        NodeOut<T> o;
        collide<T>(d, g, (T)chi, (T)usx, (T)usy, out, o);
        const long long base = (long long)j * d.pitch + i;
#pragma unroll
        for (int a = 0; a < NQ; ++a) Codec<S>::store(fout, a * d.ps + base, out[a], d.scale);
        if (!(o.rho > T(0)) || !__builtin_isfinite(o.ux) || !__builtin_isfinite(o.uy))
            atomicOr(d.flag, 1);
        if (part) {
            const double dFx = (double)o.dFx, dFy = (double)o.dFy;
            const double rho = (double)o.rho, ux = (double)o.ux, uy = (double)o.uy;
            acc[0] = dFx;
            acc[1] = dFy;
            acc[2] = rx * dFy - ry * dFx;
            acc[3] = chi * rho * ux;
            acc[4] = chi * rho * uy;
            acc[5] = chi * rho * (rx * uy - ry * ux);
        }
    }
    if (!part) return;  // uniform over the workgroup

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = s;
    }
    __syncthreads();
    const int nbx = bx1 - bx0 + 1;
    const int nb = nbx * (by1 - by0 + 1);
    if (threadIdx.x == 0) {
        const int slot = (ty - by0) * nbx + (tx - bx0);
        for (int k = 0; k < 6; ++k) {
            double s = red[0][k];
            for (int w = 1; w < NWAVE; ++w) s += red[w][k];
            d.partials[(long long)slot * 6 + k] = s;
        }
        __threadfence();
        const unsigned prev = atomicAdd(d.counter, 1u);
        last = (prev == (unsigned)(nb - 1));
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double t[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = threadIdx.x; s < nb; s += TILE_X)
        for (int k = 0; k < 6; ++k) t[k] += d.partials[(long long)s * 6 + k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double s = wave_sum(t[k]);
        if (lane == 0) red[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[6];
        for (int k = 0; k < 6; ++k) {
            double s = red[0][k];
            for (int w = 1; w < NWAVE; ++w) s += red[w][k];
            tot[k] = s;
        }
        body_advance(d, p, tot);
        atomicExch(d.counter, 0u);
    }
}

}  // namespace vplbm
