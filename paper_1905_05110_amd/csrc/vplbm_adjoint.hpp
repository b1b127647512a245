// vplbm_adjoint.hpp -- reverse-mode (adjoint) step of the VP-LBM scheme for gfx950.
//
// Objective: J = sum_{n<N} (w_x F_x(n) + w_y F_y(n)), F(n) the penalization force on a
// body held at a fixed pose with a rigid velocity field u_s = V + Omega e_z x (x - X)
// (Sec. 2.1, the force as the volume integral of the penalization term).  The step
// (Sec. 2.2: pull streaming with boundary rules, Eq. (18); implicit penalized velocity
// and force density, Eqs. (19)-(22); MRT collision with the Guo source, Eqs. (8),
// (12)-(17)) is written P^n = A(f^n, O^n), f^{n+1} = C(P^n), O^{n+1} = E P^n with A the
// linear pull (O the convective-outflow memory), C the node-wise collision and E the
// east-column selection.  The adjoint recursion runs on the pulled populations:
//
//   Pbar^n = (dC/dP)^T [A_f^T Pbar^{n+1}] + dJ_n/dP^n + E^T A_O^T Pbar^{n+1},
//
// with Pbar^N = 0.  A_f^T is a gather: away from the domain edge, population b of node
// y is read by node y + c_b alone, so (A_f^T Pbar)_b(y) = Pbar_b(y + c_b); nodes on the
// edge use a table of their readers built on the host from the boundary rules.  The
// outflow memory contributes Pbar_a(east, j) / (1 + U_c) for a in {3, 6, 7}.  Each
// adjoint step re-pulls P^n from the stored state f^n (recomputed segment by segment
// from checkpoints) and differentiates C by hand:
//
//   forward   rho, j = M rows 0, 3, 5 of P;  lam = chi/eta;  r = (j + rho g/2 - rho u_s)
//             / (rho (1 + lam/2));  u = u_s + r;  G = rho g - rho lam r;  dF = rho lam r
//             m* = m - S (m - m_eq(rho, u)) + (I - S/2) m_F(u, G), conserved exact
//   reverse   mbar* = M^-T fbar, then through the relaxation, m_eq, m_F, G, dF (seeded
//             with w), r, u back to rho, j, lam and u_s;  Pbar = M^T (rhobar, (1 - s_k)
//             mbar*_k, jbar ...)
//
// and accumulates dJ/dchi = lambar / eta per node and the u_s adjoint per tile (for
// dJ/dV, dJ/dOmega and the u_s part of dJ/dX).
#pragma once

#include <hip/hip_runtime.h>

#include "vplbm_device.hpp"

namespace vplbm {

// One reader of an edge population: w_b(y) += coef * Pbar_a(i, j).
struct RingEntry {
    int i, j, a, pad;
    double coef;
};

// One reader of an edge population in the transposed pull, as the kernel reads it: the
// element index (a * ps + j * pitch + i) of the reader's adjoint value and the
// weight of the read.  Unused slots have weight 0 and index 0.
struct RingSlot {
    long long idx;
    double coef;
};

struct AdjDesc {
    char* seg_pop;          // K + 1 population buffers of a segment, seg_stride bytes apart
    long long seg_stride;
    char* seg_out;          // K + 1 outflow memories (3 x ny values), out_stride bytes apart
    long long out_stride;
    const char* ckpt_pop;   // one checkpoint per segment (state at the segment start)
    const char* ckpt_out;
    void* abar[2];          // Pbar of the two parities, 9 planes of ps values
    double* chibar;         // dJ/dchi accumulated over the steps, FP64 [ny][fpitch]
    double* tile_acc;       // per tile of the adjoint grid: u_s adjoint sums (x, y, angular)
    const RingSlot* ring;   // ring_k readers per (edge node, direction)
    const int* ring_kn;     // per edge node: the slots it visits (its longest list)
    int* seg_index;         // segment being reversed (device counter for graph replays)
    double pose[6];         // X, Y, theta, Vx, Vy, Omega
    double wx, wy;          // objective weights
    int box[4];             // adjoint tiles (x range, rows) that may hold chi > 0
    int nbox[4];            // nodes (i0, i1, j0, j1) where d(chi)/d(X, Y) may be non-zero
    long long pop_bytes, out_bytes;
    int tiles_x, ring_k;
};

// Index of an edge node in the ring (bottom row, top row, left column, right column).
__host__ __device__ __forceinline__ int ring_index(int nx, int ny, int i, int j) {
    if (j == 0) return i;
    if (j == ny - 1) return nx + i;
    if (i == 0) return 2 * nx + (j - 1);
    if (i == nx - 1) return 2 * nx + (ny - 2) + (j - 1);
    return -1;
}

__host__ __device__ __forceinline__ int ring_count(int nx, int ny) { return 2 * nx + 2 * (ny - 2); }

// The adjoint of one step for node (i, j) of adjoint tile (blockIdx.x, row blockIdx.y).
template <class S>
__device__ __forceinline__ void adjoint_node(const SimDesc& d, const AdjDesc& a, int iseg) {
    using T = S;
    const Consts<T>& c = consts_of<T>(d);
    const int i = (int)blockIdx.x * TILE_X + (int)threadIdx.x;
    const int j = (int)blockIdx.y;
    const int nx = d.nx, ny = d.ny;
    const DiscParams B = disc_params(d.body);  // ahead of the population loads
    const long long ps = d.ps;
    const T* __restrict__ Ain = reinterpret_cast<const T*>(a.abar[(iseg + 1) & 1]);
    T* __restrict__ Aout = reinterpret_cast<T*>(a.abar[iseg & 1]);
    const void* fin = a.seg_pop + (long long)iseg * a.seg_stride;
    const void* outk = a.seg_out + (long long)iseg * a.out_stride;
    double usum[3] = {0.0, 0.0, 0.0};
    const bool in_box = (int)blockIdx.x >= a.box[0] && (int)blockIdx.x <= a.box[1] &&
                        (int)blockIdx.y >= a.box[2] && (int)blockIdx.y <= a.box[3];

    if (i < nx) {
        // 1. the pulled populations of this step (offsets from f_ref)
        T g[NQ];
        const bool inner = i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2;
        if (__all(inner)) {  // one pull path per wave (the boundary-rule pull handles all)
            const char* P[NQ];
#pragma unroll
            for (int b = 0; b < NQ; ++b) P[b] = plane<S>(d, fin, b);
            // 32-bit offsets: the adjoint refuses grids whose direction arrays reach 4 GiB
            pull_interior<S>(P, (unsigned)node_off<S>(d, i, j), (unsigned)d.pitch * (unsigned)sizeof(S),
                             1.0f, g);
        } else {
            pull_edge<S>(d, fin, outk, i, j, g, false);
        }
        // 2. indicator and rigid velocity at this node
        const double rxg = (double)i - a.pose[0], ryg = (double)j - a.pose[1];
        const double chi = B.active ? disc_chi(B, disc_d2(rxg, ryg)) + chi_add_at(B, i, j) : 0.0;
        const double usx_d = a.pose[3] - a.pose[5] * ryg;
        const double usy_d = a.pose[4] + a.pose[5] * rxg;
        const T usx = (T)usx_d, usy = (T)usy_d;
        // 3. adjoint of the post-collision populations: transpose of the next pull (issued
        // before the arithmetic below, so that both sets of loads are in flight together)
        T w[NQ];
        const unsigned row = (unsigned)d.pitch;
        const unsigned o0 = (unsigned)j * row + (unsigned)i;
        // dJ/dchi adds one term per step over the N steps: accumulated in FP64 whatever
        // the storage, so that the sum carries no rounding beyond its terms' (the pose
        // gradient takes it against d(chi)/dX, where front and back nearly cancel)
        double* chib = a.chibar + ((long long)j * d.fpitch + i);
        const double chib_old = gld(chib);
        if (inner) {
#pragma unroll
            for (int b = 0; b < NQ; ++b)
                w[b] = gld(Ain + (long long)b * ps + (o0 + (unsigned)(dir_cy(b) * (int)row + dir_cx(b))));
        } else {
            // an edge node: the readers of its populations through the boundary rules, ring_k
            // table slots per direction; slot k of the nine directions is read at once, then
            // the nine adjoint values it names (two rounds of loads per slot, not two per
            // reader one after another)
            const int r = ring_index(nx, ny, i, j);
            const int K = a.ring_k;
            const RingSlot* rs = a.ring + (long long)r * NQ * K;
            // slots beyond the node's longest list hold weight 0 and are not visited (the
            // count is read with the first slot; every list has at least one slot)
            const int kn = gld(a.ring_kn + r);
#pragma unroll
            for (int b = 0; b < NQ; ++b) w[b] = T(0);
            for (int k = 0; k < K; ++k) {
                if (k > 0 && k >= kn) break;
                long long ix[NQ];
                T cf[NQ];
#pragma unroll
                for (int b = 0; b < NQ; ++b) {
                    ix[b] = gld(&rs[b * K + k].idx);
                    cf[b] = (T)gld(&rs[b * K + k].coef);
                }
#pragma unroll
                for (int b = 0; b < NQ; ++b) w[b] += cf[b] * gld(Ain + ix[b]);
            }
        }
        // 4. forward node quantities
        NodeOut<T> o;
        macros<T, true>(c, g, (T)chi, (T)(usx_d - d.u0x), (T)(usy_d - d.u0y), o);
        const T rho = o.rho, ux = o.ux, uy = o.uy, Gx = o.Gx, Gy = o.Gy;
        const T rx = o.dux - (T)(usx_d - d.u0x), ry = o.duy - (T)(usy_d - d.u0y);
        const T lam = (T)chi * c.inv_eta;
        // 5. reverse of the collision.  mbar* = M^-T w = diag(1/|row|^2) M w; the rows of
        // the conserved moments divide as the forward step does (correctly rounded, see
        // div_small), so that the sweep is the transpose of the step it reverses rather
        // than one with a constant relative bias repeated over the N steps
        const T s1234 = (w[1] + w[2]) + (w[3] + w[4]);
        const T s5678 = (w[5] + w[6]) + (w[7] + w[8]);
        const T dx5 = (w[5] - w[6]) + (w[8] - w[7]);
        const T dy5 = (w[5] + w[6]) - (w[7] + w[8]);
        const T ms0 = div_small(w[0] + s1234 + s5678, T(9), T(1.0 / 9.0));
        const T ms1 = (T(2) * s5678 - T(4) * w[0] - s1234) * T(1.0 / 36.0);
        const T ms2 = (T(4) * w[0] - T(2) * s1234 + s5678) * T(1.0 / 36.0);
        const T ms3 = div_small((w[1] - w[3]) + dx5, T(6), T(1.0 / 6.0));
        const T ms4 = (dx5 - T(2) * (w[1] - w[3])) * T(1.0 / 12.0);
        const T ms5 = div_small((w[2] - w[4]) + dy5, T(6), T(1.0 / 6.0));
        const T ms6 = (dy5 - T(2) * (w[2] - w[4])) * T(1.0 / 12.0);
        const T ms7 = ((w[1] + w[3]) - (w[2] + w[4])) * T(0.25);
        const T ms8 = ((w[5] + w[7]) - (w[6] + w[8])) * T(0.25);
        // relaxation: m* = (1 - s) m + s m_eq + (1 - s/2) m_F for the non-conserved moments
        const T v1 = (T(1) - c.s_e) * ms1, v2 = (T(1) - c.s_eps) * ms2;
        const T v4 = (T(1) - c.s_q) * ms4, v6 = (T(1) - c.s_q) * ms6;
        const T v7 = (T(1) - c.s_nu) * ms7, v8 = (T(1) - c.s_nu) * ms8;
        const T E1 = c.s_e * ms1, E2 = c.s_eps * ms2, E4 = c.s_q * ms4, E6 = c.s_q * ms6;
        const T E7 = c.s_nu * ms7, E8 = c.s_nu * ms8;
        // m_F = (., 6 u.G, -6 u.G, ., -Gx, ., -Gy, 2 (ux Gx - uy Gy), ux Gy + uy Gx)
        const T A6 = T(6) * (c.h_e * ms1 - c.h_eps * ms2);
        const T B7 = T(2) * c.h_nu * ms7, C8 = c.h_nu * ms8;
        // conserved moments: m*_0 = rho, m*_3,5 = j + G
        T rhob = ms0, jbx = ms3, jby = ms5;
        T Gbx = ms3 + (A6 + B7) * ux + C8 * uy - c.h_q * ms4;
        T Gby = ms5 + (A6 - B7) * uy + C8 * ux - c.h_q * ms6;
        T ubx = (A6 + B7) * Gx + C8 * Gy;
        T uby = (A6 - B7) * Gy + C8 * Gx;
        // m_eq = (rho, rho(-2 + 3|u|^2), rho(1 - 3|u|^2), ., -rho ux, ., -rho uy,
        //         rho (ux^2 - uy^2), rho ux uy)
        const T usq = ux * ux + uy * uy;
        rhob += E1 * (T(3) * usq - T(2)) + E2 * (T(1) - T(3) * usq) - E4 * ux - E6 * uy +
                E7 * (ux * ux - uy * uy) + E8 * (ux * uy);
        const T K3 = T(6) * rho * (E1 - E2);  // 2 x 3 rho (E1 - E2): d|u|^2/du = 2u
        ubx += K3 * ux + rho * (T(2) * E7 * ux + E8 * uy - E4);
        uby += K3 * uy + rho * (E8 * ux - T(2) * E7 * uy - E6);
        // dF = rho lam r (seeded with w) and G = rho g - rho lam r
        const T fx = (T)a.wx - Gbx, fy = (T)a.wy - Gby;
        const T fr = fx * rx + fy * ry;
        rhob += lam * fr + Gbx * c.gx + Gby * c.gy;
        T lamb = rho * fr;
        const T rbx = rho * lam * fx + ubx, rby = rho * lam * fy + uby;
        T usbx = ubx, usby = uby;  // u = u_s + r
        // r = N / D with N = j + rho g/2 - rho u_s and D = rho (1 + lam/2)
        const T half = T(1) + T(0.5) * lam;
        const T inv = T(1) / (rho * half);
        const T Nbx = rbx * inv, Nby = rby * inv;
        const T Db = -(rbx * rx + rby * ry) * inv;
        jbx += Nbx;
        jby += Nby;
        rhob += Nbx * (T(0.5) * c.gx - usx) + Nby * (T(0.5) * c.gy - usy) + Db * half;
        usbx -= rho * Nbx;
        usby -= rho * Nby;
        lamb += Db * rho * T(0.5);
        // Pbar = M^T (rhob, v1, v2, jbx, v4, jby, v6, v7, v8)
        T pb[NQ];
        const T bb = rhob - v1 - T(2) * v2;
        const T cc = rhob + T(2) * v1 + v2;
        const T x1 = jbx - T(2) * v4, y1 = jby - T(2) * v6;
        const T x2 = jbx + v4, y2 = jby + v6;
        pb[0] = rhob - T(4) * v1 + T(4) * v2;
        pb[1] = bb + x1 + v7;
        pb[2] = bb + y1 - v7;
        pb[3] = bb - x1 + v7;
        pb[4] = bb - y1 - v7;
        pb[5] = cc + x2 + y2 + v8;
        pb[6] = cc - x2 + y2 - v8;
        pb[7] = cc - x2 - y2 + v8;
        pb[8] = cc + x2 - y2 - v8;
        // 6. the outflow memory carries the east column's 3, 6, 7 into the next step
        if (i == nx - 1 && d.bc[1] == BC_OUTFLOW) {
            pb[3] += c.inv1uc * gld(Ain + 3 * ps + o0);
            pb[6] += c.inv1uc * gld(Ain + 6 * ps + o0);
            pb[7] += c.inv1uc * gld(Ain + 7 * ps + o0);
        }
#pragma unroll
        for (int b = 0; b < NQ; ++b) gst(Aout + (long long)b * ps + o0, pb[b]);
        gst(chib, chib_old + (double)(lamb * c.inv_eta));
        if (chi != 0.0) {  // where chi = 0 the step does not depend on u_s
            usum[0] = (double)usbx;
            usum[1] = (double)usby;
            usum[2] = (double)usby * rxg - (double)usbx * ryg;
        }
    }
    if (!in_box) return;  // uniform over the workgroup
    __shared__ double red[NWAVE][3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = wave_sum(usum[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int q = 1; q < NWAVE; ++q) v += red[q][k];
        double* slot = a.tile_acc + ((long long)blockIdx.y * a.tiles_x + blockIdx.x) * 3;
        slot[k] += v;
    }
}

// d(chi)/d(X, Y) at node (i, j) for the pose (X, Y): chi = 1 / (1 + exp(2 z)),
// z = (d - R)/delta, so dchi/dX = 2 chi (1 - chi) (i - X) / (delta d); zero where the
// indicator is clamped (|z| > 20), at d = 0 and for the sharp indicator.
__device__ __forceinline__ void chi_pose_derivative(const BodyDev& B, double rx, double ry,
                                                    double& dX, double& dY) {
    dX = dY = 0.0;
    if (!B.active || !B.smooth) return;
    const double d2 = disc_d2(rx, ry);
    if (!(d2 > 0.0)) return;
    const double dd = sqrt(d2);
    const double z = (dd - B.R) / B.delta;
    if (z > 20.0 || z < -20.0) return;
    const double chi = 1.0 / (1.0 + exp(2.0 * z));
    const double k = 2.0 * chi * (1.0 - chi) / (B.delta * dd);
    dX = k * rx;
    dY = k * ry;
}

}  // namespace vplbm

namespace vplbm {

template <class S>
__global__ __launch_bounds__(TILE_X) void k_adjoint(const SimDesc* __restrict__ dp,
                                                    const AdjDesc* __restrict__ ap, int iseg) {
    adjoint_node<S>(*dp, *ap, iseg);
}

// Segment bookkeeping kernels (defined once, in the adjoint host translation unit):
// copy the checkpoint of segment *seg_index into the first slot of the segment store;
// move the counter to the previous segment; clear n 4-byte words.
__global__ void k_adj_load_segment(const AdjDesc* __restrict__ ap);
__global__ void k_adj_next_segment(const AdjDesc* __restrict__ ap);
__global__ void k_adj_zero(int* __restrict__ p, long long n);

// Fixed-order FP64 reduction (one workgroup): out = (dJ/dX, dJ/dY, dJ/dVx, dJ/dVy,
// dJ/dOmega) from dJ/dchi and the per-tile u_s adjoint sums.
template <class S>
__global__ __launch_bounds__(TILE_X) void k_adj_reduce(const SimDesc* __restrict__ dp,
                                                       const AdjDesc* __restrict__ ap,
                                                       double* __restrict__ out) {
    const SimDesc& d = *dp;
    const AdjDesc& a = *ap;
    const BodyDev& B = *d.body;
    const double* chib = a.chibar;
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int bw = a.nbox[1] - a.nbox[0] + 1, bh = a.nbox[3] - a.nbox[2] + 1;
    const long long nb = (bw > 0 && bh > 0) ? (long long)bw * bh : 0;
    for (long long k = threadIdx.x; k < nb; k += TILE_X) {
        const int i = a.nbox[0] + (int)(k % bw), j = a.nbox[2] + (int)(k / bw);
        double dX, dY;
        chi_pose_derivative(B, (double)i - a.pose[0], (double)j - a.pose[1], dX, dY);
        const double cb = chib[(long long)j * d.fpitch + i];
        t[0] += cb * dX;
        t[1] += cb * dY;
    }
    const long long ntile = (long long)a.tiles_x * d.ny;
    for (long long k = threadIdx.x; k < ntile; k += TILE_X)
        for (int q = 0; q < 3; ++q) t[2 + q] += a.tile_acc[k * 3 + q];
    __shared__ double red[NWAVE][5];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = 0; q < 5; ++q) {
        const double v = wave_sum(t[q]);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[5];
        for (int q = 0; q < 5; ++q) {
            s[q] = red[0][q];
            for (int w = 1; w < NWAVE; ++w) s[q] += red[w][q];
        }
        const double om = a.pose[5];
        // u_s = (Vx - Omega (y - Y), Vy + Omega (x - X))
        out[0] = s[0] - om * s[3];
        out[1] = s[1] + om * s[2];
        out[2] = s[2];
        out[3] = s[3];
        out[4] = s[4];
    }
}

// dJ/dchi as FP64 [ny][nx].
template <class S>
__global__ void k_adj_export(const SimDesc* __restrict__ dp, const AdjDesc* __restrict__ ap,
                             double* __restrict__ out) {
    const SimDesc& d = *dp;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    out[(long long)j * d.nx + i] =
        ap->chibar[(long long)j * d.fpitch + i];
}

// Launch interface, instantiated for S = double and float in adj_<storage>.hip.
template <class S>
struct AdjLaunch {
    static void step(const SimDesc* dd, const AdjDesc* ad, dim3 grid, int iseg, hipStream_t st);
    static void reduce(const SimDesc* dd, const AdjDesc* ad, double* out, hipStream_t st);
    static void export_chi(const SimDesc* dd, const AdjDesc* ad, double* out, dim3 grid,
                           hipStream_t st);
};

#define VPLBM_DEFINE_ADJ_LAUNCH(S)                                                           \
    template <>                                                                              \
    void AdjLaunch<S>::step(const SimDesc* dd, const AdjDesc* ad, dim3 grid, int iseg,       \
                            hipStream_t st) {                                                \
        hipLaunchKernelGGL(k_adjoint<S>, grid, dim3(TILE_X), 0, st, dd, ad, iseg);           \
    }                                                                                        \
    template <>                                                                              \
    void AdjLaunch<S>::reduce(const SimDesc* dd, const AdjDesc* ad, double* out,             \
                              hipStream_t st) {                                              \
        hipLaunchKernelGGL(k_adj_reduce<S>, dim3(1), dim3(TILE_X), 0, st, dd, ad, out);      \
    }                                                                                        \
    template <>                                                                              \
    void AdjLaunch<S>::export_chi(const SimDesc* dd, const AdjDesc* ad, double* out,         \
                                  dim3 grid, hipStream_t st) {                               \
        hipLaunchKernelGGL(k_adj_export<S>, grid, dim3(TILE_X), 0, st, dd, ad, out);         \
    }

}  // namespace vplbm
