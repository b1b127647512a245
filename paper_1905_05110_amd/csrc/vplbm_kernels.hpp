// vplbm_kernels.hpp -- kernel templates of the VP-LBM library and the launch interface
// between the host runtime (vplbm.hip) and the per-storage translation units
// (kern_<storage>.hip), which are compiled separately and in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "vplbm_device.hpp"

namespace vplbm {

// Launch entry points, one instantiation per storage type S (double, float,
// _Float16, bf16s), each defined in its own translation unit.
template <class S>
struct Launch {
    // the kernel of one time step (parity p; rows per lane 1, 2 or 4; nt selects
    // nontemporal stores; tile_w columns per tile, TILE_NARROW, TILE_X or TILE_WIDE;
    // grid from step_grid; tile rows dispatched from row_shift on, 0 <= row_shift <
    // tiles_y; the partial force slots in sa.slots when that is set, else in the
    // simulation's own array)
    static void step(const SimDesc* dd, dim3 grid, int rows, bool nt, int tile_w, int p,
                     hipStream_t st, int row_shift = 0, SlotArray sa = SlotArray{nullptr, 0});
    // one time step of several simulations in one launch: workgroup b handles the tile
    // sched[b] = (simulation, by << 16 | bx) of descs[simulation]
    static void step_batch(const SimDesc* descs, const int2* sched, int nsched, int rows, bool nt,
                           int tile_w, int p, hipStream_t st);
    static void fill(const SimDesc& d, const double g[NQ], int buf, hipStream_t st);
    static void set_pop(const SimDesc& d, const double* f, int buf, hipStream_t st);
    static void get_pop(const SimDesc& d, double* f, int buf, hipStream_t st);
    static void fields(const SimDesc& d, double* out, int p, hipStream_t st);
};

// ---------------------------------------------------------------------------------
// Grid of the step kernel for a single simulation.  Tiles of TILE_X or TILE_WIDE
// columns: tiles_x x tiles_y workgroups.  TILE_NARROW tiles: 8 tiles_x x ceil(tiles_y / 8)
// workgroups, see k_step.
inline dim3 step_grid(const SimDesc& d) {
    if (d.tile_w == TILE_NARROW) return dim3(8 * d.tiles_x, (d.tiles_y + 7) / 8);
    return dim3(d.tiles_x, d.tiles_y);
}

// One kernel serves a single simulation (sched == nullptr) and a batch (1D grid over
// sched, whose order the host chooses; an entry with a negative simulation index is a
// gap and does nothing).  The tile body has a single call site, so a simulation computes
// bitwise the same inside a batch as alone.  Consecutive workgroups go to the eight XCDs
// in turn.  A single simulation with wide tiles (2D grid of its tiles) takes tile row
// (blockIdx.y + row_shift) mod tiles_y and tile column (blockIdx.x + blockIdx.y) mod
// tiles_x: skewing the column by the row spreads each column, and so the longer work of
// the body's tiles, over all XCDs instead of one or two.  With narrow tiles, XCD x walks
// the tile rows x, x + 8, x + 16, ... (before the rotation by row_shift), each from left
// to right: horizontally adjacent tiles, which share the cache lines their x-shifted
// pulls straddle, run one after the other on one XCD, and every XCD meets the body's
// rows.
// Single-row tiles of 4-byte or narrower storage fit in 64 registers without spilling:
// eight waves per SIMD then hide more memory latency.
template <class S, int ROWS>
constexpr int step_waves() { return (sizeof(S) <= 4 && ROWS == 1) ? 8 : 1; }

template <class S, int ROWS, bool NT, int TW>
__global__ __launch_bounds__(tile_lanes(TW)) __attribute__((amdgpu_waves_per_eu(step_waves<S, ROWS>())))
void k_step(const SimDesc* __restrict__ descs,
                                                 const int2* __restrict__ sched, int p,
                                                 int row_shift, SlotArray sa) {
    const SimDesc* d;
    int tx, ty;
    if (sched) {  // entry: (simulation, ty << 16 | tx)
        const int2 e = sched[blockIdx.x];
        if (e.x < 0) return;  // a gap (uniform)
        d = descs + e.x;
        tx = e.y & 0xffff;
        ty = e.y >> 16;
    } else if constexpr (TW == TILE_NARROW) {
        d = descs;
        const int tiles_y = d->tiles_y;
        const int x = (int)(blockIdx.x & 7);
        tx = (int)(blockIdx.x >> 3);
        ty = (int)blockIdx.y * 8 + x;
        if (ty >= tiles_y) return;  // beyond the last tile row (uniform)
        ty += row_shift;
        if (ty >= tiles_y) ty -= tiles_y;
    } else {
        d = descs;
        const int gx = (int)gridDim.x;
        const int t = (int)blockIdx.x + (int)(blockIdx.y % gridDim.x);
        tx = t >= gx ? t - gx : t;
        ty = (int)blockIdx.y + row_shift;
        if (ty >= (int)gridDim.y) ty -= (int)gridDim.y;
    }
    step_tile<S, ROWS, NT, TW>(*d, tx, ty, p, sa);
}

__global__ __launch_bounds__(TILE_X) void k_finalize(const SimDesc* __restrict__ dp, int p,
                                                     SlotArray sa);
// the same for several simulations: workgroup b finalizes descs[members[b]]
__global__ __launch_bounds__(TILE_X) void k_finalize_batch(const SimDesc* __restrict__ descs,
                                                           const int* __restrict__ members, int p);

struct Offsets9 {
    double g[NQ];
};

// Fill one buffer's planes with constant offsets (initial equilibrium).
template <class S>
__global__ void k_fill(SimDesc d, Offsets9 go, int buf) {
    using T = typename Codec<S>::T;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const double* g = go.g;
    const long long off = node_off<S>(d, i, j);
    for (int a = 0; a < NQ; ++a)
        Codec<S>::template store<false>(const_cast<char*>(plane<S>(d, d.pop[buf], a)) + off, 0u,
                                        (T)g[a], d.scale);
}

// Host FP64 populations f [9][ny][nx] <-> stored offsets.
template <class S>
__global__ void k_set_pop(SimDesc d, const double* __restrict__ f, int buf) {
    using T = typename Codec<S>::T;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const long long plane_n = (long long)d.nx * d.ny;
    const long long off = node_off<S>(d, i, j);
    for (int a = 0; a < NQ; ++a) {
        const double v = f[a * plane_n + (long long)j * d.nx + i] - d.fref[a];
        Codec<S>::template store<false>(const_cast<char*>(plane<S>(d, d.pop[buf], a)) + off, 0u,
                                        (T)v, d.scale);
    }
}

template <class S>
__global__ void k_get_pop(SimDesc d, double* __restrict__ f, int buf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const long long plane_n = (long long)d.nx * d.ny;
    const long long off = node_off<S>(d, i, j);
    for (int a = 0; a < NQ; ++a)
        f[a * plane_n + (long long)j * d.nx + i] =
            (double)Codec<S>::load(plane<S>(d, d.pop[buf], a) + off, 0u, d.inv_scale) + d.fref[a];
}

// Density and penalized velocity of the current state, body at its current pose.
template <class S>
__global__ void k_fields(SimDesc d, double* __restrict__ out, int p) {
    using T = typename Codec<S>::T;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    T g[NQ];
    pull_edge<S>(d, d.pop[p], d.outlet, i, j, g, false);
    const BodyDev& B = *d.body;
    const BodyState& st = B.st[p];  // final: the host flushes before reading fields
    double chi = 0.0, dsx = 0.0, dsy = 0.0;
    if (B.active) {
        const double rx = (double)i - st.q[0], ry = (double)j - st.q[1];
        chi = disc_chi(B, disc_d2(rx, ry)) + chi_add_at(B, i, j);
        if (chi != 0.0) {
            dsx = (st.v[0] - st.v[2] * ry) - d.u0x;
            dsy = (st.v[1] + st.v[2] * rx) - d.u0y;
        }
    }
    NodeOut<T> o;
    macros<T>(consts_of<T>(d), g, (T)chi, (T)dsx, (T)dsy, o);
    const long long plane_n = (long long)d.nx * d.ny, o_ = (long long)j * d.nx + i;
    out[o_] = (double)o.rho;
    out[plane_n + o_] = d.u0x + (double)o.dux;
    out[2 * plane_n + o_] = d.u0y + (double)o.duy;
}


inline dim3 grid_rows(const SimDesc& d) { return dim3((d.nx + 255) / 256, d.ny); }

template <class S, bool NT, int TW>
static void launch_step_tw(const SimDesc* dd, const int2* sched, dim3 grid, int rows, int p,
                           hipStream_t st, int row_shift, SlotArray sa) {
    switch (rows) {
        case 1: hipLaunchKernelGGL((k_step<S, 1, NT, TW>), grid, dim3(tile_lanes(TW)), 0, st, dd, sched, p, row_shift, sa); break;
        case 2: hipLaunchKernelGGL((k_step<S, 2, NT, TW>), grid, dim3(tile_lanes(TW)), 0, st, dd, sched, p, row_shift, sa); break;
        default: hipLaunchKernelGGL((k_step<S, 4, NT, TW>), grid, dim3(tile_lanes(TW)), 0, st, dd, sched, p, row_shift, sa); break;
    }
}

template <class S, bool NT>
static void launch_step_rows(const SimDesc* dd, const int2* sched, dim3 grid, int rows, int tile_w,
                             int p, hipStream_t st, int row_shift, SlotArray sa) {
    if (tile_w == TILE_WIDE)
        launch_step_tw<S, NT, TILE_WIDE>(dd, sched, grid, rows, p, st, row_shift, sa);
    else if (tile_w == TILE_NARROW)
        launch_step_tw<S, NT, TILE_NARROW>(dd, sched, grid, rows, p, st, row_shift, sa);
    else
        launch_step_tw<S, NT, TILE_X>(dd, sched, grid, rows, p, st, row_shift, sa);
}

// Body of one translation unit: defines Launch<S>.
#define VPLBM_DEFINE_LAUNCH(S)                                                                \
    template <>                                                                             \
    void Launch<S>::step(const SimDesc* dd, dim3 grid, int rows, bool nt, int tile_w, int p, \
                         hipStream_t st, int row_shift, SlotArray sa) {                     \
        if (nt)                                                                             \
            launch_step_rows<S, true>(dd, nullptr, grid, rows, tile_w, p, st, row_shift, sa); \
        else                                                                                \
            launch_step_rows<S, false>(dd, nullptr, grid, rows, tile_w, p, st, row_shift, sa); \
    }                                                                                       \
    template <>                                                                             \
    void Launch<S>::step_batch(const SimDesc* descs, const int2* sched, int nsched, int rows, \
                               bool nt, int tile_w, int p, hipStream_t st) {                \
        if (nt)                                                                             \
            launch_step_rows<S, true>(descs, sched, dim3(nsched), rows, tile_w, p, st, 0,   \
                                      SlotArray{nullptr, 0});                               \
        else                                                                                \
            launch_step_rows<S, false>(descs, sched, dim3(nsched), rows, tile_w, p, st, 0,  \
                                       SlotArray{nullptr, 0});                              \
    }                                                                                       \
    template <>                                                                             \
    void Launch<S>::fill(const SimDesc& d, const double g[NQ], int buf, hipStream_t st) {   \
        Offsets9 go;                                                                        \
        for (int a = 0; a < NQ; ++a) go.g[a] = g[a];                                        \
        hipLaunchKernelGGL(k_fill<S>, grid_rows(d), dim3(256), 0, st, d, go, buf);          \
    }                                                                                       \
    template <>                                                                             \
    void Launch<S>::set_pop(const SimDesc& d, const double* f, int buf, hipStream_t st) {   \
        hipLaunchKernelGGL(k_set_pop<S>, grid_rows(d), dim3(256), 0, st, d, f, buf);        \
    }                                                                                       \
    template <>                                                                             \
    void Launch<S>::get_pop(const SimDesc& d, double* f, int buf, hipStream_t st) {         \
        hipLaunchKernelGGL(k_get_pop<S>, grid_rows(d), dim3(256), 0, st, d, f, buf);        \
    }                                                                                       \
    template <>                                                                             \
    void Launch<S>::fields(const SimDesc& d, double* out, int p, hipStream_t st) {          \
        hipLaunchKernelGGL(k_fields<S>, grid_rows(d), dim3(256), 0, st, d, out, p);         \
    }

}  // namespace vplbm
