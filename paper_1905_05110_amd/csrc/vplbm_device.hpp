// vplbm_device.hpp -- device-side data structures and per-node arithmetic of the
// VP-LBM time step for gfx950 (MI355X).
//
// Populations are held as offsets g = f - f_ref from a reference equilibrium
// f_ref = f_eq(1, u_ref) in every storage precision (u_ref = 0 gives the rest-state
// weights w_a).  The moment transform works on the offsets directly, using
// M f_ref = m_eq(1, u_ref), and the macroscopic velocity is carried as du = u - u_ref,
// so that a flow near the reference state is stored and updated without cancelling
// against u_ref.
// Method: Liberge & Beghein (arXiv 1905.05110), Sec. 2.1-2.3 and Algorithm 1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <stdint.h>

namespace vplbm {

constexpr int NQ = 9;
// A tile is TW columns; the step kernel is built for TW = TILE_NARROW, TILE_X and
// TILE_WIDE, chosen per launch.  With TW = TILE_X or TILE_WIDE a tile is one row of TW
// columns per row of a TW-thread workgroup (each lane walks ROWS rows down its column);
// with TW = TILE_NARROW the TILE_X-thread workgroup stacks its four waves, one per row,
// so that a tile is 64 columns x 4 ROWS rows: a row's ragged end then leaves at most
// part of one wave idle, not whole waves of a wide tile.  TILE_X is also the width of
// the adjoint's tiles and the workgroup size of the body-state sums.
constexpr int TILE_NARROW = 64;
constexpr int TILE_X = 256;
constexpr int TILE_WIDE = 512;
constexpr int NWAVE = TILE_X / 64;
// threads of the step kernel's workgroup, and its rows of lanes, for tiles TW wide
__host__ __device__ constexpr int tile_lanes(int tw) { return tw == TILE_NARROW ? TILE_X : tw; }
__host__ __device__ constexpr int tile_stack(int tw) { return tile_lanes(tw) / tw; }
// per-step FP64 sums: penalization force (2) and torque (1); momentum inside the body
// after collision (2 + 1 angular) and before it (2 + 1); momentum-exchange force (2)
// and torque (1)
constexpr int NRED = 12;

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
// Tile ranges are (tx0, tx1, ty0, ty1), inclusive.
struct BodyState {
    double q[3], v[3];   // pose (X, Y, theta) and velocities used by the step
    double pin_prev[3];  // internal momentum P_in of the previous step
    long long t_body;    // steps since the body was set (phase of the imposed motion)
    long long step;      // index of the step that uses this state
    int pin_valid;       // 0 on the first step after the body is set
    int fresh;           // 1: written by the host or a flush; the step takes it as is
    int boxM[4];         // tiles within the support of this pose plus a 3-node margin
    int part_box[4];     // tiles that took part in this state's step (its partial slots)
};

struct BodyDev {
    // constants of the disc and its motion law
    int active, mode;
    unsigned free_mask;
    int imc;  // internal-fluid momentum correction for FREE bodies
    int smooth;
    int mem;  // momentum-exchange sum: 0 not evaluated, 1 evaluated and drives FREE bodies,
              // 2 evaluated and recorded only
    double R, R2, delta, reach;
    double mass, inertia;
    double k[3], c[3], q0[3], fext[3];
    double amp, freq, y0, phase;
    // optional additive indicator (FP64, row-major over the node window cwin = (i0, i1,
    // j0, j1), which lies inside the body's participating tiles): chi(i, j) becomes the
    // disc's indicator plus chi_add there; used by the adjoint, whose body is fixed
    const double* chi_add;
    int cwin[4];
    // State of step n in st[n & 1].  Step n's kernel derives it from st[(n - 1) & 1] and
    // the partial sums of step n - 1 (every tile that needs it, identically) unless the
    // host or a flush already wrote it ("fresh").
    BodyState st[2];
};

struct Record {  // same layout as lbm_force_rec
    long long step;
    double fvp[2], tvp, pin[3], fh[2], th, q[3], v[3], fmem[2], tmem;
};

// Per-simulation constants in the arithmetic precision T, precomputed on the host.
template <class T>
struct Consts {
    T s_e, s_eps, s_q, s_nu;      // MRT rates of the non-conserved moments
    T h_e, h_eps, h_q, h_nu;      // 1 - s/2 (source weights of Eq. (8))
    T inv_eta, gx, gy, u0x, u0y;  // 1/eta, fluid body force, reference velocity
    T uc, inv1uc;                 // convective outflow velocity, 1/(1 + U_c)
    T bb[4][NQ];                  // bounce-back increment per side and direction
    T dref[NQ][NQ];               // f_ref[b] - f_ref[a]: correction when a pulls b
    T xadd[2][3];                 // x-edge rule (west, east) for the three directions whose
                                  // source lies outside: the additive constant
};

struct SimDesc {
    void* pop[2];        // two population buffers, 9 planes of ps elements each
    void* outlet;        // 3 x ny offsets (directions 3, 6, 7) of the outflow memory
    void* outlet_out;    // where the step writes the next memory (normally == outlet)
    BodyDev* body;
    double* partials;    // NRED FP64 sums per participating tile, two parities
    long long part_stride;  // doubles per parity in partials
    Record* hist;        // ring of per-step records
    int* flag;           // set to 1 when an unstable node is met
    long long ps;        // stride between the population arrays of two directions (elements)
    int nx, ny;
    int pitch;           // stride between two rows of one direction's populations (elements)
    int fpitch;          // row stride of a single-field array such as dJ/dchi (elements)
    int layout;          // LBM_LAYOUT_ROWS or LBM_LAYOUT_PLANES (pitch and ps follow from it)
    int rows;            // rows per tile: rows per lane x the workgroup's rows of lanes
    int tiles_x, tiles_y, hist_cap;
    int tile_w;          // columns per tile of the step kernel: TILE_NARROW, TILE_X or TILE_WIDE
    int bc[4];
    // x-edge rule (west, east) for the three directions whose source lies outside (1, 5, 8
    // at the west side, 3, 6, 7 at the east): source (i + dx, j + dy) and its plane
    int xsrc[2][3][3];
    double u0x, u0y;     // reference velocity u_ref of the offsets
    double fref[NQ];     // f_eq(1, u_ref)
    float scale, inv_scale;  // storage scale of 16-bit offsets
    Consts<double> cd;
    Consts<float> cf;
};

template <class T>
__device__ __forceinline__ const Consts<T>& consts_of(const SimDesc& d);
template <>
__device__ __forceinline__ const Consts<double>& consts_of<double>(const SimDesc& d) {
    return d.cd;
}
template <>
__device__ __forceinline__ const Consts<float>& consts_of<float>(const SimDesc& d) {
    return d.cf;
}

// ---- storage codecs (byte offsets from a plane base) -----------------------------------
struct bf16s {
    uint16_t bits;
};

template <class S>
struct Codec;

// Population buffers live in global memory: accesses through these address-space-1
// pointers compile to global loads and stores with a uniform (scalar) base and a
// 32-bit lane offset, instead of flat accesses with 64-bit lane addresses.
typedef __attribute__((address_space(1))) const double g_cdouble;
typedef __attribute__((address_space(1))) double g_double;
typedef __attribute__((address_space(1))) const float g_cfloat;
typedef __attribute__((address_space(1))) float g_float;
typedef __attribute__((address_space(1))) _Float16 g_half;
typedef __attribute__((address_space(1))) const uint16_t g_cu16;
typedef __attribute__((address_space(1))) uint16_t g_u16;

template <>
struct Codec<double> {
    using T = double;
    static __device__ __forceinline__ T load(const char* base, unsigned off, float) {
        return *(g_cdouble*)(base + off);
    }
    template <bool NT>
    static __device__ __forceinline__ void store(char* base, unsigned off, T v, float) {
        g_double* q = (g_double*)(base + off);
        if (NT) __builtin_nontemporal_store(v, q); else *q = v;
    }
};

template <>
struct Codec<float> {
    using T = float;
    static __device__ __forceinline__ T load(const char* base, unsigned off, float) {
        return *(g_cfloat*)(base + off);
    }
    template <bool NT>
    static __device__ __forceinline__ void store(char* base, unsigned off, T v, float) {
        g_float* q = (g_float*)(base + off);
        if (NT) __builtin_nontemporal_store(v, q); else *q = v;
    }
};

template <>
struct Codec<_Float16> {
    using T = float;
    // stored value: round-to-nearest-even of g * 2^k
    static __device__ __forceinline__ T decode(uint16_t bits, float inv_scale) {
        return (float)__builtin_bit_cast(_Float16, bits) * inv_scale;
    }
    static __device__ __forceinline__ T load(const char* base, unsigned off, float inv_scale) {
        return decode(*(g_cu16*)(base + off), inv_scale);
    }
    template <bool NT>
    static __device__ __forceinline__ void store(char* base, unsigned off, T v, float scale) {
        g_half* q = (g_half*)(base + off);
        const _Float16 h = (_Float16)(v * scale);
        if (NT) __builtin_nontemporal_store(h, q); else *q = h;
    }
};

template <>
struct Codec<bf16s> {
    using T = float;
    static __device__ __forceinline__ T decode(uint16_t bits, float inv_scale) {
        return __builtin_bit_cast(float, (uint32_t)bits << 16) * inv_scale;
    }
    static __device__ __forceinline__ T load(const char* base, unsigned off, float inv_scale) {
        return decode(*(g_cu16*)(base + off), inv_scale);
    }
    template <bool NT>
    static __device__ __forceinline__ void store(char* base, unsigned off, T v, float scale) {
        g_u16* q = (g_u16*)(base + off);
        // round to nearest even: one conversion instruction on this architecture
        const uint16_t b = __builtin_bit_cast(uint16_t, (__bf16)(v * scale));
        if (NT) __builtin_nontemporal_store(b, q); else *q = b;
    }
};

// Fourth word of a raw buffer resource descriptor on this architecture (32-bit data
// format; no swizzle, no index stride).
constexpr int BUFFER_RSRC_WORD3 = 0x00020000;

// Global-memory load and store of a T through an address-space-1 pointer.
template <class T>
__device__ __forceinline__ T gld(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ void gst(T* p, T v) {
    *(__attribute__((address_space(1))) T*)p = v;
}

// Raise bits of the simulation's status flag with a global (not flat) atomic: a flat
// memory operation is also counted by the scalar-load counter, so later waits for
// scalar loads would wait for it too.
__device__ __forceinline__ void raise_flag(int* flag, int bits) {
    __hip_atomic_fetch_or((__attribute__((address_space(1))) int*)flag, bits, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
}

// Byte offset of node (i, j) from a direction's base, 64-bit: the paths off the tile's
// fast path (edge pulls, import, export, the exchange pass) address any buffer size this
// way, at the cost of a per-lane 64-bit address.
template <class S>
__device__ __forceinline__ long long node_off(const SimDesc& d, int i, int j) {
    return ((long long)j * d.pitch + i) * (long long)sizeof(S);
}

template <class S>
__device__ __forceinline__ const char* plane(const SimDesc& d, const void* buf, int a) {
    return reinterpret_cast<const char*>(buf) + (long long)a * d.ps * (long long)sizeof(S);
}

// The scalars of a step that a tile's fast path uses (buffers, layout, the collision
// constants), read once at the start of the tile.  Read there, ahead of every other
// memory operation of the tile, they come in with one round of scalar loads and stay in
// scalar registers; read from the descriptor where they are used, after a load or an
// atomic the compiler has to order them behind, each came back as a vector load with
// a full memory round trip of its own.
// The fast path addresses populations with 32-bit lane offsets from bases that the tile
// moves to its own rows: fin and fout point at row jb, the row above the tile's first
// (-1 for the first tile row: an address below the buffer that is never accessed), and a
// node (i, j) of the tile or of the rows next to it lies at byte offset
// ((j - jb) pitch + i) sizeof(S) from them, whatever the size of the buffer.
template <class T>
struct TileScalars {
    const char* fin;   // populations read by the step, from row jb on
    char* fout;        // populations written, from row jb on
    long long psb;     // plane stride in bytes
    unsigned rowb;     // row pitch in bytes
    int jb;            // the row fin and fout point at
    int pitch, nx, ny;
    float scale, inv_scale;
    int* flag;
    T s_e, s_eps, s_q, s_nu, h_e, h_eps, h_q, h_nu, inv_eta, gx, gy, u0x, u0y;
};

template <class S>
__device__ __forceinline__ TileScalars<typename Codec<S>::T> tile_scalars(const SimDesc& d, int p,
                                                                         int jb) {
    using T = typename Codec<S>::T;
    const Consts<T>& c = consts_of<T>(d);
    TileScalars<T> t;
    // integer arithmetic: the base of the first tile row lies below the buffer
    const long long rel = (long long)jb * d.pitch * (long long)sizeof(S);
    t.fin = reinterpret_cast<const char*>(reinterpret_cast<uintptr_t>(d.pop[p]) + rel);
    t.fout = reinterpret_cast<char*>(reinterpret_cast<uintptr_t>(d.pop[p ^ 1]) + rel);
    t.jb = jb;
    t.psb = d.ps * (long long)sizeof(S);
    t.pitch = d.pitch;
    t.rowb = (unsigned)d.pitch * (unsigned)sizeof(S);
    t.nx = d.nx;
    t.ny = d.ny;
    t.scale = d.scale;
    t.inv_scale = d.inv_scale;
    t.flag = d.flag;
    t.s_e = c.s_e;
    t.s_eps = c.s_eps;
    t.s_q = c.s_q;
    t.s_nu = c.s_nu;
    t.h_e = c.h_e;
    t.h_eps = c.h_eps;
    t.h_q = c.h_q;
    t.h_nu = c.h_nu;
    t.inv_eta = c.inv_eta;
    t.gx = c.gx;
    t.gy = c.gy;
    t.u0x = c.u0x;
    t.u0y = c.u0y;
    return t;
}

// ---- streaming with boundary rules (Eq. (18) applied as a pull) -----------------------
// Value pulled by node (i, j) for direction a.  Returns false when the source crosses
// an OUTFLOW side (the caller then applies the convective rule).
template <class S>
__device__ bool pull_rules(const SimDesc& d, const void* fin, int a, int i, int j,
                           typename Codec<S>::T& out) {
    using T = typename Codec<S>::T;
    const Consts<T>& c = consts_of<T>(d);
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
            out = Codec<S>::load(plane<S>(d, fin, dir_opp(a)) + node_off<S>(d, i, j), 0u, d.inv_scale) +
                  c.bb[side][a];
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
            out = Codec<S>::load(plane<S>(d, fin, dir_opp(a)) + node_off<S>(d, i, j), 0u, d.inv_scale) +
                  c.bb[side][a];
            return true;
        }
    }
    out = Codec<S>::load(plane<S>(d, fin, dir) + node_off<S>(d, si, sj), 0u, d.inv_scale);
    if (dir != a) out += c.dref[a][dir];  // specular reflection between directions
    return true;
}

// Index of a direction in the 3-slot outflow memory (directions 3, 6, 7).
__device__ __forceinline__ int outflow_slot(int a) { return a == 3 ? 0 : (a == 6 ? 1 : 2); }

// A uniform value held in a scalar register.  Selecting between two such values keeps
// the choice in registers; selecting between two loads would let the compiler turn it
// into one load from a per-lane address, a memory round trip on the critical path.
__device__ __forceinline__ float uniform_value(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double uniform_value(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Pulled offsets of a node on the domain edge, through the boundary rules; outlet_in
// is the outflow memory of the previous step.  The source of every direction is
// resolved first (pure arithmetic: the rules of pull_rules, with the convective outflow
// reading its value one node in), then the nine loads are issued together, so an edge
// node costs one memory round trip like an interior one.  When update_outlet is set,
// the east column stores its pulled values 3, 6, 7 into d.outlet_out as the memory of
// the next step (in place when outlet_out == outlet_in: each element is read and
// written by the same thread).
template <class S>
__device__ __forceinline__ void pull_edge(const SimDesc& d, const void* fin, const void* outlet_in, int i, int j,
                          typename Codec<S>::T g[NQ], bool update_outlet) {
    using T = typename Codec<S>::T;
    const Consts<T>& c = consts_of<T>(d);
    // uniform parameters, read together ahead of the lane-dependent logic
    const int nx = d.nx, ny = d.ny;
    const int kW = d.bc[0], kE = d.bc[1], kS = d.bc[2], kN = d.bc[3];
    const long long pitch = d.pitch;
    const long long psb = d.ps * (long long)sizeof(S);
    const float is = d.inv_scale;
    const T uc = c.uc, inv1uc = c.inv1uc;
    // additive constants: bounce-back increments bb[side][a] and reflection corrections
    // dref[a][b] (zero where b == a), addressed per lane as byte offsets into the block
    const char* cbase = reinterpret_cast<const char*>(&c);
    constexpr unsigned o_bb = (unsigned)offsetof(Consts<T>, bb);
    constexpr unsigned o_dr = (unsigned)offsetof(Consts<T>, dref);
    const char* base = reinterpret_cast<const char*>(fin);
    // Each direction is resolved (integer arithmetic only) and its two loads, the
    // population and its additive constant, issued at once; with the outflow memory
    // below they make one round of loads.
    T v[NQ], add[NQ];
    unsigned outflow = 0;  // bit a: direction a takes the convective outflow rule
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
        int si = i - dir_cx(a), sj = j - dir_cy(a);
        int pi = i;  // node whose pull this is (nx - 2 for the outflow's inner value)
        bool fx = false, fy = false, of = false;
        int bbside = -1;
        if (si < 0 || si >= nx) {
            const bool west = si < 0;
            const int kind = west ? kW : kE;
            if (kind == BC_PERIODIC) {
                si += west ? nx : -nx;
            } else if (kind == BC_SYMMETRY) {
                fx = true;
                si = i;
            } else if (kind == BC_OUTFLOW) {
                of = true;  // value pulled by (nx - 2, j): its x source is in range
                pi = nx - 2;
                si = nx - 2 - dir_cx(a);
            } else {  // WALL or VELOCITY: half-way bounce-back at (i, j)
                bbside = west ? 0 : 1;
            }
        }
        if (bbside < 0 && (sj < 0 || sj >= ny)) {
            const bool south = sj < 0;
            const int kind = south ? kS : kN;
            if (kind == BC_PERIODIC) {
                sj += south ? ny : -ny;
            } else if (kind == BC_SYMMETRY) {
                fy = true;
                sj = j;
            } else {
                bbside = south ? 2 : 3;
            }
        }
        const int ax = dir_flip_x(a), ay = dir_flip_y(a), ao = dir_opp(a);
        int dir;
        unsigned to;  // byte offset of the additive constant
        if (bbside >= 0) {
            dir = ao;
            si = pi;
            sj = j;
            to = o_bb + (unsigned)(bbside * NQ + a) * (unsigned)sizeof(T);
        } else {
            dir = (fx && fy) ? ao : (fx ? ax : (fy ? ay : a));  // specular reflection
            to = o_dr + (unsigned)(a * NQ + dir) * (unsigned)sizeof(T);
        }
        v[a] = Codec<S>::load(base + (long long)dir * psb +
                                  ((long long)sj * pitch + si) * (long long)sizeof(S), 0u, is);
        add[a] = gld(reinterpret_cast<const T*>(cbase + to));
        if (of) outflow |= 1u << a;
    }
    const T* outlet = reinterpret_cast<const T*>(outlet_in);
    T om[3] = {T(0), T(0), T(0)};
    if (kE == BC_OUTFLOW) {
#pragma unroll
        for (int k = 0; k < 3; ++k) om[k] = gld(outlet + k * ny + j);
    }
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
        T x = v[a] + add[a];
        // convective outflow: implicit upwind step of df/dt + U_c df/dx = 0 using last
        // step's value at the east column and this step's value one node in
        if (outflow & (1u << a)) x = (om[outflow_slot(a)] + uc * x) * inv1uc;
        g[a] = x;
    }
    if (update_outlet && i == nx - 1 && kE == BC_OUTFLOW) {
        T* next = reinterpret_cast<T*>(d.outlet_out);
        gst(next + 0 * ny + j, g[3]);
        gst(next + 1 * ny + j, g[6]);
        gst(next + 2 * ny + j, g[7]);
    }
}

// Interior node: the nine shifted planes are read directly (pull of Eq. (18)).
template <class S>
__device__ __forceinline__ void pull_interior(const char* const P[NQ], unsigned off, unsigned rowb,
                                              float is, typename Codec<S>::T g[NQ]) {
    constexpr unsigned e = sizeof(S);
    const unsigned o[NQ] = {off,        off - e,           off - rowb,        off + e,          off + rowb,
                            off - rowb - e, off - rowb + e, off + rowb + e, off + rowb - e};
    if constexpr (sizeof(S) == 2) {
        // 16-bit storage: the nine loads are all issued before the first is decoded.
        // Otherwise the scheduler may place a decode (and its wait) among them, and a
        // wave then waits for one round trip before issuing its last loads.
        uint16_t h[NQ];
#pragma unroll
        for (int a = 0; a < NQ; ++a) h[a] = *(g_cu16*)(P[a] + o[a]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < NQ; ++a) g[a] = Codec<S>::decode(h[a], is);
    } else {
#pragma unroll
        for (int a = 0; a < NQ; ++a) g[a] = Codec<S>::load(P[a], o[a], is);
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

template <class Body>
__device__ __forceinline__ double disc_chi(const Body& B, double d2) {
    if (!B.smooth) return d2 <= B.R2 ? 1.0 : 0.0;
    const double z = (sqrt(d2) - B.R) / B.delta;
    if (z > 20.0) return 0.0;
    if (z < -20.0) return 1.0;
    return 1.0 / (1.0 + exp(2.0 * z));
}

// The disc's shape parameters, read once (global loads of uniform values: scalar loads
// when nothing before them may have written the body) rather than through the generic
// body pointer, whose loads are flat and are waited for with every scalar load after.
struct DiscParams {
    int active, smooth;
    double R, R2, delta;
    const double* chi_add;
    int cwin[4];
};
__device__ __forceinline__ DiscParams disc_params(const BodyDev* B) {
    DiscParams q;
    q.active = gld(&B->active);
    q.smooth = gld(&B->smooth);
    q.R = gld(&B->R);
    q.R2 = gld(&B->R2);
    q.delta = gld(&B->delta);
    q.chi_add = gld(&B->chi_add);
#pragma unroll
    for (int k = 0; k < 4; ++k) q.cwin[k] = gld(&B->cwin[k]);
    return q;
}

// The additive indicator at node (i, j): the window's value, 0 outside it or without one.
template <class Body>
__device__ __forceinline__ double chi_add_at(const Body& B, int i, int j) {
    if (!B.chi_add || i < B.cwin[0] || i > B.cwin[1] || j < B.cwin[2] || j > B.cwin[3]) return 0.0;
    return B.chi_add[(long long)(j - B.cwin[2]) * (B.cwin[1] - B.cwin[0] + 1) + (i - B.cwin[0])];
}

// Tile range (inclusive) of the tiles that meet the support of the body; all its
// nodes with chi > 0 lie inside.  An absent or out-of-domain body maps to tile (0, 0)
// alone, so that exactly one workgroup finalises every step.
// Evaluated once per step (by the workgroup that advances the body, and on the host
// when the body is set) and stored per parity in BodyDev::box.
// margin: nodes added around the support (1 for the exact box, 3 for participation).
constexpr double BOX_MARGIN = 3.0;
__host__ __device__ inline void body_tiles(int nx, int ny, int rows, int tile_w, const BodyDev& B,
                                           double X, double Y, int box[4],
                                           double margin = BOX_MARGIN) {
    box[0] = box[1] = box[2] = box[3] = 0;
    if (!B.active) return;
    const double xl = fmax(floor(X - B.reach) - margin, 0.0);
    const double xh = fmin(ceil(X + B.reach) + margin, (double)(nx - 1));
    const double yl = fmax(floor(Y - B.reach) - margin, 0.0);
    const double yh = fmin(ceil(Y + B.reach) + margin, (double)(ny - 1));
    if (!(xl <= xh) || !(yl <= yh)) return;
    box[0] = (int)xl / tile_w;
    box[1] = (int)xh / tile_w;
    box[2] = (int)yl / rows;
    box[3] = (int)yh / rows;
}

// ---- macroscopic quantities, penalized velocity and MRT collision ------------------
template <class T>
struct NodeOut {
    T rho, drho, dux, duy, ux, uy, dFx, dFy, jgx, jgy, Gx, Gy;
};

template <class T>
__device__ __forceinline__ T recip(T x) {
    return T(1) / x;
}
template <>
__device__ __forceinline__ float recip<float>(float x) {
    return __builtin_amdgcn_rcpf(x);  // 1 ulp; FP32 arithmetic is not held to IEEE division
}

// Density, momentum and the implicit penalized velocity (Sec. 2.2, Eqs. (19)-(22)):
//   rho (1 + lam/2) u = j + rho g/2 + rho lam u_s / 2,   lam = chi / eta,
// solved for r = u - u_s; the fluid receives G = rho g - rho lam r and the body
// rho lam r.  With j = jg + u_ref (jg the momentum of the offsets) and
// ds = u_s - u_ref:  r = (jg - drho u_ref + rho g/2 - rho ds) / (rho (1 + lam/2)),
// u - u_ref = ds + r.  Where chi = 0 the result does not depend on u_s, and ds = 0
// is passed so that no term cancels against u_ref.
template <class T, bool VP = true, class C>
__device__ __forceinline__ void macros(const C& c, const T g[NQ], T chi, T dsx, T dsy,
                                       NodeOut<T>& o) {
    const T s1234 = (g[1] + g[2]) + (g[3] + g[4]);
    const T s5678 = (g[5] + g[6]) + (g[7] + g[8]);
    const T drho = g[0] + s1234 + s5678;
    const T jgx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const T jgy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const T rho = T(1) + drho;
    o.rho = rho;
    o.drho = drho;
    if (VP) {
        const T lam = chi * c.inv_eta;
        const T inv = recip<T>(rho * (T(1) + T(0.5) * lam));
        const T rx = (jgx - drho * c.u0x + T(0.5) * rho * c.gx - rho * dsx) * inv;
        const T ry = (jgy - drho * c.u0y + T(0.5) * rho * c.gy - rho * dsy) * inv;
        o.dux = dsx + rx;
        o.duy = dsy + ry;
        o.dFx = rho * lam * rx;
        o.dFy = rho * lam * ry;
    } else {  // chi = 0: plain Guo velocity, no penalization force
        const T inv = recip<T>(rho);
        o.dux = (jgx - drho * c.u0x + T(0.5) * rho * c.gx) * inv;
        o.duy = (jgy - drho * c.u0y + T(0.5) * rho * c.gy) * inv;
        o.dFx = T(0);
        o.dFy = T(0);
    }
    o.ux = c.u0x + o.dux;
    o.uy = c.u0y + o.duy;
    o.Gx = rho * c.gx - o.dFx;
    o.Gy = rho * c.gy - o.dFy;
    o.jgx = jgx;
    o.jgy = jgy;
}

// x / k for a small integer k, from the rounded reciprocal inv_k = RN(1/k).  The product
// x * inv_k alone carries the constant's own rounding, the same relative error at every
// node and step (RN(1/6) and RN(1/9) both lie above the true values in FP32); dividing
// the conserved moments that way adds momentum and mass coherently, step after step.
// One correction step from the exact residual x - k q (a single FMA: k q is within an
// ulp of x) gives the correctly rounded quotient, whose error is no longer biased.
template <class T>
__device__ __forceinline__ T div_small(T x, T k, T inv_k) {
    const T q = x * inv_k;
    return __builtin_fma(__builtin_fma(-k, q, x), inv_k, q);
}
__device__ __forceinline__ float div_small(float x, float k, float inv_k) {
    const float q = x * inv_k;
    return __builtin_fmaf(__builtin_fmaf(-k, q, x), inv_k, q);
}

// Collision in moment space with the forcing source (Eqs. (8), (14), (16), (17); the
// source enters with the sign of Eq. (8)):  m* = m - S (m - m_eq) + (I - S/2) M F,
// F the Guo forcing vector of Eq. (12) without its (1 - 1/2tau) factor, whose moments
// are (0, 6 u.G, -6 u.G, Gx, -Gx, Gy, -Gy, 2(ux Gx - uy Gy), ux Gy + uy Gx).
// The conserved moments come out as rho, j + G whatever their rates.
template <class T, bool VP = true, class C>
__device__ __forceinline__ void collide(const C& c, const T g[NQ], T chi, T dsx, T dsy,
                                        T out[NQ], NodeOut<T>& o) {
    macros<T, VP>(c, g, chi, dsx, dsy, o);
    const T drho = o.drho, Gx = o.Gx, Gy = o.Gy;
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

    const T ux = o.ux, uy = o.uy, dux = o.dux, duy = o.duy;
    const T u0x = c.u0x, u0y = c.u0y;
    const T usq = ux * ux + uy * uy;
    // equilibria of the offsets, m_eq(rho, u) - m_eq(1, u_ref), in terms of drho and du
    const T dsqx = dux * (T(2) * u0x + dux);  // ux^2 - u0x^2
    const T dsqy = duy * (T(2) * u0y + duy);
    const T dE = drho * usq + (dsqx + dsqy);  // rho |u|^2 - |u_ref|^2
    const T e_eq = T(3) * dE - T(2) * drho;
    const T ep_eq = drho - T(3) * dE;
    const T qx_eq = -(drho * ux + dux);
    const T qy_eq = -(drho * uy + duy);
    const T pxx_eq = drho * (ux * ux - uy * uy) + (dsqx - dsqy);
    const T pxy_eq = drho * ux * uy + (dux * u0y + u0x * duy + dux * duy);
    const T uG6 = T(6) * (ux * Gx + uy * Gy);

    const T e_s = e - c.s_e * (e - e_eq) + c.h_e * uG6;
    const T ep_s = ep - c.s_eps * (ep - ep_eq) - c.h_eps * uG6;
    const T qx_s = qx - c.s_q * (qx - qx_eq) - c.h_q * Gx;
    const T qy_s = qy - c.s_q * (qy - qy_eq) - c.h_q * Gy;
    const T pxx_s = pxx - c.s_nu * (pxx - pxx_eq) + c.h_nu * (T(2) * (ux * Gx - uy * Gy));
    const T pxy_s = pxy - c.s_nu * (pxy - pxy_eq) + c.h_nu * (ux * Gy + uy * Gx);
    const T jx_s = o.jgx + Gx;
    const T jy_s = o.jgy + Gy;

    // f = M^-1 m*, M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
    // The mass and momentum of the result are 9 a0 and 6 (a3, a5) exactly, so those three
    // quotients are correctly rounded (div_small); the others relax.
    const T a0 = div_small(drho, T(9), T(1.0 / 9.0));
    const T a1 = e_s * T(1.0 / 36.0);
    const T a2 = ep_s * T(1.0 / 36.0);
    const T a3 = div_small(jx_s, T(6), T(1.0 / 6.0));
    const T a4 = qx_s * T(1.0 / 12.0);
    const T a5 = div_small(jy_s, T(6), T(1.0 / 6.0));
    const T a6 = qy_s * T(1.0 / 12.0);
    const T a7 = pxx_s * T(0.25);
    const T a8 = pxy_s * T(0.25);
    const T b = a0 - a1 - T(2) * a2;
    const T cc = a0 + T(2) * a1 + a2;
    const T x1 = a3 - T(2) * a4, y1 = a5 - T(2) * a6;
    const T x2 = a3 + a4, y2 = a5 + a6;
    out[0] = a0 - T(4) * a1 + T(4) * a2;
    out[1] = b + x1 + a7;
    out[2] = b + y1 - a7;
    out[3] = b - x1 + a7;
    out[4] = b - y1 - a7;
    out[5] = cc + x2 + y2 + a8;
    out[6] = cc - x2 + y2 - a8;
    out[7] = cc - x2 - y2 + a8;
    out[8] = cc + x2 - y2 - a8;
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

// Working set, in LDS, of the body update that ends a step.
struct BodyStep {
    double tot[NRED];  // the step's FP64 sums
    double F[3];       // penalization load F_h (x, y and T_h), recorded as fh
    double qv[6];      // state of the next step: pose (X, Y, theta), then its velocities
    long long step, t_body;
    int boxM[4];       // participation box of that pose (filled by the thread that stores it)
    // the previous state's step counters and P_in flag, staged by lanes 0-2 (one copy
    // each, so that no two lanes write one location)
    long long step_prev[3], t_prev[3];
    int pin_valid[3];
};

__device__ __forceinline__ bool box_inside(const int a[4], const int b[4]) {
    return a[0] >= b[0] && a[1] <= b[1] && a[2] >= b[2] && a[3] <= b[3];
}

// Lanes of a 64-lane wave moved by one DPP pattern (lanes reading outside their row, or
// masked off, receive 0); the 64-bit value moves as two 32-bit halves.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, BANK_MASK, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, BANK_MASK, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave, returned to every lane.  Row shifts build the sum of
// each 16-lane row in its last lane, row broadcasts carry it on to lane 63 (a fixed
// order of FP64 additions, the same in every wave), which is then read by all lanes.
// Data-parallel moves between lanes: no LDS round trips.
__device__ __forceinline__ double wave_sum(double v) {
    double t = v + dpp_move<0x111, 0xf, 0xf>(v);   // row_shr:1
    t = t + dpp_move<0x112, 0xf, 0xf>(v);          // row_shr:2
    t = t + dpp_move<0x113, 0xf, 0xf>(v);          // row_shr:3
    t = t + dpp_move<0x114, 0xf, 0xe>(t);          // row_shr:4, banks 1-3
    t = t + dpp_move<0x118, 0xf, 0xc>(t);          // row_shr:8, banks 2-3
    t = t + dpp_move<0x142, 0xa, 0xf>(t);          // row_bcast:15, rows 1 and 3
    t = t + dpp_move<0x143, 0xc, 0xf>(t);          // row_bcast:31, rows 2 and 3
    const long long b = __builtin_bit_cast(long long, t);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// A wave of an interior row (1 <= j <= ny - 2) holding the west node (WEST) or the east
// node of the row but not both: every lane pulls as in the interior, except that the
// edge lane takes the three directions whose source lies outside (from x - 1 at the west
// edge, x + 1 at the east) through that side's rule.  The side, hence its rule and its
// additive constants, is the same for the whole wave, so the rule costs a few selects
// and scalar constants instead of the general per-lane resolution.  Lanes beyond the
// grid (i >= nx) load nothing.
template <class S, bool WEST>
__device__ __forceinline__ void pull_xedge(const SimDesc& d,
                                           const TileScalars<typename Codec<S>::T>& ts, int i,
                                           int j, typename Codec<S>::T g[NQ],
                                           bool update_outlet) {
    using T = typename Codec<S>::T;
    const Consts<T>& c = consts_of<T>(d);
    constexpr unsigned e = sizeof(S);
    const int nx = ts.nx;
    // outside directions (source x - 1 at the west edge, x + 1 at the east); the side's
    // rule for them (periodic wrap, reflection across the side, bounce-back, or the
    // outflow's value one node in) was resolved on the host into a source offset, a
    // plane and an additive constant, all read here in one round of scalar loads
    constexpr int A0 = WEST ? 1 : 3, A1 = WEST ? 5 : 6, A2 = WEST ? 8 : 7;
    const int side = WEST ? 0 : 1;
    const int kind = d.bc[side];
    T kadd[3];
    int sdx[3], sdy[3], spl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        sdx[k] = d.xsrc[side][k][0];
        sdy[k] = d.xsrc[side][k][1];
        spl[k] = d.xsrc[side][k][2];
        kadd[k] = c.xadd[side][k];
    }
    const bool edge = WEST ? (i == 0) : (i == nx - 1);
    const unsigned off = ((unsigned)(j - ts.jb) * (unsigned)ts.pitch + (unsigned)i) * e;
    const unsigned rowb = ts.rowb;
    const char* P[NQ];
#pragma unroll
    for (int a = 0; a < NQ; ++a) P[a] = ts.fin + (long long)a * ts.psb;
    T v[NQ];
    if (i < nx) {
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
            const int cx = dir_cx(a), cy = dir_cy(a);
            unsigned o = off - (unsigned)cx * e - (unsigned)cy * rowb;  // interior source
            const char* pl = P[a];
            const int k = a == A0 ? 0 : (a == A1 ? 1 : (a == A2 ? 2 : -1));
            if (k >= 0 && edge) {
                o = off + (unsigned)(sdx[k] * (int)e) + (unsigned)sdy[k] * rowb;
                pl = ts.fin + (long long)spl[k] * ts.psb;
            }
            v[a] = Codec<S>::load(pl, o, ts.inv_scale);
        }
    }
    T om[3] = {T(0), T(0), T(0)};
    if (!WEST && kind == BC_OUTFLOW && i < nx) {
        const T* outlet = reinterpret_cast<const T*>(d.outlet);
#pragma unroll
        for (int k = 0; k < 3; ++k) om[k] = gld(outlet + k * ts.ny + j);
    }
    if (i >= nx) return;
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
        const int k = a == A0 ? 0 : (a == A1 ? 1 : (a == A2 ? 2 : -1));
        T x = v[a];
        if (k >= 0 && edge) {
            x += kadd[k];
            // convective outflow: implicit upwind step of df/dt + U_c df/dx = 0 using
            // last step's value at the east column and this step's value one node in
            if (!WEST && kind == BC_OUTFLOW) x = (om[outflow_slot(a)] + c.uc * x) * c.inv1uc;
        }
        g[a] = x;
    }
    if (!WEST && update_outlet && edge && kind == BC_OUTFLOW) {
        T* next = reinterpret_cast<T*>(d.outlet_out);
        gst(next + 0 * ts.ny + j, g[3]);
        gst(next + 1 * ts.ny + j, g[6]);
        gst(next + 2 * ts.ny + j, g[7]);
    }
}

// Pull of row j for a wave that holds an edge node: the x-edge path when the row is
// interior and the wave holds one x edge only, else the general boundary-rule pull.
template <class S>
__device__ __forceinline__ void pull_wave_edge(const SimDesc& d,
                                               const TileScalars<typename Codec<S>::T>& ts,
                                               int i, int j, typename Codec<S>::T g[NQ]) {
    const int nx = ts.nx;
    const int i0 = __builtin_amdgcn_readfirstlane(i - (int)(threadIdx.x & 63));  // wave's first column
    const bool row_inner = j >= 1 && j <= ts.ny - 2;  // uniform: one row per wave
    const bool has_w = i0 == 0, has_e = i0 <= nx - 1 && nx - 1 < i0 + 64;
    if (row_inner && has_w && !has_e) {
        pull_xedge<S, true>(d, ts, i, j, g, true);
    } else if (row_inner && has_e && !has_w) {
        pull_xedge<S, false>(d, ts, i, j, g, true);
    } else if (i < nx && j < ts.ny) {
        pull_edge<S>(d, reinterpret_cast<const char*>(reinterpret_cast<uintptr_t>(ts.fin) -
                                                      (long long)ts.jb * ts.rowb),
                     d.outlet, i, j, g, true);
    }
}

// ---- one tile of one step ------------------------------------------------------------
// A tile is TW columns x ROWS rows; each lane walks down its column, issuing the
// next row's nine loads before colliding the current row.  Nodes are pulled,
// penalized, collided and stored.  PART tiles (those meeting the body) also rasterise
// chi and u_s and accumulate force, torque and internal momentum in FP64.
// First row of a tile: the pulled offsets of node (i, j0), interior or edge.
template <int TW, int ROWS>
__device__ __forceinline__ void tile_node(int tx, int ty, int& i, int& j0) {
    // column of this lane and first of its ROWS rows in tile (tx, ty)
    constexpr int K = tile_stack(TW);
    const int col = K == 1 ? (int)threadIdx.x : (int)(threadIdx.x & (TW - 1));
    const int grp = K == 1 ? 0 : (int)(threadIdx.x / TW);  // one wave per row group
    i = tx * TW + col;
    j0 = (ty * K + grp) * ROWS;
}

template <class S, int ROWS, int TW>
__device__ __forceinline__ void pull_first(const SimDesc& d,
                                           const TileScalars<typename Codec<S>::T>& ts, int tx,
                                           int ty, typename Codec<S>::T g[NQ]) {
    int i, j0;
    tile_node<TW, ROWS>(tx, ty, i, j0);
    // a wave with any edge node takes the boundary-rule pull for all its lanes (it
    // handles interior nodes too): one path and one round of loads per wave
    const bool inner = i >= 1 && i <= ts.nx - 2 && j0 >= 1 && j0 <= ts.ny - 2;
    if (__all(inner)) {
        const char* P[NQ];
#pragma unroll
        for (int a = 0; a < NQ; ++a) P[a] = ts.fin + (long long)a * ts.psb;
        pull_interior<S>(P, ((unsigned)(j0 - ts.jb) * (unsigned)ts.pitch + (unsigned)i) * (unsigned)sizeof(S),
                         ts.rowb, ts.inv_scale, g);
    } else {
        pull_wave_edge<S>(d, ts, i, j0, g);
    }
}

template <class S, int ROWS, bool NT, bool PART, int TW>
__device__ __forceinline__ void step_rows(const SimDesc& d,
                                          const TileScalars<typename Codec<S>::T>& c, int tx,
                                          int ty, double acc[NRED], const double* pose,
                                          typename Codec<S>::T g[NQ], bool& hit) {
    using T = typename Codec<S>::T;
    const char* fin = c.fin;
    char* fout = c.fout;
    int i, j0;
    tile_node<TW, ROWS>(tx, ty, i, j0);
    const int nx = c.nx, ny = c.ny;
    const bool col_ok = i < nx;
    const bool col_inner = i >= 1 && i <= nx - 2;

    const char* P[NQ];
    char* Q[NQ];
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
        P[a] = fin + (long long)a * c.psb;
        Q[a] = fout + (long long)a * c.psb;
    }
    const unsigned rowb = c.rowb;
    const float is = c.inv_scale;

    T gn[NQ];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int j = j0 + r;
        if (j >= ny) break;  // uniform over the wave
        if (r + 1 < ROWS && j + 1 < ny) {  // uniform
            if (__all(col_inner && j + 1 <= ny - 2))
                pull_interior<S>(P, ((unsigned)(j + 1 - c.jb) * (unsigned)c.pitch + (unsigned)i) * (unsigned)sizeof(S),
                                 rowb, is, gn);
            else
                pull_wave_edge<S>(d, c, i, j + 1, gn);
        }
        if (col_ok) {
            T out[NQ];
            NodeOut<T> o;
            if (PART) {
                const BodyDev& B = *d.body;
                double chi = 0.0, dsx = 0.0, dsy = 0.0;
                const double rx = (double)i - pose[0], ry = (double)j - pose[1];
                const double d2 = disc_d2(rx, ry);
                if (B.active) {
                    chi = disc_chi(B, d2) + chi_add_at(B, i, j);
                    if (chi != 0.0) {
                        const double om = pose[5];
                        dsx = (pose[3] - om * ry) - d.u0x;
                        dsy = (pose[4] + om * rx) - d.u0y;
                    }
                }
                if (chi != 0.0) {
                    hit = true;
                    collide<T, true>(c, g, (T)chi, (T)dsx, (T)dsy, out, o);
                    const double dFx = (double)o.dFx, dFy = (double)o.dFy;
                    const double jx = (double)o.jgx + d.u0x, jy = (double)o.jgy + d.u0y;
                    const double px = jx + (double)o.Gx, py = jy + (double)o.Gy;
                    acc[0] += dFx;
                    acc[1] += dFy;
                    acc[2] += rx * dFy - ry * dFx;
                    acc[3] += chi * px;
                    acc[4] += chi * py;
                    acc[5] += chi * (rx * py - ry * px);
                    acc[6] += chi * jx;
                    acc[7] += chi * jy;
                    acc[8] += chi * (rx * jy - ry * jx);
                } else {
                    // outside the body: the same instructions as in other tiles (nothing
                    // to accumulate), so results do not depend on which tiles take part
                    collide<T, false>(c, g, T(0), T(0), T(0), out, o);
                }
            } else {
                collide<T, false>(c, g, T(0), T(0), T(0), out, o);
            }
            const unsigned off = ((unsigned)(j - c.jb) * (unsigned)c.pitch + (unsigned)i) * (unsigned)sizeof(S);
#pragma unroll
            for (int a = 0; a < NQ; ++a) Codec<S>::template store<NT>(Q[a], off, out[a], c.scale);
            if (!(o.rho > T(0)) || !__builtin_isfinite(o.ux) || !__builtin_isfinite(o.uy))
                raise_flag(c.flag, 1);
        }
        if (r + 1 < ROWS) {
#pragma unroll
            for (int a = 0; a < NQ; ++a) g[a] = gn[a];
        }
    }
}

// Momentum-exchange load (Sec. 2.3, Eqs. (25)-(27)) of a participating tile's lane,
// m = (Fx, Fy, T), after the tile's rows are stored.  Solid nodes are those with d^2 <= R^2 (in both
// indicator modes).  A link joins a fluid node x_f to the solid node x_s = x_f + e; its
// force (e - u_G) f~_e(x_f) - (-e - u_G) f~_-e(x_s) is shared out as one term per end,
// each end evaluating x_G (the crossing of the link and the circle, taken from the fluid
// end so that both ends agree) and the rigid velocity u_G there.  A lane visits its
// nodes within one lattice step of the circle and reads back the post-collision
// populations it has just written along their links (the values that stream).  The
// directions are walked one at a time, apart from the collision, so that this adds no
// registers to it.
template <class S, int ROWS, int TW>
__device__ __forceinline__ void mem_pass(const SimDesc& d, int tx, int ty, int p,
                                         const double* pose, double m[3]) {
    const BodyDev& B = *d.body;
    int i, j0;
    tile_node<TW, ROWS>(tx, ty, i, j0);
    m[0] = m[1] = m[2] = 0.0;
    if (!B.active || !B.mem || i >= d.nx) return;
    // uniform over the workgroup: kept in scalar registers
    const double R2 = uniform_value(B.R2);
    const double band = uniform_value(B.R + 1.5), inner = uniform_value(B.R - 1.5);
    const double X = uniform_value(pose[0]), Y = uniform_value(pose[1]);
    const double Vx = uniform_value(pose[3]), Vy = uniform_value(pose[4]);
    const double Om = uniform_value(pose[5]);
    double mx = 0.0, my = 0.0, mt = 0.0;
#pragma unroll 1
    for (int r = 0; r < ROWS; ++r) {
        const int j = j0 + r;
        if (j >= d.ny) break;
        const double rx = (double)i - X, ry = (double)j - Y;
        const double d2 = disc_d2(rx, ry);
        if (d2 > band * band || (inner > 0.0 && d2 < inner * inner)) continue;
        const bool self_solid = d2 <= R2;
        const long long off = node_off<S>(d, i, j);
#pragma unroll 1
        for (int a = 1; a < NQ; ++a) {
            const int cx = dir_cx(a), cy = dir_cy(a);
            const double nrx = (double)(i + cx) - X, nry = (double)(j + cy) - Y;
            if ((disc_d2(nrx, nry) <= R2) == self_solid) continue;
            const double f = d.fref[a] + (double)Codec<S>::load(plane<S>(d, d.pop[p ^ 1], a) + off, 0u,
                                                                 d.inv_scale);
            // fluid end (relative to the centre) and link direction towards the solid
            const double fx = self_solid ? nrx : rx, fy = self_solid ? nry : ry;
            const double ex = self_solid ? -cx : cx, ey = self_solid ? -cy : cy;
            // nearer root of |f + q e|^2 = R^2, written without cancellation (c > 0, b < 0)
            const double qa = ex * ex + ey * ey, qb = ex * fx + ey * fy;
            const double qc = fx * fx + fy * fy - R2;
            const double q = qc / (-qb + sqrt(qb * qb - qa * qc));
            const double gx = fx + q * ex, gy = fy + q * ey;  // x_G - X
            const double ugx = Vx - Om * gy, ugy = Vy + Om * gx;
            const double sg = self_solid ? -1.0 : 1.0;
            const double Fx = sg * ((double)cx - ugx) * f, Fy = sg * ((double)cy - ugy) * f;
            mx += Fx;
            my += Fy;
            mt += gx * Fy - gy * Fx;
        }
    }
    m[0] = mx;
    m[1] = my;
    m[2] = mt;
}

// Fixed-order FP64 sum of a step's partial slots into tot (LDS) by the first TILE_X
// threads of a workgroup (of TILE_X or more threads; the others only meet the
// barriers): every caller, whatever its tile width, obtains bitwise the same totals.
__device__ __forceinline__ void sum_slots(const double* __restrict__ slots, int nb,
                                          double red[][NRED], double* tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < TILE_X) {  // uniform over each wave
        // the thread's first slot is loaded straight into the accumulators, all its
        // loads in flight before the first add waits (0 + v, as a sum from zero)
        double t[NRED];
        int s = threadIdx.x;
        if (s < nb) {
#pragma unroll
            for (int k = 0; k < NRED; ++k) t[k] = gld(slots + (long long)s * NRED + k);
        } else {
#pragma unroll
            for (int k = 0; k < NRED; ++k) t[k] = 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < NRED; ++k) t[k] = 0.0 + t[k];
        for (s += TILE_X; s < nb; s += TILE_X) {  // bodies of more than TILE_X tiles
#pragma unroll
            for (int h = 0; h < NRED; h += NRED / 2) {  // in halves: fewer live registers
#pragma unroll
                for (int k = h; k < h + NRED / 2; ++k) t[k] += gld(slots + (long long)s * NRED + k);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int k = 0; k < NRED; ++k) {
            const double v = wave_sum(t[k]);
            if (lane == 0) red[wave][k] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < NRED) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int w = 1; w < NWAVE; ++w) v += red[w][k];
        tot[k] = v;
    }
    __syncthreads();
}

__host__ __device__ __forceinline__ int box_count(const int b[4]) { return (b[1] - b[0] + 1) * (b[3] - b[2] + 1); }

// The body update at the end of step n - 1 (Sec. 2.3, Eqs. (23)-(24); RK4 of
// Algorithm 1), as every participating tile of step n and the flush kernel compute it:
// the fixed-order sum of step n - 1's slots, then one lane per degree of freedom
// advances it.  The hydrodynamic load is F_vp + P_in(n-1) - P_in(n-2): with P_in the
// post-collision momentum inside the body this is, for a sharp indicator, the momentum
// carried across the interface by streaming (the momentum-exchange force of Eqs.
// (25)-(27)); on the first step after the body is set the pre-collision momentum stands
// in for the previous P_in.  The result is left in bs (LDS) for all threads; the work
// runs in parallel lanes so that it needs no stack and few registers.  slots are step
// n - 1's partial slots; pbox is its participation box, which gives their count.
__device__ __forceinline__ void derive_body(const SimDesc& d, int p, double red[][NRED],
                                            BodyStep& bs, const double* slots, const int* pbox) {
    const BodyDev& B = *d.body;
    const BodyState& prev = B.st[p ^ 1];
    int nbox[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) nbox[i] = pbox[i];
    // The lanes that advance a degree of freedom stage its previous state in the LDS
    // fields they overwrite later (each lane its own): these loads return with the slot
    // count's, and their registers are free again while the slots are read.
    const int k = threadIdx.x;
    if (k < 3) {  // one block, so that a single wait covers every load
        const double q = gld(&prev.q[k]), v = gld(&prev.v[k]), pin = gld(&prev.pin_prev[k]);
        const long long sp = gld(&prev.step), tp = gld(&prev.t_body);
        const int pv = gld(&prev.pin_valid);
        bs.qv[k] = q;
        bs.qv[3 + k] = v;
        bs.F[k] = pin;
        bs.step_prev[k] = sp;
        bs.t_prev[k] = tp;
        bs.pin_valid[k] = pv;
    }
    sum_slots(slots, box_count(nbox), red, bs.tot);
    if (k < 3) {
        const double q_prev = bs.qv[k], v_prev = bs.qv[3 + k], pin_prev = bs.F[k];
        double dp = 0.0;
        if (B.imc) dp = bs.tot[3 + k] - (bs.pin_valid[k] ? pin_prev : bs.tot[6 + k]);
        bs.F[k] = bs.tot[k] + dp;
        const double F = B.mem == 1 ? bs.tot[9 + k] : bs.F[k];
        double q = q_prev, v = v_prev;
        if (B.active) {
            if (B.mode == MODE_IMPOSED_SIN) {
                if (k == 1) {
                    const double w = 6.283185307179586476925286766559 * B.freq;
                    const double ph = w * (double)(bs.t_prev[k] + 1) + B.phase;
                    q = B.y0 + B.amp * sin(ph);
                    v = w * B.amp * cos(ph);
                }
            } else if (B.mode == MODE_CONST_VEL) {
                q += v;
            } else if (B.mode == MODE_FREE && (B.free_mask & (1u << k))) {
                rk4_dof(k < 2 ? B.mass : B.inertia, B.c[k], B.k[k], B.q0[k], F + B.fext[k], q, v);
            }
        }
        bs.qv[k] = q;
        bs.qv[3 + k] = v;
    } else if (k == 3) {
        bs.step = bs.step_prev[0] + 1;  // staged before the slot sums' barriers
        bs.t_body = bs.t_prev[0] + 1;
    }
    __syncthreads();
}

// Record of step n - 1 (one thread), from the state it used and its sums.
__device__ __forceinline__ void write_record(const SimDesc& d, const BodyState& prev,
                                             const BodyStep& bs) {
    Record& r = d.hist[prev.step % d.hist_cap];
    r.step = prev.step;
    r.fvp[0] = bs.tot[0];
    r.fvp[1] = bs.tot[1];
    r.tvp = bs.tot[2];
    for (int k = 0; k < 3; ++k) {
        r.pin[k] = bs.tot[3 + k];
        r.q[k] = prev.q[k];
        r.v[k] = prev.v[k];
    }
    r.fh[0] = bs.F[0];
    r.fh[1] = bs.F[1];
    r.th = bs.F[2];
    r.fmem[0] = bs.tot[9];
    r.fmem[1] = bs.tot[10];
    r.tmem = bs.tot[11];
}

// State slot of step n from the derived update (one thread); fresh marks a flush.
__device__ __forceinline__ void store_state(BodyState& cur, const BodyState& prev,
                                            const BodyStep& bs, int fresh) {
    for (int k = 0; k < 3; ++k) {
        cur.q[k] = bs.qv[k];
        cur.v[k] = bs.qv[3 + k];
        cur.pin_prev[k] = bs.tot[3 + k];
    }
    cur.t_body = bs.t_body;
    cur.step = bs.step;
    cur.pin_valid = 1;
    for (int k = 0; k < 4; ++k) {
        cur.boxM[k] = bs.boxM[k];
        cur.part_box[k] = prev.boxM[k];
    }
    cur.fresh = fresh;
}

// Tiles that meet the body (with a margin, judged from the previous pose) obtain this
// step's body state, rasterise chi and u_s, and reduce their FP64 sums into a slot;
// the next step (or a flush) adds the slots in a fixed order.  No device-wide fence is
// needed: the kernel boundary orders producer and consumer (on this multi-XCD part such
// a fence would write back the whole L2).
// The caller maps workgroups to tiles (the host rotates the rows so that those of the
// body are dispatched early, a little into the grid: their longer work then overlaps
// the rest of the grid instead of extending the end of the kernel).
// Where a step's partial force slots live: the simulation's own array, or (slots != null)
// an array the caller names, whose two parities lie `stride` doubles apart.
struct SlotArray {
    double* slots;
    long long stride;
};
__device__ __forceinline__ double* slot_base(const SimDesc& d, SlotArray sa, int parity) {
    return sa.slots ? sa.slots + (long long)parity * sa.stride
                    : d.partials + (long long)parity * d.part_stride;
}

template <class S, int ROWS, bool NT, int TW>
__device__ __forceinline__ void step_tile(const SimDesc& d, int tx, int ty, int p, SlotArray sa) {
    using T = typename Codec<S>::T;
    constexpr int NW = tile_lanes(TW) / 64;  // waves of the workgroup
    __shared__ double red[NW][NRED];
    __shared__ double pose_set[6];
    __shared__ BodyStep bs;
    BodyDev& B = *d.body;
    // The step's scalars, then the participation box and whether this step's state is
    // final already, then the first row's populations.
    // the row above the tile's first: every row the tile reads or writes lies 1 to
    // K ROWS + 1 rows below it
    constexpr int TILE_ROWS = tile_stack(TW) * ROWS;
    const TileScalars<T> ts = tile_scalars<S>(d, p, ty * TILE_ROWS - 1);
    const double* prev_slots = slot_base(d, sa, p ^ 1);
    // The box is read with vector-memory (buffer) loads whose values stay in vector
    // registers until the pull has been issued: a uniform load result is otherwise
    // moved to scalar registers, with a wait for it, where it is loaded, and a scalar
    // or flat load would be waited for with every other scalar load.  The wait comes
    // after the population loads and is counted in order with them, so it costs no
    // round trip of its own, whatever the pull does with its values.  (The offset's
    // zero comes from a register the compiler cannot see through, which keeps the
    // loads per lane.)  The descriptor covers the two state slots exactly; reads
    // beyond it would return 0.
    const __amdgpu_buffer_rsrc_t bst = __builtin_amdgcn_make_buffer_rsrc(
        (void*)&B.st[0], (short)0, (int)sizeof(B.st), BUFFER_RSRC_WORD3);
    int vz;
    asm("v_mov_b32 %0, 0" : "=v"(vz));
    const int sp = vz + p * (int)sizeof(BodyState), sq = vz + (p ^ 1) * (int)sizeof(BodyState);
    constexpr int o_fresh = (int)offsetof(BodyState, fresh), o_box = (int)offsetof(BodyState, boxM);
    const int fresh_v = __builtin_amdgcn_raw_buffer_load_b32(bst, sp + o_fresh, 0, 0);
    int box_q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) box_q[k] = __builtin_amdgcn_raw_buffer_load_b32(bst, sq + o_box + 4 * k, 0, 0);
    T g[NQ];
    pull_first<S, ROWS, TW>(d, ts, tx, ty, g);
    const int fresh = __builtin_amdgcn_readfirstlane(fresh_v);
    // the tiles that take part: the box of the previous step's pose (with a margin that
    // covers this step's), whether this step's state is derived or was made final by a
    // flush, so that flushes do not change which slots the sums are made of
    int pb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pb[k] = __builtin_amdgcn_readfirstlane(box_q[k]);
    const int bx0 = pb[0], bx1 = pb[1], by0 = pb[2], by1 = pb[3];
    const bool part = tx >= bx0 && tx <= bx1 && ty >= by0 && ty <= by1;
    double acc[NRED];
    if (!part) {
        bool unused = false;
        step_rows<S, ROWS, NT, false, TW>(d, ts, tx, ty, acc, nullptr, g, unused);
        return;  // uniform over the workgroup
    }
    const bool writer = tx == bx0 && ty == by0;
    // pose and velocities of this step (LDS): as the host or a flush wrote them, or
    // derived from the previous step (whose last barrier makes them visible)
    const double* pose;
    if (fresh) {
        if (threadIdx.x < 3) {
            const double q = gld(&B.st[p].q[threadIdx.x]), v = gld(&B.st[p].v[threadIdx.x]);
            pose_set[threadIdx.x] = q;
            pose_set[3 + threadIdx.x] = v;
        }
        __syncthreads();
        pose = pose_set;
    } else {
        derive_body(d, p, red, bs, prev_slots, B.st[p ^ 1].part_box);
        pose = bs.qv;
    }
#pragma unroll
    for (int k = 0; k < NRED; ++k) acc[k] = 0.0;
    bool hit = false;  // a node of this lane lies in the body (chi != 0)
    step_rows<S, ROWS, NT, true, TW>(d, ts, tx, ty, acc, pose, g, hit);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // A wave none of whose nodes lies in the body holds +0 in every accumulator, whose
    // sum is +0: it skips the cross-lane sums (most waves of a tile meeting a small body).
    if (__any(hit)) {  // uniform over the wave
#pragma unroll
        for (int k = 0; k < NRED - 3; ++k) {
            const double s = wave_sum(acc[k]);
            if (lane == 0) red[wave][k] = s;
        }
    } else if (lane < NRED - 3) {
        red[wave][lane] = 0.0;
    }
    // the momentum-exchange pass runs once the other sums have left the registers
    if (B.mem) {  // uniform
        double m[3];
        mem_pass<S, ROWS, TW>(d, tx, ty, p, pose, m);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double s = wave_sum(m[k]);
            if (lane == 0) red[wave][NRED - 3 + k] = s;
        }
    } else if (lane < 3) {
        red[wave][NRED - 3 + lane] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x < NRED) {
        const int k = threadIdx.x;
        double s = red[0][k];
        for (int w = 1; w < NW; ++w) s += red[w][k];
        const int slot = (ty - by0) * (bx1 - bx0 + 1) + (tx - bx0);
        slot_base(d, sa, p)[(long long)slot * NRED + k] = s;
    }
    // the writer's global stores come last: no barrier waits for them
    if (writer && threadIdx.x == 0) {
        if (!fresh) {
            const BodyState& prev = B.st[p ^ 1];
            int exact[4];
            body_tiles(d.nx, d.ny, d.rows, d.tile_w, B, bs.qv[0], bs.qv[1], exact, 1.0);
            if (!box_inside(exact, pb)) raise_flag(d.flag, 2);  // moved >= 2 nodes in a step
            body_tiles(d.nx, d.ny, d.rows, d.tile_w, B, bs.qv[0], bs.qv[1], bs.boxM);
            write_record(d, prev, bs);
            store_state(B.st[p], prev, bs, 0);
        }
        B.st[p ^ 1].fresh = 0;  // the next step derives its state
    }
}

// Flush (one workgroup): make the state of step n (parity p) final on the host's
// request, writing the record of step n - 1.  Does nothing when the state is fresh
// already, so it may be launched any number of times.
__device__ __forceinline__ void finalize_step(const SimDesc& d, int p, SlotArray sa) {
    __shared__ double red[NWAVE][NRED];
    __shared__ BodyStep bs;
    BodyDev& B = *d.body;
    if (B.st[p].fresh) return;  // uniform
    derive_body(d, p, red, bs, slot_base(d, sa, p ^ 1),
                B.st[p ^ 1].part_box);
    if (threadIdx.x == 0) {
        const BodyState& prev = B.st[p ^ 1];
        int exact[4];
        body_tiles(d.nx, d.ny, d.rows, d.tile_w, B, bs.qv[0], bs.qv[1], exact, 1.0);
        if (!box_inside(exact, prev.boxM)) raise_flag(d.flag, 2);
        body_tiles(d.nx, d.ny, d.rows, d.tile_w, B, bs.qv[0], bs.qv[1], bs.boxM);
        write_record(d, prev, bs);
        store_state(B.st[p], prev, bs, 1);
    }
}

}  // namespace vplbm
