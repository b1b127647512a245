// vplbm.hip -- kernels and host runtime behind the C ABI of include/vplbm.h.
//
// One lbm_step launch = one fluid-structure step of Algorithm 1 (Liberge & Beghein,
// arXiv 1905.05110): every workgroup pulls, penalizes, collides and stores one row
// segment; the workgroups that meet the body reduce its force/torque in FP64 and the
// last of them advances the body on the device, so consecutive steps need no host
// round trip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "vplbm.h"
#include "vplbm_host.hpp"
#include "vplbm_kernels.hpp"

using namespace vplbm;

namespace vplbm {
__global__ __launch_bounds__(TILE_X) void k_finalize(const SimDesc* __restrict__ dp, int p,
                                                     SlotArray sa) {
    finalize_step(*dp, p, sa);
}
__global__ __launch_bounds__(TILE_X) void k_finalize_batch(const SimDesc* __restrict__ descs,
                                                           const int* __restrict__ members, int p) {
    finalize_step(descs[members[blockIdx.x]], p, SlotArray{nullptr, 0});
}
}  // namespace vplbm

// ---------------------------------------------------------------------------------
// host runtime
// ---------------------------------------------------------------------------------
namespace {
thread_local std::string g_create_error;
}  // namespace

static const double kW[NQ] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// Equilibrium f_eq(rho, u) (Eq. (11)) in FP64.
static void equilibrium(double rho, double ux, double uy, double f[NQ]) {
    const double usq = ux * ux + uy * uy;
    for (int a = 0; a < NQ; ++a) {
        const double cu = dir_cx(a) * ux + dir_cy(a) * uy;
        f[a] = kW[a] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    }
}

static int upload_desc(lbm_sim* s) {
    HIP_TRY(s, hipMemcpyAsync(s->desc_d, &s->desc, sizeof(SimDesc), hipMemcpyHostToDevice,
                              s->stream));
    return LBM_OK;
}

// First tile row in dispatch order.  Tiles that meet the body take longer than the
// others; dispatched among the last workgroups they would extend the end of the grid.
// Their rows are placed a little into the order, not at its start: the rotation is fixed
// while a captured graph is replayed, and a body that has since moved to lower rows then
// still has its tiles dispatched early rather than wrapped to the end.  How far in was
// measured on the free-VIV grid: an eighth of the rows for 32- and 64-bit populations
// (1-1.5 % faster than a sixteenth), a sixteenth for 16-bit ones (whose shorter tiles
// lost 1 % at an eighth).
static int dispatch_row_shift(const lbm_sim* s, const int boxM[4]) {
    const int tiles_y = s->desc.tiles_y;
    const bool narrow = s->storage == LBM_FP16_OFS || s->storage == LBM_BF16_OFS;
    const int r = boxM[2] - tiles_y / (narrow ? 16 : 8);
    return ((r % tiles_y) + tiles_y) % tiles_y;
}

static void drop_graph(lbm_sim* s) {
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->gexec = nullptr;
    s->graph = nullptr;
}

// Tiles of the body's participation box above which LBM_FINALIZE_AUTO finalizes by kernel:
// each of the box's P tiles reads P slots of 96 bytes when the tiles finalize, while the
// extra launch costs a few microseconds of the device's time per step.  Measured: a
// 40-node disc (about 100 tiles, 2048x1024) runs 25 us per step with the sums in its
// tiles and 32 us with the launch; a 512-node disc (about 2000 tiles, 8192^2) 813 us
// and 796 us.
constexpr int FINALIZE_TILES_MAX = 512;

// Whether the body state is made final by a launch after each step (LBM_FINALIZE_*); the
// box is that of the pose set or loaded last, in the current tiles (its size barely
// changes as the body moves).  A change takes effect at the next launch: captured graphs
// are dropped.
static void update_finalize(lbm_sim* s) {
    bool k = false;
    if (s->has_body) {
        if (s->fin_req == LBM_FINALIZE_KERNEL) {
            k = true;
        } else if (s->fin_req == LBM_FINALIZE_AUTO) {
            const BodyState& st = s->body_h.st[s->host_step & 1];
            int box[4];
            body_tiles(s->nx, s->ny, s->desc.rows, s->desc.tile_w, s->body_h, st.q[0], st.q[1], box);
            k = box_count(box) > FINALIZE_TILES_MAX;
        }
    }
    if (k != s->sep_final) {
        s->sep_final = k;
        drop_graph(s);
    }
}

// One fluid-structure step: one kernel launch (ev0/ev1, optional, bracket it); the
// partial force slots in sa.slots when that is set (lbm_step_static), else the
// simulation's own.
static int launch_step(lbm_sim* s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                       SlotArray sa = SlotArray{nullptr, 0}) {
    const int p = (int)(s->host_step & 1);
    const dim3 grid = step_grid(s->desc);
    if (ev0) HIP_TRY(s, hipEventRecord(ev0, s->stream));
    dispatch(s->storage, [&](auto* tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        Launch<S>::step(s->desc_d, grid, s->rows, s->nt, s->desc.tile_w, p, s->stream, s->row_shift,
                        sa);
        return LBM_OK;
    });
    if (ev1) HIP_TRY(s, hipEventRecord(ev1, s->stream));
    if (s->sep_final)  // the state of the next step, made final once for every tile
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(TILE_X), 0, s->stream, s->desc_d,
                           (int)((s->host_step + 1) & 1), sa);
    HIP_TRY(s, hipGetLastError());
    s->host_step += 1;
    return LBM_OK;
}

// Makes the body state of the next step final and writes the last step's record
// (the step kernels defer that work to their successor).  Enqueued on the stream.
static int flush_state(lbm_sim* s, SlotArray sa = SlotArray{nullptr, 0}) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(TILE_X), 0, s->stream, s->desc_d,
                       (int)(s->host_step & 1), sa);
    HIP_TRY(s, hipGetLastError());
    return LBM_OK;
}

// ---- partial force slots in a static device array, for lbm_step_static ------------------
// Callers that cannot allocate device memory (graph capture, serving loops) step with
// the partial slots here instead of the simulation's own array; each device holds its own
// copy for the life of the process.  STATIC_SLOT_DOUBLES / 2 per parity: 10 922 tiles of
// 12 sums.
constexpr long long STATIC_SLOT_DOUBLES = 1LL << 18;  // 2 MiB
static __device__ __align__(256) double scratch[STATIC_SLOT_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

// The device address of this device's `scratch` (the array's name in host code stands
// for it but is not a device address), looked up once per device with it current.
static int static_slots(lbm_sim* s, SlotArray& sa) {
    int dev = -1;
    HIP_TRY(s, hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(s, LBM_ERR_STATE, "device index beyond the static slot table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(s, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(s, LBM_ERR_HIP, "hipGetSymbolAddress returned no address");
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    sa.slots = g_scratch_ptr[dev];
    sa.stride = STATIC_SLOT_DOUBLES / 2;
    return LBM_OK;
}

extern "C" {

void lbm_default_opts(lbm_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    for (int k = 0; k < 4; ++k) o->bc[k] = LBM_BC_PERIODIC;
    o->rho0 = 1.0;
    o->storage = LBM_FP32;
    o->fp16_scale_log2 = 10;
    o->history_cap = 65536;
}

size_t lbm_pop_bytes(int nx, int ny, int storage) {
    if (nx < 1 || ny < 1 || storage < LBM_FP64 || storage > LBM_BF16_OFS) return 0;
    return (size_t)NQ * (size_t)plane_stride(nx, ny) * elem_size(storage);
}

const char* lbm_last_error(const lbm_sim* sim) {
    return sim ? sim->err.c_str() : g_create_error.c_str();
}

static int check_opts(int nx, int ny, lbm_rates r, double eta, const lbm_opts& o, std::string& m) {
    if (nx < 3 || ny < 3) return m = "nx and ny must be >= 3", LBM_ERR_ARG;
    if ((long long)nx * ny > (1LL << 31)) return m = "grid too large", LBM_ERR_ARG;
    const double rr[4] = {r.s_e, r.s_eps, r.s_q, r.s_nu};
    for (double x : rr)
        if (!(x > 0.0 && x < 2.0)) return m = "relaxation rates must lie in (0, 2)", LBM_ERR_ARG;
    if (!(eta > 0.0) || !std::isfinite(eta)) return m = "eta must be > 0", LBM_ERR_ARG;
    for (int k = 0; k < 4; ++k)
        if (o.bc[k] < LBM_BC_PERIODIC || o.bc[k] > LBM_BC_OUTFLOW)
            return m = "unknown boundary kind", LBM_ERR_ARG;
    if ((o.bc[0] == LBM_BC_PERIODIC) != (o.bc[1] == LBM_BC_PERIODIC) ||
        (o.bc[2] == LBM_BC_PERIODIC) != (o.bc[3] == LBM_BC_PERIODIC))
        return m = "periodic sides must come in opposite pairs", LBM_ERR_ARG;
    if (o.bc[0] == LBM_BC_OUTFLOW || o.bc[2] == LBM_BC_OUTFLOW || o.bc[3] == LBM_BC_OUTFLOW)
        return m = "OUTFLOW is only supported on the east side", LBM_ERR_ARG;
    if (!(o.u_conv >= 0.0)) return m = "u_conv must be >= 0", LBM_ERR_ARG;
    if (o.storage < LBM_FP64 || o.storage > LBM_BF16_OFS) return m = "unknown storage", LBM_ERR_ARG;
    if (o.storage == LBM_FP16_OFS && (o.fp16_scale_log2 < 0 || o.fp16_scale_log2 > 14))
        return m = "fp16_scale_log2 must lie in 0..14", LBM_ERR_ARG;
    if (o.history_cap < 1) return m = "history_cap must be >= 1", LBM_ERR_ARG;
    if (o.rows_per_tile != 0 && o.rows_per_tile != 1 && o.rows_per_tile != 2 &&
        o.rows_per_tile != 4)
        return m = "rows_per_tile must be 0, 1, 2 or 4", LBM_ERR_ARG;
    if (o.tile_width != 0 && o.tile_width != TILE_NARROW && o.tile_width != TILE_X &&
        o.tile_width != TILE_WIDE)
        return m = "tile_width must be 0, 64, 256 or 512", LBM_ERR_ARG;
    if (o.collision != LBM_COLLIDE_MRT && o.collision != LBM_COLLIDE_BGK)
        return m = "collision must be LBM_COLLIDE_MRT or LBM_COLLIDE_BGK", LBM_ERR_ARG;
    if (o.store_mode < LBM_STORE_AUTO || o.store_mode > LBM_STORE_NONTEMPORAL)
        return m = "unknown store mode", LBM_ERR_ARG;
    if (o.offset_ref != LBM_REF_AUTO && o.offset_ref != LBM_REF_INITIAL && o.offset_ref != LBM_REF_REST)
        return m = "unknown offset reference", LBM_ERR_ARG;
    if (!(o.rho0 > 0.0)) return m = "rho0 must be > 0", LBM_ERR_ARG;
    if ((o.pop_buffers[0] == nullptr) != (o.pop_buffers[1] == nullptr))
        return m = "pass both population buffers or neither", LBM_ERR_ARG;
    if (o.layout < LBM_LAYOUT_AUTO || o.layout > LBM_LAYOUT_PLANES)
        return m = "unknown layout", LBM_ERR_ARG;
    if (o.finalize < LBM_FINALIZE_AUTO || o.finalize > LBM_FINALIZE_KERNEL)
        return m = "unknown finalize mode", LBM_ERR_ARG;
    int pitch, layout;
    long long ps;
    if (!pop_geometry(nx, ny, o.storage, o.layout, pitch, ps, layout, m)) return LBM_ERR_ARG;
    return LBM_OK;
}

static void free_sim(lbm_sim* s) {
    drop_graph(s);
    if (s->own_pop) {
        if (s->pop[0]) (void)hipFree(s->pop[0]);
        if (s->pop[1]) (void)hipFree(s->pop[1]);
    }
    void* bufs[] = {s->outlet, s->body_d, s->partials, s->hist, s->flag, s->staging,
                    s->desc_d, s->chi_add_d};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

int lbm_create(int nx, int ny, lbm_rates rates, double eta, const lbm_opts* opts, lbm_sim** out) {
    if (!out) return g_create_error = "out is NULL", LBM_ERR_ARG;
    *out = nullptr;
    lbm_opts o;
    if (opts)
        o = *opts;
    else
        lbm_default_opts(&o);
    if (o.history_cap == 0) o.history_cap = 65536;
    std::string msg;
    int rc = check_opts(nx, ny, rates, eta, o, msg);
    if (rc) return g_create_error = msg, rc;
    if (o.collision == LBM_COLLIDE_BGK) rates.s_e = rates.s_eps = rates.s_q = rates.s_nu;

    lbm_sim* s = new lbm_sim();
    s->nx = nx;
    s->ny = ny;
    s->storage = o.storage;
    s->opts = o;
    s->rates = rates;
    s->eta = eta;
    s->hist_cap = o.history_cap;
    s->fin_req = o.finalize;
    s->pop_bytes = lbm_pop_bytes(nx, ny, o.storage);
    auto bail = [&](int code) {
        g_create_error = s->err;
        free_sim(s);
        return code;
    };
#define CREATE_TRY(expr)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            s->err = std::string(#expr) + ": " + hipGetErrorString(e_);                    \
            return bail(e_ == hipErrorOutOfMemory ? LBM_ERR_ALLOC : LBM_ERR_HIP);          \
        }                                                                                  \
    } while (0)
    int ndev = 0;
    CREATE_TRY(hipGetDeviceCount(&ndev));
    if (ndev < 1) return s->err = "no HIP device", bail(LBM_ERR_HIP);
    if (o.hip_stream) {
        s->stream = (hipStream_t)o.hip_stream;
    } else {
        CREATE_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        s->own_stream = true;
    }
    if (o.pop_buffers[0]) {
        s->pop[0] = o.pop_buffers[0];
        s->pop[1] = o.pop_buffers[1];
    } else {
        s->own_pop = true;
        CREATE_TRY(hipMalloc(&s->pop[0], s->pop_bytes));
        CREATE_TRY(hipMalloc(&s->pop[1], s->pop_bytes));
    }
    const size_t tsz = o.storage == LBM_FP64 ? 8 : 4;
    // Launch configuration defaults (lbm_autotune refines them): two rows per lane for
    // grids up to 2.5 M nodes with FP32 arithmetic, one otherwise; nontemporal stores once
    // the two population buffers exceed 1 GiB (far beyond the 256 MB Infinity Cache).
    s->rows = o.rows_per_tile ? o.rows_per_tile : 1;
    s->nt = o.store_mode == LBM_STORE_NONTEMPORAL ||
            (o.store_mode == LBM_STORE_AUTO && 2 * s->pop_bytes > (size_t(1) << 30));
    const int tile_w = o.tile_width ? o.tile_width : TILE_X;
    const int tile_h = s->rows * tile_stack(tile_w);
    const int tiles_x = (nx + tile_w - 1) / tile_w;
    const int tiles_y = (ny + tile_h - 1) / tile_h;
    // enough slots for any tile shape: one-row tiles of TILE_X columns, or the four-row
    // tiles of TILE_NARROW columns (more of them than of the former on grids of three rows)
    const long long ntiles = std::max((long long)((nx + TILE_X - 1) / TILE_X) * ny,
                                      (long long)((nx + TILE_NARROW - 1) / TILE_NARROW) *
                                          ((ny + 3) / 4));
    CREATE_TRY(hipMalloc(&s->outlet, 3 * (size_t)ny * tsz));
    CREATE_TRY(hipMalloc((void**)&s->body_d, sizeof(BodyDev)));
    CREATE_TRY(hipMalloc((void**)&s->partials, 2 * (size_t)ntiles * NRED * sizeof(double)));
    CREATE_TRY(hipMalloc((void**)&s->hist, (size_t)s->hist_cap * sizeof(Record)));
    CREATE_TRY(hipMalloc((void**)&s->flag, 64));
    CREATE_TRY(hipMalloc((void**)&s->desc_d, sizeof(SimDesc)));

    SimDesc& d = s->desc;
    d.pop[0] = s->pop[0];
    d.pop[1] = s->pop[1];
    d.outlet = s->outlet;
    d.outlet_out = s->outlet;
    d.body = s->body_d;
    d.partials = s->partials;
    d.part_stride = ntiles * NRED;
    d.hist = s->hist;
    d.flag = s->flag;
    {
        std::string m;
        (void)pop_geometry(nx, ny, o.storage, o.layout, d.pitch, d.ps, d.layout, m);  // checked above
    }
    d.fpitch = row_pitch(nx);
    d.nx = nx;
    d.ny = ny;
    d.rows = tile_h;
    d.tiles_x = tiles_x;
    d.tile_w = tile_w;
    d.tiles_y = tiles_y;
    d.hist_cap = s->hist_cap;
    for (int k = 0; k < 4; ++k) d.bc[k] = o.bc[k];
    // reference state of the stored offsets
    const bool ref_rest = o.offset_ref == LBM_REF_REST ||
                          (o.offset_ref == LBM_REF_AUTO &&
                           (o.storage == LBM_FP16_OFS || o.storage == LBM_BF16_OFS));
    d.u0x = ref_rest ? 0.0 : o.u0[0];
    d.u0y = ref_rest ? 0.0 : o.u0[1];
    equilibrium(1.0, d.u0x, d.u0y, d.fref);
    Consts<double>& cd = d.cd;
    cd.s_e = rates.s_e;
    cd.s_eps = rates.s_eps;
    cd.s_q = rates.s_q;
    cd.s_nu = rates.s_nu;
    cd.h_e = 1.0 - 0.5 * rates.s_e;
    cd.h_eps = 1.0 - 0.5 * rates.s_eps;
    cd.h_q = 1.0 - 0.5 * rates.s_q;
    cd.h_nu = 1.0 - 0.5 * rates.s_nu;
    cd.inv_eta = 1.0 / eta;
    cd.gx = o.g_fluid[0];
    cd.gy = o.g_fluid[1];
    cd.u0x = d.u0x;
    cd.u0y = d.u0y;
    cd.uc = o.u_conv;
    cd.inv1uc = 1.0 / (1.0 + o.u_conv);
    for (int a = 0; a < NQ; ++a)
        for (int b = 0; b < NQ; ++b) cd.dref[a][b] = d.fref[b] - d.fref[a];
    for (int side = 0; side < 4; ++side)
        for (int a = 0; a < NQ; ++a) {
            const double moving =
                o.bc[side] == LBM_BC_VELOCITY
                    ? 6.0 * kW[a] * (dir_cx(a) * o.u_wall[side][0] + dir_cy(a) * o.u_wall[side][1])
                    : 0.0;
            cd.bb[side][a] = moving + cd.dref[a][dir_opp(a)];
        }
    // the x-edge rules of the west and east sides for their three outside directions
    for (int side = 0; side < 2; ++side)
        for (int k = 0; k < 3; ++k) {
            const int a = side == 0 ? (k == 0 ? 1 : (k == 1 ? 5 : 8)) : (k == 0 ? 3 : (k == 1 ? 6 : 7));
            const int cx = dir_cx(a), cy = dir_cy(a);
            int* src = d.xsrc[side][k];
            double add = 0.0;
            switch (o.bc[side]) {
                case LBM_BC_PERIODIC:  // the node across the domain
                    src[0] = -cx + (side == 0 ? nx : -nx);
                    src[1] = -cy;
                    src[2] = a;
                    break;
                case LBM_BC_SYMMETRY:  // the mirror image (i, j - cy), reflected direction
                    src[0] = 0;
                    src[1] = -cy;
                    src[2] = dir_flip_x(a);
                    add = cd.dref[a][dir_flip_x(a)];
                    break;
                case LBM_BC_OUTFLOW:  // node nx - 2's pull of the same direction
                    src[0] = 0;
                    src[1] = -cy;
                    src[2] = a;
                    break;
                default:  // bounce-back at the node itself
                    src[0] = 0;
                    src[1] = 0;
                    src[2] = dir_opp(a);
                    add = cd.bb[side][a];
                    break;
            }
            cd.xadd[side][k] = add;
        }
    Consts<float>& cf = d.cf;
    {
        const double* src = reinterpret_cast<const double*>(&cd);
        float* dst = reinterpret_cast<float*>(&cf);
        static_assert(sizeof(Consts<double>) == 2 * sizeof(Consts<float>), "constant blocks");
        for (size_t k = 0; k < sizeof(Consts<double>) / sizeof(double); ++k) dst[k] = (float)src[k];
    }
    if (o.storage == LBM_FP16_OFS) {
        d.scale = std::ldexp(1.0f, o.fp16_scale_log2);
        d.inv_scale = std::ldexp(1.0f, -o.fp16_scale_log2);
    } else {
        d.scale = 1.0f;
        d.inv_scale = 1.0f;
    }

    // initial state: equilibrium at (rho0, u0) in both buffers, outflow memory alike
    CREATE_TRY(hipMemsetAsync(s->pop[0], 0, s->pop_bytes, s->stream));
    CREATE_TRY(hipMemsetAsync(s->pop[1], 0, s->pop_bytes, s->stream));
    CREATE_TRY(hipMemsetAsync(s->flag, 0, 64, s->stream));
    double g[NQ];
    equilibrium(o.rho0, o.u0[0], o.u0[1], g);
    for (int a = 0; a < NQ; ++a) g[a] -= d.fref[a];
    dispatch(o.storage, [&](auto* tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        for (int b = 0; b < 2; ++b) Launch<S>::fill(d, g, b, s->stream);
        return 0;
    });
    CREATE_TRY(hipGetLastError());
    {
        std::vector<double> o64(3 * (size_t)ny);
        std::vector<float> o32(3 * (size_t)ny);
        const int dirs[3] = {3, 6, 7};
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < ny; ++j) {
                o64[(size_t)k * ny + j] = g[dirs[k]];
                o32[(size_t)k * ny + j] = (float)g[dirs[k]];
            }
        if (tsz == 8)
            CREATE_TRY(hipMemcpy(s->outlet, o64.data(), o64.size() * 8, hipMemcpyHostToDevice));
        else
            CREATE_TRY(hipMemcpy(s->outlet, o32.data(), o32.size() * 4, hipMemcpyHostToDevice));
    }
    std::memset(&s->body_h, 0, sizeof(BodyDev));
    s->body_h.active = 0;
    s->body_h.st[0].fresh = 1;  // step 0 takes this (absent-body) state as is
    CREATE_TRY(hipMemcpyAsync(s->body_d, &s->body_h, sizeof(BodyDev), hipMemcpyHostToDevice,
                              s->stream));
    CREATE_TRY(hipMemcpyAsync(s->desc_d, &s->desc, sizeof(SimDesc), hipMemcpyHostToDevice,
                              s->stream));
    CREATE_TRY(hipStreamSynchronize(s->stream));
#undef CREATE_TRY
    *out = s;
    return LBM_OK;
}

int lbm_destroy(lbm_sim* s) {
    if (!s) return LBM_ERR_ARG;
    if (s->in_batch) return reject_member(s);
    // an error of the work still queued is not reported here: the handle goes either way
    (void)hipStreamSynchronize(s->stream);
    free_sim(s);
    return LBM_OK;
}

static int sync_check(lbm_sim* s) {
    int rc = flush_state(s);
    if (rc) return rc;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    int flag = 0;
    HIP_TRY(s, hipMemcpy(&flag, s->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag & 1) return fail(s, LBM_ERR_UNSTABLE, "non-positive or non-finite density/velocity met");
    if (flag & 2) return fail(s, LBM_ERR_UNSTABLE, "body moved two or more nodes in one step");
    return LBM_OK;
}

int lbm_sync(lbm_sim* s) {
    if (!s) return LBM_ERR_ARG;
    return sync_check(s);
}

int lbm_set_body(lbm_sim* s, const lbm_body* b) {
    if (!s || !b) return fail(s, LBM_ERR_ARG, "NULL argument");
    if (!(b->radius > 0.0) || !std::isfinite(b->radius))
        return fail(s, LBM_ERR_ARG, "radius must be > 0");
    if (b->mode < LBM_BODY_FIXED || b->mode > LBM_BODY_CONST_VEL)
        return fail(s, LBM_ERR_ARG, "unknown body mode");
    if (b->mode == LBM_BODY_FREE && (!(b->mass > 0.0) || !(b->inertia > 0.0)))
        return fail(s, LBM_ERR_ARG, "FREE bodies need mass > 0 and inertia > 0");
    if (!(b->smooth_delta >= 0.0)) return fail(s, LBM_ERR_ARG, "smooth_delta must be >= 0");
    if (b->free_mask > 7u) return fail(s, LBM_ERR_ARG, "free_mask has bits beyond x, y, theta");
    if (b->force_model < LBM_FORCE_VP || b->force_model > LBM_FORCE_VP_MEM)
        return fail(s, LBM_ERR_ARG, "force_model must be LBM_FORCE_VP, _MEM or _VP_MEM");
    if (!std::isfinite(b->imp_phase)) return fail(s, LBM_ERR_ARG, "non-finite imp_phase");
    const double vals[] = {b->x, b->y, b->theta, b->vx, b->vy, b->omega};
    for (double x : vals)
        if (!std::isfinite(x)) return fail(s, LBM_ERR_ARG, "non-finite pose or velocity");
    int rc = sync_check(s);  // finish pending work and its record first
    if (rc && rc != LBM_ERR_UNSTABLE) return rc;
    BodyDev B;
    std::memset(&B, 0, sizeof(B));
    B.active = 1;
    B.mode = b->mode;
    B.free_mask = b->free_mask;
    B.imc = b->internal_mass_correction ? 1 : 0;
    B.mem = b->force_model == LBM_FORCE_MEM ? 1 : (b->force_model == LBM_FORCE_VP_MEM ? 2 : 0);
    B.smooth = b->smooth_delta > 0.0;
    B.R = b->radius;
    B.R2 = b->radius * b->radius;
    B.delta = b->smooth_delta;
    B.reach = B.smooth ? b->radius + 20.0 * b->smooth_delta : b->radius;
    B.mass = b->mass;
    B.inertia = b->inertia;
    for (int k = 0; k < 3; ++k) {
        B.k[k] = b->k[k];
        B.c[k] = b->c[k];
        B.q0[k] = b->q0[k];
        B.fext[k] = b->f_ext[k];
    }
    B.amp = b->imp_amp;
    B.freq = b->imp_freq;
    B.y0 = b->imp_y0;
    B.phase = b->imp_phase;
    B.chi_add = s->chi_add_d;
    for (int k = 0; k < 4; ++k) B.cwin[k] = s->chi_win[k];
    const int p = (int)(s->host_step & 1);
    double q[3] = {b->x, b->y, b->theta}, v[3] = {b->vx, b->vy, b->omega};
    if (b->mode == LBM_BODY_IMPOSED_SIN) {
        q[1] = b->imp_y0 + b->imp_amp * std::sin(b->imp_phase);
        v[1] = 6.283185307179586476925286766559 * b->imp_freq * b->imp_amp * std::cos(b->imp_phase);
    }
    BodyState& st = B.st[p];
    for (int k = 0; k < 3; ++k) {
        st.q[k] = q[k];
        st.v[k] = v[k];
    }
    st.t_body = 0;
    st.step = s->host_step;
    st.pin_valid = 0;
    st.fresh = 1;
    body_tiles(s->nx, s->ny, s->desc.rows, s->desc.tile_w, B, q[0], q[1], st.boxM);
    for (int k = 0; k < 4; ++k) st.part_box[k] = st.boxM[k];
    // a step takes part by the box of the state before it: the other slot starts as a
    // copy of this one
    B.st[p ^ 1] = st;
    const int shift = dispatch_row_shift(s, st.boxM);
    if (s->row_shift != shift) {  // captured launches carry the row shift
        s->row_shift = shift;
        drop_graph(s);
    }
    s->body_h = B;
    s->body_desc = *b;
    if (!s->has_body) s->drained = std::max(s->drained, s->host_step);  // body-less steps
    s->has_body = true;
    update_finalize(s);
    HIP_TRY(s, hipMemcpy(s->body_d, &B, sizeof(B), hipMemcpyHostToDevice));
    return LBM_OK;
}

int lbm_clear_body(lbm_sim* s) {
    if (!s) return LBM_ERR_ARG;
    int rc = sync_check(s);
    if (rc && rc != LBM_ERR_UNSTABLE) return rc;
    BodyDev B;
    HIP_TRY(s, hipMemcpy(&B, s->body_d, sizeof(B), hipMemcpyDeviceToHost));
    const int p = (int)(s->host_step & 1);
    B.active = 0;
    BodyState& st = B.st[p];
    st.pin_valid = 0;
    st.fresh = 1;
    for (int k = 0; k < 4; ++k) st.boxM[k] = st.part_box[k] = B.st[p ^ 1].boxM[k] = 0;
    if (s->row_shift != 0) {
        s->row_shift = 0;
        drop_graph(s);
    }
    if (s->has_body) s->rec_end = s->host_step;
    s->has_body = false;
    update_finalize(s);
    HIP_TRY(s, hipMemcpy(s->body_d, &B, sizeof(B), hipMemcpyHostToDevice));
    return LBM_OK;
}

int lbm_set_graph_steps(lbm_sim* s, int k) {
    if (!s) return LBM_ERR_ARG;
    if (s->in_batch) return reject_member(s);
    if (k != 0 && (k < 2 || (k & 1))) return fail(s, LBM_ERR_ARG, "graph steps must be 0 or even >= 2");
    drop_graph(s);
    s->graph_steps = k;
    return LBM_OK;
}

static int capture_graph(lbm_sim* s) {
    // the graph holds graph_steps launches with parities 0, 1, 0, 1, ...
    const int64_t saved = s->host_step;
    s->host_step = 0;
    HIP_TRY(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    int rc = LBM_OK;
    for (int k = 0; k < s->graph_steps && rc == LBM_OK; ++k) rc = launch_step(s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    s->host_step = saved;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(s, LBM_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
    s->graph = g;
    HIP_TRY(s, hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0));
    return LBM_OK;
}

int lbm_step(lbm_sim* s, int64_t n) {
    if (!s) return LBM_ERR_ARG;
    if (s->in_batch) return reject_member(s);
    if (n < 0) return fail(s, LBM_ERR_ARG, "n must be >= 0");
    int64_t done = 0;
    if (s->graph_steps > 0 && n >= s->graph_steps) {
        if ((s->host_step & 1) && done < n) {
            int rc = launch_step(s);
            if (rc) return rc;
            ++done;
        }
        if (!s->gexec) {
            int rc = capture_graph(s);
            if (rc) return rc;
        }
        while (n - done >= s->graph_steps) {
            HIP_TRY(s, hipGraphLaunch(s->gexec, s->stream));
            s->host_step += s->graph_steps;
            done += s->graph_steps;
        }
    }
    for (; done < n; ++done) {
        int rc = launch_step(s);
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_step_static(lbm_sim* s, int64_t n) {
    if (!s) return LBM_ERR_ARG;
    if (s->in_batch) return reject_member(s);
    if (n < 0) return fail(s, LBM_ERR_ARG, "n must be >= 0");
    if (s->has_body) {
        // a step's slots: one per tile of its participation box; the box of a moving body
        // spans at most one more tile each way than that of the pose set last
        const BodyState& st = s->body_h.st[s->host_step & 1];
        int box[4];
        body_tiles(s->nx, s->ny, s->desc.rows, s->desc.tile_w, s->body_h, st.q[0], st.q[1], box);
        const long long need = (long long)(box[1] - box[0] + 3) * (box[3] - box[2] + 3) * NRED;
        if (need > STATIC_SLOT_DOUBLES / 2)
            return fail(s, LBM_ERR_ARG, "the body's tiles need more partial slots than the static array holds (" +
                                            std::to_string(STATIC_SLOT_DOUBLES / 2 / NRED) + " tiles)");
    }
    SlotArray sa;
    int rc = static_slots(s, sa);
    if (rc) return rc;
    // the pending state is made final from the simulation's own slots; the steps then
    // write and read the static ones, and the last is made final from them, so that later
    // steps of either kind find a final state and never read the other kind's slots
    rc = flush_state(s);
    for (int64_t k = 0; k < n && rc == LBM_OK; ++k) rc = launch_step(s, nullptr, nullptr, sa);
    if (rc == LBM_OK && n > 0) rc = flush_state(s, sa);
    return rc;
}

int lbm_step_timed(lbm_sim* s, int64_t n, double* kernel_ms, double* region_ms) {
    if (!s || n < 0) return fail(s, LBM_ERR_ARG, "bad argument");
    if (s->in_batch) return reject_member(s);
    // Every event created here is destroyed on every way out; the first failure is the
    // one reported, and no timing is returned after one.
    std::vector<hipEvent_t> ev;
    ev.reserve(2 * (size_t)n + 2);
    int rc = LBM_OK;
    auto check = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == LBM_OK)
            rc = fail(s, LBM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    };
    for (size_t i = 0; i < 2 * (size_t)n + 2 && rc == LBM_OK; ++i) {
        hipEvent_t e = nullptr;
        check(hipEventCreate(&e), "hipEventCreate");
        if (rc == LBM_OK) ev.push_back(e);
    }
    if (rc == LBM_OK) check(hipEventRecord(ev[0], s->stream), "hipEventRecord");
    for (int64_t k = 0; k < n && rc == LBM_OK; ++k) rc = launch_step(s, ev[2 + 2 * k], ev[3 + 2 * k]);
    if (rc == LBM_OK) check(hipEventRecord(ev[1], s->stream), "hipEventRecord");
    if (rc == LBM_OK) check(hipEventSynchronize(ev[1]), "hipEventSynchronize");
    double ksum = 0.0;
    float ms = 0.f, region = 0.f;
    for (int64_t k = 0; k < n && rc == LBM_OK; ++k) {
        check(hipEventElapsedTime(&ms, ev[2 + 2 * k], ev[3 + 2 * k]), "hipEventElapsedTime");
        ksum += ms;
    }
    if (rc == LBM_OK) check(hipEventElapsedTime(&region, ev[0], ev[1]), "hipEventElapsedTime");
    for (auto& e : ev) (void)hipEventDestroy(e);  // nothing to recover from here
    if (rc) return rc;
    if (kernel_ms) *kernel_ms = ksum;
    if (region_ms) *region_ms = region;
    return LBM_OK;
}

int64_t lbm_step_index(const lbm_sim* s) { return s ? s->host_step : -1; }

int lbm_forces(lbm_sim* s, lbm_force_rec* out, int64_t cap, int64_t* n_out) {
    if (!s || (!out && cap > 0) || cap < 0) return fail(s, LBM_ERR_ARG, "bad argument");
    int rc = sync_check(s);  // flushes: records exist for every enqueued step
    if (n_out) *n_out = 0;
    const int64_t written = s->has_body ? s->host_step : s->rec_end;
    if (s->drained < written - s->hist_cap) s->drained = written - s->hist_cap;
    int64_t n = std::min<int64_t>(written - s->drained, cap);
    static_assert(sizeof(Record) == sizeof(lbm_force_rec), "record layout");
    for (int64_t k = 0; k < n;) {
        const int64_t st = s->drained + k;
        const int64_t slot = st % s->hist_cap;
        const int64_t run = std::min<int64_t>(n - k, s->hist_cap - slot);
        HIP_TRY(s, hipMemcpy(out + k, s->hist + slot, run * sizeof(Record), hipMemcpyDeviceToHost));
        k += run;
    }
    s->drained += n;
    if (n_out) *n_out = n;
    return rc;
}

int lbm_fields(lbm_sim* s, double* rho, double* ux, double* uy) {
    if (!s || !rho || !ux || !uy) return fail(s, LBM_ERR_ARG, "NULL argument");
    const int p = (int)(s->host_step & 1);
    if (ensure_staging(s) != hipSuccess)
        return fail(s, LBM_ERR_ALLOC, "hipMalloc of the FP64 exchange buffer failed");
    int frc = flush_state(s);
    if (frc) return frc;
    dispatch(s->storage, [&](auto* tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        Launch<S>::fields(s->desc, s->staging, p, s->stream);
        return 0;
    });
    HIP_TRY(s, hipGetLastError());
    int rc = sync_check(s);
    const size_t plane = (size_t)s->nx * s->ny;
    HIP_TRY(s, hipMemcpy(rho, s->staging, plane * 8, hipMemcpyDeviceToHost));
    HIP_TRY(s, hipMemcpy(ux, s->staging + plane, plane * 8, hipMemcpyDeviceToHost));
    HIP_TRY(s, hipMemcpy(uy, s->staging + 2 * plane, plane * 8, hipMemcpyDeviceToHost));
    return rc;
}

int lbm_set_populations(lbm_sim* s, const double* f) {
    if (!s || !f) return fail(s, LBM_ERR_ARG, "NULL argument");
    if (ensure_staging(s) != hipSuccess)
        return fail(s, LBM_ERR_ALLOC, "hipMalloc of the FP64 exchange buffer failed");
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const size_t n = (size_t)NQ * s->nx * s->ny;
    HIP_TRY(s, hipMemcpy(s->staging, f, n * 8, hipMemcpyHostToDevice));
    const int p = (int)(s->host_step & 1);
    dispatch(s->storage, [&](auto* tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        Launch<S>::set_pop(s->desc, s->staging, p, s->stream);
        return 0;
    });
    HIP_TRY(s, hipGetLastError());
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

int lbm_get_populations(lbm_sim* s, double* f) {
    if (!s || !f) return fail(s, LBM_ERR_ARG, "NULL argument");
    if (ensure_staging(s) != hipSuccess)
        return fail(s, LBM_ERR_ALLOC, "hipMalloc of the FP64 exchange buffer failed");
    const int p = (int)(s->host_step & 1);
    dispatch(s->storage, [&](auto* tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        Launch<S>::get_pop(s->desc, s->staging, p, s->stream);
        return 0;
    });
    HIP_TRY(s, hipGetLastError());
    int rc = sync_check(s);
    HIP_TRY(s, hipMemcpy(f, s->staging, (size_t)NQ * s->nx * s->ny * 8, hipMemcpyDeviceToHost));
    return rc;
}

int lbm_get_body_state(lbm_sim* s, double* q, double* v) {
    if (!s || !q || !v) return fail(s, LBM_ERR_ARG, "NULL argument");
    int rc = sync_check(s);
    BodyDev B;
    HIP_TRY(s, hipMemcpy(&B, s->body_d, sizeof(B), hipMemcpyDeviceToHost));
    const int p = (int)(s->host_step & 1);
    for (int k = 0; k < 3; ++k) {
        q[k] = B.st[p].q[k];
        v[k] = B.st[p].v[k];
    }
    return rc;
}

// ---- launch configuration and its autotuning ---------------------------------------
static int apply_launch_config(lbm_sim* s, int rows, bool nt, int tile_w) {
    int rc0 = sync_check(s);  // the next step's state is then fresh
    if (rc0 && rc0 != LBM_ERR_UNSTABLE) return rc0;
    const int tile_h = rows * tile_stack(tile_w);
    s->rows = rows;
    s->nt = nt;
    s->desc.rows = tile_h;
    s->desc.tiles_y = (s->ny + tile_h - 1) / tile_h;
    s->desc.tile_w = tile_w;
    s->desc.tiles_x = (s->nx + tile_w - 1) / tile_w;
    BodyDev B;
    HIP_TRY(s, hipMemcpy(&B, s->body_d, sizeof(B), hipMemcpyDeviceToHost));
    // the boxes of the final state and of the one before it (by which the next step takes
    // part), in the new tiles
    BodyState& st = B.st[s->host_step & 1];
    BodyState& before = B.st[(s->host_step & 1) ^ 1];
    body_tiles(s->nx, s->ny, tile_h, tile_w, B, st.q[0], st.q[1], st.boxM);
    body_tiles(s->nx, s->ny, tile_h, tile_w, B, before.q[0], before.q[1], before.boxM);
    for (int k = 0; k < 4; ++k) st.part_box[k] = before.boxM[k];
    s->row_shift = dispatch_row_shift(s, st.boxM);
    HIP_TRY(s, hipMemcpy(s->body_d, &B, sizeof(B), hipMemcpyHostToDevice));
    int rc = upload_desc(s);
    if (rc) return rc;
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    drop_graph(s);
    update_finalize(s);
    return LBM_OK;
}

// The autotuners' choice among timed candidates: of those within 1 % of the fastest,
// the one of lowest rank (rank orders narrower tiles first, then fewer rows per lane,
// plain stores before nontemporal ones, the body state finalized in the tiles before
// the extra launch).  Candidates that close are equal within the timing's spread, and
// narrower tiles read fewer bytes (the cache lines that x-shifted pulls straddle are
// shared by tiles that run one after the other on one XCD); the rule also keeps the
// choice from changing with the spread from one run to the next.
constexpr double TUNE_TIE = 0.01;
static int pick_near_fastest(const double* us, const int* rank, int n) {
    double fastest = us[0];
    for (int k = 1; k < n; ++k) fastest = std::min(fastest, us[k]);
    int pick = -1;
    for (int k = 0; k < n; ++k)
        if (us[k] <= fastest * (1.0 + TUNE_TIE) && (pick < 0 || rank[k] < rank[pick])) pick = k;
    return pick;
}

static std::string tune_key(const lbm_sim* s) {
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    char buf[128];
    std::snprintf(buf, sizeof(buf), "%s/s%d/%dx%d", arch.c_str(), s->storage, s->nx, s->ny);
    return buf;
}

// Cache lines: {"key": "<arch>/s<storage>/<nx>x<ny>", "rows": r, "nt": 0|1, "tile": w,
// "us": t, "fin": f}; lines without "tile" (an earlier format) stand for 256-column tiles;
// "fin" (LBM_FINALIZE_TILES or _KERNEL) is present when a body took part in the timing.
static bool tune_lookup(const char* path, const std::string& key, int& rows, int& nt, int& tile_w,
                        int& fin) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[256];
        int r = 0, n = 0, w = TILE_X;
        double us = 0;
        const bool with_tile =
            std::sscanf(line, " {\"key\": \"%255[^\"]\", \"rows\": %d, \"nt\": %d, \"tile\": %d, \"us\": %lf",
                        k, &r, &n, &w, &us) == 5;
        if (!with_tile) {
            w = TILE_X;
            if (std::sscanf(line, " {\"key\": \"%255[^\"]\", \"rows\": %d, \"nt\": %d, \"us\": %lf", k,
                            &r, &n, &us) != 4)
                continue;
        }
        int fm = LBM_FINALIZE_AUTO;
        const char* fp = std::strstr(line, "\"fin\": ");
        if (fp && std::sscanf(fp, "\"fin\": %d", &fm) != 1) fm = LBM_FINALIZE_AUTO;
        if (key == k && (r == 1 || r == 2 || r == 4) && (n == 0 || n == 1) &&
            (w == TILE_NARROW || w == TILE_X || w == TILE_WIDE) && fm >= LBM_FINALIZE_AUTO &&
            fm <= LBM_FINALIZE_KERNEL) {
            rows = r;
            nt = n;
            tile_w = w;
            fin = fm;
            found = true;  // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

int lbm_autotune(lbm_sim* s, int trial_steps, const char* cache_path, int* rows_out, int* nt_out,
                 double* us_out) {
    if (!s || trial_steps < 1) return fail(s, LBM_ERR_ARG, "bad argument");
    if (s->in_batch) return reject_member(s);
    const std::string key = tune_key(s);
    int rows = 0, nt = 0, tile_w = TILE_X, fin = LBM_FINALIZE_AUTO;
    double best = -1.0;
    if (!(cache_path && tune_lookup(cache_path, key, rows, nt, tile_w, fin))) {
        // candidates are timed from this simulation's current state, not from the uniform
        // start (whose exactly-zero offsets the memory system moves faster)
        HIP_TRY(s, hipStreamSynchronize(s->stream));
        const int cur = (int)(s->host_step & 1);
        const size_t outlet_bytes = 3 * (size_t)s->ny * (s->storage == LBM_FP64 ? 8 : 4);
        const int cand_rows[3] = {1, 2, 4};
        const int cand_w[3] = {TILE_NARROW, TILE_X, TILE_WIDE};
        // with a body, both ways of finalizing its state are timed
        const int cand_fin[2] = {LBM_FINALIZE_TILES, LBM_FINALIZE_KERNEL};
        const int ncand = s->has_body ? 36 : 18;
        double cand_us[36];
        for (int cj = 0; cj < ncand; ++cj) {
            const int ci = cj % 18;
            lbm_opts o = s->opts;
            o.hip_stream = nullptr;
            o.pop_buffers[0] = o.pop_buffers[1] = nullptr;
            o.history_cap = 64;
            o.rows_per_tile = cand_rows[(ci / 2) % 3];
            o.store_mode = (ci & 1) ? LBM_STORE_NONTEMPORAL : LBM_STORE_PLAIN;
            o.tile_width = cand_w[ci / 6];
            o.finalize = s->has_body ? cand_fin[cj / 18] : s->fin_req;
            lbm_sim* t = nullptr;
            int rc = lbm_create(s->nx, s->ny, s->rates, s->eta, &o, &t);
            if (rc) return fail(s, rc, std::string("autotune: ") + lbm_last_error(nullptr));
            if (s->has_body && lbm_set_body(t, &s->body_desc) != LBM_OK) {
                lbm_destroy(t);
                return fail(s, LBM_ERR_HIP, "autotune: body");
            }
            // timed as the steps are meant to run, replayed from a captured graph of gs
            // steps (after four eager ones, so that each replay starts on an even step);
            // the faster of two replays
            const int gs = std::max(2, trial_steps & ~1);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            float ms = 0.f, best_ms = -1.f;
            bool ok = hipMemcpyAsync(t->pop[0], s->pop[cur], s->pop_bytes, hipMemcpyDeviceToDevice,
                                     t->stream) == hipSuccess &&
                      hipMemcpyAsync(t->outlet, s->outlet, outlet_bytes, hipMemcpyDeviceToDevice,
                                     t->stream) == hipSuccess &&
                      lbm_step(t, 4) == LBM_OK && lbm_set_graph_steps(t, gs) == LBM_OK &&
                      lbm_step(t, gs) == LBM_OK && hipEventCreate(&e0) == hipSuccess &&
                      hipEventCreate(&e1) == hipSuccess;
            for (int rep = 0; ok && rep < 2; ++rep) {
                ok = hipEventRecord(e0, t->stream) == hipSuccess && lbm_step(t, gs) == LBM_OK &&
                     hipEventRecord(e1, t->stream) == hipSuccess &&
                     hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                if (ok && (best_ms < 0.f || ms < best_ms)) best_ms = ms;
            }
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            lbm_destroy(t);
            if (!ok) return fail(s, LBM_ERR_HIP, "autotune: timing run failed");
            cand_us[cj] = 1e3 * best_ms / gs;
        }
        // candidate cj: tile width cj % 18 / 6, rows (cj % 18 / 2) % 3, store cj % 2,
        // finalization cj / 18
        int rank[36];
        for (int k = 0; k < ncand; ++k) rank[k] = 2 * (k % 18) + k / 18;
        const int cj = pick_near_fastest(cand_us, rank, ncand), ci = cj % 18;
        best = cand_us[cj];
        rows = cand_rows[(ci / 2) % 3];
        nt = ci & 1;
        tile_w = cand_w[ci / 6];
        fin = s->has_body ? cand_fin[cj / 18] : LBM_FINALIZE_AUTO;
        if (cache_path) {
            FILE* f = std::fopen(cache_path, "a");
            if (f) {
                if (s->has_body)
                    std::fprintf(f, "{\"key\": \"%s\", \"rows\": %d, \"nt\": %d, \"tile\": %d, \"us\": %.3f, \"fin\": %d}\n",
                                 key.c_str(), rows, nt, tile_w, best, fin);
                else
                    std::fprintf(f, "{\"key\": \"%s\", \"rows\": %d, \"nt\": %d, \"tile\": %d, \"us\": %.3f}\n",
                                 key.c_str(), rows, nt, tile_w, best);
                std::fclose(f);
            }
        }
    }
    if (fin != LBM_FINALIZE_AUTO) s->fin_req = fin;
    int rc = apply_launch_config(s, rows, nt != 0, tile_w);
    if (rc) return rc;
    if (rows_out) *rows_out = rows;
    if (nt_out) *nt_out = nt;
    if (us_out) *us_out = best;
    return LBM_OK;
}

int lbm_launch_config(const lbm_sim* s, int* rows_out, int* nt_out, int* tile_width_out) {
    if (!s) return LBM_ERR_ARG;
    if (rows_out) *rows_out = s->rows;
    if (nt_out) *nt_out = s->nt ? 1 : 0;
    if (tile_width_out) *tile_width_out = s->desc.tile_w;
    return LBM_OK;
}

int lbm_layout(const lbm_sim* s, int* layout_out) {
    if (!s || !layout_out) return LBM_ERR_ARG;
    *layout_out = s->desc.layout;
    return LBM_OK;
}

int lbm_finalize_by_kernel(const lbm_sim* s, int* kernel_out) {
    if (!s || !kernel_out) return LBM_ERR_ARG;
    *kernel_out = s->sep_final ? 1 : 0;
    return LBM_OK;
}

// ---- save / load -------------------------------------------------------------------
struct SaveHeader {
    char magic[8];
    int version, nx, ny, storage, layout;
    long long host_step, drained;
    unsigned long long pop_bytes, outlet_bytes;
};

int lbm_save(lbm_sim* s, void* buf, size_t cap, size_t* size_out) {
    if (!s || !size_out) return fail(s, LBM_ERR_ARG, "NULL argument");
    const size_t tsz = s->storage == LBM_FP64 ? 8 : 4;
    const size_t ob = 3 * (size_t)s->ny * tsz;
    const size_t total = sizeof(SaveHeader) + s->pop_bytes + ob + sizeof(BodyDev);
    *size_out = total;
    if (!buf) return LBM_OK;
    if (cap < total) return fail(s, LBM_ERR_ARG, "buffer too small");
    int rc = sync_check(s);
    if (rc) return rc;
    SaveHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, "VPLBMS1", 8);
    h.version = 2;
    h.nx = s->nx;
    h.ny = s->ny;
    h.storage = s->storage;
    h.layout = s->desc.layout;
    h.host_step = s->host_step;
    h.drained = s->drained;
    h.pop_bytes = s->pop_bytes;
    h.outlet_bytes = ob;
    char* c = (char*)buf;
    std::memcpy(c, &h, sizeof(h));
    c += sizeof(h);
    HIP_TRY(s, hipMemcpy(c, s->pop[s->host_step & 1], s->pop_bytes, hipMemcpyDeviceToHost));
    c += s->pop_bytes;
    HIP_TRY(s, hipMemcpy(c, s->outlet, ob, hipMemcpyDeviceToHost));
    c += ob;
    HIP_TRY(s, hipMemcpy(c, s->body_d, sizeof(BodyDev), hipMemcpyDeviceToHost));
    return LBM_OK;
}

int lbm_load(lbm_sim* s, const void* buf, size_t size) {
    if (!s || !buf) return fail(s, LBM_ERR_ARG, "NULL argument");
    if (s->in_batch) return reject_member(s);
    if (size < sizeof(SaveHeader)) return fail(s, LBM_ERR_ARG, "buffer too small");
    SaveHeader h;
    std::memcpy(&h, buf, sizeof(h));
    const size_t tsz = s->storage == LBM_FP64 ? 8 : 4;
    const size_t ob = 3 * (size_t)s->ny * tsz;
    if (std::memcmp(h.magic, "VPLBMS1", 8) != 0 || h.version != 2 || h.nx != s->nx ||
        h.ny != s->ny || h.storage != s->storage || h.layout != s->desc.layout ||
        h.pop_bytes != s->pop_bytes ||
        h.outlet_bytes != ob || size < sizeof(h) + s->pop_bytes + ob + sizeof(BodyDev))
        return fail(s, LBM_ERR_ARG, "saved state does not match this simulation");
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const char* c = (const char*)buf + sizeof(h);
    s->host_step = h.host_step;
    s->drained = h.drained;
    HIP_TRY(s, hipMemcpy(s->pop[s->host_step & 1], c, s->pop_bytes, hipMemcpyHostToDevice));
    c += s->pop_bytes;
    HIP_TRY(s, hipMemcpy(s->outlet, c, ob, hipMemcpyHostToDevice));
    c += ob;
    BodyDev B;
    std::memcpy(&B, c, sizeof(B));
    // the save flushed the state (fresh); its participation box is in the saver's tiles,
    // which may differ from this simulation's
    BodyState& st = B.st[s->host_step & 1];
    BodyState& before = B.st[(s->host_step & 1) ^ 1];
    if (st.fresh && B.active) {
        body_tiles(s->nx, s->ny, s->desc.rows, s->desc.tile_w, B, st.q[0], st.q[1], st.boxM);
        body_tiles(s->nx, s->ny, s->desc.rows, s->desc.tile_w, B, before.q[0], before.q[1], before.boxM);
        for (int k = 0; k < 4; ++k) st.part_box[k] = before.boxM[k];
    }
    HIP_TRY(s, hipMemcpy(s->body_d, &B, sizeof(BodyDev), hipMemcpyHostToDevice));
    s->has_body = B.active != 0;
    s->body_h = B;
    update_finalize(s);
    s->row_shift = dispatch_row_shift(s, B.st[s->host_step & 1].boxM);
    if (!s->has_body) s->rec_end = s->drained = std::max(s->drained, s->host_step);
    HIP_TRY(s, hipMemset(s->flag, 0, sizeof(int)));
    drop_graph(s);
    return LBM_OK;
}

}  // extern "C"

// ---- batches of independent simulations -------------------------------------------------
struct lbm_batch {
    int n = 0;
    int storage = LBM_FP32;
    std::vector<lbm_sim*> sims;
    std::vector<lbm_batch_desc> in;  // creation inputs (for the autotuner's scratch batch)
    std::vector<lbm_opts> in_opts;
    std::vector<lbm_body> in_body;
    std::vector<int> has_body;
    lbm_batch_opts bopts{};
    SimDesc* descs_d = nullptr;
    int2* sched_d = nullptr;
    int nsched = 0;
    int order = LBM_ORDER_LARGEST_FIRST;
    int rows = 1;
    bool nt = false;
    int tile_w = TILE_X;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t host_step = 0;
    int graph_steps = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<int> fin_list;  // members whose body state is finalized by kernel
    int* fin_d = nullptr;       // fin_list on the device
    std::string err;
};

static thread_local std::string g_batch_create_error;

static int bfail(lbm_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    return code;
}

#define BHIP_TRY(b, expr)                                                               \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            (b)->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
            return LBM_ERR_HIP;                                                         \
        }                                                                               \
    } while (0)

static void batch_drop_graph(lbm_batch* b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

// Work list of one step: every tile of every simulation once, in the chosen order.
static std::vector<int2> batch_schedule(const lbm_batch* b, int order) {
    std::vector<int> idx(b->n);
    for (int i = 0; i < b->n; ++i) idx[i] = i;
    auto tiles = [&](int i) {
        return (long long)b->sims[i]->desc.tiles_x * b->sims[i]->desc.tiles_y;
    };
    if (order == LBM_ORDER_LARGEST_FIRST)
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return tiles(a) > tiles(c); });
    std::vector<int2> out;
    if (b->tile_w == TILE_NARROW) {
        // The tile rows of every simulation, in the chosen order (each simulation's rows
        // rotated to put its body's rows early, as below), are dealt out to eight queues,
        // each row whole to the queue holding the fewest tiles so far; entry 8 k + x of
        // the schedule is the k-th tile of queue x.  Workgroup 8 k + x runs on XCD x, so
        // horizontally adjacent tiles, which share the cache lines their x-shifted pulls
        // straddle, run one after the other on one XCD.  Where a queue has run out, the
        // entry is a gap (simulation -1).
        std::vector<std::pair<int, int>> rows;  // (simulation, tile row)
        if (order == LBM_ORDER_INTERLEAVED) {
            int maxr = 0;
            for (int i = 0; i < b->n; ++i) maxr = std::max(maxr, b->sims[i]->desc.tiles_y);
            for (int r = 0; r < maxr; ++r)
                for (int i = 0; i < b->n; ++i)
                    if (r < b->sims[i]->desc.tiles_y) rows.emplace_back(i, r);
        } else {
            for (int i : idx) {
                const int ty = b->sims[i]->desc.tiles_y;
                for (int r0 = 0; r0 < ty; ++r0)
                    rows.emplace_back(i, (r0 + b->sims[i]->row_shift) % ty);
            }
        }
        std::vector<int2> q[8];
        for (const auto& rw : rows) {
            int x = 0;
            for (int k = 1; k < 8; ++k)
                if (q[k].size() < q[x].size()) x = k;
            for (int c = 0; c < b->sims[rw.first]->desc.tiles_x; ++c)
                q[x].push_back(make_int2(rw.first, (rw.second << 16) | c));
        }
        size_t len = 0;
        for (const auto& v : q) len = std::max(len, v.size());
        out.assign(8 * len, make_int2(-1, 0));
        for (int x = 0; x < 8; ++x)
            for (size_t k = 0; k < q[x].size(); ++k) out[8 * k + x] = q[x][k];
        while (!out.empty() && out.back().x < 0) out.pop_back();
        return out;
    }
    if (order == LBM_ORDER_INTERLEAVED) {
        // one row of tiles from each simulation in turn
        int maxr = 0;
        for (int i = 0; i < b->n; ++i) maxr = std::max(maxr, b->sims[i]->desc.tiles_y);
        for (int r = 0; r < maxr; ++r)
            for (int i = 0; i < b->n; ++i) {
                const SimDesc& d = b->sims[i]->desc;
                if (r >= d.tiles_y) continue;
                for (int x = 0; x < d.tiles_x; ++x)
                    out.push_back(make_int2(i, (r << 16) | ((x + r) % d.tiles_x)));
            }
        return out;
    }
    for (int i : idx) {
        const SimDesc& d = b->sims[i]->desc;
        for (int r0 = 0; r0 < d.tiles_y; ++r0) {
            const int r = (r0 + b->sims[i]->row_shift) % d.tiles_y;  // body rows early
            // columns skewed by the row, as in a single launch: consecutive entries go to
            // the eight XCDs in turn, and each tile column then visits all of them
            for (int x = 0; x < d.tiles_x; ++x)
                out.push_back(make_int2(i, (r << 16) | ((x + r0) % d.tiles_x)));
        }
    }
    return out;
}

// The members that finalize their body state by kernel share one launch after each
// step; the list follows their bodies (lbm_set_body on a member may change it).
static int batch_fin_refresh(lbm_batch* b) {
    std::vector<int> l;
    for (int i = 0; i < b->n; ++i)
        if (b->sims[i]->sep_final) l.push_back(i);
    if (l == b->fin_list && (b->fin_d || l.empty())) return LBM_OK;
    BHIP_TRY(b, hipStreamSynchronize(b->stream));  // no launch in flight reads the old list
    batch_drop_graph(b);
    if (b->fin_d) (void)hipFree(b->fin_d);
    b->fin_d = nullptr;
    b->fin_list = l;
    if (!l.empty()) {
        BHIP_TRY(b, hipMalloc((void**)&b->fin_d, l.size() * sizeof(int)));
        BHIP_TRY(b, hipMemcpy(b->fin_d, l.data(), l.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    return LBM_OK;
}

static int batch_upload(lbm_batch* b) {
    std::vector<SimDesc> ds(b->n);
    for (int i = 0; i < b->n; ++i) ds[i] = b->sims[i]->desc;
    BHIP_TRY(b, hipMemcpy(b->descs_d, ds.data(), ds.size() * sizeof(SimDesc), hipMemcpyHostToDevice));
    std::vector<int2> sc = batch_schedule(b, b->order);
    if (b->sched_d) (void)hipFree(b->sched_d);
    b->sched_d = nullptr;
    BHIP_TRY(b, hipMalloc((void**)&b->sched_d, sc.size() * sizeof(int2)));
    BHIP_TRY(b, hipMemcpy(b->sched_d, sc.data(), sc.size() * sizeof(int2), hipMemcpyHostToDevice));
    b->nsched = (int)sc.size();
    batch_drop_graph(b);
    return batch_fin_refresh(b);
}

static int batch_launch(lbm_batch* b) {
    const int p = (int)(b->host_step & 1);
    dispatch(b->storage, [&](auto* tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        Launch<S>::step_batch(b->descs_d, b->sched_d, b->nsched, b->rows, b->nt, b->tile_w, p,
                              b->stream);
        return 0;
    });
    if (!b->fin_list.empty())
        hipLaunchKernelGGL(k_finalize_batch, dim3((unsigned)b->fin_list.size()), dim3(TILE_X), 0,
                           b->stream, b->descs_d, b->fin_d, p ^ 1);
    BHIP_TRY(b, hipGetLastError());
    b->host_step += 1;
    for (lbm_sim* s : b->sims) s->host_step += 1;
    return LBM_OK;
}

static void batch_free(lbm_batch* b) {
    batch_drop_graph(b);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (lbm_sim* s : b->sims)
        if (s) free_sim(s);
    if (b->descs_d) (void)hipFree(b->descs_d);
    if (b->sched_d) (void)hipFree(b->sched_d);
    if (b->fin_d) (void)hipFree(b->fin_d);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

extern "C" {

void lbm_default_batch_opts(lbm_batch_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->storage = LBM_FP32;
    o->order = LBM_ORDER_LARGEST_FIRST;
}

const char* lbm_batch_last_error(const lbm_batch* b) {
    return b ? b->err.c_str() : g_batch_create_error.c_str();
}

int lbm_batch_create(int n, const lbm_batch_desc* descs, const lbm_batch_opts* opts,
                     lbm_batch** out) {
    if (!out || !descs || n < 1) return g_batch_create_error = "bad argument", LBM_ERR_ARG;
    *out = nullptr;
    lbm_batch_opts bo;
    if (opts)
        bo = *opts;
    else
        lbm_default_batch_opts(&bo);
    if (bo.order < LBM_ORDER_GIVEN || bo.order > LBM_ORDER_INTERLEAVED)
        return g_batch_create_error = "unknown order", LBM_ERR_ARG;
    if (bo.store_mode < LBM_STORE_AUTO || bo.store_mode > LBM_STORE_NONTEMPORAL)
        return g_batch_create_error = "unknown store mode", LBM_ERR_ARG;
    if (bo.storage < LBM_FP64 || bo.storage > LBM_BF16_OFS)
        return g_batch_create_error = "unknown storage", LBM_ERR_ARG;
    if (bo.rows_per_tile != 0 && bo.rows_per_tile != 1 && bo.rows_per_tile != 2 && bo.rows_per_tile != 4)
        return g_batch_create_error = "rows_per_tile must be 0, 1, 2 or 4", LBM_ERR_ARG;
    if (bo.tile_width != 0 && bo.tile_width != TILE_NARROW && bo.tile_width != TILE_X &&
        bo.tile_width != TILE_WIDE)
        return g_batch_create_error = "tile_width must be 0, 64, 256 or 512", LBM_ERR_ARG;
    if (bo.layout < LBM_LAYOUT_AUTO || bo.layout > LBM_LAYOUT_PLANES)
        return g_batch_create_error = "unknown layout", LBM_ERR_ARG;
    if (bo.finalize < LBM_FINALIZE_AUTO || bo.finalize > LBM_FINALIZE_KERNEL)
        return g_batch_create_error = "unknown finalize mode", LBM_ERR_ARG;
    lbm_batch* b = new lbm_batch();
    b->n = n;
    b->storage = bo.storage;
    b->bopts = bo;
    b->order = bo.order;
    auto bail = [&](int code) {
        g_batch_create_error = b->err;
        batch_free(b);
        return code;
    };
    if (bo.hip_stream) {
        b->stream = (hipStream_t)bo.hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return b->err = hipGetErrorString(e), bail(LBM_ERR_HIP);
        b->own_stream = true;
    }
    b->in.assign(descs, descs + n);
    b->in_opts.resize(n);
    b->in_body.resize(n);
    b->has_body.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        lbm_opts o;
        if (descs[i].opts)
            o = *descs[i].opts;
        else
            lbm_default_opts(&o);
        o.storage = bo.storage;
        o.hip_stream = b->stream;
        o.pop_buffers[0] = o.pop_buffers[1] = nullptr;
        o.rows_per_tile = bo.rows_per_tile;
        o.store_mode = bo.store_mode;
        o.tile_width = bo.tile_width;
        if (bo.layout != LBM_LAYOUT_AUTO) o.layout = bo.layout;
        if (bo.finalize != LBM_FINALIZE_AUTO) o.finalize = bo.finalize;
        b->in_opts[i] = o;
        if (descs[i].body) {
            b->in_body[i] = *descs[i].body;
            b->has_body[i] = 1;
        }
        lbm_sim* s = nullptr;
        int rc = lbm_create(descs[i].nx, descs[i].ny, descs[i].rates, descs[i].eta, &o, &s);
        if (rc) return b->err = "simulation " + std::to_string(i) + ": " + lbm_last_error(nullptr), bail(rc);
        s->in_batch = true;
        b->sims.push_back(s);
        if (descs[i].body) {
            rc = lbm_set_body(s, descs[i].body);
            if (rc) return b->err = "simulation " + std::to_string(i) + ": " + s->err, bail(rc);
        }
        // schedule entries hold 16-bit tile coordinates, in every tile shape
        if ((s->nx + TILE_NARROW - 1) / TILE_NARROW > 0xffff || s->ny > 0x7fff)
            return b->err = "grid too large for a batch", bail(LBM_ERR_ARG);
    }
    // one launch configuration for the whole batch; the defaults follow the single-grid
    // rules applied to the batch's total size
    size_t bytes = 0;
    for (lbm_sim* s : b->sims) bytes += s->pop_bytes;
    b->rows = bo.rows_per_tile ? bo.rows_per_tile : 1;
    b->nt = bo.store_mode == LBM_STORE_NONTEMPORAL ||
            (bo.store_mode == LBM_STORE_AUTO && 2 * bytes > (size_t(1) << 30));
    b->tile_w = bo.tile_width ? bo.tile_width : TILE_X;
    for (lbm_sim* s : b->sims) {
        int rc = apply_launch_config(s, b->rows, b->nt, b->tile_w);
        if (rc) return b->err = s->err, bail(rc);
    }
    hipError_t e = hipMalloc((void**)&b->descs_d, (size_t)n * sizeof(SimDesc));
    if (e != hipSuccess) return b->err = hipGetErrorString(e), bail(LBM_ERR_ALLOC);
    int rc = batch_upload(b);
    if (rc) return bail(rc);
    *out = b;
    return LBM_OK;
}

int lbm_batch_order(const lbm_batch* b, int* order_out) {
    if (!b || !order_out) return LBM_ERR_ARG;
    *order_out = b->order;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_ERR_ARG;
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    return LBM_OK;
}

int lbm_batch_size(const lbm_batch* b) { return b ? b->n : -1; }

int lbm_batch_sim(lbm_batch* b, int i, lbm_sim** out) {
    if (!b || !out || i < 0 || i >= b->n) return bfail(b, LBM_ERR_ARG, "bad argument");
    *out = b->sims[i];
    return LBM_OK;
}

int lbm_batch_set_graph_steps(lbm_batch* b, int k) {
    if (!b) return LBM_ERR_ARG;
    if (k != 0 && (k < 2 || (k & 1))) return bfail(b, LBM_ERR_ARG, "graph steps must be 0 or even >= 2");
    batch_drop_graph(b);
    b->graph_steps = k;
    return LBM_OK;
}

static int batch_capture(lbm_batch* b) {
    const int64_t saved = b->host_step;
    std::vector<int64_t> saved_s(b->n);
    for (int i = 0; i < b->n; ++i) saved_s[i] = b->sims[i]->host_step;
    b->host_step = 0;
    BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = LBM_OK;
    for (int k = 0; k < b->graph_steps && rc == LBM_OK; ++k) rc = batch_launch(b);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    b->host_step = saved;
    for (int i = 0; i < b->n; ++i) b->sims[i]->host_step = saved_s[i];
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return bfail(b, LBM_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
    b->graph = g;
    BHIP_TRY(b, hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int64_t n) {
    if (!b) return LBM_ERR_ARG;
    if (n < 0) return bfail(b, LBM_ERR_ARG, "n must be >= 0");
    for (lbm_sim* s : b->sims)
        if (s->host_step != b->host_step)
            return bfail(b, LBM_ERR_STATE, "a simulation of the batch was stepped on its own");
    int frc = batch_fin_refresh(b);
    if (frc) return frc;
    int64_t done = 0;
    if (b->graph_steps > 0 && n >= b->graph_steps) {
        if (b->host_step & 1) {
            int rc = batch_launch(b);
            if (rc) return rc;
            ++done;
        }
        if (!b->gexec) {
            int rc = batch_capture(b);
            if (rc) return rc;
        }
        while (n - done >= b->graph_steps) {
            BHIP_TRY(b, hipGraphLaunch(b->gexec, b->stream));
            b->host_step += b->graph_steps;
            for (lbm_sim* s : b->sims) s->host_step += b->graph_steps;
            done += b->graph_steps;
        }
    }
    for (; done < n; ++done) {
        int rc = batch_launch(b);
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_batch_sync(lbm_batch* b) {
    if (!b) return LBM_ERR_ARG;
    int worst = LBM_OK;
    for (lbm_sim* s : b->sims) {
        int rc = sync_check(s);
        if (rc == LBM_ERR_UNSTABLE && worst == LBM_OK) worst = rc;
        if (rc && rc != LBM_ERR_UNSTABLE) return bfail(b, rc, s->err);
    }
    return worst;
}

static int batch_apply(lbm_batch* b, int rows, bool nt, int order, int tile_w, int fin) {
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    for (lbm_sim* s : b->sims) {
        if (fin != LBM_FINALIZE_AUTO) s->fin_req = fin;
        int rc = apply_launch_config(s, rows, nt, tile_w);
        if (rc) return bfail(b, rc, s->err);
    }
    b->rows = rows;
    b->nt = nt;
    b->order = order;
    b->tile_w = tile_w;
    return batch_upload(b);
}

// Times trial_steps steps of a scratch copy of the batch for each candidate.
static int batch_time(lbm_batch* b, int rows, bool nt, int order, int tile_w, int fin,
                      int trial_steps, double& us) {
    lbm_batch_opts bo = b->bopts;
    bo.finalize = fin;
    bo.hip_stream = nullptr;
    bo.rows_per_tile = rows;
    bo.store_mode = nt ? LBM_STORE_NONTEMPORAL : LBM_STORE_PLAIN;
    bo.order = order;
    bo.tile_width = tile_w;
    std::vector<lbm_batch_desc> ds = b->in;
    for (int i = 0; i < b->n; ++i) {
        b->in_opts[i].history_cap = 64;
        b->in_opts[i].finalize = b->sims[i]->fin_req;  // as the member stands now
        ds[i].opts = &b->in_opts[i];
        ds[i].body = b->has_body[i] ? &b->in_body[i] : nullptr;
    }
    lbm_batch* t = nullptr;
    int rc = lbm_batch_create(b->n, ds.data(), &bo, &t);
    if (rc) return bfail(b, rc, std::string("autotune: ") + lbm_batch_last_error(nullptr));
    // the candidates run from the members' current states (see lbm_autotune)
    bool ok = hipStreamSynchronize(b->stream) == hipSuccess;
    for (int i = 0; ok && i < b->n; ++i) {
        const lbm_sim* m = b->sims[i];
        const size_t outlet_bytes = 3 * (size_t)m->ny * (m->storage == LBM_FP64 ? 8 : 4);
        ok = hipMemcpyAsync(t->sims[i]->pop[0], m->pop[m->host_step & 1], m->pop_bytes,
                            hipMemcpyDeviceToDevice, t->stream) == hipSuccess &&
             hipMemcpyAsync(t->sims[i]->outlet, m->outlet, outlet_bytes, hipMemcpyDeviceToDevice,
                            t->stream) == hipSuccess;
    }
    // replayed from a captured graph, as the steps are meant to run (see lbm_autotune);
    // the faster of two replays
    const int gs = std::max(2, trial_steps & ~1);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f, best_ms = -1.f;
    ok = ok && lbm_batch_step(t, 4) == LBM_OK && lbm_batch_set_graph_steps(t, gs) == LBM_OK &&
         lbm_batch_step(t, gs) == LBM_OK && hipEventCreate(&e0) == hipSuccess &&
         hipEventCreate(&e1) == hipSuccess;
    for (int rep = 0; ok && rep < 2; ++rep) {
        ok = hipEventRecord(e0, t->stream) == hipSuccess && lbm_batch_step(t, gs) == LBM_OK &&
             hipEventRecord(e1, t->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (ok && (best_ms < 0.f || ms < best_ms)) best_ms = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    lbm_batch_destroy(t);
    if (!ok) return bfail(b, LBM_ERR_HIP, "autotune: timing run failed");
    us = 1e3 * best_ms / gs;
    return LBM_OK;
}

int lbm_batch_autotune(lbm_batch* b, int trial_steps, int* rows_out, int* nt_out, int* order_out,
                       double* us_out) {
    if (!b || trial_steps < 1) return bfail(b, LBM_ERR_ARG, "bad argument");
    int best_rows = 1, best_order = LBM_ORDER_LARGEST_FIRST, best_w = TILE_X;
    int best_fin = LBM_FINALIZE_AUTO;
    bool best_nt = false;
    double best = -1.0, us = 0.0;
    const int cand_rows[3] = {1, 2, 4};
    const int cand_w[3] = {TILE_NARROW, TILE_X, TILE_WIDE};
    // two passes over the candidates, each keeping its faster pass: the first candidates
    // of a single pass run while the device is still reaching its working clocks
    double cand_us[18];
    for (int pass = 0; pass < 2; ++pass)
        for (int ci = 0; ci < 18; ++ci) {
            const int rows = cand_rows[(ci / 2) % 3], w = cand_w[ci / 6];
            int rc = batch_time(b, rows, ci & 1, LBM_ORDER_LARGEST_FIRST, w, LBM_FINALIZE_AUTO,
                                trial_steps, us);
            if (rc) return rc;
            cand_us[ci] = pass == 0 ? us : std::min(cand_us[ci], us);
        }
    int rank[18];
    for (int k = 0; k < 18; ++k) rank[k] = k;  // width ci / 6, rows (ci / 2) % 3, store ci % 2
    const int ci = pick_near_fastest(cand_us, rank, 18);
    best = cand_us[ci];
    best_rows = cand_rows[(ci / 2) % 3];
    best_nt = ci & 1;
    best_w = cand_w[ci / 6];
    for (int order : {LBM_ORDER_GIVEN, LBM_ORDER_INTERLEAVED}) {
        int rc = batch_time(b, best_rows, best_nt, order, best_w, LBM_FINALIZE_AUTO, trial_steps, us);
        if (rc) return rc;
        if (us < best) {
            best = us;
            best_order = order;
        }
    }
    bool any_body = false;
    for (int i = 0; i < b->n; ++i) any_body = any_body || b->has_body[i];
    if (any_body) {  // every member's state finalized in its tiles, or all by one launch
        for (int fin : {LBM_FINALIZE_TILES, LBM_FINALIZE_KERNEL}) {
            int rc = batch_time(b, best_rows, best_nt, best_order, best_w, fin, trial_steps, us);
            if (rc) return rc;
            if (us < best) {
                best = us;
                best_fin = fin;
            }
        }
    }
    int rc = batch_apply(b, best_rows, best_nt, best_order, best_w, best_fin);
    if (rc) return rc;
    if (rows_out) *rows_out = best_rows;
    if (nt_out) *nt_out = best_nt;
    if (order_out) *order_out = best_order;
    if (us_out) *us_out = best;
    return LBM_OK;
}

int lbm_batch_configure(lbm_batch* b, int rows, int store_mode, int order) {
    if (!b) return LBM_ERR_ARG;
    if (rows != 1 && rows != 2 && rows != 4) return bfail(b, LBM_ERR_ARG, "rows must be 1, 2 or 4");
    if (store_mode != LBM_STORE_PLAIN && store_mode != LBM_STORE_NONTEMPORAL)
        return bfail(b, LBM_ERR_ARG, "store mode must be PLAIN or NONTEMPORAL");
    if (order < LBM_ORDER_GIVEN || order > LBM_ORDER_INTERLEAVED) return bfail(b, LBM_ERR_ARG, "unknown order");
    return batch_apply(b, rows, store_mode == LBM_STORE_NONTEMPORAL, order, b->tile_w,
                       LBM_FINALIZE_AUTO);
}

}  // extern "C"
