// adjoint_host.hip -- host runtime of the reverse-mode path (lbm_adjoint_* of
// include/vplbm.h): checkpointed forward run, segment-wise recomputation and the
// adjoint sweep, reductions of the gradient.
//
// Forward: N steps of an internal simulation from a stored initial state; the state
// (populations and outflow memory) is copied aside every K steps and the objective
// J = sum_n (w_x F_x(n) + w_y F_y(n)) is summed in FP64 from the per-step records.
// Backward: for each segment, last first, the checkpoint is loaded, the K forward
// steps are recomputed into a segment store (one buffer per step), then the adjoint
// kernel runs over them in reverse.  One segment is captured once as a HIP graph and
// replayed for every segment; a device counter selects the checkpoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "vplbm.h"
#include "vplbm_adjoint.hpp"
#include "vplbm_host.hpp"

using namespace vplbm;

namespace vplbm {

// Copies the checkpoint of segment *seg_index into the first slot of the segment
// store (populations and outflow memory), in 4-byte words.
__global__ void k_adj_load_segment(const AdjDesc* __restrict__ ap) {
    const AdjDesc& a = *ap;
    const long long s = *a.seg_index;
    const int* src = reinterpret_cast<const int*>(a.ckpt_pop + s * a.pop_bytes);
    int* dst = reinterpret_cast<int*>(a.seg_pop);
    const long long n = a.pop_bytes / 4;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        dst[k] = src[k];
    const int* so = reinterpret_cast<const int*>(a.ckpt_out + s * a.out_bytes);
    int* dout = reinterpret_cast<int*>(a.seg_out);
    const long long no = a.out_bytes / 4;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < no; k += stride)
        dout[k] = so[k];
}

// Moves the device segment counter to the previous segment (one thread).
__global__ void k_adj_next_segment(const AdjDesc* __restrict__ ap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *ap->seg_index -= 1;
}

// Sets n 4-byte words to zero.
__global__ void k_adj_zero(int* __restrict__ p, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = 0;
}

}  // namespace vplbm

struct lbm_adjoint {
    lbm_sim* sim = nullptr;
    int storage = LBM_FP32, nx = 0, ny = 0;
    int64_t steps = 0;
    int K = 0, nseg = 0;
    bool graphs = true;
    double wx = 0.0, wy = 0.0;
    lbm_body body{};
    size_t tsz = 4, out_bytes = 0;
    AdjDesc ad{};
    // Two segment stores: the backward sweep over segment m (reading one store) runs
    // alongside the recomputation of segment m - 1 (writing the other) on a second stream.
    AdjDesc* ad_d = nullptr;        // adjoint descriptors of store 0 and store 1 (two)
    SimDesc* seg_descs_d = nullptr; // forward step descriptors: K for store 0, then K for 1
    char* def_pop = nullptr;  // the uniform initial state of lbm_create
    char* def_out = nullptr;
    char* init_pop = nullptr;  // initial state of the forward run
    char* init_out = nullptr;
    char* ckpt_pop = nullptr;
    char* ckpt_out = nullptr;
    char* seg_pop = nullptr;  // store 0; store 1 follows it (2 (K + 1) buffers in all)
    char* seg_out = nullptr;
    void* abar[2] = {nullptr, nullptr};
    void* chibar = nullptr;
    double* tile_acc = nullptr;
    RingSlot* ring = nullptr;
    int* ring_kn = nullptr;  // per edge node: its longest reader list (slots it must visit)
    int ring_k = 1;
    int* seg_index = nullptr;
    double* red = nullptr;
    int atx = 0;  // adjoint tiles along x (one row per tile)
    bool fwd_done = false, bwd_done = false;
    double J = 0.0;
    std::vector<lbm_force_rec> recs;
    hipStream_t aux = nullptr;  // the recomputation's stream
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};  // one backward stage per parity of m
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    std::string err;
};

namespace {

thread_local std::string g_adj_create_error;

int afail(lbm_adjoint* A, int code, const std::string& msg) {
    if (A) A->err = msg;
    return code;
}

#define AHIP_TRY(A, expr)                                                               \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            (A)->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
            return LBM_ERR_HIP;                                                         \
        }                                                                               \
    } while (0)

// One population read by a pull: (node, direction) and its coefficient.
struct Src {
    int i, j, a;
    double coef;
};

// Populations that the value pulled by node (i, j) for direction a is made of, through
// the boundary rules of the step (the x rule first, then the y rule).  The outflow
// rule contributes its value one node in, with weight U_c / (1 + U_c); its memory term
// is handled by the adjoint kernel.  Constant terms (moving walls) do not enter.
void resolve_pull(const int bc[4], int nx, int ny, double uc, int a, int i, int j, double coef,
                  std::vector<Src>& out) {
    int si = i - dir_cx(a), sj = j - dir_cy(a), dir = a;
    if (si < 0 || si >= nx) {
        const int kind = bc[si < 0 ? 0 : 1];
        if (kind == BC_PERIODIC) {
            si += si < 0 ? nx : -nx;
        } else if (kind == BC_SYMMETRY) {
            dir = dir_flip_x(a);
            si = i;
        } else if (kind == BC_OUTFLOW) {
            resolve_pull(bc, nx, ny, uc, a, nx - 2, j, coef * uc / (1.0 + uc), out);
            return;
        } else {
            out.push_back({i, j, dir_opp(a), coef});
            return;
        }
    }
    if (sj < 0 || sj >= ny) {
        const int kind = bc[sj < 0 ? 2 : 3];
        if (kind == BC_PERIODIC) {
            sj += sj < 0 ? ny : -ny;
        } else if (kind == BC_SYMMETRY) {
            dir = dir_flip_y(dir);
            sj = j;
        } else {
            out.push_back({i, j, dir_opp(a), coef});
            return;
        }
    }
    out.push_back({si, sj, dir, coef});
}

// Readers of every population of the edge nodes: the transpose of the pull there.
// Every reader of an edge population lies within one node of the edge (or on the
// opposite edge for periodic sides), so the nodes of the two outer rings are scanned.
void build_ring(const int bc[4], int nx, int ny, double uc, long long ps, int pitch,
                std::vector<RingSlot>& slots, std::vector<int>& kn, int& K) {
    const int nr = ring_count(nx, ny);
    std::vector<std::vector<RingEntry>> lists((size_t)nr * NQ);
    std::vector<Src> srcs;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (!(i <= 1 || i >= nx - 2 || j <= 1 || j >= ny - 2)) continue;
            for (int a = 0; a < NQ; ++a) {
                srcs.clear();
                resolve_pull(bc, nx, ny, uc, a, i, j, 1.0, srcs);
                for (const Src& s : srcs) {
                    const int r = ring_index(nx, ny, s.i, s.j);
                    if (r >= 0) lists[(size_t)r * NQ + s.a].push_back({i, j, a, 0, s.coef});
                }
            }
        }
    // fixed width: K slots per (node, direction), the longest list; the rest padded with
    // weight 0 (index 0)
    K = 1;
    for (const auto& l : lists) K = std::max<int>(K, (int)l.size());
    // slots an edge node visits: its longest list over the nine directions (at least one)
    kn.assign((size_t)nr, 1);
    for (int r = 0; r < nr; ++r)
        for (int a = 0; a < NQ; ++a) kn[r] = std::max<int>(kn[r], (int)lists[(size_t)r * NQ + a].size());
    slots.assign(lists.size() * (size_t)K, RingSlot{0, 0.0});
    for (size_t q = 0; q < lists.size(); ++q)
        for (size_t k = 0; k < lists[q].size(); ++k) {
            const RingEntry& re = lists[q][k];
            slots[q * K + k] = RingSlot{(long long)re.a * ps + (long long)re.j * pitch + re.i, re.coef};
        }
}

// Pose-dependent parts of the adjoint descriptor.
void set_pose(lbm_adjoint* A) {
    const lbm_body& b = A->body;
    AdjDesc& ad = A->ad;
    ad.pose[0] = b.x;
    ad.pose[1] = b.y;
    ad.pose[2] = b.theta;
    ad.pose[3] = b.vx;
    ad.pose[4] = b.vy;
    ad.pose[5] = b.omega;
    const BodyDev& B = A->sim->body_h;
    int nb[4];
    body_tiles(A->nx, A->ny, 1, TILE_X, B, b.x, b.y, nb, 1.0);  // adjoint tiles: one row each
    ad.box[0] = nb[0];
    ad.box[1] = nb[1];
    ad.box[2] = nb[2];
    ad.box[3] = nb[3];
    const double reach = B.reach;
    ad.nbox[0] = std::max(0, (int)std::floor(b.x - reach) - 1);
    ad.nbox[1] = std::min(A->nx - 1, (int)std::ceil(b.x + reach) + 1);
    ad.nbox[2] = std::max(0, (int)std::floor(b.y - reach) - 1);
    ad.nbox[3] = std::min(A->ny - 1, (int)std::ceil(b.y + reach) + 1);
}

// The adjoint descriptors of the two segment stores (they differ in the store only).
int upload_ad(lbm_adjoint* A) {
    AdjDesc two[2] = {A->ad, A->ad};
    two[1].seg_pop = A->ad.seg_pop + (A->K + 1) * A->ad.seg_stride;
    two[1].seg_out = A->ad.seg_out + (A->K + 1) * A->ad.out_stride;
    AHIP_TRY(A, hipMemcpy(A->ad_d, two, sizeof(two), hipMemcpyHostToDevice));
    return LBM_OK;
}

int zero_words(lbm_adjoint* A, void* p, size_t bytes) {
    const long long n = (long long)(bytes / 4);
    const int blocks = (int)std::min<long long>(2048, (n + 255) / 256);
    hipLaunchKernelGGL(k_adj_zero, dim3(std::max(blocks, 1)), dim3(256), 0, A->sim->stream,
                       reinterpret_cast<int*>(p), n);
    AHIP_TRY(A, hipGetLastError());
    return LBM_OK;
}

// Recomputation of the segment the device counter names, into segment store `store`:
// checkpoint -> slot 0, K forward steps (slot i -> i + 1), then the counter moves to the
// previous segment.  Enqueued on stream st.
int enqueue_recompute(lbm_adjoint* A, int store, hipStream_t st) {
    lbm_sim* s = A->sim;
    const long long words = (long long)(s->pop_bytes / 4);
    const int blocks = (int)std::min<long long>(4096, (words + 255) / 256);
    hipLaunchKernelGGL(k_adj_load_segment, dim3(blocks), dim3(256), 0, st, A->ad_d + store);
    const dim3 fgrid = step_grid(s->desc);
    const SimDesc* sd = A->seg_descs_d + (size_t)store * A->K;
    dispatch(A->storage, [&](auto* tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        for (int i = 0; i < A->K; ++i)
            Launch<S>::step(sd + i, fgrid, s->rows, s->nt, s->desc.tile_w, i & 1, st, s->row_shift);
        return 0;
    });
    hipLaunchKernelGGL(k_adj_next_segment, dim3(1), dim3(64), 0, st, A->ad_d);
    AHIP_TRY(A, hipGetLastError());
    return LBM_OK;
}

// Backward sweep over the segment held in store `store` (K adjoint steps, last first).
int enqueue_sweep(lbm_adjoint* A, int store, hipStream_t st) {
    lbm_sim* s = A->sim;
    const dim3 agrid(A->atx, A->ny);
    dispatch(A->storage, [&](auto* tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        if constexpr (std::is_same_v<S, double> || std::is_same_v<S, float>)
            for (int i = A->K - 1; i >= 0; --i) AdjLaunch<S>::step(s->desc_d, A->ad_d + store, agrid, i, st);
        return 0;
    });
    AHIP_TRY(A, hipGetLastError());
    return LBM_OK;
}

// Stage m of the backward run (m = nseg - 1 .. 1): the sweep over segment m (store
// m & 1) on the simulation's stream alongside the recomputation of segment m - 1 (the
// other store) on the second stream; the stage ends when both have.
int enqueue_stage(lbm_adjoint* A, int parity) {
    hipStream_t st = A->sim->stream;
    AHIP_TRY(A, hipEventRecord(A->ev_fork, st));
    AHIP_TRY(A, hipStreamWaitEvent(A->aux, A->ev_fork, 0));
    int rc = enqueue_recompute(A, parity ^ 1, A->aux);
    if (rc) return rc;
    rc = enqueue_sweep(A, parity, st);
    if (rc) return rc;
    AHIP_TRY(A, hipEventRecord(A->ev_join, A->aux));
    AHIP_TRY(A, hipStreamWaitEvent(st, A->ev_join, 0));
    return LBM_OK;
}

void drop_stage_graphs(lbm_adjoint* A) {
    for (int q = 0; q < 2; ++q) {
        if (A->gexec[q]) (void)hipGraphExecDestroy(A->gexec[q]);
        if (A->graph[q]) (void)hipGraphDestroy(A->graph[q]);
        A->gexec[q] = nullptr;
        A->graph[q] = nullptr;
    }
}

void adj_free(lbm_adjoint* A) {
    drop_stage_graphs(A);
    if (A->sim) (void)hipStreamSynchronize(A->sim->stream);
    if (A->aux) {
        (void)hipStreamSynchronize(A->aux);
        (void)hipStreamDestroy(A->aux);
    }
    if (A->ev_fork) (void)hipEventDestroy(A->ev_fork);
    if (A->ev_join) (void)hipEventDestroy(A->ev_join);
    void* bufs[] = {A->ad_d, A->seg_descs_d, A->def_pop, A->def_out, A->init_pop, A->init_out,
                    A->ckpt_pop, A->ckpt_out, A->seg_pop, A->seg_out, A->abar[0], A->abar[1],
                    A->chibar, A->tile_acc, A->ring, A->ring_kn, A->seg_index, A->red};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (A->sim) lbm_destroy(A->sim);
    delete A;
}

}  // namespace

extern "C" {

void lbm_default_adjoint_opts(lbm_adjoint_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->steps = 4000;
    o->checkpoint_every = 100;
    o->weight_fx = 1.0;
    o->weight_fy = 0.0;
    o->use_graphs = 1;
}

const char* lbm_adjoint_last_error(const lbm_adjoint* A) {
    return A ? A->err.c_str() : g_adj_create_error.c_str();
}

int lbm_adjoint_create(int nx, int ny, lbm_rates rates, double eta, const lbm_opts* opts,
                       const lbm_body* body, const lbm_adjoint_opts* aopts, lbm_adjoint** out) {
    if (!out || !body || !aopts) return g_adj_create_error = "NULL argument", LBM_ERR_ARG;
    *out = nullptr;
    const int64_t N = aopts->steps;
    const int K = aopts->checkpoint_every;
    if (N < 1) return g_adj_create_error = "steps must be >= 1", LBM_ERR_ARG;
    if (K < 2 || (K & 1)) return g_adj_create_error = "checkpoint_every must be even and >= 2", LBM_ERR_ARG;
    if (N % K) return g_adj_create_error = "steps must be a multiple of checkpoint_every", LBM_ERR_ARG;
    if (!std::isfinite(aopts->weight_fx) || !std::isfinite(aopts->weight_fy))
        return g_adj_create_error = "non-finite weights", LBM_ERR_ARG;
    if (body->mode != LBM_BODY_FIXED)
        return g_adj_create_error = "the adjoint needs a FIXED body", LBM_ERR_ARG;
    lbm_opts o;
    if (opts)
        o = *opts;
    else
        lbm_default_opts(&o);
    if (o.storage != LBM_FP64 && o.storage != LBM_FP32)
        return g_adj_create_error = "the adjoint runs in FP64 or FP32 storage", LBM_ERR_ARG;
    o.pop_buffers[0] = o.pop_buffers[1] = nullptr;
    o.history_cap = (int)std::min<int64_t>(std::max<int64_t>(N, 64), 1 << 20);
    lbm_adjoint* A = new lbm_adjoint();
    auto bail = [&](int code) {
        g_adj_create_error = A->err;
        adj_free(A);
        return code;
    };
    int rc = lbm_create(nx, ny, rates, eta, &o, &A->sim);
    if (rc) return A->err = lbm_last_error(nullptr), bail(rc);
    lbm_sim* s = A->sim;
    // the reverse step addresses a direction's populations with 32-bit byte offsets
    if ((long long)s->desc.pitch * ny * (long long)vplbm::elem_size(o.storage) >= (1LL << 32))
        return A->err = "grid too large for the adjoint (a direction's populations reach 4 GiB)",
               bail(LBM_ERR_ARG);
    rc = lbm_set_body(s, body);
    if (rc) return A->err = s->err, bail(rc);
    A->storage = o.storage;
    A->nx = nx;
    A->ny = ny;
    A->steps = N;
    A->K = K;
    A->nseg = (int)(N / K);
    A->wx = aopts->weight_fx;
    A->wy = aopts->weight_fy;
    A->graphs = aopts->use_graphs != 0;
    A->body = *body;
    A->tsz = elem_size(o.storage);
    A->out_bytes = 3 * (size_t)ny * A->tsz;
    A->atx = (nx + TILE_X - 1) / TILE_X;
    const size_t pb = s->pop_bytes, ob = A->out_bytes;
    const size_t plane_b = (size_t)s->desc.fpitch * ny * sizeof(double);  // dJ/dchi, [ny][fpitch]
    auto alloc = [&](void** p, size_t bytes) {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) A->err = std::string("hipMalloc: ") + hipGetErrorString(e);
        return e == hipSuccess;
    };
    if (!alloc((void**)&A->ad_d, 2 * sizeof(AdjDesc)) ||
        !alloc((void**)&A->seg_descs_d, 2 * (size_t)K * sizeof(SimDesc)) ||
        !alloc((void**)&A->def_pop, pb) || !alloc((void**)&A->def_out, ob) ||
        !alloc((void**)&A->init_pop, pb) || !alloc((void**)&A->init_out, ob) ||
        !alloc((void**)&A->ckpt_pop, pb * A->nseg) || !alloc((void**)&A->ckpt_out, ob * A->nseg) ||
        !alloc((void**)&A->seg_pop, 2 * pb * (K + 1)) || !alloc((void**)&A->seg_out, 2 * ob * (K + 1)) ||
        !alloc(&A->abar[0], pb) || !alloc(&A->abar[1], pb) || !alloc(&A->chibar, plane_b) ||
        !alloc((void**)&A->tile_acc, (size_t)A->atx * ny * 3 * sizeof(double)) ||
        !alloc((void**)&A->seg_index, 64) || !alloc((void**)&A->red, 8 * sizeof(double)))
        return bail(LBM_ERR_ALLOC);
    // readers of the edge populations
    std::vector<RingSlot> slots;
    std::vector<int> kn;
    build_ring(s->desc.bc, nx, ny, o.u_conv, s->desc.ps, s->desc.pitch, slots, kn, A->ring_k);
    if (!alloc((void**)&A->ring, slots.size() * sizeof(RingSlot)) ||
        !alloc((void**)&A->ring_kn, kn.size() * sizeof(int)))
        return bail(LBM_ERR_ALLOC);
    hipError_t e = hipMemcpy(A->ring, slots.data(), slots.size() * sizeof(RingSlot), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(A->ring_kn, kn.data(), kn.size() * sizeof(int), hipMemcpyHostToDevice);
    // the uniform initial state as lbm_create left it
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipMemcpy(A->def_pop, s->pop[s->host_step & 1], pb, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(A->def_out, s->outlet, ob, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(A->init_pop, A->def_pop, pb, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(A->init_out, A->def_out, ob, hipMemcpyDeviceToDevice);
    // forward recomputation of a segment into store q: step i reads buffer i and writes
    // buffer i + 1 of that store
    if (e == hipSuccess) {
        std::vector<SimDesc> sd(2 * (size_t)K, s->desc);
        for (int q = 0; q < 2; ++q) {
            char* pop0 = A->seg_pop + (size_t)q * (K + 1) * pb;
            char* out0 = A->seg_out + (size_t)q * (K + 1) * ob;
            for (int i = 0; i < K; ++i) {
                SimDesc& d = sd[(size_t)q * K + i];
                const int p = i & 1;
                d.pop[p] = pop0 + (size_t)i * pb;
                d.pop[p ^ 1] = pop0 + (size_t)(i + 1) * pb;
                d.outlet = out0 + (size_t)i * ob;
                d.outlet_out = out0 + (size_t)(i + 1) * ob;
            }
        }
        e = hipMemcpy(A->seg_descs_d, sd.data(), sd.size() * sizeof(SimDesc), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&A->aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&A->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&A->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) return A->err = hipGetErrorString(e), bail(LBM_ERR_HIP);
    AdjDesc& ad = A->ad;
    std::memset(&ad, 0, sizeof(ad));
    ad.seg_pop = A->seg_pop;
    ad.seg_stride = (long long)pb;
    ad.seg_out = A->seg_out;
    ad.out_stride = (long long)ob;
    ad.ckpt_pop = A->ckpt_pop;
    ad.ckpt_out = A->ckpt_out;
    ad.abar[0] = A->abar[0];
    ad.abar[1] = A->abar[1];
    ad.chibar = static_cast<double*>(A->chibar);
    ad.tile_acc = A->tile_acc;
    ad.ring = A->ring;
    ad.ring_kn = A->ring_kn;
    ad.ring_k = A->ring_k;
    ad.seg_index = A->seg_index;
    ad.wx = A->wx;
    ad.wy = A->wy;
    ad.pop_bytes = (long long)pb;
    ad.out_bytes = (long long)ob;
    ad.tiles_x = A->atx;
    set_pose(A);
    rc = upload_ad(A);
    if (rc) return bail(rc);
    if (A->graphs && K <= 1024) {
        rc = lbm_set_graph_steps(s, K);
        if (rc) return A->err = s->err, bail(rc);
    }
    *out = A;
    return LBM_OK;
}

int lbm_adjoint_destroy(lbm_adjoint* A) {
    if (!A) return LBM_ERR_ARG;
    adj_free(A);
    return LBM_OK;
}

// Removes the additive indicator (its window follows the pose it was set for).
static void drop_chi_add(lbm_sim* s) {
    if (s->chi_add_d) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipFree(s->chi_add_d);
    }
    s->chi_add_d = nullptr;
    s->chi_win[0] = s->chi_win[2] = 0;
    s->chi_win[1] = s->chi_win[3] = -1;
}

int lbm_adjoint_set_chi_add(lbm_adjoint* A, const double* field) {
    if (!A) return LBM_ERR_ARG;
    lbm_sim* s = A->sim;
    A->fwd_done = A->bwd_done = false;
    if (!field) {
        drop_chi_add(s);
        return LBM_OK;
    }
    // the window: the nodes where the disc's own indicator may change with its pose
    const int* w = A->ad.nbox;
    for (int j = 0; j < A->ny; ++j)
        for (int i = 0; i < A->nx; ++i) {
            const double v = field[(size_t)j * A->nx + i];
            if (!std::isfinite(v)) return afail(A, LBM_ERR_ARG, "non-finite additive indicator");
            const bool inside = i >= w[0] && i <= w[1] && j >= w[2] && j <= w[3];
            if (!inside && v != 0.0)
                return afail(A, LBM_ERR_ARG, "additive indicator non-zero outside the body's box");
        }
    const int ww = w[1] - w[0] + 1, wh = w[3] - w[2] + 1;
    if (ww < 1 || wh < 1) return afail(A, LBM_ERR_ARG, "the body has no box on the grid");
    std::vector<double> win((size_t)ww * wh);
    for (int j = 0; j < wh; ++j)
        for (int i = 0; i < ww; ++i) win[(size_t)j * ww + i] = field[(size_t)(w[2] + j) * A->nx + w[0] + i];
    drop_chi_add(s);
    AHIP_TRY(A, hipMalloc((void**)&s->chi_add_d, win.size() * sizeof(double)));
    AHIP_TRY(A, hipMemcpy(s->chi_add_d, win.data(), win.size() * sizeof(double), hipMemcpyHostToDevice));
    for (int k = 0; k < 4; ++k) s->chi_win[k] = w[k];
    return LBM_OK;  // the next forward run sets the body with it
}

int lbm_adjoint_set_body(lbm_adjoint* A, const lbm_body* b) {
    if (!A || !b) return afail(A, LBM_ERR_ARG, "NULL argument");
    if (b->mode != LBM_BODY_FIXED) return afail(A, LBM_ERR_ARG, "the adjoint needs a FIXED body");
    drop_chi_add(A->sim);
    int rc = lbm_set_body(A->sim, b);
    if (rc) return afail(A, rc, A->sim->err);
    A->body = *b;
    set_pose(A);
    A->fwd_done = A->bwd_done = false;
    drop_stage_graphs(A);  // the captured stages carry the row shift of the old pose
    return upload_ad(A);
}

int lbm_adjoint_set_initial(lbm_adjoint* A, const double* f, const double* outlet) {
    if (!A) return LBM_ERR_ARG;
    lbm_sim* s = A->sim;
    AHIP_TRY(A, hipStreamSynchronize(s->stream));
    if (f) {
        int rc = lbm_set_populations(s, f);
        if (rc) return afail(A, rc, s->err);
        AHIP_TRY(A, hipMemcpy(A->init_pop, s->pop[s->host_step & 1], s->pop_bytes, hipMemcpyDeviceToDevice));
    } else {
        AHIP_TRY(A, hipMemcpy(A->init_pop, A->def_pop, s->pop_bytes, hipMemcpyDeviceToDevice));
    }
    if (outlet) {
        const int dirs[3] = {3, 6, 7};
        std::vector<double> o64(3 * (size_t)A->ny);
        std::vector<float> o32(3 * (size_t)A->ny);
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < A->ny; ++j) {
                const double v = outlet[(size_t)k * A->ny + j] - s->desc.fref[dirs[k]];
                o64[(size_t)k * A->ny + j] = v;
                o32[(size_t)k * A->ny + j] = (float)v;
            }
        const void* src = A->tsz == 8 ? (const void*)o64.data() : (const void*)o32.data();
        AHIP_TRY(A, hipMemcpy(A->init_out, src, A->out_bytes, hipMemcpyHostToDevice));
    } else {
        AHIP_TRY(A, hipMemcpy(A->init_out, A->def_out, A->out_bytes, hipMemcpyDeviceToDevice));
    }
    A->fwd_done = A->bwd_done = false;
    return LBM_OK;
}

int lbm_adjoint_forward(lbm_adjoint* A, double* J) {
    if (!A) return LBM_ERR_ARG;
    lbm_sim* s = A->sim;
    A->fwd_done = A->bwd_done = false;
    AHIP_TRY(A, hipStreamSynchronize(s->stream));
    s->host_step = 0;
    s->drained = 0;
    s->rec_end = 0;
    AHIP_TRY(A, hipMemcpyAsync(s->pop[0], A->init_pop, s->pop_bytes, hipMemcpyDeviceToDevice, s->stream));
    AHIP_TRY(A, hipMemcpyAsync(s->outlet, A->init_out, A->out_bytes, hipMemcpyDeviceToDevice, s->stream));
    AHIP_TRY(A, hipMemsetAsync(s->flag, 0, sizeof(int), s->stream));
    int rc = lbm_set_body(s, &A->body);  // fresh state of step 0
    if (rc && rc != LBM_ERR_UNSTABLE) return afail(A, rc, s->err);
    AHIP_TRY(A, hipMemsetAsync(s->flag, 0, sizeof(int), s->stream));
    s->drained = 0;
    A->recs.assign((size_t)A->steps, lbm_force_rec{});
    const bool drain_each = A->steps > s->hist_cap;
    for (int c = 0; c < A->nseg; ++c) {
        AHIP_TRY(A, hipMemcpyAsync(A->ckpt_pop + (size_t)c * s->pop_bytes, s->pop[0], s->pop_bytes,
                                   hipMemcpyDeviceToDevice, s->stream));
        AHIP_TRY(A, hipMemcpyAsync(A->ckpt_out + (size_t)c * A->out_bytes, s->outlet, A->out_bytes,
                                   hipMemcpyDeviceToDevice, s->stream));
        rc = lbm_step(s, A->K);
        if (rc) return afail(A, rc, s->err);
        if (drain_each) {
            int64_t n = 0;
            rc = lbm_forces(s, A->recs.data() + (size_t)c * A->K, A->K, &n);
            if (rc) return afail(A, rc, s->err);
            if (n != A->K) return afail(A, LBM_ERR_STATE, "missing force records");
        }
    }
    if (!drain_each) {
        int64_t n = 0;
        rc = lbm_forces(s, A->recs.data(), A->steps, &n);
        if (rc) return afail(A, rc, s->err);
        if (n != A->steps) return afail(A, LBM_ERR_STATE, "missing force records");
    }
    double sum = 0.0;
    for (const lbm_force_rec& r : A->recs) sum += A->wx * r.fvp[0] + A->wy * r.fvp[1];
    A->J = sum;
    if (J) *J = sum;
    A->fwd_done = true;
    return LBM_OK;
}

int lbm_adjoint_forces(lbm_adjoint* A, lbm_force_rec* out, int64_t cap, int64_t* n_out) {
    if (!A || (!out && cap > 0) || cap < 0) return afail(A, LBM_ERR_ARG, "bad argument");
    if (!A->fwd_done) return afail(A, LBM_ERR_STATE, "no forward run");
    const int64_t n = std::min<int64_t>(cap, (int64_t)A->recs.size());
    if (n > 0) std::memcpy(out, A->recs.data(), (size_t)n * sizeof(lbm_force_rec));
    if (n_out) *n_out = n;
    return LBM_OK;
}

int lbm_adjoint_backward(lbm_adjoint* A) {
    if (!A) return LBM_ERR_ARG;
    if (!A->fwd_done) return afail(A, LBM_ERR_STATE, "lbm_adjoint_forward must run first");
    lbm_sim* s = A->sim;
    A->bwd_done = false;
    int rc = zero_words(A, A->abar[(A->steps) & 1], s->pop_bytes);
    if (!rc) rc = zero_words(A, A->chibar, (size_t)s->desc.fpitch * s->ny * sizeof(double));
    if (!rc) rc = zero_words(A, A->tile_acc, (size_t)A->atx * A->ny * 3 * sizeof(double));
    if (rc) return rc;
    const int last = A->nseg - 1;
    AHIP_TRY(A, hipMemcpyAsync(A->seg_index, &last, sizeof(int), hipMemcpyHostToDevice, s->stream));
    AHIP_TRY(A, hipStreamSynchronize(s->stream));
    // segments are swept last first; segment m's store is m & 1.  The recomputation of
    // the last segment comes first, then stages m = nseg - 1 .. 1 (sweep m alongside the
    // recomputation of m - 1), then the sweep over segment 0.
    rc = enqueue_recompute(A, last & 1, s->stream);
    if (rc) return rc;
    if (!A->graphs) {
        for (int m = last; m >= 1; --m) {
            rc = enqueue_stage(A, m & 1);
            if (rc) return rc;
        }
    } else if (last >= 1) {
        for (int q = 0; q < 2 && q < last; ++q) {
            const int parity = (last - q) & 1;  // the first two stages, one of each parity
            if (A->gexec[parity]) continue;
            AHIP_TRY(A, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
            rc = enqueue_stage(A, parity);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(s->stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return afail(A, LBM_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
            A->graph[parity] = g;
            AHIP_TRY(A, hipGraphInstantiate(&A->gexec[parity], g, nullptr, nullptr, 0));
        }
        for (int m = last; m >= 1; --m) AHIP_TRY(A, hipGraphLaunch(A->gexec[m & 1], s->stream));
    }
    rc = enqueue_sweep(A, 0, s->stream);
    if (rc) return rc;
    AHIP_TRY(A, hipStreamSynchronize(s->stream));
    A->bwd_done = true;
    return LBM_OK;
}

int lbm_adjoint_gradient(lbm_adjoint* A, double* dJ_dchi, double* dJ_dpos, double* dJ_dvel) {
    if (!A) return LBM_ERR_ARG;
    if (!A->bwd_done) return afail(A, LBM_ERR_STATE, "lbm_adjoint_backward must run first");
    lbm_sim* s = A->sim;
    if (dJ_dchi && ensure_staging(s) != hipSuccess)
        return afail(A, LBM_ERR_ALLOC, "hipMalloc of the FP64 exchange buffer failed");
    double r[5];
    dispatch(A->storage, [&](auto* tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        if constexpr (std::is_same_v<S, double> || std::is_same_v<S, float>) {
            AdjLaunch<S>::reduce(s->desc_d, A->ad_d, A->red, s->stream);
            if (dJ_dchi)
                AdjLaunch<S>::export_chi(s->desc_d, A->ad_d, s->staging,
                                         dim3((A->nx + 255) / 256, A->ny), s->stream);
        }
        return 0;
    });
    AHIP_TRY(A, hipGetLastError());
    AHIP_TRY(A, hipMemcpyAsync(r, A->red, sizeof(r), hipMemcpyDeviceToHost, s->stream));
    AHIP_TRY(A, hipStreamSynchronize(s->stream));
    if (dJ_dchi)
        AHIP_TRY(A, hipMemcpy(dJ_dchi, s->staging, (size_t)A->nx * A->ny * sizeof(double),
                              hipMemcpyDeviceToHost));
    if (dJ_dpos) {
        dJ_dpos[0] = r[0];
        dJ_dpos[1] = r[1];
    }
    if (dJ_dvel) {
        dJ_dvel[0] = r[2];
        dJ_dvel[1] = r[3];
        dJ_dvel[2] = r[4];
    }
    return LBM_OK;
}

int lbm_adjoint_time_kernels(lbm_adjoint* A, int reps, double* adjoint_us, double* step_us) {
    if (!A || reps < 1) return afail(A, LBM_ERR_ARG, "bad argument");
    if (!A->bwd_done) return afail(A, LBM_ERR_STATE, "lbm_adjoint_backward must run first");
    lbm_sim* s = A->sim;
    hipEvent_t e[3];
    for (auto& x : e) AHIP_TRY(A, hipEventCreate(&x));
    const dim3 fgrid = step_grid(s->desc), agrid(A->atx, A->ny);
    AHIP_TRY(A, hipEventRecord(e[0], s->stream));
    dispatch(A->storage, [&](auto* tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        if constexpr (std::is_same_v<S, double> || std::is_same_v<S, float>) {
            for (int k = 0; k < reps; ++k) AdjLaunch<S>::step(s->desc_d, A->ad_d, agrid, k & 1, s->stream);
            (void)hipEventRecord(e[1], s->stream);
            for (int k = 0; k < reps; ++k) {
                const int i = k % A->K;
                Launch<S>::step(A->seg_descs_d + i, fgrid, s->rows, s->nt, s->desc.tile_w, i & 1, s->stream,
                                s->row_shift);
            }
        }
        return 0;
    });
    AHIP_TRY(A, hipGetLastError());
    AHIP_TRY(A, hipEventRecord(e[2], s->stream));
    AHIP_TRY(A, hipEventSynchronize(e[2]));
    float ms1 = 0.f, ms2 = 0.f;
    AHIP_TRY(A, hipEventElapsedTime(&ms1, e[0], e[1]));
    AHIP_TRY(A, hipEventElapsedTime(&ms2, e[1], e[2]));
    for (auto& x : e) (void)hipEventDestroy(x);
    if (adjoint_us) *adjoint_us = 1e3 * ms1 / reps;
    if (step_us) *step_us = 1e3 * ms2 / reps;
    A->bwd_done = false;  // the accumulators were overwritten
    return LBM_OK;
}

}  // extern "C"
