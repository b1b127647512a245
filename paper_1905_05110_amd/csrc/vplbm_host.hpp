// vplbm_host.hpp -- host-side state of a simulation, shared by the translation units
// of the host runtime (vplbm.hip: step, batch and I/O; adjoint_host.hip: the adjoint).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "vplbm.h"
#include "vplbm_kernels.hpp"

namespace vplbm {

inline size_t elem_size(int storage) {
    switch (storage) {
        case LBM_FP64: return 8;
        case LBM_FP32: return 4;
        default: return 2;
    }
}

// Row stride of a single-field array (elements): nx rounded up to 64.
inline int row_pitch(int nx) { return (nx + 63) / 64 * 64; }

// Row stride of the population arrays (elements): nx rounded up to an odd multiple of
// 64.  Tiles of consecutive rows run at once on different XCDs; with a row stride of
// 2^k x 64 elements (k >= 2) their accesses fall on the same few memory channels, and
// 64-column tiles of 512-, 768- or 1024-column grids ran 5-10 % slower than those of
// 576 or 704 columns.  The padding columns are never read or written.
inline int pop_row_pitch(int nx) { return ((nx + 63) / 64 | 1) * 64; }

inline long long plane_stride(int nx, int ny) {
    // pad planes by 5 x 64 elements so the nine streams do not start on the same
    // large power-of-two boundary
    return (long long)pop_row_pitch(nx) * ny + 320;
}

// Strides of the population arrays of one buffer (elements): between the rows of one
// direction (SimDesc::pitch) and between directions (SimDesc::ps).  ROWS puts row j of
// direction a at (9 j + a) pop_row_pitch: the rows a node's pull reads and the row it
// writes then lie within a few row lengths of each other, which the memory system serves
// faster than nine separate planes.  The step kernel's fast path addresses populations
// with 32-bit lane offsets from per-tile bases at the tile's rows, so a buffer may be of
// any size, but the rows a tile reaches (at most 18: 16 rows of a tile and one on each
// side) must span less than 4 GiB; returns false (with a message) when the request does
// not fit.
inline bool pop_geometry(int nx, int ny, int storage, int request, int& pitch, long long& ps,
                         int& layout, std::string& msg) {
    const long long rp = pop_row_pitch(nx);
    const long long e = (long long)elem_size(storage);
    const long long lim = 1LL << 32;
    const bool rows_fit = 18 * NQ * rp * e < lim;
    const bool planes_fit = 18 * rp * e < lim;
    if (request == LBM_LAYOUT_ROWS || (request == LBM_LAYOUT_AUTO && rows_fit)) {
        if (!rows_fit) return msg = "grid too wide for the ROWS layout (18 rows span 4 GiB or more)", false;
        pitch = (int)(NQ * rp);
        ps = rp;
        layout = LBM_LAYOUT_ROWS;
        return true;
    }
    if (!planes_fit) return msg = "grid too wide: 18 rows of a plane span 4 GiB or more", false;
    pitch = (int)rp;
    ps = plane_stride(nx, ny);
    layout = LBM_LAYOUT_PLANES;
    return true;
}

}  // namespace vplbm

using vplbm::BodyDev;
using vplbm::Record;
using vplbm::SimDesc;
using vplbm::bf16s;

struct lbm_sim {
    int nx = 0, ny = 0, storage = LBM_FP32;
    size_t pop_bytes = 0;
    void* pop[2] = {nullptr, nullptr};
    bool own_pop = false;
    void* outlet = nullptr;
    BodyDev* body_d = nullptr;
    double* partials = nullptr;
    Record* hist = nullptr;
    int* flag = nullptr;
    double* staging = nullptr;  // FP64 [9][ny][nx] for set/get/fields, see ensure_staging
    SimDesc desc{};
    SimDesc* desc_d = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t host_step = 0;
    int64_t drained = 0;
    int64_t rec_end = 0;  // without a body: records exist for the steps before this one
    int hist_cap = 65536;
    lbm_opts opts{};
    lbm_rates rates{};
    double eta = 0.0;
    BodyDev body_h{};
    lbm_body body_desc{};  // last body set (used by the autotuner)
    bool has_body = false;
    std::string err;
    int graph_steps = 0;
    int rows = 1;   // rows of a tile (nodes per lane)
    bool nt = false;  // nontemporal population stores
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    bool in_batch = false;  // member of an lbm_batch: stepped, configured and freed by it
    int row_shift = 0;      // first tile row dispatched (the body's rows come a little later)
    int fin_req = LBM_FINALIZE_AUTO;  // requested finalization of the body state
    bool sep_final = false;           // in effect: a one-workgroup launch after each step
    double* chi_add_d = nullptr;      // additive indicator over chi_win (set by the adjoint)
    int chi_win[4] = {0, -1, 0, -1};  // its node window (i0, i1, j0, j1)
};

#define HIP_TRY(sim, expr)                                                             \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (sim)->err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
            return LBM_ERR_HIP;                                                        \
        }                                                                              \
    } while (0)

inline int fail(lbm_sim* s, int code, const std::string& msg) {
    if (s) s->err = msg;
    return code;
}

inline int reject_member(lbm_sim* s) {
    return fail(s, LBM_ERR_STATE, "a member of a batch is stepped, configured and freed by its batch");
}


template <class F>
inline int dispatch(int storage, F&& f) {
    switch (storage) {
        case LBM_FP64: return f((double*)nullptr);
        case LBM_FP32: return f((float*)nullptr);
        case LBM_FP16_OFS: return f((_Float16*)nullptr);
        default: return f((bf16s*)nullptr);
    }
}

// The FP64 exchange buffer [9][ny][nx] (fields, population import and export, the
// adjoint's field export), allocated on first use: a simulation that never exchanges
// whole fields with the host holds none (72 B per node; 1.1 GB for the 64-run sweep).
inline hipError_t ensure_staging(lbm_sim* s) {
    if (s->staging) return hipSuccess;
    return hipMalloc((void**)&s->staging, (size_t)vplbm::NQ * s->nx * s->ny * sizeof(double));
}
