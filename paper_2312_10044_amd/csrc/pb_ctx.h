// Internal host-side state of the library: the context (pb_ctx), its device
// buffers, error and timing helpers.  Shared by pb_capi.hip and pb_batch.hip.
#pragma once

#include "../../include/pbsolve.h"
#include "pb_host.h"
#include "pb_kernels.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

namespace pbk {

constexpr double C_UNITS = 332.0716;      // e_c^2/A -> kcal/mol (Sec. 2.1)
constexpr double TWO_PI = 6.283185307179586476925286766559;
constexpr int TARGET_WAVES = 32768;       // ~32 waves per SIMD over a launch (256 CUs x 4 SIMDs)

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct ErrorState {
    std::string msg = "no error";
};

}  // namespace pbk

struct pb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    pbk::ErrorState err;
    size_t mem_used = 0;    // bytes held in device buffers (DevBuf capacities)
    size_t mem_limit = 0;   // pb_set_memory_limit; 0 = none
    // device scratch
    pbk::DevBuf geo, geo_part, src64, src32, part, vec, V, small, dpart, chg_part, chg_per;
    pbk::DevBuf in_vert, in_tri, in_pos, in_q, io_x, io_y;
    double *hsmall = nullptr;   // pinned host staging, HSMALL doubles
    double *hgeo = nullptr;     // pinned host staging of the centroids (leaf build)
    size_t hgeo_n = 0;
    double *hchg = nullptr;     // pinned host staging of the charges' solid angles
    size_t hchg_n = 0;
    hipEvent_t ev_fetch = nullptr;   // marks the centroid copy for the leaf build
    // kernel timing (pb_profile_*)
    struct Mark {
        hipEvent_t a, b;
        int kind;
        double pairs;
    };
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<Mark> marks;
    int64_t prof_launches[PB_KERNEL_COUNT] = {};
    double prof_ms[PB_KERNEL_COUNT] = {};
    double prof_pairs[PB_KERNEL_COUNT] = {};
    // launch configuration of the FP32 forward sweep (pb_set_sweep_config / pb_autotune)
    int f32_tpt = PB_SWEEP_PAIRWISE;   // 1, 2: per-target sweep; or the pairwise sweep
    int f32_waves = 131072;
    // pairwise sweep: packed points, work items and partial sums (plan cached)
    pbk::DevBuf sym_src, sym_src64, sym_items, sym_rowstart, sym_rowpart, sym_colpart;
    int f64_kind = PB_SWEEP_PAIRWISE;   // FP64 sweep: 1 per-target, or pairwise
    int b_sym_tiles = 4;                 // batch: source tiles per pairwise work item
    pbk::SymPlan sym_plan;
    // banded pairwise FP32 sweep: items, record lists (start, index), records
    pbk::DevBuf band_items, band_lists, band_recs;
    pbk::BandPlan band_plan;
    int sym_waves = 0;
    // treecode: tree, permuted geometry and weights, moments, results
    pbk::DevBuf t_nodes, t_ctr, t_perm, t_geo, t_wv, t_out, t_mom, t_cnt;
    bool t_ready = false;     // tree of the current geometry built (reset by setup_geometry)
    int t_n0 = 0, t_n_nodes = 0;
    // treecode matvec inside solves (pb_solve_tree): FP64 forward matvecs use it
    bool t_solve = false;
    double t_theta = 0.0;
    int t_order = 0, t_solve_n0 = 0;
    // current geometry
    pbk::Geo g{};
    double center[3] = {0.0, 0.0, 0.0};
    double volume = 0.0, area_sum = 0.0;
    double sigma_min = 1.0;   // inverse length scale of the mesh (f32_sigma)
    pbk::DevBuf dup_tab;      // coincident-centroid check (launch_dup_check)
    pbk::DevBuf probe_out;    // pb_probe_valu's per-thread results
    // block-diagonal preconditioner of the current geometry
    pbk::DevBuf pc_idx, pc_inv;
    int64_t pc_leaves = 0;
    int32_t *pc_perm = nullptr, *pc_start = nullptr;
    int64_t *pc_boff = nullptr;
    int64_t *pc_pidx = nullptr, *pc_qidx = nullptr;
    // batched solves (pb_solve_batch)
    pbk::DevBuf b_geo, b_desc, b_map, b_items, b_src, b_part, b_vec, b_V, b_state, b_red, b_chg;
    pbk::DevBuf b_sitems, b_rs, b_srow, b_scol;   // pairwise sweeps of the batch
    pbk::DevBuf b_pc_idx, b_pc_inv, b_pc_sys;
    hipGraphExec_t b_graph = nullptr;
    uint64_t b_graph_key = 0;
};

namespace pbk {

constexpr int HSMALL = 4 * (MAX_RESTART + 2) + 64;
constexpr int HSMALL_DUP = HSMALL - 6;   // two int32: the coincident-centroid verdict

// Slots of the coincident-centroid hash table for n points: a power of two >= 2n.
inline int64_t dup_table_size(int64_t n)
{
    int64_t cap = 1024;
    while (cap < 2 * n)
        cap *= 2;
    return cap;
}

inline int fail(pb_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err.msg = buf;
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(c, e_ == hipErrorOutOfMemory ? PB_ERR_OOM : PB_ERR_HIP,           \
                        "%s failed: %s", #expr, hipGetErrorString(e_));                   \
    } while (0)

#define LAUNCHCHK()                                                                       \
    do {                                                                                  \
        hipError_t e_ = hipGetLastError();                                                \
        if (e_ != hipSuccess)                                                             \
            return fail(c, PB_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

#define TRY(expr)              \
    do {                       \
        int rc_ = (expr);      \
        if (rc_ < 0)           \
            return rc_;        \
    } while (0)

inline int ensure(pb_ctx *c, DevBuf &b, size_t bytes)
{
    if (bytes <= b.cap)
        return PB_OK;
    if (c->mem_limit && c->mem_used - b.cap + bytes > c->mem_limit)
        return fail(c, PB_ERR_OOM,
                    "device scratch of %zu bytes would pass the context's limit of %zu bytes "
                    "(%zu held)",
                    bytes, c->mem_limit, c->mem_used);
    if (b.p) {
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipFree(b.p));
    }
    c->mem_used -= b.cap;
    b.p = nullptr;
    b.cap = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(c, PB_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    b.cap = bytes;
    c->mem_used += bytes;
    return PB_OK;
}

template <typename T>
inline T *as(DevBuf &b) { return static_cast<T *>(b.p); }

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

inline hipEvent_t pool_event(pb_ctx *c, size_t idx)
{
    while (c->ev_pool.size() <= idx) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[idx];
}

// Brackets one kernel launch with events when profiling is on.
struct ProfScope {
    pb_ctx *c;
    int kind;
    double pairs;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(pb_ctx *c_, int kind_, double pairs_) : c(c_), kind(kind_), pairs(pairs_)
    {
        if (!c->prof_on)
            return;
        const size_t k = 2 * c->marks.size();
        a = pool_event(c, k);
        b = pool_event(c, k + 1);
        if (a && b)
            (void)hipEventRecord(a, c->stream);
    }
    ~ProfScope()
    {
        if (a && b) {
            (void)hipEventRecord(b, c->stream);
            c->marks.push_back({a, b, kind, pairs});
        }
    }
};

// Collect elapsed times of recorded launches (the stream must have drained).
inline void prof_collect(pb_ctx *c)
{
    for (const auto &m : c->marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
            c->prof_ms[m.kind] += ms;
            c->prof_launches[m.kind] += 1;
            c->prof_pairs[m.kind] += m.pairs;
        }
    }
    c->marks.clear();
}



// Batched solve of independent systems (pb_batch.hip).
int tree_matvec(pb_ctx *c, const pb_params *p, double theta, int order, int n0, const double *x,
                double *y, int64_t *counts);
int tree_prepare(pb_ctx *c, int n0);
int tree_apply(pb_ctx *c, const pb_params *p, double theta, int order, const double *x,
               double *y, int64_t *counts);
// Candidate configurations of the batch autotuner and their timings.
struct BatchTune {
    int n = 0;
    int kind[8] = {0}, tiles[8] = {0};
    double ms[8] = {0.0};
    int best = -1;
};
// No-allocation matvec (pb_noalloc.hip): set-up once per device, and the call.
int noalloc_init(int device);
int matvec_noalloc(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                   const int32_t *d_tri, const pb_params *p, const double *d_x, double *d_y,
                   int transpose, int precision);
int batch_solve(pb_ctx *c, int32_t n_sys, const pb_surface *surf, const pb_charges *chg,
                const pb_params *p, int want_forces, double *e_solv, double *dE_dpos,
                double *dE_dq, pb_info *info, BatchTune *tune = nullptr,
                bool device_inputs = false);

}  // namespace pbk
