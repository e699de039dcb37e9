// Host runtime behind the C ABI of include/cgp.h: context, mesh registry,
// per-mesh solver workspaces, cached launch plans for the persistent solver,
// HIP graph capture, and argument validation.  No C++ exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <sstream>
#include <unordered_map>

#include "cgp_internal.hpp"

namespace cgp {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

int pcg_max_blocks_per_cu();

struct Plan {
    DBuf<uint8_t> buf;
    InstDesc *d_insts = nullptr;
    int32_t *d_block_inst = nullptr;
    RowRange *d_ranges = nullptr;
    int32_t *d_done_at = nullptr;    // persistent driver: stage at which each instance finished
    int32_t *d_done = nullptr;       // staged driver: finished-instance counter
    SolveParams *d_prm = nullptr;    // staged driver: parameters of the current call
    int32_t *d_cblk_inst = nullptr;  // deflation: instance of each coarse-kernel workgroup
    CoarseRec *d_crecs = nullptr;    // deflation: per-instance coarse-step records (device)
    InstDesc one{};                  // a single instance's record (passed by value to the stage kernels)
    std::vector<CoarseRec> crecs;    // the same on the host (a single instance's goes by value)
    int cgrid = 0;                   // deflation: coarse-kernel workgroups
    int grid = 0;
    int n_inst = 0;
    int unb = 0;                     // workgroups per instance when all instances have as many, else 0
    int halo = 0;                    // widest column range of a workgroup
    hipGraph_t graph = nullptr;      // staged driver: `launches` stage launches
    hipGraphExec_t exec = nullptr;
    int launches = 0;
    hipGraph_t tail_graph = nullptr; // staged driver: TAIL_LAUNCHES stage launches for the end of a solve
    hipGraphExec_t tail_exec = nullptr;
    int32_t last_stages = 0;         // launches the previous solve of this plan needed (0 = unknown)
    ~Plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (tail_exec) (void)hipGraphExecDestroy(tail_exec);
        if (tail_graph) (void)hipGraphDestroy(tail_graph);
    }
};

constexpr int TAIL_LAUNCHES = 4;   // stage launches per graph near the predicted end of a solve

// preconditioner degrees cgp_autotune times (1 = Jacobi in the tiled iteration)
constexpr int AUTOTUNE_CANDIDATES = CGP_AUTOTUNE_CANDIDATES;
constexpr int AUTOTUNE_DEGREES[AUTOTUNE_CANDIDATES] = {1, 2, 3, 4, 5, 6, 7, 8};
struct TuneRec {
    std::vector<int32_t> degree;           // per instance
    double ms[AUTOTUNE_CANDIDATES] = {};   // the batch's best solve time at each candidate (-1: no solve)
    std::vector<int32_t> iters;            // [instance][candidate] iterations (-1: no solve)
};

struct GraphRec {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<std::shared_ptr<Plan>> plans;   // launch plans the recorded solves use
};

}  // namespace cgp

using namespace cgp;

struct cgp_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t aux = nullptr;
    int cus = 0;
    int max_blocks_per_cu = 1;
    int32_t next_mesh = 0, next_graph = 0;
    std::map<int32_t, std::unique_ptr<Mesh>> meshes;
    // (shared with the graphs that recorded solves on them, which keep them alive)
    std::unordered_map<std::string, std::shared_ptr<Plan>> plans;
    // launches the last solve of a mesh set and option set needed, whatever its vectors: the
    // prediction for a plan's first solve (plans differ by vector pointers, e.g. rotating
    // previous-solution buffers, but solve alike)
    std::unordered_map<std::string, int32_t> stage_hint;
    // cgp_autotune's choices by mesh shape (rows, nonzeros, widest row), precision and deflation
    std::unordered_map<std::string, TuneRec> tuned;
    std::map<int32_t, GraphRec> graphs;
    struct ModelDel {
        void operator()(Model *m) const { gnn_destroy(m); }
    };
    std::map<int32_t, std::unique_ptr<Model, ModelDel>> models;
    int32_t next_model = 0;
    DBuf<GridSync> sync;
    int32_t *host_flag = nullptr;     // pinned, mapped: [0] set by the device when a staged solve is
                                      // done, [1] the launches its last instance needed
    int32_t *host_flag_dev = nullptr;
    DBuf<int32_t> sink_flag;          // [2] the completion flag of solves recorded in graphs
    hipEvent_t chunk_ev[2] = {nullptr, nullptr};
    uint64_t timeout_ticks = 0;
    int64_t stage_launches = 0;
    bool capturing = false;
    std::vector<std::shared_ptr<Plan>> capture_plans;   // plans used by the capture in progress
    // stage timing (cgp_stage_timing): stage kernels launched one by one between HIP events
    bool time_stages = false;
    std::vector<hipEvent_t> tev;
    int64_t timed_launches[2] = {0, 0};   // stage kernels, coarse kernels
    double timed_us[2] = {0.0, 0.0};
};

namespace {

template <class F>
cgp_status guarded(F &&f) {
    try {
        f();
        return CGP_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return CGP_E_NOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return CGP_E_INVALID;
    }
}

void use_device(cgp_ctx ctx) {
    CGP_REQUIRE(ctx != nullptr, "null context");
    CGP_HIP(hipSetDevice(ctx->device));
}

Mesh &get_mesh(cgp_ctx ctx, cgp_mesh h) {
    auto it = ctx->meshes.find(h);
    if (it == ctx->meshes.end()) throw Error{CGP_E_INVALID, "unknown mesh handle"};
    return *it->second;
}

void ensure_work(Mesh &m, hipStream_t st) {
    const int64_t n = m.lv[0].n;
    SolveWork &w = m.work;
    if (w.n == n) return;
    w.r.alloc(2 * n);
    w.w.alloc(2 * n);
    w.s.alloc(2 * n);
    w.p.alloc(n);
    w.r32.alloc(2 * n);
    w.w32.alloc(2 * n);
    w.s32.alloc(2 * n);
    w.p32.alloc(n);
    w.c32.alloc(n);
    w.u.alloc(n);
    w.u32.alloc(n);
    w.rwsd32.alloc(8 * n);
    w.rwsd64.alloc(8 * n);
    w.up32.alloc(2 * n);
    w.up64.alloc(2 * n);
    launch_fill_rwsd(st, n, m.dinv32.p, m.dinv.p, w.rwsd32.p, w.rwsd64.p);
    w.n = n;
}

// split `grid` workgroups between the instances, proportionally to n^1.5
// (rows times the ~sqrt(n) iterations a Jacobi-CG solve needs), at least one each
std::vector<int32_t> split_blocks(const std::vector<int64_t> &rows, int grid) {
    const size_t k = rows.size();
    std::vector<double> w(k);
    double tot = 0.0;
    for (size_t i = 0; i < k; ++i) {
        w[i] = std::pow(static_cast<double>(std::max<int64_t>(rows[i], 1)), 1.5);
        tot += w[i];
    }
    std::vector<int32_t> nb(k, 1);
    int left = grid - static_cast<int>(k);
    std::vector<double> want(k);
    for (size_t i = 0; i < k; ++i) want[i] = w[i] / tot * grid;
    // greedy: give blocks to the instance with the largest remaining deficit
    while (left > 0) {
        size_t best = 0;
        double bd = -1e300;
        for (size_t i = 0; i < k; ++i) {
            const double cap = static_cast<double>(std::max<int64_t>(rows[i] / 64, 1));
            if (nb[i] >= cap) continue;
            const double d = want[i] - nb[i];
            if (d > bd) { bd = d; best = i; }
        }
        if (bd == -1e300) break;
        ++nb[best];
        --left;
    }
    return nb;
}

struct WorkPtrs {
    double *r, *w, *s, *p, *u;
    float *r32, *w32, *s32, *p32, *c32, *u32;
    float *rwsd32, *up32;
    double *rwsd64, *up64;
};

WorkPtrs work_ptrs(SolveWork &w) {
    return WorkPtrs{w.r.p,   w.w.p,   w.s.p,   w.p.p,      w.u.p,    w.r32.p,    w.w32.p, w.s32.p,
                    w.p32.p, w.c32.p, w.u32.p, w.rwsd32.p, w.up32.p, w.rwsd64.p, w.up64.p};
}

// Chebyshev iteration over [hi/1000, hi] ([hi/30, hi] with deflation, whose coarse space takes
// over the smooth end of the spectrum): the first step scales D^-1 r by 1/c, step k updates
// dz <- a1 dz + a2 D^-1 res; degree 1 is Jacobi, z = D^-1 r
void cheb_coefficients(double *cheb, int degree, double hi, bool defl) {
    if (degree <= 1) {
        cheb[0] = 1.0;
        return;
    }
    const double lo = hi / (defl ? 30.0 : 1000.0);
    const double c = 0.5 * (hi + lo), e = 0.5 * (hi - lo), sig = c / e;
    double rho = 1.0 / sig;
    cheb[0] = 1.0 / c;
    for (int k = 1; k < degree; ++k) {
        const double rn = 1.0 / (2.0 * sig - rho);
        cheb[2 * k - 1] = rn * rho;
        cheb[2 * k] = 2.0 * rn / e;
        rho = rn;
    }
}

// The record of one instance from its mesh, workspace vectors and the caller's vectors; the
// launch-specific fields (workgroups, partial sums, control state, coarse-step buffers) are
// the caller's to fill.  T: the tiled plan (null for the row-range and persistent kernels).
InstDesc describe_instance(Mesh &m, const WorkPtrs &ws, const TilePlan *T, int kwidth, int degree, bool defl,
                           bool persistent, int lanes, int guess, const double *b, double *x,
                           const double *prev1, const double *prev2, hipStream_t aux) {
    InstDesc d{};
    d.n = static_cast<int32_t>(m.lv[0].n);
    d.lanes = lanes;
    d.guess = guess;
    d.fast = (!persistent && m.max_row <= pcg_ell_max_width()) ? 1 : 0;
    d.ell_w = m.max_row;
    d.ell_col = m.ell_col.p;
    d.ell_val = m.ell_val.p;
    d.ell_val32 = m.ell_val32.p;
    d.rowptr = m.rowptr.p;
    d.col = m.col.p;
    d.val = m.val.p;
    d.val32 = m.val32.p;
    d.dinv = m.dinv.p;
    d.dinv32 = m.dinv32.p;
    d.b = b;
    d.x = x;
    d.prev1 = prev1;
    d.prev2 = prev2;
    d.r = ws.r;
    d.w = ws.w;
    d.s = ws.s;
    d.p = ws.p;
    d.u = ws.u;
    d.r32 = ws.r32;
    d.w32 = ws.w32;
    d.s32 = ws.s32;
    d.p32 = ws.p32;
    d.c32 = ws.c32;
    d.u32 = ws.u32;
    d.rwsd32 = ws.rwsd32;
    d.up32 = ws.up32;
    d.rwsd64 = ws.rwsd64;
    d.up64 = ws.up64;
    if (T) {
        d.degree = degree;
        d.tblk = T->blk.p;
        d.treg = T->reg.p;
        if (kwidth == SPLIT_WIDTH) {
            d.tcol = reinterpret_cast<const uint16_t *>(T->scol.p);
            d.tval32 = T->sval32.p;
            d.tval = T->sval64.p;
        } else {
            d.tcol = T->ecol.p;
            d.tval32 = T->eval32.p;
            d.tval = T->eval64.p;
        }
        d.agg = T->agg;
        if (defl) {
            d.defl = 1;
            d.kzk = T->kzk.p;
            d.kzv32 = T->kzv32.p;
            d.kzv = T->kzv64.p;
            d.einv = T->einv.p;
            d.einv32 = T->einv32.p;
            d.oagg = T->oagg.p;
        }
        cheb_coefficients(d.cheb, degree, degree >= 2 ? mesh_gershgorin(aux, m) : 0.0, defl);
    }
    return d;
}

// the coarse step's record of a deflated instance whose record d is complete (fp32 iterations
// read E^-1 rounded to fp32: they round mu to fp32 anyway, and the coarse step reads all of
// E^-1 every stage)
CoarseRec coarse_record(const InstDesc &d, int cblk0) {
    CoarseRec cr{};
    cr.einv = d.einv;
    cr.einv32 = d.einv32;
    cr.partials = d.partials;
    cr.mu = d.mu;
    cr.cpart = d.cpart;
    cr.m = d.agg * d.nblk;
    cr.agg = d.agg;
    cr.tiles = d.nblk;
    cr.cblk0 = cblk0;
    cr.ctl = d.ctl;
    cr.ncb = d.ncb;
    return cr;
}

void check_opts(const cgp_solve_opts &o) {
    CGP_REQUIRE(o.precision == CGP_FP64 || o.precision == CGP_FP32_IR, "unknown precision");
    CGP_REQUIRE(o.guess >= CGP_GUESS_ZERO && o.guess <= CGP_GUESS_LEARNED, "unknown guess mode");
    CGP_REQUIRE(o.tol > 0.0 && std::isfinite(o.tol), "tol must be positive");
    CGP_REQUIRE(o.refine_delta >= 0.0 && o.refine_delta < 1.0, "refine_delta must be in [0, 1)");
    CGP_REQUIRE(o.max_iter >= 0 && o.max_iter <= 10000000, "max_iter must be in [0, 1e7]");
    CGP_REQUIRE(o.spmv_lanes == 0 || o.spmv_lanes == 1 || o.spmv_lanes == 2 || o.spmv_lanes == 4 ||
                    o.spmv_lanes == 8,
                "spmv_lanes must be 0, 1, 2, 4 or 8");
    CGP_REQUIRE(o.blocks >= 0, "blocks must be >= 0");
    CGP_REQUIRE(o.engine >= CGP_ENGINE_AUTO && o.engine <= CGP_ENGINE_STAGED_ROWS, "unknown engine");
    CGP_REQUIRE(o.precond_degree == CGP_DEGREE_TUNED || (o.precond_degree >= 0 && o.precond_degree <= TILE_MAX_DEGREE),
                "precond_degree must be in [0, 8] or CGP_DEGREE_TUNED");
    CGP_REQUIRE(o.deflation == 0 || o.deflation == 1, "deflation must be 0 or 1");
    CGP_REQUIRE(o.launches_per_graph >= 0 && o.launches_per_graph % 2 == 0 && o.launches_per_graph <= 4096,
                "launches_per_graph must be even and <= 4096");
    CGP_REQUIRE(o.stage_budget >= 0 && o.stage_budget <= MAX_STAGE_BUDGET, "stage_budget must be in [0, 65536]");
}

Model &get_model(cgp_ctx ctx, cgp_model h) {
    auto it = ctx->models.find(h);
    if (it == ctx->models.end()) throw Error{CGP_E_INVALID, "unknown model handle"};
    return *it->second;
}

}  // namespace

extern "C" {

const char *cgp_last_error(cgp_ctx ctx) {
    (void)ctx;   // the message is kept per host thread
    return g_last_error.c_str();
}

cgp_status cgp_create(cgp_ctx *out, int32_t device, void *hip_stream) {
    return guarded([&] {
        CGP_REQUIRE(out != nullptr, "null output pointer");
        *out = nullptr;
        int ndev = 0;
        CGP_HIP(hipGetDeviceCount(&ndev));
        CGP_REQUIRE(device >= 0 && device < ndev, "device index out of range");
        auto ctx = std::make_unique<cgp_ctx_s>();
        ctx->device = device;
        CGP_HIP(hipSetDevice(device));
        ctx->stream = static_cast<hipStream_t>(hip_stream);
        CGP_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
        CGP_HIP(hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, device));
        ctx->max_blocks_per_cu = std::max(1, pcg_max_blocks_per_cu());
        noalloc_init(device);   // the no-allocation solve's array on this device (once per device)
        ctx->sync.alloc(1);
        ctx->sink_flag.alloc(2);
        CGP_HIP(hipMemset(ctx->sync.p, 0, sizeof(GridSync)));
        CGP_HIP(hipHostMalloc(reinterpret_cast<void **>(&ctx->host_flag), 2 * sizeof(int32_t), hipHostMallocMapped));
        ctx->host_flag[0] = ctx->host_flag[1] = 0;
        CGP_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&ctx->host_flag_dev), ctx->host_flag, 0));
        CGP_HIP(hipEventCreateWithFlags(&ctx->chunk_ev[0], hipEventDisableTiming));
        CGP_HIP(hipEventCreateWithFlags(&ctx->chunk_ev[1], hipEventDisableTiming));
        int khz = 0;
        CGP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device));
        if (khz <= 0) khz = 100000;
        ctx->timeout_ticks = static_cast<uint64_t>(khz) * 1000ull * 4ull;   // 4 s per barrier wait
        CGP_HIP(hipDeviceSynchronize());
        *out = ctx.release();
    });
}

cgp_status cgp_destroy(cgp_ctx ctx) {
    return guarded([&] {
        CGP_REQUIRE(ctx != nullptr, "null context");
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        for (auto &g : ctx->graphs) {
            if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
            if (g.second.graph) (void)hipGraphDestroy(g.second.graph);
        }
        ctx->plans.clear();
        ctx->models.clear();
        if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
        for (auto &e : ctx->tev) (void)hipEventDestroy(e);
        for (auto &e : ctx->chunk_ev)
            if (e) (void)hipEventDestroy(e);
        if (ctx->host_flag) (void)hipHostFree(ctx->host_flag);
        delete ctx;
    });
}

cgp_status cgp_set_stream(cgp_ctx ctx, void *hip_stream) {
    return guarded([&] {
        CGP_REQUIRE(ctx != nullptr, "null context");
        CGP_REQUIRE(!ctx->capturing, "cannot change the stream during graph capture");
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    });
}

cgp_status cgp_sync(cgp_ctx ctx) {
    return guarded([&] {
        use_device(ctx);
        CGP_HIP(hipStreamSynchronize(ctx->stream));
        CGP_HIP(hipGetLastError());
    });
}

int32_t cgp_device_cus(cgp_ctx ctx) { return ctx ? ctx->cus : 0; }

int64_t cgp_stage_launches(cgp_ctx ctx) { return ctx ? ctx->stage_launches : 0; }

cgp_status cgp_stage_timing(cgp_ctx ctx, int32_t enable) {
    return guarded([&] {
        CGP_REQUIRE(ctx != nullptr, "null context");
        CGP_REQUIRE(enable == 0 || enable == 1, "enable must be 0 or 1");
        CGP_REQUIRE(!ctx->capturing, "stage timing cannot change during graph capture");
        ctx->time_stages = enable == 1;
        if (enable) {
            ctx->timed_launches[0] = ctx->timed_launches[1] = 0;
            ctx->timed_us[0] = ctx->timed_us[1] = 0.0;
        }
    });
}

cgp_status cgp_stage_timing_read(cgp_ctx ctx, int64_t *h_stage_launches, double *h_stage_us,
                                 int64_t *h_coarse_launches, double *h_coarse_us) {
    return guarded([&] {
        CGP_REQUIRE(ctx != nullptr, "null context");
        if (h_stage_launches) *h_stage_launches = ctx->timed_launches[0];
        if (h_stage_us) *h_stage_us = ctx->timed_us[0];
        if (h_coarse_launches) *h_coarse_launches = ctx->timed_launches[1];
        if (h_coarse_us) *h_coarse_us = ctx->timed_us[1];
    });
}

// ------------------------------------------------------------------ meshes

cgp_status cgp_mesh_upload(cgp_ctx ctx, const double *h_xy, int64_t n_nodes, const int32_t *h_tri,
                           int64_t n_tris, const uint8_t *h_dirichlet, int32_t k_levels, cgp_mesh *out) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(out != nullptr && h_xy != nullptr && h_tri != nullptr && h_dirichlet != nullptr,
                    "null pointer argument");
        CGP_REQUIRE(n_nodes >= 3 && n_tris >= 1, "mesh needs at least one triangle");
        CGP_REQUIRE(n_nodes < INT32_MAX && 9 * n_tris < INT32_MAX, "mesh exceeds 32-bit indexing");
        CGP_REQUIRE(k_levels >= 0 && k_levels <= 6, "k_levels must be in [0, 6]");
        CGP_REQUIRE(!ctx->capturing, "cgp_mesh_upload cannot be captured in a graph");
        auto m = std::make_unique<Mesh>();
        build_hierarchy(ctx->stream, *m, h_xy, n_nodes, h_tri, n_tris, h_dirichlet, k_levels);
        const int32_t h = ctx->next_mesh++;
        ctx->meshes[h] = std::move(m);
        *out = h;
    });
}

cgp_status cgp_mesh_info(cgp_ctx ctx, cgp_mesh mesh, int32_t level, int64_t *n_nodes, int64_t *n_tris,
                         int64_t *n_edges, int64_t *nnz) {
    return guarded([&] {
        CGP_REQUIRE(ctx != nullptr, "null context");
        Mesh &m = get_mesh(ctx, mesh);
        CGP_REQUIRE(level >= 0 && level <= m.k, "level out of range");
        const Level &L = m.lv[level];
        if (n_nodes) *n_nodes = L.n;
        if (n_tris) *n_tris = L.T;
        if (n_edges) *n_edges = L.E;
        if (nnz) *nnz = level == 0 ? m.nnz : 0;
    });
}

cgp_status cgp_mesh_levels(cgp_ctx ctx, cgp_mesh mesh, int32_t *k_levels) {
    return guarded([&] {
        CGP_REQUIRE(ctx != nullptr && k_levels != nullptr, "null argument");
        *k_levels = get_mesh(ctx, mesh).k;
    });
}

cgp_status cgp_mesh_download(cgp_ctx ctx, cgp_mesh mesh, int32_t level, double *h_xy, int32_t *h_tri,
                             uint8_t *h_dirichlet, int32_t *h_edge_ends) {
    return guarded([&] {
        use_device(ctx);
        Mesh &m = get_mesh(ctx, mesh);
        CGP_REQUIRE(level >= 0 && level <= m.k, "level out of range");
        const Level &L = m.lv[level];
        CGP_HIP(hipStreamSynchronize(ctx->stream));
        if (h_xy) CGP_HIP(hipMemcpy(h_xy, L.xy.p, 2 * L.n * sizeof(double), hipMemcpyDeviceToHost));
        if (h_tri) CGP_HIP(hipMemcpy(h_tri, L.tri.p, 3 * L.T * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (h_dirichlet) CGP_HIP(hipMemcpy(h_dirichlet, L.dir.p, L.n, hipMemcpyDeviceToHost));
        if (h_edge_ends && L.E > 0)
            CGP_HIP(hipMemcpy(h_edge_ends, L.ends.p, 2 * L.E * sizeof(int32_t), hipMemcpyDeviceToHost));
    });
}

cgp_status cgp_mesh_matrix(cgp_ctx ctx, cgp_mesh mesh, int32_t *h_rowptr, int32_t *h_col, double *h_val,
                           double *h_dinv) {
    return guarded([&] {
        use_device(ctx);
        Mesh &m = get_mesh(ctx, mesh);
        const int64_t n = m.lv[0].n;
        CGP_HIP(hipStreamSynchronize(ctx->stream));
        if (h_rowptr) CGP_HIP(hipMemcpy(h_rowptr, m.rowptr.p, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (h_col) CGP_HIP(hipMemcpy(h_col, m.col.p, m.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (h_val) CGP_HIP(hipMemcpy(h_val, m.val.p, m.nnz * sizeof(double), hipMemcpyDeviceToHost));
        if (h_dinv) CGP_HIP(hipMemcpy(h_dinv, m.dinv.p, n * sizeof(double), hipMemcpyDeviceToHost));
    });
}

cgp_status cgp_mesh_free(cgp_ctx ctx, cgp_mesh mesh) {
    return guarded([&] {
        use_device(ctx);
        (void)get_mesh(ctx, mesh);
        CGP_REQUIRE(!ctx->capturing, "cannot free a mesh during graph capture");
        CGP_HIP(hipStreamSynchronize(ctx->stream));
        // launch plans that reference this mesh's buffers become stale
        ctx->plans.clear();
        ctx->stage_hint.clear();
        for (auto &md : ctx->models) gnn_release_mesh(*md.second, ctx->meshes[mesh].get());
        ctx->meshes.erase(mesh);
    });
}

// ------------------------------------------------------------------ CGP steps

cgp_status cgp_restrict(cgp_ctx ctx, cgp_mesh mesh, const double *d_uf, const double *d_vf, int32_t kind,
                        double scale, double *d_b, double *d_uc, double *d_vc) {
    return guarded([&] {
        use_device(ctx);
        Mesh &m = get_mesh(ctx, mesh);
        CGP_REQUIRE(d_uf != nullptr && d_vf != nullptr && d_b != nullptr, "null device pointer");
        CGP_REQUIRE(kind == CGP_SRC_CURL || kind == CGP_SRC_DIV, "kind must be CGP_SRC_CURL or CGP_SRC_DIV");
        CGP_REQUIRE(std::isfinite(scale), "scale must be finite");
        launch_restrict(ctx->stream, m, d_uf, d_vf, kind, scale, d_b, d_uc, d_vc);
    });
}

cgp_status cgp_prolong(cgp_ctx ctx, cgp_mesh mesh, const double *d_qc, double *d_qf) {
    return guarded([&] {
        use_device(ctx);
        Mesh &m = get_mesh(ctx, mesh);
        CGP_REQUIRE(d_qc != nullptr && d_qf != nullptr, "null device pointer");
        CGP_REQUIRE(d_qc != d_qf, "d_qc and d_qf must not alias");
        launch_prolong(ctx->stream, m, d_qc, d_qf);
    });
}

cgp_status cgp_lorentz_force(cgp_ctx ctx, cgp_mesh mesh, const double *d_phif, const double *d_uf,
                             const double *d_vf, double sigma, double B0, double *d_fx, double *d_fy,
                             double *d_grad_elem) {
    return guarded([&] {
        use_device(ctx);
        Mesh &m = get_mesh(ctx, mesh);
        CGP_REQUIRE(d_phif && d_uf && d_vf && d_fx && d_fy, "null device pointer");
        CGP_REQUIRE(std::isfinite(sigma) && std::isfinite(B0), "sigma and B0 must be finite");
        launch_lorentz(ctx->stream, m, d_phif, d_uf, d_vf, sigma, B0, d_fx, d_fy, d_grad_elem, !ctx->capturing);
    });
}

cgp_status cgp_velocity_correct(cgp_ctx ctx, cgp_mesh mesh, const double *d_pf, const double *d_ut,
                                const double *d_vt, const uint8_t *d_mask, double scale, double *d_u,
                                double *d_v) {
    return guarded([&] {
        use_device(ctx);
        Mesh &m = get_mesh(ctx, mesh);
        CGP_REQUIRE(d_pf && d_ut && d_vt && d_u && d_v, "null device pointer");
        CGP_REQUIRE(std::isfinite(scale), "scale must be finite");
        CGP_REQUIRE(d_u != d_v, "d_u and d_v must differ");
        CGP_REQUIRE(d_u != d_pf && d_v != d_pf, "the output must not overwrite d_pf");
        launch_velocity(ctx->stream, m, d_pf, d_ut, d_vt, d_mask, scale, d_u, d_v, !ctx->capturing);
    });
}

cgp_status cgp_surface_force(cgp_ctx ctx, cgp_mesh mesh, int32_t level, int64_t n_edges, const int32_t *d_edges,
                             const double *d_p, const double *d_u, const double *d_v, double mu, double *d_force) {
    return guarded([&] {
        use_device(ctx);
        Mesh &m = get_mesh(ctx, mesh);
        CGP_REQUIRE(level >= 0 && level <= m.k, "level out of range");
        CGP_REQUIRE(n_edges >= 0, "n_edges must be non-negative");
        CGP_REQUIRE(d_p && d_u && d_v && d_force && (n_edges == 0 || d_edges), "null device pointer");
        CGP_REQUIRE(std::isfinite(mu) && mu >= 0.0, "mu must be non-negative");
        launch_surface_force(ctx->stream, m, level, n_edges, d_edges, d_p, d_u, d_v, mu, d_force);
    });
}

cgp_status cgp_interpolate(cgp_ctx ctx, cgp_mesh mesh, int32_t level, int64_t n_pts, const double *d_pts,
                           const double *d_field, double *d_out, int32_t *d_tri) {
    return guarded([&] {
        use_device(ctx);
        Mesh &m = get_mesh(ctx, mesh);
        CGP_REQUIRE(level >= 0 && level <= m.k, "level out of range");
        CGP_REQUIRE(n_pts >= 0, "n_pts must be non-negative");
        CGP_REQUIRE(n_pts == 0 || (d_pts && d_field && d_out), "null device pointer");
        CGP_REQUIRE(n_pts == 0 || (d_out != d_field && static_cast<const void *>(d_out) !=
                                                             static_cast<const void *>(d_pts)),
                    "d_out must not overwrite an input");
        interpolate_points(ctx->stream, m, level, n_pts, d_pts, d_field, d_out, d_tri, !ctx->capturing);
    });
}

cgp_status cgp_momentum_step(cgp_ctx ctx, cgp_mesh mesh, const double *d_un, const double *d_vn,
                             const double *d_fx, const double *d_fy, const uint8_t *d_mask, double rho,
                             double mu, double dt, double tol, int32_t max_iter, double *d_ut, double *d_vt,
                             cgp_momentum_stats *h_stats) {
    return guarded([&] {
        use_device(ctx);
        Mesh &m = get_mesh(ctx, mesh);
        CGP_REQUIRE(!ctx->capturing, "cgp_momentum_step cannot be captured");
        CGP_REQUIRE(d_un && d_vn && d_fx && d_fy && d_ut && d_vt, "null device pointer");
        CGP_REQUIRE(std::isfinite(rho) && rho > 0.0, "rho must be positive");
        CGP_REQUIRE(std::isfinite(mu) && mu >= 0.0, "mu must be non-negative");
        CGP_REQUIRE(std::isfinite(dt) && dt > 0.0, "dt must be positive");
        CGP_REQUIRE(std::isfinite(tol) && tol > 0.0, "tol must be positive");
        CGP_REQUIRE(max_iter >= 1, "max_iter must be at least 1");
        CGP_REQUIRE(d_ut != d_vt, "d_ut and d_vt must differ");
        for (const double *in : {d_un, d_vn, d_fx, d_fy})
            CGP_REQUIRE(in != d_ut && in != d_vt, "the outputs must not overwrite an input");
        momentum_step(ctx->stream, m, d_un, d_vn, d_fx, d_fy, d_mask, rho, mu, dt, tol, max_iter, d_ut, d_vt,
                      h_stats);
    });
}

cgp_status cgp_poisson_solve(cgp_ctx ctx, int32_t n_inst, const cgp_mesh *h_meshes, const double *const *h_d_b,
                             double *const *h_d_phi, const double *const *h_d_prev1,
                             const double *const *h_d_prev2, const cgp_solve_opts *h_opts,
                             cgp_solve_stats *d_stats) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(n_inst >= 1, "n_inst must be >= 1");
        CGP_REQUIRE(h_meshes && h_d_b && h_d_phi && h_opts && d_stats, "null argument");
        const cgp_solve_opts &o = *h_opts;
        check_opts(o);
        Model *model = nullptr;
        if (o.guess == CGP_GUESS_LEARNED) {
            auto mit = ctx->models.find(o.model);
            CGP_REQUIRE(mit != ctx->models.end(), "CGP_GUESS_LEARNED needs a valid model handle");
            model = mit->second.get();
        }
        const bool need_prev = o.guess == CGP_GUESS_EXTRAP || o.guess == CGP_GUESS_LEARNED;
        std::vector<Mesh *> ms(n_inst);
        for (int i = 0; i < n_inst; ++i) {
            ms[i] = &get_mesh(ctx, h_meshes[i]);
            for (int j = 0; j < i; ++j)
                CGP_REQUIRE(h_meshes[j] != h_meshes[i], "each instance needs its own mesh");
            CGP_REQUIRE(h_d_b[i] != nullptr && h_d_phi[i] != nullptr, "null b or phi");
            CGP_REQUIRE(static_cast<const void *>(h_d_b[i]) != static_cast<const void *>(h_d_phi[i]),
                        "b and phi must not alias");
            if (need_prev) {
                CGP_REQUIRE(h_d_prev1 && h_d_prev2 && h_d_prev1[i] && h_d_prev2[i],
                            "prev1 and prev2 are required for this guess mode");
                CGP_REQUIRE(h_d_prev1[i] != h_d_phi[i] && h_d_prev2[i] != h_d_phi[i],
                            "prev1/prev2 must not alias phi");
            }
        }
        // preconditioner degree of each instance: the option's, or (CGP_DEGREE_TUNED) the one
        // cgp_autotune chose for the instance's mesh
        std::vector<int> degs(n_inst, std::max(1, o.precond_degree));
        if (o.precond_degree == CGP_DEGREE_TUNED) {
            for (int i = 0; i < n_inst; ++i) {
                degs[i] = ms[i]->tuned_degree[o.precision][o.deflation];
                CGP_REQUIRE(degs[i] >= 1, "CGP_DEGREE_TUNED: a mesh has no autotuned degree for this precision and "
                                          "deflation (call cgp_autotune)");
            }
        }
        const int degree = *std::max_element(degs.begin(), degs.end());
        // AUTO under graph capture: the persistent engine for plain Jacobi, the staged engine's
        // recorded launches for the Chebyshev preconditioner or deflation
        const bool persistent = o.engine == CGP_ENGINE_PERSISTENT ||
                                (o.engine == CGP_ENGINE_AUTO && ctx->capturing && degree < 2 && o.deflation != 1);
        if (degree >= 2 && (persistent || o.engine == CGP_ENGINE_STAGED_ROWS))
            throw Error{CGP_E_UNSUPPORTED, "the Chebyshev preconditioner needs CGP_ENGINE_STAGED"};
        // tiled iteration when every instance's mesh fits it with one matrix width (AUTO: only
        // for the Chebyshev preconditioner; the row-range kernel is the faster Jacobi iteration)
        std::vector<TilePlan *> tp(n_inst, nullptr);
        bool tiled = !persistent && o.engine != CGP_ENGINE_STAGED_ROWS &&
                     (o.engine == CGP_ENGINE_STAGED || degree >= 2 || o.deflation == 1);
        for (int i = 0; i < n_inst && tiled; ++i) {
            tp[i] = tile_plan(ctx->aux, *ms[i], degs[i]);
            tiled = tp[i] != nullptr && tp[i]->width == tp[0]->width;
        }
        // the records the stage kernel reads: split (off-diagonal) records when every instance
        // has them, else the plans' common width
        int kwidth = 0;
        if (tiled) {
            kwidth = SPLIT_WIDTH;
            for (int i = 0; i < n_inst; ++i)
                if (tp[i]->kwidth != SPLIT_WIDTH) kwidth = tp[0]->width;
        }
        if (degree >= 2 && !tiled)
            throw Error{CGP_E_UNSUPPORTED, "a mesh does not fit the tiled iteration the Chebyshev preconditioner needs"};
        const bool defl = o.deflation == 1;
        if (defl) {
            if (!tiled) throw Error{CGP_E_UNSUPPORTED, "deflation needs the tiled iteration (CGP_ENGINE_STAGED)"};
            for (int i = 0; i < n_inst; ++i)
                if (!tile_deflation(ctx->aux, *ms[i], *tp[i]))
                    throw Error{CGP_E_UNSUPPORTED, "a mesh does not fit deflation (tiles or couplings)"};
        }
        SolveParams prm{};
        prm.tol = o.tol;
        // fewer iterations between refinements with the Chebyshev preconditioner: longer fp32 runs
        prm.delta = o.refine_delta > 0.0 ? o.refine_delta : (degree >= 2 ? 0.01 : 0.1);
        prm.max_iter = o.max_iter > 0 ? o.max_iter : 100000;
        prm.precision = o.precision;
        const int launches = o.launches_per_graph > 0 ? o.launches_per_graph : 16;

        const int max_grid = ctx->cus * ctx->max_blocks_per_cu;
        // the persistent engine takes every co-resident workgroup slot by default: each of its
        // workgroups walks thousands of rows per stage, and more of them in flight hide the
        // latency of the row gathers
        int grid = o.blocks > 0 ? o.blocks : (persistent ? max_grid : ctx->cus);
        grid = std::min(grid, max_grid);
        for (int i = 0; i < n_inst; ++i) ensure_work(*ms[i], ctx->stream);

        // instances in groups of at most `grid` (one workgroup minimum each)
        for (int g0 = 0; g0 < n_inst; g0 += (persistent ? grid : n_inst)) {
            const int gn = persistent ? std::min(grid, n_inst - g0) : n_inst;
            std::vector<int64_t> rows(gn);
            for (int i = 0; i < gn; ++i) rows[i] = ms[g0 + i]->lv[0].n;
            // staged: one row per thread, so ceil(n / block) workgroups per instance;
            // persistent: the co-resident grid split between the instances
            std::vector<int32_t> nb;
            if (persistent) {
                nb = split_blocks(rows, grid);
            } else if (tiled) {
                for (int i = 0; i < gn; ++i) nb.push_back(tp[g0 + i]->nparts);
            } else {
                for (int64_t r : rows) nb.push_back(static_cast<int32_t>((r + pcg_block_size() - 1) / pcg_block_size()));
            }
            int used = 0;
            for (int v : nb) used += v;
            // lanes per matrix row of the general row-range stages: 4 for the staged engines' row
            // blocks of at most a few hundred rows; 1 for the persistent engine, whose workgroups
            // own thousands of rows (one row per thread keeps BLOCK rows' gathers in flight per
            // pass, where 8 lanes would take 8 times the passes)
            auto lanes_of = [&](Mesh &m) {
                (void)m;
                return o.spmv_lanes ? o.spmv_lanes : (persistent ? 1 : 4);
            };
            // cache key: everything the launch records depend on
            std::ostringstream key;
            key << o.precision << ':' << o.guess << ':' << used << ':' << launches << ':' << persistent << ':'
                << tiled << ':' << defl << ':';
            for (int i = 0; i < gn; ++i) {
                const int ii = g0 + i;
                key << h_meshes[ii] << ',' << degs[ii] << ',' << lanes_of(*ms[ii]) << ',' << nb[i] << ','
                    << (const void *)h_d_b[ii]
                    << ',' << (const void *)h_d_phi[ii] << ','
                    << (const void *)(need_prev ? h_d_prev1[ii] : nullptr) << ','
                    << (const void *)(need_prev ? h_d_prev2[ii] : nullptr) << ';';
            }
            // the same key without the vectors, for the stage-count prediction
            std::ostringstream hkey;
            hkey << o.precision << ':' << o.guess << ':' << launches << ':' << tiled << ':' << defl << ':' << o.tol
                 << ':';
            for (int i = 0; i < gn; ++i) hkey << h_meshes[g0 + i] << ',' << degs[g0 + i] << ';';
            auto it = ctx->plans.find(key.str());
            std::shared_ptr<Plan> plan_sp;
            if (it != ctx->plans.end()) {
                plan_sp = it->second;
            } else {
                if (ctx->capturing && !persistent)
                    throw Error{CGP_E_INVALID, "a staged solve recorded in a graph needs an uncaptured solve of the "
                                               "same meshes, vectors and options first (its launch records and "
                                               "stage count)"};
                auto p = std::make_shared<Plan>();
                size_t npart = 0, nmu = 0, ncb_total = 0;
                for (int i = 0; i < gn; ++i) {
                    const int v = nb[i], A = tiled ? tp[g0 + i]->agg : 0;
                    npart += static_cast<size_t>(2) * NPART * v;
                    nmu += A * v;
                    ncb_total += (A * v + COARSE_ROWS - 1) / COARSE_ROWS;
                }
                if (!defl) nmu = ncb_total = 0;
                auto align = [](size_t x) { return (x + 255) / 256 * 256; };
                const size_t off_bi = align(sizeof(InstDesc) * gn);
                const size_t off_rng = align(off_bi + sizeof(int32_t) * used);
                const size_t off_ctl = align(off_rng + sizeof(RowRange) * used);
                const size_t off_done_at = align(off_ctl + sizeof(Ctl) * 2 * gn);
                const size_t off_done = align(off_done_at + sizeof(int32_t) * gn);
                const size_t off_prm = align(off_done + sizeof(int32_t));
                const size_t off_part = align(off_prm + sizeof(SolveParams));
                const size_t off_mu = align(off_part + sizeof(double) * npart);
                const size_t off_cpart = align(off_mu + sizeof(double) * nmu);
                const size_t off_cbi = align(off_cpart + sizeof(double) * (NRED + 1) * ncb_total);
                const size_t off_crec = align(off_cbi + sizeof(int32_t) * ncb_total);
                const size_t total = off_crec + (defl ? sizeof(CoarseRec) * gn : 0);
                p->buf.alloc(total);
                std::vector<uint8_t> host(off_ctl, 0);
                InstDesc *hd = reinterpret_cast<InstDesc *>(host.data());
                int32_t *hbi = reinterpret_cast<int32_t *>(host.data() + off_bi);
                double *dpart = reinterpret_cast<double *>(p->buf.p + off_part);
                Ctl *dctl = reinterpret_cast<Ctl *>(p->buf.p + off_ctl);
                int blk = 0, cblk = 0;
                size_t poff = 0;
                double *dmu = reinterpret_cast<double *>(p->buf.p + off_mu);
                double *dcpart = reinterpret_cast<double *>(p->buf.p + off_cpart);
                std::vector<int32_t> hcbi;
                for (int i = 0; i < gn; ++i) {
                    const int ii = g0 + i;
                    Mesh &m = *ms[ii];
                    InstDesc d = describe_instance(m, work_ptrs(m.work), tiled ? tp[ii] : nullptr, kwidth, degs[ii], defl,
                                                   persistent, lanes_of(m), o.guess, h_d_b[ii], h_d_phi[ii],
                                                   need_prev ? h_d_prev1[ii] : nullptr,
                                                   need_prev ? h_d_prev2[ii] : nullptr, ctx->aux);
                    d.blk0 = blk;
                    d.nblk = nb[i];
                    d.stats_index = i;
                    d.chunk = static_cast<int32_t>((m.lv[0].n + nb[i] - 1) / nb[i]);
                    d.partials = dpart + poff;
                    d.ctl = dctl + 2 * i;
                    if (defl) {
                        d.ncb = (d.agg * nb[i] + COARSE_ROWS - 1) / COARSE_ROWS;
                        d.cblk0 = cblk;
                        d.mu = dmu;
                        d.cpart = dcpart;
                        dmu += d.agg * nb[i];
                        dcpart += static_cast<size_t>(NRED + 1) * d.ncb;
                        for (int v = 0; v < d.ncb; ++v) hcbi.push_back(i);
                        p->crecs.push_back(coarse_record(d, cblk));
                        cblk += d.ncb;
                    }
                    hd[i] = d;
                    for (int v = 0; v < nb[i]; ++v) hbi[blk + v] = i;
                    blk += nb[i];
                    poff += static_cast<size_t>(2) * NPART * nb[i];
                }
                CGP_HIP(hipMemcpyAsync(p->buf.p, host.data(), off_rng, hipMemcpyHostToDevice, ctx->aux));
                p->one = hd[0];
                if (defl) {
                    // mu and the coarse records start at zero: the first stages read them before
                    // any coarse step has produced values for them
                    CGP_HIP(hipMemsetAsync(p->buf.p + off_mu, 0, off_cbi - off_mu, ctx->aux));
                    CGP_HIP(hipMemcpyAsync(p->buf.p + off_cbi, hcbi.data(), sizeof(int32_t) * hcbi.size(),
                                           hipMemcpyHostToDevice, ctx->aux));
                    p->d_cblk_inst = reinterpret_cast<int32_t *>(p->buf.p + off_cbi);
                    p->d_crecs = reinterpret_cast<CoarseRec *>(p->buf.p + off_crec);
                    CGP_HIP(hipMemcpyAsync(p->d_crecs, p->crecs.data(), sizeof(CoarseRec) * p->crecs.size(),
                                           hipMemcpyHostToDevice, ctx->aux));
                    p->cgrid = cblk;
                }
                p->d_insts = reinterpret_cast<InstDesc *>(p->buf.p);
                p->d_block_inst = reinterpret_cast<int32_t *>(p->buf.p + off_bi);
                p->d_ranges = reinterpret_cast<RowRange *>(p->buf.p + off_rng);
                p->d_done_at = reinterpret_cast<int32_t *>(p->buf.p + off_done_at);
                p->d_done = reinterpret_cast<int32_t *>(p->buf.p + off_done);
                p->d_prm = reinterpret_cast<SolveParams *>(p->buf.p + off_prm);
                p->grid = used;
                p->n_inst = gn;
                p->unb = std::all_of(nb.begin(), nb.end(), [&](int32_t v) { return v == nb[0]; }) ? nb[0] : 0;
                launch_ranges(ctx->aux, p->d_insts, p->d_block_inst, used, p->d_ranges);
                std::vector<RowRange> hr(used);
                CGP_HIP(hipMemcpyAsync(hr.data(), p->d_ranges, sizeof(RowRange) * used, hipMemcpyDeviceToHost,
                                       ctx->aux));
                CGP_HIP(hipStreamSynchronize(ctx->aux));
                for (const RowRange &r : hr) p->halo = std::max(p->halo, r.c1 - r.c0 + 1);
                plan_sp = p;
                ctx->plans[key.str()] = std::move(p);
            }
            Plan *plan = plan_sp.get();
            if (ctx->capturing) ctx->capture_plans.push_back(plan_sp);
            SolveParams gp = prm;
            gp.n_inst = gn;
            gp.stats = d_stats + g0;
            if (model)   // the network's guess goes into phi; the solver judges it against prev1
                for (int i = 0; i < gn; ++i)
                    gnn_predict(ctx->stream, *model, *ms[g0 + i], h_d_b[g0 + i], h_d_prev1[g0 + i],
                                h_d_prev2[g0 + i], h_d_phi[g0 + i], !ctx->capturing);
            if (persistent) {
                launch_cg_persistent(ctx->stream, plan->d_insts, gn, plan->d_block_inst, plan->d_ranges, plan->grid,
                                     gp, ctx->sync.p, plan->d_done_at, ctx->timeout_ticks);
                continue;
            }
            // staged: graphs of stage launches (an even count each, so that the buffer parity runs
            // on from one graph to the next), replayed until every instance is done
            // `count` stage launches (and with deflation the coarse step after each) on stream st;
            // ev (optional): a start and a stop event per kernel, recorded by the dispatches themselves
            const int kps = (tiled && defl) ? 2 : 1;
            // completion flag: the host's, or under capture a device word nobody reads (a replay
            // still running must not signal the end of a later uncaptured solve)
            int32_t *done_flag = ctx->capturing ? ctx->sink_flag.p : ctx->host_flag_dev;
            auto enqueue = [&](int64_t count, hipStream_t st, hipEvent_t *ev) {
                auto evs = [&](int k) { return ev ? KernelEvents{ev[2 * k], ev[2 * k + 1]} : KernelEvents{}; };
                for (int64_t l = 0; l < count; ++l) {
                    if (tiled) {
                        launch_cg_tile(st, o.precision == CGP_FP32_IR, kwidth, defl, plan->unb, plan->d_insts,
                                       gn == 1 ? &plan->one : nullptr,
                                       plan->d_block_inst, plan->d_ranges, plan->grid, plan->d_prm,
                                       static_cast<int>(l & 1), plan->d_done, done_flag, evs(kps * l));
                        if (defl)
                            launch_cg_coarse(st, o.precision == CGP_FP32_IR, gn == 1 ? plan->crecs.data() : nullptr,
                                             plan->d_crecs, plan->d_cblk_inst, plan->cgrid, static_cast<int>(l & 1),
                                             evs(kps * l + 1));
                    } else {
                        launch_cg_step(st, o.precision == CGP_FP32_IR, plan->halo, gn, plan->d_insts,
                                       gn == 1 ? &plan->one : nullptr,
                                       plan->d_block_inst, plan->d_ranges, plan->grid, plan->d_prm,
                                       static_cast<int>(l & 1), plan->d_done, done_flag, evs(l));
                    }
                }
            };
            auto capture = [&](int count, hipGraph_t &graph, hipGraphExec_t &exec) {
                // the launch template is recorded on the private stream (the caller's may be the null stream)
                CGP_HIP(hipStreamBeginCapture(ctx->aux, hipStreamCaptureModeRelaxed));
                enqueue(count, ctx->aux, nullptr);
                CGP_HIP(hipStreamEndCapture(ctx->aux, &graph));
                CGP_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            };
            if (ctx->capturing) {
                // recorded in the caller's graph: the boot, a fixed number of stage launches (stages
                // past an instance's end find it done and return) and the closing kernel, which
                // marks instances still running after the last launch as aborted
                CGP_REQUIRE(o.stage_budget > 0 || plan->last_stages > 0,
                            "no stage count to size the recorded solve (stage_budget = 0 and no finished "
                            "uncaptured solve of this launch plan)");
                const int64_t budget = o.stage_budget > 0 ? o.stage_budget
                                                          : (static_cast<int64_t>(plan->last_stages) * 5) / 4 + 8;
                CGP_REQUIRE(budget <= MAX_STAGE_BUDGET, "stage budget above the limit of a recorded solve");
                launch_cg_boot(ctx->stream, plan->d_insts, gn, gp, plan->d_prm, plan->d_done);
                enqueue(budget, ctx->stream, nullptr);
                launch_cg_close(ctx->stream, plan->d_insts, gn, plan->d_prm, static_cast<int>((budget - 1) & 1));
                continue;
            }
            if (!plan->exec) {
                capture(launches, plan->graph, plan->exec);
                plan->launches = launches;
                if (launches > TAIL_LAUNCHES) capture(TAIL_LAUNCHES, plan->tail_graph, plan->tail_exec);
            }
            volatile int32_t *flag = ctx->host_flag;
            flag[0] = 0;
            launch_cg_boot(ctx->stream, plan->d_insts, gn, gp, plan->d_prm, plan->d_done);
            // each instance needs at most max_iter iterations plus three stages per
            // refinement (at most one per iteration) plus a few set-up stages
            const int64_t max_stages = 4 * static_cast<int64_t>(prm.max_iter) + 16;
            // full graphs while they end before the launch count the previous solve of this plan
            // needed, then short ones, so that little runs past the end
            int64_t predicted = plan->last_stages;
            if (predicted == 0) {
                auto h = ctx->stage_hint.find(hkey.str());
                if (h != ctx->stage_hint.end()) predicted = h->second;
            }
            int64_t issued = 0;
            int64_t chunk = 0;
            bool finished = false;
            if (ctx->time_stages) {
                // the same chunks, enqueued launch by launch between events; each chunk is waited
                // for and its kernels' durations added up before the next one is enqueued
                while (!*flag) {
                    if (issued >= max_stages + 2 * plan->launches)
                        throw Error{CGP_E_ABORTED, "staged solve did not terminate"};
                    const bool tail = plan->tail_exec && predicted > 0 && issued + plan->launches > predicted;
                    const int count = tail ? TAIL_LAUNCHES : plan->launches;
                    const size_t nk = static_cast<size_t>(kps) * count;   // kernels in the chunk
                    while (ctx->tev.size() < 2 * nk) {
                        hipEvent_t e;
                        CGP_HIP(hipEventCreate(&e));
                        ctx->tev.push_back(e);
                    }
                    enqueue(count, ctx->stream, ctx->tev.data());
                    CGP_HIP(hipEventSynchronize(ctx->tev[2 * nk - 1]));
                    for (size_t q = 0; q < nk; ++q) {
                        float msec = 0.f;
                        CGP_HIP(hipEventElapsedTime(&msec, ctx->tev[2 * q], ctx->tev[2 * q + 1]));
                        const int kind = (kps == 2 && (q % 2) == 1) ? 1 : 0;
                        ctx->timed_us[kind] += 1e3 * static_cast<double>(msec);
                        ++ctx->timed_launches[kind];
                    }
                    ctx->stage_launches += count;
                    issued += count;
                }
                finished = true;
            }
            while (!finished) {
                // two chunks in flight, but none beyond the predicted end before the device has
                // had the chance to report completion (every launch past the end costs a stage
                // that finds the solve done)
                const bool past = predicted > 0 && issued >= predicted;
                if (chunk >= 2 || (past && chunk >= 1)) {
                    // wait for the older chunk in flight, or past the prediction for the newest
                    // (or for the device to report completion)
                    hipEvent_t old = ctx->chunk_ev[(past ? chunk - 1 : chunk) & 1];
                    for (;;) {
                        if (*flag) {
                            finished = true;
                            break;
                        }
                        const hipError_t q = hipEventQuery(old);
                        if (q == hipSuccess) break;
                        if (q != hipErrorNotReady) CGP_HIP(q);
                    }
                    if (finished) break;
                    if (*flag) break;
                }
                if (issued >= max_stages + 2 * plan->launches)
                    throw Error{CGP_E_ABORTED, "staged solve did not terminate"};
                const bool tail = plan->tail_exec && predicted > 0 && issued + plan->launches > predicted;
                CGP_HIP(hipGraphLaunch(tail ? plan->tail_exec : plan->exec, ctx->stream));
                CGP_HIP(hipEventRecord(ctx->chunk_ev[chunk & 1], ctx->stream));
                const int count = tail ? TAIL_LAUNCHES : plan->launches;
                ctx->stage_launches += count;
                issued += count;
                ++chunk;
            }
            plan->last_stages = flag[1];
            ctx->stage_hint[hkey.str()] = flag[1];
        }
    });
}

cgp_status cgp_solve_check(cgp_ctx ctx, int32_t n_inst, const cgp_solve_stats *d_stats, cgp_solve_stats *h_stats) {
    cgp_status result = CGP_OK;
    cgp_status rc = guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(n_inst >= 1 && d_stats != nullptr, "bad arguments");
        std::vector<cgp_solve_stats> tmp(n_inst);
        CGP_HIP(hipStreamSynchronize(ctx->stream));
        CGP_HIP(hipMemcpy(tmp.data(), d_stats, n_inst * sizeof(cgp_solve_stats), hipMemcpyDeviceToHost));
        if (h_stats) std::copy(tmp.begin(), tmp.end(), h_stats);
        for (int i = 0; i < n_inst && result == CGP_OK; ++i) {
            switch (tmp[i].status) {
            case CGP_SOLVE_OK: break;
            case CGP_SOLVE_NOCONV: result = CGP_E_NOCONV; break;
            case CGP_SOLVE_BREAKDOWN: result = CGP_E_BREAKDOWN; break;
            default: result = CGP_E_ABORTED; break;
            }
            if (result != CGP_OK) set_error("instance " + std::to_string(i) + " did not converge");
        }
    });
    return rc != CGP_OK ? rc : result;
}

cgp_status cgp_poisson_solve_noalloc(cgp_ctx ctx, cgp_mesh mesh, const double *d_b, double *d_phi,
                                     const double *d_prev1, const double *d_prev2, const cgp_solve_opts *h_opts,
                                     cgp_solve_stats *d_stats) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(d_b && d_phi && h_opts && d_stats, "null argument");
        CGP_REQUIRE(static_cast<const void *>(d_b) != static_cast<const void *>(d_phi), "b and phi must not alias");
        const cgp_solve_opts &o = *h_opts;
        check_opts(o);
        CGP_REQUIRE(!ctx->capturing, "cgp_poisson_solve_noalloc waits for the device: it cannot be captured");
        if (o.guess == CGP_GUESS_LEARNED)
            throw Error{CGP_E_UNSUPPORTED, "the learned guess allocates the network's activations per mesh"};
        if (o.engine == CGP_ENGINE_PERSISTENT)
            throw Error{CGP_E_UNSUPPORTED, "the no-allocation solve runs the staged engine"};
        if (o.precond_degree == CGP_DEGREE_TUNED)
            throw Error{CGP_E_UNSUPPORTED, "the no-allocation solve takes an explicit preconditioner degree"};
        if (o.guess == CGP_GUESS_EXTRAP) {
            CGP_REQUIRE(d_prev1 && d_prev2, "prev1 and prev2 are required for this guess mode");
            CGP_REQUIRE(d_prev1 != d_phi && d_prev2 != d_phi, "prev1/prev2 must not alias phi");
        }
        Mesh &m = get_mesh(ctx, mesh);
        const int64_t n = m.lv[0].n;
        const int degree = std::max(1, o.precond_degree);
        const bool defl = o.deflation == 1;
        const bool tiled = o.engine != CGP_ENGINE_STAGED_ROWS && (o.engine == CGP_ENGINE_STAGED || degree >= 2 || defl);
        if ((degree >= 2 || defl) && !tiled)
            throw Error{CGP_E_UNSUPPORTED, "the Chebyshev preconditioner and deflation need the tiled iteration"};
        TilePlan *T = nullptr;
        if (tiled) {
            T = m.tiles[degree] ? m.tiles[degree].get() : nullptr;
            CGP_REQUIRE(T != nullptr && T->nparts > 0,
                        "the mesh's tiled plan of this degree is not built: call cgp_poisson_solve with this "
                        "degree on the mesh first");
            CGP_REQUIRE(degree < 2 || m.gershgorin > 0.0,
                        "the mesh's spectral bound is not computed: call cgp_poisson_solve with this degree first");
            CGP_REQUIRE(!defl || T->defl_state == 1,
                        "the mesh's deflation data is not built: call cgp_poisson_solve with deflation first");
        }
        const int nblk = tiled ? T->nparts : static_cast<int>((n + pcg_block_size() - 1) / pcg_block_size());
        const int na = defl ? T->agg * nblk : 0;
        const int ncb = defl ? (na + COARSE_ROWS - 1) / COARSE_ROWS : 0;
        // layout of the scratch array (every piece 256-byte aligned)
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t at = off;
            off = (off + bytes + 255) / 256 * 256;
            return at;
        };
        // the iteration's vectors: the row-range kernel's separate arrays, or the tiled
        // iteration's row-interleaved (r, w, s, D^-1) and (u, p) in the solve's precision and c
        const bool mixed = o.precision == CGP_FP32_IR;
        size_t o_r = 0, o_w = 0, o_s = 0, o_p = 0, o_u = 0, o_r32 = 0, o_w32 = 0, o_s32 = 0, o_p32 = 0, o_c32 = 0,
               o_u32 = 0, o_rwsd = 0, o_up = 0;
        if (!tiled) {
            o_r = take(2 * n * sizeof(double));
            o_w = take(2 * n * sizeof(double));
            o_s = take(2 * n * sizeof(double));
            o_p = take(n * sizeof(double));
            o_u = take(n * sizeof(double));
            o_r32 = take(2 * n * sizeof(float));
            o_w32 = take(2 * n * sizeof(float));
            o_s32 = take(2 * n * sizeof(float));
            o_p32 = take(n * sizeof(float));
            o_c32 = take(n * sizeof(float));
            o_u32 = take(n * sizeof(float));
            o_rwsd = o_up = o_r;   // not read by the row-range kernel
        } else {
            const size_t e = mixed ? sizeof(float) : sizeof(double);
            o_rwsd = take(8 * n * e);
            o_up = take(2 * n * e);
            o_c32 = take(n * sizeof(float));
            // the row-range arrays are not read by the tiled kernel; they alias the interleaved buffer
            o_r = o_w = o_s = o_p = o_u = o_r32 = o_w32 = o_s32 = o_p32 = o_u32 = o_rwsd;
        }
        const size_t o_inst = take(sizeof(InstDesc)), o_bi = take(sizeof(int32_t) * nblk),
                     o_rng = take(sizeof(RowRange) * nblk), o_ctl = take(2 * sizeof(Ctl)), o_done = take(sizeof(int32_t)),
                     o_prm = take(sizeof(SolveParams)), o_part = take(sizeof(double) * 2 * NPART * nblk),
                     o_zero = take(sizeof(double) * (na + (NRED + 1) * ncb)),
                     o_cbi = take(sizeof(int32_t) * std::max(ncb, 1)),
                     o_crec = take(sizeof(CoarseRec));
        if (off > CGP_NOALLOC_SCRATCH_BYTES) {
            std::ostringstream msg;
            msg << "the solve needs " << off << " bytes of scratch; the no-allocation array holds "
                << CGP_NOALLOC_SCRATCH_BYTES;
            throw Error{CGP_E_INVALID, msg.str()};
        }
        uint8_t *base = noalloc_scratch(ctx->device);
        CGP_REQUIRE(base != nullptr, "the no-allocation array of this device was not looked up");
        auto at = [&](size_t o_) { return base + o_; };
        WorkPtrs ws{reinterpret_cast<double *>(at(o_r)),   reinterpret_cast<double *>(at(o_w)),
                    reinterpret_cast<double *>(at(o_s)),   reinterpret_cast<double *>(at(o_p)),
                    reinterpret_cast<double *>(at(o_u)),   reinterpret_cast<float *>(at(o_r32)),
                    reinterpret_cast<float *>(at(o_w32)),  reinterpret_cast<float *>(at(o_s32)),
                    reinterpret_cast<float *>(at(o_p32)),  reinterpret_cast<float *>(at(o_c32)),
                    reinterpret_cast<float *>(at(o_u32)),  reinterpret_cast<float *>(at(o_rwsd)),
                    reinterpret_cast<float *>(at(o_up)),   reinterpret_cast<double *>(at(o_rwsd)),
                    reinterpret_cast<double *>(at(o_up))};
        const bool extrap = o.guess == CGP_GUESS_EXTRAP;
        const int lanes = o.spmv_lanes ? o.spmv_lanes : 4;
        InstDesc d = describe_instance(m, ws, T, T ? T->kwidth : 0, degree, defl, false, lanes, o.guess, d_b, d_phi,
                                       extrap ? d_prev1 : nullptr, extrap ? d_prev2 : nullptr, ctx->aux);
        d.blk0 = 0;
        d.nblk = nblk;
        d.stats_index = 0;
        d.chunk = static_cast<int32_t>((n + nblk - 1) / nblk);
        d.partials = reinterpret_cast<double *>(at(o_part));
        d.ctl = reinterpret_cast<Ctl *>(at(o_ctl));
        double *zero = reinterpret_cast<double *>(at(o_zero));
        CoarseRec cr{};
        if (defl) {
            d.ncb = ncb;
            d.cblk0 = 0;
            d.mu = zero;
            d.cpart = zero + na;
            cr = coarse_record(d, 0);
        }
        SolveParams prm{};
        prm.tol = o.tol;
        prm.delta = o.refine_delta > 0.0 ? o.refine_delta : (o.precond_degree >= 2 ? 0.01 : 0.1);
        prm.max_iter = o.max_iter > 0 ? o.max_iter : 100000;
        prm.precision = o.precision;
        prm.n_inst = 1;
        prm.stats = d_stats;
        InstDesc *d_insts = reinterpret_cast<InstDesc *>(at(o_inst));
        int32_t *d_bi = reinterpret_cast<int32_t *>(at(o_bi));
        RowRange *d_rng = reinterpret_cast<RowRange *>(at(o_rng));
        int32_t *d_done = reinterpret_cast<int32_t *>(at(o_done));
        SolveParams *d_prm = reinterpret_cast<SolveParams *>(at(o_prm));
        int32_t *d_cbi = reinterpret_cast<int32_t *>(at(o_cbi));
        CoarseRec *d_crec = reinterpret_cast<CoarseRec *>(at(o_crec));
        hipStream_t st = ctx->stream;
        launch_noalloc_setup(st, d_insts, d, d_bi, nblk, d_cbi, ncb, zero, na + (NRED + 1) * ncb,
                             defl ? d_crec : nullptr, cr);
        if (tiled)   // D^-1 into the interleaved vectors (the array keeps whatever the last call left)
            launch_fill_rwsd(st, n, m.dinv32.p, m.dinv.p, mixed ? ws.rwsd32 : nullptr, mixed ? nullptr : ws.rwsd64);
        launch_ranges(st, d_insts, d_bi, nblk, d_rng);
        volatile int32_t *flag = ctx->host_flag;
        flag[0] = 0;
        launch_cg_boot(st, d_insts, 1, prm, d_prm, d_done);
        // chunks of stage launches enqueued directly, two in flight, until the device reports
        // completion (the row-range kernel's widest staging variant covers any halo: a row range
        // whose halo does not fit takes the general stage path)
        const int launches = o.launches_per_graph > 0 ? o.launches_per_graph : 16;
        const int64_t max_stages = 4 * static_cast<int64_t>(prm.max_iter) + 16;
        int64_t issued = 0, chunk = 0;
        for (;;) {
            if (chunk >= 2) {
                hipEvent_t old = ctx->chunk_ev[chunk & 1];
                for (;;) {
                    if (*flag) break;
                    const hipError_t q = hipEventQuery(old);
                    if (q == hipSuccess) break;
                    if (q != hipErrorNotReady) CGP_HIP(q);
                }
            }
            if (*flag) break;
            if (issued >= max_stages + 2 * launches) throw Error{CGP_E_ABORTED, "staged solve did not terminate"};
            for (int l = 0; l < launches; ++l) {
                if (tiled) {
                    launch_cg_tile(st, mixed, T->kwidth, defl, 0, d_insts, &d, d_bi, d_rng, nblk, d_prm, l & 1, d_done,
                                   ctx->host_flag_dev);
                    if (defl) launch_cg_coarse(st, mixed, &cr, d_crec, d_cbi, ncb, l & 1);
                } else {
                    launch_cg_step(st, mixed, INT32_MAX, 1, d_insts, &d, d_bi, d_rng, nblk, d_prm, l & 1, d_done,
                                   ctx->host_flag_dev);
                }
            }
            CGP_HIP(hipEventRecord(ctx->chunk_ev[chunk & 1], st));
            ctx->stage_launches += launches;
            issued += launches;
            ++chunk;
        }
    });
}

cgp_status cgp_autotune(cgp_ctx ctx, int32_t n, const cgp_mesh *h_meshes, int32_t precision, int32_t deflation,
                        int32_t *h_degree_out, double *h_ms_out, int32_t *h_iters_out) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(n >= 1 && h_meshes != nullptr, "bad arguments");
        CGP_REQUIRE(precision == CGP_FP64 || precision == CGP_FP32_IR, "unknown precision");
        CGP_REQUIRE(deflation == 0 || deflation == 1, "deflation must be 0 or 1");
        CGP_REQUIRE(!ctx->capturing, "cgp_autotune cannot be captured");
        std::vector<Mesh *> ms(n);
        std::ostringstream shape;   // the batch's shapes (rows, nonzeros, widest row), precision, deflation
        shape << precision << ':' << deflation << ':';
        for (int i = 0; i < n; ++i) {
            ms[i] = &get_mesh(ctx, h_meshes[i]);
            for (int j = 0; j < i; ++j) CGP_REQUIRE(h_meshes[j] != h_meshes[i], "each instance needs its own mesh");
            shape << ms[i]->lv[0].n << ',' << ms[i]->nnz << ',' << ms[i]->max_row << ';';
        }
        auto emit = [&](const TuneRec &rec) {
            for (int i = 0; i < n; ++i) {
                ms[i]->tuned_degree[precision][deflation] = rec.degree[i];
                if (h_degree_out) h_degree_out[i] = rec.degree[i];
                if (h_iters_out)
                    for (int c = 0; c < AUTOTUNE_CANDIDATES; ++c)
                        h_iters_out[i * AUTOTUNE_CANDIDATES + c] = rec.iters[static_cast<size_t>(i) * AUTOTUNE_CANDIDATES + c];
            }
            if (h_ms_out)
                for (int c = 0; c < AUTOTUNE_CANDIDATES; ++c) h_ms_out[c] = rec.ms[c];
        };
        auto hit = ctx->tuned.find(shape.str());
        if (hit != ctx->tuned.end()) {   // a batch of the same shapes was tuned: same choices
            emit(hit->second);
            return;
        }
        hipEvent_t e0, e1;
        CGP_HIP(hipEventCreate(&e0));
        CGP_HIP(hipEventCreate(&e1));
        struct EvGuard {
            hipEvent_t a, b;
            ~EvGuard() {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } guard{e0, e1};
        // per instance: the load of a unit source (b_i = 1 on free rows), a smooth field like the
        // sources of the time steps, solved from zero to 1e-8
        std::vector<DBuf<double>> bs(n), xs(n);
        std::vector<const double *> bp(n);
        std::vector<double *> xp(n);
        for (int i = 0; i < n; ++i) {
            const int64_t nn = ms[i]->lv[0].n;
            bs[i].alloc(nn);
            xs[i].alloc(nn);
            std::vector<uint8_t> dir(nn);
            CGP_HIP(hipMemcpy(dir.data(), ms[i]->lv[0].dir.p, nn, hipMemcpyDeviceToHost));
            std::vector<double> hb(nn);
            for (int64_t j = 0; j < nn; ++j) hb[j] = dir[j] ? 0.0 : 1.0;
            CGP_HIP(hipMemcpy(bs[i].p, hb.data(), nn * sizeof(double), hipMemcpyHostToDevice));
            bp[i] = bs[i].p;
            xp[i] = xs[i].p;
        }
        DBuf<cgp_solve_stats> st;
        st.alloc(n);
        std::vector<cgp_solve_stats> hs(n);
        TuneRec rec;
        rec.degree.assign(n, 0);
        rec.iters.assign(static_cast<size_t>(n) * AUTOTUNE_CANDIDATES, -1);
        // every candidate degree on the whole batch at once (the regime the solves run in)
        int best = -1;
        for (int c = 0; c < AUTOTUNE_CANDIDATES; ++c) {
            cgp_solve_opts o{};
            o.precision = precision;
            o.guess = CGP_GUESS_ZERO;
            o.tol = 1e-8;
            o.precond_degree = AUTOTUNE_DEGREES[c];
            o.deflation = deflation;
            o.engine = CGP_ENGINE_STAGED;
            float ms_best = 1e30f;
            bool ok = true;
            for (int rep = 0; rep < 3 && ok; ++rep) {   // the first solve also builds the tiled plans
                CGP_HIP(hipEventRecord(e0, ctx->stream));
                const cgp_status rc = cgp_poisson_solve(ctx, n, h_meshes, bp.data(), xp.data(), nullptr, nullptr, &o,
                                                        st.p);
                if (rc == CGP_E_UNSUPPORTED) {   // a mesh does not fit the tiled plan of this degree
                    ok = false;
                    break;
                }
                if (rc != CGP_OK) throw Error{rc, g_last_error};
                CGP_HIP(hipEventRecord(e1, ctx->stream));
                CGP_HIP(hipEventSynchronize(e1));
                CGP_HIP(hipMemcpy(hs.data(), st.p, n * sizeof(cgp_solve_stats), hipMemcpyDeviceToHost));
                for (int i = 0; i < n && ok; ++i) ok = hs[i].status == CGP_SOLVE_OK;
                float msec = 0.f;
                CGP_HIP(hipEventElapsedTime(&msec, e0, e1));
                if (rep > 0) ms_best = std::min(ms_best, msec);
            }
            rec.ms[c] = ok ? ms_best : -1.0;
            if (!ok) continue;
            for (int i = 0; i < n; ++i) rec.iters[static_cast<size_t>(i) * AUTOTUNE_CANDIDATES + c] = hs[i].iters;
            if (best < 0 || ms_best < rec.ms[best]) best = c;
        }
        CGP_REQUIRE(best >= 0, "no preconditioner degree solved the tuning problem");
        // the batch takes as many stages as its slowest instance at the fastest degree; every
        // instance then runs the lowest degree that needs no more iterations than that (a lower
        // degree has a smaller region: fewer bytes per stage, the same number of stages)
        int smax = 0;
        for (int i = 0; i < n; ++i) smax = std::max(smax, rec.iters[static_cast<size_t>(i) * AUTOTUNE_CANDIDATES + best]);
        for (int i = 0; i < n; ++i) {
            rec.degree[i] = AUTOTUNE_DEGREES[best];
            for (int c = 0; c < best; ++c) {
                const int it = rec.iters[static_cast<size_t>(i) * AUTOTUNE_CANDIDATES + c];
                if (it >= 0 && it <= smax) {
                    rec.degree[i] = AUTOTUNE_DEGREES[c];
                    break;
                }
            }
        }
        ctx->tuned[shape.str()] = rec;
        emit(rec);
        // the tuning solves' launch plans point at the buffers freed on return
        ctx->plans.clear();
    });
}

// ------------------------------------------------------------------ learned guess

int64_t cgp_model_param_count(void) { return gnn_param_count(); }

cgp_status cgp_model_create(cgp_ctx ctx, int32_t hidden, int32_t layers, uint64_t seed, cgp_model *out) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(out != nullptr, "null output pointer");
        CGP_REQUIRE(!ctx->capturing, "cgp_model_create cannot be captured");
        if (hidden != CGP_MODEL_HIDDEN || layers != CGP_MODEL_LAYERS)
            throw Error{CGP_E_UNSUPPORTED, "the network has 64 hidden features and 3 message layers"};
        std::unique_ptr<Model, cgp_ctx_s::ModelDel> md(gnn_create(ctx->stream, seed));
        const int32_t h = ctx->next_model++;
        ctx->models[h] = std::move(md);
        *out = h;
    });
}

cgp_status cgp_model_free(cgp_ctx ctx, cgp_model model) {
    return guarded([&] {
        use_device(ctx);
        (void)get_model(ctx, model);
        CGP_HIP(hipStreamSynchronize(ctx->stream));
        ctx->models.erase(model);
    });
}

cgp_status cgp_model_get_params(cgp_ctx ctx, cgp_model model, float *h_params) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(h_params != nullptr, "null output pointer");
        gnn_get_params(ctx->stream, get_model(ctx, model), h_params);
    });
}

cgp_status cgp_model_set_params(cgp_ctx ctx, cgp_model model, const float *h_params) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(h_params != nullptr, "null input pointer");
        gnn_set_params(ctx->stream, get_model(ctx, model), h_params);
    });
}

cgp_status cgp_model_predict(cgp_ctx ctx, cgp_model model, cgp_mesh mesh, const double *d_b, const double *d_prev1,
                             const double *d_prev2, double *d_guess) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(d_b && d_prev1 && d_prev2 && d_guess, "null device pointer");
        gnn_predict(ctx->stream, get_model(ctx, model), get_mesh(ctx, mesh), d_b, d_prev1, d_prev2, d_guess,
                    !ctx->capturing);
    });
}

cgp_status cgp_model_grad(cgp_ctx ctx, cgp_model model, cgp_mesh mesh, const double *d_b, const double *d_prev1,
                          const double *d_prev2, const double *d_target, double *h_loss, float *h_grad) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(d_b && d_prev1 && d_prev2 && d_target, "null device pointer");
        CGP_REQUIRE(!ctx->capturing, "cgp_model_grad cannot be captured");
        gnn_grad(ctx->stream, get_model(ctx, model), get_mesh(ctx, mesh), d_b, d_prev1, d_prev2, d_target, h_loss,
                 h_grad);
    });
}

cgp_status cgp_model_train(cgp_ctx ctx, cgp_model model, cgp_mesh mesh, int32_t n_samples,
                           const double *const *h_d_b, const double *const *h_d_prev1,
                           const double *const *h_d_prev2, const double *const *h_d_target, int32_t epochs, double lr,
                           uint64_t seed, double *h_loss_history) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(n_samples >= 1 && epochs >= 1, "need at least one sample and one epoch");
        CGP_REQUIRE(h_d_b && h_d_prev1 && h_d_prev2 && h_d_target, "null sample arrays");
        for (int i = 0; i < n_samples; ++i)
            CGP_REQUIRE(h_d_b[i] && h_d_prev1[i] && h_d_prev2[i] && h_d_target[i], "null sample pointer");
        CGP_REQUIRE(lr > 0.0 && std::isfinite(lr), "lr must be positive");
        CGP_REQUIRE(!ctx->capturing, "cgp_model_train cannot be captured");
        gnn_train(ctx->stream, get_model(ctx, model), get_mesh(ctx, mesh), n_samples, h_d_b, h_d_prev1, h_d_prev2,
                  h_d_target, epochs, lr, seed, h_loss_history);
    });
}

cgp_status cgp_model_save(cgp_ctx ctx, cgp_model model, const char *path) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(path != nullptr, "null path");
        std::vector<float> h(gnn_param_count());
        gnn_get_params(ctx->stream, get_model(ctx, model), h.data());
        FILE *f = std::fopen(path, "wb");
        if (!f) throw Error{CGP_E_INVALID, std::string("cannot open ") + path};
        const char tag[8] = {'C', 'G', 'P', 'G', 'N', 'N', '1', 0};
        const int64_t cnt = static_cast<int64_t>(h.size());
        bool ok = std::fwrite(tag, 1, 8, f) == 8 && std::fwrite(&cnt, sizeof cnt, 1, f) == 1 &&
                  std::fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
        ok = (std::fclose(f) == 0) && ok;
        if (!ok) throw Error{CGP_E_INVALID, std::string("cannot write ") + path};
    });
}

cgp_status cgp_model_load(cgp_ctx ctx, const char *path, cgp_model *out) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(path != nullptr && out != nullptr, "null argument");
        FILE *f = std::fopen(path, "rb");
        if (!f) throw Error{CGP_E_INVALID, std::string("cannot open ") + path};
        char tag[8] = {0};
        int64_t cnt = 0;
        std::vector<float> h(gnn_param_count());
        bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, "CGPGNN1", 8) == 0 &&
                  std::fread(&cnt, sizeof cnt, 1, f) == 1 && cnt == gnn_param_count() &&
                  std::fread(h.data(), sizeof(float), h.size(), f) == h.size();
        std::fclose(f);
        if (!ok) throw Error{CGP_E_INVALID, std::string("not a model file: ") + path};
        std::unique_ptr<Model, cgp_ctx_s::ModelDel> md(gnn_create(ctx->stream, 0));
        gnn_set_params(ctx->stream, *md, h.data());
        const int32_t hd = ctx->next_model++;
        ctx->models[hd] = std::move(md);
        *out = hd;
    });
}

// ------------------------------------------------------------------ graphs

cgp_status cgp_graph_begin(cgp_ctx ctx) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(ctx->stream != nullptr, "graph capture needs a non-null stream");
        CGP_REQUIRE(!ctx->capturing, "capture already in progress");
        CGP_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
        ctx->capturing = true;
        ctx->capture_plans.clear();
    });
}

cgp_status cgp_graph_end(cgp_ctx ctx, cgp_graph *out) {
    return guarded([&] {
        use_device(ctx);
        CGP_REQUIRE(out != nullptr, "null output pointer");
        CGP_REQUIRE(ctx->capturing, "no capture in progress");
        ctx->capturing = false;
        GraphRec g;
        g.plans = std::move(ctx->capture_plans);
        ctx->capture_plans.clear();
        CGP_HIP(hipStreamEndCapture(ctx->stream, &g.graph));
        CGP_HIP(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
        const int32_t h = ctx->next_graph++;
        ctx->graphs[h] = g;
        *out = h;
    });
}

cgp_status cgp_graph_launch(cgp_ctx ctx, cgp_graph graph) {
    return guarded([&] {
        use_device(ctx);
        auto it = ctx->graphs.find(graph);
        CGP_REQUIRE(it != ctx->graphs.end(), "unknown graph handle");
        CGP_HIP(hipGraphLaunch(it->second.exec, ctx->stream));
    });
}

cgp_status cgp_graph_free(cgp_ctx ctx, cgp_graph graph) {
    return guarded([&] {
        use_device(ctx);
        auto it = ctx->graphs.find(graph);
        CGP_REQUIRE(it != ctx->graphs.end(), "unknown graph handle");
        CGP_HIP(hipStreamSynchronize(ctx->stream));
        (void)hipGraphExecDestroy(it->second.exec);
        (void)hipGraphDestroy(it->second.graph);
        ctx->graphs.erase(it);
    });
}

}  // extern "C"
