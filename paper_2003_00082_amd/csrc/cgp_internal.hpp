// Internal declarations shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "../../include/cgp.h"

namespace cgp {

// ------------------------------------------------------------------ error handling

void set_error(const std::string &msg);

struct Error {
    cgp_status code;
    std::string msg;
};

#define CGP_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::cgp::Error{CGP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define CGP_REQUIRE(cond, msg)                                        \
    do {                                                              \
        if (!(cond)) throw ::cgp::Error{CGP_E_INVALID, (msg)};        \
    } while (0)

// ------------------------------------------------------------------ device buffers

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            throw Error{CGP_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
        }
        n = count;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// ------------------------------------------------------------------ mesh hierarchy

struct Level {
    int64_t n = 0, T = 0, E = 0;
    DBuf<double> xy;        // [2n]
    DBuf<int32_t> tri;      // [3T]
    DBuf<uint8_t> dir;      // [n]
    DBuf<int32_t> ne_ptr;   // [n+1] node -> incident triangles (ascending triangle id)
    DBuf<int32_t> ne_idx;   // [3T]
    DBuf<int32_t> ends;     // [2E] edge end points (levels < k)
    DBuf<double> tmp;       // [n] prolongation staging (levels 1..k-1)
};

// per-instance solver workspace, owned by the mesh (r, w, s double-buffered;
// u = M^-1 r of the tiled iteration single-buffered: only its own row reads it).  The
// tiled iteration keeps its vectors row-interleaved instead: rwsd [2][n][4] = (r, w, s,
// D^-1) of a row by stage parity (one 16-byte gather per region row in fp32; D^-1 written
// once, when the buffers are made), and up [n][2] = (u, p) by own slot (a tile's own rows
// are consecutive slots, TileBlk::own_off on), which only the owning tile reads.
struct SolveWork {
    int64_t n = 0;
    DBuf<double> r, w, s, p, u;
    DBuf<float> r32, w32, s32, p32, c32, u32;
    DBuf<float> rwsd32, up32;
    DBuf<double> rwsd64, up64;
};

// ------------------------------------------------------------------ tiled iteration

constexpr int TILE_ROWS = 512;        // own rows per workgroup at one per thread (the preferred tile)
constexpr int TILE_OWN = 2;           // own rows a thread can hold
constexpr int TILE_ROWS_MAX = TILE_OWN * TILE_ROWS;   // own rows per workgroup
constexpr int TILE_GRID = 256;        // tiles aimed for when the rows need more than this many
                                      // preferred tiles: one per compute unit of the chip
constexpr int TILE_REGION = 2048;     // region rows per workgroup (own rows + halo to distance d)
constexpr int TILE_SPMV = 1536;       // region rows that carry a local matrix row
constexpr int TILE_MAX_DEGREE = 8;

// One workgroup of the tiled iteration: a compact tile of own rows (recursive
// coordinate bisection of the node coordinates) and its region, the rows within
// graph distance d of the tile, listed own rows first and then by distance.
struct TileBlk {
    int32_t reg_off;                  // first entry of the region in TilePlan::reg
    int32_t ell_off;                  // first local matrix row record of the tile
    int32_t nreg;                     // region rows (= nt[degree])
    int32_t nspmv;                    // rows with a local matrix row (= nt[max(degree - 1, 0)])
    int32_t nt[TILE_MAX_DEGREE + 2];  // nt[t]: region rows at distance <= t
    int32_t kz_off;                   // deflation: first coupling record of the tile
    int32_t nkz;                      // deflation: coupling records (<= TILE_ROWS)
    int32_t own_off;                  // first own slot of the tile (own rows of tiles 0..t-1)
};

// 16-bit column entries per local matrix row record (a multiple of 8: 16-byte loads)
constexpr int tile_col_stride(int width) { return width <= 8 ? 8 : 16; }

// Partition and local matrices of one mesh for one preconditioner degree.  Local
// matrix row t of a tile: columns (region indices) at (ell_off + t) * tile_col_stride,
// values at (ell_off + t) * width.
struct TilePlan {
    int32_t degree = 0, width = 0, nparts = 0;
    // records the CG stage kernel reads: SPLIT_WIDTH (rows of at most SPLIT_WIDTH off-diagonal
    // entries: the split records below) or width (the records above)
    int32_t kwidth = 0;
    int32_t agg = 0;          // deflation aggregates per tile (each tile's own rows bisected into agg parts)
    std::vector<TileBlk> hblk;
    std::vector<int32_t> hreg;
    DBuf<TileBlk> blk;
    DBuf<int32_t> reg;
    DBuf<uint16_t> ecol;
    DBuf<float> eval32;
    DBuf<double> eval64;
    // split records: the off-diagonal entries only (the kernel forms the diagonal as 1 / D^-1
    // from the row's vector record), padded with the row's own region index and value 0; per
    // tile column-major, so that one load instruction of a wavefront reads consecutive rows:
    // value pair q (entries 2q, 2q + 1) of local row t at SPLIT_WIDTH ell_off + 2 (q nspmv + t),
    // column pair q (two 16-bit region indices) at (SPLIT_WIDTH / 2) ell_off + q nspmv + t
    DBuf<uint32_t> scol;
    DBuf<float> sval32;
    DBuf<double> sval64;
    // subdomain deflation, each tile's own rows cut into agg aggregates (agg t .. agg t +
    // agg - 1) by bisection (built on first use; defl_state 0 = not built, 1 = built, -1 = not
    // supported for this mesh)
    int32_t defl_state = 0;
    DBuf<int8_t> oagg;        // per region entry, own rows only: 0 Dirichlet, 1 + aggregate within the tile
    DBuf<uint64_t> kzk;       // coupling record: the region index of the row (bits 0..11) and the
                              // KZ_PER_ROW aggregates it couples to (12 bits each from bit 12 on)
    DBuf<float> kzv32;        // [4] per record: (K Z)_{row, aggregate}
    DBuf<double> kzv64;
    DBuf<double> einv;        // [m x einv_stride(m)] (Z^T K Z)^-1, row-major, m = agg * nparts
    DBuf<float> einv32;       // the same rounded to fp32 (the coarse step of fp32 iterations)
};

constexpr int SPLIT_WIDTH = 6;             // off-diagonal entries of a split record
constexpr int MAX_STAGE_BUDGET = 65536;    // stage launches a solve recorded in a graph may take
constexpr int AGG_TILE = 2;              // deflation aggregates per tile of TILE_ROWS-row tiles
constexpr int AGG_MAX = 8;               // aggregates a tile may carry
constexpr int NRED = 4;                  // reduced sums of a stage: gamma, delta, sigma, r.r
constexpr int NPART = NRED + AGG_MAX;    // partial-sum slots per workgroup (NRED + aggregate sums)
constexpr int KZ_PER_ROW = 4;            // aggregates one row may couple to
constexpr int KZ_BITS = 12;              // bits of a region index or aggregate in a coupling record
constexpr int MAX_DEFL_AGGREGATES = 2048;   // the coarse step holds a row of E^-1 in 32 registers per lane
static_assert(TILE_REGION <= (1 << KZ_BITS) && MAX_DEFL_AGGREGATES <= (1 << KZ_BITS) &&
                  KZ_BITS * (1 + KZ_PER_ROW) <= 64, "a coupling record packs into 64 bits");

// The nodal gradient of the finest level as a sparse operator: G_i = sum_j (cx_ij, cy_ij) q_j
// (the area-weighted mean of the element gradients around node i), column-major ELL of
// width W (entry k of node i at k * n + i; padding: the node itself with zero weights).
constexpr int GRAD_MAX_W = 32;
struct NodalGrad {
    int32_t W = 0;        // entries per node (its other vertices, padded to 6 or 8); 0: not built; -1: a
                          // node has more than GRAD_MAX_W - 1 neighbours
    DBuf<int32_t> col;
    DBuf<double> cx, cy;
};

// Workgroups are dispatched to the 8 XCDs round robin (workgroup v to XCD v % 8).  This
// maps dispatch index v to a logical block so that every XCD takes a contiguous range of
// row blocks or tiles: neighbouring blocks share halo rows, which are then read through
// one L2 rather than fetched by several.  A bijection of [0, G), so every block and
// partial-sum slot is still covered once.
__device__ inline int xcd_block(int v, int G) {
    const int x = v % 8, k = v / 8, q = G / 8, rm = G % 8;
    return x * q + (x < rm ? x : rm) + k;
}

// Workspace of the momentum step on the finest level, in its own numbering of the nodes
// (along a Z curve of their coordinates, so that a row's neighbours lie close in memory;
// perm: own -> mesh, inv: mesh -> own): the adjacency pattern (self included, sorted; CSR
// and a column-major ELL copy) with the operator's values (ELL), its Jacobi inverse, the
// rows' Dirichlet bits, the two right-hand sides, the iterate of both components and the
// BiCGStab vectors ([n][2] each, interleaved; p and v by parity).
struct MomentumWork {
    int64_t n = 0, nnz = 0;
    int32_t width = 0;       // the ELL width: the longest row rounded up to a bin
    int32_t last_iters = 0;  // BiCGStab iterations of the previous call (0: none yet)
    DBuf<int32_t> perm, inv;
    DBuf<uint8_t> rowmask;
    DBuf<double> x;          // [2][n]: u, then v
    DBuf<int32_t> ptr, col;  // CSR pattern (built once)
    DBuf<int32_t> ecol;      // ELL columns: entry k of row i at k * n + i (padding: i)
    DBuf<double> val, dinv, b, r, rh, p, v, s, t;
    DBuf<double> part;       // per-workgroup partial sums of the start and of the two launches
    DBuf<double> scal;       // recurrence scalars and norms
    DBuf<int32_t> state;     // two copies (by launch parity) of each component's status and iterations
};

// Point location on one level: a uniform grid of square cells of side h from (x0, y0),
// gx x gy cells, each listing (CSR) the triangles whose bounding box overlaps it.
struct Locator {
    double x0 = 0.0, y0 = 0.0, h = 1.0;
    int32_t gx = 1, gy = 1;
    const int32_t *cell_ptr = nullptr, *cell_tri = nullptr;
};
struct LocatorData {
    Locator loc;
    DBuf<int32_t> cell_ptr, cell_tri;
};

constexpr int NBR_NARROW = 6;   // neighbour-table width of a regular triangulation
constexpr int NBR_WIDE = 8;

struct Mesh {
    int32_t k = 0;
    std::vector<Level> lv;
    // level-0 full adjacency (sorted, self included) kept for the learned guess
    DBuf<int32_t> adj_ptr, adj_col;
    int64_t adj_nnz = 0;
    // the same neighbours (self excluded) as a column-major table: neighbour k of node i at
    // k * n + i, padded with n; width nbr_w = NBR_NARROW, or a multiple of NBR_WIDE
    DBuf<int32_t> nbr;
    int32_t nbr_w = 0;
    // level-0 system matrix
    int64_t nnz = 0;
    int32_t max_row = 0;
    DBuf<int32_t> rowptr, col;
    DBuf<double> val, dinv;
    DBuf<float> val32, dinv32;
    // column-major ELL copy, width max_row: entry k of row i at k * n + i
    DBuf<int32_t> ell_col;
    DBuf<double> ell_val;
    DBuf<float> ell_val32;
    SolveWork work;
    int32_t tuned_degree[2][2] = {{0, 0}, {0, 0}};   // cgp_autotune's degree per precision and deflation (0: none)
    double gershgorin = 0.0;           // max_i sum_j |K_ij| / K_ii (0 = not computed)
    std::unique_ptr<TilePlan> tiles[TILE_MAX_DEGREE + 1];   // per preconditioner degree
    NodalGrad grad;                     // finest level, built on the first force or correction
    std::unique_ptr<MomentumWork> mom;  // finest level, built on the first momentum step
    std::vector<std::unique_ptr<LocatorData>> loc;   // per level, built on the first interpolation
};

// builds (or returns) the tiled plan of a mesh for degree d; nullptr when the
// mesh does not fit the tiled iteration (rows wider than 12, regions too large)
TilePlan *tile_plan(hipStream_t s, Mesh &m, int degree);
double mesh_gershgorin(hipStream_t s, Mesh &m);
// builds (or reports) the deflation data of a tile plan; false when the mesh does not fit
// it (too many aggregates, a row coupled to more than KZ_PER_ROW aggregates, more
// coupled rows in a region than a workgroup has threads)
bool tile_deflation(hipStream_t s, Mesh &m, TilePlan &P);

// ------------------------------------------------------------------ solver launch records

// per-instance control state of the CG stage machine
struct Ctl {
    int32_t state, it, refinements, status, guess_used, stages, restart, first;   // stages: launches decoded
    double gamma, alpha, beta, pap, bnorm, rmax, rel_res, rel_res_guess;
};

// rows [r0, r1) of one workgroup and the column range [c0, c1] they touch
struct RowRange {
    int32_t r0, r1, c0, c1;
};

// per-workgroup partial sums of a stage (NPART slots, defined with the tile constants):
// gamma, delta, sigma, r.r (NRED, reduced over the instance by the next stage, which puts
// the coarse term c in S[NRED]) and (deflation) the sums of w or r over the free rows of
// each of the tile's aggregates (slots NRED + a)

// device-side description of one instance of a (batched) solve
struct InstDesc {
    int32_t n;            // rows
    int32_t blk0;         // first workgroup of this instance
    int32_t nblk;         // workgroups of this instance
    int32_t lanes;        // SpMV lanes per row (1, 2, 4, 8)
    int32_t guess;        // CGP_GUESS_*
    int32_t stats_index;  // record of this instance in SolveParams::stats
    int32_t chunk;        // rows per workgroup
    int32_t fast;         // every row fits the one-row-per-thread iteration (ELL width <= its limit)
    int32_t ell_w;        // ELL width
    int32_t pad2_;
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
    const float *val32;
    const double *dinv;
    const float *dinv32;
    const double *b;
    double *x;
    const double *prev1;
    const double *prev2;
    double *r, *w, *s, *p;               // fp64 recurrences (r, w, s: 2n each)
    float *r32, *w32, *s32, *p32, *c32;  // fp32 recurrences and correction
    double *partials;                    // [2][NPART][nblk]
    Ctl *ctl;                            // [2]
    const int32_t *ell_col;              // column-major ELL copy of the matrix
    const double *ell_val;
    const float *ell_val32;
    // tiled iteration (degree >= 1; 0 = not tiled)
    int32_t degree;
    int32_t pad3_;
    const TileBlk *tblk;                 // [nblk]
    const int32_t *treg;
    const uint16_t *tcol;
    const float *tval32;
    const double *tval;
    double *u;                           // M^-1 r (own rows)
    float *u32;
    float *rwsd32;                       // tiled iteration: (r, w, s, D^-1) [2][n][4] and (u, p) [n][2]
    float *up32;
    double *rwsd64;
    double *up64;
    double cheb[2 * TILE_MAX_DEGREE];    // [0]: scale of the first step; [2k-1], [2k]: step k coefficients
    // subdomain deflation (tiled iteration only; agg aggregates in each of the instance's tiles)
    int32_t defl;                        // 0 off, 1 on
    int32_t ncb;                         // workgroups of the coarse kernel for this instance
    int32_t cblk0;                       // first of them
    int32_t agg;                         // deflation aggregates per tile
    const uint64_t *kzk;
    const float *kzv32;
    const double *kzv;
    const double *einv;                  // [m x einv_stride(m)], m = agg * nblk
    const float *einv32;                 // the same in fp32
    double *mu;                          // [m] E^-1 Z^T v of the last stage
    double *cpart;                       // [ncb][NRED + 1] coarse step records: a slice of the tiles' NRED
                                         // sums and a partial of mu . Z^T v
    const int8_t *oagg;                  // own rows (by region entry): 0 Dirichlet, 1 + aggregate within the tile
};

struct SolveParams {
    double tol;
    double delta;
    int32_t max_iter;
    int32_t precision;
    int32_t n_inst;
    int32_t pad_;
    cgp_solve_stats *stats;   // caller's stats array (per call, not part of the cached plan)
};

// grid-wide barrier state of the persistent driver (one per context, zeroed at creation)
struct GridSync {
    uint32_t arrive;
    uint32_t gen;
    int32_t abort;
    int32_t pad_;
};

// solver launches (pcg.hip)
int pcg_block_size();
int pcg_max_blocks_per_cu();
void launch_ranges(hipStream_t s, const InstDesc *d_insts, const int32_t *d_block_inst, int grid,
                   RowRange *d_ranges);
void launch_cg_boot(hipStream_t s, InstDesc *d_insts, int n_inst, const SolveParams &prm, SolveParams *d_prm,
                    int32_t *d_done);
// after the recorded launches of a captured staged solve (par: parity of the last launch)
void launch_cg_close(hipStream_t s, const InstDesc *d_insts, int n_inst, const SolveParams *d_prm, int par);
// D^-1 into the fourth component of both parities of the row-interleaved vectors (either may be null)
void launch_fill_rwsd(hipStream_t s, int64_t n, const float *dinv32, const double *dinv, float *rwsd32,
                      double *rwsd64);
// start and stop events of one kernel dispatch (stage timing): recorded by the dispatch itself
// (hipExtLaunchKernelGGL), so their interval is the kernel's own execution; null: plain launch
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
// h_one: the record of a single-instance solve (passed by value to the kernel), else null
void launch_cg_step(hipStream_t s, bool mixed, int halo, int n_inst, const InstDesc *d_insts, const InstDesc *h_one,
                    const int32_t *d_block_inst, const RowRange *d_ranges, int grid, const SolveParams *d_prm,
                    int par, int32_t *d_done, int32_t *d_host_flag, KernelEvents ev = {});
// unb: the workgroups of each instance when all instances have that many (the stage kernel then
// finds its instance without reading d_block_inst), else 0
void launch_cg_tile(hipStream_t s, bool mixed, int width, bool defl, int unb, const InstDesc *d_insts,
                    const InstDesc *h_one, const int32_t *d_block_inst, const RowRange *d_ranges, int grid,
                    const SolveParams *d_prm, int par, int32_t *d_done, int32_t *d_host_flag, KernelEvents ev = {});
// the coarse step of deflation after a tiled stage launch: mu = E^-1 (aggregate sums), c partials
constexpr int COARSE_WAVES = 8;                  // wavefronts per coarse workgroup
constexpr int COARSE_ROWS = 2 * COARSE_WAVES;    // aggregates (rows of E^-1) per coarse workgroup
// row stride of both copies of E^-1: m rounded up to a multiple of 4 entries (zero padded), so
// that every row starts 16-byte aligned
constexpr int einv_stride(int m) { return (m + 3) & ~3; }
struct CoarseRec {               // what the coarse step of one instance touches
    const double *einv;          // [m x einv_stride(m)]
    const float *einv32;         // the same in fp32 (read by the coarse step of fp32 iterations)
    const double *partials;      // the instance's [2][NPART][tiles] stage partials
    double *mu;                  // [m]
    double *cpart;               // [ncb][NRED + 1]
    int32_t m;                   // aggregates (agg per tile)
    int32_t tiles;               // workgroups of the tiled stage
    int32_t cblk0;               // first coarse workgroup of the instance
    int32_t agg;                 // aggregates per tile: aggregate a is part a % agg of tile a / agg
    const Ctl *ctl;              // the instance's control state, by stage parity
    int32_t ncb;                 // coarse workgroups of the instance (ceil(m / COARSE_ROWS))
    int32_t pad_;
};
// h_single: the record of a single-instance solve (passed by value), else the device records
// e32: read the fp32 copy of E^-1 (fp32 iterations)
void launch_cg_coarse(hipStream_t s, bool e32, const CoarseRec *h_single, const CoarseRec *d_recs,
                      const int32_t *d_cblk_inst, int grid, int par, KernelEvents ev = {});
int pcg_ell_max_width();
void launch_cg_persistent(hipStream_t s, const InstDesc *d_insts, int n_inst, const int32_t *d_block_inst,
                          const RowRange *d_ranges, int grid, const SolveParams &prm, GridSync *d_sync,
                          int32_t *d_done_at, uint64_t timeout_ticks);

// the no-allocation solve's device array (noalloc.hip): noalloc_init looks its address up on
// `device` (which must be current), noalloc_scratch returns it (null before noalloc_init)
void noalloc_init(int device);
uint8_t *noalloc_scratch(int device);
void launch_noalloc_setup(hipStream_t s, InstDesc *insts, const InstDesc &d, int32_t *block_inst, int nblk,
                          int32_t *cblk_inst, int ncb, double *zero, int nzero, CoarseRec *crec,
                          const CoarseRec &c);

// mesh build (mesh_build.hip)
void build_hierarchy(hipStream_t s, Mesh &m, const double *h_xy, int64_t n, const int32_t *h_tri,
                     int64_t T, const uint8_t *h_dir, int32_t k);

// transfer kernels (transfer.hip)
void launch_restrict(hipStream_t s, const Mesh &m, const double *uf, const double *vf, int kind,
                     double scale, double *b, double *uc, double *vc);
void launch_prolong(hipStream_t s, Mesh &m, const double *qc, double *qf);
// build: may build the nodal-gradient operator now (not while the stream is captured)
void launch_lorentz(hipStream_t s, Mesh &m, const double *phif, const double *uf,
                    const double *vf, double sigma, double b0, double *fx, double *fy,
                    double *grad_elem, bool build);
void launch_velocity(hipStream_t s, Mesh &m, const double *pf, const double *ut, const double *vt,
                     const uint8_t *mask, double scale, double *u, double *v, bool build);
// the force of the fluid on a body over its boundary edges (a, b, t) of a level: out[5]
void launch_surface_force(hipStream_t s, Mesh &m, int level, int64_t n_edges, const int32_t *edges,
                          const double *p, const double *u, const double *v, double mu, double *out);

// learned initial guess (gnn.hip)
struct Model;
int64_t gnn_param_count();
Model *gnn_create(hipStream_t s, uint64_t seed);   // owned by the caller, freed by gnn_destroy
void gnn_set_params(hipStream_t s, Model &md, const float *h);
void gnn_get_params(hipStream_t s, Model &md, float *h);
// the finest level's adjacency (self included, sorted rows)
void level_adjacency(hipStream_t s, const Level &L, DBuf<int32_t> &adj_ptr, DBuf<int32_t> &adj_col,
                     int64_t &adj_nnz);
// a level's P1 field at np points (x, y interleaved): out (NaN outside the mesh) and, when
// tri_out is not null, the containing triangle (-1 outside); build: the level's locator
// may be built here (a host synchronisation), else it must exist
void interpolate_points(hipStream_t s, Mesh &m, int level, int64_t np, const double *pts, const double *field,
                        double *out, int32_t *tri_out, bool build);
// the momentum step of Eqs. 13-14 on the finest level (synchronises the stream)
void momentum_step(hipStream_t s, Mesh &m, const double *un, const double *vn, const double *fx,
                   const double *fy, const uint8_t *mask, double rho, double mu, double dt, double tol, int max_iter, double *ut,
                   double *vt, cgp_momentum_stats *stats);

// guess from the network, then smoothed; build: the smoothing's tiled plan may be built here
// (a host synchronisation: not under graph capture), else it is used when already built
void gnn_predict(hipStream_t s, Model &md, Mesh &m, const double *b, const double *p1, const double *p2,
                 double *guess, bool build);
void gnn_grad(hipStream_t s, Model &md, const Mesh &m, const double *b, const double *p1, const double *p2,
              const double *target, double *h_loss, float *h_grad);
void gnn_train(hipStream_t s, Model &md, const Mesh &m, int n_samples, const double *const *b,
               const double *const *p1, const double *const *p2, const double *const *target, int epochs,
               double lr, uint64_t seed, double *h_loss);
void gnn_release_mesh(Model &md, const Mesh *m);
void gnn_destroy(Model *md);

// scan (mesh_build.hip): out[0..n] exclusive prefix sums of in[0..n-1]; returns total
int64_t exclusive_scan(hipStream_t s, const int32_t *in, int32_t *out, int64_t n);

inline unsigned blocks_for(int64_t n, int threads) {
    return static_cast<unsigned>((n + threads - 1) / threads);
}

}  // namespace cgp
