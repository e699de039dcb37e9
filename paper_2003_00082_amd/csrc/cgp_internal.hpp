// Internal declarations shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
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

// per-instance solver workspace, owned by the mesh
struct SolveWork {
    int64_t n = 0;
    DBuf<double> r, z, p0, p1, q;                   // fp64 recurrences
    DBuf<float> c32, r32, z32, p32a, p32b, q32;     // fp32 inner recurrences
};

struct Mesh {
    int32_t k = 0;
    std::vector<Level> lv;
    // level-0 full adjacency (sorted, self included) kept for the learned guess
    DBuf<int32_t> adj_ptr, adj_col;
    int64_t adj_nnz = 0;
    // level-0 system matrix
    int64_t nnz = 0;
    int32_t max_row = 0;
    DBuf<int32_t> rowptr, col;
    DBuf<double> val, dinv;
    DBuf<float> val32, dinv32;
    SolveWork work;
    int32_t tuned_lanes[2] = {0, 0};   // autotuned SpMV lanes per precision (0 = not tuned)
};

// ------------------------------------------------------------------ solver launch records

// device-side description of one instance of a (batched) persistent solve
struct InstDesc {
    int32_t n;          // rows
    int32_t blk0;       // first persistent workgroup of this instance
    int32_t nblk;       // workgroups of this instance
    int32_t lanes;      // SpMV lanes per row (1, 2, 4, 8)
    int32_t guess;      // CGP_GUESS_*
    int32_t pad_;
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
    double *r, *z, *p0, *p1, *q;
    float *c32, *r32, *z32, *p32a, *p32b, *q32;
    double *partials;   // [2][NPART][nblk]
    cgp_solve_stats *stats;
};

constexpr int NPART = 4;

struct SolveParams {
    double tol;
    double delta;
    int32_t max_iter;
    int32_t precision;
    int32_t n_inst;
    int32_t pad_;
};

// grid-wide barrier state (one per context, zeroed at creation)
struct GridSync {
    uint32_t arrive;
    uint32_t gen;
    int32_t abort;
    int32_t pad_;
};

// launch the persistent solver (pcg.hip)
void launch_pcg(hipStream_t s, const InstDesc *d_insts, int n_inst, const int32_t *d_block_inst,
                int grid, int block, const SolveParams &prm, GridSync *d_sync, int32_t *d_done_at,
                size_t lds_bytes);
int pcg_block_size();
size_t pcg_lds_bytes();

// mesh build (mesh_build.hip)
void build_hierarchy(hipStream_t s, Mesh &m, const double *h_xy, int64_t n, const int32_t *h_tri,
                     int64_t T, const uint8_t *h_dir, int32_t k);

// transfer kernels (transfer.hip)
void launch_restrict(hipStream_t s, const Mesh &m, const double *uf, const double *vf, int kind,
                     double scale, double *b, double *uc, double *vc);
void launch_prolong(hipStream_t s, Mesh &m, const double *qc, double *qf);
void launch_lorentz(hipStream_t s, const Mesh &m, const double *phif, const double *uf,
                    const double *vf, double sigma, double b0, double *fx, double *fy,
                    double *grad_elem);
void launch_guess_prep(hipStream_t s, int guess, int64_t n, double *x, const double *prev1,
                       const double *prev2);

// scan (mesh_build.hip): out[0..n] exclusive prefix sums of in[0..n-1]; returns total
int64_t exclusive_scan(hipStream_t s, const int32_t *in, int32_t *out, int64_t n);

inline unsigned blocks_for(int64_t n, int threads) {
    return static_cast<unsigned>((n + threads - 1) / threads);
}

}  // namespace cgp
