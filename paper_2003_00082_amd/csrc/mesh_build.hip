// Mesh hierarchy on the device: validation, node->triangle incidence, node
// adjacency, edge numbering, uniform 4-way refinement (Section 2.3, Eq. 18) and
// the Galerkin P1 stiffness matrix of the coarse Poisson problems (Eqs. 12, 15).
//
// Everything here is gather-based and free of floating-point atomics: integer
// atomics only count or claim slots, and every list they fill is sorted
// afterwards, so the result is independent of scheduling.
#include "cgp_internal.hpp"

namespace cgp {
namespace {

constexpr int TPB = 256;

// ------------------------------------------------------------------ exclusive scan

constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t *wave_tot, int32_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const int nw = blockDim.x >> 6;
        int32_t w = lane < nw ? wave_tot[lane] : 0;
        int32_t wi = w;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            int32_t t = __shfl_up(wi, d, 64);
            if (lane >= d) wi += t;
        }
        if (lane < nw) wave_tot[lane] = wi - w;   // exclusive wave offsets
        if (lane == nw - 1) *total = wi;
    }
    __syncthreads();
    return incl - v + wave_tot[wave];
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(const int32_t *in, int32_t *out,
                                                             int64_t n, int32_t *tile_sums) {
    __shared__ int32_t wave_tot[SCAN_THREADS / 64];
    __shared__ int32_t total;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    int32_t off = block_exclusive_scan(s, wave_tot, &total);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = off;
        off += v[i];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_add(int32_t *out, int64_t n, const int32_t *tile_off) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_off[i / SCAN_TILE];
}

__global__ void k_store_total(int32_t *out, int64_t n, const int32_t *tile_off, const int32_t *tile_sums,
                              int64_t ntiles) {
    out[n] = tile_off[ntiles - 1] + tile_sums[ntiles - 1];
}

void scan_rec(hipStream_t s, const int32_t *in, int32_t *out, int64_t n) {
    // out[0..n] exclusive sums of in[0..n-1], out[n] = total
    const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    DBuf<int32_t> sums, offs;
    sums.alloc(ntiles);
    offs.alloc(ntiles + 1);
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(SCAN_THREADS), 0, s, in, out, n, sums.p);
    CGP_HIP(hipGetLastError());
    if (ntiles > 1) {
        scan_rec(s, sums.p, offs.p, ntiles);
        hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(n, TPB)), dim3(TPB), 0, s, out, n, offs.p);
        CGP_HIP(hipGetLastError());
    } else {
        CGP_HIP(hipMemsetAsync(offs.p, 0, sizeof(int32_t), s));
    }
    hipLaunchKernelGGL(k_store_total, dim3(1), dim3(1), 0, s, out, n, offs.p, sums.p, ntiles);
    CGP_HIP(hipGetLastError());
    CGP_HIP(hipStreamSynchronize(s));   // scratch buffers are freed on return
}

// ------------------------------------------------------------------ validation

__global__ void k_validate(int64_t n, int64_t T, const double *xy, const int32_t *tri, int32_t *flag) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n) {
        atomicOr(flag, 1);
        return;
    }
    if (a == b || b == c || c == a) {
        atomicOr(flag, 2);
        return;
    }
    const double xa = xy[2 * a], ya = xy[2 * a + 1];
    const double xb = xy[2 * b], yb = xy[2 * b + 1];
    const double xc = xy[2 * c], yc = xy[2 * c + 1];
    const double twice_area = (xb - xa) * (yc - ya) - (xc - xa) * (yb - ya);
    if (!(twice_area > 0.0)) atomicOr(flag, 4);
}

__global__ void k_isolated(int64_t n, const int32_t *cnt, int32_t *flag) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && cnt[i] == 0) atomicOr(flag, 8);
}

// ------------------------------------------------------------------ incidence and adjacency

__global__ void k_count_incident(int64_t T, const int32_t *tri, int32_t *cnt) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= T) return;
    for (int c = 0; c < 3; ++c) atomicAdd(&cnt[tri[3 * t + c]], 1);
}

__global__ void k_fill_incident(int64_t T, const int32_t *tri, const int32_t *ptr, int32_t *cursor,
                                int32_t *idx) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= T) return;
    for (int c = 0; c < 3; ++c) {
        const int32_t v = tri[3 * t + c];
        const int32_t slot = atomicAdd(&cursor[v], 1);
        idx[ptr[v] + slot] = static_cast<int32_t>(t);
    }
}

__device__ inline void insertion_sort(int32_t *a, int m) {
    for (int i = 1; i < m; ++i) {
        const int32_t key = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > key) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = key;
    }
}

__global__ void k_sort_segments(int64_t n, const int32_t *ptr, int32_t *idx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    insertion_sort(idx + ptr[i], ptr[i + 1] - ptr[i]);
}

// candidate neighbours of node i (all vertices of its triangles), sorted and de-duplicated
// in place in cand[3*ne_ptr[i] ...]; the unique count goes to cnt[i]
__global__ void k_adj_candidates(int64_t n, const int32_t *ne_ptr, const int32_t *ne_idx,
                                 const int32_t *tri, int32_t *cand, int32_t *cnt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t *c = cand + 3 * static_cast<int64_t>(ne_ptr[i]);
    int m = 0;
    for (int32_t k = ne_ptr[i]; k < ne_ptr[i + 1]; ++k) {
        const int64_t t = ne_idx[k];
        c[m++] = tri[3 * t];
        c[m++] = tri[3 * t + 1];
        c[m++] = tri[3 * t + 2];
    }
    insertion_sort(c, m);
    int u = 0;
    for (int k = 0; k < m; ++k)
        if (u == 0 || c[k] != c[u - 1]) c[u++] = c[k];
    cnt[i] = u;
}

__global__ void k_adj_compact(int64_t n, const int32_t *ne_ptr, const int32_t *cand,
                              const int32_t *adj_ptr, int32_t *adj_col) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t *c = cand + 3 * static_cast<int64_t>(ne_ptr[i]);
    const int32_t m = adj_ptr[i + 1] - adj_ptr[i];
    for (int k = 0; k < m; ++k) adj_col[adj_ptr[i] + k] = c[k];
}

// ------------------------------------------------------------------ edges

__global__ void k_edge_count(int64_t n, const int32_t *adj_ptr, const int32_t *adj_col, int32_t *cnt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t u = 0;
    for (int32_t k = adj_ptr[i]; k < adj_ptr[i + 1]; ++k) u += adj_col[k] > i;
    cnt[i] = u;
}

// number of triangles shared by nodes a and b (merge of two sorted incidence lists)
__device__ inline int shared_triangles(const int32_t *ne_ptr, const int32_t *ne_idx, int32_t a, int32_t b) {
    int32_t i = ne_ptr[a], ie = ne_ptr[a + 1], j = ne_ptr[b], je = ne_ptr[b + 1];
    int s = 0;
    while (i < ie && j < je) {
        const int32_t x = ne_idx[i], y = ne_idx[j];
        if (x == y) { ++s; ++i; ++j; }
        else if (x < y) ++i;
        else ++j;
    }
    return s;
}

__global__ void k_edge_fill(int64_t n, const int32_t *adj_ptr, const int32_t *adj_col,
                            const int32_t *edge_ptr, const int32_t *ne_ptr, const int32_t *ne_idx,
                            int32_t *ends, uint8_t *boundary) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t e = edge_ptr[i];
    for (int32_t k = adj_ptr[i]; k < adj_ptr[i + 1]; ++k) {
        const int32_t j = adj_col[k];
        if (j <= i) continue;
        ends[2 * e] = static_cast<int32_t>(i);
        ends[2 * e + 1] = j;
        boundary[e] = shared_triangles(ne_ptr, ne_idx, static_cast<int32_t>(i), j) == 1;
        ++e;
    }
}

// ------------------------------------------------------------------ refinement

__global__ void k_refine_nodes(int64_t n, int64_t E, const double *xy, const uint8_t *dir,
                               const int32_t *ends, const uint8_t *boundary, double *xy_f, uint8_t *dir_f) {
    const int64_t id = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= n + E) return;
    if (id < n) {
        xy_f[2 * id] = xy[2 * id];
        xy_f[2 * id + 1] = xy[2 * id + 1];
        dir_f[id] = dir[id];
        return;
    }
    const int64_t e = id - n;
    const int32_t a = ends[2 * e], b = ends[2 * e + 1];
    xy_f[2 * id] = (xy[2 * a] + xy[2 * b]) * 0.5;
    xy_f[2 * id + 1] = (xy[2 * a + 1] + xy[2 * b + 1]) * 0.5;
    dir_f[id] = (boundary[e] && dir[a] && dir[b]) ? 1 : 0;
}

// id of edge {a, b}: the entries of node lo's sorted adjacency row that exceed lo
// are its edges in order, starting at edge_ptr[lo]
__device__ inline int32_t edge_id(const int32_t *adj_ptr, const int32_t *adj_col, const int32_t *edge_ptr,
                                  int32_t a, int32_t b) {
    const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
    int32_t rank = 0;
    for (int32_t k = adj_ptr[lo]; k < adj_ptr[lo + 1]; ++k) {
        const int32_t c = adj_col[k];
        if (c > lo && c < hi) ++rank;
    }
    return edge_ptr[lo] + rank;
}

__global__ void k_refine_tris(int64_t T, int64_t n, const int32_t *tri, const int32_t *adj_ptr,
                              const int32_t *adj_col, const int32_t *edge_ptr, int32_t *tri_f) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    const int32_t mab = static_cast<int32_t>(n) + edge_id(adj_ptr, adj_col, edge_ptr, a, b);
    const int32_t mbc = static_cast<int32_t>(n) + edge_id(adj_ptr, adj_col, edge_ptr, b, c);
    const int32_t mca = static_cast<int32_t>(n) + edge_id(adj_ptr, adj_col, edge_ptr, c, a);
    int32_t *o = tri_f + 12 * t;
    o[0] = a;   o[1] = mab;  o[2] = mca;
    o[3] = mab; o[4] = b;    o[5] = mbc;
    o[6] = mca; o[7] = mbc;  o[8] = c;
    o[9] = mab; o[10] = mbc; o[11] = mca;
}

// ------------------------------------------------------------------ P1 stiffness (level 0)

__global__ void k_csr_count(int64_t n, const int32_t *adj_ptr, const int32_t *adj_col, const uint8_t *dir,
                            int32_t *cnt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (dir[i]) {
        cnt[i] = 1;
        return;
    }
    int32_t u = 0;
    for (int32_t k = adj_ptr[i]; k < adj_ptr[i + 1]; ++k) u += dir[adj_col[k]] == 0;
    cnt[i] = u;
}

// Row i of K: sum over the triangles e around i (ascending e) of
// A_e grad(psi_i).grad(psi_j) = (beta_i . beta_j) / (2 D_e), with D_e = 2 A_e and
// beta_a = (y_b - y_c, x_c - x_b) (cyclic), skipping Dirichlet columns;
// Dirichlet rows are identity rows.
__global__ void k_csr_fill(int64_t n, const int32_t *adj_ptr, const int32_t *adj_col, const uint8_t *dir,
                           const int32_t *rowptr, const int32_t *ne_ptr, const int32_t *ne_idx,
                           const int32_t *tri, const double *xy, int32_t *col, double *val, double *dinv,
                           float *val32, float *dinv32) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r0 = rowptr[i], r1 = rowptr[i + 1];
    if (dir[i]) {
        col[r0] = static_cast<int32_t>(i);
        val[r0] = 1.0;
        val32[r0] = 1.0f;
        dinv[i] = 1.0;
        dinv32[i] = 1.0f;
        return;
    }
    int32_t w = r0;
    for (int32_t k = adj_ptr[i]; k < adj_ptr[i + 1]; ++k) {
        const int32_t j = adj_col[k];
        if (dir[j] == 0) {
            col[w] = j;
            val[w] = 0.0;
            ++w;
        }
    }
    for (int32_t k = ne_ptr[i]; k < ne_ptr[i + 1]; ++k) {
        const int64_t e = ne_idx[k];
        int32_t v[3];
        double x[3], y[3];
        int li = 0;
        for (int c = 0; c < 3; ++c) {
            v[c] = tri[3 * e + c];
            x[c] = xy[2 * v[c]];
            y[c] = xy[2 * v[c] + 1];
            if (v[c] == i) li = c;
        }
        const double d = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
        double bx[3], by[3];
        for (int c = 0; c < 3; ++c) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            bx[c] = y[c1] - y[c2];
            by[c] = x[c2] - x[c1];
        }
        for (int c = 0; c < 3; ++c) {
            const int32_t j = v[c];
            if (dir[j]) continue;
            const double kij = (bx[li] * bx[c] + by[li] * by[c]) / (2.0 * d);
            int32_t pos = r0;
            while (col[pos] != j) ++pos;
            val[pos] += kij;
        }
    }
    double diag = 0.0;
    for (int32_t k = r0; k < r1; ++k) {
        val32[k] = static_cast<float>(val[k]);
        if (col[k] == i) diag = val[k];
    }
    dinv[i] = 1.0 / diag;
    dinv32[i] = static_cast<float>(1.0 / diag);
}

__global__ void k_max_row(int64_t n, const int32_t *rowptr, int32_t *out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(out, rowptr[i + 1] - rowptr[i]);
}

// ------------------------------------------------------------------ neighbour table

// longest list of mesh neighbours (self excluded) over the nodes
__global__ void k_nbr_width(int64_t n, const int32_t *adj_ptr, const int32_t *adj_col, int32_t *out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = 0;
    for (int32_t k = adj_ptr[i]; k < adj_ptr[i + 1]; ++k) c += adj_col[k] != i;
    atomicMax(out, c);
}

// Column-major neighbour table: neighbour k (adjacency order, self skipped) of node i at
// k * n + i, padded with n (a row past the end that the reader keeps at zero), so that a
// gather of all neighbours of 64 consecutive nodes is a fixed number of coalesced index
// loads with no per-row lookup and no branch.
__global__ void k_nbr_fill(int64_t n, int32_t width, const int32_t *adj_ptr, const int32_t *adj_col,
                           int32_t *nbr) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = 0;
    for (int32_t k = adj_ptr[i]; k < adj_ptr[i + 1]; ++k)
        if (adj_col[k] != i) nbr[static_cast<int64_t>(c++) * n + i] = adj_col[k];
    for (; c < width; ++c) nbr[static_cast<int64_t>(c) * n + i] = static_cast<int32_t>(n);
}

// ------------------------------------------------------------------ ELL copy of K

// Column-major ELL: entry k of row i at k * n + i, width = the longest row.  A
// wavefront reads entry k of 64 consecutive rows with one coalesced load and the
// address needs no per-row lookup.  Shorter rows are padded with (column = the
// row itself, value = 0).
__global__ void k_ell_fill(int64_t n, int32_t width, const int32_t *rowptr, const int32_t *col, const double *val,
                           const float *val32, int32_t *ecol, double *eval, float *eval32) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t k0 = rowptr[i], len = rowptr[i + 1] - k0;
    for (int32_t k = 0; k < width; ++k) {
        const int64_t o = static_cast<int64_t>(k) * n + i;
        if (k < len) {
            ecol[o] = col[k0 + k];
            eval[o] = val[k0 + k];
            eval32[o] = val32[k0 + k];
        } else {
            ecol[o] = static_cast<int32_t>(i);
            eval[o] = 0.0;
            eval32[o] = 0.0f;
        }
    }
}

template <class T>
void h2d(hipStream_t s, DBuf<T> &dst, const T *src, size_t count) {
    dst.alloc(count);
    CGP_HIP(hipMemcpyAsync(dst.p, src, count * sizeof(T), hipMemcpyHostToDevice, s));
}

int32_t read_i32(hipStream_t s, const int32_t *d) {
    int32_t v = 0;
    CGP_HIP(hipMemcpyAsync(&v, d, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CGP_HIP(hipStreamSynchronize(s));
    return v;
}

void build_incidence(hipStream_t s, Level &L) {
    DBuf<int32_t> cnt, cursor;
    cnt.alloc(L.n);
    cursor.alloc(L.n);
    CGP_HIP(hipMemsetAsync(cnt.p, 0, L.n * sizeof(int32_t), s));
    CGP_HIP(hipMemsetAsync(cursor.p, 0, L.n * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_count_incident, dim3(blocks_for(L.T, TPB)), dim3(TPB), 0, s, L.T, L.tri.p, cnt.p);
    L.ne_ptr.alloc(L.n + 1);
    scan_rec(s, cnt.p, L.ne_ptr.p, L.n);
    L.ne_idx.alloc(3 * L.T);
    hipLaunchKernelGGL(k_fill_incident, dim3(blocks_for(L.T, TPB)), dim3(TPB), 0, s, L.T, L.tri.p,
                       L.ne_ptr.p, cursor.p, L.ne_idx.p);
    hipLaunchKernelGGL(k_sort_segments, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, L.ne_ptr.p,
                       L.ne_idx.p);
    CGP_HIP(hipGetLastError());
    CGP_HIP(hipStreamSynchronize(s));
}

void build_adjacency(hipStream_t s, const Level &L, DBuf<int32_t> &adj_ptr, DBuf<int32_t> &adj_col,
                     int64_t &adj_nnz) {
    DBuf<int32_t> cand, cnt;
    cand.alloc(9 * L.T);
    cnt.alloc(L.n);
    hipLaunchKernelGGL(k_adj_candidates, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, L.ne_ptr.p,
                       L.ne_idx.p, L.tri.p, cand.p, cnt.p);
    CGP_HIP(hipGetLastError());
    adj_ptr.alloc(L.n + 1);
    scan_rec(s, cnt.p, adj_ptr.p, L.n);
    adj_nnz = read_i32(s, adj_ptr.p + L.n);
    adj_col.alloc(adj_nnz);
    hipLaunchKernelGGL(k_adj_compact, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, L.ne_ptr.p, cand.p,
                       adj_ptr.p, adj_col.p);
    CGP_HIP(hipGetLastError());
    CGP_HIP(hipStreamSynchronize(s));
}

}  // namespace

void level_adjacency(hipStream_t s, const Level &L, DBuf<int32_t> &adj_ptr, DBuf<int32_t> &adj_col,
                     int64_t &adj_nnz) {
    build_adjacency(s, L, adj_ptr, adj_col, adj_nnz);
}

int64_t exclusive_scan(hipStream_t s, const int32_t *in, int32_t *out, int64_t n) {
    scan_rec(s, in, out, n);
    return read_i32(s, out + n);
}

void build_hierarchy(hipStream_t s, Mesh &m, const double *h_xy, int64_t n, const int32_t *h_tri,
                     int64_t T, const uint8_t *h_dir, int32_t k) {
    m.k = k;
    m.lv.clear();
    m.lv.resize(k + 1);
    {
        Level &L = m.lv[0];
        L.n = n;
        L.T = T;
        h2d(s, L.xy, h_xy, 2 * n);
        h2d(s, L.tri, h_tri, 3 * T);
        h2d(s, L.dir, h_dir, n);
        DBuf<int32_t> flag;
        flag.alloc(1);
        CGP_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_validate, dim3(blocks_for(T, TPB)), dim3(TPB), 0, s, n, T, L.xy.p, L.tri.p, flag.p);
        CGP_HIP(hipGetLastError());
        const int32_t f = read_i32(s, flag.p);
        if (f & 1) throw Error{CGP_E_MESH, "triangle vertex id out of range"};
        if (f & 2) throw Error{CGP_E_MESH, "triangle with a repeated vertex"};
        if (f & 4) throw Error{CGP_E_MESH, "triangle with non-positive signed area (must be CCW)"};
    }
    for (int32_t l = 0; l <= k; ++l) {
        Level &L = m.lv[l];
        build_incidence(s, L);
        if (l == k && l != 0) break;   // the finest level needs incidence only
        // adjacency: kept for level 0, temporary above
        DBuf<int32_t> tptr, tcol;
        int64_t tnnz = 0;
        DBuf<int32_t> &adj_ptr = (l == 0) ? m.adj_ptr : tptr;
        DBuf<int32_t> &adj_col = (l == 0) ? m.adj_col : tcol;
        int64_t &adj_nnz = (l == 0) ? m.adj_nnz : tnnz;
        build_adjacency(s, L, adj_ptr, adj_col, adj_nnz);
        if (l == 0) {
            // row lengths of the system matrix; a free node without triangles has
            // an empty row (K singular) and is rejected
            DBuf<int32_t> flag, deg;
            flag.alloc(1);
            deg.alloc(L.n);
            CGP_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
            hipLaunchKernelGGL(k_csr_count, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, adj_ptr.p,
                               adj_col.p, L.dir.p, deg.p);
            hipLaunchKernelGGL(k_isolated, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, deg.p, flag.p);
            CGP_HIP(hipGetLastError());
            if (read_i32(s, flag.p) & 8) throw Error{CGP_E_MESH, "a free node belongs to no triangle"};
            m.rowptr.alloc(L.n + 1);
            m.nnz = exclusive_scan(s, deg.p, m.rowptr.p, L.n);
            m.col.alloc(m.nnz);
            m.val.alloc(m.nnz);
            m.val32.alloc(m.nnz);
            m.dinv.alloc(L.n);
            m.dinv32.alloc(L.n);
            hipLaunchKernelGGL(k_csr_fill, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, adj_ptr.p,
                               adj_col.p, L.dir.p, m.rowptr.p, L.ne_ptr.p, L.ne_idx.p, L.tri.p, L.xy.p,
                               m.col.p, m.val.p, m.dinv.p, m.val32.p, m.dinv32.p);
            CGP_HIP(hipGetLastError());
            DBuf<int32_t> mr;
            mr.alloc(1);
            CGP_HIP(hipMemsetAsync(mr.p, 0, sizeof(int32_t), s));
            hipLaunchKernelGGL(k_max_row, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, m.rowptr.p, mr.p);
            CGP_HIP(hipGetLastError());
            m.max_row = read_i32(s, mr.p);
            // ELL copy
            m.ell_col.alloc(static_cast<size_t>(m.max_row) * L.n);
            m.ell_val.alloc(static_cast<size_t>(m.max_row) * L.n);
            m.ell_val32.alloc(static_cast<size_t>(m.max_row) * L.n);
            hipLaunchKernelGGL(k_ell_fill, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, m.max_row, m.rowptr.p,
                               m.col.p, m.val.p, m.val32.p, m.ell_col.p, m.ell_val.p, m.ell_val32.p);
            CGP_HIP(hipGetLastError());
            // neighbour table of the learned guess: width 6 when it fits, else a multiple of 8
            CGP_HIP(hipMemsetAsync(mr.p, 0, sizeof(int32_t), s));
            hipLaunchKernelGGL(k_nbr_width, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, adj_ptr.p,
                               adj_col.p, mr.p);
            CGP_HIP(hipGetLastError());
            const int32_t nw = read_i32(s, mr.p);
            m.nbr_w = nw <= NBR_NARROW ? NBR_NARROW : (nw + NBR_WIDE - 1) / NBR_WIDE * NBR_WIDE;
            m.nbr.alloc(static_cast<size_t>(m.nbr_w) * L.n);
            hipLaunchKernelGGL(k_nbr_fill, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, m.nbr_w, adj_ptr.p,
                               adj_col.p, m.nbr.p);
            CGP_HIP(hipGetLastError());
            CGP_HIP(hipStreamSynchronize(s));
        }
        if (l == k) break;
        // edges of level l
        DBuf<int32_t> ecnt, edge_ptr;
        DBuf<uint8_t> boundary;
        ecnt.alloc(L.n);
        edge_ptr.alloc(L.n + 1);
        hipLaunchKernelGGL(k_edge_count, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, adj_ptr.p,
                           adj_col.p, ecnt.p);
        CGP_HIP(hipGetLastError());
        L.E = exclusive_scan(s, ecnt.p, edge_ptr.p, L.n);
        L.ends.alloc(2 * L.E);
        boundary.alloc(L.E);
        hipLaunchKernelGGL(k_edge_fill, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, adj_ptr.p,
                           adj_col.p, edge_ptr.p, L.ne_ptr.p, L.ne_idx.p, L.ends.p, boundary.p);
        CGP_HIP(hipGetLastError());
        // level l+1
        Level &F = m.lv[l + 1];
        F.n = L.n + L.E;
        F.T = 4 * L.T;
        if (F.n > INT32_MAX || 9 * F.T > INT32_MAX)
            throw Error{CGP_E_INVALID, "refined mesh exceeds 32-bit indexing"};
        F.xy.alloc(2 * F.n);
        F.dir.alloc(F.n);
        F.tri.alloc(3 * F.T);
        hipLaunchKernelGGL(k_refine_nodes, dim3(blocks_for(F.n, TPB)), dim3(TPB), 0, s, L.n, L.E, L.xy.p,
                           L.dir.p, L.ends.p, boundary.p, F.xy.p, F.dir.p);
        hipLaunchKernelGGL(k_refine_tris, dim3(blocks_for(L.T, TPB)), dim3(TPB), 0, s, L.T, L.n, L.tri.p,
                           adj_ptr.p, adj_col.p, edge_ptr.p, F.tri.p);
        CGP_HIP(hipGetLastError());
        CGP_HIP(hipStreamSynchronize(s));
        if (l + 1 < k) F.tmp.alloc(F.n);
    }
    CGP_HIP(hipStreamSynchronize(s));
}

}  // namespace cgp
