// The semi-implicit momentum step of the CGP algorithm (step 4, Eqs. 13-14; the general
// scheme Eq. 8) on the finest level, Galerkin P1 (Section 2.3): for w = u and w = v
//
//   A w~ = b,  A = (rho/dt) M + rho C(u^n) + mu K,  b = (rho/dt) M w^n + M f,
//
// M_ij = int psi_i psi_j, C_ij = int psi_i (u^n . grad psi_j) (u^n in P1), K the
// stiffness; Dirichlet rows are identity rows with the caller's boundary values.  The
// Dirichlet rows of the two components may differ (a slip wall fixes v only, a natural
// outflow neither: Section 3): such a row is assembled in full and each product replaces
// it by the identity for the component that is fixed there.
//
// The operator is assembled row by row (one thread per row: the incident triangles in
// ascending id order, no atomics) into a column-major ELL copy of the finest level's
// adjacency pattern (entry k of row i at k * n + i, width = the longest row rounded up to 7,
// 8, 12, 16, 24 or 33, padding: the
// row itself with value 0, so that a wavefront reads entry k of 64 consecutive rows with
// one coalesced load), together with both right-hand sides.  Both components share it and are solved together by
// Jacobi-preconditioned BiCGStab (van der Vorst) in fp64: a thread applies each matrix
// row it reads to both components.  An iteration is two launches,
//   HA  x += alpha D^-1 p + omega D^-1 s, r = s - omega t (the end of the previous
//       iteration), p' = r + beta (p - omega v), v' = A D^-1 p'    partials  rh.v', r.r
//   HB  s = r - alpha v', t = A D^-1 s                             partials  t.s, t.t, rh.t, rh.s
// with omega = t.s / t.t and rh.r = rh.s - omega rh.t formed from HB's partials, so that
// the update of x and r needs no launch of its own; the test on
// |r| uses r.r summed row by row in HA.  The preconditioned vectors of the neighbours are
// formed on the fly from the previous launch's vectors (so no launch waits on another's
// row updates), and every
// workgroup derives the scalars it needs from the previous launch's per-workgroup
// partials in a fixed order (no floating-point atomics: bitwise reproducible).  The
// grid is one workgroup per compute unit, each over a contiguous block of rows.
#include <algorithm>
#include <cmath>

#include "cgp_internal.hpp"

namespace cgp {

namespace {

constexpr int MB = 512;          // threads per workgroup
constexpr int MG = 256;          // workgroups of the BiCGStab launches
constexpr int MAX_ROW = 33;      // a node and at most 32 neighbours
constexpr int MQ = 4;            // partial sums per component and launch
constexpr int CHECK_EVERY = 4;   // iterations between the host's looks at the status near the
                                 // predicted end (the previous call's count), 32 before it

// scalar slots per component (scal[c * NS + ...]); slots indexed by parity hold the
// values of iteration it at it & 1
enum { S_BB = 0, S_RHO = 1, S_ALPHA = 3, S_RR = 5, NS = 6 };
// state per component: status (-1 running, ST_SUSPECT: HA found beta undefined and HB
// decides between converged and breakdown, else CGP_SOLVE_*), iterations
enum { ST_STATUS = 0, ST_ITERS = 1, NSTATE = 2 };
constexpr int ST_SUSPECT = -2;

// one thread per row: the operator row and both right-hand sides
__global__ __launch_bounds__(256) void k_mom_assemble(int64_t n, int width, const int32_t *ecol,
                                                      const int32_t *perm, const int32_t *inv,
                                                      const int32_t *ne_ptr, const int32_t *ne_idx,
                                                      const int32_t *tri, const double *xy, const uint8_t *mask,
                                                      int both, uint8_t *rowmask, const double *un, const double *vn, const double *fx,
                                                      const double *fy, const double *gu, const double *gv,
                                                      double rho, double mu, double dt, double *val, double *dinv,
                                                      double *b) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t pd = i;   // the diagonal entry (the first entry whose column is the row)
    for (int k = width - 1; k >= 0; --k) {
        const int64_t o = static_cast<int64_t>(k) * n + i;
        val[o] = 0.0;
        if (ecol[o] == i) pd = o;
    }
    // row i of the own numbering is mesh node o; the mesh's arrays are read at mesh indices
    const int32_t o = perm[i];
    const int rm = both ? (mask[o] ? 3 : 0) : (mask[o] & 3);
    rowmask[i] = static_cast<uint8_t>(rm);
    if (rm == 3) {
        val[pd] = 1.0;
        dinv[i] = 1.0;
        b[2 * i] = gu[o];
        b[2 * i + 1] = gv[o];
        return;
    }
    const double rdt = rho / dt;
    double bu = 0.0, bv = 0.0;
    for (int32_t q = ne_ptr[o]; q < ne_ptr[o + 1]; ++q) {
        const int64_t e = ne_idx[q];
        const int32_t v3[3] = {tri[3 * e], tri[3 * e + 1], tri[3 * e + 2]};
        const int li = v3[0] == o ? 0 : (v3[1] == o ? 1 : 2);
        const double xa = xy[2 * v3[0]], ya = xy[2 * v3[0] + 1];
        const double xb = xy[2 * v3[1]], yb = xy[2 * v3[1] + 1];
        const double xc = xy[2 * v3[2]], yc = xy[2 * v3[2] + 1];
        const double twice = (xb - xa) * (yc - ya) - (xc - xa) * (yb - ya);
        const double area = 0.5 * twice;
        const double gx[3] = {(yb - yc) / twice, (yc - ya) / twice, (ya - yb) / twice};
        const double gy[3] = {(xc - xb) / twice, (xa - xc) / twice, (xb - xa) / twice};
        // int psi_i psi_k = A (1 + delta_ik) / 12: the advecting velocity's weight in row i
        const double ax = area / 12.0 * (un[v3[0]] + un[v3[1]] + un[v3[2]] + un[o]);
        const double ay = area / 12.0 * (vn[v3[0]] + vn[v3[1]] + vn[v3[2]] + vn[o]);
        for (int lj = 0; lj < 3; ++lj) {
            const int32_t j = v3[lj], jo = inv[j];   // mesh index, own index
            const double mij = area * (lj == li ? 2.0 : 1.0) / 12.0;
            const double a = rdt * mij + rho * (ax * gx[lj] + ay * gy[lj]) +
                             mu * area * (gx[li] * gx[lj] + gy[li] * gy[lj]);
            int k = 0;   // j is in the row (a vertex of a triangle of node i); padding comes last
            while (k < width - 1 && ecol[static_cast<int64_t>(k) * n + i] != jo) ++k;
            val[static_cast<int64_t>(k) * n + i] += a;
            bu += mij * (rdt * un[j] + fx[j]);
            bv += mij * (rdt * vn[j] + fy[j]);
        }
    }
    // a component with its own Dirichlet row keeps the full row here; the products replace
    // that component's row by the identity
    dinv[i] = 1.0 / val[pd];
    b[2 * i] = (rm & 1) ? gu[o] : bu;
    b[2 * i + 1] = (rm & 2) ? gv[o] : bv;
}

// the iterate in the own numbering from the caller's vectors, and back
__global__ void k_mom_gather(int64_t n, const int32_t *perm, const double *u, const double *v, double *x) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t o = perm[i];
    x[i] = u[o];
    x[n + i] = v[o];
}
__global__ void k_mom_scatter(int64_t n, const int32_t *perm, const double *x, double *u, double *v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t o = perm[i];
    u[o] = x[i];
    v[o] = x[n + i];
}

// the workgroup's partial sums (q values per component) in a fixed order, to
// part[(c * MQ + q) * MG + block]
__device__ inline void block_partials(const double (&v)[2][MQ], double *part, int blk) {
    __shared__ double red[MB / 64][2][MQ];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < MQ; ++q) {
            double x = v[c][q];
            for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
            if (lane == 0) red[wave][c][q] = x;
        }
    __syncthreads();
    if (threadIdx.x < 2 * MQ) {
        const int c = threadIdx.x / MQ, q = threadIdx.x % MQ;
        double t = 0.0;
        for (int w = 0; w < MB / 64; ++w) t += red[w][c][q];
        part[(c * MQ + q) * MG + blk] = t;
    }
}

// the sums of a launch's partials (every workgroup, the same fixed order): sums[c][q]; the
// first wavefront issues all its loads before the first add (a fixed trip count), so the
// reduction costs one memory latency, not one per load
static_assert(MG % 64 == 0, "the partials are reduced by one wavefront");
__device__ inline void reduce_partials(const double *part, double (*sums)[MQ]) {
    __shared__ double red[2 * MQ];
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        double x[2 * MQ][MG / 64];
#pragma unroll
        for (int cq = 0; cq < 2 * MQ; ++cq)
#pragma unroll
            for (int t = 0; t < MG / 64; ++t) x[cq][t] = part[cq * MG + t * 64 + lane];
#pragma unroll
        for (int cq = 0; cq < 2 * MQ; ++cq) {
            double y = 0.0;
#pragma unroll
            for (int t = 0; t < MG / 64; ++t) y += x[cq][t];
            for (int m = 32; m >= 1; m >>= 1) y += __shfl_xor(y, m, 64);
            if (lane == 0) red[cq] = y;
        }
    }
    __syncthreads();
    for (int cq = 0; cq < 2 * MQ; ++cq) sums[cq / MQ][cq % MQ] = red[cq];
}

// both components of row j of an interleaved [n][2] vector
__device__ inline double2 ld2(const double *v, int64_t j) { return reinterpret_cast<const double2 *>(v)[j]; }

struct Rows {
    int64_t r0, r1;
};
// contiguous row blocks, consecutive ones on the same XCD (its L2 holds the neighbours)
__device__ inline Rows block_rows(int64_t n) {
    const int64_t per = (n + MG - 1) / MG;
    const int64_t r0 = static_cast<int64_t>(xcd_block(blockIdx.x, MG)) * per;
    return {r0, r0 + per < n ? r0 + per : n};
}

// column-major ELL copy of the CSR pattern (padding: the row itself)
__global__ void k_mom_ell(int64_t n, int width, const int32_t *ptr, const int32_t *col, int32_t *ecol) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t p0 = ptr[i], len = ptr[i + 1] - p0;
    for (int k = 0; k < width; ++k) ecol[static_cast<int64_t>(k) * n + i] = k < len ? col[p0 + k] : static_cast<int32_t>(i);
}

struct Vecs {
    int64_t n;
    int width;
    const int32_t *col;   // ELL: entry k of row i at k * n + i
    const double *val, *dinv, *b;
    const uint8_t *mask;   // per row: bit c = component c has a Dirichlet (identity) row
    double *x[2];
    double *r, *rh, *p, *v, *s, *t;   // [n][2] (the components interleaved); p and v: [2 parities][n][2]
    double *part1, *part2, *part3;
    double *scal;
    int32_t *state;
    double tol;
    int max_iter;
};

__device__ inline int row_mask(const Vecs &V, int64_t i) { return V.mask[i]; }

// The product kernels are instantiated for the ELL width W (the longest row rounded up to
// a bin, the padding: the row itself with value 0): the loop over a row's entries unrolls,
// so a thread issues a row's gathers before the first one returns.

// rows of up to 12 entries unroll fully; longer ones by 8 (a full unroll would spill);
// HA, which gathers four vectors per entry, unrolls rows of 12 by 6
template <int W>
constexpr int UNROLL = W <= 12 ? W : 8;
template <int W>
constexpr int UNROLL_HA = W <= 8 ? W : (W == 12 ? 6 : 8);

// H0: r = b - A x, rh = s = r, t = 0, p = v = 0 (parity 0); partials rh.r, r.r, b.b
template <int W>
__global__ __launch_bounds__(MB) void k_mom_start(Vecs V) {
    const Rows R = block_rows(V.n);
    double acc[2][MQ] = {};
    const int64_t n = V.n;
    for (int64_t i = R.r0 + threadIdx.x; i < R.r1; i += MB) {
        double ax0 = 0.0, ax1 = 0.0;
#pragma unroll UNROLL<W>
        for (int k = 0; k < W; ++k) {
            const int64_t o = static_cast<int64_t>(k) * n + i;
            const int32_t j = V.col[o];
            ax0 += V.val[o] * V.x[0][j];
            ax1 += V.val[o] * V.x[1][j];
        }
        const int rm = row_mask(V, i);
        if (rm & 1) ax0 = V.x[0][i];
        if (rm & 2) ax1 = V.x[1][i];
        const double rr[2] = {V.b[2 * i] - ax0, V.b[2 * i + 1] - ax1};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            V.r[2 * i + c] = rr[c];
            V.rh[2 * i + c] = rr[c];
            V.s[2 * i + c] = rr[c];
            V.t[2 * i + c] = 0.0;
            V.p[2 * i + c] = 0.0;
            V.v[2 * i + c] = 0.0;
            acc[c][0] += rr[c] * rr[c];
            acc[c][1] += rr[c] * rr[c];
            acc[c][2] += V.b[2 * i + c] * V.b[2 * i + c];
        }
    }
    block_partials(acc, V.part3, blockIdx.x);
}

// The status of a component as the previous launch left it (every launch reads the
// previous launch's copy and its workgroup 0 writes its own, so no workgroup reads what
// another one of the same launch writes).  Launch q (H0 = 0, HA of iteration it = 2 it - 1,
// HB of iteration it = 2 it) reads copy (q - 1) & 1 and writes copy q & 1.
__device__ inline const int32_t *state_in(const Vecs &V, int q, int c) {
    return V.state + ((q - 1) & 1) * 2 * NSTATE + c * NSTATE;
}
__device__ inline int32_t *state_out(const Vecs &V, int q, int c) {
    return V.state + (q & 1) * 2 * NSTATE + c * NSTATE;
}

// HA of iteration it >= 1: the end of iteration it - 1 and the start of iteration it.
// From HB's partials of it - 1 (t.s, t.t, rh.t, rh.s):
//   omega = t.s / t.t,  rho = rh.r = rh.s - omega rh.t,  beta = (rho / rho')(alpha / omega)
// (rho' = rh.r of it - 2, alpha of it - 1; every inner product summed afresh, so that no
// rounding error is carried from one iteration to the next);
// per row
//   x += alpha D^-1 p + omega D^-1 s,  r = s - omega t,
//   p' = r + beta (p - omega v),  v' = A D^-1 p'          partials rh.v', r.r
// with the neighbours' p' formed from their s, t, p, v.  Iteration 1 starts from H0's
// partials: rho = rh.r, b.b, and the test of the initial residual.
template <int W>
__global__ __launch_bounds__(MB) void k_mom_ha(Vecs V, int it) {
    __shared__ double sums[2][MQ];
    __shared__ double al_s[2], om_s[2], be_s[2];
    __shared__ int upd_s[2], run_s[2], zero_s[2];
    reduce_partials(it == 1 ? V.part3 : V.part2, sums);
    const int q = 2 * it - 1, rd = (it - 1) & 1, wr = it & 1;
    if (threadIdx.x < 2) {
        const int c = threadIdx.x;
        double *sc = V.scal + c * NS;
        const int32_t *si = state_in(V, q, c);
        int status = si[ST_STATUS], iters = si[ST_ITERS];
        const int was = status < 0;
        int upd = 0, zero = 0;
        double alpha = 0.0, omega = 0.0, beta = 0.0;
        if (was) {
            if (it == 1) {
                const double rho = sums[c][0], rr = sums[c][1], bb = sums[c][2];
                if (bb == 0.0) {
                    status = CGP_SOLVE_OK;   // b = 0: the solution is 0
                    zero = 1;
                } else if (rr <= V.tol * V.tol * bb) {
                    status = CGP_SOLVE_OK;
                }
                if (status >= 0) iters = 0;
                if (blockIdx.x == 0) {
                    sc[S_BB] = bb;
                    sc[S_RHO + 0] = rho;
                    sc[S_RR] = rr;
                }
            } else {
                const double ts = sums[c][0], tt = sums[c][1], rht = sums[c][2], rhs = sums[c][3];
                alpha = sc[S_ALPHA + rd];
                // t = 0 (s = 0 or a singular operator): omega = 0, r = s
                omega = tt != 0.0 ? ts / tt : 0.0;
                const double rho_p = sc[S_RHO + (it & 1)];   // rho of iteration it - 2
                const double rho = rhs - omega * rht;
                upd = 1;
                if (it <= V.max_iter) {
                    beta = (rho / rho_p) * (alpha / omega);
                    // near convergence t.t or rho can vanish: HB tests the residual first
                    if (!std::isfinite(beta) || rho == 0.0) {
                        status = ST_SUSPECT;
                        iters = it - 1;
                    }
                }
                if (blockIdx.x == 0) sc[S_RHO + rd] = rho;
            }
        }
        if (blockIdx.x == 0) {
            int32_t *so = state_out(V, q, c);
            so[ST_STATUS] = status;
            so[ST_ITERS] = iters;
        }
        upd_s[c] = upd;
        zero_s[c] = zero;
        run_s[c] = status == -1 && it <= V.max_iter;
        al_s[c] = alpha;
        om_s[c] = omega;
        be_s[c] = beta;
    }
    __syncthreads();
    const Rows R = block_rows(V.n);
    const int64_t n = V.n;
#pragma unroll
    for (int c = 0; c < 2; ++c)
        if (zero_s[c])
            for (int64_t i = R.r0 + threadIdx.x; i < R.r1; i += MB) V.x[c][i] = 0.0;
    const double *pr = V.p + rd * 2 * n, *vr = V.v + rd * 2 * n;
    double *pw = V.p + wr * 2 * n, *vw = V.v + wr * 2 * n;
    const double al[2] = {al_s[0], al_s[1]}, om[2] = {om_s[0], om_s[1]}, be[2] = {be_s[0], be_s[1]};
    const bool upd[2] = {upd_s[0] != 0, upd_s[1] != 0}, run[2] = {run_s[0] != 0, run_s[1] != 0};
    double acc[2][MQ] = {};
    if (upd[0] || upd[1] || run[0] || run[1]) {
        for (int64_t i = R.r0 + threadIdx.x; i < R.r1; i += MB) {
            const double di = V.dinv[i];
            double rn[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double sv = V.s[2 * i + c];
                rn[c] = sv - om[c] * V.t[2 * i + c];
                if (upd[c]) {
                    V.x[c][i] += al[c] * di * pr[2 * i + c] + om[c] * di * sv;
                    V.r[2 * i + c] = rn[c];
                }
                // r.r whenever r is new or in use: HB tests it even when no product follows
                if (upd[c] || run[c]) acc[c][1] += rn[c] * rn[c];
            }
            if (!run[0] && !run[1]) continue;
            double y[2] = {0.0, 0.0};
#pragma unroll UNROLL_HA<W>
            for (int k = 0; k < W; ++k) {
                const int64_t o = static_cast<int64_t>(k) * n + i;
                const int32_t j = V.col[o];
                const double a = V.val[o] * V.dinv[j];
                // the neighbour's p' from its s, t, p, v (one 16-byte load per vector)
                const double2 sj = ld2(V.s, j), tj = ld2(V.t, j), pj = ld2(pr, j), vj = ld2(vr, j);
                y[0] += a * ((sj.x - om[0] * tj.x) + be[0] * (pj.x - om[0] * vj.x));
                y[1] += a * ((sj.y - om[1] * tj.y) + be[1] * (pj.y - om[1] * vj.y));
            }
            const int rm = row_mask(V, i);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (!run[c]) continue;
                const double pi = rn[c] + be[c] * (pr[2 * i + c] - om[c] * vr[2 * i + c]);
                if (rm & (1 << c)) y[c] = di * pi;   // identity row of this component
                pw[2 * i + c] = pi;
                vw[2 * i + c] = y[c];
                acc[c][0] += V.rh[2 * i + c] * y[c];
            }
        }
    }
    block_partials(acc, V.part1, blockIdx.x);
}

// HB of iteration it (reads HA's partials rh.v', r.r): the test of r (the residual after
// iteration it - 1, summed row by row), then alpha = rho / rh.v',
//   s = r - alpha v',  t = A D^-1 s                             partials t.s, t.t, rh.t, rh.s
template <int W>
__global__ __launch_bounds__(MB) void k_mom_hb(Vecs V, int it) {
    __shared__ double sums[2][MQ];
    __shared__ double alpha_s[2];
    __shared__ int run_s[2];
    reduce_partials(V.part1, sums);
    const int q = 2 * it, wr = it & 1;
    if (threadIdx.x < 2) {
        const int c = threadIdx.x;
        double *sc = V.scal + c * NS;
        const int32_t *si = state_in(V, q, c);
        int status = si[ST_STATUS], iters = si[ST_ITERS];
        double alpha = 0.0;
        if (status < 0) {
            const double rhv = sums[c][0], rr = sums[c][1];
            if (status == ST_SUSPECT) {
                status = rr <= V.tol * V.tol * sc[S_BB] ? CGP_SOLVE_OK : CGP_SOLVE_BREAKDOWN;
                iters = it - 1;
            } else if (rr <= V.tol * V.tol * sc[S_BB]) {
                status = CGP_SOLVE_OK;
                iters = it - 1;
            } else if (it > V.max_iter) {
                status = CGP_SOLVE_NOCONV;
                iters = it - 1;
            } else {
                alpha = sc[S_RHO + ((it - 1) & 1)] / rhv;
                if (!std::isfinite(alpha)) {
                    status = CGP_SOLVE_BREAKDOWN;
                    iters = it - 1;
                }
            }
            if (blockIdx.x == 0) {
                sc[S_RR] = rr;
                sc[S_ALPHA + wr] = alpha;   // (unused once the component has finished)
            }
        }
        if (blockIdx.x == 0) {
            int32_t *so = state_out(V, q, c);
            so[ST_STATUS] = status;
            so[ST_ITERS] = iters;
        }
        run_s[c] = status < 0;
        alpha_s[c] = alpha;
    }
    __syncthreads();
    const Rows R = block_rows(V.n);
    const int64_t n = V.n;
    const double *vw = V.v + wr * 2 * n;
    const double al[2] = {alpha_s[0], alpha_s[1]};
    const bool run[2] = {run_s[0] != 0, run_s[1] != 0};
    double acc[2][MQ] = {};
    if (run[0] || run[1]) {
        for (int64_t i = R.r0 + threadIdx.x; i < R.r1; i += MB) {
            double t[2] = {0.0, 0.0};
#pragma unroll UNROLL<W>
            for (int k = 0; k < W; ++k) {
                const int64_t o = static_cast<int64_t>(k) * n + i;
                const int32_t j = V.col[o];
                const double a = V.val[o] * V.dinv[j];
                const double2 rj = ld2(V.r, j), vj = ld2(vw, j);
                t[0] += a * (rj.x - al[0] * vj.x);
                t[1] += a * (rj.y - al[1] * vj.y);
            }
            const int rm = row_mask(V, i);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (!run[c]) continue;
                const double si = V.r[2 * i + c] - al[c] * vw[2 * i + c];
                if (rm & (1 << c)) t[c] = V.dinv[i] * si;
                V.s[2 * i + c] = si;
                V.t[2 * i + c] = t[c];
                acc[c][0] += t[c] * si;
                acc[c][1] += t[c] * t[c];
                acc[c][2] += V.rh[2 * i + c] * t[c];
                acc[c][3] += V.rh[2 * i + c] * si;
            }
        }
    }
    block_partials(acc, V.part2, blockIdx.x);
}

struct MomKernels {
    void (*start)(Vecs);
    void (*ha)(Vecs, int);
    void (*hb)(Vecs, int);
};
template <int W>
MomKernels mom_kernels() {
    return {k_mom_start<W>, k_mom_ha<W>, k_mom_hb<W>};
}
// the ELL width of a longest row of `len` entries
int width_bin(int len) {
    for (int w : {7, 8, 12, 16, 24})
        if (len <= w) return w;
    return MAX_ROW;
}
MomKernels pick_kernels(int width) {
    switch (width) {
    case 7: return mom_kernels<7>();
    case 8: return mom_kernels<8>();
    case 12: return mom_kernels<12>();
    case 16: return mom_kernels<16>();
    case 24: return mom_kernels<24>();
    default: return mom_kernels<MAX_ROW>();
    }
}

__global__ void k_mom_reset(int32_t *state) {
    if (threadIdx.x < 4) {   // both copies, both components
        state[threadIdx.x * NSTATE + ST_STATUS] = -1;
        state[threadIdx.x * NSTATE + ST_ITERS] = 0;
    }
}

MomentumWork &momentum_work(hipStream_t s, Mesh &m) {
    Level &L = m.lv[m.k];
    if (!m.mom) {
        auto w = std::make_unique<MomentumWork>();
        w->n = L.n;
        const size_t n = static_cast<size_t>(L.n);
        // the mesh's adjacency and coordinates on the host
        DBuf<int32_t> mptr, mcol;
        level_adjacency(s, L, mptr, mcol, w->nnz);
        std::vector<int32_t> hp(n + 1), hc(static_cast<size_t>(w->nnz));
        std::vector<double> hxy(2 * n);
        CGP_HIP(hipMemcpyAsync(hp.data(), mptr.p, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CGP_HIP(hipMemcpyAsync(hc.data(), mcol.p, hc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CGP_HIP(hipMemcpyAsync(hxy.data(), L.xy.p, hxy.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        CGP_HIP(hipStreamSynchronize(s));
        int width = 1;
        for (size_t i = 0; i < n; ++i) width = std::max(width, hp[i + 1] - hp[i]);
        if (width > MAX_ROW) throw Error{CGP_E_UNSUPPORTED, "a node has more than 32 neighbours"};
        // own numbering: the nodes sorted along a Z curve of 2^20 x 2^20 cells of the bounding box
        double x0 = hxy[0], x1 = hxy[0], y0 = hxy[1], y1 = hxy[1];
        for (size_t i = 0; i < n; ++i) {
            x0 = std::min(x0, hxy[2 * i]);
            x1 = std::max(x1, hxy[2 * i]);
            y0 = std::min(y0, hxy[2 * i + 1]);
            y1 = std::max(y1, hxy[2 * i + 1]);
        }
        const double sx = x1 > x0 ? 1048575.0 / (x1 - x0) : 0.0, sy = y1 > y0 ? 1048575.0 / (y1 - y0) : 0.0;
        std::vector<uint64_t> code(n);
        for (size_t i = 0; i < n; ++i) {
            const uint64_t cx = static_cast<uint64_t>((hxy[2 * i] - x0) * sx);
            const uint64_t cy = static_cast<uint64_t>((hxy[2 * i + 1] - y0) * sy);
            uint64_t z = 0;
            for (int bit = 0; bit < 20; ++bit) z |= ((cx >> bit) & 1) << (2 * bit) | ((cy >> bit) & 1) << (2 * bit + 1);
            code[i] = z;
        }
        std::vector<int32_t> perm(n), inv(n);
        for (size_t i = 0; i < n; ++i) perm[i] = static_cast<int32_t>(i);
        std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return code[a] < code[b]; });
        for (size_t i = 0; i < n; ++i) inv[perm[i]] = static_cast<int32_t>(i);
        // the pattern in the own numbering (rows sorted)
        std::vector<int32_t> np(n + 1, 0), nc(hc.size());
        for (size_t i = 0; i < n; ++i) np[i + 1] = np[i] + (hp[perm[i] + 1] - hp[perm[i]]);
        for (size_t i = 0; i < n; ++i) {
            const int32_t o = perm[i];
            int32_t *dst = &nc[np[i]];
            for (int32_t q = hp[o]; q < hp[o + 1]; ++q) dst[q - hp[o]] = inv[hc[q]];
            std::sort(dst, dst + (hp[o + 1] - hp[o]));
        }
        w->ptr.alloc(n + 1);
        w->col.alloc(nc.size());
        w->perm.alloc(n);
        w->inv.alloc(n);
        CGP_HIP(hipMemcpyAsync(w->ptr.p, np.data(), np.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        CGP_HIP(hipMemcpyAsync(w->col.p, nc.data(), nc.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        CGP_HIP(hipMemcpyAsync(w->perm.p, perm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
        CGP_HIP(hipMemcpyAsync(w->inv.p, inv.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
        CGP_HIP(hipStreamSynchronize(s));
        w->rowmask.alloc(n);
        w->x.alloc(2 * n);
        w->width = width_bin(width);
        width = w->width;
        w->ecol.alloc(static_cast<size_t>(width) * n);
        hipLaunchKernelGGL(k_mom_ell, dim3(blocks_for(L.n, 256)), dim3(256), 0, s, L.n, width, w->ptr.p, w->col.p,
                           w->ecol.p);
        CGP_HIP(hipGetLastError());
        w->val.alloc(static_cast<size_t>(width) * n);
        w->dinv.alloc(n);
        w->b.alloc(2 * n);
        w->r.alloc(2 * n);
        w->rh.alloc(2 * n);
        w->p.alloc(4 * n);
        w->v.alloc(4 * n);
        w->s.alloc(2 * n);
        w->t.alloc(2 * n);
        w->part.alloc(3 * 2 * MQ * MG);
        w->scal.alloc(2 * NS);
        w->state.alloc(2 * 2 * NSTATE);
        m.mom = std::move(w);
    }
    return *m.mom;
}

}  // namespace

void momentum_step(hipStream_t s, Mesh &m, const double *un, const double *vn, const double *fx,
                   const double *fy, const uint8_t *mask, double rho, double mu, double dt, double tol, int max_iter, double *ut,
                   double *vt, cgp_momentum_stats *stats) {
    Level &L = m.lv[m.k];
    MomentumWork &w = momentum_work(s, m);
    const int64_t n = L.n;
    hipLaunchKernelGGL(k_mom_assemble, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, w.width, w.ecol.p, w.perm.p,
                       w.inv.p, L.ne_ptr.p, L.ne_idx.p, L.tri.p, L.xy.p, mask ? mask : L.dir.p, mask ? 0 : 1,
                       w.rowmask.p, un, vn, fx, fy, ut, vt, rho, mu, dt, w.val.p, w.dinv.p, w.b.p);
    hipLaunchKernelGGL(k_mom_gather, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, w.perm.p, ut, vt, w.x.p);
    Vecs V{};
    V.n = n;
    V.width = w.width;
    V.col = w.ecol.p;
    V.val = w.val.p;
    V.dinv = w.dinv.p;
    V.b = w.b.p;
    V.mask = w.rowmask.p;
    V.x[0] = w.x.p;
    V.x[1] = w.x.p + n;
    V.r = w.r.p;
    V.rh = w.rh.p;
    V.p = w.p.p;
    V.v = w.v.p;
    V.s = w.s.p;
    V.t = w.t.p;
    V.part1 = w.part.p;
    V.part2 = w.part.p + 2 * MQ * MG;
    V.part3 = w.part.p + 4 * MQ * MG;
    V.scal = w.scal.p;
    V.state = w.state.p;
    V.tol = tol;
    V.max_iter = max_iter;
    hipLaunchKernelGGL(k_mom_reset, dim3(1), dim3(64), 0, s, w.state.p);
    const MomKernels K = pick_kernels(w.width);
    hipLaunchKernelGGL(K.start, dim3(MG), dim3(MB), 0, s, V);
    CGP_HIP(hipGetLastError());
    int32_t hs[2 * NSTATE] = {-1, 0, -1, 0};
    // HA and HB of iteration max_iter + 1 only finish iteration max_iter and record the
    // outcome; the host looks at the status (the copy HB writes) every 32 iterations, and
    // every CHECK_EVERY from shortly before the iteration count of the previous call (the
    // kernels of a finished component do nothing)
    for (int it = 1; it <= max_iter + 1; ++it) {
        hipLaunchKernelGGL(K.ha, dim3(MG), dim3(MB), 0, s, V, it);
        hipLaunchKernelGGL(K.hb, dim3(MG), dim3(MB), 0, s, V, it);
        CGP_HIP(hipGetLastError());
        const bool near = it + CHECK_EVERY > w.last_iters;
        if ((near ? it % CHECK_EVERY : it % 32) == 0 || it == max_iter + 1) {
            CGP_HIP(hipMemcpyAsync(hs, w.state.p, sizeof(hs), hipMemcpyDeviceToHost, s));
            CGP_HIP(hipStreamSynchronize(s));
            if (hs[ST_STATUS] >= 0 && hs[NSTATE + ST_STATUS] >= 0) break;
        }
    }
    hipLaunchKernelGGL(k_mom_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, w.perm.p, w.x.p, ut, vt);
    CGP_HIP(hipGetLastError());
    w.last_iters = std::max(hs[ST_ITERS], hs[NSTATE + ST_ITERS]);
    double sc[2 * NS];
    CGP_HIP(hipMemcpyAsync(sc, w.scal.p, sizeof(sc), hipMemcpyDeviceToHost, s));
    CGP_HIP(hipStreamSynchronize(s));
    if (stats) {
        for (int c = 0; c < 2; ++c) {
            stats->iters[c] = hs[c * NSTATE + ST_ITERS];
            stats->status[c] = hs[c * NSTATE + ST_STATUS] < 0 ? CGP_SOLVE_ABORTED : hs[c * NSTATE + ST_STATUS];
            const double bb = sc[c * NS + S_BB], rr = sc[c * NS + S_RR];
            stats->rel_res[c] = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
        }
    }
    for (int c = 0; c < 2; ++c) {
        if (hs[c * NSTATE + ST_STATUS] == CGP_SOLVE_NOCONV) throw Error{CGP_E_NOCONV, "momentum step did not converge"};
        if (hs[c * NSTATE + ST_STATUS] == CGP_SOLVE_BREAKDOWN) throw Error{CGP_E_BREAKDOWN, "momentum step broke down"};
        if (hs[c * NSTATE + ST_STATUS] < 0) throw Error{CGP_E_ABORTED, "momentum step did not finish"};
    }
}

}  // namespace cgp
