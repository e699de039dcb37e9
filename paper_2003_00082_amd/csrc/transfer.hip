// Two-grid transfer work of a CGP step (Section 2.2, steps 1, 3, 5, 7 and the
// source of step 4):
//   k_restrict_source  injection of the fine velocity (Eq. 19) fused with the
//                      assembly of the coarse right-hand side of Eq. 12 / Eq. 15
//   k_prolong_level    P1 prolongation from one level to the next (Eq. 20)
//   k_lorentz          nodal grad(phi_f) and the Lorentz source of Eqs. 13-14
//   k_velocity         nodal grad(p_f) and the velocity correction of Eqs. 16-17
//
// All four are per-node gathers over the node->triangle incidence lists
// (ascending triangle id), one thread per node: no atomics, deterministic.
// They are HBM-bound streaming kernels (coordinates, connectivity and fields
// read once per incident triangle from L2).
#include "cgp_internal.hpp"

namespace cgp {
namespace {

constexpr int TPB = 256;

// b_i = -scale/3 * sum_{e ni i} q_e A_e with q_e the element-constant curl or
// divergence of the P1 interpolant.  With beta_a = (y_b - y_c, x_c - x_b)
// (cyclic) and D_e = 2 A_e, grad(psi_a) = beta_a / D_e, so
//   curl_e A_e = 1/2 sum_a (v_a beta_a.x - u_a beta_a.y)
//   div_e  A_e = 1/2 sum_a (u_a beta_a.x + v_a beta_a.y)
// and the element area cancels.
__global__ __launch_bounds__(TPB) void k_restrict_source(
    int64_t n, const int32_t *__restrict__ ne_ptr, const int32_t *__restrict__ ne_idx,
    const int32_t *__restrict__ tri, const double *__restrict__ xy, const uint8_t *__restrict__ dir,
    const double *__restrict__ uf, const double *__restrict__ vf, int kind, double scale,
    double *__restrict__ b, double *__restrict__ uc, double *__restrict__ vc) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (uc) uc[i] = uf[i];   // coarse node i is fine node i (hierarchical numbering)
    if (vc) vc[i] = vf[i];
    if (dir[i]) {
        b[i] = 0.0;
        return;
    }
    double acc = 0.0;
    for (int32_t k = ne_ptr[i]; k < ne_ptr[i + 1]; ++k) {
        const int64_t e = ne_idx[k];
        const int32_t a0 = tri[3 * e], a1 = tri[3 * e + 1], a2 = tri[3 * e + 2];
        const double x0 = xy[2 * a0], y0 = xy[2 * a0 + 1];
        const double x1 = xy[2 * a1], y1 = xy[2 * a1 + 1];
        const double x2 = xy[2 * a2], y2 = xy[2 * a2 + 1];
        const double bx0 = y1 - y2, bx1 = y2 - y0, bx2 = y0 - y1;
        const double by0 = x2 - x1, by1 = x0 - x2, by2 = x1 - x0;
        const double u0 = uf[a0], u1 = uf[a1], u2 = uf[a2];
        const double v0 = vf[a0], v1 = vf[a1], v2 = vf[a2];
        double qa;
        if (kind == CGP_SRC_CURL)
            qa = (v0 * bx0 + v1 * bx1 + v2 * bx2) - (u0 * by0 + u1 * by1 + u2 * by2);
        else
            qa = (u0 * bx0 + u1 * bx1 + u2 * bx2) + (v0 * by0 + v1 * by1 + v2 * by2);
        acc += 0.5 * qa;
    }
    b[i] = -scale * acc / 3.0;
}

// level l -> l+1: kept nodes copy, midpoint N_l + e of edge (a, b) = (q_a + q_b) * 0.5
__global__ __launch_bounds__(TPB) void k_prolong_level(int64_t n, int64_t E, const int32_t *__restrict__ ends,
                                                       const double *__restrict__ q, double *__restrict__ qf) {
    const int64_t id = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id < n) {
        qf[id] = q[id];
    } else if (id < n + E) {
        const int64_t e = id - n;
        qf[id] = (q[ends[2 * e]] + q[ends[2 * e + 1]]) * 0.5;
    }
}

// nodal gradient G_i = sum_e A_e g_e / sum_e A_e over the triangles around i, with
// A_e g_e = 1/2 sum_a phi_a beta_a
__device__ inline void nodal_gradient(int64_t i, const int32_t *__restrict__ ne_ptr,
                                      const int32_t *__restrict__ ne_idx, const int32_t *__restrict__ tri,
                                      const double *__restrict__ xy, const double *__restrict__ phi, double &Gx,
                                      double &Gy) {
    double gx = 0.0, gy = 0.0, area = 0.0;
    for (int32_t k = ne_ptr[i]; k < ne_ptr[i + 1]; ++k) {
        const int64_t e = ne_idx[k];
        const int32_t a0 = tri[3 * e], a1 = tri[3 * e + 1], a2 = tri[3 * e + 2];
        const double x0 = xy[2 * a0], y0 = xy[2 * a0 + 1];
        const double x1 = xy[2 * a1], y1 = xy[2 * a1 + 1];
        const double x2 = xy[2 * a2], y2 = xy[2 * a2 + 1];
        const double p0 = phi[a0], p1 = phi[a1], p2 = phi[a2];
        gx += 0.5 * (p0 * (y1 - y2) + p1 * (y2 - y0) + p2 * (y0 - y1));
        gy += 0.5 * (p0 * (x2 - x1) + p1 * (x0 - x2) + p2 * (x1 - x0));
        area += 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
    }
    Gx = gx / area;
    Gy = gy / area;
}

// F = sigma B0 (-G_y - B0 u, G_x - B0 v)
__global__ __launch_bounds__(TPB) void k_lorentz(
    int64_t n, const int32_t *__restrict__ ne_ptr, const int32_t *__restrict__ ne_idx,
    const int32_t *__restrict__ tri, const double *__restrict__ xy, const double *__restrict__ phi,
    const double *__restrict__ u, const double *__restrict__ v, double sigma, double b0,
    double *__restrict__ fx, double *__restrict__ fy) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double gx, gy;
    nodal_gradient(i, ne_ptr, ne_idx, tri, xy, phi, gx, gy);
    fx[i] = sigma * b0 * (-gy - b0 * u[i]);
    fy[i] = sigma * b0 * (gx - b0 * v[i]);
}

// u = ut - scale G_x, v = vt - scale G_y (scale = dt / rho); u may alias ut and v vt,
// since thread i reads and writes only entry i of them
__global__ __launch_bounds__(TPB) void k_velocity(
    int64_t n, const int32_t *__restrict__ ne_ptr, const int32_t *__restrict__ ne_idx,
    const int32_t *__restrict__ tri, const double *__restrict__ xy, const double *__restrict__ p,
    const double *ut, const double *vt, const uint8_t *mask, double scale, double *u, double *v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double gx, gy;
    nodal_gradient(i, ne_ptr, ne_idx, tri, xy, p, gx, gy);
    const double a = ut[i], b = vt[i];
    const int m = mask ? mask[i] : 0;
    u[i] = (m & 1) ? a : a - scale * gx;
    v[i] = (m & 2) ? b : b - scale * gy;
}

// The nodal gradient as an operator (built once per mesh): node i's vertices of its
// incident triangles, ascending and unique, and their weights in G_i = sum_e A_e g_e /
// sum_e A_e with A_e g_e = 1/2 sum_a q_a beta_a.
__device__ inline int grad_vertices(int64_t i, const int32_t *__restrict__ ne_ptr, const int32_t *__restrict__ ne_idx,
                                    const int32_t *__restrict__ tri, int32_t (&ids)[GRAD_MAX_W]) {
    int cnt = 0;
    for (int32_t k = ne_ptr[i]; k < ne_ptr[i + 1]; ++k) {
        const int64_t e = ne_idx[k];
        for (int a = 0; a < 3; ++a) {
            const int32_t v = tri[3 * e + a];
            int p = 0;
            while (p < cnt && ids[p] < v) ++p;
            if (p < cnt && ids[p] == v) continue;
            if (cnt == GRAD_MAX_W) return -1;
            for (int q = cnt; q > p; --q) ids[q] = ids[q - 1];
            ids[p] = v;
            ++cnt;
        }
    }
    return cnt;
}

__global__ __launch_bounds__(TPB) void k_grad_count(int64_t n, const int32_t *__restrict__ ne_ptr,
                                                    const int32_t *__restrict__ ne_idx,
                                                    const int32_t *__restrict__ tri, int32_t *wmax) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t ids[GRAD_MAX_W];
    const int cnt = grad_vertices(i, ne_ptr, ne_idx, tri, ids);
    atomicMax(wmax, cnt < 0 ? GRAD_MAX_W + 1 : cnt);
}

__global__ __launch_bounds__(TPB) void k_grad_fill(int64_t n, int W, const int32_t *__restrict__ ne_ptr,
                                                   const int32_t *__restrict__ ne_idx,
                                                   const int32_t *__restrict__ tri, const double *__restrict__ xy,
                                                   int32_t *__restrict__ col, double *__restrict__ cx,
                                                   double *__restrict__ cy) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t ids[GRAD_MAX_W];
    double wx[GRAD_MAX_W], wy[GRAD_MAX_W];
    const int cnt = grad_vertices(i, ne_ptr, ne_idx, tri, ids);   // <= W (counted before)
    for (int p = 0; p < GRAD_MAX_W; ++p) wx[p] = wy[p] = 0.0;
    double area = 0.0;
    for (int32_t k = ne_ptr[i]; k < ne_ptr[i + 1]; ++k) {
        const int64_t e = ne_idx[k];
        const int32_t a0 = tri[3 * e], a1 = tri[3 * e + 1], a2 = tri[3 * e + 2];
        const double x0 = xy[2 * a0], y0 = xy[2 * a0 + 1];
        const double x1 = xy[2 * a1], y1 = xy[2 * a1 + 1];
        const double x2 = xy[2 * a2], y2 = xy[2 * a2 + 1];
        const int32_t vs[3] = {a0, a1, a2};
        const double bx[3] = {y1 - y2, y2 - y0, y0 - y1}, by[3] = {x2 - x1, x0 - x2, x1 - x0};
        for (int a = 0; a < 3; ++a) {
            int p = 0;
            while (ids[p] != vs[a]) ++p;
            wx[p] += 0.5 * bx[a];
            wy[p] += 0.5 * by[a];
        }
        area += 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
    }
    // the node's own entry is left out: every row of the operator sums to zero (a constant has
    // no gradient), so G_i q = sum_j c_ij (q_j - q_i) over the other vertices
    int q = 0;
    for (int p = 0; p < cnt; ++p) {
        if (ids[p] == i) continue;
        col[static_cast<int64_t>(q) * n + i] = ids[p];
        cx[static_cast<int64_t>(q) * n + i] = wx[p] / area;
        cy[static_cast<int64_t>(q) * n + i] = wy[p] / area;
        ++q;
    }
    for (; q < W; ++q) {   // padding: the node itself, coefficient 0
        col[static_cast<int64_t>(q) * n + i] = static_cast<int32_t>(i);
        cx[static_cast<int64_t>(q) * n + i] = 0.0;
        cy[static_cast<int64_t>(q) * n + i] = 0.0;
    }
}

// G_i from the operator (coalesced column-major entries of the other vertices, gathered q):
// sum_j c_ij (q_j - q_i).  WT > 0: the operator's width, every load of the row issued before
// the first is used; 0: the width W at run time.
template <int WT>
__device__ inline void grad_apply(int64_t i, int64_t n, int W, const int32_t *__restrict__ col,
                                  const double *__restrict__ cx, const double *__restrict__ cy,
                                  const double *__restrict__ q, double &gx, double &gy) {
    const double qi = q[i];
    gx = 0.0;
    gy = 0.0;
    if constexpr (WT > 0) {
        int32_t c[WT];
        double a[WT], b[WT], qj[WT];
#pragma unroll
        for (int p = 0; p < WT; ++p) {
            const int64_t o = static_cast<int64_t>(p) * n + i;
            c[p] = col[o];
            a[p] = cx[o];
            b[p] = cy[o];
        }
#pragma unroll
        for (int p = 0; p < WT; ++p) qj[p] = q[c[p]];
#pragma unroll
        for (int p = 0; p < WT; ++p) {
            const double d = qj[p] - qi;
            gx += a[p] * d;
            gy += b[p] * d;
        }
    } else {
        for (int p = 0; p < W; ++p) {
            const int64_t o = static_cast<int64_t>(p) * n + i;
            const double d = q[col[o]] - qi;
            gx += cx[o] * d;
            gy += cy[o] * d;
        }
    }
}

template <int WT>
__global__ __launch_bounds__(TPB) void k_lorentz_op(int64_t n, int W, const int32_t *__restrict__ col,
                                                    const double *__restrict__ cx, const double *__restrict__ cy,
                                                    const double *__restrict__ phi, const double *__restrict__ u,
                                                    const double *__restrict__ v, double sigma, double b0,
                                                    double *__restrict__ fx, double *__restrict__ fy) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double gx, gy;
    grad_apply<WT>(i, n, W, col, cx, cy, phi, gx, gy);
    fx[i] = sigma * b0 * (-gy - b0 * u[i]);
    fy[i] = sigma * b0 * (gx - b0 * v[i]);
}

// u may alias ut and v vt (thread i reads and writes only entry i of them)
template <int WT>
__global__ __launch_bounds__(TPB) void k_velocity_op(int64_t n, int W, const int32_t *__restrict__ col,
                                                     const double *__restrict__ cx, const double *__restrict__ cy,
                                                     const double *__restrict__ p, const double *ut,
                                                     const double *vt, const uint8_t *mask, double scale,
                                                     double *u, double *v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double gx, gy;
    grad_apply<WT>(i, n, W, col, cx, cy, p, gx, gy);
    const double a = ut[i], b = vt[i];
    const int m = mask ? mask[i] : 0;
    u[i] = (m & 1) ? a : a - scale * gx;
    v[i] = (m & 2) ? b : b - scale * gy;
}

constexpr int SF_BLOCK = 256;

// The force of the fluid on a body over its boundary edges (a, b, t), t the fluid triangle
// owning edge ab: -int p n ds (p linear along the edge) and int mu (grad w + grad w^T) n ds
// (t's constant gradient), n the unit normal out of the body (towards t's third vertex).
// One workgroup, the edges strided over its threads, a fixed-order reduction: out[0..1]
// pressure, out[2..3] viscous, out[4] the number of edges skipped (an index out of range,
// or a or b not a vertex of t).
__global__ __launch_bounds__(SF_BLOCK) void k_surface_force(int64_t ne, const int32_t *edges, int64_t n,
                                                            int64_t T, const int32_t *tri, const double *xy,
                                                            const double *p, const double *u, const double *v,
                                                            double mu, double *out) {
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t k = threadIdx.x; k < ne; k += SF_BLOCK) {
        const int32_t a = edges[3 * k], b = edges[3 * k + 1], t = edges[3 * k + 2];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b || t < 0 || t >= T) {
            acc[4] += 1.0;
            continue;
        }
        const int32_t v0 = tri[3 * t], v1 = tri[3 * t + 1], v2 = tri[3 * t + 2];
        const int ha = (v0 == a) + (v1 == a) + (v2 == a), hb = (v0 == b) + (v1 == b) + (v2 == b);
        if (ha != 1 || hb != 1) {
            acc[4] += 1.0;
            continue;
        }
        const int32_t c = v0 != a && v0 != b ? v0 : (v1 != a && v1 != b ? v1 : v2);
        const double ax = xy[2 * a], ay = xy[2 * a + 1];
        const double dx = xy[2 * b] - ax, dy = xy[2 * b + 1] - ay;
        const double len = sqrt(dx * dx + dy * dy);
        double nx = dy / len, ny = -dx / len;
        if ((xy[2 * c] - ax) * nx + (xy[2 * c + 1] - ay) * ny < 0.0) {
            nx = -nx;
            ny = -ny;
        }
        const double pm = 0.5 * (p[a] + p[b]);
        acc[0] -= pm * nx * len;
        acc[1] -= pm * ny * len;
        // the triangle's constant gradients of u and v
        const double x0 = xy[2 * v0], y0 = xy[2 * v0 + 1], x1 = xy[2 * v1], y1 = xy[2 * v1 + 1];
        const double x2 = xy[2 * v2], y2 = xy[2 * v2 + 1];
        const double d = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
        const double ux = (u[v0] * (y1 - y2) + u[v1] * (y2 - y0) + u[v2] * (y0 - y1)) / d;
        const double uy = (u[v0] * (x2 - x1) + u[v1] * (x0 - x2) + u[v2] * (x1 - x0)) / d;
        const double vx = (v[v0] * (y1 - y2) + v[v1] * (y2 - y0) + v[v2] * (y0 - y1)) / d;
        const double vy = (v[v0] * (x2 - x1) + v[v1] * (x0 - x2) + v[v2] * (x1 - x0)) / d;
        const double sxy = uy + vx;
        acc[2] += mu * (2.0 * ux * nx + sxy * ny) * len;
        acc[3] += mu * (sxy * nx + 2.0 * vy * ny) * len;
    }
    __shared__ double red[SF_BLOCK / 64][5];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        double x = acc[q];
        for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
        if (lane == 0) red[wave][q] = x;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double x = 0.0;
        for (int w = 0; w < SF_BLOCK / 64; ++w) x += red[w][threadIdx.x];
        out[threadIdx.x] = x;
    }
}

// element gradient g_e = sum_a phi_a beta_a / D_e
__global__ __launch_bounds__(TPB) void k_elem_grad(int64_t T, const int32_t *__restrict__ tri,
                                                   const double *__restrict__ xy, const double *__restrict__ phi,
                                                   double *__restrict__ g) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= T) return;
    const int32_t a0 = tri[3 * e], a1 = tri[3 * e + 1], a2 = tri[3 * e + 2];
    const double x0 = xy[2 * a0], y0 = xy[2 * a0 + 1];
    const double x1 = xy[2 * a1], y1 = xy[2 * a1 + 1];
    const double x2 = xy[2 * a2], y2 = xy[2 * a2 + 1];
    const double p0 = phi[a0], p1 = phi[a1], p2 = phi[a2];
    const double d = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
    g[2 * e] = (p0 * (y1 - y2) + p1 * (y2 - y0) + p2 * (y0 - y1)) / d;
    g[2 * e + 1] = (p0 * (x2 - x1) + p1 * (x0 - x2) + p2 * (x1 - x0)) / d;
}

}  // namespace

void launch_restrict(hipStream_t s, const Mesh &m, const double *uf, const double *vf, int kind,
                     double scale, double *b, double *uc, double *vc) {
    const Level &L = m.lv[0];
    hipLaunchKernelGGL(k_restrict_source, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, L.ne_ptr.p,
                       L.ne_idx.p, L.tri.p, L.xy.p, L.dir.p, uf, vf, kind, scale, b, uc, vc);
    CGP_HIP(hipGetLastError());
}

void launch_prolong(hipStream_t s, Mesh &m, const double *qc, double *qf) {
    if (m.k == 0) {
        CGP_HIP(hipMemcpyAsync(qf, qc, m.lv[0].n * sizeof(double), hipMemcpyDeviceToDevice, s));
        return;
    }
    const double *src = qc;
    for (int32_t l = 0; l < m.k; ++l) {
        const Level &L = m.lv[l];
        double *dst = (l + 1 == m.k) ? qf : m.lv[l + 1].tmp.p;
        hipLaunchKernelGGL(k_prolong_level, dim3(blocks_for(L.n + L.E, TPB)), dim3(TPB), 0, s, L.n, L.E,
                           L.ends.p, src, dst);
        CGP_HIP(hipGetLastError());
        src = dst;
    }
}

// builds the nodal-gradient operator of the finest level on first use (unless `build` is
// false: inside a stream capture); false when it is not there or a node has more than
// GRAD_MAX_W neighbours (the per-triangle kernels are used then)
bool nodal_grad(hipStream_t s, Mesh &m, bool build) {
    NodalGrad &G = m.grad;
    if (G.W == 0 && build) {
        const Level &L = m.lv[m.k];
        DBuf<int32_t> w;
        w.alloc(1);
        CGP_HIP(hipMemsetAsync(w.p, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_grad_count, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, L.ne_ptr.p, L.ne_idx.p,
                           L.tri.p, w.p);
        CGP_HIP(hipGetLastError());
        int32_t W = 0;
        CGP_HIP(hipMemcpyAsync(&W, w.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CGP_HIP(hipStreamSynchronize(s));
        // W counts the node itself, which the operator leaves out; widths up to 6 and 8 are padded
        // to those (the unrolled kernels)
        W -= 1;
        if (W > 0 && W <= 6) W = 6;
        else if (W > 6 && W <= 8) W = 8;
        if (W > GRAD_MAX_W || W < 1) {
            G.W = -1;
        } else {
            G.col.alloc(static_cast<size_t>(W) * L.n);
            G.cx.alloc(static_cast<size_t>(W) * L.n);
            G.cy.alloc(static_cast<size_t>(W) * L.n);
            hipLaunchKernelGGL(k_grad_fill, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, W, L.ne_ptr.p,
                               L.ne_idx.p, L.tri.p, L.xy.p, G.col.p, G.cx.p, G.cy.p);
            CGP_HIP(hipGetLastError());
            G.W = W;
        }
    }
    return G.W > 0;
}

void launch_lorentz(hipStream_t s, Mesh &m, const double *phif, const double *uf, const double *vf,
                    double sigma, double b0, double *fx, double *fy, double *grad_elem, bool build) {
    const Level &L = m.lv[m.k];
    if (nodal_grad(s, m, build)) {
#define CGP_LORENTZ(WT)                                                                                     \
    hipLaunchKernelGGL(k_lorentz_op<WT>, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, m.grad.W,      \
                       m.grad.col.p, m.grad.cx.p, m.grad.cy.p, phif, uf, vf, sigma, b0, fx, fy)
        if (m.grad.W == 6)
            CGP_LORENTZ(6);
        else if (m.grad.W == 8)
            CGP_LORENTZ(8);
        else
            CGP_LORENTZ(0);
#undef CGP_LORENTZ
    } else
        hipLaunchKernelGGL(k_lorentz, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, L.ne_ptr.p, L.ne_idx.p,
                           L.tri.p, L.xy.p, phif, uf, vf, sigma, b0, fx, fy);
    CGP_HIP(hipGetLastError());
    if (grad_elem) {
        hipLaunchKernelGGL(k_elem_grad, dim3(blocks_for(L.T, TPB)), dim3(TPB), 0, s, L.T, L.tri.p, L.xy.p,
                           phif, grad_elem);
        CGP_HIP(hipGetLastError());
    }
}

void launch_velocity(hipStream_t s, Mesh &m, const double *pf, const double *ut, const double *vt,
                     const uint8_t *mask, double scale, double *u, double *v, bool build) {
    const Level &L = m.lv[m.k];
    if (nodal_grad(s, m, build)) {
#define CGP_VELOCITY(WT)                                                                                    \
    hipLaunchKernelGGL(k_velocity_op<WT>, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, m.grad.W,     \
                       m.grad.col.p, m.grad.cx.p, m.grad.cy.p, pf, ut, vt, mask, scale, u, v)
        if (m.grad.W == 6)
            CGP_VELOCITY(6);
        else if (m.grad.W == 8)
            CGP_VELOCITY(8);
        else
            CGP_VELOCITY(0);
#undef CGP_VELOCITY
    } else
        hipLaunchKernelGGL(k_velocity, dim3(blocks_for(L.n, TPB)), dim3(TPB), 0, s, L.n, L.ne_ptr.p, L.ne_idx.p,
                           L.tri.p, L.xy.p, pf, ut, vt, mask, scale, u, v);
    CGP_HIP(hipGetLastError());
}

void launch_surface_force(hipStream_t s, Mesh &m, int level, int64_t n_edges, const int32_t *edges,
                          const double *p, const double *u, const double *v, double mu, double *out) {
    const Level &L = m.lv[level];
    hipLaunchKernelGGL(k_surface_force, dim3(1), dim3(SF_BLOCK), 0, s, n_edges, edges, L.n, L.T, L.tri.p, L.xy.p,
                       p, u, v, mu, out);
    CGP_HIP(hipGetLastError());
}

}  // namespace cgp
