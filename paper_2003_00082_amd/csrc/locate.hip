// P1 interpolation of a level's field at arbitrary points (the general restriction of
// Section 2.3 for a coarse mesh that is not nested in the fine one: every coarse node is
// located in a fine triangle and the fine field evaluated there).
//
// Location: a uniform grid over the level's bounding box, cells of about two triangles'
// size, each listing the triangles whose bounding box (widened by a relative 1e-9)
// overlaps it, built once per level on the host (CSR; an entry is the triangle's id and its
// three node ids in one 16-byte record, so that a candidate costs one load before its
// coordinates).  A group of lanes per point tests its
// cell's triangles and keeps the one with the largest smallest barycentric coordinate (the
// lowest id on a tie); the point is inside when that coordinate is >= -1e-12.
// A triangle that contains the point overlaps the point's cell, so the scan is exact.
#include <algorithm>
#include <cmath>

#include "cgp_internal.hpp"

namespace cgp {

namespace {

constexpr double LOC_EPS = 1e-12;    // tolerance on the barycentric coordinates
constexpr double BOX_SLACK = 1e-9;   // relative widening of the triangles' boxes when binned

constexpr int LANES = 8;               // lanes per point: each tests every LANES-th candidate
constexpr int LOC_BLOCK = 256;

// One group of LANES lanes per point.  Each lane keeps its best candidate by the order
// (smallest barycentric coordinate descending, triangle id ascending); the order is total, so
// the butterfly over the group gives every lane the same winner as a serial scan would.
__global__ __launch_bounds__(LOC_BLOCK) void k_interpolate(int64_t np, const double *pts, const double *xy,
                                                           Locator L, const double *field,
                                                           double *out, int32_t *tri_out) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * LOC_BLOCK + threadIdx.x;
    const int64_t q = gid / LANES;
    const int lane = static_cast<int>(gid % LANES);
    const bool valid = q < np;
    int32_t best = -1;
    double bl0 = 0.0, bl1 = 0.0, bl2 = 0.0, bmin = -INFINITY;
    int32_t bv0 = 0, bv1 = 0, bv2 = 0;   // the best triangle's nodes
    if (valid) {
        const double px = pts[2 * q], py = pts[2 * q + 1];
        const double fx = (px - L.x0) / L.h, fy = (py - L.y0) / L.h;
        if (fx >= -1.0 && fy >= -1.0 && fx <= L.gx + 1.0 && fy <= L.gy + 1.0) {
            const int cx = std::min(std::max(static_cast<int>(floor(fx)), 0), L.gx - 1);
            const int cy = std::min(std::max(static_cast<int>(floor(fy)), 0), L.gy - 1);
            const int64_t c = static_cast<int64_t>(cy) * L.gx + cx;
            const int32_t end = L.cell_ptr[c + 1];
            for (int32_t k = L.cell_ptr[c] + lane; k < end; k += LANES) {
                const int4 en = reinterpret_cast<const int4 *>(L.cell_tri)[k];
                const int32_t t = en.x, a = en.y, b = en.z, d = en.w;
                const double ax = xy[2 * a], ay = xy[2 * a + 1];
                const double e1x = xy[2 * b] - ax, e1y = xy[2 * b + 1] - ay;
                const double e2x = xy[2 * d] - ax, e2y = xy[2 * d + 1] - ay;
                const double dx = px - ax, dy = py - ay;
                const double det = e1x * e2y - e1y * e2x;
                const double l1 = (dx * e2y - dy * e2x) / det, l2 = (e1x * dy - e1y * dx) / det;
                const double l0 = 1.0 - l1 - l2;
                const double m = fmin(l0, fmin(l1, l2));
                if (m > bmin || (m == bmin && t < best)) {
                    bmin = m;
                    best = t;
                    bl0 = l0;
                    bl1 = l1;
                    bl2 = l2;
                    bv0 = a;
                    bv1 = b;
                    bv2 = d;
                }
            }
        }
    }
    // every lane of the wave takes part (groups never straddle a wave: LANES divides 64)
    double wmin = bmin;
    int32_t wbest = best;
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) {
        const double om = __shfl_xor(wmin, o, LANES);
        const int32_t ob = __shfl_xor(wbest, o, LANES);
        if (ob >= 0 && (wbest < 0 || om > wmin || (om == wmin && ob < wbest))) {
            wmin = om;
            wbest = ob;
        }
    }
    if (!valid) return;
    if (wbest >= 0 && wmin >= -LOC_EPS) {
        if (best != wbest) return;   // the winner's lane writes (a triangle is listed once per cell)
        out[q] = bl0 * field[bv0] + bl1 * field[bv1] + bl2 * field[bv2];
        if (tri_out) tri_out[q] = best;
    } else if (lane == 0) {
        out[q] = NAN;
        if (tri_out) tri_out[q] = -1;
    }
}

// the bucket grid of one level, from its coordinates and triangles (host)
std::unique_ptr<LocatorData> build_locator(hipStream_t s, const Level &L) {
    std::vector<double> xy(2 * L.n);
    std::vector<int32_t> tri(3 * L.T);
    CGP_HIP(hipMemcpyAsync(xy.data(), L.xy.p, xy.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    CGP_HIP(hipMemcpyAsync(tri.data(), L.tri.p, tri.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CGP_HIP(hipStreamSynchronize(s));
    double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
    for (int64_t i = 0; i < L.n; ++i) {
        x0 = std::min(x0, xy[2 * i]);
        x1 = std::max(x1, xy[2 * i]);
        y0 = std::min(y0, xy[2 * i + 1]);
        y1 = std::max(y1, xy[2 * i + 1]);
    }
    const double w = std::max(x1 - x0, 1e-300), hgt = std::max(y1 - y0, 1e-300);
    // cells of about two triangles' area, at most ~4 M cells
    double h = std::sqrt(2.0 * w * hgt / std::max<int64_t>(L.T, 1));
    h = std::max(h, std::sqrt(w * hgt / 4.0e6));
    auto out = std::make_unique<LocatorData>();
    Locator &G = out->loc;
    G.x0 = x0;
    G.y0 = y0;
    G.h = h;
    G.gx = std::max(1, static_cast<int>(std::ceil(w / h)));
    G.gy = std::max(1, static_cast<int>(std::ceil(hgt / h)));
    const int64_t nc = static_cast<int64_t>(G.gx) * G.gy;
    std::vector<int32_t> cnt(nc + 1, 0);
    auto cells = [&](int64_t t, int &cx0, int &cx1, int &cy0, int &cy1) {
        double bx0 = INFINITY, by0 = INFINITY, bx1 = -INFINITY, by1 = -INFINITY;
        for (int a = 0; a < 3; ++a) {
            const int32_t v = tri[3 * t + a];
            bx0 = std::min(bx0, xy[2 * v]);
            bx1 = std::max(bx1, xy[2 * v]);
            by0 = std::min(by0, xy[2 * v + 1]);
            by1 = std::max(by1, xy[2 * v + 1]);
        }
        const double sx = BOX_SLACK * w + BOX_SLACK * (bx1 - bx0), sy = BOX_SLACK * hgt + BOX_SLACK * (by1 - by0);
        cx0 = std::min(std::max(static_cast<int>(std::floor((bx0 - sx - x0) / h)), 0), G.gx - 1);
        cx1 = std::min(std::max(static_cast<int>(std::floor((bx1 + sx - x0) / h)), 0), G.gx - 1);
        cy0 = std::min(std::max(static_cast<int>(std::floor((by0 - sy - y0) / h)), 0), G.gy - 1);
        cy1 = std::min(std::max(static_cast<int>(std::floor((by1 + sy - y0) / h)), 0), G.gy - 1);
    };
    for (int64_t t = 0; t < L.T; ++t) {
        int cx0, cx1, cy0, cy1;
        cells(t, cx0, cx1, cy0, cy1);
        for (int cy = cy0; cy <= cy1; ++cy)
            for (int cx = cx0; cx <= cx1; ++cx) ++cnt[static_cast<int64_t>(cy) * G.gx + cx + 1];
    }
    for (int64_t c = 0; c < nc; ++c) cnt[c + 1] += cnt[c];
    std::vector<int32_t> list(4 * static_cast<size_t>(cnt[nc]));
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t t = 0; t < L.T; ++t) {   // ascending triangle id within every cell
        int cx0, cx1, cy0, cy1;
        cells(t, cx0, cx1, cy0, cy1);
        for (int cy = cy0; cy <= cy1; ++cy)
            for (int cx = cx0; cx <= cx1; ++cx) {
                int32_t *en = &list[4 * static_cast<size_t>(fill[static_cast<int64_t>(cy) * G.gx + cx]++)];
                en[0] = static_cast<int32_t>(t);
                en[1] = tri[3 * t];
                en[2] = tri[3 * t + 1];
                en[3] = tri[3 * t + 2];
            }
    }
    out->cell_ptr.alloc(cnt.size());
    out->cell_tri.alloc(list.size());
    CGP_HIP(hipMemcpyAsync(out->cell_ptr.p, cnt.data(), cnt.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (!list.empty())
        CGP_HIP(hipMemcpyAsync(out->cell_tri.p, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    CGP_HIP(hipStreamSynchronize(s));
    G.cell_ptr = out->cell_ptr.p;
    G.cell_tri = out->cell_tri.p;
    return out;
}

}  // namespace

void interpolate_points(hipStream_t s, Mesh &m, int level, int64_t np, const double *pts, const double *field,
                        double *out, int32_t *tri_out, bool build) {
    if (m.loc.size() < m.lv.size()) m.loc.resize(m.lv.size());
    auto &slot = m.loc[level];
    if (!slot) {
        if (!build) throw Error{CGP_E_INVALID, "the point locator of this level is built outside graph capture"};
        slot = build_locator(s, m.lv[level]);
    }
    if (np == 0) return;
    const Level &L = m.lv[level];
    hipLaunchKernelGGL(k_interpolate, dim3(blocks_for(np * LANES, LOC_BLOCK)), dim3(LOC_BLOCK), 0, s, np, pts, L.xy.p,
                       slot->loc, field, out, tri_out);
    CGP_HIP(hipGetLastError());
}

}  // namespace cgp
