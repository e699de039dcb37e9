// Tiles of the coarse mesh for the tiled CG iteration (host side).
//
// Each workgroup of the tiled iteration owns a compact tile of at most 512 rows,
// cut by recursive coordinate bisection of the node coordinates, and works on
// the tile's region: the rows within graph distance d of the tile in the matrix
// graph (d = degree of the polynomial preconditioner, 1 for Jacobi), listed own
// rows first and then by distance, so that "distance <= t" is a prefix of the
// list.  A local ELL copy of the matrix rows at distance <= d - 1, with columns
// given as region indices, lets the workgroup apply the preconditioner and the
// matrix to its own rows from the region's values alone.  Its rows are records:
// the columns of local row t (16-bit, padded to 8 or 16 entries) at
// (ell_off + t) * cols_per_row, its values (width entries) at (ell_off + t) * width,
// so that a thread reads a row with a few 16-byte loads.
#include <algorithm>
#include <cmath>
#include <limits>

#include "cgp_internal.hpp"

namespace cgp {
namespace {

template <class T>
std::vector<T> d2h(hipStream_t s, const T *p, size_t n) {
    std::vector<T> h(n);
    if (n) CGP_HIP(hipMemcpyAsync(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
    CGP_HIP(hipStreamSynchronize(s));
    return h;
}

template <class T>
void h2d(hipStream_t s, DBuf<T> &d, const std::vector<T> &h) {
    d.alloc(h.size());
    if (!h.empty()) CGP_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// split ids[lo, hi) into `parts` pieces of nearly equal size, each cut across the
// longer side of the piece's bounding box; appends the end of every piece to cuts
void bisect(std::vector<int32_t> &ids, size_t lo, size_t hi, int parts, const std::vector<double> &xy,
            std::vector<size_t> &cuts) {
    if (parts <= 1) {
        cuts.push_back(hi);
        return;
    }
    double mn[2] = {std::numeric_limits<double>::infinity(), std::numeric_limits<double>::infinity()};
    double mx[2] = {-mn[0], -mn[1]};
    for (size_t q = lo; q < hi; ++q)
        for (int a = 0; a < 2; ++a) {
            const double v = xy[2 * static_cast<size_t>(ids[q]) + a];
            mn[a] = std::min(mn[a], v);
            mx[a] = std::max(mx[a], v);
        }
    const int ax = (mx[0] - mn[0] >= mx[1] - mn[1]) ? 0 : 1;
    const int pl = parts / 2;
    const size_t nl = (hi - lo) * static_cast<size_t>(pl) / static_cast<size_t>(parts);
    std::nth_element(ids.begin() + lo, ids.begin() + lo + nl, ids.begin() + hi, [&](int32_t a, int32_t b) {
        const double xa = xy[2 * static_cast<size_t>(a) + ax], xb = xy[2 * static_cast<size_t>(b) + ax];
        return xa < xb || (xa == xb && a < b);
    });
    bisect(ids, lo, lo + nl, pl, xy, cuts);
    bisect(ids, lo + nl, hi, parts - pl, xy, cuts);
}

// the tiles for `parts` pieces, or an empty plan when a region or its matrix rows
// exceed the workgroup's capacity
bool build_tiles(int64_t n, int parts, int degree, int width, const std::vector<int32_t> &rowptr,
                 const std::vector<int32_t> &col, const std::vector<double> &val, const std::vector<double> &xy,
                 std::vector<TileBlk> &blk, std::vector<int32_t> &reg, std::vector<uint16_t> &ecol,
                 std::vector<double> &eval) {
    std::vector<int32_t> ids(n);
    for (int64_t i = 0; i < n; ++i) ids[i] = static_cast<int32_t>(i);
    std::vector<size_t> cuts;
    bisect(ids, 0, static_cast<size_t>(n), parts, xy, cuts);
    std::vector<int32_t> mark(n, -1), loc(n, -1);
    blk.assign(parts, TileBlk{});
    reg.clear();
    ecol.clear();
    eval.clear();
    size_t b0 = 0;
    for (int p = 0; p < parts; ++p) {
        const size_t b1 = cuts[p];
        if (b1 - b0 > static_cast<size_t>(TILE_ROWS_MAX)) return false;
        TileBlk &B = blk[p];
        B.reg_off = static_cast<int32_t>(reg.size());
        B.ell_off = static_cast<int32_t>(eval.size() / width);
        std::vector<int32_t> list(ids.begin() + b0, ids.begin() + b1);
        std::sort(list.begin(), list.end());
        for (int32_t g : list) mark[g] = p;
        B.nt[0] = static_cast<int32_t>(list.size());
        size_t f0 = 0;
        for (int t = 1; t <= degree; ++t) {
            const size_t f1 = list.size();
            std::vector<int32_t> next;
            for (size_t q = f0; q < f1; ++q) {
                const int32_t g = list[q];
                for (int32_t k = rowptr[g]; k < rowptr[g + 1]; ++k) {
                    const int32_t j = col[k];
                    if (mark[j] != p) {
                        mark[j] = p;
                        next.push_back(j);
                    }
                }
            }
            std::sort(next.begin(), next.end());
            list.insert(list.end(), next.begin(), next.end());
            B.nt[t] = static_cast<int32_t>(list.size());
            f0 = f1;
        }
        for (int t = degree + 1; t < TILE_MAX_DEGREE + 2; ++t) B.nt[t] = B.nt[degree];
        B.kz_off = 0;
        B.nkz = 0;
        B.own_off = static_cast<int32_t>(b0);
        B.nreg = B.nt[degree];
        B.nspmv = B.nt[std::max(degree - 1, 0)];
        if (B.nreg > TILE_REGION || B.nspmv > TILE_SPMV) return false;
        for (int32_t t = 0; t < B.nreg; ++t) loc[list[t]] = t;
        const int cw = tile_col_stride(width);
        ecol.resize(ecol.size() + static_cast<size_t>(cw) * B.nspmv);
        eval.resize(eval.size() + static_cast<size_t>(width) * B.nspmv);
        for (int32_t t = 0; t < B.nspmv; ++t) {
            const int32_t g = list[t];
            const int32_t len = rowptr[g + 1] - rowptr[g];
            const size_t oc = (static_cast<size_t>(B.ell_off) + t) * cw, ov = (static_cast<size_t>(B.ell_off) + t) * width;
            for (int k = 0; k < cw; ++k) {
                if (k < len) {
                    const int32_t lc = loc[col[rowptr[g] + k]];
                    if (lc < 0) throw Error{CGP_E_HIP, "tile region misses a matrix neighbour"};
                    ecol[oc + k] = static_cast<uint16_t>(lc);
                    if (k < width) eval[ov + k] = val[rowptr[g] + k];
                } else {
                    ecol[oc + k] = static_cast<uint16_t>(t);
                    if (k < width) eval[ov + k] = 0.0;
                }
            }
        }
        for (int32_t g : list) loc[g] = -1;
        reg.insert(reg.end(), list.begin(), list.end());
        b0 = b1;
    }
    // every row owned by exactly one tile; every index inside its array
    std::vector<int32_t> owned(n, 0);
    for (const TileBlk &B : blk) {
        for (int32_t t = 0; t < B.nt[0]; ++t) ++owned[reg[static_cast<size_t>(B.reg_off) + t]];
        for (int32_t t = 0; t < B.nreg; ++t) {
            const int32_t g = reg[static_cast<size_t>(B.reg_off) + t];
            if (g < 0 || g >= n) throw Error{CGP_E_HIP, "tile region row out of range"};
        }
        const size_t cw = static_cast<size_t>(tile_col_stride(width));
        for (size_t q = 0; q < cw * B.nspmv; ++q)
            if (ecol[static_cast<size_t>(B.ell_off) * cw + q] >= B.nreg)
                throw Error{CGP_E_HIP, "tile matrix column out of range"};
    }
    for (int64_t i = 0; i < n; ++i)
        if (owned[i] != 1) throw Error{CGP_E_HIP, "tiles do not partition the rows"};
    return true;
}

// The split records of a plan built with width-8 records (tile_col_stride 8): every local row's
// entries other than its own column (the diagonal, and the padding, which names the row itself),
// in the same order.  False if a row has more than SPLIT_WIDTH of them.
bool split_records(const std::vector<TileBlk> &blk, const std::vector<uint16_t> &ecol,
                   const std::vector<double> &eval, TilePlan &plan, hipStream_t s) {
    constexpr int W = 8, SW = SPLIT_WIDTH;
    static_assert(SW % 2 == 0 && SW <= W, "split records hold pairs of entries");
    const size_t rows = eval.size() / W;
    std::vector<double> sv(rows * SW, 0.0);
    std::vector<uint32_t> sc(rows * (SW / 2), 0u);
    for (const TileBlk &B : blk) {
        const size_t ns = static_cast<size_t>(B.nspmv);
        for (size_t t = 0; t < ns; ++t) {
            const size_t r = static_cast<size_t>(B.ell_off) + t;
            uint16_t c[SW];
            double v[SW];
            int cnt = 0;
            for (int k = 0; k < W; ++k) {
                const uint16_t lc = ecol[r * tile_col_stride(W) + k];
                if (lc == t) continue;
                if (cnt == SW) return false;
                c[cnt] = lc;
                v[cnt] = eval[r * W + k];
                ++cnt;
            }
            for (; cnt < SW; ++cnt) {
                c[cnt] = static_cast<uint16_t>(t);
                v[cnt] = 0.0;
            }
            for (int q = 0; q < SW / 2; ++q) {
                const size_t vo = static_cast<size_t>(SW) * B.ell_off + 2 * (q * ns + t);
                sv[vo] = v[2 * q];
                sv[vo + 1] = v[2 * q + 1];
                sc[static_cast<size_t>(SW / 2) * B.ell_off + q * ns + t] =
                    static_cast<uint32_t>(c[2 * q]) | (static_cast<uint32_t>(c[2 * q + 1]) << 16);
            }
        }
    }
    h2d(s, plan.scol, sc);
    h2d(s, plan.sval64, sv);
    std::vector<float> s32(sv.begin(), sv.end());
    h2d(s, plan.sval32, s32);
    CGP_HIP(hipStreamSynchronize(s));
    return true;
}

}  // namespace

double mesh_gershgorin(hipStream_t s, Mesh &m) {
    if (m.gershgorin > 0.0) return m.gershgorin;
    const int64_t n = m.lv[0].n;
    const auto rowptr = d2h(s, m.rowptr.p, n + 1);
    const auto val = d2h(s, m.val.p, m.nnz);
    const auto col = d2h(s, m.col.p, m.nnz);
    double hi = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double sum = 0.0, diag = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            sum += std::fabs(val[k]);
            if (col[k] == i) diag = val[k];
        }
        if (diag > 0.0) hi = std::max(hi, sum / diag);
    }
    m.gershgorin = hi;
    return hi;
}

TilePlan *tile_plan(hipStream_t s, Mesh &m, int degree) {
    CGP_REQUIRE(degree >= 1 && degree <= TILE_MAX_DEGREE, "preconditioner degree out of range");
    if (m.tiles[degree]) return m.tiles[degree]->nparts > 0 ? m.tiles[degree].get() : nullptr;
    auto plan = std::make_unique<TilePlan>();
    TilePlan *out = nullptr;
    const int width = m.max_row <= 8 ? 8 : (m.max_row <= 12 ? 12 : 0);
    if (width > 0) {
        const int64_t n = m.lv[0].n;
        const auto rowptr = d2h(s, m.rowptr.p, n + 1);
        const auto col = d2h(s, m.col.p, m.nnz);
        const auto val = d2h(s, m.val.p, m.nnz);
        const auto xy = d2h(s, m.lv[0].xy.p, 2 * n);
        std::vector<TileBlk> blk;
        std::vector<int32_t> reg;
        std::vector<uint16_t> ecol;
        std::vector<double> eval;
        // tiles of up to TILE_ROWS rows (one own row per thread); a mesh that needs more than
        // TILE_GRID of them takes TILE_GRID larger ones while they fit a workgroup (a grid
        // just above the compute-unit count would run a few compute units two workgroups
        // deep); then more, smaller tiles until every region fits (at least 64 rows)
        int parts = static_cast<int>((n + TILE_ROWS - 1) / TILE_ROWS);
        if (parts > TILE_GRID)
            parts = std::max(TILE_GRID, static_cast<int>((n + TILE_ROWS_MAX - 1) / TILE_ROWS_MAX));
        const int max_parts = static_cast<int>((n + 63) / 64);
        bool ok = false;
        while (!ok && parts <= max_parts) {
            ok = build_tiles(n, parts, degree, width, rowptr, col, val, xy, blk, reg, ecol, eval);
            if (!ok) parts = parts + std::max(1, parts / 8);
        }
        if (ok) {
            plan->degree = degree;
            plan->width = width;
            plan->kwidth = width;
            if (m.max_row <= SPLIT_WIDTH + 1 && split_records(blk, ecol, eval, *plan, s)) plan->kwidth = SPLIT_WIDTH;
            plan->nparts = parts;
            plan->agg = AGG_TILE;
            plan->hblk = blk;
            plan->hreg = reg;
            h2d(s, plan->blk, blk);
            h2d(s, plan->reg, reg);
            h2d(s, plan->ecol, ecol);
            h2d(s, plan->eval64, eval);
            std::vector<float> e32(eval.begin(), eval.end());
            h2d(s, plan->eval32, e32);
            CGP_HIP(hipStreamSynchronize(s));
            out = plan.get();
        }
    }
    m.tiles[degree] = std::move(plan);
    return out;
}

// Deflation data of the tiled iteration.  Aggregates: every tile's own rows cut into
// P.agg parts by bisection (aggregates agg t .. agg t + agg - 1; Z: their free-row indicators).  For
// every region row that couples to an aggregate through K, a record (region index, up to
// KZ_PER_ROW aggregates, (K Z)_{row, a}); a row whose couplings cancel (an interior row:
// zero row sum) gets none.  E = Z^T K Z is inverted on the host (Cholesky), an aggregate
// without free rows getting E_aa = 1.
bool tile_deflation(hipStream_t s, Mesh &m, TilePlan &P) {
    if (P.defl_state != 0) return P.defl_state > 0;
    P.defl_state = -1;
    const int nt = P.nparts, A = P.agg, na = A * nt;
    if (na > MAX_DEFL_AGGREGATES) return false;
    const int64_t n = m.lv[0].n;
    const auto rowptr = d2h(s, m.rowptr.p, n + 1);
    const auto col = d2h(s, m.col.p, m.nnz);
    const auto val = d2h(s, m.val.p, m.nnz);
    const auto dir = d2h(s, m.lv[0].dir.p, n);
    const auto xy = d2h(s, m.lv[0].xy.p, 2 * n);
    std::vector<int32_t> agg(n, -1);
    std::vector<int8_t> oagg(P.hreg.size(), 0);
    for (int t = 0; t < nt; ++t) {
        const TileBlk &B = P.hblk[t];
        std::vector<int32_t> ids(P.hreg.begin() + B.reg_off, P.hreg.begin() + B.reg_off + B.nt[0]);
        std::vector<size_t> cuts;
        bisect(ids, 0, ids.size(), A, xy, cuts);
        size_t lo = 0;
        for (int h = 0; h < A; ++h) {
            for (size_t q = lo; q < cuts[h]; ++q)
                if (!dir[ids[q]]) agg[ids[q]] = A * t + h;
            lo = cuts[h];
        }
        for (int32_t q = 0; q < B.nt[0]; ++q) {
            const int32_t j = P.hreg[static_cast<size_t>(B.reg_off) + q];
            oagg[static_cast<size_t>(B.reg_off) + q] = agg[j] < 0 ? 0 : static_cast<int8_t>(1 + agg[j] - A * t);
        }
    }
    // coupling records
    std::vector<TileBlk> blk = P.hblk;
    std::vector<uint64_t> kzk;
    std::vector<double> kzv;
    for (int t = 0; t < nt; ++t) {
        const TileBlk &B = P.hblk[t];
        blk[t].kz_off = static_cast<int32_t>(kzk.size());
        for (int32_t q = 0; q < B.nreg; ++q) {
            const int32_t j = P.hreg[static_cast<size_t>(B.reg_off) + q];
            int32_t ids[16];
            double sums[16];
            int cnt = 0;
            double scale = 0.0;
            for (int32_t k = rowptr[j]; k < rowptr[j + 1]; ++k) {
                scale += std::fabs(val[k]);
                const int32_t a = agg[col[k]];
                if (a < 0) continue;
                int e = 0;
                while (e < cnt && ids[e] != a) ++e;
                if (e == cnt) {
                    if (cnt == 16) return false;
                    ids[cnt] = a;
                    sums[cnt] = 0.0;
                    ++cnt;
                }
                sums[e] += val[k];
            }
            // drop couplings that cancel to rounding (row sums of interior rows)
            int keep = 0;
            for (int e = 0; e < cnt; ++e)
                if (std::fabs(sums[e]) > 1e-13 * scale) {
                    ids[keep] = ids[e];
                    sums[keep] = sums[e];
                    ++keep;
                }
            if (keep == 0) continue;
            if (keep > KZ_PER_ROW) return false;
            uint64_t rec = static_cast<uint64_t>(q);
            for (int e = 0; e < KZ_PER_ROW; ++e) {
                rec |= static_cast<uint64_t>(e < keep ? ids[e] : A * t) << (KZ_BITS * (1 + e));
                kzv.push_back(e < keep ? sums[e] : 0.0);
            }
            kzk.push_back(rec);
        }
        blk[t].nkz = static_cast<int32_t>(kzk.size()) - blk[t].kz_off;
        if (blk[t].nkz > TILE_ROWS) return false;   // one record per thread
    }
    // one record past the last tile's: every thread of the stage kernel loads record
    // kz_off + min(t, nkz) (no branch around the loads) and ignores it unless t < nkz
    kzk.push_back(0);
    for (int e = 0; e < KZ_PER_ROW; ++e) kzv.push_back(0.0);
    // E = Z^T K Z and its inverse
    std::vector<double> E(static_cast<size_t>(na) * na, 0.0);
    std::vector<int32_t> nfree(na, 0);
    for (int64_t j = 0; j < n; ++j) {
        const int32_t a = agg[j];
        if (a < 0) continue;
        ++nfree[a];
        for (int32_t k = rowptr[j]; k < rowptr[j + 1]; ++k) {
            const int32_t b = agg[col[k]];
            if (b >= 0) E[static_cast<size_t>(a) * na + b] += val[k];
        }
    }
    for (int a = 0; a < na; ++a)
        if (nfree[a] == 0) E[static_cast<size_t>(a) * na + a] = 1.0;
    // Cholesky E = L L^T (lower triangle in place), then E^-1 = L^-T L^-1
    std::vector<double> L = E;
    for (int j = 0; j < na; ++j) {
        double d = L[static_cast<size_t>(j) * na + j];
        for (int k = 0; k < j; ++k) d -= L[static_cast<size_t>(j) * na + k] * L[static_cast<size_t>(j) * na + k];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        L[static_cast<size_t>(j) * na + j] = d;
        for (int i = j + 1; i < na; ++i) {
            double v = L[static_cast<size_t>(i) * na + j];
            for (int k = 0; k < j; ++k) v -= L[static_cast<size_t>(i) * na + k] * L[static_cast<size_t>(j) * na + k];
            L[static_cast<size_t>(i) * na + j] = v / d;
        }
    }
    // Li = L^-1 (lower triangular) by forward substitution, one row at a time: row i of Li is
    // (e_i - sum_{k<i} L_ik Li_k) / L_ii, the update running along contiguous rows
    std::vector<double> Li(static_cast<size_t>(na) * na, 0.0);
    for (int i = 0; i < na; ++i) {
        double *xi = &Li[static_cast<size_t>(i) * na];
        xi[i] = 1.0;
        for (int k = 0; k < i; ++k) {
            const double a = L[static_cast<size_t>(i) * na + k];
            const double *xk = &Li[static_cast<size_t>(k) * na];
            for (int c = 0; c <= k; ++c) xi[c] -= a * xk[c];
        }
        const double d = L[static_cast<size_t>(i) * na + i];
        for (int c = 0; c <= i; ++c) xi[c] /= d;
    }
    // E^-1 = Li^T Li as a sum of rank-one updates by the rows of Li (lower triangle), mirrored
    std::vector<double> Ei(static_cast<size_t>(na) * na, 0.0);
    for (int k = 0; k < na; ++k) {
        const double *lk = &Li[static_cast<size_t>(k) * na];
        for (int a = 0; a <= k; ++a) {
            const double la = lk[a];
            double *ea = &Ei[static_cast<size_t>(a) * na];
            for (int b = 0; b <= a; ++b) ea[b] += la * lk[b];
        }
    }
    for (int a = 0; a < na; ++a)
        for (int b = 0; b < a; ++b) Ei[static_cast<size_t>(b) * na + a] = Ei[static_cast<size_t>(a) * na + b];
    // in place: cached launch records of earlier solves point at this buffer
    P.hblk = blk;
    CGP_HIP(hipMemcpyAsync(P.blk.p, blk.data(), blk.size() * sizeof(TileBlk), hipMemcpyHostToDevice, s));
    h2d(s, P.oagg, oagg);
    h2d(s, P.kzk, kzk);
    h2d(s, P.kzv64, kzv);
    std::vector<float> kzv32(kzv.begin(), kzv.end());
    h2d(s, P.kzv32, kzv32);
    // rows padded with zeros to einv_stride(na) entries (16-byte aligned rows for the coarse step)
    const int ms = einv_stride(na);
    std::vector<double> Ep(static_cast<size_t>(na) * ms, 0.0);
    for (int a = 0; a < na; ++a)
        std::copy(Ei.begin() + static_cast<size_t>(a) * na, Ei.begin() + static_cast<size_t>(a + 1) * na,
                  Ep.begin() + static_cast<size_t>(a) * ms);
    h2d(s, P.einv, Ep);
    std::vector<float> ep32(Ep.begin(), Ep.end());
    h2d(s, P.einv32, ep32);
    CGP_HIP(hipStreamSynchronize(s));
    P.defl_state = 1;
    return true;
}

}  // namespace cgp
