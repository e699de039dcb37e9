// Jacobi-preconditioned conjugate gradients for the coarse Poisson systems
// K phi = b of Eqs. 12 and 15 (the paper solves them with GMRES(m)+ILU(0),
// Section 2.3; after Dirichlet elimination K is symmetric positive definite,
// so CG applies).
//
// Single-reduction form: one grid-wide synchronisation per iteration.  With
// u = M^-1 r, w = K u and s = K p carried by recurrences,
//   p_i = u_i + beta_i p_{i-1},   s_i = w_i + beta_i s_{i-1}
//   x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i
//   u_{i+1} = M^-1 r_{i+1},       w_{i+1} = K u_{i+1}
//   gamma = r.u, delta = w.u, sigma = u.s_i   (one fused reduction)
//   beta_{i+1}  = gamma_{i+1} / gamma_i
//   alpha_{i+1} = gamma_{i+1} / (delta + 2 beta sigma + beta^2 gamma_i / alpha_i)
// The denominator is p_{i+1}.K p_{i+1} expanded exactly, so it stays valid when
// the residual is replaced by a true residual (mixed precision, below).
//
// Halo: the product w_{i+1} = K u_{i+1} needs u_{i+1} at neighbouring rows owned
// by other workgroups.  Those values are recomputed from r_i, w_i, s_{i-1}
// (written by the previous stage, hence stable) into LDS over the workgroup's
// column range, so neither a second synchronisation nor a global gather of a
// freshly written vector is needed.  r, w, s are double-buffered by stage
// parity: every stage reads buffer par^1 and writes buffer par (copying what it
// does not change), so the buffers a stage reads are known before its state is.
//
// Mixed precision (CGP_FP32_IR): matrix, recurrences and products in fp32, dot
// products accumulated in fp64; the fp32 correction c is folded into the fp64
// iterate and the residual replaced by fl32(b - K x) computed in fp64 whenever
// ||r|| has dropped by `delta` since the last replacement.  Convergence is
// decided on true fp64 residuals only.
//
// Two drivers run the same stages:
//   k_cg_step       one stage per launch, one row per thread; the host replays
//                   a captured graph of launches until the instances are done
//                   (kernel boundaries are the cheapest grid-wide
//                   synchronisation on this GPU).  Every global load an
//                   iteration needs (sliced-ELL row, vectors over the halo range)
//                   is issued at kernel start, before the stage is decoded, so an
//                   iteration costs about one memory round trip.
//   k_cg_persistent all stages in one co-resident launch with a grid barrier
//                   (fits inside a caller's graph capture of a whole step)
#include <hip/hip_ext.h>

#include "cgp_internal.hpp"

namespace cgp {
namespace {

constexpr int BLOCK = 512;
constexpr int NWAVE = BLOCK / 64;
constexpr int LDS_DOUBLES = 8192;   // 64 KB staging buffer
constexpr int LDS_FLOATS = 2 * LDS_DOUBLES;
constexpr int KMAX = 12;            // widest ELL row the one-row-per-thread iteration holds in registers
constexpr int HMAX = 8;             // most staged entries per thread in that iteration (4096 per workgroup)

// Pointers read from a launch record are generic (flat) to the compiler; these
// casts let it emit global-memory loads and stores, which it can keep in flight.
#define CGP_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const CGP_GLOBAL T *gld(const T *p) {
    return (const CGP_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ CGP_GLOBAL T *gst(T *p) {
    return (CGP_GLOBAL T *)p;
}
// Memory that no thread writes while the kernel runs, read at a uniform address: through the
// constant address space the compiler loads it with scalar loads, which complete apart from
// the vector loads in flight.
#define CGP_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const CGP_CONST T *cld(const T *p) {
    return (const CGP_CONST T *)p;
}
// a whole record that way (word by word: structs do not copy across address spaces)
template <class T>
__device__ __forceinline__ T cld_record(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "records of whole 32-bit words");
    const CGP_CONST uint32_t *src = (const CGP_CONST uint32_t *)p;
    uint32_t w[sizeof(T) / 4];
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 4; ++i) w[i] = src[i];
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

enum State : int32_t {
    ST_BOOT = 0,  // before the first stage
    ST_JUDGE,     // LEARNED: energy-norm comparison of the network guess with prev1
    ST_RES,       // r = b - K x (fp64); the first one also stores the initial x
    ST_START,     // u = M^-1 r, w = K u, reductions gamma, delta, sigma
    ST_ITER,      // one CG iteration
    ST_FOLD,      // mixed, last stage: x += c, c = 0 (refinements fold c at START)
    ST_ZEROX,     // ||b|| = 0: x = 0
    ST_DONE
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// block-wide sums of NS values into out[] (valid for every thread after return)
template <int NS>
__device__ inline void block_sums(double (&v)[NS], double (*red)[NPART], double *out) {
    static_assert(NS <= NPART, "the reduction rows hold NPART values");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = wave_sum(v[s]);
    if (lane == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) red[wave][s] = v[s];
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        double t = 0.0;
        for (int w = 0; w < NWAVE; ++w) t += red[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// the workgroup's NS sums written to part[s * stride], s < NS, in block_sums' order; one
// barrier (no thread reads the sums afterwards)
template <int NS>
__device__ inline void block_partials(double (&v)[NS], double (*red)[NPART], double *part, int stride) {
    static_assert(NS <= NPART, "the reduction rows hold NPART values");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = wave_sum(v[s]);
    if (lane == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) red[wave][s] = v[s];
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        double t = 0.0;
        for (int w = 0; w < NWAVE; ++w) t += red[w][threadIdx.x];
        part[static_cast<size_t>(threadIdx.x) * stride] = t;
    }
}

// sum of an instance's per-workgroup partials (same order in every workgroup); out[NRED],
// the deflation term of the transitions, is zero (the persistent engine does not deflate)
__device__ inline void reduce_partials(const double *part, int nblk, double (*red)[NPART], double *out) {
    double t[NRED + 1] = {};
    for (int j = threadIdx.x; j < nblk; j += BLOCK) {
#pragma unroll
        for (int s = 0; s < NRED; ++s) t[s] += part[s * nblk + j];
    }
    block_sums(t, red, out);
}

// ------------------------------------------------------------------ state transitions

// After a true residual ||r||^2 = rr of the iterate (on the first, also ||b||^2 = bb): the end,
// a stop, or the restart of the recurrences.  Executed by one thread.
__device__ inline Ctl after_residual(Ctl c, double rr, double bb, const SolveParams &prm, int guess) {
    const bool mixed = prm.precision == CGP_FP32_IR;
    const double tol = prm.tol;
    if (c.first) {
        c.bnorm = sqrt(bb);
        if (bb == 0.0) {
            c.state = ST_ZEROX;
            return c;
        }
        if (!isfinite(bb)) {
            c.status = CGP_SOLVE_BREAKDOWN;
            c.state = ST_DONE;
            return c;
        }
    }
    if (!isfinite(rr)) {
        c.status = CGP_SOLVE_BREAKDOWN;
        c.state = ST_DONE;
        return c;
    }
    const double rn = sqrt(rr);
    c.rel_res = rn / c.bnorm;
    if (c.first && guess != CGP_GUESS_LEARNED) c.rel_res_guess = c.rel_res;
    if (!c.first) ++c.refinements;
    // mixed: the residual was of x + c, and c is folded into x before the end
    const int32_t end = (mixed && !c.first) ? ST_FOLD : ST_DONE;
    if (rn <= tol * c.bnorm) {
        c.status = CGP_SOLVE_OK;
        c.state = end;
        return c;
    }
    if (c.it >= prm.max_iter) {
        c.status = CGP_SOLVE_NOCONV;
        c.state = end;
        return c;
    }
    // fp64: a failed verification restarts CG; mixed: a replaced residual keeps p and s
    c.restart = (c.first || !mixed) ? 1 : 0;
    c.first = 0;
    // the phase's refinement point delta rn, unless the phase after it would be short (the
    // tolerance within a factor delta^(1/4) of that point: half a decade at delta = 0.01):
    // then this phase runs to the tolerance (rmax = 0 leaves only the stopping test)
    c.rmax = (mixed && prm.delta * sqrt(sqrt(prm.delta)) * rn <= tol * c.bnorm) ? 0.0 : rn;
    c.state = ST_START;
    return c;
}

// Decide the next stage from the stage just executed and its reductions S.  judge_res: the
// kernel's judge stage also leaves the guess's residual as the first residual stage does.
// Executed by one thread; every workgroup of the instance computes the same result.
__device__ inline Ctl transition(Ctl c, const double *S, const SolveParams &prm, int guess, bool judge_res = true) {
    const bool mixed = prm.precision == CGP_FP32_IR;
    const double tol = prm.tol;
    switch (c.state) {
    case ST_BOOT:
        c.it = c.refinements = 0;
        c.status = CGP_SOLVE_OK;
        c.guess_used = guess;
        c.restart = 1;
        c.first = 1;
        c.gamma = c.alpha = c.beta = c.pap = 0.0;
        c.bnorm = c.rmax = c.rel_res = c.rel_res_guess = 0.0;
        c.state = guess == CGP_GUESS_LEARNED ? ST_JUDGE : ST_RES;
        break;
    case ST_JUDGE: {
        const double rl = S[0], rp = S[1], gain = S[3];
        const double bn = sqrt(S[2]) > 0.0 ? sqrt(S[2]) : 1.0;
        if (gain >= 0.0 && isfinite(rl) && isfinite(gain)) {   // a non-finite network output is rejected
            c.guess_used = CGP_GUESS_LEARNED;
            c.rel_res_guess = sqrt(rl) / bn;
            if (judge_res)
                c = after_residual(c, rl, S[2], prm, guess);
            else
                c.state = ST_RES;
        } else {   // the first residual stage starts from prev1 instead
            c.guess_used = CGP_GUESS_GIVEN;
            c.rel_res_guess = sqrt(rp) / bn;
            c.state = ST_RES;
        }
        break;
    }
    case ST_RES:
        c = after_residual(c, S[0], S[1], prm, guess);
        break;
    case ST_START: {
        const double g = S[0], dl = S[1], sg = S[2];
        double denom;
        // with deflation S[NRED] = mu . Z^T K u: p = u + beta p - Z mu stays K-orthogonal to range(Z)
        if (c.restart) {
            c.beta = 0.0;
            denom = dl - S[NRED];
        } else {
            c.beta = g / c.gamma;
            denom = dl + 2.0 * c.beta * sg + c.beta * c.beta * c.pap - S[NRED];
        }
        if (!(denom > 0.0) || !isfinite(denom) || !isfinite(g)) {
            c.status = CGP_SOLVE_BREAKDOWN;
            c.state = ST_DONE;
            break;
        }
        c.alpha = g / denom;
        c.gamma = g;
        c.state = ST_ITER;
        break;
    }
    case ST_ITER: {
        const double g = S[0], dl = S[1], sg = S[2], rr = S[3];
        ++c.it;
        if (!isfinite(rr) || !isfinite(g)) {
            c.status = CGP_SOLVE_BREAKDOWN;
            c.state = ST_DONE;
            break;
        }
        const double rn = sqrt(rr);
        const bool stop = rn <= tol * c.bnorm || c.it >= prm.max_iter;
        c.pap = c.gamma / c.alpha;   // p.Kp of the direction just used
        if (!mixed && stop) {
            c.state = ST_RES;   // verify on the true residual
            break;
        }
        if (mixed && (stop || rn <= prm.delta * c.rmax)) {
            c.state = ST_RES;   // refine from the true residual of x + c; p (and s = K p) are kept
            break;
        }
        c.beta = g / c.gamma;
        const double denom = dl + 2.0 * c.beta * sg + c.beta * c.beta * c.pap - S[NRED];
        if (!(denom > 0.0) || !isfinite(denom)) {
            c.status = CGP_SOLVE_BREAKDOWN;
            c.state = ST_DONE;
            break;
        }
        c.alpha = g / denom;
        c.gamma = g;
        c.restart = 0;
        break;
    }
    case ST_FOLD:
        c.state = ST_DONE;
        break;
    case ST_ZEROX:
        c.rel_res = c.rel_res_guess = 0.0;
        c.status = CGP_SOLVE_OK;
        c.state = ST_DONE;
        break;
    default:
        break;
    }
    return c;
}

// The iterate a solve's first residual stage starts from, which that stage also stores in x
// for its rows: zero, the extrapolation 2 prev1 - prev2, prev1 (a network guess the judge
// rejected), or x as the caller or the network left it.  The stage reads it from its source,
// never from x, so the rows of other workgroups are never read while they are written.
enum FirstIterate : int { X0_AS_IS = 0, X0_ZERO, X0_EXTRAP, X0_PREV1 };
__device__ inline int first_iterate(const Ctl &c, int guess) {
    if (!c.first) return X0_AS_IS;
    if (guess == CGP_GUESS_ZERO) return X0_ZERO;
    if (guess == CGP_GUESS_EXTRAP) return X0_EXTRAP;
    if (guess == CGP_GUESS_LEARNED && c.guess_used != CGP_GUESS_LEARNED) return X0_PREV1;
    return X0_AS_IS;
}
template <class PX, class PP>
__device__ inline double first_x(int src, PX x, PP p1, PP p2, int64_t j) {
    return src == X0_ZERO ? 0.0 : src == X0_EXTRAP ? 2.0 * p1[j] - p2[j] : src == X0_PREV1 ? p1[j] : x[j];
}

// ------------------------------------------------------------------ stage work

// The matrix of a row-range product: CSR, and the column-major ELL copy (entry k of row i
// at k * n + i, padded with the row itself and value 0; width ew, 0 when absent).
template <class V>
struct RowMat {
    const int32_t *rowptr, *col;
    const V *val;
    const int32_t *ecol;
    const V *eval;
    int ew;
    int64_t n;
};

// y_i = sum_k val[k] * g(col[k]) for the workgroup's rows, `lanes` threads per row;
// emit(i, y_i) from each row's first lane.  With one lane per row and an ELL copy of at
// most KMAX columns, a thread issues its row's loads together from the ELL copy (same
// terms, same order) instead of walking the CSR row one dependent load at a time.
template <bool ELL, class V, class Gather, class Emit>
__device__ inline void spmv_rows(const RowRange &R, int lanes, const RowMat<V> &A, Gather g, Emit emit) {
    if (ELL && lanes == 1 && A.ecol && A.ew <= KMAX) {
        const CGP_GLOBAL int32_t *ec = gld(A.ecol);
        const CGP_GLOBAL V *ev = gld(A.eval);
        for (int32_t base = R.r0; base < R.r1; base += BLOCK) {
            const int32_t i = base + threadIdx.x;
            if (i >= R.r1) continue;
            int32_t c[KMAX];
            V v[KMAX];
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                if (k < A.ew) {
                    c[k] = ec[k * A.n + i];
                    v[k] = ev[k * A.n + i];
                }
            }
            V acc = V(0);
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < A.ew) acc += v[k] * g(c[k]);
            emit(i, acc);
        }
        return;
    }
    const int32_t *__restrict__ rowptr = A.rowptr;
    const int32_t *__restrict__ col = A.col;
    const V *__restrict__ val = A.val;
    const int per_pass = BLOCK / lanes;
    const int sub = threadIdx.x % lanes;
    for (int32_t base = R.r0; base < R.r1; base += per_pass) {
        const int32_t i = base + threadIdx.x / lanes;
        V acc = V(0);
        if (i < R.r1) {
            const int32_t k1 = rowptr[i + 1];
            for (int32_t k = rowptr[i] + sub; k < k1; k += lanes) acc += val[k] * g(col[k]);
        }
        for (int m = lanes >> 1; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
        if (i < R.r1 && sub == 0) emit(i, acc);
    }
}

// Fill LDS with src(j) over the column range (calling own(j, v) for the
// workgroup's own rows) and multiply from LDS; without room in LDS, own(j, v)
// runs over the own rows and the product gathers src(col) directly.
template <bool ELL, class V, class Src, class Own, class Emit>
__device__ inline void staged_product(const RowRange &R, bool staged, int lanes, const RowMat<V> &A, V *lds,
                                      Src src, Own own, Emit emit) {
    if (staged) {
        for (int32_t j = R.c0 + threadIdx.x; j <= R.c1; j += BLOCK) {
            const V v = src(j);
            lds[j - R.c0] = v;
            if (j >= R.r0 && j < R.r1) own(j, v);
        }
        __syncthreads();
        spmv_rows<ELL, V>(R, lanes, A, [&](int32_t j) { return lds[j - R.c0]; },
                     [&](int32_t i, V y) { emit(i, y, lds[i - R.c0]); });
        __syncthreads();
    } else {
        for (int32_t j = R.r0 + threadIdx.x; j < R.r1; j += BLOCK) own(j, src(j));
        spmv_rows<ELL, V>(R, lanes, A, src, [&](int32_t i, V y) { emit(i, y, src(i)); });
    }
}

struct Shared {
    double lds[LDS_DOUBLES];
    double red[NWAVE][NPART];
    double sums[NPART];
    Ctl ctl;
};

// One stage of instance D over the workgroup's rows (any number of rows per
// thread); reads buffers rd = par^1, writes buffers wr = par; partial sums into v[].
// ELL: the one-lane products may read the rows from the ELL copy (the persistent engine's
// workgroups own thousands of rows); the staged kernels leave it out, where its registers
// would crowd the prefetched iteration
template <bool ELL>
__device__ inline void stage_work(const Ctl &c, const InstDesc &D, const RowRange &R,
                                        const SolveParams &prm, Shared &sh, int par, double (&v)[NRED]) {
    const bool mixed = prm.precision == CGP_FP32_IR;
    const int lanes = D.lanes;
    const double *__restrict__ b = D.b;
    double *__restrict__ x = D.x;
    const int64_t n = D.n;
    const int rd = par ^ 1, wr = par;
    const bool staged64 = R.c1 >= R.c0 && R.c1 - R.c0 + 1 <= LDS_DOUBLES;
    const bool staged32 = R.c1 >= R.c0 && R.c1 - R.c0 + 1 <= LDS_FLOATS;
    double *lds64 = sh.lds;
    float *lds32 = reinterpret_cast<float *>(sh.lds);
    const RowMat<double> A64{D.rowptr, D.col, D.val, D.ell_col, D.ell_val, D.ell_w, n};
    const RowMat<float> A32{D.rowptr, D.col, D.val32, D.ell_col, D.ell_val32, D.ell_w, n};
    auto nop = [](int32_t, auto) {};
    // carry the recurrence vectors of untouched rows into the write buffers
    auto carry = [&](bool cr, bool cw, bool cs) {
        for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) {
            if (mixed) {
                if (cr) D.r32[wr * n + i] = D.r32[rd * n + i];
                if (cw) D.w32[wr * n + i] = D.w32[rd * n + i];
                if (cs) D.s32[wr * n + i] = D.s32[rd * n + i];
            } else {
                if (cr) D.r[wr * n + i] = D.r[rd * n + i];
                if (cw) D.w[wr * n + i] = D.w[rd * n + i];
                if (cs) D.s[wr * n + i] = D.s[rd * n + i];
            }
        }
    };

    switch (c.state) {
    case ST_ZEROX:
        for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) x[i] = 0.0;
        break;
    case ST_FOLD:
        for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) {
            x[i] += static_cast<double>(D.c32[i]);
            D.c32[i] = 0.0f;
        }
        break;
    case ST_JUDGE: {
        const double *p1 = D.prev1;
        // J(x) = x.Kx / 2 - b.x = -x.(b + r) / 2 differs from the energy-norm error
        // |x - x*|_K^2 / 2 by a constant, so v[3] = J(prev1) - J(guess) (times 2) > 0
        // says the network's guess is the closer one in the norm CG minimises
        // the guess's residual is also left as the first residual stage would leave it (r, and
        // c = 0 when mixed): an accepted guess goes on to the restart directly
        staged_product<ELL, double>(R, staged64, lanes, A64, lds64, [&](int32_t j) { return x[j]; },
                               nop, [&](int32_t i, double y, double) {
                                   const double r = b[i] - y;
                                   if (mixed) {
                                       D.r32[wr * n + i] = static_cast<float>(r);
                                       D.c32[i] = 0.0f;
                                   } else {
                                       D.r[wr * n + i] = r;
                                   }
                                   v[0] += r * r;
                                   v[2] += b[i] * b[i];
                                   v[3] += x[i] * (b[i] + r);
                               });
        staged_product<ELL, double>(R, staged64, lanes, A64, lds64, [&](int32_t j) { return p1[j]; },
                               nop, [&](int32_t i, double y, double) {
                                   const double r = b[i] - y;
                                   v[1] += r * r;
                                   v[3] -= p1[i] * (b[i] + r);
                               });
        break;
    }
    case ST_RES: {
        const bool first = c.first;
        const int src = first_iterate(c, D.guess);
        const double *p1 = D.prev1, *p2 = D.prev2;
        if (mixed) {
            // after the first, the iterate is x + c (c: the fp32 correction since the last START)
            float *r32 = D.r32 + wr * n;
            float *c32 = D.c32;
            staged_product<ELL, double>(R, staged64, lanes, A64, lds64,
                                   [&](int32_t j) {
                                       return first ? first_x(src, x, p1, p2, j) : x[j] + static_cast<double>(c32[j]);
                                   },
                                   nop, [&](int32_t i, double y, double xi) {
                                       const double ri = b[i] - y;
                                       r32[i] = static_cast<float>(ri);
                                       if (first) c32[i] = 0.0f;
                                       if (src != X0_AS_IS) x[i] = xi;
                                       v[0] += ri * ri;
                                       if (first) v[1] += b[i] * b[i];
                                   });
        } else {
            double *r = D.r + wr * n;
            staged_product<ELL, double>(R, staged64, lanes, A64, lds64,
                                   [&](int32_t j) { return first_x(src, x, p1, p2, j); },
                                   nop, [&](int32_t i, double y, double xi) {
                                       const double ri = b[i] - y;
                                       r[i] = ri;
                                       if (src != X0_AS_IS) x[i] = xi;
                                       v[0] += ri * ri;
                                       if (first) v[1] += b[i] * b[i];
                                   });
        }
        if (!first && mixed) carry(false, false, true);   // START keeps the direction: it needs s
        break;
    }
    case ST_START: {
        const bool keep = !c.restart;
        if (mixed) {
            const float *r = D.r32 + rd * n, *s = D.s32 + rd * n, *dv = D.dinv32;
            float *w = D.w32 + wr * n;
            staged_product<ELL, float>(R, staged32, lanes, A32, lds32,
                                  [&](int32_t j) { return dv[j] * r[j]; },
                                  [&](int32_t j, float u) {
                                      v[0] += static_cast<double>(r[j]) * static_cast<double>(u);
                                      if (keep) v[2] += static_cast<double>(u) * static_cast<double>(s[j]);
                                  },
                                  [&](int32_t i, float y, float u) {
                                      w[i] = y;
                                      v[1] += static_cast<double>(y) * static_cast<double>(u);
                                  });
            // fold the correction the residual stage saw into x; the next one starts at zero
            for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) {
                x[i] += static_cast<double>(D.c32[i]);
                D.c32[i] = 0.0f;
            }
        } else {
            const double *r = D.r + rd * n, *s = D.s + rd * n, *dv = D.dinv;
            double *w = D.w + wr * n;
            staged_product<ELL, double>(R, staged64, lanes, A64, lds64,
                                   [&](int32_t j) { return dv[j] * r[j]; },
                                   [&](int32_t j, double u) {
                                       v[0] += r[j] * u;
                                       if (keep) v[2] += u * s[j];
                                   },
                                   [&](int32_t i, double y, double u) {
                                       w[i] = y;
                                       v[1] += y * u;
                                   });
        }
        carry(true, false, keep);
        break;
    }
    case ST_ITER: {
        const bool rs = c.restart;
        if (mixed) {
            const float al = static_cast<float>(c.alpha), be = static_cast<float>(c.beta);
            const float *r = D.r32 + rd * n, *w = D.w32 + rd * n, *so = D.s32 + rd * n, *dv = D.dinv32;
            float *rn = D.r32 + wr * n, *wn = D.w32 + wr * n, *sn = D.s32 + wr * n;
            float *p = D.p32, *cc = D.c32;
            // u_{i+1} at row j from the stable r_i, w_i, s_{i-1}
            auto s_new = [&](int32_t j) { return rs ? w[j] : w[j] + be * so[j]; };
            staged_product<ELL, float>(R, staged32, lanes, A32, lds32,
                                  [&](int32_t j) { return dv[j] * (r[j] - al * s_new(j)); },
                                  [&](int32_t j, float u1) {
                                      const float sj = s_new(j);
                                      const float u0 = dv[j] * r[j];
                                      const float pj = rs ? u0 : u0 + be * p[j];
                                      const float rj = r[j] - al * sj;
                                      p[j] = pj;
                                      sn[j] = sj;
                                      rn[j] = rj;
                                      cc[j] += al * pj;
                                      v[0] += static_cast<double>(rj) * static_cast<double>(u1);
                                      v[2] += static_cast<double>(u1) * static_cast<double>(sj);
                                      v[3] += static_cast<double>(rj) * static_cast<double>(rj);
                                  },
                                  [&](int32_t i, float y, float u1) {
                                      wn[i] = y;
                                      v[1] += static_cast<double>(y) * static_cast<double>(u1);
                                  });
        } else {
            const double al = c.alpha, be = c.beta;
            const double *r = D.r + rd * n, *w = D.w + rd * n, *so = D.s + rd * n, *dv = D.dinv;
            double *rn = D.r + wr * n, *wn = D.w + wr * n, *sn = D.s + wr * n;
            double *p = D.p;
            auto s_new = [&](int32_t j) { return rs ? w[j] : w[j] + be * so[j]; };
            staged_product<ELL, double>(R, staged64, lanes, A64, lds64,
                                   [&](int32_t j) { return dv[j] * (r[j] - al * s_new(j)); },
                                   [&](int32_t j, double u1) {
                                       const double sj = s_new(j);
                                       const double u0 = dv[j] * r[j];
                                       const double pj = rs ? u0 : u0 + be * p[j];
                                       const double rj = r[j] - al * sj;
                                       p[j] = pj;
                                       sn[j] = sj;
                                       rn[j] = rj;
                                       x[j] += al * pj;
                                       v[0] += rj * u1;
                                       v[2] += u1 * sj;
                                       v[3] += rj * rj;
                                   },
                                   [&](int32_t i, double y, double u1) {
                                       wn[i] = y;
                                       v[1] += y * u1;
                                   });
        }
        break;
    }
    default:
        break;
    }
}

// ------------------------------------------------------------------ one-row-per-thread iteration

// Values an iteration needs, loaded before the stage is decoded: the ELL row of
// the thread's row and r, w, s, D^-1 over the staged halo range.
template <class T, int H>
struct IterPrefetch {
    T hd[H], hr[H], hw[H], hs[H];                // staged entries c0 + tid + h*BLOCK
    T od, orr, ow, os, op, ox;                   // own row: D^-1, r, w, s, p, c (mixed) or x (fp64)
    T sv[KMAX];
    int32_t sc[KMAX];
};

template <class T>
__device__ inline const T *vec_of(const InstDesc &D, int which);   // 0 r, 1 w, 2 s, 3 dinv, 4 p
template <>
__device__ inline const double *vec_of<double>(const InstDesc &D, int which) {
    return which == 0 ? D.r : which == 1 ? D.w : which == 2 ? D.s : which == 3 ? D.dinv : D.p;
}
template <>
__device__ inline const float *vec_of<float>(const InstDesc &D, int which) {
    return which == 0 ? D.r32 : which == 1 ? D.w32 : which == 2 ? D.s32 : which == 3 ? D.dinv32 : D.p32;
}

template <class T, int H>
__device__ inline void iter_prefetch(IterPrefetch<T, H> &f, const InstDesc &D, const RowRange &R, int rd) {
    const int64_t n = D.n;
    const CGP_GLOBAL T *r = gld(vec_of<T>(D, 0) + rd * n), *w = gld(vec_of<T>(D, 1) + rd * n);
    const CGP_GLOBAL T *s = gld(vec_of<T>(D, 2) + rd * n);
    const CGP_GLOBAL T *dv = gld(vec_of<T>(D, 3)), *p = gld(vec_of<T>(D, 4));
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int32_t j = R.c0 + threadIdx.x + h * BLOCK;
        if (j <= R.c1) {
            f.hd[h] = dv[j];
            f.hr[h] = r[j];
            f.hw[h] = w[j];
            f.hs[h] = s[j];
        }
    }
    const int32_t i = R.r0 + threadIdx.x;
    if (i < R.r1) {
        f.od = dv[i];
        f.orr = r[i];
        f.ow = w[i];
        f.os = s[i];
        f.op = p[i];
        if constexpr (sizeof(T) == 4)
            f.ox = gld(D.c32)[i];
        else
            f.ox = gld(D.x)[i];
        const CGP_GLOBAL T *ev = gld(sizeof(T) == 4 ? reinterpret_cast<const T *>(D.ell_val32)
                                                     : reinterpret_cast<const T *>(D.ell_val));
        const CGP_GLOBAL int32_t *ec = gld(D.ell_col);
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k < D.ell_w) {
                f.sv[k] = ev[k * n + i];
                f.sc[k] = ec[k * n + i];
            }
        }
    }
}

// one CG iteration for the workgroup's rows (at most BLOCK of them) from prefetched values
template <class T, int H>
__device__ inline void iter_fast(const IterPrefetch<T, H> &f, const Ctl &c, const InstDesc &D, const RowRange &R,
                                 int wr, T *lds, double (&v)[NRED]) {
    const int64_t n = D.n;
    const T al = static_cast<T>(c.alpha), be = static_cast<T>(c.beta);
    const bool rs = c.restart;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int32_t j = R.c0 + threadIdx.x + h * BLOCK;
        if (j <= R.c1) {
            const T sj = rs ? f.hw[h] : f.hw[h] + be * f.hs[h];
            lds[j - R.c0] = f.hd[h] * (f.hr[h] - al * sj);
        }
    }
    __syncthreads();
    const int32_t i = R.r0 + threadIdx.x;
    if (i < R.r1) {
        const T sj = rs ? f.ow : f.ow + be * f.os;
        const T rj = f.orr - al * sj;
        const T u1 = lds[i - R.c0];
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < D.ell_w) acc += f.sv[k] * lds[f.sc[k] - R.c0];
        const T u0 = f.od * f.orr;
        const T pj = rs ? u0 : u0 + be * f.op;
        gst(const_cast<T *>(vec_of<T>(D, 4)))[i] = pj;
        gst(const_cast<T *>(vec_of<T>(D, 2)) + wr * n)[i] = sj;
        gst(const_cast<T *>(vec_of<T>(D, 0)) + wr * n)[i] = rj;
        gst(const_cast<T *>(vec_of<T>(D, 1)) + wr * n)[i] = acc;
        if constexpr (sizeof(T) == 4)
            gst(D.c32)[i] = f.ox + al * pj;
        else
            gst(D.x)[i] = f.ox + al * pj;
        const double r64 = static_cast<double>(rj), u64 = static_cast<double>(u1);
        v[0] += r64 * u64;
        v[1] += static_cast<double>(acc) * u64;
        v[2] += u64 * static_cast<double>(sj);
        v[3] += r64 * r64;
    }
}

__device__ inline void write_stats(const Ctl &c, const SolveParams &prm, int idx) {
    cgp_solve_stats o;
    o.iters = c.it;
    o.refinements = c.refinements;
    o.status = c.status;
    o.guess_used = c.guess_used;
    o.rel_res = c.rel_res;
    o.rel_res_guess = c.rel_res_guess;
    prm.stats[idx] = o;
}

// The previous stage's sums of an instance, by every thread of the workgroup: the first
// NRED of its per-workgroup partials, and S[NRED] = 0 (the stages of a deflated solve
// decode from the coarse step's records instead: reduced_decode).  Each thread adds the
// slots t, t + BLOCK, ..., then block_sums adds threads and wavefronts in a fixed order, so
// every workgroup of the instance gets the same sums.  One round of loads for up to BLOCK workgroups, instead of a wavefront walking
// the slots 64 at a time.
__device__ inline void stage_sums(const InstDesc &D, int rd, double (*red)[NPART], double *out) {
    const int nblk = D.nblk;
    const CGP_GLOBAL double *pg = gld(D.partials + static_cast<size_t>(rd) * NPART * nblk);
    double t[NRED + 1] = {};
    for (int j = threadIdx.x; j < nblk; j += BLOCK) {
        double a[NRED];
#pragma unroll
        for (int q = 0; q < NRED; ++q) a[q] = pg[q * nblk + j];
#pragma unroll
        for (int q = 0; q < NRED; ++q) t[q] += a[q];
    }
    block_sums(t, red, out);   // t[NRED] = 0: deflated stages decode from the coarse step's sums
}

// The common transition, an iteration followed by another one, kept short and
// inline; every other case goes through transition().  Same arithmetic.
__device__ inline Ctl next_state(const Ctl &prev, const double *S, const SolveParams &prm, int guess,
                                 bool judge_res = true) {
    if (prev.state == ST_ITER) {
        const double g = S[0], dl = S[1], sg = S[2], rr = S[3];
        // the stopping tests of transition() on squares: rn <= t  <=>  rr <= t^2 (t >= 0)
        const double t_conv = prm.tol * prev.bnorm, t_ref = prm.delta * prev.rmax;
        const bool mixed = prm.precision == CGP_FP32_IR;
        const bool go_on = isfinite(rr) && isfinite(g) && !(rr <= t_conv * t_conv) &&
                           prev.it + 1 < prm.max_iter && !(mixed && rr <= t_ref * t_ref);
        if (go_on) {
            Ctl c = prev;
            ++c.it;
            c.pap = c.gamma / c.alpha;
            c.beta = g / c.gamma;
            const double denom = dl + 2.0 * c.beta * sg + c.beta * c.beta * c.pap - S[NRED];
            if (denom > 0.0 && isfinite(denom)) {
                c.alpha = g / denom;
                c.gamma = g;
                c.restart = 0;
                return c;
            }
        }
    }
    return transition(prev, S, prm, guess, judge_res);
}

// What workgroup 0 of an instance does after a transition (one thread): carry the state
// forward and, when the instance finished, write its stats and report completion.  A stage
// whose successor is the end whatever it sums (the fold of a mixed solve, x = 0 for b = 0)
// is the instance's last: this launch does its work and carries the end forward, so no
// further launch is needed to find it.
__device__ inline void stage_bookkeeping(const InstDesc &D, int par, const Ctl &prev, const Ctl &c,
                                         const SolveParams &prm, int32_t *done_count, int32_t *host_flag) {
    const double none[NRED + 1] = {};
    const Ctl out = (c.state == ST_FOLD || c.state == ST_ZEROX) ? transition(c, none, prm, D.guess) : c;
    D.ctl[par] = out;   // carried forward every launch, DONE included
    if (out.state == ST_DONE && prev.state != ST_DONE) {
        write_stats(out, prm, D.stats_index);
        // the last instance to finish reports the launches it needed, then completion
        if (atomicAdd(done_count, 1) == prm.n_inst - 1) {
            __hip_atomic_store(host_flag + 1, out.stages, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(host_flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// Decode the stage: the workgroup sums the previous stage's partials, thread 0 applies
// the transition into sh.ctl (workgroup 0 of the instance also carries the state forward
// and reports completion); the other threads wait at the barrier.
__device__ inline void decode_stage(const InstDesc &D, int lb, int rd, int par, bool judge_res, const SolveParams *prm_dev,
                                    Shared &sh, int32_t *done_count, int32_t *host_flag) {
    Ctl prev{};
    if (threadIdx.x == 0) prev = D.ctl[rd];   // in flight while the sums are loaded
    stage_sums(D, rd, sh.red, sh.sums);
    if (threadIdx.x == 0) {
        const SolveParams prm = *prm_dev;
        Ctl c = prev;
        if (prev.state != ST_DONE) {
            c = next_state(prev, sh.sums, prm, D.guess, judge_res);
            c.stages = prev.stages + 1;
        }
        sh.ctl = c;
        if (lb == 0) stage_bookkeeping(D, par, prev, c, prm, done_count, host_flag);
    }
    __syncthreads();
}

// A deflated tiled stage finds the previous stage's sums in the records of that stage's
// coarse step (ncb records per instance, each a slice of the tiles' NRED sums and a partial
// of c): wavefront 0 adds them (lanes over the records, then across the wavefront: a fixed
// order) instead of the whole workgroup reducing every tile's partials, and thread 0 applies
// the transition.  The control state and the parameters come through scalar loads (the
// stage writes ctl[par], never ctl[rd], and no parameter).
__device__ inline Ctl reduced_decode(const InstDesc &D, int lb, int rd, int par, bool judge_res, const SolveParams *prm_dev,
                                     Shared &sh, int32_t *done_count, int32_t *host_flag) {
    const Ctl prev = cld_record(D.ctl + rd);
    const SolveParams prm = cld_record(prm_dev);
    if (threadIdx.x < 64) {
        const CGP_GLOBAL double *cp = gld(D.cpart);
        double S[NRED + 1] = {};
        for (int j = static_cast<int>(threadIdx.x); j < D.ncb; j += 64) {
#pragma unroll
            for (int q = 0; q <= NRED; ++q) S[q] += cp[j * (NRED + 1) + q];
        }
#pragma unroll
        for (int q = 0; q <= NRED; ++q) S[q] = wave_sum(S[q]);
        if (threadIdx.x == 0) {
            Ctl c = prev;
            if (prev.state != ST_DONE) {
                c = next_state(prev, S, prm, D.guess, judge_res);
                c.stages = prev.stages + 1;
            }
            sh.ctl = c;
            if (lb == 0) stage_bookkeeping(D, par, prev, c, prm, done_count, host_flag);
        }
    }
    __syncthreads();
    return sh.ctl;
}

// ------------------------------------------------------------------ driver 1: one stage per launch

// The staged kernels renumber an instance's workgroups with xcd_block, so that every XCD
// takes a contiguous run of row blocks or tiles.
// ONE: a single instance, whose record arrives by value in the kernel arguments (one
// dependent load less on every pointer the stage follows)
template <class T, int H, bool ONE>
__global__ __launch_bounds__(BLOCK) void k_cg_step(const InstDesc *__restrict__ insts, const InstDesc one,
                                                   const int32_t *__restrict__ block_inst, int n_inst,
                                                   const RowRange *__restrict__ ranges,
                                                   const SolveParams *__restrict__ prm_dev, int par,
                                                   int32_t *done_count, int32_t *host_flag) {
    __shared__ Shared sh;
    const InstDesc &D = ONE ? one : insts[block_inst[blockIdx.x]];
    const int lb = xcd_block(blockIdx.x - D.blk0, D.nblk);
    const RowRange R = ranges[D.blk0 + lb];
    const int rd = par ^ 1;
    const bool fast = D.fast && R.r1 - R.r0 <= BLOCK && R.c1 >= R.c0 && R.c1 - R.c0 + 1 <= H * BLOCK;
    // speculative loads for an iteration, in flight while the state is decoded
    IterPrefetch<T, H> f;
    if (fast) iter_prefetch<T, H>(f, D, R, rd);
    decode_stage(D, lb, rd, par, true, prm_dev, sh, done_count, host_flag);
    const Ctl c = sh.ctl;
    if (c.state == ST_DONE) return;
    double v[NRED] = {};
    if (fast && c.state == ST_ITER) {
        iter_fast<T, H>(f, c, D, R, par, reinterpret_cast<T *>(sh.lds), v);
    } else {
        const SolveParams prm = *prm_dev;
        stage_work<false>(c, D, R, prm, sh, par, v);
    }
    block_partials(v, sh.red, D.partials + static_cast<size_t>(par) * NPART * D.nblk + lb, D.nblk);
}

// ------------------------------------------------------------------ tiled iteration

// One CG stage (iteration or restart of the recurrences) for a workgroup's tile,
// with the preconditioner M^-1 = Jacobi (degree 1) or a Chebyshev polynomial of
// degree d in D^-1 K: the workgroup gathers r, w, s and D^-1 over its region
// (distance <= d), updates r there, runs the d-step Chebyshev iteration for
// K z = r' on shrinking prefixes of the region (each product with K loses one
// distance level) and ends with u' = z and w' = K u' on its own rows — one
// global reduction per iteration however large d is.  Region row t belongs to
// thread t % BLOCK; the own rows come first, so a thread holds one own row, or two
// in a tile of more than BLOCK rows.
constexpr int TH = TILE_REGION / BLOCK;   // region rows per thread
constexpr int TS = TILE_SPMV / BLOCK;     // local matrix rows per thread
static_assert(BLOCK == TILE_ROWS, "one own row per thread in a tile of TILE_ROWS rows");
static_assert(TILE_OWN * BLOCK == TILE_ROWS_MAX && TILE_OWN <= TS, "own rows are local matrix rows");
static_assert(4 * TILE_REGION * sizeof(double) <= LDS_DOUBLES * sizeof(double),
              "three region vectors and the deflation term in LDS");

template <class T>
__device__ inline T *rwsd_of(const InstDesc &D);
template <>
__device__ inline double *rwsd_of<double>(const InstDesc &D) { return D.rwsd64; }
template <>
__device__ inline float *rwsd_of<float>(const InstDesc &D) { return D.rwsd32; }
template <class T>
__device__ inline T *up_of(const InstDesc &D);
template <>
__device__ inline double *up_of<double>(const InstDesc &D) { return D.up64; }
template <>
__device__ inline float *up_of<float>(const InstDesc &D) { return D.up32; }

template <class T, int W>
struct TilePrefetch {
    int32_t g[TH];                 // region rows t = tid + h * BLOCK (global ids, -1 past the end)
    T r[TH], w[TH], s[TH], dv[TH];
    T ou[TILE_OWN], op[TILE_OWN], ox[TILE_OWN];   // own rows: u = M^-1 r, p, c (mixed) or x (fp64)
    T ev[TS][W];                   // local matrix rows t = tid + h * BLOCK
    uint32_t ec[TS][W / 2];        // their region columns, two 16-bit indices per register
};

template <class T>
__device__ inline const T *tile_val(const InstDesc &D);
template <>
__device__ inline const double *tile_val<double>(const InstDesc &D) { return D.tval; }
template <>
__device__ inline const float *tile_val<float>(const InstDesc &D) { return D.tval32; }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <class T, int W>
__device__ inline void tile_prefetch(TilePrefetch<T, W> &f, const InstDesc &D, const TileBlk &B, int rd) {
    // Every load is issued by every thread, at a clamped index where the thread has no row
    // (its values are then replaced by zeros): with no branch around the loads the compiler
    // can wait for exactly the loads a step needs, so the gathers that follow the region's
    // row list go out as soon as that list has arrived, while the matrix records are in flight.
    const int64_t n = D.n;
    constexpr int CW = tile_col_stride(W);   // 16-bit columns per record
    constexpr int VP = 16 / sizeof(T);        // values per 16-byte load
    static_assert(W == SPLIT_WIDTH || W % VP == 0, "value records are whole 16-byte loads");
    const int tid = static_cast<int>(threadIdx.x);
    // the region's global rows first (the gathers below wait for them, not for the records)
    const CGP_GLOBAL int32_t *reg = gld(D.treg + B.reg_off);
#pragma unroll
    for (int h = 0; h < TH; ++h) {
        const int t = tid + h * BLOCK;
        const int32_t g = reg[min(t, B.nreg - 1)];
        f.g[h] = t < B.nreg ? g : -1;
    }
    // local matrix rows (rows past nspmv gather entry 0 times 0)
#pragma unroll
    for (int h = 0; h < TS; ++h) {
        const int t = tid + h * BLOCK;
        const bool live = t < B.nspmv;
        const size_t tc = static_cast<size_t>(min(t, B.nspmv - 1));
        if constexpr (W == SPLIT_WIDTH) {
            // split records, column-major over the tile's rows: pair q of every row in turn
            const size_t ns = static_cast<size_t>(B.nspmv);
            const CGP_GLOBAL uint32_t *sc = reinterpret_cast<const CGP_GLOBAL uint32_t *>(gld(D.tcol)) +
                                            (SPLIT_WIDTH / 2) * static_cast<size_t>(B.ell_off) + tc;
            const CGP_GLOBAL T *sv = gld(tile_val<T>(D)) + SPLIT_WIDTH * static_cast<size_t>(B.ell_off) + 2 * tc;
#pragma unroll
            for (int q = 0; q < SPLIT_WIDTH / 2; ++q) {
                const uint32_t c = sc[q * ns];
                f.ec[h][q] = live ? c : 0u;
                if constexpr (sizeof(T) == 4) {
                    const u32x2 u = *reinterpret_cast<const CGP_GLOBAL u32x2 *>(sv + 2 * q * ns);
                    f.ev[h][2 * q] = live ? __uint_as_float(u.x) : 0.0f;
                    f.ev[h][2 * q + 1] = live ? __uint_as_float(u.y) : 0.0f;
                } else {
                    const u32x4 u = *reinterpret_cast<const CGP_GLOBAL u32x4 *>(sv + 2 * q * ns);
                    f.ev[h][2 * q] = live ? __hiloint2double(static_cast<int>(u.y), static_cast<int>(u.x)) : 0.0;
                    f.ev[h][2 * q + 1] = live ? __hiloint2double(static_cast<int>(u.w), static_cast<int>(u.z)) : 0.0;
                }
            }
        } else {
            const size_t row = static_cast<size_t>(B.ell_off) + tc;
            const CGP_GLOBAL u32x4 *ec = reinterpret_cast<const CGP_GLOBAL u32x4 *>(gld(D.tcol) + row * CW);
            const u32x4 c0 = ec[0];
            f.ec[h][0] = live ? c0.x : 0u;
            f.ec[h][1] = live ? c0.y : 0u;
            f.ec[h][2] = live ? c0.z : 0u;
            f.ec[h][3] = live ? c0.w : 0u;
            if constexpr (W > 8) {
                const u32x4 c1 = ec[1];
                f.ec[h][4] = live ? c1.x : 0u;
                f.ec[h][5] = live ? c1.y : 0u;
            }
            const CGP_GLOBAL u32x4 *ev = reinterpret_cast<const CGP_GLOBAL u32x4 *>(gld(tile_val<T>(D)) + row * W);
#pragma unroll
            for (int q = 0; q < W / VP; ++q) {
                const u32x4 u = ev[q];
                if constexpr (sizeof(T) == 4) {
                    f.ev[h][4 * q] = live ? __uint_as_float(u.x) : 0.0f;
                    f.ev[h][4 * q + 1] = live ? __uint_as_float(u.y) : 0.0f;
                    f.ev[h][4 * q + 2] = live ? __uint_as_float(u.z) : 0.0f;
                    f.ev[h][4 * q + 3] = live ? __uint_as_float(u.w) : 0.0f;
                } else {
                    f.ev[h][2 * q] = live ? __hiloint2double(static_cast<int>(u.y), static_cast<int>(u.x)) : 0.0;
                    f.ev[h][2 * q + 1] = live ? __hiloint2double(static_cast<int>(u.w), static_cast<int>(u.z)) : 0.0;
                }
            }
        }
    }
    // own rows: (u, p) by own slot, consecutive over the tile
    const CGP_GLOBAL T *up = gld(up_of<T>(D)) + 2 * static_cast<int64_t>(B.own_off);
#pragma unroll
    for (int h = 0; h < TILE_OWN; ++h) {
        const int t = tid + h * BLOCK;
        const bool live = t < B.nt[0];
        const int tc = min(t, B.nt[0] - 1);
        const T u = up[2 * tc], p = up[2 * tc + 1];
        f.ou[h] = live ? u : T(0);
        f.op[h] = live ? p : T(0);
    }
    // (r, w, s, D^-1) of a region row: one 16-byte load (fp32) or two (fp64)
    const CGP_GLOBAL u32x4 *q = reinterpret_cast<const CGP_GLOBAL u32x4 *>(gld(rwsd_of<T>(D)) + rd * n * 4);
#pragma unroll
    for (int h = 0; h < TH; ++h) {
        const int32_t j = f.g[h];
        const int64_t jc = j >= 0 ? j : 0;
        const bool live = j >= 0;
        if constexpr (sizeof(T) == 4) {
            const u32x4 a = q[jc];
            f.r[h] = live ? __uint_as_float(a.x) : 0.0f;
            f.w[h] = live ? __uint_as_float(a.y) : 0.0f;
            f.s[h] = live ? __uint_as_float(a.z) : 0.0f;
            f.dv[h] = live ? __uint_as_float(a.w) : 1.0f;
        } else {
            const u32x4 a = q[2 * jc], b = q[2 * jc + 1];
            f.r[h] = live ? __hiloint2double(static_cast<int>(a.y), static_cast<int>(a.x)) : 0.0;
            f.w[h] = live ? __hiloint2double(static_cast<int>(a.w), static_cast<int>(a.z)) : 0.0;
            f.s[h] = live ? __hiloint2double(static_cast<int>(b.y), static_cast<int>(b.x)) : 0.0;
            f.dv[h] = live ? __hiloint2double(static_cast<int>(b.w), static_cast<int>(b.z)) : 1.0;
        }
    }
    // own rows: c (fp32) or x (fp64) by row
#pragma unroll
    for (int h = 0; h < TILE_OWN; ++h) {
        const int32_t j = f.g[h];
        const int64_t jc = j >= 0 ? j : 0;
        const bool live = tid + h * BLOCK < B.nt[0];
        T x;
        if constexpr (sizeof(T) == 4)
            x = gld(D.c32)[jc];
        else
            x = gld(D.x)[jc];
        f.ox[h] = live ? x : T(0);
    }
}

// Deflation (aggregates: every tile's own rows cut into D.agg parts by bisection, Z their
// free-row indicators): the coarse coefficients mu = E^-1 Z^T v written by the coarse
// kernel after the previous stage, the thread's coupling record (a region row and its
// (K Z) entries) with the mu of the aggregates it names, and the own row's aggregate code.
template <class T>
struct DeflPrefetch {
    int32_t kr;                // region index of the record, -1 for none
    uint32_t kg[KZ_PER_ROW];   // the aggregates it names
    double mu_own;             // thread a < agg: mu of the tile's aggregate a
    T kv[KZ_PER_ROW];          // (K Z)_{row, a}
    T km[KZ_PER_ROW];          // mu_a (rounded to the iteration's precision)
    int32_t code[TILE_OWN];    // own rows: 0 Dirichlet (or none), 1 + part of the tile
};

template <class T>
__device__ inline const T *kz_val(const InstDesc &D);
template <>
__device__ inline const double *kz_val<double>(const InstDesc &D) { return D.kzv; }
template <>
__device__ inline const float *kz_val<float>(const InstDesc &D) { return D.kzv32; }

// (1) the loads that depend on nothing: coupling record, aggregate codes, own-aggregate mu;
// issued ahead of the tile's loads, so that (2), the gathers of the named aggregates' mu,
// waits for them alone
template <class T>
__device__ inline void defl_records(DeflPrefetch<T> &f, const InstDesc &D, const TileBlk &B, int lb) {
    const int tid = static_cast<int>(threadIdx.x);
    const double m = gld(D.mu)[D.agg * lb + min(tid, D.agg - 1)];
    f.mu_own = tid < D.agg ? m : 0.0;
#pragma unroll
    for (int h = 0; h < TILE_OWN; ++h) {
        const int t = tid + h * BLOCK;
        const int32_t code = gld(D.oagg)[static_cast<size_t>(B.reg_off) + min(t, B.nt[0] - 1)];
        f.code[h] = t < B.nt[0] ? code : 0;
    }
    // record kz_off + min(t, nkz): the records of the next tile, or the one past the last
    // tile's, where the thread has none (kg, kv and km are read only where kr >= 0)
    const size_t q = static_cast<size_t>(B.kz_off) + min(tid, B.nkz);
    const uint64_t k = gld(D.kzk)[q];
    constexpr uint64_t MASK = (uint64_t(1) << KZ_BITS) - 1;
    f.kr = tid < B.nkz ? static_cast<int32_t>(k & MASK) : -1;
#pragma unroll
    for (int e = 0; e < KZ_PER_ROW; ++e) f.kg[e] = static_cast<uint32_t>((k >> (KZ_BITS * (1 + e))) & MASK);
    const CGP_GLOBAL T *kv = gld(kz_val<T>(D)) + q * KZ_PER_ROW;
#pragma unroll
    for (int e = 0; e < KZ_PER_ROW; ++e) f.kv[e] = kv[e];
}

template <class T>
__device__ inline void defl_mu(DeflPrefetch<T> &f, const InstDesc &D) {
    const CGP_GLOBAL double *mu = gld(D.mu);
#pragma unroll
    for (int e = 0; e < KZ_PER_ROW; ++e) f.km[e] = static_cast<T>(mu[f.kg[e]]);
}

// y_t = sum_k ev[h][k] * x[ec[h][k]] for the thread's local matrix row h; with split records
// (W = SPLIT_WIDTH) the diagonal term dg x_t comes first (own = x_t, held by the thread)
template <class T, int W>
__device__ inline T tile_row(const TilePrefetch<T, W> &f, int h, const T *x, T own, T dg) {
    T acc = W == SPLIT_WIDTH ? dg * own : T(0);
#pragma unroll
    for (int k = 0; k < W; ++k) acc += f.ev[h][k] * x[(f.ec[h][k / 2] >> (16 * (k & 1))) & 0xffffu];
    return acc;
}

// nt: the tile's distance prefix counts, cheb: the Chebyshev coefficients (both in LDS).
// Each Chebyshev step is one pass over the rows that still need it: the step's
// residual update (one product with K, reading the previous step's dz of the
// neighbours from LDS) and its dz and z updates; r', the residual and z of a row
// stay in the thread's registers (no other row reads them), dz alternates
// between two LDS buffers, and the last step leaves the final z there for w = K z.
// With deflation, kzm holds (K Z mu) over the region and zm = (Z mu) at the own rows
// (their aggregate's mu), code their aggregate: ITER takes p = u + beta p - Z mu,
// s = w + beta s - K Z mu (mu = E^-1 Z^T w of the previous stage); START applies the
// coarse correction x += Z mu, r -= K Z mu (mu = E^-1 Z^T r of the residual stage before
// it).  Both emit Z^T w' (the sums over the tile's aggregates) as the partials after the
// NRED sums.
template <class T, int W>
__device__ inline void tile_iter(const TilePrefetch<T, W> &f, const Ctl &c, const InstDesc &D, const TileBlk &B,
                                 const int32_t *nt, const double *cheb, int wr, T *lds, const T *kzm, bool defl,
                                 const T (&zm)[TILE_OWN], double (&v)[NRED], double (&av)[TILE_OWN]) {
    const int64_t n = D.n;
    const bool start = c.state == ST_START;
    const bool rs = c.restart;
    const T al = start ? T(0) : static_cast<T>(c.alpha), be = static_cast<T>(c.beta);
    T *Zl = lds, *Da = lds + TILE_REGION, *Db = Da + TILE_REGION;
    const int deg = D.degree;
    const T c0 = static_cast<T>(cheb[0]);
    T s_own[TILE_OWN] = {}, r_own[TILE_OWN] = {};
    T rr[TS], zz[TS], qq[TS], dd[TS];
    // split records: the diagonal of a local matrix row, 1 / D^-1 (rounded to T)
    T dg[TS];
#pragma unroll
    for (int h = 0; h < TS; ++h)
        dg[h] = (W == SPLIT_WIDTH && static_cast<int>(threadIdx.x) + h * BLOCK < B.nspmv) ? T(1) / f.dv[h] : T(0);
    // r' = r - alpha (w + beta s) over the region; first Chebyshev step z = c0 D^-1 r'
#pragma unroll
    for (int h = 0; h < TH; ++h) {
        const int t = threadIdx.x + h * BLOCK;
        if (t < B.nreg) {
            const T kz = defl ? kzm[t] : T(0);
            const T sj = start ? f.s[h] : (rs ? f.w[h] : f.w[h] + be * f.s[h]) - kz;
            const T rj = start ? f.r[h] - kz : f.r[h] - al * sj;
            if (h < TILE_OWN) {
                s_own[h] = sj;
                r_own[h] = rj;
            }
            const T z = f.dv[h] * rj * c0;
            Zl[t] = z;
            if (h < TS) {
                rr[h] = rj;
                zz[h] = z;
                dd[h] = z;
            }
        }
    }
    __syncthreads();
    const T *Uz = Zl;   // where the final z ends up
    for (int k = 1; k < deg; ++k) {
        // step k on rows at distance <= d-k: res_k = res_{k-1} - K dz_{k-1} (res_1 = r' - K z_1),
        // dz_k = a1 dz_{k-1} + a2 D^-1 res_k, z += dz_k
        const T a1 = static_cast<T>(cheb[2 * k - 1]), a2 = static_cast<T>(cheb[2 * k]);
        const int lim = nt[deg - k];
        const T *src = k == 1 ? Zl : ((k & 1) ? Db : Da);
        T *dst = (k & 1) ? Da : Db;
        const bool last = k + 1 == deg;
        // the gathers of all of the thread's rows first (in flight together), then the updates
        T kx[TS];
#pragma unroll
        for (int h = 0; h < TS; ++h) kx[h] = tile_row(f, h, src, dd[h], dg[h]);
#pragma unroll
        for (int h = 0; h < TS; ++h) {
            const int t = threadIdx.x + h * BLOCK;
            if (t < lim) {
                qq[h] = k == 1 ? rr[h] - kx[h] : qq[h] - kx[h];
                const T dz = a1 * dd[h] + a2 * (f.dv[h] * qq[h]);
                dd[h] = dz;
                zz[h] += dz;
                dst[t] = last ? zz[h] : dz;
            }
        }
        __syncthreads();
        Uz = dst;
    }
    // own rows: u' = z, w' = K u', the recurrences and the reductions
#pragma unroll
    for (int h = 0; h < TILE_OWN; ++h) {
        if (static_cast<int>(threadIdx.x) + h * BLOCK >= nt[0]) continue;
        const int32_t j = f.g[h];
        const T u1 = zz[h];
        const T wn = tile_row(f, h, Uz, zz[h], dg[h]);
        // (r, w, s) of the row into the write parity (D^-1 stays in the fourth slot)
        CGP_GLOBAL T *q = gst(rwsd_of<T>(D)) + (wr * n + j) * 4;
        q[0] = r_own[h];
        q[1] = wn;
        q[2] = s_own[h];
        CGP_GLOBAL T *up = gst(up_of<T>(D)) + 2 * (static_cast<int64_t>(B.own_off) + threadIdx.x + h * BLOCK);
        if (!start) {
            const T pj = (rs ? f.ou[h] : f.ou[h] + be * f.op[h]) - zm[h];
            up[0] = u1;
            up[1] = pj;
            if constexpr (sizeof(T) == 4)
                gst(D.c32)[j] = f.ox[h] + al * pj;
            else
                gst(D.x)[j] = f.ox[h] + al * pj;
        } else {
            up[0] = u1;
            up[1] = f.op[h];   // the direction carried (a refinement that keeps it reads it next)
            if constexpr (sizeof(T) == 4) {
                // mixed: fold the correction the residual stage saw (f.ox = c) into x; the next
                // correction starts with the coarse step (deflation) or at zero
                gst(D.x)[j] = gld(D.x)[j] + static_cast<double>(f.ox[h]);
                gst(D.c32)[j] = zm[h];
            } else if (defl) {
                gst(D.x)[j] = f.ox[h] + zm[h];   // fp64: the coarse correction of x
            }
        }
        const double r64 = static_cast<double>(r_own[h]), u64 = static_cast<double>(u1);
        v[0] += r64 * u64;
        v[1] += static_cast<double>(wn) * u64;
        v[2] += u64 * static_cast<double>(s_own[h]);
        v[3] += r64 * r64;
        av[h] = static_cast<double>(wn);   // the row's term of its aggregate's sum Z^T w'

    }
}

// The residual stage of a tiled solve, over the tile's own rows (so that, with deflation, the
// aggregate partials are the tile's sums Z^T r): r = b - K x in fp64 from the CSR matrix.
__device__ inline void tile_res_row(const Ctl &c, const InstDesc &D, int32_t own, bool mixed, int par,
                                    double (&v)[NRED], double &av) {
    const int64_t n = D.n;
    const int wr = par, rd = par ^ 1;
    const CGP_GLOBAL int32_t *rowptr = gld(D.rowptr), *col = gld(D.col);
    const CGP_GLOBAL double *val = gld(D.val), *x = gld(D.x);
    const CGP_GLOBAL float *cc = gld(D.c32);
    const bool with_c = mixed && !c.first;   // the iterate is x + c after the first residual
    const int src = first_iterate(c, D.guess);
    const CGP_GLOBAL double *p1 = gld(D.prev1), *p2 = gld(D.prev2);
    double kx = 0.0;
    for (int32_t k = rowptr[own]; k < rowptr[own + 1]; ++k) {
        const int32_t j = col[k];
        kx += val[k] * (with_c ? x[j] + static_cast<double>(cc[j]) : first_x(src, x, p1, p2, j));
    }
    if (src != X0_AS_IS) gst(D.x)[own] = first_x(src, x, p1, p2, own);
    const double bi = gld(D.b)[own], ri = bi - kx;
    if (mixed) {
        CGP_GLOBAL float *q = gst(D.rwsd32);
        q[(wr * n + own) * 4] = static_cast<float>(ri);
        if (c.first)
            gst(D.c32)[own] = 0.0f;
        else
            q[(wr * n + own) * 4 + 2] = q[(rd * n + own) * 4 + 2];   // START keeps the direction: it needs s
    } else {
        gst(D.rwsd64)[(wr * n + own) * 4] = ri;
    }
    v[0] += ri * ri;
    if (c.first) v[1] += bi * bi;
    av = ri;   // the row's term of its aggregate's sum Z^T r
}

// The judge of a learned guess over the tile's own rows: the fp64 residuals of the guess (in x)
// and of prev1, b.b and the energy-norm comparison x.(b + r_x) - prev1.(b + r_prev1), and for the
// guess what the first residual stage leaves (r with the same arithmetic, c = 0 when mixed, the
// row's term of its aggregate's sum Z^T r), so that an accepted guess goes on to the restart.
__device__ inline void tile_judge_row(const InstDesc &D, int32_t own, bool mixed, int par, double (&v)[NRED],
                                      double &av) {
    const int64_t n = D.n;
    const CGP_GLOBAL int32_t *rowptr = gld(D.rowptr), *col = gld(D.col);
    const CGP_GLOBAL double *val = gld(D.val), *x = gld(D.x), *p1 = gld(D.prev1);
    const int32_t k0 = rowptr[own], k1 = rowptr[own + 1];
    const double bi = gld(D.b)[own];
    // the guess first (its residual is kept), then prev1: one product in flight at a time
    double kx = 0.0;
    for (int32_t k = k0; k < k1; ++k) kx += val[k] * x[col[k]];
    const double rg = bi - kx;
    if (mixed) {
        gst(D.rwsd32)[(par * n + own) * 4] = static_cast<float>(rg);
        gst(D.c32)[own] = 0.0f;
    } else {
        gst(D.rwsd64)[(par * n + own) * 4] = rg;
    }
    v[0] += rg * rg;
    v[2] += bi * bi;
    v[3] += x[own] * (bi + rg);
    av = rg;
    double kp = 0.0;
    for (int32_t k = k0; k < k1; ++k) kp += val[k] * p1[col[k]];
    const double rp = bi - kp;
    v[1] += rp * rp;
    v[3] -= p1[own] * (bi + rp);
}

template <class T, int W>
__device__ inline void tile_res(const Ctl &c, const InstDesc &D, const TileBlk &B, const TilePrefetch<T, W> &f,
                                bool mixed, int par, double (&v)[NRED], double (&av)[TILE_OWN]) {
#pragma unroll
    for (int h = 0; h < TILE_OWN; ++h)
        if (static_cast<int>(threadIdx.x) + h * BLOCK < B.nt[0]) tile_res_row(c, D, f.g[h], mixed, par, v, av[h]);
}

// fp32: at most 128 VGPRs, so that two workgroups share a compute unit and a grid of
// up to twice the compute units (a 131841-row mesh cuts into 258 tiles) runs at once.
// DEFL: the deflated iteration (its coupling records and coefficients take registers
// the plain one does not need)
template <class T, int W, bool DEFL, bool ONE>
__global__ __launch_bounds__(BLOCK, sizeof(T) == 4 ? 4 : 1) void k_cg_tile(const InstDesc *__restrict__ insts,
                                                   const InstDesc one, const int32_t *__restrict__ block_inst,
                                                   int unb, const RowRange *__restrict__ ranges,
                                                   const SolveParams *__restrict__ prm_dev, int par,
                                                   int32_t *done_count, int32_t *host_flag) {
    __shared__ Shared sh;
    __shared__ int32_t s_nt[TILE_MAX_DEGREE + 2];
    __shared__ double s_cheb[2 * TILE_MAX_DEGREE];
    // unb > 0: every instance has unb workgroups, and the instance follows from the workgroup
    // index (one dependent load less before the tile's record and its prefetch)
    const InstDesc &D = ONE ? one : insts[unb > 0 ? static_cast<int>(blockIdx.x) / unb : block_inst[blockIdx.x]];
    const int lb = xcd_block(blockIdx.x - D.blk0, D.nblk);
    const TileBlk B = D.tblk[lb];
    const int rd = par ^ 1;
    // an instance that finished before this launch (the launches that run past the end of a
    // batch's slowest instance): workgroup 0 carries its state forward, and nothing is
    // prefetched.  The state arrives through a scalar load beside the tile's record, which the
    // prefetch waits for anyway.
    if (cld(&D.ctl[rd].state)[0] == ST_DONE) {
        if (lb == 0 && threadIdx.x == 0) D.ctl[par] = cld_record(D.ctl + rd);
        return;
    }
    // speculative loads for an iteration, in flight while the state is decoded
    constexpr bool defl = DEFL;
    // the fp32 split-record kernel judges a learned guess over the tile's own rows and leaves its
    // residual (the first residual stage's work) on the way; the others, whose registers are
    // fuller, judge over row ranges and run the residual stage after it
    constexpr bool JUDGE_RES = W == SPLIT_WIDTH && sizeof(T) == 4;
    DeflPrefetch<T> df;
    df.kr = -1;
#pragma unroll
    for (int h = 0; h < TILE_OWN; ++h) df.code[h] = 0;
    if (defl) defl_records<T>(df, D, B, lb);
    TilePrefetch<T, W> f;
    tile_prefetch<T, W>(f, D, B, rd);
    __shared__ double s_mu[AGG_MAX];
    static_assert(AGG_TILE <= AGG_MAX, "the partial slots hold the tile's aggregates");
    T *kzm = reinterpret_cast<T *>(sh.lds) + 3 * TILE_REGION;
    if (defl) {
        defl_mu<T>(df, D);
#pragma unroll
        for (int h = 0; h < TH; ++h) {
            const int t = threadIdx.x + h * BLOCK;
            if (t < B.nreg) kzm[t] = T(0);
        }
    }
    // per-distance row counts and coefficients, indexed by a run-time degree: LDS (from the
    // records already loaded, read after the barriers below)
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < TILE_MAX_DEGREE + 2; ++k) s_nt[k] = B.nt[k];
#pragma unroll
        for (int k = 0; k < 2 * TILE_MAX_DEGREE; ++k) s_cheb[k] = D.cheb[k];
    }
    Ctl c;
    if constexpr (DEFL) {
        c = reduced_decode(D, lb, rd, par, JUDGE_RES, prm_dev, sh, done_count, host_flag);
    } else {
        decode_stage(D, lb, rd, par, JUDGE_RES, prm_dev, sh, done_count, host_flag);
        c = sh.ctl;
    }
    if (c.state == ST_DONE) return;
    double v[NRED] = {};
    double av[TILE_OWN] = {};   // per own row: its term of its aggregate's sum (deflation)
    if (c.state == ST_ITER || c.state == ST_START) {
        if (defl) {
            // K Z mu over the region: one coupling record per thread, zero elsewhere (the
            // decode's barrier put every thread's zeros in place first); the tile's own mu
            if (static_cast<int>(threadIdx.x) < D.agg) s_mu[threadIdx.x] = df.mu_own;
            if (df.kr >= 0) {
                T a = T(0);
#pragma unroll
                for (int e = 0; e < KZ_PER_ROW; ++e) a += df.kv[e] * df.km[e];
                kzm[df.kr] = a;
            }
            __syncthreads();
        }
        T zm[TILE_OWN];   // Z mu at the own rows: the mu of the row's aggregate
#pragma unroll
        for (int h = 0; h < TILE_OWN; ++h) zm[h] = df.code[h] > 0 ? static_cast<T>(s_mu[df.code[h] - 1]) : T(0);
        tile_iter<T, W>(f, c, D, B, s_nt, s_cheb, par, reinterpret_cast<T *>(sh.lds), kzm, defl, zm, v, av);
    } else if (c.state == ST_RES) {
        // the residual over the tile's own rows (its vectors are the tiled iteration's own)
        tile_res<T, W>(c, D, B, f, sizeof(T) == 4, par, v, av);
    } else if (JUDGE_RES && c.state == ST_JUDGE) {
#pragma unroll
        for (int h = 0; h < TILE_OWN; ++h)
            if (static_cast<int>(threadIdx.x) + h * BLOCK < B.nt[0]) tile_judge_row(D, f.g[h], sizeof(T) == 4, par, v, av[h]);
    } else {
        const SolveParams prm = *prm_dev;
        const RowRange R = ranges[D.blk0 + lb];
        stage_work<false>(c, D, R, prm, sh, par, v);
    }
    // the partials: NRED sums and (deflation) the tile's aggregate sums, each own row's term
    // added to its aggregate's slot
    constexpr int NS = DEFL ? NRED + AGG_TILE : NRED;
    double vs[NS];
#pragma unroll
    for (int q = 0; q < NRED; ++q) vs[q] = v[q];
#pragma unroll
    for (int a = 0; a < NS - NRED; ++a) {
        double t = 0.0;
#pragma unroll
        for (int h = 0; h < TILE_OWN; ++h)
            if (df.code[h] == a + 1) t += av[h];
        vs[NRED + a] = t;
    }
    block_partials(vs, sh.red, D.partials + static_cast<size_t>(par) * NPART * D.nblk + lb, D.nblk);
}

// Coarse step of deflation after a tiled stage: mu = E^-1 q with q the stage's aggregate
// sums (the fifth partial of its workgroups), one wavefront per row of E^-1 (two rows per
// wavefront, COARSE_ROWS per workgroup), and per workgroup the partial sum of mu_a q_a
// (fixed order); the next stage reads both.  A row is read with 16-byte loads (E^-1 rows
// start 16-byte aligned: stride einv_stride(m), zero padded); fp32 iterations read the fp32
// copy (both rows' loads in flight together), fp64 ones the fp64 copy (a row at a time).
// Every stage gets one (only those after a residual, restart or iteration stage are read);
// the record of a single instance arrives in the kernel arguments, so the row loads are
// the first memory accesses.
template <class E>
__device__ inline const E *einv_of(const CoarseRec &C);
template <>
__device__ inline const double *einv_of<double>(const CoarseRec &C) { return C.einv; }
template <>
__device__ inline const float *einv_of<float>(const CoarseRec &C) { return C.einv32; }

// BOTH: the two rows' loads of E^-1 at once (fp32 only: registers), for the single-instance
// step, whose few workgroups leave the compute units' wave slots free; the batched step loads a
// row at a time, so that all of its workgroups fit the chip at once (80 registers, six
// wavefronts per SIMD) instead of running a second, partly filled round
template <class E, bool BOTH>
__device__ inline void coarse_rows(const CoarseRec &C, int cb, int par) {
    constexpr int VE = 16 / static_cast<int>(sizeof(E));        // entries per 16-byte load
    constexpr int CH = MAX_DEFL_AGGREGATES / (64 * VE);         // loads per lane and row, at most
    __shared__ double red[COARSE_ROWS];
    __shared__ __attribute__((aligned(16))) double qs[MAX_DEFL_AGGREGATES];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = C.m, ms = einv_stride(m), nt = C.tiles, nch = ms / VE;
    const int a0 = cb * COARSE_ROWS + wave, a1 = a0 + COARSE_WAVES;
    const E *einv = einv_of<E>(C);
    // Loads without branches around them (clamped indices, zeros selected afterwards), q
    // first: its LDS copy then waits for q alone while the rows of E^-1 are in flight.
    // q_a, the partial NRED + (a % agg) of tile a / agg (zero past m)
    constexpr int QT = MAX_DEFL_AGGREGATES / (64 * COARSE_WAVES);   // q entries per thread, at most
    const CGP_GLOBAL double *q = gld(C.partials) + static_cast<size_t>(par) * NPART * nt + static_cast<size_t>(NRED) * nt;
    const int A = C.agg;
    double qv[QT];
#pragma unroll
    for (int k = 0; k < QT; ++k) {
        const int i = static_cast<int>(threadIdx.x) + k * 64 * COARSE_WAVES;
        const int ic = min(i, m - 1);
        const double v = q[static_cast<size_t>(ic % A) * nt + ic / A];
        qv[k] = i < m ? v : 0.0;
    }
    u32x4 e0[CH], e1[BOTH ? CH : 1];
    auto load_row = [&](int a, u32x4 *e) {
        const CGP_GLOBAL u32x4 *er =
            reinterpret_cast<const CGP_GLOBAL u32x4 *>(gld(einv) + static_cast<size_t>(a < m ? a : 0) * ms);
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int c = lane + 64 * k;
            const u32x4 v = er[min(c, nch - 1)];
            e[k] = (a < m && c < nch) ? v : u32x4{0u, 0u, 0u, 0u};
        }
    };
    load_row(a0, e0);
    if constexpr (BOTH) load_row(a1, e1);
    // wave 1: the first 64 tiles of the workgroup's slice of the tiles' NRED partials (tiles
    // [cb nt / ncb, (cb + 1) nt / ncb): about COARSE_ROWS / agg of them), requested behind the
    // rows of E^-1 and summed at the end
    const int j0 = static_cast<int>(static_cast<int64_t>(cb) * nt / C.ncb);
    const int j1 = static_cast<int>(static_cast<int64_t>(cb + 1) * nt / C.ncb);
    const CGP_GLOBAL double *pg = gld(C.partials) + static_cast<size_t>(par) * NPART * nt;
    double tp[NRED] = {};
    if (wave == 1) {
        const int j = min(j0 + lane, j1 - 1);
#pragma unroll
        for (int q = 0; q < NRED; ++q) {
            const double v = pg[q * nt + max(j, 0)];
            tp[q] = j0 + lane < j1 ? v : 0.0;
        }
    }
    // a stage that found the instance finished (launches past the end of the solve) has
    // nothing for the next one; its state was stored by the stage kernel before this launch
    // (a scalar load: no wait for the loads in flight)
    if ((cld(C.ctl) + par)->state == ST_DONE) return;
#pragma unroll
    for (int k = 0; k < QT; ++k) {
        const int i = static_cast<int>(threadIdx.x) + k * 64 * COARSE_WAVES;
        if (i < ms) qs[i] = qv[k];
    }
    __syncthreads();
    auto dot = [&](const u32x4 *e) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int c = lane + 64 * k;
            if (c < nch) {
                if constexpr (sizeof(E) == 4) {
                    acc += static_cast<double>(__uint_as_float(e[k].x)) * qs[4 * c] +
                           static_cast<double>(__uint_as_float(e[k].y)) * qs[4 * c + 1] +
                           static_cast<double>(__uint_as_float(e[k].z)) * qs[4 * c + 2] +
                           static_cast<double>(__uint_as_float(e[k].w)) * qs[4 * c + 3];
                } else {
                    acc += __hiloint2double(static_cast<int>(e[k].y), static_cast<int>(e[k].x)) * qs[2 * c] +
                           __hiloint2double(static_cast<int>(e[k].w), static_cast<int>(e[k].z)) * qs[2 * c + 1];
                }
            }
        }
        return wave_sum(acc);
    };
    const double mu0 = dot(e0);
    double mu1;
    if constexpr (BOTH) {
        mu1 = dot(e1);
    } else {
        load_row(a1, e0);
        mu1 = dot(e0);
    }
    if (lane == 0) {
        red[wave] = a0 < m ? mu0 * qs[a0] : 0.0;
        red[wave + COARSE_WAVES] = a1 < m ? mu1 * qs[a1] : 0.0;
        if (a0 < m) gst(C.mu)[a0] = mu0;
        if (a1 < m) gst(C.mu)[a1] = mu1;
    }
    __syncthreads();
    // the workgroup's record for the next stage's decode: its partial of c = mu . q, and its
    // slice of the tiles' NRED partials (tiles [cb nt / ncb, (cb + 1) nt / ncb), lanes over
    // the slice, then across the wavefront), so that the next stage adds ncb records
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < COARSE_ROWS; ++w) t += red[w];
        gst(C.cpart)[cb * (NRED + 1) + NRED] = t;
    }
    if (wave == 1) {
        double t[NRED];
#pragma unroll
        for (int q = 0; q < NRED; ++q) t[q] = tp[q];
        for (int j = j0 + 64 + lane; j < j1; j += 64) {   // (slices past 64 tiles)
#pragma unroll
            for (int q = 0; q < NRED; ++q) t[q] += pg[q * nt + j];
        }
#pragma unroll
        for (int q = 0; q < NRED; ++q) t[q] = wave_sum(t[q]);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < NRED; ++q) gst(C.cpart)[cb * (NRED + 1) + q] = t[q];
        }
    }
}

template <class E>
__global__ __launch_bounds__(64 * COARSE_WAVES) void k_cg_coarse1(const CoarseRec C, int par) {
    coarse_rows<E, sizeof(E) == 4>(C, blockIdx.x, par);
}

template <class E>
__global__ __launch_bounds__(64 * COARSE_WAVES) __attribute__((amdgpu_waves_per_eu(sizeof(E) == 4 ? 6 : 1))) void
k_cg_coarse(const CoarseRec *__restrict__ recs,
                                                                const int32_t *__restrict__ cblk_inst, int par) {
    const CoarseRec C = recs[cblk_inst[blockIdx.x]];
    coarse_rows<E, false>(C, blockIdx.x - C.cblk0, par);
}

__global__ void k_fill_rwsd(int64_t n, const float *dinv32, const double *dinv, float *rwsd32, double *rwsd64) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= 2 * n) return;
    const int64_t row = i < n ? i : i - n;
    if (rwsd32) rwsd32[i * 4 + 3] = dinv32[row];
    if (rwsd64) rwsd64[i * 4 + 3] = dinv[row];
}

__global__ void k_cg_boot(InstDesc *insts, int n_inst, const SolveParams prm, SolveParams *prm_dev,
                          int32_t *done_count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *prm_dev = prm;
        *done_count = 0;
    }
    if (i < n_inst) {
        Ctl c{};
        c.state = ST_BOOT;
        insts[i].ctl[1] = c;   // read by the first launch (par = 0)
    }
}

// After the recorded launches of a captured staged solve: an instance whose last decoded
// stage (carried in ctl[par] by its first workgroup) is not the end was cut off by the
// stage budget, and its statistics say so (status aborted, counters as far as it got).
__global__ void k_cg_close(const InstDesc *insts, int n_inst, const SolveParams *prm_dev, int par) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    Ctl c = insts[i].ctl[par];
    if (c.state != ST_DONE) {
        c.status = CGP_SOLVE_ABORTED;
        write_stats(c, *prm_dev, insts[i].stats_index);
    }
}

// ------------------------------------------------------------------ driver 2: persistent launch

// Grid barrier (arrive counter + generation) with a bounded wait: past `timeout`
// ticks of the constant-rate clock the workgroup raises the abort flag and
// every waiter leaves once it sees it.  Returns false when aborted.
__device__ inline bool grid_barrier(GridSync *gs, uint32_t nblocks, uint32_t &my_gen, uint64_t timeout, int *s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __threadfence();
        const uint32_t old = atomicAdd(&gs->arrive, 1u);
        if (old == nblocks - 1) {
            atomicExch(&gs->arrive, 0u);
            __threadfence();
            atomicAdd(&gs->gen, 1u);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == my_gen) {
                if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > timeout) {
                    atomicExch(&gs->abort, 1);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __threadfence();
        if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        ++my_gen;
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

__global__ __launch_bounds__(BLOCK) void k_cg_persistent(const InstDesc *__restrict__ insts,
                                                         const int32_t *__restrict__ block_inst,
                                                         const RowRange *__restrict__ ranges, SolveParams prm,
                                                         GridSync *gs, int32_t *done_at, uint64_t timeout) {
    __shared__ Shared sh;
    __shared__ int s_ok, s_exit;
    const int inst = block_inst[blockIdx.x];
    const InstDesc &D = insts[inst];
    const int lb = blockIdx.x - D.blk0;
    const RowRange R = ranges[blockIdx.x];
    uint32_t my_gen = 0;
    if (threadIdx.x == 0) {
        my_gen = __hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Ctl c{};
        c.state = ST_BOOT;
        sh.ctl = transition(c, sh.sums, prm, D.guess);
    }
    __syncthreads();
    for (int32_t stage = 0;; ++stage) {
        const int par = stage & 1;
        double *part = D.partials + static_cast<size_t>(par) * NPART * D.nblk;
        const Ctl c = sh.ctl;
        double v[NRED] = {};
        if (c.state != ST_DONE) stage_work<true>(c, D, R, prm, sh, par, v);
        block_sums(v, sh.red, sh.sums);
        if (threadIdx.x < NRED) part[threadIdx.x * D.nblk + lb] = sh.sums[threadIdx.x];
        if (!grid_barrier(gs, gridDim.x, my_gen, timeout, &s_ok)) {
            if (lb == 0 && threadIdx.x == 0 && c.state != ST_DONE) {
                Ctl a = c;
                a.status = CGP_SOLVE_ABORTED;
                write_stats(a, prm, D.stats_index);
            }
            return;
        }
        if (c.state != ST_DONE) {
            reduce_partials(part, D.nblk, sh.red, sh.sums);
            if (threadIdx.x == 0) {
                sh.ctl = transition(c, sh.sums, prm, D.guess);
                if (sh.ctl.state == ST_DONE && lb == 0) {
                    write_stats(sh.ctl, prm, D.stats_index);
                    done_at[inst] = stage;
                }
            }
        }
        // leave once every instance finished at an earlier stage (values written
        // after this barrier are not counted, so all workgroups agree)
        if (threadIdx.x == 0) s_exit = 1;
        __syncthreads();
        for (int i = threadIdx.x; i < prm.n_inst; i += BLOCK)
            if (__hip_atomic_load(&done_at[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > stage - 1) s_exit = 0;
        __syncthreads();
        if (s_exit) return;
    }
}

__global__ void k_persistent_setup(GridSync *gs, int32_t *done_at, int n_inst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        gs->arrive = 0u;
        gs->abort = 0;
    }
    if (i < n_inst) done_at[i] = INT32_MAX;
}

// ------------------------------------------------------------------ plan set-up

// rows [r0, r1) of each workgroup and the column range they touch
__global__ void k_ranges(const InstDesc *insts, const int32_t *block_inst, int grid, RowRange *ranges) {
    const int blk = blockIdx.x;
    if (blk >= grid) return;
    __shared__ int s_lo, s_hi;
    const InstDesc &D = insts[block_inst[blk]];
    const int lb = blk - D.blk0;
    const int32_t r0 = min(D.n, lb * D.chunk), r1 = min(D.n, r0 + D.chunk);
    if (threadIdx.x == 0) {
        s_lo = INT32_MAX;
        s_hi = -1;
    }
    __syncthreads();
    int32_t lo = INT32_MAX, hi = -1;
    for (int32_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const int32_t k0 = D.rowptr[i], k1 = D.rowptr[i + 1];
        if (k1 > k0) {
            lo = min(lo, D.col[k0]);
            hi = max(hi, D.col[k1 - 1]);
        }
    }
    if (hi >= 0) {
        atomicMin(&s_lo, lo);
        atomicMax(&s_hi, hi);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        RowRange R;
        R.r0 = r0;
        R.r1 = r1;
        R.c0 = s_lo;
        R.c1 = s_hi;
        ranges[blk] = R;
    }
}

}  // namespace

int pcg_block_size() { return BLOCK; }

int pcg_max_blocks_per_cu() {
    int a = 0;
    CGP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_cg_persistent, BLOCK, 0));
    return a;
}

int pcg_ell_max_width() { return KMAX; }

void launch_ranges(hipStream_t s, const InstDesc *d_insts, const int32_t *d_block_inst, int grid, RowRange *d_ranges) {
    hipLaunchKernelGGL(k_ranges, dim3(grid), dim3(256), 0, s, d_insts, d_block_inst, grid, d_ranges);
    CGP_HIP(hipGetLastError());
}

void launch_cg_boot(hipStream_t s, InstDesc *d_insts, int n_inst, const SolveParams &prm, SolveParams *d_prm,
                    int32_t *d_done) {
    hipLaunchKernelGGL(k_cg_boot, dim3((n_inst + 255) / 256), dim3(256), 0, s, d_insts, n_inst, prm, d_prm, d_done);
    CGP_HIP(hipGetLastError());
}

void launch_cg_close(hipStream_t s, const InstDesc *d_insts, int n_inst, const SolveParams *d_prm, int par) {
    hipLaunchKernelGGL(k_cg_close, dim3((n_inst + 255) / 256), dim3(256), 0, s, d_insts, n_inst, d_prm, par);
    CGP_HIP(hipGetLastError());
}

void launch_fill_rwsd(hipStream_t s, int64_t n, const float *dinv32, const double *dinv, float *rwsd32,
                      double *rwsd64) {
    hipLaunchKernelGGL(k_fill_rwsd, dim3(blocks_for(2 * n, 256)), dim3(256), 0, s, n, dinv32, dinv, rwsd32, rwsd64);
    CGP_HIP(hipGetLastError());
}

// a kernel launch, with the dispatch's own start and stop timestamps in ev when ev.start is set
#define CGP_LAUNCH(K, G, B, S, EV, ...)                                                                  \
    do {                                                                                                \
        if ((EV).start)                                                                                 \
            hipExtLaunchKernelGGL(K, G, B, 0, S, (EV).start, (EV).stop, 0, __VA_ARGS__);                \
        else                                                                                            \
            hipLaunchKernelGGL(K, G, B, 0, S, __VA_ARGS__);                                             \
    } while (0)

void launch_cg_tile(hipStream_t s, bool mixed, int width, bool defl, int unb, const InstDesc *d_insts,
                    const InstDesc *h_one, const int32_t *d_block_inst, const RowRange *d_ranges, int grid,
                    const SolveParams *d_prm, int par, int32_t *d_done, int32_t *d_host_flag, KernelEvents ev) {
    const InstDesc none{};
#define CGP_TILE(T, W, F)                                                                                          \
    do {                                                                                                           \
        if (h_one)                                                                                                 \
            CGP_LAUNCH((k_cg_tile<T, W, F, true>), dim3(grid), dim3(BLOCK), s, ev, d_insts, *h_one, d_block_inst,  \
                       0, d_ranges, d_prm, par, d_done, d_host_flag);                                             \
        else                                                                                                       \
            CGP_LAUNCH((k_cg_tile<T, W, F, false>), dim3(grid), dim3(BLOCK), s, ev, d_insts, none, d_block_inst,   \
                       unb, d_ranges, d_prm, par, d_done, d_host_flag);                                           \
    } while (0)
#define CGP_TILE_W(T, F)                     \
    if (width == SPLIT_WIDTH) CGP_TILE(T, SPLIT_WIDTH, F); \
    else if (width <= 8) CGP_TILE(T, 8, F); \
    else CGP_TILE(T, 12, F)
    if (mixed) {
        if (defl) { CGP_TILE_W(float, true); } else { CGP_TILE_W(float, false); }
    } else {
        if (defl) { CGP_TILE_W(double, true); } else { CGP_TILE_W(double, false); }
    }
#undef CGP_TILE_W
#undef CGP_TILE
    CGP_HIP(hipGetLastError());
}

void launch_cg_coarse(hipStream_t s, bool e32, const CoarseRec *h_single, const CoarseRec *d_recs,
                      const int32_t *d_cblk_inst, int grid, int par, KernelEvents ev) {
#define CGP_COARSE(E)                                                                                             \
    do {                                                                                                          \
        if (h_single)                                                                                             \
            CGP_LAUNCH(k_cg_coarse1<E>, dim3(grid), dim3(64 * COARSE_WAVES), s, ev, *h_single, par);             \
        else                                                                                                      \
            CGP_LAUNCH(k_cg_coarse<E>, dim3(grid), dim3(64 * COARSE_WAVES), s, ev, d_recs, d_cblk_inst, par);    \
    } while (0)
    if (e32)
        CGP_COARSE(float);
    else
        CGP_COARSE(double);
#undef CGP_COARSE
    CGP_HIP(hipGetLastError());
}

void launch_cg_step(hipStream_t s, bool mixed, int halo, int n_inst, const InstDesc *d_insts,
                    const InstDesc *h_one, const int32_t *d_block_inst, const RowRange *d_ranges, int grid,
                    const SolveParams *d_prm, int par, int32_t *d_done, int32_t *d_host_flag, KernelEvents ev) {
    // staged entries per thread: 4 covers workgroups whose column range spans <= 2048 rows
    const bool small = halo <= 4 * BLOCK;
    const InstDesc none{};
#define CGP_STEP(T, H)                                                                                            \
    do {                                                                                                          \
        if (h_one)                                                                                                \
            CGP_LAUNCH((k_cg_step<T, H, true>), dim3(grid), dim3(BLOCK), s, ev, d_insts, *h_one, d_block_inst,   \
                       n_inst, d_ranges, d_prm, par, d_done, d_host_flag);                                       \
        else                                                                                                      \
            CGP_LAUNCH((k_cg_step<T, H, false>), dim3(grid), dim3(BLOCK), s, ev, d_insts, none, d_block_inst,    \
                       n_inst, d_ranges, d_prm, par, d_done, d_host_flag);                                       \
    } while (0)
    if (mixed) {
        if (small) CGP_STEP(float, 4);
        else CGP_STEP(float, HMAX);
    } else {
        if (small) CGP_STEP(double, 4);
        else CGP_STEP(double, HMAX);
    }
#undef CGP_STEP
    CGP_HIP(hipGetLastError());
}

void launch_cg_persistent(hipStream_t s, const InstDesc *d_insts, int n_inst, const int32_t *d_block_inst,
                          const RowRange *d_ranges, int grid, const SolveParams &prm, GridSync *d_sync,
                          int32_t *d_done_at, uint64_t timeout_ticks) {
    hipLaunchKernelGGL(k_persistent_setup, dim3((n_inst + 255) / 256), dim3(256), 0, s, d_sync, d_done_at, n_inst);
    CGP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cg_persistent, dim3(grid), dim3(BLOCK), 0, s, d_insts, d_block_inst, d_ranges, prm, d_sync,
                       d_done_at, timeout_ticks);
    CGP_HIP(hipGetLastError());
}

}  // namespace cgp
