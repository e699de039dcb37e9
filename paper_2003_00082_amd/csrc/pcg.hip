// Persistent Jacobi-preconditioned CG for the coarse Poisson systems K phi = b
// of Eqs. 12 and 15 (the paper solves them with GMRES(m)+ILU(0), Section 2.3;
// K is symmetric positive definite, so CG applies).
//
// One launch solves a batch of independent instances.  The grid is co-resident
// (one or two workgroups per compute unit) and split statically between the
// instances; each workgroup owns a contiguous range of rows of one instance.
// The solve is a sequence of stages separated by grid-wide barriers; after each
// barrier every workgroup of an instance reduces that instance's per-workgroup
// partial sums in the same fixed order, so all of them take the same decision
// (bitwise) without a further barrier.
//
// Iteration (2 barriers): with p double-buffered,
//   stage A: p_new = z + beta p_old ; q = K p_new ; partial p_new.q
//   stage B: x += alpha p_new ; r -= alpha q ; z = D^-1 r ; partials r.r, r.z
// Stage A gathers p_new at neighbouring rows by recomputing z_j + beta p_old_j
// (both stable during the stage), staged once per stage into LDS when the
// workgroup's column range fits, so the product reads LDS instead of scattered
// global memory.
//
// Mixed mode (CGP_FP32_IR): the same recurrences in fp32 (matrix, vectors,
// products) with fp64 dot accumulation; the fp32 residual is replaced by the
// true fp64 residual b - K x after folding the fp32 correction into the fp64
// iterate whenever the fp32 residual has dropped by `delta` since the last
// replacement.  Convergence is only decided on a true fp64 residual.
#include "cgp_internal.hpp"

namespace cgp {
namespace {

constexpr int BLOCK = 512;
constexpr int NWAVE = BLOCK / 64;
constexpr int LDS_DOUBLES = 8192;          // 64 KB staging buffer
constexpr int LDS_FLOATS = 2 * LDS_DOUBLES;

enum State : int32_t {
    ST_PREP = 0,   // x = initial guess (ZERO / EXTRAP)
    ST_JUDGE,      // LEARNED: residual norms of the network guess and of prev1
    ST_PICK,       // LEARNED rejected: x = prev1
    ST_INIT,       // fp64: r = b - K x, z = D^-1 r, p_old = 0
    ST_A,          // fp64: p_new = z + beta p_old, q = K p_new
    ST_B,          // fp64: x += alpha p_new, r -= alpha q, z = D^-1 r
    ST_VERIFY,     // fp64: true residual when the recurrence says converged
    MX_INIT,       // mixed: r64 = b - K x, r32 = fl32(r64), c32 = 0, z32, p_old32 = 0
    MX_A,          // mixed: p_new32 = z32 + beta p_old32, q32 = K32 p_new32
    MX_B,          // mixed: c32 += alpha p_new32, r32 -= alpha q32, z32 = D32^-1 r32
    MX_FOLD,       // mixed: x += c32, c32 = 0
    MX_RES,        // mixed: r64 = b - K x, r32 = fl32(r64), z32
    ST_ZEROX,      // ||b|| = 0: x = 0
    ST_DONE
};

struct Ctl {
    int32_t state, it, refinements, status, guess_used, par, done;
    int32_t pad_;
    double rho, alpha, beta, bnorm, rmax, rel_res, rel_res_guess;
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// block-wide sums of NPART values; result valid in every thread after return
__device__ inline void block_sums(double (&v)[NPART], double (*red)[NPART], double *out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < NPART; ++s) v[s] = wave_sum(v[s]);
    if (lane == 0) {
#pragma unroll
        for (int s = 0; s < NPART; ++s) red[wave][s] = v[s];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < NPART; ++s) {
            double t = 0.0;
            for (int w = 0; w < NWAVE; ++w) t += red[w][s];
            out[s] = t;
        }
    }
    __syncthreads();
}

// Grid barrier: arrive counter + generation.  The wait is bounded: past
// `timeout` ticks of the constant-rate wall clock the workgroup raises the
// abort flag, and every waiter leaves once it sees the flag.  Returns false
// when the solve was aborted.
__device__ inline bool grid_barrier(GridSync *gs, uint32_t nblocks, uint32_t &my_gen, uint64_t timeout,
                                    int *s_ok) {
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

// ------------------------------------------------------------------ row kernels of the stages

struct Rows {
    int32_t r0, r1;       // rows of this workgroup
    int32_t c0, c1;       // column range [c0, c1] touched by those rows
    bool staged;          // gathers go through LDS
};

// y_i = sum_k val[k] * src(col[k]) for the workgroup's rows, `lanes` threads per
// row; calls emit(i, y_i) once per row (from the row's first lane).
template <class V, class Src, class Emit>
__device__ inline void spmv_rows(const Rows &R, int lanes, const int32_t *__restrict__ rowptr,
                                 const int32_t *__restrict__ col, const V *__restrict__ val, V *lds,
                                 Src src, Emit emit) {
    if (R.staged) {
        for (int32_t j = R.c0 + threadIdx.x; j <= R.c1; j += BLOCK) lds[j - R.c0] = src(j);
        __syncthreads();
    }
    const int per_pass = BLOCK / lanes;
    const int sub = threadIdx.x % lanes;
    for (int32_t base = R.r0; base < R.r1; base += per_pass) {
        const int32_t i = base + threadIdx.x / lanes;
        V acc = V(0);
        if (i < R.r1) {
            const int32_t k1 = rowptr[i + 1];
            if (R.staged) {
                for (int32_t k = rowptr[i] + sub; k < k1; k += lanes) acc += val[k] * lds[col[k] - R.c0];
            } else {
                for (int32_t k = rowptr[i] + sub; k < k1; k += lanes) acc += val[k] * src(col[k]);
            }
        }
        for (int m = lanes >> 1; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
        if (i < R.r1 && sub == 0) emit(i, acc);
    }
    if (R.staged) __syncthreads();   // LDS is reused by the next product
}

// ------------------------------------------------------------------ the persistent kernel

__global__ __launch_bounds__(BLOCK) void k_pcg(const InstDesc *__restrict__ insts,
                                               const int32_t *__restrict__ block_inst, SolveParams prm,
                                               GridSync *gs, int32_t *done_at, uint64_t timeout) {
    __shared__ double lds_raw[LDS_DOUBLES];
    __shared__ double red[NWAVE][NPART];
    __shared__ double sums[NPART];
    __shared__ Ctl ctl;
    __shared__ int s_ok, s_cmin, s_cmax, s_exit;

    const int inst = block_inst[blockIdx.x];
    const InstDesc D = insts[inst];
    const int lb = blockIdx.x - D.blk0;
    const int32_t chunk = (D.n + D.nblk - 1) / D.nblk;
    Rows R;
    R.r0 = min(D.n, lb * chunk);
    R.r1 = min(D.n, R.r0 + chunk);
    const bool mixed = prm.precision == CGP_FP32_IR;
    const int lanes = D.lanes;

    // column range of the workgroup's rows (columns are sorted within a row)
    if (threadIdx.x == 0) {
        s_cmin = INT32_MAX;
        s_cmax = -1;
    }
    __syncthreads();
    {
        int32_t lo = INT32_MAX, hi = -1;
        for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) {
            const int32_t k0 = D.rowptr[i], k1 = D.rowptr[i + 1];
            if (k1 > k0) {
                lo = min(lo, D.col[k0]);
                hi = max(hi, D.col[k1 - 1]);
            }
        }
        if (hi >= 0) {
            atomicMin(&s_cmin, lo);
            atomicMax(&s_cmax, hi);
        }
    }
    __syncthreads();
    R.c0 = s_cmin;
    R.c1 = s_cmax;
    const int cap = mixed ? LDS_FLOATS : LDS_DOUBLES;
    R.staged = (R.c1 >= R.c0) && (R.c1 - R.c0 + 1 <= cap);
    double *lds64 = lds_raw;
    float *lds32 = reinterpret_cast<float *>(lds_raw);

    uint32_t my_gen = 0;
    if (threadIdx.x == 0) {
        my_gen = __hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ctl.it = 0;
        ctl.refinements = 0;
        ctl.status = CGP_SOLVE_OK;
        ctl.par = 0;
        ctl.done = 0;
        ctl.rho = ctl.alpha = ctl.beta = 0.0;
        ctl.bnorm = ctl.rmax = 0.0;
        ctl.rel_res = ctl.rel_res_guess = 0.0;
        ctl.guess_used = D.guess;
        if (D.guess == CGP_GUESS_LEARNED)
            ctl.state = ST_JUDGE;
        else if (D.guess == CGP_GUESS_GIVEN)
            ctl.state = mixed ? MX_INIT : ST_INIT;
        else
            ctl.state = ST_PREP;
    }
    __syncthreads();

    const double *__restrict__ b = D.b;
    double *__restrict__ x = D.x;
    const double *__restrict__ dinv = D.dinv;
    const float *__restrict__ dinv32 = D.dinv32;

    for (int32_t stage = 0;; ++stage) {
        const int par = stage & 1;
        double *part = D.partials + static_cast<size_t>(par) * NPART * D.nblk;
        double v[NPART] = {0.0, 0.0, 0.0, 0.0};
        const int32_t st = ctl.state;
        const double alpha = ctl.alpha, beta = ctl.beta;
        double *pold = ctl.par ? D.p1 : D.p0;
        double *pnew = ctl.par ? D.p0 : D.p1;
        float *pold32 = ctl.par ? D.p32b : D.p32a;
        float *pnew32 = ctl.par ? D.p32a : D.p32b;

        // ---------------------------------------------------------- row work
        switch (st) {
        case ST_PREP:
            for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK)
                x[i] = (D.guess == CGP_GUESS_EXTRAP) ? 2.0 * D.prev1[i] - D.prev2[i] : 0.0;
            break;
        case ST_JUDGE: {
            // |b - K x|^2 (network guess) in v[0], |b - K prev1|^2 in v[1], |b|^2 in v[2]
            spmv_rows<double>(R, lanes, D.rowptr, D.col, D.val, lds64, [&](int32_t j) { return x[j]; },
                              [&](int32_t i, double y) {
                                  const double r = b[i] - y;
                                  v[0] += r * r;
                                  v[2] += b[i] * b[i];
                              });
            const double *p1v = D.prev1;
            spmv_rows<double>(R, lanes, D.rowptr, D.col, D.val, lds64, [&](int32_t j) { return p1v[j]; },
                              [&](int32_t i, double y) {
                                  const double r = b[i] - y;
                                  v[1] += r * r;
                              });
            break;
        }
        case ST_PICK:
            for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) x[i] = D.prev1[i];
            break;
        case ST_INIT:
        case ST_VERIFY: {
            double *r = D.r, *z = D.z;
            const bool init = st == ST_INIT;
            spmv_rows<double>(R, lanes, D.rowptr, D.col, D.val, lds64, [&](int32_t j) { return x[j]; },
                              [&](int32_t i, double y) {
                                  const double ri = b[i] - y;
                                  const double zi = dinv[i] * ri;
                                  r[i] = ri;
                                  z[i] = zi;
                                  pold[i] = 0.0;
                                  v[0] += ri * ri;
                                  v[1] += ri * zi;
                                  if (init) v[2] += b[i] * b[i];
                              });
            break;
        }
        case ST_A: {
            const double *z = D.z;
            double *q = D.q;
            const double *po = pold;
            spmv_rows<double>(R, lanes, D.rowptr, D.col, D.val, lds64,
                              [&](int32_t j) { return z[j] + beta * po[j]; },
                              [&](int32_t i, double y) {
                                  q[i] = y;
                                  v[0] += (z[i] + beta * po[i]) * y;
                              });
            for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) pnew[i] = z[i] + beta * po[i];
            break;
        }
        case ST_B: {
            double *r = D.r, *z = D.z;
            const double *q = D.q;
            for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) {
                x[i] += alpha * pnew[i];
                const double ri = r[i] - alpha * q[i];
                const double zi = dinv[i] * ri;
                r[i] = ri;
                z[i] = zi;
                v[0] += ri * ri;
                v[1] += ri * zi;
            }
            break;
        }
        case MX_INIT:
        case MX_RES: {
            float *r32 = D.r32, *z32 = D.z32, *c32 = D.c32;
            const bool init = st == MX_INIT;
            spmv_rows<double>(R, lanes, D.rowptr, D.col, D.val, lds64, [&](int32_t j) { return x[j]; },
                              [&](int32_t i, double y) {
                                  const double ri = b[i] - y;
                                  const float r32i = static_cast<float>(ri);
                                  const float z32i = dinv32[i] * r32i;
                                  r32[i] = r32i;
                                  z32[i] = z32i;
                                  v[0] += ri * ri;
                                  v[1] += static_cast<double>(r32i) * static_cast<double>(z32i);
                                  if (init) {
                                      c32[i] = 0.0f;
                                      pold32[i] = 0.0f;
                                      v[2] += b[i] * b[i];
                                  }
                              });
            break;
        }
        case MX_A: {
            const float *z32 = D.z32;
            float *q32 = D.q32;
            const float *po = pold32;
            const float bf = static_cast<float>(beta);
            spmv_rows<float>(R, lanes, D.rowptr, D.col, D.val32, lds32,
                             [&](int32_t j) { return z32[j] + bf * po[j]; },
                             [&](int32_t i, float y) {
                                 q32[i] = y;
                                 const float pi = z32[i] + bf * po[i];
                                 v[0] += static_cast<double>(pi) * static_cast<double>(y);
                             });
            for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) pnew32[i] = z32[i] + bf * po[i];
            break;
        }
        case MX_B: {
            float *r32 = D.r32, *z32 = D.z32, *c32 = D.c32;
            const float *q32 = D.q32;
            const float af = static_cast<float>(alpha);
            for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) {
                c32[i] += af * pnew32[i];
                const float ri = r32[i] - af * q32[i];
                const float zi = dinv32[i] * ri;
                r32[i] = ri;
                z32[i] = zi;
                v[0] += static_cast<double>(ri) * static_cast<double>(ri);
                v[1] += static_cast<double>(ri) * static_cast<double>(zi);
            }
            break;
        }
        case MX_FOLD: {
            float *c32 = D.c32;
            for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) {
                x[i] += static_cast<double>(c32[i]);
                c32[i] = 0.0f;
            }
            break;
        }
        case ST_ZEROX:
            for (int32_t i = R.r0 + threadIdx.x; i < R.r1; i += BLOCK) x[i] = 0.0;
            break;
        default:
            break;
        }

        // ---------------------------------------------------------- partial sums of this workgroup
        block_sums(v, red, sums);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int s = 0; s < NPART; ++s) part[s * D.nblk + lb] = sums[s];
        }

        if (!grid_barrier(gs, gridDim.x, my_gen, timeout, &s_ok)) {
            if (lb == 0 && threadIdx.x == 0 && !ctl.done) {
                cgp_solve_stats o;
                o.iters = ctl.it;
                o.refinements = ctl.refinements;
                o.status = CGP_SOLVE_ABORTED;
                o.guess_used = ctl.guess_used;
                o.rel_res = ctl.rel_res;
                o.rel_res_guess = ctl.rel_res_guess;
                *D.stats = o;
            }
            return;
        }

        // ---------------------------------------------------------- instance decision
        if (!ctl.done) {
            double t[NPART] = {0.0, 0.0, 0.0, 0.0};
            for (int j = threadIdx.x; j < D.nblk; j += BLOCK) {
#pragma unroll
                for (int s = 0; s < NPART; ++s) t[s] += part[s * D.nblk + j];
            }
            block_sums(t, red, sums);
            if (threadIdx.x == 0) {
                Ctl &c = ctl;
                const double tol = prm.tol;
                auto finish = [&](int status) {
                    c.status = status;
                    c.done = 1;
                    c.state = ST_DONE;
                };
                switch (st) {
                case ST_PREP:
                    c.state = mixed ? MX_INIT : ST_INIT;
                    break;
                case ST_JUDGE: {
                    c.bnorm = sqrt(sums[2]);
                    const double rl = sums[0], rp = sums[1];
                    const double bn = c.bnorm > 0.0 ? c.bnorm : 1.0;
                    if (rl <= rp && isfinite(rl)) {   // NaN/Inf network output is rejected
                        c.guess_used = CGP_GUESS_LEARNED;
                        c.rel_res_guess = sqrt(rl) / bn;
                        c.state = mixed ? MX_INIT : ST_INIT;
                    } else {
                        c.guess_used = CGP_GUESS_GIVEN;
                        c.rel_res_guess = sqrt(rp) / bn;
                        c.state = ST_PICK;
                    }
                    break;
                }
                case ST_PICK:
                    c.state = mixed ? MX_INIT : ST_INIT;
                    break;
                case ST_INIT:
                case MX_INIT: {
                    const double rr = sums[0], rz = sums[1], bb = sums[2];
                    c.bnorm = sqrt(bb);
                    if (bb == 0.0) {
                        c.state = ST_ZEROX;
                        break;
                    }
                    if (!isfinite(rr) || !isfinite(bb)) {
                        finish(CGP_SOLVE_BREAKDOWN);
                        break;
                    }
                    const double rn = sqrt(rr);
                    c.rel_res = rn / c.bnorm;
                    if (D.guess != CGP_GUESS_LEARNED) c.rel_res_guess = c.rel_res;
                    if (rn <= tol * c.bnorm) {
                        finish(CGP_SOLVE_OK);
                        break;
                    }
                    c.rmax = rn;
                    c.rho = rz;
                    c.beta = 0.0;
                    c.state = (st == ST_INIT) ? ST_A : MX_A;
                    break;
                }
                case ST_A:
                case MX_A: {
                    const double pq = sums[0];
                    if (!(pq > 0.0) || !isfinite(pq)) {
                        finish(CGP_SOLVE_BREAKDOWN);
                        break;
                    }
                    c.alpha = c.rho / pq;
                    c.state = (st == ST_A) ? ST_B : MX_B;
                    break;
                }
                case ST_B: {
                    const double rr = sums[0], rz = sums[1];
                    ++c.it;
                    if (!isfinite(rr)) {
                        finish(CGP_SOLVE_BREAKDOWN);
                        break;
                    }
                    if (sqrt(rr) <= tol * c.bnorm || c.it >= prm.max_iter) {
                        c.state = ST_VERIFY;
                        c.par ^= 1;   // p_new becomes p_old (zeroed by VERIFY)
                        break;
                    }
                    c.beta = rz / c.rho;
                    c.rho = rz;
                    c.par ^= 1;
                    c.state = ST_A;
                    break;
                }
                case ST_VERIFY: {
                    const double rr = sums[0], rz = sums[1];
                    const double rn = sqrt(rr);
                    c.rel_res = rn / c.bnorm;
                    if (!isfinite(rr)) {
                        finish(CGP_SOLVE_BREAKDOWN);
                        break;
                    }
                    if (rn <= tol * c.bnorm) {
                        finish(CGP_SOLVE_OK);
                        break;
                    }
                    if (c.it >= prm.max_iter) {
                        finish(CGP_SOLVE_NOCONV);
                        break;
                    }
                    c.rho = rz;   // restart from the current iterate
                    c.beta = 0.0;
                    c.state = ST_A;
                    break;
                }
                case MX_B: {
                    const double rr = sums[0], rz = sums[1];
                    ++c.it;
                    const double rn = sqrt(rr);
                    if (!isfinite(rr)) {
                        finish(CGP_SOLVE_BREAKDOWN);
                        break;
                    }
                    if (rn <= prm.delta * c.rmax || rn <= tol * c.bnorm || c.it >= prm.max_iter) {
                        c.state = MX_FOLD;
                        break;
                    }
                    c.beta = rz / c.rho;
                    c.rho = rz;
                    c.par ^= 1;
                    c.state = MX_A;
                    break;
                }
                case MX_FOLD:
                    c.state = MX_RES;
                    break;
                case MX_RES: {
                    const double rr = sums[0], rz = sums[1];
                    ++c.refinements;
                    const double rn = sqrt(rr);
                    c.rel_res = rn / c.bnorm;
                    if (!isfinite(rr)) {
                        finish(CGP_SOLVE_BREAKDOWN);
                        break;
                    }
                    if (rn <= tol * c.bnorm) {
                        finish(CGP_SOLVE_OK);
                        break;
                    }
                    if (c.it >= prm.max_iter) {
                        finish(CGP_SOLVE_NOCONV);
                        break;
                    }
                    c.rmax = rn;
                    c.beta = rz / c.rho;   // keep the search direction
                    c.rho = rz;
                    c.par ^= 1;
                    c.state = MX_A;
                    break;
                }
                case ST_ZEROX:
                    c.rel_res = 0.0;
                    c.rel_res_guess = 0.0;
                    finish(CGP_SOLVE_OK);
                    break;
                default:
                    break;
                }
                if (c.done && lb == 0) {
                    cgp_solve_stats o;
                    o.iters = c.it;
                    o.refinements = c.refinements;
                    o.status = c.status;
                    o.guess_used = c.guess_used;
                    o.rel_res = c.rel_res;
                    o.rel_res_guess = c.rel_res_guess;
                    *D.stats = o;
                    done_at[inst] = stage;
                }
            }
        }
        // ---------------------------------------------------------- global exit: every instance
        // finished at an earlier stage (values written after this barrier are not counted)
        if (threadIdx.x == 0) s_exit = 1;
        __syncthreads();
        for (int i = threadIdx.x; i < prm.n_inst; i += BLOCK)
            if (__hip_atomic_load(&done_at[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > stage - 1)
                s_exit = 0;
        __syncthreads();
        if (s_exit) return;
    }
}

__global__ void k_pcg_setup(GridSync *gs, int32_t *done_at, int n_inst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        gs->arrive = 0u;
        gs->abort = 0;
    }
    if (i < n_inst) done_at[i] = INT32_MAX;
}

}  // namespace

int pcg_block_size() { return BLOCK; }
size_t pcg_lds_bytes() { return sizeof(double) * LDS_DOUBLES; }

int pcg_max_blocks_per_cu() {
    int nb = 0;
    CGP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pcg, BLOCK, 0));
    return nb;
}

void launch_pcg(hipStream_t s, const InstDesc *d_insts, int n_inst, const int32_t *d_block_inst, int grid,
                int block, const SolveParams &prm, GridSync *d_sync, int32_t *d_done_at, size_t) {
    (void)block;
    int dev = 0;
    CGP_HIP(hipGetDevice(&dev));
    int khz = 0;
    CGP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) khz = 100000;
    const uint64_t timeout = static_cast<uint64_t>(khz) * 1000ull * 4ull;   // 4 s per barrier wait
    hipLaunchKernelGGL(k_pcg_setup, dim3((n_inst + 255) / 256), dim3(256), 0, s, d_sync, d_done_at, n_inst);
    CGP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_pcg, dim3(grid), dim3(BLOCK), 0, s, d_insts, d_block_inst, prm, d_sync, d_done_at,
                       timeout);
    CGP_HIP(hipGetLastError());
}

}  // namespace cgp
