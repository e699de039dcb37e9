// Learned initial guess of the coarse Poisson solve: a small graph network on the
// coarse mesh that corrects the extrapolation 2 phi^{n-1} - phi^{n-2} (the guess
// is then judged against phi^{n-1} by the solver; see pcg.hip).
//
//   features  X = [b/s_b, p1/s_p, p2/s_p, r_e/s_r, K d/s_r, d/s_d, dirichlet, 1]
//             e = 2 p1 - p2, d = p1 - p2, r_e = b - K e, s_* = RMS over all nodes
//   encoder   h0 = relu(X W0 + c0)                          8 (padded to 16) -> 64
//   layers    h <- relu([h, mean_nbr(h)] W_l + c_l) + h      128 -> 64, l = 1..3
//   decoder   y = h w_d + c_d;  guess = (e + s_d y) on free nodes
//
// Dense products run on the matrix cores (v_mfma_f32_32x32x16_bf16) with
// bfloat16 weights and fp32 accumulation.  Activations, features and neighbour
// means are fp32; the forward pass feeds each as two bfloat16 operands, its high
// part and the remainder (a + b with a = bf16(v), b = bf16(v - a) carries v to
// about 2^-17), so the network's output carries no per-node bfloat16 noise.  The
// gradient products take single bfloat16 operands (layer inputs, features,
// activation gradients).  Biases, decoder, reductions and master weights in fp32.  Training minimises the
// energy norm (delta^T K delta)/N_free of the scaled output error with Adam.
// Every reduction is a per-workgroup partial followed by a fixed-order sum: no
// floating-point atomics, bitwise reproducible.
#include <cmath>
#include <fstream>
#include <map>
#include <memory>

#include "cgp_internal.hpp"

namespace cgp {

constexpr int GH = 64;                 // hidden width
constexpr int GF = 8;                  // input features
constexpr int GFP = 16;                // padded to the MFMA K step
constexpr int GL = 3;                  // message-passing layers
constexpr int P_W0 = 0;
constexpr int P_C0 = P_W0 + GFP * GH;
constexpr int P_L0 = P_C0 + GH;                       // layer l: W at P_L0 + (l-1)*(2GH*GH+GH), c after it
constexpr int P_LSTRIDE = 2 * GH * GH + GH;
constexpr int P_WD = P_L0 + GL * P_LSTRIDE;
constexpr int P_CD = P_WD + GH;
constexpr int P_COUNT = P_CD + 1;
constexpr int Q_W0 = 0;                               // bf16 copies: W0 then W1..W3
constexpr int Q_COUNT = GFP * GH + GL * 2 * GH * GH;

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct GnnWork {
    int64_t n = 0;
    DBuf<double> e, d, re, kd, part, scales, delta;
    DBuf<float> x;                // [n, 16] features (training)
    DBuf<float> h[GL + 1];        // [n + 1, 64] activations; row n stays zero (neighbour-table padding)
    DBuf<float> a[GL + 1];        // pre-activations [n, 64] (training)
    DBuf<float> y;                // [n]
    DBuf<float> dy, dh, dhp, dm;  // training
    DBuf<float> gpart;            // per-workgroup gradient partials
    DBuf<float> gred;             // their sums over RED_CHUNKS ranges of workgroups
    DBuf<float> grad;             // [P_COUNT]
    DBuf<double> lpart;
};

struct Model {
    DBuf<float> theta, m1, m2;
    DBuf<bf16> wq, wqT;       // bf16 weight matrices, row-major and transposed
    int64_t step = 0;
    std::map<const Mesh *, std::unique_ptr<GnnWork>> work;
};

namespace {

constexpr int TPB = 256;
constexpr int TM = 64;                 // rows per forward workgroup
constexpr int SMOOTH_SWEEPS = 4;       // damped Jacobi sweeps applied to the network's guess
constexpr double SMOOTH_OMEGA = 2.0 / 3.0;
constexpr int BW_SUB = 4;              // 64-row sub-tiles per backward workgroup

__device__ inline bf16 to_bf16(float v) { return static_cast<bf16>(v); }
__device__ inline float from_bf16(bf16 v) { return static_cast<float>(v); }

// acc[32x32] += A[32 x K] B[K x 32], A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn] (LDS)
__device__ inline void mfma_tile(f32x16 &acc, const bf16 *A, int sam, int sak, const bf16 *B, int sbk, int sbn,
                                 int K) {
    const int l = threadIdx.x & 63;
    const int mi = l & 31, kh = (l >> 5) * 8;
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            a[i] = A[mi * sam + (k0 + kh + i) * sak];
            b[i] = B[(k0 + kh + i) * sbk + mi * sbn];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
}
// element v of lane l of a 32x32 accumulator tile
__device__ inline int acc_row(int v) { return (v >> 2) * 8 + ((threadIdx.x & 63) >> 5) * 4 + (v & 3); }
__device__ inline int acc_col() { return threadIdx.x & 31; }

// ------------------------------------------------------------------ features

// scales[q] = sqrt(sum / n) (1 when zero), q = b, p1, r_e, d, from per-block partials, by
// a TPB-thread workgroup in a fixed order
__device__ inline void reduce_scales(int64_t n, const double *part, int nblk, double *out) {
    __shared__ double red[TPB / 64][4];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < nblk; j += TPB)
        for (int q = 0; q < 4; ++q) s[q] += part[static_cast<int64_t>(q) * nblk + j];
    for (int q = 0; q < 4; ++q) {
        double v = s[q];
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < TPB / 64; ++w) t += red[w][threadIdx.x];
        const double r = sqrt(t / static_cast<double>(n));
        out[threadIdx.x] = r > 0.0 ? r : 1.0;
    }
}

// e, d, r_e = b - K e, K d per row (K from its column-major ELL copy: coalesced entries, the
// CSR rows' summation order); per-block partial sums of b^2, p1^2, r_e^2, d^2
__global__ __launch_bounds__(TPB) void k_gnn_prep(int64_t n, int width, const int32_t *ecol, const double *eval,
                                                  const double *b, const double *p1, const double *p2, double *e,
                                                  double *d, double *re, double *kd, double *part) {
    __shared__ double red[TPB / 64][4];
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i = static_cast<int64_t>(lb) * TPB + threadIdx.x;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < n) {
        double ke = 0.0, kdd = 0.0;
        for (int k = 0; k < width; ++k) {
            const int64_t o = static_cast<int64_t>(k) * n + i;
            const int32_t j = ecol[o];
            const double v = eval[o], a = p1[j], c = p2[j];
            ke += v * (2.0 * a - c);
            kdd += v * (a - c);
        }
        const double ei = 2.0 * p1[i] - p2[i], di = p1[i] - p2[i], ri = b[i] - ke;
        e[i] = ei;
        d[i] = di;
        re[i] = ri;
        kd[i] = kdd;
        s[0] = b[i] * b[i];
        s[1] = p1[i] * p1[i];
        s[2] = ri * ri;
        s[3] = di * di;
    }
    for (int q = 0; q < 4; ++q) {
        double v = s[q];
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < TPB / 64; ++w) t += red[w][threadIdx.x];
        part[static_cast<int64_t>(threadIdx.x) * gridDim.x + lb] = t;
    }
}

// the feature scales from k_gnn_prep's partials, by one workgroup
__global__ __launch_bounds__(TPB) void k_gnn_scales(int64_t n, const double *part, int nblk, double *scales) {
    reduce_scales(n, part, nblk, scales);
}

// ------------------------------------------------------------------ forward layers

// Z tile [TM x 128] in LDS: own h row and the mean of the neighbours' h rows
__device__ inline void build_z(bf16 *Z, int64_t r0, int64_t n, const float *h, const int32_t *adj_ptr,
                               const int32_t *adj_col) {
    for (int task = threadIdx.x; task < TM * (GH / 8); task += blockDim.x) {
        const int r = task / (GH / 8), c = (task % (GH / 8)) * 8;
        const int64_t i = r0 + r;
        float self[8], acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) self[q] = acc[q] = 0.0f;
        if (i < n) {
#pragma unroll
            for (int q = 0; q < 8; ++q) self[q] = h[i * GH + c + q];
            int deg = 0;
            for (int32_t k = adj_ptr[i]; k < adj_ptr[i + 1]; ++k) {
                const int32_t j = adj_col[k];
                if (j == i) continue;
                ++deg;
#pragma unroll
                for (int q = 0; q < 8; ++q) acc[q] += h[static_cast<int64_t>(j) * GH + c + q];
            }
            const float inv = deg > 0 ? 1.0f / static_cast<float>(deg) : 0.0f;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] *= inv;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            Z[r * (2 * GH) + c + q] = to_bf16(self[q]);
            Z[r * (2 * GH) + GH + c + q] = to_bf16(acc[q]);
        }
    }
}

// Forward layer, one wavefront per 32-row tile; a workgroup takes groups of four
// consecutive tiles (grid-stride, the same trip count for all its wavefronts; groups
// numbered so that every XCD takes a contiguous range, whose rows' mesh neighbours
// are then mostly in its own L2).  Global memory is read and written row-coalesced:
// lane l covers columns 4(l%16)..+3 of rows l/16 + 4k, k = 0..7, so that 16 lanes move
// one 256-byte row.  A 32 x 64 fp32 tile per wavefront in LDS turns these rows into the
// MFMA A operand (lane l: row l%32, columns 8(l/32)..+7 of each 16-wide k step), fed as
// its bfloat16 high part and remainder (two MFMAs per k step): first the rows' own
// activations, then their neighbour means, and finally takes the accumulators back to
// the row layout for the epilogue.  Neighbour lists come from the column-major table
// (lanes 0..31 load those of the tile's rows, a shuffle hands them to the row layout).
// Weights arrive transposed ([64 x K] bf16) and are shared through LDS rows padded by
// 16 bytes.
//   MODE 0  encoder: features of the row computed here from b, p1, p2, r_e, K d, d
//   MODE 1  message layer: h' = relu([h, mean_nbr h] W + c) + h
//   MODE 2  message layer + decoder: y = h' w_d + c_d, guess = e + s_d y on free nodes
struct FwdArgs {
    int64_t n;
    const int32_t *nbr;   // message layers: the mesh's neighbour table, width nbw (a multiple of NB)
    int nbw;
    const float *hin;
    const double *b, *p1, *p2, *re, *kd, *d, *e, *scales;
    const uint8_t *dir;
    const bf16 *wT;
    const float *bias;
    const float *wd;      // w_d [64] then c_d
    float *hout;
    float *aout;          // pre-activations (training) or null
    float *xout;          // encoder: features (training) or null
    float *yout;          // decoder: network output or null
    double *guess;        // decoder: guess or null
};

constexpr int FWD_WAVES = TPB / 64;
constexpr int ZS = GH + 4;   // padded row of a wavefront's 32 x 64 LDS tile (floats)

__device__ inline bf16x8 ld8(const bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

struct F8 {
    float v[8];
};
__device__ inline F8 ldf8(const float *p) {
    const float4 a = reinterpret_cast<const float4 *>(p)[0], b = reinterpret_cast<const float4 *>(p)[1];
    return F8{{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w}};
}
__device__ inline void stf8(float *p, const float (&v)[8]) {
    reinterpret_cast<float4 *>(p)[0] = make_float4(v[0], v[1], v[2], v[3]);
    reinterpret_cast<float4 *>(p)[1] = make_float4(v[4], v[5], v[6], v[7]);
}
__device__ inline float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ inline void st4(float *p, float4 v) { *reinterpret_cast<float4 *>(p) = v; }
__device__ inline float4 add4(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
// orders a wavefront's LDS writes before its later LDS reads (of other lanes' values): the
// accesses of one wavefront are performed in order, so only code motion has to be stopped
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// v = hi + lo with hi = bf16(v), lo = bf16(v - hi), by pairs (one conversion instruction per
// two values; the hi pair back in fp32 by a shift and a mask)
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ inline void split8(const float (&v)[8], bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
        const f32x2 x = {v[q], v[q + 1]};
        const bf16x2 h = __builtin_convertvector(x, bf16x2);
        const bf16x2 l = __builtin_convertvector(x - __builtin_convertvector(h, f32x2), bf16x2);
        hi[q] = h[0];
        hi[q + 1] = h[1];
        lo[q] = l[0];
        lo[q + 1] = l[1];
    }
}

// column c of activation row r, addressed as the buffer's base plus a 32-bit unsigned byte
// offset (activation buffers are smaller than 4 GiB, checked on the host), so that a load or
// store takes the kernel argument's base and one 32-bit register instead of a 64-bit pointer
// per lane
__device__ inline uint32_t row_off(int64_t r, int c) {
    return (static_cast<uint32_t>(r) * GH + static_cast<uint32_t>(c)) * static_cast<uint32_t>(sizeof(float));
}
__device__ inline float4 ld4o(const float *base, uint32_t off) {
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + off);
}
__device__ inline void st4o(float *base, uint32_t off, float4 v) {
    *reinterpret_cast<float4 *>(reinterpret_cast<char *>(base) + off) = v;
}

template <int MODE, int NB>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(3))) void k_gnn_fwd(FwdArgs A) {
    constexpr int K = MODE == 0 ? GFP : 2 * GH;
    constexpr int KP = K + 8;
    __shared__ __align__(16) bf16 Wl[GH * KP];
    __shared__ __align__(16) float Zt[FWD_WAVES][32 * ZS];
    __shared__ float ys[FWD_WAVES][32];   // decoder: the network output of the tile's rows
    for (int t = threadIdx.x; t < GH * (K / 8); t += TPB) {
        const int row = t / (K / 8), ch = t % (K / 8);
        *reinterpret_cast<bf16x8 *>(Wl + row * KP + ch * 8) = ld8(A.wT + row * K + ch * 8);
    }
    __syncthreads();
    const int l = threadIdx.x & 63, r = l & 31, half = l >> 5, wave = threadIdx.x >> 6;
    const int rg = l >> 4, c4 = (l & 15) * 4;   // row layout: rows rg + 4k, columns c4..c4+3
    float *Z = Zt[wave];
    const int64_t n = A.n, ntiles = (n + 31) / 32, ngroups = (ntiles + FWD_WAVES - 1) / FWD_WAVES;
    const double sd = MODE == 2 ? A.scales[3] : 0.0;
    for (int64_t g = xcd_block(blockIdx.x, gridDim.x); g < ngroups; g += gridDim.x) {
        const int64_t row0 = (g * FWD_WAVES + wave) * 32, i = row0 + r;
        const bool valid = i < n;
        // decoder: the row's extrapolation and Dirichlet flag, loaded now so that they arrive
        // with the layer's first loads
        double e_row = 0.0;
        bool dir_row = true;
        if (MODE == 2 && A.guess && valid && half == 0) {
            e_row = A.e[i];
            dir_row = A.dir[i] != 0;
        }
        // the two 32-column halves of the output accumulate over the k steps in order: the
        // row's own activations (k steps 0..3) before its neighbour mean (4..7)
        f32x16 c[2] = {};
        auto products = [&](const bf16x8 *ah, const bf16x8 *al, int s0, int s1) {
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int s = s0; s < s1; ++s) {
                    const bf16x8 w = ld8(Wl + (ct * 32 + r) * KP + 16 * s + 8 * half);
                    c[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s - s0], w, c[ct], 0, 0, 0);
                    c[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s - s0], w, c[ct], 0, 0, 0);
                }
        };
        // a 32 x 64 block of the tile in the operand layout, as high parts and remainders
        auto operands = [&](bf16x8 *ah, bf16x8 *al) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const F8 v = ldf8(Z + r * ZS + (2 * j + half) * 8);
                split8(v.v, ah[j], al[j]);
            }
        };
        if constexpr (MODE == 0) {
            float f[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            if (valid && half == 0) {
                const double sb = A.scales[0], sp = A.scales[1], sr = A.scales[2], sd = A.scales[3];
                f[0] = static_cast<float>(A.b[i] / sb);
                f[1] = static_cast<float>(A.p1[i] / sp);
                f[2] = static_cast<float>(A.p2[i] / sp);
                f[3] = static_cast<float>(A.re[i] / sr);
                f[4] = static_cast<float>(A.kd[i] / sr);
                f[5] = static_cast<float>(A.d[i] / sd);
                f[6] = static_cast<float>(A.dir[i]);
                f[7] = 1.0f;
            }
            bf16x8 ah[1], al[1];
            split8(f, ah[0], al[0]);
            if (A.xout && valid) stf8(A.xout + i * GFP + 8 * half, f);
            products(ah, al, 0, 1);
        } else {
            const float *h = A.hin;
            // the rows' own activations, through the tile into the operand layout (a row past
            // the end reads the zero row n)
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int64_t ir = row0 + rg + 4 * k;
                st4(Z + (rg + 4 * k) * ZS + c4, ld4o(h, row_off(ir < n ? ir : n, c4)));
            }
            wave_lds_sync();
            {
                bf16x8 ah[4], al[4];
                operands(ah, al);
                products(ah, al, 0, 4);
            }
            wave_lds_sync();
            // neighbour means, in table order; padding slots, and every slot of a row past the
            // end, name row n of h, which is zero
            if constexpr (NB > 0) {
                // a table of width NB: lanes 0..31 hold their row's neighbours, handed to the
                // row layout by a shuffle; two rows' gathers in flight at a time
                const int64_t ic = valid ? i : n - 1;
                int32_t nb[NB];
                int deg = 0;
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const int32_t v = A.nbr[static_cast<int64_t>(u) * n + ic];
                    nb[u] = valid ? v : static_cast<int32_t>(n);
                    deg += nb[u] != n ? 1 : 0;
                }
                const float inv_row = deg > 0 ? 1.0f / static_cast<float>(deg) : 0.0f;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    float4 v[NB];
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const int32_t j = __shfl(nb[u], rg + 4 * k, 64);
                        v[u] = ld4o(h, row_off(j, c4));
                    }
                    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                    for (int u = 0; u < NB; ++u) acc = add4(acc, v[u]);
                    const float inv = __shfl(inv_row, rg + 4 * k, 64);
                    st4(Z + (rg + 4 * k) * ZS + c4, make_float4(acc.x * inv, acc.y * inv, acc.z * inv, acc.w * inv));
                    if (k & 1) __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                // a wider table: the row-layout lanes walk their rows' slots themselves
#pragma unroll 1
                for (int k = 0; k < 8; ++k) {
                    const int64_t ir = row0 + rg + 4 * k;
                    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    int dg = 0;
                    for (int u = 0; u < A.nbw; ++u) {
                        const int32_t j = ir < n ? A.nbr[static_cast<int64_t>(u) * n + ir] : static_cast<int32_t>(n);
                        dg += j != n ? 1 : 0;
                        acc = add4(acc, ld4(h + static_cast<int64_t>(j) * GH + c4));
                    }
                    const float inv = dg > 0 ? 1.0f / static_cast<float>(dg) : 0.0f;
                    st4(Z + (rg + 4 * k) * ZS + c4, make_float4(acc.x * inv, acc.y * inv, acc.z * inv, acc.w * inv));
                }
            }
            wave_lds_sync();
            {
                bf16x8 ah[4], al[4];
                operands(ah, al);
                products(ah, al, 4, 8);
            }
            wave_lds_sync();
        }
        // the accumulators go back to the row layout through the tile
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int v = 0; v < 16; ++v) Z[acc_row(v) * ZS + ct * 32 + acc_col()] = c[ct][v];
        wave_lds_sync();
        const float4 bias = ld4(A.bias + c4);
        float4 wd = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if constexpr (MODE == 2) wd = ld4(A.wd + c4);
        // the residual input is read again (cache hits) rather than kept in registers, all
        // eight rows before the first store (which the compiler cannot move loads across); a
        // row past the end reads the zero row n
        float4 res[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t ir = row0 + rg + 4 * k;
            res[k] = MODE != 0 ? ld4o(A.hin, row_off(ir < n ? ir : n, c4)) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t ir = row0 + rg + 4 * k;
            const bool ok = ir < n;
            const float4 z = ld4(Z + (rg + 4 * k) * ZS + c4);
            const float4 pre = make_float4(z.x + bias.x, z.y + bias.y, z.z + bias.z, z.w + bias.w);
            float4 hv = make_float4(fmaxf(pre.x, 0.0f), fmaxf(pre.y, 0.0f), fmaxf(pre.z, 0.0f), fmaxf(pre.w, 0.0f));
            if constexpr (MODE != 0) hv = add4(hv, res[k]);
            if (ok) {
                st4o(A.hout, row_off(ir, c4), hv);
                if (A.aout) st4o(A.aout, row_off(ir, c4), pre);
            }
            if constexpr (MODE == 2) {
                float y = hv.x * wd.x + hv.y * wd.y + hv.z * wd.z + hv.w * wd.w;
#pragma unroll
                for (int m = 8; m >= 1; m >>= 1) y += __shfl_xor(y, m, 64);
                if ((l & 15) == 0) ys[wave][rg + 4 * k] = y + A.wd[GH];
            }
        }
        if constexpr (MODE == 2) {
            // output and guess row by row in the operand layout's lanes 0..31: coalesced
            wave_lds_sync();
            if (valid && half == 0) {
                const float y = ys[wave][r];
                if (A.yout) A.yout[i] = y;
                if (A.guess) A.guess[i] = dir_row ? 0.0 : e_row + sd * static_cast<double>(y);
            }
        }
        wave_lds_sync();   // the tile is written again by the next group
    }
}

__global__ void k_gnn_zero(float *p, int64_t count) {
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0.0f;
}

// one damped Jacobi sweep xout = xin + omega D^-1 (b - K xin); Dirichlet rows (identity, b = 0)
// keep their zero
// (the column-major ELL copy of K: coalesced entries, the same summation order as the CSR rows)
__global__ __launch_bounds__(TPB) void k_gnn_smooth(int64_t n, int width, const int32_t *ecol, const double *eval,
                                                    const double *dinv, const double *b, const double *xin,
                                                    double *xout, double omega) {
    const int64_t i = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * TPB + threadIdx.x;
    if (i >= n) return;
    double kx = 0.0;
    for (int k = 0; k < width; ++k) {
        const int64_t o = static_cast<int64_t>(k) * n + i;
        kx += eval[o] * xin[ecol[o]];
    }
    xout[i] = xin[i] + omega * dinv[i] * (b[i] - kx);
}

// All SMOOTH_SWEEPS sweeps in one launch: a workgroup per tile of the mesh's tiled
// partition for distance SMOOTH_SWEEPS holds the guess over the tile's region (the rows
// within graph distance SMOOTH_SWEEPS, own rows first, then by distance) in LDS; sweep k
// updates the rows at distance <= SMOOTH_SWEEPS - k from the previous sweep's values of
// their neighbours (two LDS buffers), so that the own rows end with the values of
// SMOOTH_SWEEPS global sweeps.  Local matrix rows: the tiles' 16-bit region columns and
// fp64 values in CSR order (padding: the row itself with value 0), as the ELL sweep sums.
constexpr int SM_BLOCK = TILE_ROWS;
template <int W>
__global__ __launch_bounds__(SM_BLOCK) void k_gnn_smooth_tiles(const TileBlk *blk, const int32_t *reg,
                                                               const uint16_t *ecol, const double *eval,
                                                               const double *dinv, const double *b,
                                                               const double *xin, double *xout, double omega) {
    constexpr int TH = TILE_REGION / SM_BLOCK, TS = TILE_SPMV / SM_BLOCK, CW = tile_col_stride(W);
    static_assert(TILE_OWN <= TS && TILE_OWN * SM_BLOCK == TILE_ROWS_MAX, "own rows are local matrix rows");
    __shared__ double xa[TILE_REGION], xb[TILE_REGION];
    __shared__ int32_t s_nt[TILE_MAX_DEGREE + 2];
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const TileBlk &B = blk[lb];
    const int nreg = B.nreg, nspmv = B.nspmv, nown = B.nt[0];
    if (threadIdx.x < TILE_MAX_DEGREE + 2) s_nt[threadIdx.x] = B.nt[threadIdx.x];
    int32_t g[TH];
#pragma unroll
    for (int h = 0; h < TH; ++h) {
        const int t = threadIdx.x + h * SM_BLOCK;
        g[h] = t < nreg ? reg[B.reg_off + t] : -1;
    }
    double bb[TS], dd[TS], ev[TS][W];
    uint16_t ec[TS][W];
#pragma unroll
    for (int h = 0; h < TS; ++h) {
        const int t = threadIdx.x + h * SM_BLOCK;
        bb[h] = dd[h] = 0.0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            ev[h][q] = 0.0;
            ec[h][q] = 0;
        }
        if (t < nspmv) {
            const size_t row = static_cast<size_t>(B.ell_off) + t;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                ec[h][q] = ecol[row * CW + q];
                ev[h][q] = eval[row * W + q];
            }
            bb[h] = b[g[h]];
            dd[h] = dinv[g[h]];
        }
    }
#pragma unroll
    for (int h = 0; h < TH; ++h) {
        const int t = threadIdx.x + h * SM_BLOCK;
        if (t < nreg) xa[t] = xin[g[h]];
    }
    __syncthreads();
    double *src = xa, *dst = xb;
    for (int k = 1; k <= SMOOTH_SWEEPS; ++k) {
        const int lim = s_nt[SMOOTH_SWEEPS - k];
#pragma unroll
        for (int h = 0; h < TS; ++h) {
            const int t = threadIdx.x + h * SM_BLOCK;
            if (t < lim) {
                double kx = 0.0;
#pragma unroll
                for (int q = 0; q < W; ++q) kx += ev[h][q] * src[ec[h][q]];
                dst[t] = src[t] + omega * dd[h] * (bb[h] - kx);
            }
        }
        __syncthreads();
        double *tmp = src;
        src = dst;
        dst = tmp;
    }
#pragma unroll
    for (int h = 0; h < TILE_OWN; ++h) {
        const int t = threadIdx.x + h * SM_BLOCK;
        if (t < nown) xout[g[h]] = src[t];
    }
}

// ------------------------------------------------------------------ training

// delta = (y - (target - e)/s_d) on free nodes
__global__ __launch_bounds__(TPB) void k_gnn_delta(int64_t n, const float *y, const double *target, const double *e,
                                                   const double *scales, const uint8_t *dir, double *delta) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * TPB + threadIdx.x;
    if (i >= n) return;
    delta[i] = dir[i] ? 0.0 : static_cast<double>(y[i]) - (target[i] - e[i]) / scales[3];
}

// dy = 2 K delta / N_free on free nodes; per-block partial of delta.K delta
__global__ __launch_bounds__(TPB) void k_gnn_dy(int64_t n, const int32_t *rowptr, const int32_t *col,
                                                const double *val, const double *delta, const uint8_t *dir,
                                                double nfree, float *dy, double *lpart) {
    __shared__ double red[TPB / 64];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * TPB + threadIdx.x;
    double l = 0.0;
    if (i < n) {
        double kd = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) kd += val[k] * delta[col[k]];
        dy[i] = dir[i] ? 0.0f : static_cast<float>(2.0 * kd / nfree);
        l = delta[i] * kd;
    }
    for (int m = 32; m >= 1; m >>= 1) l += __shfl_xor(l, m, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < TPB / 64; ++w) t += red[w];
        lpart[blockIdx.x] = t;
    }
}

// loss = sum(lpart) / N_free, added to *out
__global__ void k_gnn_loss(const double *lpart, int nblk, double nfree, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double t = 0.0;
    for (int j = 0; j < nblk; ++j) t += lpart[j];
    *out += t / nfree;
}

// dh3 = dy w_d^T; partials of h3^T dy (64) and sum(dy) (1) per block: gpart[blk][65]
__global__ __launch_bounds__(TPB) void k_gnn_dec_bwd(int64_t n, const float *dy, const float *h, const float *theta,
                                                     float *dh, float *gpart) {
    __shared__ float red[TPB / 64][GH + 1];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * TPB + threadIdx.x;
    const float g = i < n ? dy[i] : 0.0f;
    for (int q = 0; q <= GH; ++q) {
        float v;
        if (q < GH) {
            if (i < n) dh[i * GH + q] = g * theta[P_WD + q];
            v = i < n ? h[i * GH + q] * g : 0.0f;
        } else {
            v = g;
        }
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x <= GH) {
        float t = 0.0f;
        for (int w = 0; w < TPB / 64; ++w) t += red[w][threadIdx.x];
        gpart[static_cast<int64_t>(blockIdx.x) * (GH + 1) + threadIdx.x] = t;
    }
}

// message layer backward for BW_SUB*TM rows: da = dh * (a > 0);
// dW partial = Z^T bf16(da), dc partial = colsum(da); dZ = bf16(da) W^T ->
// dhp = dh + dZ[:, :64], dm = dZ[:, 64:] / deg
__global__ __launch_bounds__(TPB) void k_gnn_layer_bwd(int64_t n, const float *hin, const int32_t *adj_ptr,
                                                       const int32_t *adj_col, const bf16 *W, const float *a,
                                                       const float *dh, float *dhp, float *dm, float *gpart) {
    constexpr int K = 2 * GH;
    __shared__ bf16 Z[TM * K];
    __shared__ bf16 Ws[K * GH];
    __shared__ bf16 Dq[TM * GH];
    __shared__ float Df[TM * GH];
    __shared__ int deg_s[TM];
    for (int t = threadIdx.x; t < K * GH; t += TPB) Ws[t] = W[t];
    const int wave = threadIdx.x >> 6;
    f32x16 gw0 = {}, gw1 = {};         // dW tiles (rows wave*32.., cols 0..31 / 32..63)
    float dc = 0.0f;                   // column threadIdx.x (< 64) sum of da
    for (int sub = 0; sub < BW_SUB; ++sub) {
        const int64_t r0 = (static_cast<int64_t>(blockIdx.x) * BW_SUB + sub) * TM;
        build_z(Z, r0, n, hin, adj_ptr, adj_col);
        for (int t = threadIdx.x; t < TM * GH; t += TPB) {
            const int64_t i = r0 + t / GH;
            const float v = (i < n && a[r0 * GH + t] > 0.0f) ? dh[r0 * GH + t] : 0.0f;
            Df[t] = v;
            Dq[t] = to_bf16(v);
        }
        for (int r = threadIdx.x; r < TM; r += TPB) {
            const int64_t i = r0 + r;
            int dg = 0;
            if (i < n)
                for (int32_t k = adj_ptr[i]; k < adj_ptr[i + 1]; ++k) dg += adj_col[k] != i;
            deg_s[r] = dg;
        }
        __syncthreads();
        if (threadIdx.x < GH)
            for (int r = 0; r < TM; ++r) dc += Df[r * GH + threadIdx.x];
        // dW += Z^T Dq  (K = rows of the sub-tile)
        mfma_tile(gw0, Z + wave * 32, 1, K, Dq, GH, 1, TM);
        mfma_tile(gw1, Z + wave * 32, 1, K, Dq + 32, GH, 1, TM);
        // dZ = Dq W^T: output [TM x 128]; wave: row tile (wave>>1)*32, column tiles 2*(wave&1), +1
        const int tr = (wave >> 1) * 32;
        for (int ct = 0; ct < 2; ++ct) {
            const int tc = (2 * (wave & 1) + ct) * 32;
            f32x16 acc = {};
            mfma_tile(acc, Dq + tr * GH, GH, 1, Ws + tc * GH, 1, GH, GH);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = tr + acc_row(v), colx = tc + acc_col();
                const int64_t i = r0 + row;
                if (i >= n) continue;
                if (colx < GH)
                    dhp[i * GH + colx] = dh[i * GH + colx] + acc[v];
                else
                    dm[i * GH + colx - GH] = deg_s[row] > 0 ? acc[v] / static_cast<float>(deg_s[row]) : 0.0f;
            }
        }
        __syncthreads();
    }
    float *g = gpart + static_cast<int64_t>(blockIdx.x) * (K * GH + GH);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = wave * 32 + acc_row(v), colx = acc_col();
        g[row * GH + colx] = gw0[v];
        g[row * GH + 32 + colx] = gw1[v];
    }
    if (threadIdx.x < GH) g[K * GH + threadIdx.x] = dc;
}

// dh_prev_j = dhp_j + sum over neighbours i of dm_i (the mean's transpose; adjacency is symmetric)
__global__ __launch_bounds__(TPB) void k_gnn_agg_bwd(int64_t n, const int32_t *adj_ptr, const int32_t *adj_col,
                                                     const float *dhp, const float *dm, float *dh) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * TPB + threadIdx.x;
    const int64_t j = t / (GH / 8);
    if (j >= n) return;
    const int c = static_cast<int>(t % (GH / 8)) * 8;
    float s[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] = dhp[j * GH + c + q];
    for (int32_t k = adj_ptr[j]; k < adj_ptr[j + 1]; ++k) {
        const int32_t i = adj_col[k];
        if (i == j) continue;
#pragma unroll
        for (int q = 0; q < 8; ++q) s[q] += dm[static_cast<int64_t>(i) * GH + c + q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) dh[j * GH + c + q] = s[q];
}

// encoder backward for BW_SUB*TM rows: partials of X^T bf16(da0) (16x64) and colsum(da0)
__global__ __launch_bounds__(TPB) void k_gnn_enc_bwd(int64_t n, const float *x, const float *a, const float *dh,
                                                     float *gpart) {
    __shared__ float Xs[TM * GFP];
    __shared__ float Dq[TM * GH];
    __shared__ float Df[TM * GH];
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // outputs threadIdx.x + 256 q of the 16x64 block
    float dc = 0.0f;
    for (int sub = 0; sub < BW_SUB; ++sub) {
        const int64_t r0 = (static_cast<int64_t>(blockIdx.x) * BW_SUB + sub) * TM;
        for (int t = threadIdx.x; t < TM * GFP; t += TPB) {
            const int64_t i = r0 + t / GFP;
            Xs[t] = i < n ? from_bf16(to_bf16(x[r0 * GFP + t])) : 0.0f;
        }
        for (int t = threadIdx.x; t < TM * GH; t += TPB) {
            const int64_t i = r0 + t / GH;
            const float v = (i < n && a[r0 * GH + t] > 0.0f) ? dh[r0 * GH + t] : 0.0f;
            Df[t] = v;
            Dq[t] = from_bf16(to_bf16(v));
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int o = threadIdx.x + TPB * q, k = o / GH, c = o % GH;
            for (int r = 0; r < TM; ++r) acc[q] += Xs[r * GFP + k] * Dq[r * GH + c];
        }
        if (threadIdx.x < GH)
            for (int r = 0; r < TM; ++r) dc += Df[r * GH + threadIdx.x];
        __syncthreads();
    }
    float *g = gpart + static_cast<int64_t>(blockIdx.x) * (GFP * GH + GH);
#pragma unroll
    for (int q = 0; q < 4; ++q) g[threadIdx.x + TPB * q] = acc[q];
    if (threadIdx.x < GH) g[GFP * GH + threadIdx.x] = dc;
}

// grad[off + p] = sum over blocks of gpart[blk * stride + p], p < count (fixed order)
__global__ __launch_bounds__(TPB) void k_gnn_reduce(const float *gpart, int nblk, int stride, int count, float *grad,
                                                    int off) {
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= count) return;
    float t = 0.0f;
    for (int b = 0; b < nblk; ++b) t += gpart[static_cast<int64_t>(b) * stride + p];
    grad[off + p] = t;
}

// the same sum in two passes when there are many blocks: range c of the blocks ([c nblk / RED_CHUNKS,
// (c + 1) nblk / RED_CHUNKS), in order) by workgroup row c, then the RED_CHUNKS range sums in order
// by k_gnn_reduce; a fixed order either way, with RED_CHUNKS times the workgroups streaming the partials
constexpr int RED_CHUNKS = 32;
__global__ __launch_bounds__(TPB) void k_gnn_reduce_chunks(const float *gpart, int nblk, int stride, int count,
                                                           float *part) {
    const int p = blockIdx.x * TPB + threadIdx.x, c = blockIdx.y;
    if (p >= count) return;
    const int b0 = static_cast<int>(static_cast<int64_t>(c) * nblk / RED_CHUNKS);
    const int b1 = static_cast<int>(static_cast<int64_t>(c + 1) * nblk / RED_CHUNKS);
    float t = 0.0f;
    for (int b = b0; b < b1; ++b) t += gpart[static_cast<int64_t>(b) * stride + p];
    part[static_cast<int64_t>(c) * count + p] = t;
}

// Adam on the fp32 master weights, then the bf16 copies of the matrices
__global__ __launch_bounds__(TPB) void k_gnn_adam(float *theta, float *m1, float *m2, const float *grad, float lr,
                                                  float b1, float b2, float c1, float c2, float eps) {
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= P_COUNT) return;
    const float g = grad[p];
    const float m = b1 * m1[p] + (1.0f - b1) * g;
    const float v = b2 * m2[p] + (1.0f - b2) * g * g;
    m1[p] = m;
    m2[p] = v;
    theta[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// bf16 copies of the weight matrices: row-major (backward) and transposed (forward)
__global__ __launch_bounds__(TPB) void k_gnn_quantize(const float *theta, bf16 *wq, bf16 *wqT) {
    const int q = blockIdx.x * TPB + threadIdx.x;
    if (q >= Q_COUNT) return;
    int src, srcT;
    if (q < GFP * GH) {
        src = P_W0 + q;
        srcT = P_W0 + (q % GFP) * GH + q / GFP;
    } else {
        const int l = (q - GFP * GH) / (2 * GH * GH), o = (q - GFP * GH) % (2 * GH * GH);
        src = P_L0 + l * P_LSTRIDE + o;
        srcT = P_L0 + l * P_LSTRIDE + (o % (2 * GH)) * GH + o / (2 * GH);
    }
    wq[q] = to_bf16(theta[src]);
    wqT[q] = to_bf16(theta[srcT]);
}

// ------------------------------------------------------------------ host side

GnnWork &work_for(hipStream_t s, Model &md, const Mesh &m, bool training) {
    auto &slot = md.work[&m];
    if (!slot) slot = std::make_unique<GnnWork>();
    GnnWork &w = *slot;
    const int64_t n = m.lv[0].n;
    if (w.n != n) {
        w = GnnWork();
        w.n = n;
        w.e.alloc(n);
        w.d.alloc(n);
        w.re.alloc(n);
        w.kd.alloc(n);
        w.part.alloc(4 * blocks_for(n, TPB));
        w.scales.alloc(4);
        w.x.alloc(n * GFP);
        for (auto &h : w.h) {
            h.alloc((n + 1) * GH);
            hipLaunchKernelGGL(k_gnn_zero, dim3(1), dim3(GH), 0, s, h.p + n * GH, static_cast<int64_t>(GH));
        }
        CGP_HIP(hipGetLastError());
        w.y.alloc(n);
    }
    if (training && w.dy.n == 0) {
        for (auto &a : w.a) a.alloc(n * GH);
        w.delta.alloc(n);
        w.dy.alloc(n);
        w.dh.alloc(n * GH);
        w.dhp.alloc(n * GH);
        w.dm.alloc(n * GH);
        const int64_t nbw = (n + BW_SUB * TM - 1) / (BW_SUB * TM);
        w.gpart.alloc(std::max<int64_t>(nbw * (2 * GH * GH + GH), blocks_for(n, TPB) * (GH + 1)));
        w.grad.alloc(P_COUNT);
        w.gred.alloc(static_cast<size_t>(RED_CHUNKS) * (2 * GH * GH + GH));
        w.lpart.alloc(blocks_for(n, TPB));
    }
    return w;
}

// features + forward; x, a[] and y saved when training; guess written when non-null
void forward(hipStream_t s, Model &md, const Mesh &m, GnnWork &w, const double *b, const double *p1,
             const double *p2, double *guess, bool training, const TilePlan *smooth_plan = nullptr) {
    const int64_t n = m.lv[0].n;
    const unsigned nb = blocks_for(n, TPB);
    hipLaunchKernelGGL(k_gnn_prep, dim3(nb), dim3(TPB), 0, s, n, m.max_row, m.ell_col.p, m.ell_val.p, b, p1, p2,
                       w.e.p, w.d.p, w.re.p, w.kd.p, w.part.p);
    hipLaunchKernelGGL(k_gnn_scales, dim3(1), dim3(TPB), 0, s, n, w.part.p, static_cast<int>(nb), w.scales.p);
    CGP_REQUIRE((n + 1) * GH * static_cast<int64_t>(sizeof(float)) <= static_cast<int64_t>(UINT32_MAX),
                "mesh too large for the network's activations");
    const int64_t ngroups = ((n + 31) / 32 + FWD_WAVES - 1) / FWD_WAVES;
    // one workgroup per group of tiles (capping the grid at 2048 workgroups of about two groups
    // each, to load the weights into LDS fewer times, measured 3 % slower at 525825 rows)
    const unsigned nf = static_cast<unsigned>(ngroups);
    const float *th = md.theta.p;
    FwdArgs A{};
    A.n = n;
    A.nbr = m.nbr.p;
    A.nbw = m.nbr_w;
    A.b = b;
    A.p1 = p1;
    A.p2 = p2;
    A.re = w.re.p;
    A.kd = w.kd.p;
    A.d = w.d.p;
    A.e = w.e.p;
    A.scales = w.scales.p;
    A.dir = m.lv[0].dir.p;
    A.wd = th + P_WD;
    A.wT = md.wqT.p + Q_W0;
    A.bias = th + P_C0;
    A.hout = w.h[0].p;
    A.aout = training ? w.a[0].p : nullptr;
    A.xout = training ? w.x.p : nullptr;
    hipLaunchKernelGGL((k_gnn_fwd<0, 0>), dim3(nf), dim3(TPB), 0, s, A);
    const int nbw = m.nbr_w == NBR_NARROW ? NBR_NARROW : m.nbr_w == NBR_WIDE ? NBR_WIDE : 0;
    A.xout = nullptr;
    for (int l = 1; l <= GL; ++l) {
        A.hin = w.h[l - 1].p;
        A.hout = w.h[l].p;
        A.aout = training ? w.a[l].p : nullptr;
        A.wT = md.wqT.p + GFP * GH + (l - 1) * 2 * GH * GH;
        A.bias = th + P_L0 + (l - 1) * P_LSTRIDE + 2 * GH * GH;
        if (l < GL) {
            if (nbw == NBR_NARROW)
                hipLaunchKernelGGL((k_gnn_fwd<1, NBR_NARROW>), dim3(nf), dim3(TPB), 0, s, A);
            else if (nbw == NBR_WIDE)
                hipLaunchKernelGGL((k_gnn_fwd<1, NBR_WIDE>), dim3(nf), dim3(TPB), 0, s, A);
            else
                hipLaunchKernelGGL((k_gnn_fwd<1, 0>), dim3(nf), dim3(TPB), 0, s, A);
        } else {
            A.yout = w.y.p;
            // with a tiled plan the raw guess goes to re (no longer needed) and the one-launch
            // smoothing writes the result into guess
            A.guess = guess && smooth_plan ? w.re.p : guess;
            if (nbw == NBR_NARROW)
                hipLaunchKernelGGL((k_gnn_fwd<2, NBR_NARROW>), dim3(nf), dim3(TPB), 0, s, A);
            else if (nbw == NBR_WIDE)
                hipLaunchKernelGGL((k_gnn_fwd<2, NBR_WIDE>), dim3(nf), dim3(TPB), 0, s, A);
            else
                hipLaunchKernelGGL((k_gnn_fwd<2, 0>), dim3(nf), dim3(TPB), 0, s, A);
        }
    }
    if (guess && smooth_plan) {
        const TilePlan &P = *smooth_plan;
        if (P.width == 8)
            hipLaunchKernelGGL(k_gnn_smooth_tiles<8>, dim3(P.nparts), dim3(SM_BLOCK), 0, s, P.blk.p, P.reg.p, P.ecol.p,
                               P.eval64.p, m.dinv.p, b, w.re.p, guess, SMOOTH_OMEGA);
        else
            hipLaunchKernelGGL(k_gnn_smooth_tiles<12>, dim3(P.nparts), dim3(SM_BLOCK), 0, s, P.blk.p, P.reg.p,
                               P.ecol.p, P.eval64.p, m.dinv.p, b, w.re.p, guess, SMOOTH_OMEGA);
        CGP_HIP(hipGetLastError());
        return;
    }
    // else one launch per sweep, ping-pong through re (no longer needed): an even number of
    // sweeps ends in guess
    static_assert(SMOOTH_SWEEPS % 2 == 0, "sweeps must end in the guess buffer");
    for (int q = 0; guess && q < SMOOTH_SWEEPS; ++q) {
        const double *xin = (q & 1) ? w.re.p : guess;
        double *xout = (q & 1) ? guess : w.re.p;
        hipLaunchKernelGGL(k_gnn_smooth, dim3(nb), dim3(TPB), 0, s, n, m.max_row, m.ell_col.p, m.ell_val.p,
                           m.dinv.p, b, xin, xout, SMOOTH_OMEGA);
    }
    CGP_HIP(hipGetLastError());
}

double count_free(hipStream_t s, const Mesh &m) {
    std::vector<uint8_t> d(m.lv[0].n);
    CGP_HIP(hipMemcpyAsync(d.data(), m.lv[0].dir.p, d.size(), hipMemcpyDeviceToHost, s));
    CGP_HIP(hipStreamSynchronize(s));
    double f = 0.0;
    for (uint8_t v : d) f += v ? 0.0 : 1.0;
    return f > 0.0 ? f : 1.0;
}

// w.grad[off + p] = the fixed-order sum of the nblk partials of gradient entry p
void reduce_grad(hipStream_t s, GnnWork &w, int nblk, int stride, int count, int off) {
    if (nblk <= 2 * RED_CHUNKS) {
        hipLaunchKernelGGL(k_gnn_reduce, dim3(blocks_for(count, TPB)), dim3(TPB), 0, s, w.gpart.p, nblk, stride, count,
                           w.grad.p, off);
        return;
    }
    hipLaunchKernelGGL(k_gnn_reduce_chunks, dim3(blocks_for(count, TPB), RED_CHUNKS), dim3(TPB), 0, s, w.gpart.p, nblk,
                       stride, count, w.gred.p);
    hipLaunchKernelGGL(k_gnn_reduce, dim3(blocks_for(count, TPB)), dim3(TPB), 0, s, w.gred.p, RED_CHUNKS, count, count,
                       w.grad.p, off);
}

// one sample: forward, loss (added to *loss_dev), gradient into w.grad
void loss_grad(hipStream_t s, Model &md, const Mesh &m, GnnWork &w, const double *b, const double *p1,
               const double *p2, const double *target, double nfree, double *loss_dev) {
    const int64_t n = m.lv[0].n;
    const unsigned nb = blocks_for(n, TPB);
    forward(s, md, m, w, b, p1, p2, nullptr, true);
    hipLaunchKernelGGL(k_gnn_delta, dim3(nb), dim3(TPB), 0, s, n, w.y.p, target, w.e.p, w.scales.p,
                       m.lv[0].dir.p, w.delta.p);
    hipLaunchKernelGGL(k_gnn_dy, dim3(nb), dim3(TPB), 0, s, n, m.rowptr.p, m.col.p, m.val.p, w.delta.p,
                       m.lv[0].dir.p, nfree, w.dy.p, w.lpart.p);
    hipLaunchKernelGGL(k_gnn_loss, dim3(1), dim3(64), 0, s, w.lpart.p, static_cast<int>(nb), nfree, loss_dev);
    // decoder
    hipLaunchKernelGGL(k_gnn_dec_bwd, dim3(nb), dim3(TPB), 0, s, n, w.dy.p, w.h[GL].p, md.theta.p, w.dh.p,
                       w.gpart.p);
    reduce_grad(s, w, static_cast<int>(nb), GH + 1, GH + 1, P_WD);
    const unsigned nbw = static_cast<unsigned>((n + BW_SUB * TM - 1) / (BW_SUB * TM));
    const int lstride = 2 * GH * GH + GH;
    for (int l = GL; l >= 1; --l) {
        hipLaunchKernelGGL(k_gnn_layer_bwd, dim3(nbw), dim3(TPB), 0, s, n, w.h[l - 1].p, m.adj_ptr.p, m.adj_col.p,
                           md.wq.p + GFP * GH + (l - 1) * 2 * GH * GH, w.a[l].p, w.dh.p, w.dhp.p, w.dm.p,
                           w.gpart.p);
        reduce_grad(s, w, static_cast<int>(nbw), lstride, lstride, P_L0 + (l - 1) * P_LSTRIDE);
        hipLaunchKernelGGL(k_gnn_agg_bwd, dim3(blocks_for(n * (GH / 8), TPB)), dim3(TPB), 0, s, n, m.adj_ptr.p,
                           m.adj_col.p, w.dhp.p, w.dm.p, w.dh.p);
    }
    hipLaunchKernelGGL(k_gnn_enc_bwd, dim3(nbw), dim3(TPB), 0, s, n, w.x.p, w.a[0].p, w.dh.p, w.gpart.p);
    reduce_grad(s, w, static_cast<int>(nbw), GFP * GH + GH, GFP * GH + GH, P_W0);
    CGP_HIP(hipGetLastError());
}

uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double gauss(uint64_t &st) {
    const double u1 = (static_cast<double>(splitmix64(st) >> 11) + 0.5) / 9007199254740992.0;
    const double u2 = (static_cast<double>(splitmix64(st) >> 11) + 0.5) / 9007199254740992.0;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

void upload_params(hipStream_t s, Model &md, const float *h) {
    CGP_HIP(hipMemcpyAsync(md.theta.p, h, P_COUNT * sizeof(float), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_gnn_quantize, dim3(blocks_for(Q_COUNT, TPB)), dim3(TPB), 0, s, md.theta.p, md.wq.p,
                       md.wqT.p);
    CGP_HIP(hipGetLastError());
    CGP_HIP(hipStreamSynchronize(s));
}

}  // namespace

int64_t gnn_param_count() { return P_COUNT; }

Model *gnn_create(hipStream_t s, uint64_t seed) {
    auto md = std::make_unique<Model>();
    md->theta.alloc(P_COUNT);
    md->m1.alloc(P_COUNT);
    md->m2.alloc(P_COUNT);
    md->wq.alloc(Q_COUNT);
    md->wqT.alloc(Q_COUNT);
    CGP_HIP(hipMemsetAsync(md->m1.p, 0, P_COUNT * sizeof(float), s));
    CGP_HIP(hipMemsetAsync(md->m2.p, 0, P_COUNT * sizeof(float), s));
    // He-normal weights (std sqrt(2 / fan_in)) from a splitmix64 stream; zero biases;
    // a small decoder so the first guesses stay close to the extrapolation
    std::vector<float> h(P_COUNT, 0.0f);
    uint64_t st = seed;
    for (int k = 0; k < GF; ++k)
        for (int c = 0; c < GH; ++c) h[P_W0 + k * GH + c] = static_cast<float>(gauss(st) * std::sqrt(2.0 / GF));
    for (int l = 0; l < GL; ++l)
        for (int q = 0; q < 2 * GH * GH; ++q)
            h[P_L0 + l * P_LSTRIDE + q] = static_cast<float>(gauss(st) * std::sqrt(2.0 / (2 * GH)) * 0.5);
    for (int q = 0; q < GH; ++q) h[P_WD + q] = static_cast<float>(gauss(st) * 0.01);
    upload_params(s, *md, h.data());
    return md.release();
}

void gnn_set_params(hipStream_t s, Model &md, const float *h) {
    upload_params(s, md, h);
    CGP_HIP(hipMemsetAsync(md.m1.p, 0, P_COUNT * sizeof(float), s));
    CGP_HIP(hipMemsetAsync(md.m2.p, 0, P_COUNT * sizeof(float), s));
    md.step = 0;
}

void gnn_get_params(hipStream_t s, Model &md, float *h) {
    CGP_HIP(hipMemcpyAsync(h, md.theta.p, P_COUNT * sizeof(float), hipMemcpyDeviceToHost, s));
    CGP_HIP(hipStreamSynchronize(s));
}

void gnn_predict(hipStream_t s, Model &md, Mesh &m, const double *b, const double *p1, const double *p2,
                 double *guess, bool build) {
    GnnWork &w = work_for(s, md, m, false);
    // the tiled partition for the smoothing's distance (shared with the solver's plans of that
    // degree), built on first use where that may synchronise the stream
    const auto &cached = m.tiles[SMOOTH_SWEEPS];
    const TilePlan *plan = build ? tile_plan(s, m, SMOOTH_SWEEPS)
                                 : (cached && cached->nparts > 0 ? cached.get() : nullptr);
    forward(s, md, m, w, b, p1, p2, guess, false, plan);
}

void gnn_grad(hipStream_t s, Model &md, const Mesh &m, const double *b, const double *p1, const double *p2,
              const double *target, double *h_loss, float *h_grad) {
    GnnWork &w = work_for(s, md, m, true);
    const double nfree = count_free(s, m);
    DBuf<double> loss;
    loss.alloc(1);
    CGP_HIP(hipMemsetAsync(loss.p, 0, sizeof(double), s));
    loss_grad(s, md, m, w, b, p1, p2, target, nfree, loss.p);
    if (h_loss) CGP_HIP(hipMemcpyAsync(h_loss, loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
    if (h_grad) CGP_HIP(hipMemcpyAsync(h_grad, w.grad.p, P_COUNT * sizeof(float), hipMemcpyDeviceToHost, s));
    CGP_HIP(hipStreamSynchronize(s));
}

void gnn_train(hipStream_t s, Model &md, const Mesh &m, int n_samples, const double *const *b,
               const double *const *p1, const double *const *p2, const double *const *target, int epochs,
               double lr, uint64_t seed, double *h_loss) {
    GnnWork &w = work_for(s, md, m, true);
    const double nfree = count_free(s, m);
    DBuf<double> losses;
    losses.alloc(epochs);
    CGP_HIP(hipMemsetAsync(losses.p, 0, epochs * sizeof(double), s));
    std::vector<int> order(n_samples);
    for (int i = 0; i < n_samples; ++i) order[i] = i;
    uint64_t st = seed;
    const float b1 = 0.9f, b2 = 0.999f;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = n_samples - 1; i > 0; --i) std::swap(order[i], order[splitmix64(st) % (i + 1)]);
        for (int k = 0; k < n_samples; ++k) {
            const int q = order[k];
            loss_grad(s, md, m, w, b[q], p1[q], p2[q], target[q], nfree, losses.p + ep);
            ++md.step;
            const float c1 = 1.0f - std::pow(b1, static_cast<float>(md.step));
            const float c2 = 1.0f - std::pow(b2, static_cast<float>(md.step));
            hipLaunchKernelGGL(k_gnn_adam, dim3(blocks_for(P_COUNT, TPB)), dim3(TPB), 0, s, md.theta.p, md.m1.p,
                               md.m2.p, w.grad.p, static_cast<float>(lr), b1, b2, c1, c2, 1e-8f);
            hipLaunchKernelGGL(k_gnn_quantize, dim3(blocks_for(Q_COUNT, TPB)), dim3(TPB), 0, s, md.theta.p,
                               md.wq.p, md.wqT.p);
            CGP_HIP(hipGetLastError());
        }
    }
    std::vector<double> hl(epochs);
    CGP_HIP(hipMemcpyAsync(hl.data(), losses.p, epochs * sizeof(double), hipMemcpyDeviceToHost, s));
    CGP_HIP(hipStreamSynchronize(s));
    if (h_loss)
        for (int e = 0; e < epochs; ++e) h_loss[e] = hl[e] / n_samples;
}

void gnn_release_mesh(Model &md, const Mesh *m) { md.work.erase(m); }

void gnn_destroy(Model *md) { delete md; }

}  // namespace cgp
