// Learned temporal-block preconditioner for the GMRES solve of V_h w = b
// (not in the paper, whose GMRES is unpreconditioned, Section 5).
//
// A small FP32 multilayer perceptron maps the local space-time neighbourhood
// of a residual to a correction.  With u = r / (D s) (D_k the diagonal entry
// of V_h: same triangle, same step; s the root-mean-square of r / D) the
// features of the DOF (step j, triangle k) are, for the lags f = 0 .. FT-1
// (0 before the first step),
//   x_{3f}     = u(j - f, k),
//   x_{3f + 1} = mean of u(j - f, k') over the 3 edge neighbours k' of k,
//   x_{3f + 2} = mean of u(j - f, k'') over the neighbours k'' of those
//                neighbours, k'' != k (the second ring, with multiplicity),
// and the correction is z(j, k) = s (c . x + N(x)) with
//   N(x) = w3 . tanh(W2^T tanh(W1^T x))   (no biases: N is odd),
// c . x a linear space-time stencil.  c is the least-squares fit of the
// pairs (convex: the same c for every seed); N is then trained on what c
// leaves, so the stencil is the deterministic part of the map and the
// perceptron a correction to it.  With hidden width 0 the preconditioner is
// the stencil alone.
// The rings are symmetric in the neighbours, so N does not depend on how
// the mesh numbers its triangles or orders their edges.  V_h is block
// lower-triangular in time, so the history carries the temporal part of
// V_h^{-1}; N(x) = x_0 would be Jacobi.  Training pairs (r, e) with V_h e = r come from the library's own
// FP64 GMRES solves: e = x* - x_k and r = b - V_h x_k at snapshot
// iterations k.  Training (mean-squared error on normalised pairs, Adam)
// and inference are hand-written FP32 kernels below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pfmm.h"

using namespace pfmm;

struct pfmm_precond {
    int device = 0;
    int FT = 8;              // time lags
    int F = 24, H = 256;     // all features (3 rings x FT lags), hidden width
    float* W1 = nullptr;     // F x H
    float* W2 = nullptr;     // H x H
    float* w3 = nullptr;     // H
    float* wl = nullptr;     // F: the linear stencil c (zero until trained)
    float* W1p = nullptr;    // packed for inference: Fp x Hp (Fp = F rounded up to 4)
    float* W2t = nullptr;    // Hp x Hp (FP32, transposed)
    float* w3p = nullptr;    // Hp
    int Hp = 256;            // padded hidden width (64, 128 or 256)
    std::vector<void*> owned;
    float last_loss = 0.f;
};

namespace {

constexpr int kT = 256;          // threads per block

#define HIP_CHECK(expr)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return set_error(PFMM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

template <class T>
pfmm_status palloc(std::vector<void*>& owned, T** p, size_t n) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, n * sizeof(T));
    if (e != hipSuccess) return set_error(PFMM_ENOMEM, std::string("preconditioner: ") + hipGetErrorString(e));
    owned.push_back(q);
    *p = (T*)q;
    return PFMM_OK;
}

// splitmix64 (Steele, Lea, Flood): counter-based random numbers
__device__ __host__ inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

constexpr int kRings = 3;        // features per time lag: the triangle, first ring, second ring

// The three normalised fields of a residual r at DOF i (natural order
// i = j E_x + k), scaled by inv = 1 / s: u(i) = r_i / D_k, the mean of u over
// the edge neighbours of k and over their neighbours other than k (same
// step).  Feature 3 f + ring of DOF i is field `ring` at DOF i - f E_x
// (0 before the first step).
__device__ __forceinline__ float ring_field(const double* __restrict__ r, const double* __restrict__ D, int64_t i,
                                            int64_t ex, int ring, const int* __restrict__ adj, double inv) {
    const int64_t j = i / ex;
    const int k = (int)(i - j * ex);
    const double* rj = r + j * ex;
    double a = 0.0;
    if (ring == 0) {
        a = rj[k] / D[k];
    } else if (ring == 1) {
        for (int e = 0; e < 3; ++e) {
            const int q = adj[3 * k + e];
            a += rj[q] / D[q];
        }
        a *= 1.0 / 3.0;
    } else {
        int c = 0;
        for (int e = 0; e < 3; ++e) {
            const int q = adj[3 * k + e];
            for (int g = 0; g < 3; ++g) {
                const int q2 = adj[3 * q + g];
                if (q2 != k) { a += rj[q2] / D[q2]; ++c; }
            }
        }
        a *= c ? 1.0 / c : 0.0;
    }
    return (float)(a * inv);
}

// U[ring][i] = ring_field(r, i, ring) for every DOF (the inverse rms read from rms[0])
__global__ void __launch_bounds__(kT) k_rings(const double* __restrict__ r, const double* __restrict__ D,
                                               const double* __restrict__ rms, const int* __restrict__ adj,
                                               int64_t ex, int64_t n, float* __restrict__ U) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const double s = rms[0];
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (int ring = 0; ring < kRings; ++ring) U[ring * n + i] = ring_field(r, D, i, ex, ring, adj, inv);
}

// sum of squares of (v / D) in fixed order: partials per block, then one block
__global__ void __launch_bounds__(kT) k_ssq(const double* __restrict__ v, const double* __restrict__ D, int64_t ex,
                                             int64_t n, double* __restrict__ part) {
    __shared__ double red[kT];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        const double q = v[i] / D[i % ex];
        s += q * q;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kT) k_ssq_final(double* __restrict__ part, int nb, int64_t n) {
    __shared__ double red[kT];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kT) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[0] = sqrt(red[0] / (double)n);   // rms of v / D
}

// ---------------------------------------------------------------- inference
// The hidden width is padded to Hp = 64 NCT (NCT = 1, 2 or 4) and the
// feature count to Fp = F rounded up to a multiple of 4, with zero weights,
// which leaves N unchanged (tanh 0 = 0).  Packed operands, rebuilt from the
// FP32 weights before every application:
//   W1p [Fp][Hp] FP32,
//   W2t [Hp][Hp] FP32, transposed (output unit first, input unit second),
//   w3p [Hp]     FP32.
typedef float f4v_t __attribute__((ext_vector_type(4)));

constexpr int kMR = 64;          // DOFs (rows) per inference block, 4 waves

__global__ void k_pack(const float* __restrict__ W1, const float* __restrict__ W2, const float* __restrict__ w3,
                       float* __restrict__ W1p, float* __restrict__ W2t, float* __restrict__ w3p, int F, int Fp,
                       int H, int Hp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < Hp * Hp) {
        const int j = i / Hp, a = i % Hp;                 // W2t[j][a] = W2[a][j]
        W2t[i] = j < H && a < H ? W2[a * H + j] : 0.f;
    }
    if (i < Fp * Hp) {
        const int f = i / Hp, h = i % Hp;
        W1p[i] = h < H && f < F ? W1[f * H + h] : 0.f;
    }
    if (i < Hp) w3p[i] = i < H ? w3[i] : 0.f;
}

// tanh x = 1 - 2 / (e^{2x} + 1) with the hardware exponential and
// reciprocal: exact limits +-1 for large |x| (rcp(inf) = 0), absolute error a
// few FP32 ulps of 1
__device__ __forceinline__ float fast_tanh(float x) {
    return 1.f - 2.f * __builtin_amdgcn_rcpf(__expf(2.f * x) + 1.f);
}

// z(i) = s N(x(i)) for the DOFs i0 .. i0 + kMR - 1 (natural order).
//  1. features X[kMR][Fp + 1] (FP32, read from the ring fields U; the odd
//     row stride spreads the rows over the LDS banks) into LDS;
//  2. first layer on the matrix cores in FP32 (v_mfma_f32_16x16x4f32: exact
//     products, FP32 accumulation); tanh into A[kMR][Hp + 1] (FP32, LDS; the
//     odd row stride spreads the rows over the banks);
//  3. second layer on the matrix cores in FP32 as well (FP32 inputs and
//     accumulation: the network applied is the one trained, in FP32).
//  In both layers wave w owns the hidden units [16 NCT w, 16 NCT (w+1)) for
//  all 64 rows (4 x NCT tiles of 16 x 16);
//  4. tanh and the output layer in FP32: the 16 lanes that hold one row's
//     units reduce by shuffles, the 4 waves through LDS.
template <int NCT>
__global__ void __launch_bounds__(256) k_mlp_mfma(const float* __restrict__ U, const double* __restrict__ rms,
                                                  const float* __restrict__ W1p, const float* __restrict__ W2t,
                                                  const float* __restrict__ w3p, const float* __restrict__ wl,
                                                  double* __restrict__ z, int64_t ex, int64_t n, int F, int Fp) {
    constexpr int Hp = 64 * NCT, AS = Hp + 1;
    const int XS = Fp + 1;
    extern __shared__ float smf[];
    float* red = smf;                                     // [4][kMR]
    float* A = red + 4 * kMR;                             // [kMR][AS]
    float* X = A + kMR * AS;                              // [kMR][XS]
    const int64_t i0 = (int64_t)blockIdx.x * kMR;
    const double s = rms[0];
    for (int e = threadIdx.x; e < kMR * Fp; e += 256) {  // lanes take consecutive rows: coalesced reads
        const int f = e / kMR, r = e - f * kMR;
        const int lag = f / kRings, ring = f - lag * kRings;
        const int64_t i = i0 + r, q = i - (int64_t)lag * ex;
        X[r * XS + f] = f < F && i < n && q >= 0 ? U[ring * n + q] : 0.f;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    {
        f4v_t c1[4][NCT];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) c1[rt][ct] = f4v_t{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < Fp; k0 += 4) {
            float b[NCT];
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)  // B[k][j] = W1[k][j]: lane j + 16 k
                b[ct] = W1p[(k0 + lk) * Hp + (wv * NCT + ct) * 16 + li];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {  // A[i][k] = X[i][k]: lane i + 16 k
                const float a = X[(rt * 16 + li) * XS + k0 + lk];
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct)
                    c1[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ct], c1[rt][ct], 0, 0, 0);
            }
        }
        // D[i][j]: lane j + 16 (i/4), element i % 4
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    A[(rt * 16 + 4 * lk + q) * AS + (wv * NCT + ct) * 16 + li] = fast_tanh(c1[rt][ct][q]);
    }
    __syncthreads();
    f4v_t acc[4][NCT];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[rt][ct] = f4v_t{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < Hp; k0 += 4) {
        float b[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)      // B[k][j] = W2[k][j]: lane j + 16 k
            b[ct] = W2t[(int64_t)((wv * NCT + ct) * 16 + li) * Hp + k0 + lk];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {      // A[i][k]: lane i + 16 k
            const float a = A[(rt * 16 + li) * AS + k0 + lk];
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[ct], acc[rt][ct], 0, 0, 0);
        }
    }
    // D[i][j]: lane j + 16 (i/4), element i % 4 -> this lane holds rows 4 lk + q of unit li of each tile
    float p[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float t = 0.f;
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) t += fast_tanh(acc[rt][ct][q]) * w3p[(wv * NCT + ct) * 16 + li];
            p[rt][q] = t;
        }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float t = p[rt][q];
            for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o, 16);
            if (li == 0) red[wv * kMR + rt * 16 + 4 * lk + q] = t;
        }
    __syncthreads();
    if (threadIdx.x < kMR && i0 + threadIdx.x < n) {   // plus the linear stencil c . x
        const int r = threadIdx.x;
        float lin = 0.f;
        for (int f = 0; f < F; ++f) lin += wl[f] * X[r * XS + f];
        z[i0 + r] = s * ((double)(red[r] + red[kMR + r] + red[2 * kMR + r] + red[3 * kMR + r]) + (double)lin);
    }
}

// The stencil alone (hidden width 0): z(i) = s c . x(i), same summation order
// over the features as the perceptron kernel's linear term.
__global__ void __launch_bounds__(kT) k_lin_apply(const float* __restrict__ U, const double* __restrict__ rms,
                                                   const float* __restrict__ wl, double* __restrict__ z, int64_t ex,
                                                   int64_t n, int F) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    float lin = 0.f;
    for (int f = 0; f < F; ++f) {
        const int lag = f / kRings, ring = f - lag * kRings;
        const int64_t q = i - (int64_t)lag * ex;
        lin += wl[f] * (q >= 0 ? U[ring * n + q] : 0.f);
    }
    z[i] = rms[0] * (double)lin;
}

// T[b] -= y[b]
__global__ void k_sub_f(float* __restrict__ T, const float* __restrict__ y, int B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) T[b] -= y[b];
}

// ---------------------------------------------------------------- training
// Minibatch gather: sample b draws (pair p, DOF i) from a counter-based hash;
// X[b][f] = feature f of r_p at i (scaled by 1 / s_p), T[b] = e_p(i) / s_p.
__global__ void __launch_bounds__(kT) k_gather(const double* __restrict__ R, const double* __restrict__ E,
                                                const double* __restrict__ S, const double* __restrict__ D,
                                                int npair, int64_t ex, int64_t n, int F, uint64_t seed, int step,
                                                int B, const int* __restrict__ adj, float* __restrict__ X,
                                                float* __restrict__ T) {
    const int b = blockIdx.x * kT + threadIdx.x;
    if (b >= B) return;
    const uint64_t h = mix64(seed ^ mix64(((uint64_t)step << 32) | (uint64_t)b));
    const int p = (int)(h % (uint64_t)npair);
    const int64_t i = (int64_t)((h >> 20) % (uint64_t)n);
    const double inv = S[p] > 0.0 ? 1.0 / S[p] : 0.0;
    const double* r = R + (int64_t)p * n;
    for (int f = 0; f < F; ++f) {
        const int lag = f / kRings;
        X[b * F + f] = i - (int64_t)lag * ex >= 0 ? ring_field(r, D, i - (int64_t)lag * ex, ex, f - lag * kRings, adj, inv)
                                                  : 0.f;
    }
    T[b] = (float)(E[(int64_t)p * n + i] * inv);
}

// C[M x N] (+)= op(A) op(B), FP32, row-major; op(A) = A (M x K) or A^T
// (A stored K x M); op(B) = B (K x N) or B^T (B stored N x K).  16 x 16
// output tiles, 16-deep K chunks through LDS.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(const float* __restrict__ A, const float* __restrict__ B,
                                               float* __restrict__ C, int M, int N, int K, int accumulate) {
    __shared__ float sa[16][17], sb[16][17];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
    float acc = 0.f;
    for (int k0 = 0; k0 < K; k0 += 16) {
        {   // A tile: rows blockIdx.y*16 + ty, k = k0 + tx
            const int r = blockIdx.y * 16 + ty, k = k0 + tx;
            float v = 0.f;
            if (r < M && k < K) v = TA ? A[(int64_t)k * M + r] : A[(int64_t)r * K + k];
            sa[ty][tx] = v;
        }
        {   // B tile: k = k0 + ty, cols blockIdx.x*16 + tx
            const int k = k0 + ty, c = blockIdx.x * 16 + tx;
            float v = 0.f;
            if (k < K && c < N) v = TB ? B[(int64_t)c * K + k] : B[(int64_t)k * N + c];
            sb[ty][tx] = v;
        }
        __syncthreads();
        for (int kk = 0; kk < 16; ++kk) acc += sa[ty][kk] * sb[kk][tx];
        __syncthreads();
    }
    if (row < M && col < N) {
        float* c = C + (int64_t)row * N + col;
        *c = accumulate ? *c + acc : acc;
    }
}

__global__ void k_tanh(float* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = tanhf(x[i]);
}

// dy[b] = 2 (y[b] - t[b]) / B; loss partial per block
__global__ void __launch_bounds__(kT) k_loss_grad(const float* __restrict__ y, const float* __restrict__ t,
                                                   float* __restrict__ dy, int B, float* __restrict__ loss) {
    __shared__ float red[kT];
    float l = 0.f;
    for (int b = threadIdx.x; b < B; b += kT) {
        const float d = y[b] - t[b];
        dy[b] = 2.f * d / (float)B;
        l += d * d;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (float)B;
}

// G[b][h] = G[b][h] * (1 - Hact[b][h]^2)   (back through tanh)
__global__ void k_dtanh(float* __restrict__ G, const float* __restrict__ Hact, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) G[i] *= 1.f - Hact[i] * Hact[i];
}

// Adam (Kingma and Ba) step on one parameter array
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, int64_t n, float lr, float b1t, float b2t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b1 = 0.9f, b2 = 0.999f;
    m1[i] = b1 * m1[i] + (1.f - b1) * g[i];
    m2[i] = b2 * m2[i] + (1.f - b2) * g[i] * g[i];
    const float mh = m1[i] / (1.f - b1t), vh = m2[i] / (1.f - b2t);
    w[i] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

template <bool TA, bool TB>
void gemm(const float* A, const float* B, float* C, int M, int N, int K, bool acc, hipStream_t st) {
    hipLaunchKernelGGL((k_gemm<TA, TB>), dim3((N + 15) / 16, (M + 15) / 16), dim3(256), 0, st, A, B, C, M, N, K,
                       acc ? 1 : 0);
}

unsigned nblk(int64_t n, int t = kT) { return (unsigned)((n + t - 1) / t); }

}  // namespace

namespace pfmm {

// rms of v / D into rms_dev[0] (scratch part: >= 1024 doubles).
pfmm_status precond_rms(const double* v, const double* D, int64_t ex, int64_t n, double* part, hipStream_t st) {
    const int nb = (int)std::min<int64_t>(1024, (n + kT - 1) / kT);
    hipLaunchKernelGGL(k_ssq, dim3(nb), dim3(kT), 0, st, v, D, ex, n, part);
    hipLaunchKernelGGL(k_ssq_final, dim3(1), dim3(kT), 0, st, part, nb, n);
    HIP_CHECK(hipGetLastError());
    return PFMM_OK;
}

size_t precond_scratch_doubles(int64_t n) { return 1024 + (size_t)(kRings * n + 1) / 2; }

// z = s N(x(v)) for the whole vector (natural order); part: scratch of
// precond_scratch_doubles(n) doubles (reduction partials, then the ring fields).
pfmm_status precond_apply(const pfmm_precond* pc, const double* v, double* z, const double* D, const int* adj,
                          int64_t ex, int64_t n, double* part, hipStream_t st) {
    if (precond_rms(v, D, ex, n, part, st) != PFMM_OK) return PFMM_EDEVICE;
    float* U = (float*)(part + 1024);
    hipLaunchKernelGGL(k_rings, dim3(nblk(n)), dim3(kT), 0, st, v, D, part, adj, ex, n, U);
    if (pc->H == 0) {
        hipLaunchKernelGGL(k_lin_apply, dim3(nblk(n)), dim3(kT), 0, st, U, part, pc->wl, z, ex, n, pc->F);
        HIP_CHECK(hipGetLastError());
        return PFMM_OK;
    }
    const int Hp = pc->Hp, Fp = (pc->F + 3) & ~3;
    hipLaunchKernelGGL(k_pack, dim3(nblk((int64_t)Hp * std::max(Hp, Fp))), dim3(kT), 0, st, pc->W1, pc->W2, pc->w3,
                       pc->W1p, pc->W2t, pc->w3p, pc->F, Fp, pc->H, Hp);
    const size_t shm = 4 * kMR * sizeof(float) + (size_t)kMR * (Hp + 1) * sizeof(float) +
                       (size_t)kMR * (Fp + 1) * sizeof(float);
    const dim3 g(nblk(n, kMR));
    if (Hp == 64)
        hipLaunchKernelGGL(k_mlp_mfma<1>, g, dim3(256), shm, st, U, part, pc->W1p, pc->W2t, pc->w3p, pc->wl, z,
                           ex, n, pc->F, Fp);
    else if (Hp == 128)
        hipLaunchKernelGGL(k_mlp_mfma<2>, g, dim3(256), shm, st, U, part, pc->W1p, pc->W2t, pc->w3p, pc->wl, z,
                           ex, n, pc->F, Fp);
    else
        hipLaunchKernelGGL(k_mlp_mfma<4>, g, dim3(256), shm, st, U, part, pc->W1p, pc->W2t, pc->w3p, pc->wl, z,
                           ex, n, pc->F, Fp);
    HIP_CHECK(hipGetLastError());
    return PFMM_OK;
}

// Train on npair pairs (R[p], E[p]) of length n (device, natural order).
pfmm_status precond_fit(pfmm_precond* pc, const double* R, const double* E, int npair, const double* D,
                        const int* adj, int64_t ex, int64_t n, int steps, int batch, float lr, uint64_t seed,
                        hipStream_t st) {
    const int F = pc->F, H = std::max(pc->H, 1), B = batch;   // (buffers of width 1 when hidden is 0)
    std::vector<void*> tmp;
    struct Free { std::vector<void*>& v; ~Free() { for (void* p : v) (void)hipFree(p); } } fr{tmp};
    double *S, *part;
    float *X, *T, *H1, *H2, *y, *dy, *G2, *G1, *g1, *g2, *g3, *m[6], *loss;
    if (palloc(tmp, &S, (size_t)npair) || palloc(tmp, &part, 1024) || palloc(tmp, &X, (size_t)B * F) ||
        palloc(tmp, &T, (size_t)B) || palloc(tmp, &H1, (size_t)B * H) || palloc(tmp, &H2, (size_t)B * H) ||
        palloc(tmp, &y, (size_t)B) || palloc(tmp, &dy, (size_t)B) || palloc(tmp, &G2, (size_t)B * H) ||
        palloc(tmp, &G1, (size_t)B * H) || palloc(tmp, &g1, (size_t)F * H) || palloc(tmp, &g2, (size_t)H * H) ||
        palloc(tmp, &g3, (size_t)H) || palloc(tmp, &loss, 1))
        return PFMM_ENOMEM;
    const size_t sizes[3] = {(size_t)F * H, (size_t)H * H, (size_t)H};
    for (int i = 0; i < 6; ++i) {
        if (palloc(tmp, &m[i], sizes[i % 3])) return PFMM_ENOMEM;
        HIP_CHECK(hipMemsetAsync(m[i], 0, sizes[i % 3] * sizeof(float), st));
    }
    for (int p = 0; p < npair; ++p) {
        if (precond_rms(R + (int64_t)p * n, D, ex, n, part, st) != PFMM_OK) return PFMM_EDEVICE;
        HIP_CHECK(hipMemcpyAsync(S + p, part, sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    // 1. the linear stencil c: least squares over about 2^20 samples drawn like
    //    the minibatches (normal equations per batch in FP32 on the GPU, summed
    //    in FP64 on the host), a ridge of 1e-8 trace / F, Cholesky
    {
        float *Gd, *rd, *ttd;
        if (palloc(tmp, &Gd, (size_t)F * F) || palloc(tmp, &rd, (size_t)F) || palloc(tmp, &ttd, 1))
            return PFMM_ENOMEM;
        std::vector<double> G((size_t)F * F, 0.0), r(F, 0.0), c(F, 0.0);
        std::vector<float> hG((size_t)F * F), hr(F);
        double tt = 0.0;
        float htt = 0.f;
        const int chunks = std::max(1, (1 << 20) / B);
        for (int ch = 0; ch < chunks; ++ch) {
            hipLaunchKernelGGL(k_gather, dim3(nblk(B)), dim3(kT), 0, st, R, E, S, D, npair, ex, n, F,
                               seed ^ 0x6c73717561726573ull, ch, B, adj, X, T);
            gemm<true, false>(X, X, Gd, F, F, B, false, st);   // X^T X
            gemm<true, false>(X, T, rd, F, 1, B, false, st);   // X^T t
            gemm<true, false>(T, T, ttd, 1, 1, B, false, st);  // t^T t
            HIP_CHECK(hipMemcpyAsync(hG.data(), Gd, hG.size() * sizeof(float), hipMemcpyDeviceToHost, st));
            HIP_CHECK(hipMemcpyAsync(hr.data(), rd, hr.size() * sizeof(float), hipMemcpyDeviceToHost, st));
            HIP_CHECK(hipMemcpyAsync(&htt, ttd, sizeof(float), hipMemcpyDeviceToHost, st));
            HIP_CHECK(hipStreamSynchronize(st));
            for (size_t i = 0; i < G.size(); ++i) G[i] += hG[i];
            for (int i = 0; i < F; ++i) r[i] += hr[i];
            tt += htt;
        }
        double tr = 0.0;
        for (int i = 0; i < F; ++i) tr += G[(size_t)i * F + i];
        for (int i = 0; i < F; ++i) G[(size_t)i * F + i] += 1e-8 * tr / F + 1e-300;
        // Cholesky G = L L^T in place (lower triangle), then two triangular solves
        for (int j = 0; j < F; ++j) {
            double d = G[(size_t)j * F + j];
            for (int k = 0; k < j; ++k) d -= G[(size_t)j * F + k] * G[(size_t)j * F + k];
            if (!(d > 0.0)) return set_error(PFMM_ENONFINITE, "preconditioner stencil: normal equations not positive definite");
            const double ljj = std::sqrt(d);
            G[(size_t)j * F + j] = ljj;
            for (int i = j + 1; i < F; ++i) {
                double v = G[(size_t)i * F + j];
                for (int k = 0; k < j; ++k) v -= G[(size_t)i * F + k] * G[(size_t)j * F + k];
                G[(size_t)i * F + j] = v / ljj;
            }
        }
        for (int i = 0; i < F; ++i) {
            double v = r[i];
            for (int k = 0; k < i; ++k) v -= G[(size_t)i * F + k] * c[k];
            c[i] = v / G[(size_t)i * F + i];
        }
        for (int i = F - 1; i >= 0; --i) {
            double v = c[i];
            for (int k = i + 1; k < F; ++k) v -= G[(size_t)k * F + i] * c[k];
            c[i] = v / G[(size_t)i * F + i];
        }
        std::vector<float> cf(F);
        double rc = 0.0;
        for (int i = 0; i < F; ++i) {
            cf[i] = (float)c[i];
            rc += r[i] * c[i];
        }
        HIP_CHECK(hipMemcpyAsync(pc->wl, cf.data(), F * sizeof(float), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipStreamSynchronize(st));
        // mean squared residual of the fit: (t^T t - r^T c) / samples (normal equations)
        pc->last_loss = (float)((tt - rc) / ((double)chunks * B));
    }
    if (pc->H == 0) return PFMM_OK;
    // 2. the perceptron, on the targets minus the stencil's prediction
    float b1t = 1.f, b2t = 1.f;
    for (int it = 0; it < steps; ++it) {
        hipLaunchKernelGGL(k_gather, dim3(nblk(B)), dim3(kT), 0, st, R, E, S, D, npair, ex, n, F, seed, it, B, adj,
                           X, T);
        gemm<false, false>(X, pc->wl, dy, B, 1, F, false, st);          // stencil prediction X c
        hipLaunchKernelGGL(k_sub_f, dim3(nblk(B)), dim3(kT), 0, st, T, dy, B);
        gemm<false, false>(X, pc->W1, H1, B, H, F, false, st);          // H1 = tanh(X W1)
        hipLaunchKernelGGL(k_tanh, dim3(nblk((int64_t)B * H)), dim3(kT), 0, st, H1, (int64_t)B * H);
        gemm<false, false>(H1, pc->W2, H2, B, H, H, false, st);         // H2 = tanh(H1 W2)
        hipLaunchKernelGGL(k_tanh, dim3(nblk((int64_t)B * H)), dim3(kT), 0, st, H2, (int64_t)B * H);
        gemm<false, false>(H2, pc->w3, y, B, 1, H, false, st);          // y = H2 w3
        hipLaunchKernelGGL(k_loss_grad, dim3(1), dim3(kT), 0, st, y, T, dy, B, loss);
        gemm<true, false>(H2, dy, g3, H, 1, B, false, st);               // g3 = H2^T dy
        gemm<false, true>(dy, pc->w3, G2, B, H, 1, false, st);          // G2 = dy w3^T
        hipLaunchKernelGGL(k_dtanh, dim3(nblk((int64_t)B * H)), dim3(kT), 0, st, G2, H2, (int64_t)B * H);
        gemm<true, false>(H1, G2, g2, H, H, B, false, st);               // g2 = H1^T G2
        gemm<false, true>(G2, pc->W2, G1, B, H, H, false, st);          // G1 = G2 W2^T
        hipLaunchKernelGGL(k_dtanh, dim3(nblk((int64_t)B * H)), dim3(kT), 0, st, G1, H1, (int64_t)B * H);
        gemm<true, false>(X, G1, g1, F, H, B, false, st);                // g1 = X^T G1
        b1t *= 0.9f;
        b2t *= 0.999f;
        // cosine decay of the step size to zero over the run (Loshchilov and Hutter)
        const float lrt = 0.5f * lr * (1.f + std::cos(3.14159265f * (float)it / (float)steps));
        hipLaunchKernelGGL(k_adam, dim3(nblk(sizes[0])), dim3(kT), 0, st, pc->W1, g1, m[0], m[3], (int64_t)sizes[0], lrt, b1t, b2t);
        hipLaunchKernelGGL(k_adam, dim3(nblk(sizes[1])), dim3(kT), 0, st, pc->W2, g2, m[1], m[4], (int64_t)sizes[1], lrt, b1t, b2t);
        hipLaunchKernelGGL(k_adam, dim3(nblk(sizes[2])), dim3(kT), 0, st, pc->w3, g3, m[2], m[5], (int64_t)sizes[2], lrt, b1t, b2t);
    }
    HIP_CHECK(hipGetLastError());
    if (steps > 0) HIP_CHECK(hipMemcpyAsync(&pc->last_loss, loss, sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    return PFMM_OK;
}

float precond_last_loss(const pfmm_precond* pc) { return pc->last_loss; }

}  // namespace pfmm

extern "C" {

pfmm_status pfmm_precond_create(int32_t device, int32_t features, int32_t hidden, uint64_t seed, pfmm_precond** out) {
    if (!out) return set_error(PFMM_EINVAL, "NULL output pointer");
    *out = nullptr;
    if (features < 1 || features > 32 || hidden < 0 || hidden > kT)
        return set_error(PFMM_EINVAL, "features must be in 1..32 and hidden in 0..256");
    if (hipSetDevice(device) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    pfmm_precond* p = new (std::nothrow) pfmm_precond();
    if (!p) return set_error(PFMM_ENOMEM, "host allocation failed");
    p->device = device;
    p->FT = features;
    p->F = features * kRings;
    p->H = hidden;
    // Glorot-uniform initial weights from splitmix64
    auto init = [&](float** w, int fan_in, int fan_out, uint64_t tag) -> pfmm_status {
        const size_t n = (size_t)fan_in * fan_out;
        std::vector<float> h(n);
        const double lim = std::sqrt(6.0 / (fan_in + fan_out));
        for (size_t i = 0; i < n; ++i) {
            const double u = (double)(mix64(seed ^ (tag << 48) ^ i) >> 11) * (1.0 / 9007199254740992.0);
            h[i] = (float)((2.0 * u - 1.0) * lim);
        }
        if (palloc(p->owned, w, n)) return PFMM_ENOMEM;
        if (hipMemcpy(*w, h.data(), n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return set_error(PFMM_EDEVICE, "hipMemcpy failed");
        return PFMM_OK;
    };
    p->Hp = hidden <= 64 ? 64 : hidden <= 128 ? 128 : 256;
    pfmm_status s = palloc(p->owned, &p->wl, (size_t)p->F);
    if (s == PFMM_OK && hipMemset(p->wl, 0, (size_t)p->F * sizeof(float)) != hipSuccess)
        s = set_error(PFMM_EDEVICE, "hipMemset failed");
    if (hidden > 0) {
        if (s == PFMM_OK) s = init(&p->W1, p->F, hidden, 1);
        if (s == PFMM_OK) s = init(&p->W2, hidden, hidden, 2);
        if (s == PFMM_OK) s = init(&p->w3, hidden, 1, 3);
        if (s == PFMM_OK) s = palloc(p->owned, &p->W1p, (size_t)((p->F + 3) & ~3) * p->Hp);
        if (s == PFMM_OK) s = palloc(p->owned, &p->W2t, (size_t)p->Hp * p->Hp);
        if (s == PFMM_OK) s = palloc(p->owned, &p->w3p, (size_t)p->Hp);
    }
    if (s != PFMM_OK) {
        pfmm_precond_destroy(p);
        return s;
    }
    *out = p;
    return PFMM_OK;
}

pfmm_status pfmm_precond_save(const pfmm_precond* p, const char* path) {
    if (!p || !path) return set_error(PFMM_EINVAL, "NULL argument");
    if (hipSetDevice(p->device) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    std::vector<float> l(p->F), a((size_t)p->F * p->H), b((size_t)p->H * p->H), c(p->H);
    bool ok = hipMemcpy(l.data(), p->wl, l.size() * 4, hipMemcpyDeviceToHost) == hipSuccess;
    if (ok && p->H > 0)
        ok = hipMemcpy(a.data(), p->W1, a.size() * 4, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(b.data(), p->W2, b.size() * 4, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(c.data(), p->w3, c.size() * 4, hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok) return set_error(PFMM_EDEVICE, "hipMemcpy failed");
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(PFMM_EINVAL, std::string("cannot open ") + path);
    const int32_t hdr[4] = {0x4d4c5031, 4, p->FT, p->H};   // magic, version, time lags, hidden
    ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1 && std::fwrite(l.data(), 4, l.size(), f) == l.size() &&
         std::fwrite(a.data(), 4, a.size(), f) == a.size() && std::fwrite(b.data(), 4, b.size(), f) == b.size() &&
         std::fwrite(c.data(), 4, c.size(), f) == c.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? PFMM_OK : set_error(PFMM_EINVAL, std::string("write failed: ") + path);
}

pfmm_status pfmm_precond_load(const char* path, int32_t device, pfmm_precond** out) {
    if (!path || !out) return set_error(PFMM_EINVAL, "NULL argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(PFMM_EINVAL, std::string("cannot open ") + path);
    int32_t hdr[4];
    if (std::fread(hdr, sizeof(hdr), 1, f) != 1 || hdr[0] != 0x4d4c5031 || hdr[1] != 4 || hdr[2] < 1 || hdr[2] > 32 ||
        hdr[3] < 0 || hdr[3] > kT) {
        std::fclose(f);
        return set_error(PFMM_EINVAL, std::string("not a preconditioner file: ") + path);
    }
    const size_t F = (size_t)hdr[2] * kRings, H = (size_t)hdr[3];
    std::vector<float> l(F), a(F * H), b(H * H), c(H);
    const bool ok = std::fread(l.data(), 4, l.size(), f) == l.size() && std::fread(a.data(), 4, a.size(), f) == a.size() &&
                    std::fread(b.data(), 4, b.size(), f) == b.size() && std::fread(c.data(), 4, c.size(), f) == c.size();
    std::fclose(f);
    if (!ok) return set_error(PFMM_EINVAL, std::string("truncated preconditioner file: ") + path);
    pfmm_precond* p = nullptr;
    pfmm_status s = pfmm_precond_create(device, hdr[2], hdr[3], 0, &p);
    if (s != PFMM_OK) return s;
    bool cp = hipMemcpy(p->wl, l.data(), l.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    if (cp && H > 0)
        cp = hipMemcpy(p->W1, a.data(), a.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(p->W2, b.data(), b.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(p->w3, c.data(), c.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    if (!cp) {
        pfmm_precond_destroy(p);
        return set_error(PFMM_EDEVICE, "hipMemcpy failed");
    }
    *out = p;
    return PFMM_OK;
}

void pfmm_precond_destroy(pfmm_precond* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    for (void* q : p->owned) (void)hipFree(q);
    delete p;
}

}  // extern "C"
