// Dirichlet solve of the Galerkin system  V_h w = (1/2 M_h + K_h) g
// (Section 2, system 02:linear:system) by GMRES without restart and without
// preconditioner, as in the experiments of Section 5, stopped at a relative
// residual (Saad and Schultz's estimate ||b - V_h w_k|| / ||b||).
//
// Arnoldi runs on the GPU in FP64 with classical Gram-Schmidt applied twice
// (CGS2): per iteration two passes of "coefficients = basis^T w" and
// "w -= basis coefficients" over the Krylov basis, one norm, and one scaling.
// Every reduction is a two-level fixed-order sum (block partials, then one
// block per column), so solves are bitwise reproducible.  The small
// Hessenberg least-squares problem (Givens rotations) is updated on the host,
// which reads m+3 doubles per iteration.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pfmm.h"

using namespace pfmm;

namespace {

constexpr int kBlock = 256;        // threads per block of the vector kernels
constexpr int kMaxBlocks = 1024;   // row blocks of a multi-dot (partials per column)
constexpr int kCols = 8;           // basis columns per pass of a multi-dot

#define HIP_CHECK(expr)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return set_error(PFMM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

// Sum of the kBlock values of `v` held one per thread; result valid in thread 0.
__device__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

// partial[j * gridDim.x + b] = sum over rows i of block b of V_j[i] w[i]
// for the columns j < ncols of V (column j at basis + j * ld).  Blocks own
// contiguous row ranges; each pass loads w once for kCols columns.
__global__ void __launch_bounds__(kBlock) k_multidot(const double* __restrict__ basis, int64_t ld, int ncols,
                                                      const double* __restrict__ w, int64_t n,
                                                      double* __restrict__ partial) {
    __shared__ double red[kBlock / 64];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    for (int j0 = 0; j0 < ncols; j0 += kCols) {
        double acc[kCols];
#pragma unroll
        for (int c = 0; c < kCols; ++c) acc[c] = 0.0;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
            const double wi = w[i];
#pragma unroll
            for (int c = 0; c < kCols; ++c)
                if (j0 + c < ncols) acc[c] += basis[(int64_t)(j0 + c) * ld + i] * wi;
        }
#pragma unroll
        for (int c = 0; c < kCols; ++c) {
            if (j0 + c >= ncols) break;
            const double s = block_sum(acc[c], red);
            if (threadIdx.x == 0) partial[(int64_t)(j0 + c) * gridDim.x + blockIdx.x] = s;
        }
    }
}

// out[j] = sum_b partial[j * nb + b], one block per column, fixed order.
__global__ void __launch_bounds__(kBlock) k_sum_partials(const double* __restrict__ partial, int nb,
                                                          double* __restrict__ out) {
    __shared__ double red[kBlock / 64];
    const int j = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) v += partial[(int64_t)j * nb + b];
    const double s = block_sum(v, red);
    if (threadIdx.x == 0) out[j] = s;
}

// y[i] = (base ? base[i] : 0) + sgn * sum_{j < ncols} c[j] V_j[i]
__global__ void __launch_bounds__(kBlock) k_combine(const double* basis, int64_t ld, int ncols,
                                                     const double* __restrict__ c, double sgn,
                                                     const double* base, double* y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < ncols; ++j) s += c[j] * basis[(int64_t)j * ld + i];
    y[i] = (base ? base[i] : 0.0) + sgn * s;
}

// y[i] = a * x[i]
__global__ void __launch_bounds__(kBlock) k_scale(const double* x, double* y, double a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

// b[i] += 1/2 M_h g: mass[k_x] = |gamma_kx| h_t for the index i = k_t E_x + k_x.
__global__ void __launch_bounds__(kBlock) k_half_mass(const double* __restrict__ g, const double* __restrict__ mass,
                                                       double* __restrict__ b, int64_t ex, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] += 0.5 * mass[i % ex] * g[i];
}

// b[i] -= a[i]
__global__ void __launch_bounds__(kBlock) k_sub(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] -= a[i];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

struct Workspace {
    double* basis = nullptr;   // (m + 1) columns of n
    double* b = nullptr;       // right-hand side (dirichlet solve only)
    double* partial = nullptr; // kMaxBlocks * (m + 1)
    double* col = nullptr;     // 2 (m + 1) + 1 reduced values
    double* coef = nullptr;    // m + 1 host-computed coefficients
    std::vector<void*> owned;
    ~Workspace() {
        for (void* p : owned) (void)hipFree(p);
    }
    pfmm_status alloc(double** p, size_t n) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, n * sizeof(double));
        if (e != hipSuccess) return set_error(PFMM_ENOMEM, std::string("solve workspace: ") + hipGetErrorString(e));
        owned.push_back(q);
        *p = (double*)q;
        return PFMM_OK;
    }
};

#define PS_TRY(expr)                       \
    do {                                   \
        pfmm_status s_ = (expr);           \
        if (s_ != PFMM_OK) return s_;      \
    } while (0)

// coefficients V_j^T x for j < ncols into dst (device), via partials.
void multidot(Workspace& ws, const double* V, int64_t ld, int ncols, const double* x, int64_t n, int nb, double* dst,
              hipStream_t st) {
    hipLaunchKernelGGL(k_multidot, dim3(nb), dim3(kBlock), 0, st, V, ld, ncols, x, n, ws.partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(ncols), dim3(kBlock), 0, st, ws.partial, nb, dst);
}

pfmm_status gmres(pfmm_tree* t, const double* b, double* x, const pfmm_solve_opts& o, pfmm_solve_info* info,
                  Workspace& ws, hipStream_t st) {
    const int64_t n = tree_dofs(t);
    const int m = o.max_iter;
    const int64_t ld = n;
    const int nb = (int)std::min<int64_t>(kMaxBlocks, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
    PS_TRY(ws.alloc(&ws.basis, (size_t)(m + 1) * n));
    PS_TRY(ws.alloc(&ws.partial, (size_t)kMaxBlocks * (m + 1)));
    PS_TRY(ws.alloc(&ws.col, (size_t)2 * (m + 1) + 1));
    PS_TRY(ws.alloc(&ws.coef, (size_t)m + 1));
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), e(m + 2, 0.0), hbuf(2 * (m + 1) + 1);
    auto Hij = [&](int i, int j) -> double& { return H[(size_t)j * (m + 1) + i]; };

    // beta = ||b||, v_0 = b / beta
    multidot(ws, b, ld, 1, b, n, nb, ws.col, st);
    HIP_CHECK(hipMemcpyAsync(hbuf.data(), ws.col, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    const double beta = std::sqrt(hbuf[0]);
    if (info) { info->history_len = 0; info->iters = 0; }
    auto record = [&](double r) {
        if (info && info->history && info->history_len < info->history_cap) info->history[info->history_len++] = r;
    };
    record(1.0);
    if (!(beta > 0.0) || !std::isfinite(beta)) {
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, x, 0.0, n);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipStreamSynchronize(st));
        if (!std::isfinite(beta)) return set_error(PFMM_ENONFINITE, "right-hand side is not finite");
        if (info) { info->converged = 1; info->rel_residual = 0.0; info->true_rel_residual = 0.0; }
        return PFMM_OK;
    }
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, ws.basis, 1.0 / beta, n);
    e[0] = beta;
    int k = 0;
    double est = 1.0;
    for (int j = 0; j < m; ++j) {
        double* vj = ws.basis + (int64_t)j * ld;
        double* w = ws.basis + (int64_t)(j + 1) * ld;
        PS_TRY(tree_apply(t, false, vj, w, st));
        // CGS2: two projections against v_0 .. v_j
        for (int pass = 0; pass < 2; ++pass) {
            double* h = ws.col + pass * (m + 1);
            multidot(ws, ws.basis, ld, j + 1, w, n, nb, h, st);
            hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kBlock), 0, st, ws.basis, ld, j + 1, h, -1.0,
                               w, w, n);
        }
        multidot(ws, w, ld, 1, w, n, nb, ws.col + 2 * (m + 1), st);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(hbuf.data(), ws.col, hbuf.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        for (int i = 0; i <= j; ++i) Hij(i, j) = hbuf[i] + hbuf[(m + 1) + i];
        const double hn = std::sqrt(hbuf[2 * (m + 1)]);
        if (!std::isfinite(hn)) return set_error(PFMM_ENONFINITE, "non-finite value in the Arnoldi process");
        Hij(j + 1, j) = hn;
        if (hn > 0.0)
            hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, w, w, 1.0 / hn, n);
        for (int i = 0; i < j; ++i) {   // earlier rotations on the new column
            const double a = Hij(i, j), c = Hij(i + 1, j);
            Hij(i, j) = cs[i] * a + sn[i] * c;
            Hij(i + 1, j) = -sn[i] * a + cs[i] * c;
        }
        const double r = std::hypot(Hij(j, j), Hij(j + 1, j));
        if (!(r > 0.0)) return set_error(PFMM_ENOTCONV, "GMRES breakdown: V_h maps a Krylov vector to zero");
        cs[j] = Hij(j, j) / r;
        sn[j] = Hij(j + 1, j) / r;
        Hij(j, j) = r;
        Hij(j + 1, j) = 0.0;
        e[j + 1] = -sn[j] * e[j];
        e[j] = cs[j] * e[j];
        k = j + 1;
        est = std::fabs(e[j + 1]) / beta;
        record(est);
        if (est <= o.rtol || hn == 0.0) break;
    }
    // x = V_k y with the triangular solve R y = e
    std::vector<double> y(k);
    for (int i = k - 1; i >= 0; --i) {
        double s = e[i];
        for (int l = i + 1; l < k; ++l) s -= Hij(i, l) * y[l];
        y[i] = s / Hij(i, i);
    }
    HIP_CHECK(hipMemcpyAsync(ws.coef, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kBlock), 0, st, ws.basis, ld, k, ws.coef, 1.0,
                       (const double*)nullptr, x, n);
    // true residual: V x - b in the first basis column (no longer needed)
    PS_TRY(tree_apply(t, false, x, ws.basis, st));
    hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, ws.basis, n);
    multidot(ws, ws.basis, ld, 1, ws.basis, n, nb, ws.col, st);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(hbuf.data(), ws.col, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    if (info) {
        info->iters = k;
        info->rel_residual = est;
        info->true_rel_residual = std::sqrt(hbuf[0]) / beta;
        info->converged = est <= o.rtol ? 1 : 0;
    }
    if (est > o.rtol)
        return set_error(PFMM_ENOTCONV, "GMRES reached max_iter = " + std::to_string(m) +
                                            " with relative residual " + std::to_string(est));
    return PFMM_OK;
}

pfmm_status check_opts(const pfmm_solve_opts* o, pfmm_solve_opts& out) {
    pfmm_default_solve_opts(&out);
    if (o) out = *o;
    if (!(out.rtol >= 0.0) || !std::isfinite(out.rtol)) return set_error(PFMM_EINVAL, "rtol must be finite and >= 0");
    if (out.max_iter < 1 || out.max_iter > 100000) return set_error(PFMM_EINVAL, "max_iter must be in 1..100000");
    return PFMM_OK;
}

pfmm_status solve_common(pfmm_tree* t, const double* b_or_g, double* w, const pfmm_solve_opts* o,
                         pfmm_solve_info* info, void* stream, bool dirichlet) {
    if (!t || !b_or_g || !w) return set_error(PFMM_EINVAL, "NULL argument");
    if (!tree_has(t, PFMM_OP_V)) return set_error(PFMM_EINVAL, "V_h was not built for this tree");
    if (dirichlet && !tree_has(t, PFMM_OP_K)) return set_error(PFMM_EINVAL, "K_h was not built for this tree");
    pfmm_solve_opts opt;
    PS_TRY(check_opts(o, opt));
    if (hipSetDevice(tree_device(t)) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    const int64_t n = tree_dofs(t);
    size_t fr = 0, tot = 0;
    HIP_CHECK(hipMemGetInfo(&fr, &tot));
    const uint64_t need = ((uint64_t)opt.max_iter + 2) * n * 8 + (uint64_t)kMaxBlocks * (opt.max_iter + 1) * 8;
    if (need > fr)
        return set_error(PFMM_ENOMEM, "GMRES workspace needs " + std::to_string(need) + " bytes, " +
                                          std::to_string(fr) + " free (lower max_iter)");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    Workspace ws;
    const double* b = b_or_g;
    if (dirichlet) {
        PS_TRY(ws.alloc(&ws.b, (size_t)n));
        PS_TRY(pfmm_dirichlet_rhs(t, b_or_g, ws.b, stream));
        b = ws.b;
    }
    pfmm_status s = gmres(t, b, w, opt, info, ws, st);
    const hipError_t e = hipStreamSynchronize(st);
    if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (s == PFMM_OK && e != hipSuccess) return set_error(PFMM_EDEVICE, hipGetErrorString(e));
    return s;
}

}  // namespace

extern "C" {

pfmm_status pfmm_default_solve_opts(pfmm_solve_opts* out) {
    if (!out) return set_error(PFMM_EINVAL, "NULL options");
    std::memset(out, 0, sizeof(*out));
    out->rtol = 1e-8;
    out->max_iter = 200;
    return PFMM_OK;
}

pfmm_status pfmm_dirichlet_rhs(pfmm_tree* t, const double* g_dev, double* b_dev, void* stream) {
    if (!t || !g_dev || !b_dev) return set_error(PFMM_EINVAL, "NULL argument");
    if (!tree_has(t, PFMM_OP_K)) return set_error(PFMM_EINVAL, "K_h was not built for this tree");
    if (hipSetDevice(tree_device(t)) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    const int64_t n = tree_dofs(t);
    hipStream_t st = (hipStream_t)stream;
    PS_TRY(tree_apply(t, true, g_dev, b_dev, st));
    hipLaunchKernelGGL(k_half_mass, dim3(blocks_for(n)), dim3(kBlock), 0, st, g_dev, tree_mass(t), b_dev,
                       tree_triangles(t), n);
    HIP_CHECK(hipGetLastError());
    return PFMM_OK;
}

pfmm_status pfmm_solve_V(pfmm_tree* t, const double* b_dev, double* w_dev, const pfmm_solve_opts* o,
                         pfmm_solve_info* info, void* stream) {
    return solve_common(t, b_dev, w_dev, o, info, stream, false);
}

pfmm_status pfmm_solve_dirichlet(pfmm_tree* t, const double* g_dev, double* w_dev, const pfmm_solve_opts* o,
                                 pfmm_solve_info* info, void* stream) {
    return solve_common(t, g_dev, w_dev, o, info, stream, true);
}

}  // extern "C"
