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

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
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

// b[i] += 1/2 M_h g: M_h[i, i] = |gamma_kx| (t_{kt+1} - t_kt) for the index i = k_t E_x + k_x.
__global__ void __launch_bounds__(kBlock) k_half_mass(const double* __restrict__ g, const double* __restrict__ area,
                                                       const double* __restrict__ hstep, double* __restrict__ b,
                                                       int64_t ex, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] += 0.5 * (area[i % ex] * hstep[i / ex]) * g[i];
}

// b[kt E_x + kx] += 1/2 (M_h g): the mixed p0 x p1 mass, (t_{kt+1} - t_kt)
// |gamma_kx| / 3 times the sum of g over the three vertices of kx.
__global__ void __launch_bounds__(kBlock) k_half_mass_p1(const double* __restrict__ g, const double* __restrict__ area,
                                                          const double* __restrict__ hstep, const int* __restrict__ tris,
                                                          double* __restrict__ b, int64_t ex, int n_v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t kt = i / ex;
    const int kx = (int)(i - kt * ex);
    const double* gk = g + kt * n_v;
    const double sg = gk[tris[3 * kx]] + gk[tris[3 * kx + 1]] + gk[tris[3 * kx + 2]];
    b[i] += 0.5 * (area[kx] * hstep[kt] / 3.0) * sg;
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

// snaps (optional, ascending): iterations k at which x_k = V_k y_k is formed
// into snap_x + i n (the training pairs of the learned preconditioner).
// With n_snap > 0, the iterates x_k at n_snap iteration counts spread over
// the solve are written to snap_x (n_snap vectors; the counts, distinct, to
// snaps_out).  They are formed after the loop: Givens rotations leave the
// leading k x k block of R and the first k entries of the rotated right-hand
// side as they were after step k, so x_k = V_k R_k^{-1} e_k.
pfmm_status gmres(pfmm_tree* t, const double* b, double* x, const pfmm_solve_opts& o, pfmm_solve_info* info,
                  Workspace& ws, hipStream_t st, int n_snap = 0, double* snap_x = nullptr,
                  std::vector<int>* snaps_out = nullptr) {
    const int64_t n = tree_dofs(t);
    const int m = o.max_iter;
    const int64_t ld = n;
    const int nb = (int)std::min<int64_t>(kMaxBlocks, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
    const double* x0 = o.x0_dev;   // initial iterate (NULL = 0); may equal x
    if (x0 && n_snap > 0) return set_error(PFMM_EINVAL, "internal: snapshots need a zero initial iterate");
    PS_TRY(ws.alloc(&ws.basis, (size_t)(m + 1) * n));
    PS_TRY(ws.alloc(&ws.partial, (size_t)kMaxBlocks * (m + 1)));
    PS_TRY(ws.alloc(&ws.col, (size_t)2 * (m + 1) + 1));
    PS_TRY(ws.alloc(&ws.coef, (size_t)m + 1));
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), e(m + 2, 0.0), hbuf(2 * (m + 1) + 1);
    auto Hij = [&](int i, int j) -> double& { return H[(size_t)j * (m + 1) + i]; };

    // bnorm = ||b||; r_0 = b - V_h x_0 in the first basis column (b when x_0 = 0)
    multidot(ws, b, ld, 1, b, n, nb, ws.col, st);
    HIP_CHECK(hipMemcpyAsync(hbuf.data(), ws.col, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    const double bnorm = std::sqrt(hbuf[0]);
    if (info) { info->history_len = 0; info->iters = 0; }
    auto record = [&](double r) {
        if (info && info->history && info->history_len < info->history_cap) info->history[info->history_len++] = r;
    };
    if (!(bnorm > 0.0) || !std::isfinite(bnorm)) {
        record(1.0);
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, x, 0.0, n);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipStreamSynchronize(st));
        if (!std::isfinite(bnorm)) return set_error(PFMM_ENONFINITE, "right-hand side is not finite");
        if (info) { info->converged = 1; info->rel_residual = 0.0; info->true_rel_residual = 0.0; }
        return PFMM_OK;
    }
    double beta = bnorm;
    if (x0) {
        PS_TRY(tree_apply(t, false, x0, ws.basis, st));
        hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, ws.basis, n);           // V x0 - b
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, ws.basis, ws.basis, -1.0, n);
        multidot(ws, ws.basis, ld, 1, ws.basis, n, nb, ws.col, st);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipMemcpyAsync(hbuf.data(), ws.col, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        beta = std::sqrt(hbuf[0]);
        if (!std::isfinite(beta)) return set_error(PFMM_ENONFINITE, "initial iterate gives a non-finite residual");
    }
    record(beta / bnorm);
    if (x0 && beta <= o.rtol * bnorm) {
        // the initial iterate already meets the tolerance: returned unchanged
        if (x0 != x) HIP_CHECK(hipMemcpyAsync(x, x0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIP_CHECK(hipStreamSynchronize(st));
        if (info) {
            info->iters = 0;
            info->rel_residual = beta / bnorm;
            info->true_rel_residual = beta / bnorm;
            info->converged = 1;
        }
        return PFMM_OK;
    }
    if (!(beta > 0.0)) return set_error(PFMM_ENOTCONV, "zero residual with rtol = 0");
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, x0 ? ws.basis : b, ws.basis, 1.0 / beta, n);
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
        est = std::fabs(e[j + 1]) / bnorm;
        record(est);
        if (est <= o.rtol || hn == 0.0) break;
    }
    if (n_snap > 0 && snap_x && snaps_out) {
        snaps_out->clear();
        for (int i = 0; i < n_snap; ++i) {
            const int ks = std::max(1, (int)((double)(i + 1) * (k - 1) / (n_snap + 1)));
            if (snaps_out->empty() || ks > snaps_out->back()) snaps_out->push_back(ks);
        }
        for (size_t si = 0; si < snaps_out->size(); ++si) {
            const int ks = (*snaps_out)[si];
            std::vector<double> ys(ks);
            for (int i = ks - 1; i >= 0; --i) {
                double sum = e[i];
                for (int l = i + 1; l < ks; ++l) sum -= Hij(i, l) * ys[l];
                ys[i] = sum / Hij(i, i);
            }
            HIP_CHECK(hipMemcpyAsync(ws.coef, ys.data(), ks * sizeof(double), hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kBlock), 0, st, ws.basis, ld, ks, ws.coef, 1.0,
                               (const double*)nullptr, snap_x + (int64_t)si * n, n);
            HIP_CHECK(hipStreamSynchronize(st));   // ys is released at the end of this block
        }
    }
    // x = V_k y with the triangular solve R y = e
    std::vector<double> y(k);
    for (int i = k - 1; i >= 0; --i) {
        double s = e[i];
        for (int l = i + 1; l < k; ++l) s -= Hij(i, l) * y[l];
        y[i] = s / Hij(i, i);
    }
    HIP_CHECK(hipMemcpyAsync(ws.coef, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
    // x = x_0 + V_k y (element-wise, so x_0 may be x itself)
    hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kBlock), 0, st, ws.basis, ld, k, ws.coef, 1.0, x0, x, n);
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
        info->true_rel_residual = std::sqrt(hbuf[0]) / bnorm;
        info->converged = est <= o.rtol ? 1 : 0;
    }
    if (est > o.rtol)
        return set_error(PFMM_ENOTCONV, "GMRES reached max_iter = " + std::to_string(m) +
                                            " with relative residual " + std::to_string(est));
    return PFMM_OK;
}

// Flexible GMRES (right preconditioning z_j = M(v_j), Saad 1993) for
// A d = r with A the tree's apply in its current precision, from d = 0,
// stopping at a relative reduction inner_rtol or m iterations.  Z and the
// basis live in ws (allocated by the caller).  iters += iterations done.
pfmm_status fgmres(pfmm_tree* t, const pfmm_precond* pc, const double* D, const double* r, double* d,
                   double inner_rtol, int m, Workspace& ws, double* Z, double* part, hipStream_t st, int& iters) {
    const int64_t n = tree_dofs(t);
    const int64_t ld = n;
    const int nb = (int)std::min<int64_t>(kMaxBlocks, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), e(m + 2, 0.0), hbuf(2 * (m + 1) + 1);
    auto Hij = [&](int i, int j) -> double& { return H[(size_t)j * (m + 1) + i]; };
    multidot(ws, r, ld, 1, r, n, nb, ws.col, st);
    HIP_CHECK(hipMemcpyAsync(hbuf.data(), ws.col, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    const double beta = std::sqrt(hbuf[0]);
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, r, d, 0.0, n);
    if (!(beta > 0.0)) return std::isfinite(beta) ? PFMM_OK : set_error(PFMM_ENONFINITE, "residual not finite");
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, r, ws.basis, 1.0 / beta, n);
    e[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
        double* vj = ws.basis + (int64_t)j * ld;
        double* zj = Z + (int64_t)j * ld;
        double* w = ws.basis + (int64_t)(j + 1) * ld;
        if (pc)
            PS_TRY(precond_apply(pc, vj, zj, D, tree_adjacency(t), tree_triangles(t), n, part, st));
        else hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, vj, zj, 1.0, n);
        PS_TRY(tree_apply(t, false, zj, w, st));
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
        if (!std::isfinite(hn)) return set_error(PFMM_ENONFINITE, "non-finite value in the flexible Arnoldi process");
        Hij(j + 1, j) = hn;
        if (hn > 0.0) hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, w, w, 1.0 / hn, n);
        for (int i = 0; i < j; ++i) {
            const double a = Hij(i, j), c = Hij(i + 1, j);
            Hij(i, j) = cs[i] * a + sn[i] * c;
            Hij(i + 1, j) = -sn[i] * a + cs[i] * c;
        }
        const double rr = std::hypot(Hij(j, j), Hij(j + 1, j));
        if (!(rr > 0.0)) break;   // breakdown: keep what was built
        cs[j] = Hij(j, j) / rr;
        sn[j] = Hij(j + 1, j) / rr;
        Hij(j, j) = rr;
        Hij(j + 1, j) = 0.0;
        e[j + 1] = -sn[j] * e[j];
        e[j] = cs[j] * e[j];
        k = j + 1;
        ++iters;
        if (std::fabs(e[j + 1]) / beta <= inner_rtol || hn == 0.0) break;
    }
    std::vector<double> y(k);
    for (int i = k - 1; i >= 0; --i) {
        double sum = e[i];
        for (int l = i + 1; l < k; ++l) sum -= Hij(i, l) * y[l];
        y[i] = sum / Hij(i, i);
    }
    if (k > 0) {
        HIP_CHECK(hipMemcpyAsync(ws.coef, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kBlock), 0, st, Z, ld, k, ws.coef, 1.0,
                           (const double*)nullptr, d, n);
    }
    HIP_CHECK(hipStreamSynchronize(st));
    return PFMM_OK;
}

// ||v||_2 (device vector) on the host, through the multi-dot kernels.
pfmm_status norm2(Workspace& ws, const double* v, int64_t n, hipStream_t st, double& out) {
    const int nb = (int)std::min<int64_t>(kMaxBlocks, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
    multidot(ws, v, n, 1, v, n, nb, ws.col, st);
    double h = 0.0;
    HIP_CHECK(hipMemcpyAsync(&h, ws.col, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    out = std::sqrt(h);
    return PFMM_OK;
}

// Iterative refinement in FP64 around flexible GMRES (see pfmm_solve_V_precond).
pfmm_status solve_ir(pfmm_tree* t, const pfmm_precond* pc, int inner_prec, const double* b, double* x,
                     const pfmm_solve_opts& o, pfmm_solve_info* info, hipStream_t st) {
    const int64_t n = tree_dofs(t);
    const int m = o.max_iter;
    Workspace ws;
    double *Z, *r, *dvec, *D = nullptr, *part;
    PS_TRY(ws.alloc(&ws.basis, (size_t)(m + 1) * n));
    PS_TRY(ws.alloc(&Z, (size_t)m * n));
    PS_TRY(ws.alloc(&ws.partial, (size_t)kMaxBlocks * (m + 1)));
    PS_TRY(ws.alloc(&ws.col, (size_t)2 * (m + 1) + 1));
    PS_TRY(ws.alloc(&ws.coef, (size_t)m + 1));
    PS_TRY(ws.alloc(&r, (size_t)n));
    PS_TRY(ws.alloc(&dvec, (size_t)n));
    PS_TRY(ws.alloc(&part, pc ? precond_scratch_doubles(n) : 1024));
    if (pc) {
        PS_TRY(ws.alloc(&D, (size_t)tree_triangles(t)));
        PS_TRY(tree_near_diag(t, D, st));
    }
    if (info) { info->history_len = 0; info->iters = 0; info->outer = 0; info->precond_fallback = 0; }
    auto record = [&](double v) {
        if (info && info->history && info->history_len < info->history_cap) info->history[info->history_len++] = v;
    };
    double nb_ = 0.0;
    PS_TRY(norm2(ws, b, n, st, nb_));
    if (!std::isfinite(nb_)) return set_error(PFMM_ENONFINITE, "right-hand side is not finite");
    if (!(nb_ > 0.0)) {
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, x, 0.0, n);
        HIP_CHECK(hipStreamSynchronize(st));
        if (info) { info->converged = 1; info->rel_residual = 0.0; info->true_rel_residual = 0.0; }
        return PFMM_OK;
    }
    const int saved = tree_precision(t);
    // r = b - V_h x (FP64) for the current x
    auto residual = [&](double& res_out) -> pfmm_status {
        (void)pfmm_set_precision(t, PFMM_FP64);
        pfmm_status s2 = tree_apply(t, false, x, r, st);
        (void)pfmm_set_precision(t, saved);
        if (s2 != PFMM_OK) return s2;
        hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, r, n);           // r = V x - b
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, r, r, -1.0, n);   // r = b - V x
        double rn = 0.0;
        s2 = norm2(ws, r, n, st, rn);
        res_out = rn / nb_;
        return s2;
    };
    int iters = 0, outer = 0;
    double res = 1.0, prev = 2.0;
    pfmm_status status = PFMM_OK;
    if (o.x0_dev) {
        if (o.x0_dev != x)
            HIP_CHECK(hipMemcpyAsync(x, o.x0_dev, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
        PS_TRY(residual(res));
        if (!std::isfinite(res)) return set_error(PFMM_ENONFINITE, "initial iterate gives a non-finite residual");
    } else {
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, x, 0.0, n);
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, r, 1.0, n);
    }
    bool fallback = false;
    while (true) {
        record(res);
        if (res <= o.rtol || iters >= m * 20) break;
        if (res > 0.5 * prev) { fallback = true; break; }
        prev = res;
        (void)pfmm_set_precision(t, inner_prec);
        status = fgmres(t, pc, D, r, dvec, std::max(1e-4, 0.5 * o.rtol / res), m, ws, Z, part, st, iters);
        (void)pfmm_set_precision(t, saved);
        if (status == PFMM_ENONFINITE) {
            // the preconditioned inner solve broke down (a non-finite
            // preconditioner output): x and r are untouched, solve on plainly
            status = PFMM_OK;
            fallback = true;
            break;
        }
        if (status != PFMM_OK) break;
        // x += d; r = b - V_h x (FP64)
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, dvec, dvec, -1.0, n);
        hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kBlock), 0, st, dvec, x, n);
        ++outer;
        double rnew = 0.0;
        status = residual(rnew);
        if (status != PFMM_OK) break;
        if (!std::isfinite(rnew) || rnew > res) {
            // the step made things worse: undo it (x -= d) and fall back
            hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, dvec, dvec, -1.0, n);
            hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kBlock), 0, st, dvec, x, n);
            status = residual(rnew);
            if (status != PFMM_OK) break;
            res = rnew;
            fallback = true;
            break;
        }
        res = rnew;
    }
    (void)pfmm_set_precision(t, saved);
    if (status != PFMM_OK) return status;
    if (!std::isfinite(res)) return set_error(PFMM_ENONFINITE, "non-finite residual");
    if (fallback && res <= o.rtol) fallback = false;
    if (fallback) {
        // plain FP64 GMRES on the current residual: x += V_h^{-1} r
        (void)pfmm_set_precision(t, PFMM_FP64);
        Workspace w2;
        pfmm_solve_opts o2 = o;
        o2.x0_dev = nullptr;
        o2.rtol = std::min(1.0, o.rtol / res);
        pfmm_solve_info i2{};
        status = gmres(t, r, dvec, o2, &i2, w2, st);
        (void)pfmm_set_precision(t, saved);
        if (status != PFMM_OK && status != PFMM_ENOTCONV) return status;
        iters += i2.iters;
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, dvec, dvec, -1.0, n);
        hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kBlock), 0, st, dvec, x, n);
        (void)pfmm_set_precision(t, PFMM_FP64);
        status = tree_apply(t, false, x, r, st);
        (void)pfmm_set_precision(t, saved);
        if (status != PFMM_OK) return status;
        hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kBlock), 0, st, b, r, n);
        double rn = 0.0;
        PS_TRY(norm2(ws, r, n, st, rn));
        res = rn / nb_;
        record(res);
    }
    if (info) {
        info->iters = iters;
        info->outer = outer;
        info->precond_fallback = fallback ? 1 : 0;
        info->rel_residual = res;
        info->true_rel_residual = res;
        info->converged = res <= o.rtol ? 1 : 0;
    }
    if (res > o.rtol)
        return set_error(PFMM_ENOTCONV, "preconditioned solve stopped at relative residual " + std::to_string(res));
    return PFMM_OK;
}

pfmm_status check_opts(const pfmm_solve_opts* o, pfmm_solve_opts& out) {
    pfmm_default_solve_opts(&out);
    if (o) out = *o;
    if (!(out.rtol >= 0.0) || !std::isfinite(out.rtol)) return set_error(PFMM_EINVAL, "rtol must be finite and >= 0");
    if (out.max_iter < 1 || out.max_iter > 100000) return set_error(PFMM_EINVAL, "max_iter must be in 1..100000");
    if (out.inner_precision != PFMM_FP64 && out.inner_precision != PFMM_MIXED_FP32 &&
        out.inner_precision != PFMM_MIXED_BF16)
        return set_error(PFMM_EINVAL, "unknown inner precision");
    return PFMM_OK;
}

// dirichlet: 0 b given, 1 p0 datum g (b = (1/2 M_h + K_h) g), 2 p1 datum.
pfmm_status solve_common(pfmm_tree* t, const double* b_or_g, double* w, const pfmm_solve_opts* o,
                         pfmm_solve_info* info, void* stream, int dirichlet) {
    if (!t || !b_or_g || !w) return set_error(PFMM_EINVAL, "NULL argument");
    if (b_or_g == w) return set_error(PFMM_EINVAL, "the right-hand side and the solution must not alias");
    if (!tree_has(t, PFMM_OP_V)) return set_error(PFMM_EINVAL, "V_h was not built for this tree");
    if (dirichlet == 1 && !tree_has(t, PFMM_OP_K)) return set_error(PFMM_EINVAL, "K_h was not built for this tree");
    if (dirichlet == 2 && !tree_has(t, PFMM_OP_K1))
        return set_error(PFMM_EINVAL, "the p1 double layer was not built for this tree");
    pfmm_solve_opts opt;
    PS_TRY(check_opts(o, opt));
    if (opt.x0_dev == b_or_g) return set_error(PFMM_EINVAL, "x0 must not alias the right-hand side");
    if (hipSetDevice(tree_device(t)) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    const bool refine = opt.precond || opt.precond_path || opt.inner_precision != PFMM_FP64;
    if (refine) {
        // the inner precision must be available on this tree
        const int saved = tree_precision(t);
        PS_TRY(pfmm_set_precision(t, opt.inner_precision));
        (void)pfmm_set_precision(t, saved);
    }
    const int64_t n = tree_dofs(t);
    size_t fr = 0, tot = 0;
    HIP_CHECK(hipMemGetInfo(&fr, &tot));
    const uint64_t need = (refine ? 2 * (uint64_t)opt.max_iter + 5 : (uint64_t)opt.max_iter + 2) * n * 8 +
                          (uint64_t)kMaxBlocks * (opt.max_iter + 1) * 8;
    if (need > fr)
        return set_error(PFMM_ENOMEM, "solve workspace needs " + std::to_string(need) + " bytes, " +
                                          std::to_string(fr) + " free (lower max_iter)");
    // a weights file is loaded for the call
    pfmm_precond* loaded = nullptr;
    const pfmm_precond* pc = opt.precond;
    if (!pc && opt.precond_path) {
        const pfmm_status ls = pfmm_precond_load(opt.precond_path, tree_device(t), &loaded);
        if (ls != PFMM_OK) return ls;
        pc = loaded;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    Workspace ws;
    const double* b = b_or_g;
    pfmm_status s = PFMM_OK;
    if (dirichlet) {
        s = ws.alloc(&ws.b, (size_t)n);
        if (s == PFMM_OK)
            s = dirichlet == 2 ? pfmm_dirichlet_rhs_p1(t, b_or_g, ws.b, stream) : pfmm_dirichlet_rhs(t, b_or_g, ws.b, stream);
        b = ws.b;
    }
    if (s == PFMM_OK) s = refine ? solve_ir(t, pc, opt.inner_precision, b, w, opt, info, st)
                                 : gmres(t, b, w, opt, info, ws, st);
    const hipError_t e = hipStreamSynchronize(st);
    if (loaded) pfmm_precond_destroy(loaded);
    if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (s == PFMM_OK && e != hipSuccess) return set_error(PFMM_EDEVICE, hipGetErrorString(e));
    return s;
}

// Scratch of pfmm_precond_apply_noalloc: the diagonal of V_h per triangle,
// the reduction partials and the three FP32 feature fields of one vector.
// One copy per GPU (each device holds the array from the library's first use
// on it until the process ends).  Host code never passes `scratch` itself to
// a kernel: it is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, looked up once per device.
constexpr size_t kScratchDoubles = (size_t)PFMM_NOALLOC_SCRATCH_BYTES / sizeof(double);
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev` (looked up on the
// first call for that device).
pfmm_status scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return set_error(PFMM_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(PFMM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
    return PFMM_OK;
}

}  // namespace

extern "C" {

pfmm_status pfmm_default_solve_opts(pfmm_solve_opts* out) {
    if (!out) return set_error(PFMM_EINVAL, "NULL options");
    std::memset(out, 0, sizeof(*out));
    out->rtol = 1e-8;
    out->max_iter = 200;
    out->inner_precision = PFMM_FP64;
    out->x0_dev = nullptr;
    out->precond = nullptr;
    out->precond_path = nullptr;
    return PFMM_OK;
}

pfmm_status pfmm_dirichlet_rhs(pfmm_tree* t, const double* g_dev, double* b_dev, void* stream) {
    if (!t || !g_dev || !b_dev) return set_error(PFMM_EINVAL, "NULL argument");
    if (!tree_has(t, PFMM_OP_K)) return set_error(PFMM_EINVAL, "K_h was not built for this tree");
    if (hipSetDevice(tree_device(t)) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    const int64_t n = tree_dofs(t);
    hipStream_t st = (hipStream_t)stream;
    PS_TRY(tree_apply(t, true, g_dev, b_dev, st));
    hipLaunchKernelGGL(k_half_mass, dim3(blocks_for(n)), dim3(kBlock), 0, st, g_dev, tree_area(t), tree_steps(t),
                       b_dev, tree_triangles(t), n);
    HIP_CHECK(hipGetLastError());
    return PFMM_OK;
}

pfmm_status pfmm_solve_V(pfmm_tree* t, const double* b_dev, double* w_dev, const pfmm_solve_opts* o,
                         pfmm_solve_info* info, void* stream) {
    return solve_common(t, b_dev, w_dev, o, info, stream, 0);
}

pfmm_status pfmm_dirichlet_rhs_p1(pfmm_tree* t, const double* g_dev, double* b_dev, void* stream) {
    if (!t || !g_dev || !b_dev) return set_error(PFMM_EINVAL, "NULL argument");
    if (!tree_has(t, PFMM_OP_K1)) return set_error(PFMM_EINVAL, "the p1 double layer was not built for this tree");
    if (hipSetDevice(tree_device(t)) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    const int64_t n = tree_dofs(t);
    hipStream_t st = (hipStream_t)stream;
    PS_TRY(tree_apply_p1(t, g_dev, b_dev, st));
    hipLaunchKernelGGL(k_half_mass_p1, dim3(blocks_for(n)), dim3(kBlock), 0, st, g_dev, tree_area(t), tree_steps(t),
                       tree_tris(t), b_dev, tree_triangles(t), tree_vertices(t), n);
    HIP_CHECK(hipGetLastError());
    return PFMM_OK;
}

pfmm_status pfmm_solve_dirichlet_p1(pfmm_tree* t, const double* g_dev, double* w_dev, const pfmm_solve_opts* o,
                                    pfmm_solve_info* info, void* stream) {
    return solve_common(t, g_dev, w_dev, o, info, stream, 2);
}

pfmm_status pfmm_solve_dirichlet(pfmm_tree* t, const double* g_dev, double* w_dev, const pfmm_solve_opts* o,
                                 pfmm_solve_info* info, void* stream) {
    return solve_common(t, g_dev, w_dev, o, info, stream, 1);
}

pfmm_status pfmm_solve_V_precond(pfmm_tree* t, const pfmm_precond* pc, int32_t inner_precision, const double* b_dev,
                                 double* w_dev, const pfmm_solve_opts* o, pfmm_solve_info* info, void* stream) {
    if (!t || !b_dev || !w_dev) return set_error(PFMM_EINVAL, "NULL argument");
    if (b_dev == w_dev) return set_error(PFMM_EINVAL, "the right-hand side and the solution must not alias");
    if (!tree_has(t, PFMM_OP_V)) return set_error(PFMM_EINVAL, "V_h was not built for this tree");
    pfmm_solve_opts opt;
    PS_TRY(check_opts(o, opt));
    if (opt.x0_dev == b_dev) return set_error(PFMM_EINVAL, "x0 must not alias the right-hand side");
    if (hipSetDevice(tree_device(t)) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    // the inner precision must be available on this tree
    const int saved = tree_precision(t);
    PS_TRY(pfmm_set_precision(t, inner_precision));
    (void)pfmm_set_precision(t, saved);
    const int64_t n = tree_dofs(t);
    size_t fr = 0, tot = 0;
    HIP_CHECK(hipMemGetInfo(&fr, &tot));
    const uint64_t need = (2 * (uint64_t)opt.max_iter + 5) * n * 8 + (uint64_t)kMaxBlocks * (opt.max_iter + 1) * 8;
    if (need > fr)
        return set_error(PFMM_ENOMEM, "solve workspace needs " + std::to_string(need) + " bytes, " +
                                          std::to_string(fr) + " free (lower max_iter)");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    pfmm_status s = solve_ir(t, pc, inner_precision, b_dev, w_dev, opt, info, st);
    const hipError_t e = hipStreamSynchronize(st);
    if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (s == PFMM_OK && e != hipSuccess) return set_error(PFMM_EDEVICE, hipGetErrorString(e));
    return s;
}

pfmm_status pfmm_precond_apply(const pfmm_precond* pc, pfmm_tree* t, const double* v_dev, double* z_dev,
                               void* stream) {
    if (!pc || !t || !v_dev || !z_dev) return set_error(PFMM_EINVAL, "NULL argument");
    if (!tree_has(t, PFMM_OP_V)) return set_error(PFMM_EINVAL, "V_h was not built for this tree");
    if (v_dev == z_dev) return set_error(PFMM_EINVAL, "v and z must not alias");
    if (hipSetDevice(tree_device(t)) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    Workspace ws;
    double *D, *part;
    pfmm_status s = ws.alloc(&D, (size_t)tree_triangles(t));
    if (s == PFMM_OK) s = ws.alloc(&part, precond_scratch_doubles(tree_dofs(t)));
    if (s == PFMM_OK) s = tree_near_diag(t, D, st);
    if (s == PFMM_OK) s = precond_apply(pc, v_dev, z_dev, D, tree_adjacency(t), tree_triangles(t), tree_dofs(t), part, st);
    if (s == PFMM_OK && hipStreamSynchronize(st) != hipSuccess) s = set_error(PFMM_EDEVICE, "hipStreamSynchronize failed");
    return s;
}

pfmm_status pfmm_precond_apply_noalloc(const pfmm_precond* pc, pfmm_tree* t, const double* v_dev, double* z_dev,
                                       void* stream) {
    if (!pc || !t || !v_dev || !z_dev) return set_error(PFMM_EINVAL, "NULL argument");
    if (!tree_has(t, PFMM_OP_V)) return set_error(PFMM_EINVAL, "V_h was not built for this tree");
    if (v_dev == z_dev) return set_error(PFMM_EINVAL, "v and z must not alias");
    const int64_t n = tree_dofs(t), ex = tree_triangles(t);
    // layout: [0, ex) the diagonal D, then (from a 256-byte boundary) the
    // partials and feature fields of precond_apply
    const int64_t off = (ex + 31) & ~(int64_t)31;
    const size_t need = (size_t)off + precond_scratch_doubles(n);
    if (need > kScratchDoubles)
        return set_error(PFMM_EINVAL, "tree too large for the no-allocation scratch: needs " +
                                          std::to_string(need * sizeof(double)) + " bytes, limit " +
                                          std::to_string((size_t)PFMM_NOALLOC_SCRATCH_BYTES));
    const int dev = tree_device(t);
    if (hipSetDevice(dev) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    double* base = nullptr;
    PS_TRY(scratch_address(dev, &base));
    // every scratch value is written before it is read (the diagonal covers all
    // triangles, the partials all blocks, the fields all DOFs): nothing to clear
    double* D = base;
    double* part = base + off;
    hipStream_t st = (hipStream_t)stream;
    PS_TRY(tree_near_diag(t, D, st));
    PS_TRY(precond_apply(pc, v_dev, z_dev, D, tree_adjacency(t), ex, n, part, st));
    return PFMM_OK;
}

pfmm_status pfmm_precond_train(pfmm_precond* pc, pfmm_tree* t, const double* b_dev, int32_t n_snap, int32_t steps,
                               int32_t batch, float lr, uint64_t seed, float* final_loss, void* stream) {
    if (!pc || !t || !b_dev) return set_error(PFMM_EINVAL, "NULL argument");
    if (!tree_has(t, PFMM_OP_V)) return set_error(PFMM_EINVAL, "V_h was not built for this tree");
    if (n_snap < 1 || n_snap > 64 || steps < 0 || batch < 1 || batch > (1 << 20) || !(lr > 0.f))
        return set_error(PFMM_EINVAL, "n_snap in 1..64, steps >= 0, batch in 1..2^20 and lr > 0 required");
    if (hipSetDevice(tree_device(t)) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    const int64_t n = tree_dofs(t);
    hipStream_t st = (hipStream_t)stream;
    const int saved = tree_precision(t);
    (void)pfmm_set_precision(t, PFMM_FP64);
    // 1. a plain FP64 solve to 1e-10, with the iterates x_k at n_snap
    //    iteration counts spread over it
    pfmm_solve_opts o;
    pfmm_default_solve_opts(&o);
    o.rtol = 1e-10;
    o.max_iter = 400;
    Workspace ws, ws2;
    double *xs, *snap, *R, *E, *D;
    pfmm_status s = ws.alloc(&xs, (size_t)n);
    if (s == PFMM_OK) s = ws2.alloc(&snap, (size_t)n_snap * n);
    pfmm_solve_info i1{};
    std::vector<int> snaps;
    if (s == PFMM_OK) s = gmres(t, b_dev, xs, o, &i1, ws, st, n_snap, snap, &snaps);
    if (s != PFMM_OK) { (void)pfmm_set_precision(t, saved); return s; }
    if (i1.iters < 2) { (void)pfmm_set_precision(t, saved); return set_error(PFMM_EINVAL, "training solve too short"); }
    const int ns = (int)snaps.size();
    const int np = 2 * ns;   // error snapshots, then Krylov basis vectors
    s = ws2.alloc(&R, (size_t)np * n);
    if (s == PFMM_OK) s = ws2.alloc(&E, (size_t)np * n);
    // 2. Krylov basis vectors v_j of the solve (columns 1.. of ws.basis),
    //    spread over it: exact pairs (V_h v_j, v_j) on the space GMRES explores
    for (int i = 0; i < ns && s == PFMM_OK; ++i) {
        const int j = 1 + (int)((double)i * std::max(1, i1.iters - 1) / ns);
        hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, ws.basis + (int64_t)j * n,
                           E + (int64_t)(ns + i) * n, 1.0, n);
    }
    if (s == PFMM_OK) s = ws2.alloc(&D, (size_t)tree_triangles(t));
    if (s != PFMM_OK) { (void)pfmm_set_precision(t, saved); return s; }
    // 3. pairs: e = x* - x_k (and the basis vectors above), r = V_h e
    for (int p = 0; p < np && s == PFMM_OK; ++p) {
        double* ep = E + (int64_t)p * n;
        if (p < ns) {
            hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, xs, ep, 1.0, n);
            hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kBlock), 0, st, snap + (int64_t)p * n, ep, n);
        }
        s = tree_apply(t, false, ep, R + (int64_t)p * n, st);
    }
    if (s == PFMM_OK) s = tree_near_diag(t, D, st);
    (void)pfmm_set_precision(t, saved);
    if (s != PFMM_OK) return s;
    // 4. fit
    s = precond_fit(pc, R, E, np, D, tree_adjacency(t), tree_triangles(t), n, steps, batch, lr, seed, st);
    if (s == PFMM_OK && final_loss) *final_loss = precond_last_loss(pc);
    return s;
}

}  // extern "C"
