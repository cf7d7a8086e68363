// Representation formula at interior points (Section 2): with zero initial
// data the solution of the heat equation inside the domain is
//     u(x, t) = (V~ w)(x, t) - (W u)(x, t),
// the single-layer potential V~ (kernel G) of the Neumann trace w and the
// double-layer potential W (kernel alpha dG/dn_y) of the Dirichlet trace,
// here for piecewise-constant data in space and time.  The time integral
// over a step is closed-form through the first antiderivatives
//     G1(r, s) = erfc(z) / (4 pi alpha r),                       dG1/ds = G,
//     K1(r, s) = [erfc(z) + r exp(-z^2) / sqrt(pi alpha s)] / (4 pi r^3),
//                                                       dK1/ds = G / (2 s),
// with z = r / (2 sqrt(alpha s)); a step [t_j, t_{j+1}] contributes
// F(t - t_j) - F(max(t - t_{j+1}, 0)), F(., 0) = 0.  Summed over the steps
// before t this telescopes to sum_j (w_j - w_{j-1}) F(t - t_j) (w_{-1} = 0),
// one antiderivative per time node (minus w_last F(t - t_E) for t past the
// last node).  The space integral over each triangle
// is the collapsed Gauss rule with q points per direction.
//
// Direct summation over all space-time elements: one workgroup per target
// point, its threads over (triangle, quadrature point) pairs, each looping
// over the time nodes before the target time; a fixed-order block reduction
// makes the result deterministic.  Work per target: n_tri q^2 (steps before
// t) antiderivative pairs (erfc, exp): ALU-bound.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pfmm.h"
#include "plan.hpp"

using namespace pfmm;

namespace {

constexpr int kT = 256;
constexpr int kMaxQ = 16;

struct Rule1D {
    double g[kMaxQ], w[kMaxQ];   // Gauss-Legendre on [0, 1]
    int q;
};

#define HIP_CHECK(expr)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return set_error(PFMM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

__global__ void __launch_bounds__(kT) k_represent(const double* __restrict__ verts, const int* __restrict__ tris,
                                                  const double* __restrict__ area, const double* __restrict__ normal,
                                                  const double* __restrict__ tn, int n_tri, int n_steps, double alpha,
                                                  const double* __restrict__ w, const double* __restrict__ u,
                                                  const double* __restrict__ xt, double* __restrict__ out, Rule1D R) {
    __shared__ double red[kT];
    const int64_t i = blockIdx.x;
    const double x0 = xt[4 * i], x1 = xt[4 * i + 1], x2 = xt[4 * i + 2], t = xt[4 * i + 3];
    const int q = R.q, q2 = q * q;
    // steps that start before t
    int J = 0;
    while (J < n_steps && tn[J] < t) ++J;
    const double inv4pa = 1.0 / (4.0 * M_PI * alpha);
    const double isa = 1.0 / sqrt(M_PI * alpha);
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)n_tri * q2; e += kT) {
        const int k = (int)(e / q2), p = (int)(e - (int64_t)k * q2);
        const int a = p / q, b = p - a * q;
        // collapsed rule: y = A + s (B - A) + s v (C - B), weight 2 |gamma| w_a w_b s
        const double s = R.g[a], sv = R.g[a] * R.g[b];
        const double* A = verts + 3 * tris[3 * k];
        const double* B = verts + 3 * tris[3 * k + 1];
        const double* C = verts + 3 * tris[3 * k + 2];
        const double y0 = A[0] + s * (B[0] - A[0]) + sv * (C[0] - B[0]);
        const double y1 = A[1] + s * (B[1] - A[1]) + sv * (C[1] - B[1]);
        const double y2 = A[2] + s * (B[2] - A[2]) + sv * (C[2] - B[2]);
        const double wq = 2.0 * area[k] * R.w[a] * R.w[b] * s;
        const double d0 = x0 - y0, d1 = x1 - y1, d2 = x2 - y2;
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double dn = d0 * normal[3 * k] + d1 * normal[3 * k + 1] + d2 * normal[3 * k + 2];
        const double ir = 1.0 / r;
        double sv_acc = 0.0, sk_acc = 0.0, wp = 0.0, up = 0.0;
        for (int j = 0; j < J; ++j) {
            const double sl = t - tn[j];                     // > 0
            const double z = 0.5 * r / sqrt(alpha * sl);
            const double ec = erfc(z);
            if (w) {
                const double wj = w[(int64_t)j * n_tri + k];
                sv_acc += (wj - wp) * (ec * inv4pa * ir);
                wp = wj;
            }
            if (u) {
                const double uj = u[(int64_t)j * n_tri + k];
                const double k1 = (ec + r * exp(-z * z) * isa / sqrt(sl)) * (0.25 / M_PI) * ir * ir * ir;
                sk_acc += (uj - up) * k1;
                up = uj;
            }
        }
        if (J > 0 && tn[J] < t) {
            // t after the last node: the last step ends before t
            const double sl = t - tn[J];
            const double z = 0.5 * r / sqrt(alpha * sl);
            const double ec = erfc(z);
            sv_acc -= wp * (ec * inv4pa * ir);
            sk_acc -= up * ((ec + r * exp(-z * z) * isa / sqrt(sl)) * (0.25 / M_PI) * ir * ir * ir);
        }
        acc += wq * (sv_acc - dn * sk_acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
}

}  // namespace

extern "C" {

pfmm_status pfmm_representation(pfmm_tree* t, const double* w_dev, const double* u_dev, const double* xt_dev,
                                int64_t n_points, int32_t q, double* out_dev, void* stream) {
    if (!t || !xt_dev || !out_dev) return set_error(PFMM_EINVAL, "NULL argument");
    if (n_points < 0 || n_points > (int64_t)INT32_MAX) return set_error(PFMM_EINVAL, "n_points out of range");
    if (q < 1 || q > kMaxQ) return set_error(PFMM_EINVAL, "q must be in 1..16");
    if (hipSetDevice(tree_device(t)) != hipSuccess) return set_error(PFMM_EDEVICE, "hipSetDevice failed");
    TreeGeom G{};
    const pfmm_status s = tree_geometry(t, &G);
    if (s != PFMM_OK) return s;
    if (n_points == 0) return PFMM_OK;
    Rule1D R{};
    std::vector<double> g, w;
    gauss_legendre01(q, g, w);
    for (int i = 0; i < q; ++i) { R.g[i] = g[i]; R.w[i] = w[i]; }
    R.q = q;
    hipLaunchKernelGGL(k_represent, dim3((unsigned)n_points), dim3(kT), 0, (hipStream_t)stream, G.verts, G.tris,
                       G.area, G.normal, G.tnodes, G.n_tri, G.n_steps, G.alpha, w_dev, u_dev, xt_dev, out_dev, R);
    HIP_CHECK(hipGetLastError());
    return PFMM_OK;
}

}  // extern "C"
