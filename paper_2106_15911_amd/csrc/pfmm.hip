// MI355X (gfx950) space-time FMM for the heat equation: device kernels and
// the C ABI declared in include/pfmm.h.
//
// Apply pipeline (Algorithm 2 of the paper), all on one stream:
//   permute w into tree order (time-major, spatially sorted triangles)
//   S2M on leaves, M2M for levels p-1..2, M2L for levels 2..p,
//   L2L for levels 3..p, L2T on leaves (overwrites f),
//   nearfield product over the stored causal blocks (adds to f),
//   permute f back to the natural order.
// Everything is FP64.  Each output value is owned by exactly one thread, so
// applies are deterministic (no floating-point atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <map>
#include <vector>

#include "internal.hpp"
#include "near_kernels.hpp"
#include "pfmm.h"
#include "plan.hpp"
#include "tables.hpp"

using namespace pfmm;

namespace {

thread_local std::string g_err;

pfmm_status fail(pfmm_status s, const std::string& m) {
    g_err = m;
    return s;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(PFMM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

constexpr int kChunk = 32;          // M2L output rows per wave
constexpr int kWave = 64;


// ------------------------------------------------------------------ permutations

__global__ void k_permute_in(const double* __restrict__ w, double* __restrict__ wd,
                             const int* __restrict__ inv_sigma, int E_x, int64_t N) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int64_t t = i / E_x;
    int p = (int)(i - t * E_x);
    wd[i] = w[t * E_x + inv_sigma[p]];
}

// p1 trial functions: the vertex values u[jt][v] (natural order) as local
// values per triangle position and vertex, w3[jt][3 p + i] = u[jt][vertex i
// of the triangle at position p].
__global__ void k_gather_p1(const double* __restrict__ u, double* __restrict__ w3, const int* __restrict__ inv_sigma,
                            const int* __restrict__ tris, int n_v, int E_x, int64_t n3) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const int64_t jt = i / (3 * (int64_t)E_x);
    const int rem = (int)(i - jt * 3 * (int64_t)E_x);
    const int p = rem / 3, c = rem - 3 * p;
    w3[i] = u[jt * n_v + tris[3 * inv_sigma[p] + c]];
}

// f = far + near, back to the natural order.  A sum of two FP64 terms is
// rounded once, so it already equals what a compensated (Neumaier) sum
// returns: no correction term is needed here.
__global__ void k_permute_out(const double* __restrict__ fd, const double* __restrict__ fn, double* __restrict__ f,
                              const int* __restrict__ sigma, int E_x, int64_t N) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int64_t t = i / E_x;
    int k = (int)(i - t * E_x);
    const int64_t p = t * E_x + sigma[k];
    f[i] = fd[p] + fn[p];
}

__global__ void k_fill(double* __restrict__ x, double v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// ------------------------------------------------------------------ far field

struct CoefMaps {
    const int* coef_a;      // Nc
    const int* coef_deg;    // Nc
    const int* coef_k;      // Nc x 3
    const int* coef_kpos;   // Nc: position of the multi-index in the Nk list
    const int* kidx;        // Nk x 3 (degree-sorted multi-indices)
    const int* kposmap;     // (m+1)^3 -> position in the Nk list
    const int* cidx;        // (m_t+1) x Nk -> coefficient index
    int Nc, Nk, mt, mx;
};

// M2L operator generation: op[(class, Delta)][chunk][c_in][r] =
//   C_ab prod_j E_{kappa_j, nu_j}(r_j, d_ab)  if |kappa| + |nu| <= m_x  (eq. exp_coeffs_3d)
__global__ void k_m2l_opgen(double* __restrict__ ops, const double* __restrict__ E1, const double* __restrict__ Cab,
                            const int* __restrict__ off3, const int* __restrict__ chunk_cols,
                            const int64_t* __restrict__ chunk_off, CoefMaps cm, int n_chunks, int64_t op_size,
                            int R, int64_t total) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t opi = i / op_size;
    int64_t e = i - opi * op_size;
    int j = 0;
    while (j + 1 < n_chunks && chunk_off[j + 1] <= e) ++j;
    e -= chunk_off[j];
    const int cin = (int)(e / kChunk), rr = (int)(e % kChunk);
    const int row = j * kChunk + rr;
    const int cls = (int)(opi / 2), D = (int)(opi % 2);
    double v = 0.0;
    if (row < cm.Nc && cin < chunk_cols[j]) {
        const int b = cm.coef_a[row], a = cm.coef_a[cin];
        if (cm.coef_deg[row] + cm.coef_deg[cin] <= cm.mx) {
            const int nt1 = cm.mt + 1, nx1 = cm.mx + 1, nR = 2 * R + 1;
            v = Cab[((int64_t)D * nt1 + a) * nt1 + b];
            for (int ax = 0; ax < 3; ++ax) {
                const int o = off3[3 * cls + ax] + R;
                const double* E = E1 + ((((int64_t)D * nR + o) * nt1 + a) * nt1 + b) * nx1 * nx1;
                v *= E[cm.coef_k[3 * cin + ax] * nx1 + cm.coef_k[3 * row + ax]];
            }
        }
    }
    ops[i] = v;
}

// M2L (eq. m2l): lambda[X, rows of chunk, k] = sum over sources (Y, Delta) of
// op(X-Y, Delta)[rows, c] * mu[Y, c, k - Delta].  One wave per
// (target slot, 64 intervals, 32-row chunk); lane = interval.
__global__ void __launch_bounds__(64) k_m2l(const double* __restrict__ mu, double* __restrict__ lam,
                                            const double* __restrict__ ops, const int* __restrict__ ptr,
                                            const int* __restrict__ src, const int* __restrict__ cls,
                                            const int* __restrict__ chunk_cols, const int64_t* __restrict__ chunk_off,
                                            int Nc, int n_int, int64_t op_size) {
    const int xs = blockIdx.x;
    const int k = blockIdx.y * kWave + threadIdx.x;
    const int j = blockIdx.z;
    const int ncol = chunk_cols[j];
    double acc[kChunk];
#pragma unroll
    for (int r = 0; r < kChunk; ++r) acc[r] = 0.0;
    for (int s = ptr[xs]; s < ptr[xs + 1]; ++s) {
        const int ys = src[s];
        const int oc = cls[s];
        for (int D = 2; D <= 3; ++D) {
            const int ks = k - D;
            const bool valid = (k < n_int) && (ks >= 0) && (D == 2 || (k & 1));
            const double* op = ops + (int64_t)(2 * oc + (D - 2)) * op_size + chunk_off[j];
            const double* m = mu + (int64_t)ys * Nc * n_int + (valid ? ks : 0);
            for (int c = 0; c < ncol; ++c) {
                const double mv = valid ? m[(int64_t)c * n_int] : 0.0;
                const double* o = op + c * kChunk;
#pragma unroll
                for (int r = 0; r < kChunk; ++r) acc[r] = fma(o[r], mv, acc[r]);
            }
        }
    }
    if (k < n_int) {
#pragma unroll
        for (int r = 0; r < kChunk; ++r) {
            const int row = j * kChunk + r;
            if (row < Nc) lam[((int64_t)xs * Nc + row) * n_int + k] = acc[r];
        }
    }
}

#include "m2l_kernels.hpp"


// Index data of the separable re-expansions, shared by k_m2m_sep and
// k_l2l_sep.  Inside a block, moments and locals are held as [a][p][kk]:
// time index a, position p of the spatial multi-index in the degree-sorted
// list (kidx), interval kk of the block innermost.  ax[(j * Nk + p) * (m_x+1) + t]
// is the position of multi-index p with its component j replaced by t, or -1
// when that exceeds the total degree m_x.
constexpr int kMaxT = 17;   // time nodes per interval at the largest Lagrange degree (16)

struct SepMaps {
    const int* coef_a;      // Nc: time index of coefficient c
    const int* coef_kpos;   // Nc: spatial position of coefficient c
    const int* cidx;        // (m_t+1) x Nk -> coefficient index
    const int* kidx;        // Nk x 3 multi-indices
    const int* ax;          // 3 x Nk x (m_x+1)
    int Nc, Nk, mt, mx;
};

// Block of a (slot, interval block) grid (S2M, M2M, L2L).  Workgroups are
// dealt to the 8 XCDs round-robin by linear id; remap so that each XCD runs
// a contiguous range of slots with the interval blocks of a slot
// consecutive: the blocks of one slot read and write neighbouring pieces of
// the slot's [coefficient][interval] rows, which then meet in one L2
// (measured at 3072 x 1024: S2M 1.30 -> 0.70 ms, M2M 1.98 -> 1.61, L2L
// 1.69 -> 1.51; L2T, whose blocks are row chunks, 1.34 -> 1.39, kept in
// grid order).
__device__ __forceinline__ int2 slot_block() {
    const int ns = gridDim.x, nb = gridDim.y;
    const int lin = blockIdx.x + ns * blockIdx.y;
    const int per = (ns * nb) / 8;
    const int lm = lin < per * 8 ? (lin % 8) * per + lin / 8 : lin;
    return int2{lm / nb, lm % nb};
}

// One 1D re-expansion pass along axis j over a [nt1][Nk][KI] block.
// Forward (M2M): out[a][p] = sum_{t <= n_j(p)} Q_j[t][n_j(p)] in[a][p with n_j = t].
// Transposed (L2L): out[a][p] = sum_{t >= n_j(p)} Q_j[n_j(p)][t] in[a][p with n_j = t].
template <bool TRANSPOSED, bool ACCUMULATE>
__device__ __forceinline__ void sep_pass(const double* __restrict__ in, double* __restrict__ out,
                                         const double* __restrict__ Qj, const int* __restrict__ axj,
                                         const int* __restrict__ kid, int j, int nt1, int Nk, int nx1, int KI,
                                         int nk) {
    const int total = nt1 * Nk * KI;
    for (int o = threadIdx.x; o < total; o += blockDim.x) {
        const int kk = o % KI;
        if (kk >= nk) continue;
        const int ap = o / KI;            // a * Nk + p
        const int pp = ap % Nk, a = ap / Nk;
        const int n = kid[3 * pp + j];
        const int* src = axj + pp * nx1;
        const double* row = in + (int64_t)a * Nk * KI + kk;
        double acc = 0.0;
        if (!TRANSPOSED) {
            for (int t = 0; t <= n; ++t) acc += Qj[t * nx1 + n] * row[src[t] * KI];
        } else {
            for (int t = n; t < nx1; ++t) {
                const int q = src[t];
                if (q < 0) break;
                acc += Qj[n * nx1 + t] * row[q * KI];
            }
        }
        if (ACCUMULATE) out[o] += acc; else out[o] = acc;
    }
}

// M2M (eqs. temp_m2m, st_m2m) from level l+1 into the boxes of level l that
// have children (inner[xs * n_int_p + k] = 1).  Block = (parent slot, KI parent intervals).  Per child:
// the temporal re-expansion of the child's two intervals per parent interval
// (read straight from HBM, intervals contiguous), then the spatial
// re-expansion as three 1D passes in LDS, accumulated over the children.
__global__ void __launch_bounds__(256) k_m2m_sep(const double* __restrict__ mu_c, double* __restrict__ mu_p,
                                                 const int* __restrict__ par_xs, const int* __restrict__ ch_ptr,
                                                 const int* __restrict__ ch, const double* __restrict__ qt,
                                                 const double* __restrict__ qx, SepMaps m, int n_int_p, int n_int_c,
                                                 int KI, const uint8_t* __restrict__ inner) {
    extern __shared__ double sm[];
    const int nt1 = m.mt + 1, nx1 = m.mx + 1, Nk = m.Nk, Nc = m.Nc;
    const int blk = Nc * KI;
    double* T = sm;                    // [nt1][Nk][KI]
    double* U = T + blk;
    double* Acc = U + blk;
    double* sq = Acc + blk;            // Q of the current child: 3 x nx1 x nx1
    double* sqt = sq + 3 * nx1 * nx1;  // q_t of the block's child intervals: [2 KI][nt1][nt1]
    const SepMaps& L = m;
    const int2 sb = slot_block();
    const int xs = par_xs[sb.x];
    const int k0 = sb.y * KI;
    const int nk = min(KI, n_int_p - k0);
    for (int i = threadIdx.x; i < blk; i += blockDim.x) Acc[i] = 0.0;
    for (int i = threadIdx.x; i < 2 * nk * nt1 * nt1; i += blockDim.x)
        sqt[i] = qt[(int64_t)2 * k0 * nt1 * nt1 + i];
    for (int ci = ch_ptr[xs]; ci < ch_ptr[xs + 1]; ++ci) {
        const int xc = ch[ci];
        __syncthreads();   // previous child's last pass is done with T, U and sq
        for (int i = threadIdx.x; i < 3 * nx1 * nx1; i += blockDim.x) sq[i] = qx[(int64_t)xc * 3 * nx1 * nx1 + i];
        // temporal: T[ap][p][kk] = sum_{b, ac} q_t[2kk+b][ac][ap] mu_c[(ac, p)][2(k0+kk)+b]
        for (int it = threadIdx.x; it < Nk * KI; it += blockDim.x) {
            const int kk = it % KI, pp = it / KI;
            if (kk >= nk) continue;
            double acc[kMaxT];
#pragma unroll
            for (int a = 0; a < kMaxT; ++a) acc[a] = 0.0;
            for (int ac = 0; ac < nt1; ++ac) {
                const double* src = mu_c + ((int64_t)xc * Nc + m.cidx[ac * Nk + pp]) * n_int_c + 2 * (k0 + kk);
                const double v0 = src[0], v1 = src[1];
                const double* q0 = sqt + ((2 * kk) * nt1 + ac) * nt1;
                const double* q1 = q0 + nt1 * nt1;
#pragma unroll
                for (int ap = 0; ap < kMaxT; ++ap)
                    if (ap < nt1) acc[ap] += q0[ap] * v0 + q1[ap] * v1;
            }
#pragma unroll
            for (int ap = 0; ap < kMaxT; ++ap)
                if (ap < nt1) T[((int64_t)ap * Nk + pp) * KI + kk] = acc[ap];
        }
        __syncthreads();
        sep_pass<false, false>(T, U, sq, L.ax, L.kidx, 0, nt1, Nk, nx1, KI, nk);
        __syncthreads();
        sep_pass<false, false>(U, T, sq + nx1 * nx1, L.ax + Nk * nx1, L.kidx, 1, nt1, Nk, nx1, KI, nk);
        __syncthreads();
        sep_pass<false, true>(T, Acc, sq + 2 * nx1 * nx1, L.ax + 2 * Nk * nx1, L.kidx, 2, nt1, Nk, nx1, KI, nk);
    }
    __syncthreads();
    // only boxes with children: a leaf parent keeps its S2M moments, an
    // absent one its zeros
    for (int o = threadIdx.x; o < blk; o += blockDim.x) {
        const int kk = o % KI, c = o / KI;
        if (kk >= nk || !inner[(int64_t)xs * n_int_p + k0 + kk]) continue;
        mu_p[((int64_t)xs * Nc + c) * n_int_p + k0 + kk] = Acc[((int64_t)m.coef_a[c] * Nk + m.coef_kpos[c]) * KI + kk];
    }
}

// L2L (transposes of eqs. temp_m2m / st_m2m) from level l-1 into every box
// of level l.  Block = (child slot, 2 KI child intervals): the parent's
// locals of KI intervals are re-expanded in space by three transposed 1D
// passes in LDS, then in time into the child's intervals (added to the
// child's M2L result; intervals contiguous).
__global__ void __launch_bounds__(256) k_l2l_sep(const double* __restrict__ lam_p, double* __restrict__ lam_c,
                                                 const int* __restrict__ parent, const double* __restrict__ qt,
                                                 const double* __restrict__ qx, SepMaps m, int n_int_c, int n_int_p,
                                                 int KI) {
    extern __shared__ double sm[];
    const int nt1 = m.mt + 1, nx1 = m.mx + 1, Nk = m.Nk, Nc = m.Nc;
    const int blk = Nc * KI;
    double* T = sm;                    // [nt1][Nk][KI] (parent intervals)
    double* U = T + blk;
    double* sq = U + blk;
    double* sqt = sq + 3 * nx1 * nx1;  // q_t of the block's child intervals: [2 KI][nt1][nt1]
    const SepMaps& L = m;
    const int2 sb = slot_block();
    const int xs = sb.x, ps = parent[xs];
    const int kp0 = sb.y * KI;                     // first parent interval
    const int nk = min(KI, n_int_p - kp0);
    for (int i = threadIdx.x; i < 3 * nx1 * nx1; i += blockDim.x) sq[i] = qx[(int64_t)xs * 3 * nx1 * nx1 + i];
    for (int i = threadIdx.x; i < 2 * nk * nt1 * nt1; i += blockDim.x)
        sqt[i] = qt[(int64_t)2 * kp0 * nt1 * nt1 + i];
    for (int o = threadIdx.x; o < blk; o += blockDim.x) {
        const int kk = o % KI, c = o / KI;
        if (kk >= nk) continue;
        T[((int64_t)m.coef_a[c] * Nk + m.coef_kpos[c]) * KI + kk] = lam_p[((int64_t)ps * Nc + c) * n_int_p + kp0 + kk];
    }
    __syncthreads();
    sep_pass<true, false>(T, U, sq, L.ax, L.kidx, 0, nt1, Nk, nx1, KI, nk);
    __syncthreads();
    sep_pass<true, false>(U, T, sq + nx1 * nx1, L.ax + Nk * nx1, L.kidx, 1, nt1, Nk, nx1, KI, nk);
    __syncthreads();
    sep_pass<true, false>(T, U, sq + 2 * nx1 * nx1, L.ax + 2 * Nk * nx1, L.kidx, 2, nt1, Nk, nx1, KI, nk);
    __syncthreads();
    // temporal: lam_c[(bc, p)][kc] += sum_bp q_t[kc][bc][bp] U[bp][p][kc/2 - kp0]
    const int KC = 2 * KI;
    for (int o = threadIdx.x; o < Nc * KC; o += blockDim.x) {
        const int kc = o % KC, c = o / KC;
        if (kc >= 2 * nk) continue;
        const int bc = m.coef_a[c], pp = m.coef_kpos[c];
        const double* q = sqt + (kc * nt1 + bc) * nt1;
        const double* u = U + (int64_t)pp * KI + kc / 2;
        double acc = 0.0;
        for (int bp = 0; bp < nt1; ++bp) acc += q[bp] * u[(int64_t)bp * Nk * KI];
        lam_c[((int64_t)xs * Nc + c) * n_int_c + 2 * kp0 + kc] += acc;
    }
}

// S2M (eq. s2m) by leaf blocks: block = (leaf, KI intervals).  The time
// integrals are applied first, W[a][r][kk] = sum_j A_t[j][a] w[j][r] (the
// densities of the leaf's triangles are contiguous in tree order), then the
// space integrals, mu[(a, p)][kk] = sum_r W[a][r][kk] A_x[r][p], written with
// the intervals contiguous.  A_x of the leaf's spatial box is staged in LDS.
__global__ void __launch_bounds__(256) k_s2m_blk(const double* __restrict__ wd, double* __restrict__ mu,
                                                 const int* __restrict__ leaf_xs, const int64_t* __restrict__ ax_off,
                                                 const int* __restrict__ tb, const int* __restrict__ te,
                                                 const double* __restrict__ At, const double* __restrict__ Ax,
                                                 SepMaps m, int n_int, const int* __restrict__ ist,
                                                 const int* __restrict__ ilen, const uint8_t* __restrict__ lflag,
                                                 int E_x, int KI, int stageA) {
    extern __shared__ double sm[];
    const int nt1 = m.mt + 1, Nk = m.Nk, Nc = m.Nc;
    const int2 sb = slot_block();
    const int li = sb.x, xs = leaf_xs[li];
    const int k0 = sb.y * KI, nk = min(KI, n_int - k0);
    // leaves of more than 64 triangles (single-step intervals) in row chunks
    // of 64, accumulated by the thread that owns each moment (fixed order)
    for (int r0 = 0; r0 < te[xs] - tb[xs]; r0 += 64) {
        const int t0 = tb[xs] + r0, nX = min(64, te[xs] - t0);
        const double* A = Ax + ax_off[li] + (int64_t)r0 * Nk;
        double* W = sm;                                     // [nt1][nX][KI]
        double* sAl = W + nt1 * nX * KI;                    // [nX][Nk] when staged
        if (r0 > 0) __syncthreads();                        // the previous chunk is done with W and sAl
        if (stageA)
            for (int i = threadIdx.x; i < nX * Nk; i += blockDim.x) sAl[i] = A[i];
        const double* sA = stageA ? sAl : A;
        for (int o = threadIdx.x; o < nt1 * nX * KI; o += blockDim.x) {
            const int r = o % nX, rest = o / nX;
            const int kk = rest % KI, a = rest / KI;
            double acc = 0.0;
            if (kk < nk) {
                const int k = k0 + kk;
                const int j0 = ist[k], ns = lflag[(int64_t)li * n_int + k] ? ilen[k] : 0;
                const double* T = At + (int64_t)j0 * nt1 + a;
                const double* wr = wd + (int64_t)j0 * E_x + t0 + r;
                for (int j = 0; j < ns; ++j) acc += T[j * nt1] * wr[(int64_t)j * E_x];
            }
            W[((int64_t)a * nX + r) * KI + kk] = acc;
        }
        __syncthreads();
        // moments of the leaf boxes only (the slot's other intervals belong to
        // boxes with children, filled by M2M, or to absent boxes, kept zero)
        for (int o = threadIdx.x; o < Nc * KI; o += blockDim.x) {
            const int kk = o % KI, c = o / KI;
            if (kk >= nk || !lflag[(int64_t)li * n_int + k0 + kk]) continue;
            const int a = m.coef_a[c], pp = m.coef_kpos[c];
            const double* wv = W + (int64_t)a * nX * KI + kk;
            double acc = 0.0;
            for (int r = 0; r < nX; ++r) acc += wv[r * KI] * sA[r * Nk + pp];
            double* dst = mu + ((int64_t)xs * Nc + c) * n_int + k0 + kk;
            if (r0 == 0) *dst = acc; else *dst += acc;
        }
    }
}

// L2T (eq. l2t) by leaf blocks: block = (leaf, KI intervals).  The leaf's
// locals of KI intervals are loaded with the intervals contiguous, the space
// basis is applied first, U[a][r][kk] = sum_p lambda[(a, p)][kk] A_x[r][p],
// then the time basis, f[j][r] = sum_a A_t[j][a] U[a][r][kk] (overwrites f,
// triangles contiguous).
__global__ void __launch_bounds__(256) k_l2t_blk(const double* __restrict__ lam, double* __restrict__ fd,
                                                 const int* __restrict__ leaf_xs, const int64_t* __restrict__ ax_off,
                                                 const int* __restrict__ tb, const int* __restrict__ te,
                                                 const double* __restrict__ At, const double* __restrict__ Ax,
                                                 SepMaps m, int n_int, const int* __restrict__ ist,
                                                 const int* __restrict__ ilen, const uint8_t* __restrict__ lflag,
                                                 const int2* __restrict__ chunks, int maxlen, int E_x, int KI,
                                                 int stageA) {
    extern __shared__ double sm[];
    const int nt1 = m.mt + 1, Nk = m.Nk, Nc = m.Nc;
    const int2 ch = chunks[blockIdx.x];       // (leaf slot, first row) of a chunk of <= 64 rows
    const int li = ch.x, xs = leaf_xs[li];
    const int t0 = tb[xs] + ch.y, nX = min(64, te[xs] - t0);
    const int k0 = blockIdx.y * KI, nk = min(KI, n_int - k0);
    const double* A = Ax + ax_off[li] + (int64_t)ch.y * Nk;
    double* L = sm;                                     // [nt1][Nk][KI]
    double* U = L + Nc * KI;                            // [nt1][nX][KI]
    double* sAl = U + nt1 * nX * KI;                    // [nX][Nk] when staged
    if (stageA)
        for (int i = threadIdx.x; i < nX * Nk; i += blockDim.x) sAl[i] = A[i];
    const double* sA = stageA ? sAl : A;
    for (int o = threadIdx.x; o < Nc * KI; o += blockDim.x) {
        const int kk = o % KI, c = o / KI;
        L[((int64_t)m.coef_a[c] * Nk + m.coef_kpos[c]) * KI + kk] =
            kk < nk ? lam[((int64_t)xs * Nc + c) * n_int + k0 + kk] : 0.0;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < nt1 * nX * KI; o += blockDim.x) {
        const int kk = o % KI, rest = o / KI;
        const int r = rest % nX, a = rest / nX;
        const double* lv = L + (int64_t)a * Nk * KI + kk;
        const double* ar = sA + r * Nk;
        double acc = 0.0;
        for (int pp = 0; pp < Nk; ++pp) acc += lv[pp * KI] * ar[pp];
        U[((int64_t)a * nX + r) * KI + kk] = acc;
    }
    __syncthreads();
    // f at the steps of the leaf boxes (intervals where the slot is a leaf)
    for (int o = threadIdx.x; o < nk * maxlen * nX; o += blockDim.x) {
        const int r = o % nX, rest = o / nX;
        const int j = rest % maxlen, kk = rest / maxlen;
        const int k = k0 + kk;
        if (j >= ilen[k] || !lflag[(int64_t)li * n_int + k]) continue;
        const double* T = At + ((int64_t)ist[k] + j) * nt1;
        double acc = 0.0;
        for (int a = 0; a < nt1; ++a) acc += T[a] * U[((int64_t)a * nX + r) * KI + kk];
        fd[((int64_t)ist[k] + j) * E_x + t0 + r] = acc;
    }
}

// ------------------------------------------------------------------ nearfield

struct NearGeom {
    const double* verts;    // natural vertices
    const int* tris;        // natural triangles
    const double* area;
    const double* normal;
    const double* centroid;
    const double* maxedge;
    const int* inv_sigma;   // position -> natural triangle
    double h, alpha;
};

struct GroupDev {
    int tb, te, dmax, usize;
    int64_t uoff, toff, mapoff;
};

__device__ __forceinline__ void tri_vertices(const NearGeom& G, int t, double P[3][3]) {
    for (int v = 0; v < 3; ++v) {
        const double* x = G.verts + 3 * G.tris[3 * t + v];
        P[v][0] = x[0]; P[v][1] = x[1]; P[v][2] = x[2];
    }
}

__device__ __forceinline__ bool coplanar(const NearGeom& G, int a, int b) {
    const double* na = G.normal + 3 * a;
    const double* nb = G.normal + 3 * b;
    const double* ca = G.centroid + 3 * a;
    const double* cb = G.centroid + 3 * b;
    const double L = fmax(G.maxedge[a], G.maxedge[b]);
    const double dn = na[0] * nb[0] + na[1] * nb[1] + na[2] * nb[2];
    const double dc = (ca[0] - cb[0]) * nb[0] + (ca[1] - cb[1]) * nb[1] + (ca[2] - cb[2]) * nb[2];
    return fabs(1.0 - fabs(dn)) < 1e-10 && fabs(dc) < 1e-10 * L;
}

// Point pairs (x - y, weight) of the tensor collapsed-Gauss rule on two
// regular panels, passed to f(dv, W, lam) with lam the barycentric
// coordinates of the source point y (in the order of the source triangle's
// vertices; p0 kernels ignore them).
template <class Fn>
__device__ __forceinline__ void regular_points(const NearGeom& G, const QuadRules& Q, int kx, int jx, Fn&& f) {
    double P[3][3], S[3][3];
    tri_vertices(G, kx, P);
    tri_vertices(G, jx, S);
    const double aP = 2.0 * G.area[kx], aS = 2.0 * G.area[jx];
    const int q = Q.q_reg;
    for (int i1 = 0; i1 < q; ++i1)
        for (int j1 = 0; j1 < q; ++j1) {
            const double s1 = Q.g_reg[i1], t1 = Q.g_reg[i1] * Q.g_reg[j1];
            const double w1 = aP * (Q.w_reg[i1] * Q.w_reg[j1] * Q.g_reg[i1]);
            double x[3];
            for (int c = 0; c < 3; ++c) x[c] = P[0][c] + s1 * (P[1][c] - P[0][c]) + t1 * (P[2][c] - P[1][c]);
            for (int i2 = 0; i2 < q; ++i2)
                for (int j2 = 0; j2 < q; ++j2) {
                    const double s2 = Q.g_reg[i2], t2 = Q.g_reg[i2] * Q.g_reg[j2];
                    const double w2 = aS * (Q.w_reg[i2] * Q.w_reg[j2] * Q.g_reg[i2]);
                    double dv[3];
                    for (int c = 0; c < 3; ++c) dv[c] = x[c] - (S[0][c] + s2 * (S[1][c] - S[0][c]) + t2 * (S[2][c] - S[1][c]));
                    const double lam[3] = {1.0 - s2, s2 - t2, t2};
                    f(dv, w1 * w2, lam);
                }
        }
}

__constant__ double c_edge_tets[6][3][3] = {
    {{0, 1, 0}, {1, 0, 0}, {1, 0, 1}},
    {{0, 1, 0}, {1, 0, 1}, {0, 1, 1}},
    {{0, 0, 1}, {1, 0, 1}, {0, 1, 1}},
    {{0, 1, 0}, {-1, 1, 0}, {0, 1, 1}},
    {{0, 0, 1}, {-1, 0, 0}, {-1, 1, 0}},
    {{0, 0, 1}, {-1, 1, 0}, {0, 1, 1}},
};
__constant__ double c_hex[6][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 0}, {-1, -1}, {0, -1}};

// Point pairs of the singular rules for touching panels (nshared = 3:
// identical, 2: common edge, 1: common vertex), passed to f(dv, W, lam).
// lam: barycentric coordinates of y in the source triangle's vertex order.
// The common-edge rule integrates the position along the shared edge in
// closed form; lam is affine in it, so its average is its value at the
// middle of that position's range.  The identical-panel rule integrates the
// position out as an area and passes lam = (1/3, 1/3, 1/3): only its sum is
// meaningful there (the double layer, the one kernel weighted by lam,
// vanishes on a panel with itself).
template <class Fn>
__device__ __forceinline__ void singular_points(const NearGeom& G, const QuadRules& Q, int kx, int jx, int nshared,
                                                Fn&& f) {
    const int q = Q.q_sing;
    const int* ta = G.tris + 3 * kx;
    const int* tb = G.tris + 3 * jx;
    if (nshared == 3) {
        double P[3][3];
        tri_vertices(G, kx, P);
        const double a2 = 2.0 * G.area[kx];
        for (int sct = 0; sct < 6; ++sct) {
            const double va0 = c_hex[sct][0], va1 = c_hex[sct][1];
            const double vb0 = c_hex[(sct + 1) % 6][0], vb1 = c_hex[(sct + 1) % 6][1];
            for (int ir = 0; ir < q; ++ir)
                for (int iu = 0; iu < q; ++iu) {
                    const double rho = Q.g_sing[ir], u = Q.g_sing[iu];
                    const double z1 = rho * (va0 + u * (vb0 - va0));
                    const double z2 = rho * (va1 + u * (vb1 - va1));
                    double dv[3];
                    for (int c = 0; c < 3; ++c) dv[c] = -(z1 * (P[1][c] - P[0][c]) + z2 * (P[2][c] - P[1][c]));
                    const double W = a2 * a2 * 0.5 * (1.0 - rho) * (1.0 - rho) * rho * (Q.w_sing[ir] * Q.w_sing[iu]);
                    const double lam[3] = {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0};
                    f(dv, W, lam);
                }
        }
    } else if (nshared == 2) {
        int ia = 0;
        for (int v = 0; v < 3; ++v) {
            bool sh = false;
            for (int w = 0; w < 3; ++w) sh |= ta[v] == tb[w];
            if (!sh) ia = v;
        }
        int q2 = 0;
        for (int w = 0; w < 3; ++w) {
            bool sh = false;
            for (int v = 0; v < 3; ++v) sh |= tb[w] == ta[v];
            if (!sh) q2 = tb[w];
        }
        const double* E0 = G.verts + 3 * ta[(ia + 1) % 3];
        const double* E1 = G.verts + 3 * ta[(ia + 2) % 3];
        const double* P2 = G.verts + 3 * ta[ia];
        const double* Q2 = G.verts + 3 * q2;
        double e[3], c1[3], c2[3];
        for (int c = 0; c < 3; ++c) { e[c] = E1[c] - E0[c]; c1[c] = P2[c] - E1[c]; c2[c] = Q2[c] - E1[c]; }
        const double aa = 2.0 * G.area[kx] * 2.0 * G.area[jx];
        // source vertex order (E0, E1, Q2) -> position in tb
        int pe0 = 0, pe1 = 0, pq2 = 0;
        for (int w = 0; w < 3; ++w) {
            if (tb[w] == ta[(ia + 1) % 3]) pe0 = w;
            else if (tb[w] == ta[(ia + 2) % 3]) pe1 = w;
            else pq2 = w;
        }
        for (int tt = 0; tt < 6; ++tt) {
            const double (*tv)[3] = c_edge_tets[tt];
            const double det = fabs(tv[0][0] * (tv[1][1] * tv[2][2] - tv[1][2] * tv[2][1])
                                    - tv[0][1] * (tv[1][0] * tv[2][2] - tv[1][2] * tv[2][0])
                                    + tv[0][2] * (tv[1][0] * tv[2][1] - tv[1][1] * tv[2][0]));
            for (int ir = 0; ir < q; ++ir)
                for (int i1 = 0; i1 < q; ++i1)
                    for (int i2 = 0; i2 < q; ++i2) {
                        const double rho = Q.g_sing[ir], u1 = Q.g_sing[i1], u2 = Q.g_sing[i2];
                        double p[3];
                        for (int c = 0; c < 3; ++c)
                            p[c] = rho * (tv[0][c] + u1 * (tv[1][c] - tv[0][c]) + (u1 * u2) * (tv[2][c] - tv[1][c]));
                        double dv[3];
                        for (int c = 0; c < 3; ++c) dv[c] = -p[0] * e[c] + p[1] * c1[c] - p[2] * c2[c];
                        const double W = aa * det * (1.0 - rho) * rho * rho * u1 * (Q.w_sing[ir] * Q.w_sing[i1] * Q.w_sing[i2]);
                        // p = (y1 - x1, x2, y2); x1 runs over [max(x2, y2 - z), min(1, 1 - z)]
                        const double x1m = 0.5 * (fmax(p[1], p[2] - p[0]) + fmin(1.0, 1.0 - p[0]));
                        const double y1 = x1m + p[0];
                        double lam[3];
                        lam[pe0] = 1.0 - y1;
                        lam[pe1] = y1 - p[2];
                        lam[pq2] = p[2];
                        f(dv, W, lam);
                    }
        }
    } else {
        int va = 0, vb = 0;
        for (int v = 0; v < 3; ++v)
            for (int w = 0; w < 3; ++w)
                if (ta[v] == tb[w]) { va = v; vb = w; }
        const double* V0 = G.verts + 3 * ta[va];
        const double* P1 = G.verts + 3 * ta[(va + 1) % 3];
        const double* P2 = G.verts + 3 * ta[(va + 2) % 3];
        const double* Q1 = G.verts + 3 * tb[(vb + 1) % 3];
        const double* Q2 = G.verts + 3 * tb[(vb + 2) % 3];
        double a1[3], b1[3], a2[3], b2[3];
        for (int c = 0; c < 3; ++c) { a1[c] = P1[c] - V0[c]; b1[c] = P2[c] - P1[c]; a2[c] = Q1[c] - V0[c]; b2[c] = Q2[c] - Q1[c]; }
        const double aa = 2.0 * G.area[kx] * 2.0 * G.area[jx];
        for (int ix = 0; ix < q; ++ix)
            for (int ie = 0; ie < q; ++ie)
                for (int i1 = 0; i1 < q; ++i1)
                    for (int i2 = 0; i2 < q; ++i2) {
                        const double xi = Q.g_sing[ix], eta = Q.g_sing[ie];
                        const double u1 = Q.g_sing[i1], u2 = Q.g_sing[i2];
                        const double W = aa * xi * xi * xi * eta *
                                         (Q.w_sing[ix] * Q.w_sing[ie] * Q.w_sing[i1] * Q.w_sing[i2]);
                        double A1[3], A2[3], dA[3], dB[3];
                        for (int c = 0; c < 3; ++c) {
                            A1[c] = a1[c] + u1 * b1[c];
                            A2[c] = a2[c] + u2 * b2[c];
                            dA[c] = xi * (A1[c] - eta * A2[c]);
                            dB[c] = xi * (eta * A1[c] - A2[c]);
                        }
                        // y = V0 + xi eta A2 (first region), V0 + xi A2 (second):
                        // reference coordinates (s, s u2) with s = xi eta or xi
                        double lA[3], lB[3];
                        const double sA = xi * eta, sB = xi;
                        lA[vb] = 1.0 - sA; lA[(vb + 1) % 3] = sA - sA * u2; lA[(vb + 2) % 3] = sA * u2;
                        lB[vb] = 1.0 - sB; lB[(vb + 1) % 3] = sB - sB * u2; lB[(vb + 2) % 3] = sB * u2;
                        f(dA, W, lA);
                        f(dB, W, lB);
                    }
    }
}

// Regular panel pairs: tensor collapsed-Gauss rule, d = d0 .. d0 + DMAX.
// NC = 3: the double layer with p1 trial functions, one table column per
// local vertex of the source triangle (column NC u + i of gr.usize = NC U).
template <bool K, int DMAX, int NC = 1>
__global__ void k_near_regular(double* __restrict__ table, const GroupDev* __restrict__ groups,
                               const int* __restrict__ blk_group, const int64_t* __restrict__ blk_base,
                               const int* __restrict__ upos, NearGeom G, QuadRules Q, int d0) {
    const int g = blk_group[blockIdx.x];
    const GroupDev gr = groups[g];
    const int nX = gr.te - gr.tb;
    const int U = gr.usize / NC;
    const int64_t idx = blk_base[blockIdx.x] + threadIdx.x;
    if (idx >= (int64_t)nX * U || d0 > gr.dmax) return;
    const int r = (int)(idx % nX), u = (int)(idx / nX);
    const int kx = G.inv_sigma[gr.tb + r];
    const int jx = G.inv_sigma[upos[gr.uoff + u]];
    double acc[NC][DMAX + 1];
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int d = 0; d <= DMAX; ++d) acc[i][d] = 0.0;
    if (kx != jx && !(K && coplanar(G, kx, jx))) {
        const double* ny = G.normal + 3 * jx;
        regular_points(G, Q, kx, jx, [&](const double* dv, double W, const double* lam) {
            if constexpr (NC == 1) {
                accumulate_point<K, DMAX>(acc[0], dv, ny, W, d0, gr.dmax, G.h, G.alpha, Q);
            } else {
#pragma unroll
                for (int i = 0; i < NC; ++i)
                    accumulate_point<K, DMAX>(acc[i], dv, ny, W * lam[i], d0, gr.dmax, G.h, G.alpha, Q);
            }
        });
    }
    double* out = table + gr.toff;
    for (int dd = 0; dd <= DMAX && d0 + dd <= gr.dmax; ++dd)
#pragma unroll
        for (int i = 0; i < NC; ++i) out[((int64_t)(d0 + dd) * gr.usize + NC * u + i) * nX + r] = acc[i][dd];
}

struct TouchDev { int group, r, u, nshared; };

// Touching panel pairs: identical (all d), common edge / vertex (d = 0, 1).
template <bool K, int DMAX, int NC = 1>
__global__ void k_near_singular(double* __restrict__ table, const GroupDev* __restrict__ groups,
                                const TouchDev* __restrict__ touch, int n_touch, const int* __restrict__ upos,
                                NearGeom G, QuadRules Q, int d0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_touch) return;
    const TouchDev tp = touch[i];
    const GroupDev gr = groups[tp.group];
    const int nX = gr.te - gr.tb;
    const int kx = G.inv_sigma[gr.tb + tp.r];
    const int jx = G.inv_sigma[upos[gr.uoff + tp.u]];
    const int dlast = (tp.nshared == 3) ? gr.dmax : min(1, gr.dmax);
    if (d0 > dlast) return;
    double acc[NC][DMAX + 1];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int d = 0; d <= DMAX; ++d) acc[c][d] = 0.0;
    const double* ny = G.normal + 3 * jx;
    if (!(K && coplanar(G, kx, jx)))
        singular_points(G, Q, kx, jx, tp.nshared, [&](const double* dv, double W, const double* lam) {
            if constexpr (NC == 1) {
                accumulate_point<K, DMAX>(acc[0], dv, ny, W, d0, dlast, G.h, G.alpha, Q);
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    accumulate_point<K, DMAX>(acc[c], dv, ny, W * lam[c], d0, dlast, G.h, G.alpha, Q);
            }
        });
    double* out = table + gr.toff;
    for (int dd = 0; dd <= DMAX && d0 + dd <= dlast; ++dd)
#pragma unroll
        for (int c = 0; c < NC; ++c) out[((int64_t)(d0 + dd) * gr.usize + NC * tp.u + c) * nX + tp.r] = acc[c][dd];
}

struct NearLayout {
    const int* rg_leaf;      // row group -> leaf
    const int* rg_kt;
    const int64_t* rg_boff;
    const int* lf_tb;        // leaf -> first triangle position
    const int* lf_nx;
    const int* lf_rect0;
    const int* lf_rect1;
    const int* lf_group;
    const int* rc_j0;
    const int* rc_j1;
    const int* rc_set;
    const int* set_off;
    const int* set_size;
    const int* set_pos;
    int E_x;
    int64_t n_rows;
    int E_src;               // stride of a source step in the density vector
                             // (E_x; 3 E_x for the p1 double layer's local values)
};

// Expand the distinct-integral table into the causal block storage:
// B[boff + c * nX + r] = T[d = kt - jt][u(y)][r].  One wave per row group.
__global__ void __launch_bounds__(256) k_near_expand(double* __restrict__ B, const double* __restrict__ table,
                                                     const GroupDev* __restrict__ groups, const int* __restrict__ umap,
                                                     NearLayout L) {
    const int64_t rg = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (rg >= L.n_rows) return;
    const int lane = threadIdx.x % kWave;
    const int leaf = L.rg_leaf[rg], kt = L.rg_kt[rg];
    const int nX = L.lf_nx[leaf];
    const int cpi = kWave / nX;
    const int cs = lane / nX, r = lane % nX;
    if (cs >= cpi) return;
    const GroupDev gr = groups[L.lf_group[leaf]];
    const int* um = umap + gr.mapoff;
    const double* T = table + gr.toff;
    double* out = B + L.rg_boff[rg];
    int64_t colbase = 0;
    for (int q = L.lf_rect0[leaf]; q < L.lf_rect1[leaf]; ++q) {
        const int j0 = L.rc_j0[q];
        const int ns = min(L.rc_j1[q], kt + 1) - j0;
        if (ns <= 0) continue;
        const int S = L.set_size[L.rc_set[q]];
        const int* pos = L.set_pos + L.set_off[L.rc_set[q]];
        const int64_t total = (int64_t)ns * S;
        int jt = j0, i = cs;
        while (i >= S) { i -= S; ++jt; }
        for (int64_t c = cs; c < total; c += cpi) {
            const int d = kt - jt;
            out[(colbase + c) * nX + r] = T[((int64_t)d * gr.usize + um[pos[i]]) * nX + r];
            i += cpi;
            while (i >= S) { i -= S; ++jt; }
        }
        colbase += total;
    }
}

// Steps of different lengths (no Toeplitz reuse): every stored entry
// V_h[(kt, kx), (jt, jx)] integrated directly into the causal blocks, with
// the same spatial rules as the table kernels (singular rules for the
// identical panel at every lag and for panels sharing an edge or a vertex at
// lags 0 and 1) and the time factor of the step pair.  One wave per row
// group, lanes over (column slot, row) as in k_near_expand.
template <bool K, int NC = 1>
__global__ void __launch_bounds__(256) k_near_direct(double* __restrict__ B, const double* __restrict__ tn,
                                                     NearLayout L, NearGeom G, QuadRules Q) {
    const int64_t rg = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (rg >= L.n_rows) return;
    const int lane = threadIdx.x % kWave;
    const int leaf = L.rg_leaf[rg], kt = L.rg_kt[rg];
    const int nX = L.lf_nx[leaf];
    const int cpi = kWave / nX;
    const int cs = lane / nX, r = lane % nX;
    if (cs >= cpi) return;
    const int kx = G.inv_sigma[L.lf_tb[leaf] + r];
    const double tk0 = tn[kt], tk1 = tn[kt + 1];
    double* out = B + L.rg_boff[rg];
    int64_t colbase = 0;
    for (int q = L.lf_rect0[leaf]; q < L.lf_rect1[leaf]; ++q) {
        const int j0 = L.rc_j0[q];
        const int ns = min(L.rc_j1[q], kt + 1) - j0;
        if (ns <= 0) continue;
        const int S = L.set_size[L.rc_set[q]];
        const int* pos = L.set_pos + L.set_off[L.rc_set[q]];
        const int64_t total = (int64_t)ns * S;
        int jt = j0, i = cs;
        while (i >= S) { i -= S; ++jt; }
        for (int64_t c = cs; c < total; c += cpi) {
            // column (jt, source position, local vertex) for NC = 3
            const int jx = G.inv_sigma[pos[i] / NC];
            const int iv = pos[i] % NC;
            const int d = kt - jt;
            const double tj0 = tn[jt], tj1 = tn[jt + 1];
            double acc = 0.0;
            if (!(K && coplanar(G, kx, jx))) {
                const double* ny = G.normal + 3 * jx;
                auto point = [&](const double* dv, double W, const double* lam) {
                    const double rr = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
                    double fac = K ? W * (dv[0] * ny[0] + dv[1] * ny[1] + dv[2] * ny[2]) : W;
                    if constexpr (NC == 3) fac *= lam[iv];
                    acc += fac * time_factor_pair<K>(rr, tk0, tk1, tj0, tj1, d, G.alpha, Q);
                };
                int nsh = 0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) nsh += G.tris[3 * kx + a] == G.tris[3 * jx + b];
                if (nsh == 3 || (nsh > 0 && d <= 1)) singular_points(G, Q, kx, jx, nsh, point);
                else regular_points(G, Q, kx, jx, point);
            }
            out[(colbase + c) * nX + r] = acc;
            i += cpi;
            while (i >= S) { i -= S; ++jt; }
        }
        colbase += total;
    }
}

#include "near_apply.hpp"

// Diagonal entries V_h[(j, k), (j, k)] (d = 0, the triangle with itself) per
// triangle, natural order: one wave per leaf, lane = row of the leaf.
__global__ void __launch_bounds__(256) k_near_diag(const double* __restrict__ table, const GroupDev* __restrict__ groups,
                                                   const int* __restrict__ umap, NearLayout L, int n_leaves,
                                                   const int* __restrict__ inv_sigma, double* __restrict__ diag) {
    const int leaf = blockIdx.x * 4 + threadIdx.x / kWave, r = threadIdx.x % kWave;
    if (leaf >= n_leaves) return;
    const int nX = L.lf_nx[leaf];
    if (r >= nX) return;
    const GroupDev gr = groups[L.lf_group[leaf]];
    const int pos = L.lf_tb[leaf] + r;
    const int u = umap[gr.mapoff + pos];
    if (u >= 0) diag[inv_sigma[pos]] = table[gr.toff + (int64_t)u * nX + r];
}


}  // namespace

// ====================================================================== tree

namespace {

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
};

struct DevLevel {
    int l = 0, nx = 0, n_int = 0, n_leafx = 0, n_par = 0;
    int* ist = nullptr;           // first step of interval k
    int* ilen = nullptr;          // steps of interval k (0: absent)
    int maxlen = 0;               // most steps of an interval
    uint8_t* lflag = nullptr;     // [leaf slot][k]: (leaf_xs[li], k) is a leaf box
    int2* lchunk = nullptr;       // S2M / L2T blocks: (leaf slot, first row) of <= 64 rows
    int n_lchunk = 0;
    uint8_t* inner = nullptr;     // [slot][k]: (xs, k) has children
    bool uniform = true;          // batched-in-time M2L kernels apply (Level::uniform)
    int2* ccols[2] = {nullptr, nullptr};   // class-aware M2L: columns (k, class) per time offset 2, 3
    int2* cbr[2] = {nullptr, nullptr};     // first and last class of each column block
    int nccb[2] = {0, 0};                  // column blocks per time offset
    int ncp[2] = {0, 0};                   // columns (16 kClsNB nccb) per time offset
    int* cperm[2] = {nullptr, nullptr};    // source interval k - D of each column (-1: padding)
    double* mup[2] = {nullptr, nullptr};   // moments gathered into column order [slot][coef][column]
    float* mup32[2] = {nullptr, nullptr};  // the same in FP32 (BF16 values for that mode)
    double* mu = nullptr;
    double* lam = nullptr;
    int* leaf_xs = nullptr;
    int64_t* ax_off = nullptr;
    int* tb = nullptr;
    int* te = nullptr;
    int* tb3 = nullptr;           // 3 tb, 3 te and 3 ax_off: rows of the p1 double layer's S2M
    int* te3 = nullptr;
    int64_t* ax_off3 = nullptr;
    int* parent = nullptr;
    int* par_xs = nullptr;        // slots with children (non-leaf)
    int* ch_ptr = nullptr;
    int* ch = nullptr;
    int* m2l_ptr = nullptr;
    int* m2l_src = nullptr;
    int* m2l_cls = nullptr;
    // class-aware M2L (levels with unequal intervals): groups of kClsKT
    // consecutive target slots and the merged offsets of each group
    int* tg_x = nullptr;          // [group][kClsKT] target slots, -1 padded
    int* tg_ptr = nullptr;        // CSR over groups
    int* tg_cls = nullptr;        //   spatial offset class
    int* tg_src = nullptr;        //   [entry][kClsKT] source slot per target, -1 where absent
    int ntg = 0;
    double* ops = nullptr;
    double* lam_parts = nullptr;  // extra shares of a split interaction list
    int parts_cap = 1;            // shares lam_parts holds room for (1 + extra buffers)
    int64_t slot_pairs = 0;       // (target slot, source slot) pairs of the interaction lists
    int nsplit = 1;
    int nsplit_q[2] = {1, 1};     // per precision (0 FP64, 1 FP32): interaction-list shares
    int m2l_nb[2] = {0, 0};       // per precision: wide M2L interval blocks per workgroup; 0: k_m2l_mfma / k_m2l
    int ncb[2] = {1, 1};          // per precision: wide M2L column blocks of 32 m2l_nb intervals
    float* mu32 = nullptr;        // FP32 moments (mixed mode), same layout as mu
    int* off3 = nullptr;
    int64_t at_off = 0, qt_off = -1, qx_off = -1, e1_off = 0, cab_off = 0, e1s_off = 0;
    int n_off = 0, R = 0;
};

struct NearOp {
    double* B = nullptr;          // causal block storage
    double* table = nullptr;      // distinct integrals
};

}  // namespace

struct pfmm_tree {
    int device = 0;
    Plan P;
    FarTables F;
    std::vector<void*> allocs;
    uint64_t bytes = 0;
    // device data
    int* sigma = nullptr;
    int* adj = nullptr;           // E_x x 3 edge neighbours (natural order)
    int* inv_sigma = nullptr;
    double* wd = nullptr;
    double* fd = nullptr;         // farfield result, tree order
    double* fn = nullptr;         // nearfield result, tree order
    hipStream_t side = nullptr;   // the nearfield runs here, beside the farfield chain
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    double* mass = nullptr;       // |gamma_k| per triangle (natural order)
    double* hstep = nullptr;      // t_{k+1} - t_k per step
    double *At = nullptr, *Ax = nullptr, *AxK = nullptr, *qt = nullptr, *qx = nullptr;
    int* chunk_cols = nullptr;
    int64_t* chunk_off = nullptr;
    double* E1 = nullptr;
    double* Cab = nullptr;
    double* E1s = nullptr;        // matrix-core M2L: staged tables [level][Delta][offset][x (C_ab folded in) | y,z][TSp]
    int TSp = 0;                  // padded table length (multiple of 128 doubles)
    int* packinfo = nullptr;      // per coefficient: a | k1<<4 | k2<<8 | k3<<12 | deg<<16
    int* slot_tile = nullptr;     // [groups][mfma_slots] row tiles per wave group (-1 = none)
    int* tile_ks = nullptr;       // K-steps per 16-row tile
    int mfma_slots = 0;           // 0: matrix-core M2L not used
    int n_partial = 0;            // split-K partial segments
    size_t m2l_shm = 0;           // dynamic LDS of the matrix-core M2L
    // wide matrix-core M2L: [0] two interval blocks / two slots, [1] four blocks / one slot
    struct Wide { int* plan = nullptr; int G = 0, stride = 0; size_t shm = 0; bool ok = false; } wide[3][3];
    Wide wcls[3];                 // class-aware M2L (levels with unequal or missing intervals), per precision
    int prec = PFMM_FP64;         // farfield precision of the next applies
    bool has_f32 = false;         // FP32/BF16 moments and tables allocated (tree built in a mixed mode)
    // wide M2L: compact 1D tables (entries with kappa + nu <= m_x per time pair),
    // rows [level][Delta][offset][x (C_ab folded in) | y,z] of TSc64 doubles / TSc32 floats
    double* E1c = nullptr;
    float* E1c32 = nullptr;
    float* E1c16 = nullptr;       // the FP32 rows rounded to bfloat16 values
    int TSc64 = 0, TSc32 = 0;
    CoefMaps cm{};
    SepMaps sm{};
    int ki_m2m = 0, ki_l2l = 0;   // intervals per block of k_m2m_sep / k_l2l_sep
    int ki_s2m = 0, ki_l2t = 0;   // intervals per block of k_s2m_blk / k_l2t_blk
    int stage_s2m = 0, stage_l2t = 0;   // A_x staged in LDS
    std::vector<DevLevel> lv;
    bool low_leaves = false;      // leaves at levels < 2 (no far field)
    NearLayout nl{};
    GroupDev* groups = nullptr;
    int* umap = nullptr;
    NearOp opV, opK;
    bool hasV = false, hasK = false;
    // the double layer with p1 trial functions: expanded nearfield layout
    // (three columns per source triangle), its groups and position map, the
    // local values per (step, triangle position, vertex) in tree order, and
    // the S2M table with three rows per triangle
    NearLayout nl3{};
    GroupDev* groups3 = nullptr;
    int* umap3 = nullptr;
    NearOp opK1;
    bool hasK1 = false;
    double* wd3 = nullptr;
    double* AxK1 = nullptr;
    int n_verts = 0;
    NearGeom geom{};              // mesh on the device (natural order)
    double* tnodes_dev = nullptr; // time nodes on the device
    bool geom_ok = false;
    int nf_mode = PFMM_NF_STORED;
    int64_t* ru_off = nullptr;    // Toeplitz nearfield: per leaf rectangle, offset into ru
    int* ru = nullptr;            // table columns u of the rectangles' source triangles
    NearGemmGroup* ngg = nullptr; // Toeplitz groups applied as GEMMs, sorted by row tiles
    int* nue = nullptr;           // their per-column records: U positions, then per x U packed (a_u, b_u)
    int* nlst = nullptr;          // leaf starts (and E_t) of the groups whose leaves differ in length
    int ngg_start[5] = {0, 0, 0, 0, 0};   // groups with 1..4 row tiles: [ngg_start[t-1], ngg_start[t])
    int ngg_lds[4] = {0, 0, 0, 0};        // per row-tile class: most dynamic LDS bytes of a group
    int* nsel = nullptr;          // row groups of the other groups (matrix-vector kernel)
    int64_t n_sel = 0;
    int nf_gemm = 1;              // pfmm_params.nearfield_gemm
    // profiling
    bool prof = false;
    std::vector<hipEvent_t> ev;   // pairs per stage
    std::vector<std::pair<int, int>> ev_used;   // (stage, event index)
    double prof_ms[8] = {0};
    int64_t prof_cnt[8] = {0};
};

namespace {

template <class T>
pfmm_status upload(pfmm_tree* t, T** dst, const T* src, size_t n) {
    *dst = nullptr;
    if (n == 0) return PFMM_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) return fail(PFMM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    t->allocs.push_back(p);
    t->bytes += n * sizeof(T);
    HIP_TRY(hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice));
    *dst = (T*)p;
    return PFMM_OK;
}

template <class T>
pfmm_status dalloc(pfmm_tree* t, T** dst, size_t n) {
    *dst = nullptr;
    if (n == 0) return PFMM_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) return fail(PFMM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    t->allocs.push_back(p);
    t->bytes += n * sizeof(T);
    *dst = (T*)p;
    return PFMM_OK;
}

#define PF_TRY(expr)                                  \
    do {                                              \
        pfmm_status s_ = (expr);                      \
        if (s_ != PFMM_OK) return s_;                 \
    } while (0)

int dmax_class(int dmax) {
    if (dmax <= 7) return 7;
    if (dmax <= 15) return 15;
    return 31;
}

// Device memory the build will need (bytes), computed before allocating.
uint64_t estimate_bytes(const Plan& P, const FarTables& F, int ops_mask, int precision, int nf_mode) {
    uint64_t b = 0;
    const uint64_t N = (uint64_t)P.E_t * P.E_x;
    // explicit M2L operators exist only on the vector-unit fallback (degrees
    // above 15, or 1D tables too large for the matrix-core kernel's LDS)
    const int TS = (P.m_t + 1) * (P.m_t + 1) * (P.m_x + 1) * (P.m_x + 1);
    const size_t shm = (size_t)6 * ((TS + 127) / 128 * 128) * 8 + (size_t)(((P.Nc + 3) & ~3) + 16) * 16;
    const bool explicit_ops = P.m_t > 15 || P.m_x > 15 || shm > 163840;
    b += 3 * N * 8;                                   // w, far and near results in tree order
    for (int l = 2; l <= P.depth; ++l) {
        const FarLevel& L = F.lv[l];
        b += 2ull * L.nx * P.Nc * L.n_int * 8;        // mu, lambda
        if (precision != PFMM_FP64) b += (uint64_t)L.nx * P.Nc * L.n_int * 4;   // FP32 moments
        if (explicit_ops) b += (uint64_t)L.n_off * 2 * F.op_size * 8;
    }
    int nop = ((ops_mask & PFMM_OP_V) ? 1 : 0) + ((ops_mask & PFMM_OP_K) ? 1 : 0);
    b += (uint64_t)nop * ((nf_mode == PFMM_NF_STORED ? (uint64_t)P.near_entries * 8 : 0) + (uint64_t)P.table_size * 8);
    if (ops_mask & PFMM_OP_K1)   // three columns per source triangle; local values; the S2M rows
        b += (uint64_t)(P.p1.near_entries + P.p1.table_size + 3 * N) * 8 + P.p1.umap.size() * 4 +
             P.p1.set_pos.size() * 4 + F.AxK1.size() * 8;
    if (nf_mode == PFMM_NF_TOEPLITZ) b += P.rects.size() * 8 + P.set_pos.size() * 4;
    b += P.umap.size() * 4 + P.set_pos.size() * 4 + P.upos.size() * 4;
    b += (F.At.size() + F.Ax.size() + F.AxK.size() + F.qt.size() + F.qx.size() + 4 * F.E1.size()) * 8;
    b += P.rows.size() * 16;
    return b;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// Mesh geometry and time nodes on the device (uploaded once per tree).
pfmm_status upload_geometry(pfmm_tree* t) {
    if (t->geom_ok) return PFMM_OK;
    const Plan& P = t->P;
    NearGeom& G = t->geom;
    double *verts, *area, *normal, *centroid, *maxedge;
    int* tris;
    PF_TRY(upload(t, &verts, P.verts.data(), P.verts.size()));
    PF_TRY(upload(t, &tris, P.tris.data(), P.tris.size()));
    PF_TRY(upload(t, &area, P.area.data(), P.area.size()));
    PF_TRY(upload(t, &normal, P.normal.data(), P.normal.size()));
    PF_TRY(upload(t, &centroid, P.centroid.data(), P.centroid.size()));
    PF_TRY(upload(t, &maxedge, P.maxedge.data(), P.maxedge.size()));
    PF_TRY(upload(t, &t->tnodes_dev, P.tnodes.data(), P.tnodes.size()));
    G.verts = verts; G.tris = tris; G.area = area; G.normal = normal; G.centroid = centroid; G.maxedge = maxedge;
    G.inv_sigma = t->inv_sigma;
    G.h = P.h; G.alpha = P.alpha;
    t->geom_ok = true;
    return PFMM_OK;
}

// Nearfield entries of one operator: kind 0 V_h, 1 K_h (p0 trial
// functions), 2 K_h with p1 trial functions (three table columns and block
// columns per source triangle: its local vertices).
pfmm_status assemble_near(pfmm_tree* t, int kind, NearOp& op, hipStream_t st) {
    Plan& P = t->P;
    const bool K = kind >= 1, p1 = kind == 2;
    const bool stored = t->nf_mode == PFMM_NF_STORED;
    PF_TRY(dalloc(t, &op.table, (size_t)(p1 ? P.p1.table_size : P.table_size)));
    if (stored) PF_TRY(dalloc(t, &op.B, (size_t)(p1 ? P.p1.near_entries : P.near_entries)));
    const GroupDev* groups = p1 ? t->groups3 : t->groups;
    const int* umap = p1 ? t->umap3 : t->umap;
    const NearLayout& NL = p1 ? t->nl3 : t->nl;
    // quadrature rules
    QuadRules Q{};
    std::vector<double> g, w;
    gauss_legendre01(P.q_reg, g, w);
    for (int i = 0; i < P.q_reg; ++i) { Q.g_reg[i] = g[i]; Q.w_reg[i] = w[i]; }
    gauss_legendre01(P.q_sing, g, w);
    for (int i = 0; i < P.q_sing; ++i) { Q.g_sing[i] = g[i]; Q.w_sing[i] = w[i]; }
    gauss_legendre01(kHat, g, w);
    for (int i = 0; i < kHat; ++i) { Q.g_hat[i] = g[i]; Q.w_hat[i] = w[i]; }
    Q.q_reg = P.q_reg;
    Q.q_sing = P.q_sing;
    // geometry
    static_assert(sizeof(TouchDev) == sizeof(TouchPair), "layout");
    PF_TRY(upload_geometry(t));
    const NearGeom G = t->geom;
    if (!P.uniform_steps) {
        // steps of different lengths: stored blocks only (the planner refuses
        // the Toeplitz mode), each entry integrated on its own
        const int64_t nrg = (int64_t)P.rows.size();
        const dim3 grid((unsigned)((nrg + 3) / 4));
        if (nrg > 0) {
            if (p1) hipLaunchKernelGGL((k_near_direct<true, 3>), grid, dim3(256), 0, st, op.B, t->tnodes_dev, NL, G, Q);
            else if (K) hipLaunchKernelGGL(k_near_direct<true>, grid, dim3(256), 0, st, op.B, t->tnodes_dev, NL, G, Q);
            else hipLaunchKernelGGL(k_near_direct<false>, grid, dim3(256), 0, st, op.B, t->tnodes_dev, NL, G, Q);
            HIP_TRY(hipGetLastError());
        }
        return PFMM_OK;
    }
    int* upos;
    PF_TRY(upload(t, &upos, P.upos.data(), P.upos.size()));
    // regular blocks
    std::vector<int> bg;
    std::vector<int64_t> bb;
    int dmx = 0;
    for (size_t i = 0; i < P.groups.size(); ++i) {
        const AsmGroup& A = P.groups[i];
        dmx = std::max(dmx, A.dmax);
        int64_t n = (int64_t)(A.te - A.tb) * A.usize;
        for (int64_t s = 0; s < n; s += 256) { bg.push_back((int)i); bb.push_back(s); }
    }
    int* d_bg;
    int64_t* d_bb;
    PF_TRY(upload(t, &d_bg, bg.data(), bg.size()));
    PF_TRY(upload(t, &d_bb, bb.data(), bb.size()));
    // time offsets 0..dmax in passes of at most 32 (d0 = 0, 32, ...); the
    // three-column kernels in passes of 8
    const int dc = p1 ? 7 : dmax_class(dmx);
#define LAUNCH_REG(KK, DD, NC) hipLaunchKernelGGL((k_near_regular<KK, DD, NC>), dim3((unsigned)bg.size()), dim3(256), \
                                                  0, st, op.table, groups, d_bg, d_bb, upos, G, Q, d0)
    for (int d0 = 0; d0 <= dmx && !bg.empty(); d0 += dc + 1) {
        if (p1) {
            LAUNCH_REG(true, 7, 3);
        } else if (K) {
            if (dc == 7) LAUNCH_REG(true, 7, 1); else if (dc == 15) LAUNCH_REG(true, 15, 1); else LAUNCH_REG(true, 31, 1);
        } else {
            if (dc == 7) LAUNCH_REG(false, 7, 1); else if (dc == 15) LAUNCH_REG(false, 15, 1); else LAUNCH_REG(false, 31, 1);
        }
        HIP_TRY(hipGetLastError());
    }
#undef LAUNCH_REG
    TouchDev* d_touch;
    PF_TRY(upload(t, (TouchPair**)&d_touch, P.touch.data(), P.touch.size()));
    const int nT = (int)P.touch.size();
#define LAUNCH_SING(KK, DD, NC) hipLaunchKernelGGL((k_near_singular<KK, DD, NC>), dim3((nT + 63) / 64), dim3(64), 0, \
                                                   st, op.table, groups, d_touch, nT, upos, G, Q, d0)
    for (int d0 = 0; d0 <= dmx && nT > 0; d0 += dc + 1) {
        if (p1) {
            LAUNCH_SING(true, 7, 3);
        } else if (K) {
            if (dc == 7) LAUNCH_SING(true, 7, 1); else if (dc == 15) LAUNCH_SING(true, 15, 1); else LAUNCH_SING(true, 31, 1);
        } else {
            if (dc == 7) LAUNCH_SING(false, 7, 1); else if (dc == 15) LAUNCH_SING(false, 15, 1); else LAUNCH_SING(false, 31, 1);
        }
        HIP_TRY(hipGetLastError());
    }
#undef LAUNCH_SING
    // expand into the causal blocks
    const int64_t nrg = (int64_t)P.rows.size();
    if (stored && nrg > 0) {
        hipLaunchKernelGGL(k_near_expand, dim3((unsigned)((nrg + 3) / 4)), dim3(256), 0, st, op.B, op.table, groups,
                           umap, NL);
        HIP_TRY(hipGetLastError());
    }
    return PFMM_OK;
}

// Split-K plan of one row group of the wide matrix-core M2L.  For an even
// block length T every tile's K-range is cut at multiples of T; segments with
// the same start share their moment operands and are grouped (by descending
// end) up to maxs per wave; waves go to the 4 SIMDs of the CU (wave w runs on
// SIMD w % 4) by longest-processing-time on their slot-steps.  T minimises
// the busiest SIMD's slot-steps plus the longest wave (its dependent chain).
struct WideSeg { int tile, start, end; };

bool plan_row_group(const std::vector<int>& tiles, const std::vector<int>& ks, int maxs, int waves_max,
                    std::vector<std::vector<WideSeg>>& best, int& best_cost) {
    best_cost = INT32_MAX;
    best.clear();
    int maxks = 0;
    for (int tt : tiles) maxks = std::max(maxks, ks[tt]);
    for (int T = 2; T <= maxks + 1; T += 2) {
        const int nblk = (maxks + T - 1) / T;
        std::vector<std::vector<WideSeg>> waves;
        for (int b = 0; b < nblk; ++b) {
            std::vector<WideSeg> sg;
            for (int tt : tiles)
                if (ks[tt] > b * T) sg.push_back({tt, b * T, std::min((b + 1) * T, ks[tt])});
            std::stable_sort(sg.begin(), sg.end(), [](const WideSeg& x, const WideSeg& y) { return x.end > y.end; });
            for (size_t i = 0; i < sg.size(); i += maxs)
                waves.emplace_back(sg.begin() + i, sg.begin() + std::min(sg.size(), i + (size_t)maxs));
        }
        if ((int)waves.size() > waves_max) continue;
        // every end but a wave's largest must lie an even number of K-steps
        // after its start: only a tile's last segment can be odd, and one more
        // K-step there only meets columns beyond the tile's degree limit
        for (auto& wv : waves)
            for (size_t i = 1; i < wv.size(); ++i)
                if (wv[i].end < wv[0].end && ((wv[i].end - wv[i].start) & 1)) wv[i].end += 1;
        auto load = [&](int i) { int l = 0; for (auto& s : waves[i]) l += s.end - s.start; return l; };
        std::vector<int> order(waves.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return load(x) > load(y); });
        int simd_load[4] = {0, 0, 0, 0}, simd_n[4] = {0, 0, 0, 0};
        std::vector<std::vector<WideSeg>> placed(waves_max);
        int longest = 0;
        for (int i : order) {
            int pick = -1;
            for (int q = 0; q < 4; ++q)
                if (simd_n[q] < waves_max / 4 && (pick < 0 || simd_load[q] < simd_load[pick])) pick = q;
            placed[simd_n[pick] * 4 + pick] = waves[i];
            simd_n[pick] += 1;
            simd_load[pick] += load(i);
            longest = std::max(longest, waves[i][0].end - waves[i][0].start);
        }
        const int cost = *std::max_element(simd_load, simd_load + 4) + longest;
        if (cost < best_cost) { best_cost = cost; best = placed; }
    }
    return !best.empty();
}

// Row groups of the wide M2L with `waves` waves of maxs slots.  Tiles are
// dealt to G groups either by longest-processing-time on their K-lengths or
// as contiguous runs of the length-sorted tiles (so that few groups contain
// the long low-degree tiles); every group gets a split-K plan.  The choice
// minimises, summed over groups, max(plan cost, half the group's longest
// K-range) plus a fixed per-workgroup overhead: a workgroup streams the
// source moments of its longest K-range once per source, which bounds it
// from below when the moment stream, not the matrix cores, is the limit.
// Fills the per-group tables of k_m2l_wide.
bool plan_wide(const std::vector<int>& ks, int maxs, int waves, std::vector<int>& tab, int& G_out, int& stride,
               int& max_partial) {
    const int ntile = (int)ks.size();
    stride = 2 * waves + 4 * waves * maxs + 1;
    double best_total = 1e300;
    std::vector<std::vector<std::vector<WideSeg>>> best_groups;
    const int gmin = std::max(1, (ntile + waves * maxs - 1) / (waves * maxs));
    std::vector<int> order(ntile);
    for (int i = 0; i < ntile; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ks[a] > ks[b]; });
    int ktot = 0;
    for (int k : ks) ktot += k;
    for (int mode = 0; mode < 2; ++mode)
        for (int G = gmin; G <= 12; ++G) {
            std::vector<std::vector<int>> gt(G);
            std::vector<int> tot(G, 0);
            int q = 0;
            for (int tt : order) {
                if (mode == 0) q = (int)(std::min_element(tot.begin(), tot.end()) - tot.begin());
                else if (tot[q] * G >= ktot && q < G - 1) ++q;
                gt[q].push_back(tt);
                tot[q] += ks[tt];
            }
            double total = 0;
            bool ok = true;
            std::vector<std::vector<std::vector<WideSeg>>> groups(G);
            for (int g = 0; g < G && ok; ++g) {
                int c = 0;
                if (gt[g].empty() || !plan_row_group(gt[g], ks, maxs, waves, groups[g], c)) { ok = false; break; }
                int mk = 0;
                for (int tt : gt[g]) mk = std::max(mk, ks[tt]);
                total += std::max((double)c, 0.5 * mk) + 8;
            }
            if (ok && total < best_total) { best_total = total; best_groups = groups; }
        }
    if (best_groups.empty()) return false;
    const int G = (int)best_groups.size();
    tab.assign((size_t)G * stride, -1);
    max_partial = 0;
    for (int q = 0; q < G; ++q) {
        int* gp = &tab[(size_t)q * stride];
        std::vector<int> red;
        for (int wv = 0; wv < waves; ++wv) {
            const auto& g = best_groups[q][wv];
            const int start = g.empty() ? 0 : g[0].start;
            gp[2 * wv] = start;
            gp[2 * wv + 1] = (int)g.size();
            for (int i = 0; i < maxs; ++i) {
                int* e = gp + 2 * waves + (wv * maxs + i) * 3;
                if (i < (int)g.size()) {
                    e[0] = g[i].tile;
                    e[1] = g[i].end;
                    e[2] = -1;
                    if (g[i].start > 0) { e[2] = (int)red.size(); red.push_back(g[i].tile); }
                } else {
                    e[0] = -1; e[1] = start; e[2] = -1;   // empty slot: ends where the wave starts
                }
            }
        }
        gp[2 * waves + 3 * waves * maxs] = (int)red.size();
        for (size_t i = 0; i < red.size(); ++i) gp[2 * waves + 3 * waves * maxs + 1 + i] = red[i];
        max_partial = std::max(max_partial, (int)red.size());
    }
    G_out = G;
    return true;
}

// Toeplitz nearfield groups that can run as GEMMs (k_near_gemm): the group's
// leaves cover all steps in order (one leaf per time interval of the group's
// level, of equal or unequal lengths), and for every table column u the
// source steps of a leaf (clipped at the leaf's last step: later ones are
// causal zeros) form one range [s0 + a_u, s0 + b_u) clipped at step 0.  With
// leaves of one length s the ranges usually repeat with the leaf index
// modulo a period of 1, 2, 4 or 8 (neighbouring leaves of a coarser level
// span 2, 4, ... intervals) and one record set per phase is kept; otherwise
// every leaf has its own (and, for unequal lengths, the leaf starts are
// kept).  All other groups keep the matrix-vector kernel over their row
// groups.
pfmm_status plan_near_gemm(pfmm_tree* t) {
    const Plan& P = t->P;
    const int ng = (int)P.groups.size();
    std::vector<std::vector<int>> gl(ng);
    for (int i = 0; i < (int)P.leaves.size(); ++i) gl[P.leaves[i].group].push_back(i);
    std::vector<uint8_t> elig(ng, 0);
    std::vector<NearGemmGroup> gg[4];
    std::vector<std::vector<int>> ue(4);
    std::vector<int> lstart;                 // leaf starts of the groups with unequal leaves
    int lds_max[4] = {0, 0, 0, 0};
    std::vector<int> lo, hi, cov;
    for (int g = 0; g < ng && t->nf_gemm; ++g) {
        const AsmGroup& A = P.groups[g];
        std::vector<int>& L = gl[g];
        if (L.empty()) continue;
        std::sort(L.begin(), L.end(), [&](int x, int y) { return P.leaves[x].s0 < P.leaves[y].s0; });
        const int nl = (int)L.size();
        const int s = P.leaves[L[0]].s1 - P.leaves[L[0]].s0;
        const int nX = A.te - A.tb, U = A.usize;
        // limits of k_near_gemm: 32-bit buffer offsets into the table and into
        // the density rows one workgroup reads, 16-bit packed step ranges
        bool ok = s > 0 && A.dmax < 32768 && nX >= 1 && nX <= 64 && U >= 1 &&
                  (int64_t)(A.dmax + 1) * U * nX * 8 < INT32_MAX && (int64_t)(A.dmax + 32) * P.E_x * 8 < INT32_MAX;
        bool equal = true;
        int prev = 0;
        for (int i = 0; ok && i < nl; ++i) {
            const LeafRec& R = P.leaves[L[i]];
            ok = R.s0 == prev && R.s1 > R.s0 && R.s1 - R.s0 < 32768 && R.tb == A.tb && R.te == A.te;
            equal = equal && R.s1 - R.s0 == s;
            prev = R.s1;
        }
        ok = ok && prev == P.E_t;
        for (int u = 0; ok && u < U; ++u) {
            const int pos = P.upos[A.uoff + u];
            ok = pos >= 0 && pos < P.E_x && P.umap[A.mapoff + pos] == u;
        }
        if (!ok) continue;
        // source-step range of every column for leaf li: false if not one range
        auto ranges = [&](int li) -> bool {
            const LeafRec& R = P.leaves[li];
            lo.assign(U, INT32_MAX);
            hi.assign(U, INT32_MIN);
            cov.assign(U, 0);
            for (int q = R.rect0; q < R.rect1; ++q) {
                const Rect& rc = P.rects[q];
                for (int i = 0; i < P.set_size[rc.set]; ++i) {
                    const int u = P.umap[A.mapoff + P.set_pos[P.set_off[rc.set] + i]];
                    if (u < 0 || u >= U) return false;
                    lo[u] = std::min(lo[u], rc.j0);
                    hi[u] = std::max(hi[u], rc.j1);
                    cov[u] += rc.j1 - rc.j0;
                }
            }
            for (int u = 0; u < U; ++u)
                if (cov[u] && cov[u] != hi[u] - lo[u]) return false;
            return true;
        };
        int per_ok = 0;
        std::vector<int> ar, br;
        for (int per = 1; equal && per <= 8 && !per_ok; per *= 2) {
            if (nl % per) break;
            ar.assign((size_t)per * U, 0);
            br.assign((size_t)per * U, 0);
            bool bad = false;
            for (int ph = 0; ph < per && !bad; ++ph) {   // reference: the last leaf of each phase
                const int li = L[nl - per + ph];
                if (!ranges(li)) { bad = true; break; }
                const int s0 = P.leaves[li].s0, s1 = P.leaves[li].s1;
                for (int u = 0; u < U; ++u) {
                    const int h = cov[u] ? std::min(hi[u], s1) : 0;
                    if (!cov[u] || lo[u] >= h) continue;
                    ar[(size_t)ph * U + u] = lo[u] - s0;
                    br[(size_t)ph * U + u] = h - s0;
                    if ((s - 1) - (lo[u] - s0) > A.dmax) bad = true;   // time offsets inside the table
                }
            }
            for (int i = 0; !bad && i < nl; ++i) {
                if (!ranges(L[i])) { bad = true; break; }
                const int ph = i % per, s0 = P.leaves[L[i]].s0, s1 = P.leaves[L[i]].s1;
                for (int u = 0; u < U && !bad; ++u) {
                    const int a = ar[(size_t)ph * U + u], b = br[(size_t)ph * U + u];
                    const int elo = std::max(0, s0 + a), ehi = s0 + b;
                    const bool want = a < b && elo < ehi;
                    const int h = cov[u] ? std::min(hi[u], s1) : 0;
                    const bool have = cov[u] && lo[u] < h;
                    bad = want ? !(have && lo[u] == elo && h == ehi) : have;
                }
            }
            if (!bad) per_ok = per;
        }
        if (!per_ok) {   // one record set per leaf
            ar.assign((size_t)nl * U, 0);
            br.assign((size_t)nl * U, 0);
            bool bad = false;
            for (int i = 0; !bad && i < nl; ++i) {
                if (!ranges(L[i])) { bad = true; break; }
                const int s0 = P.leaves[L[i]].s0, s1 = P.leaves[L[i]].s1;
                for (int u = 0; u < U; ++u) {
                    const int h = cov[u] ? std::min(hi[u], s1) : 0;
                    if (!cov[u] || lo[u] >= h) continue;
                    ar[(size_t)i * U + u] = lo[u] - s0;
                    br[(size_t)i * U + u] = h - s0;
                    if ((s1 - 1) - lo[u] > A.dmax) bad = true;   // time offsets inside the table
                }
            }
            if (!bad) per_ok = nl;
        }
        if (!per_ok) continue;
        // the most leaves one block of 16 target steps meets: a workgroup
        // stages their records, or one set per phase when the period is shorter
        int nlb = 0;
        for (int b0 = 0, li = 0; b0 < P.E_t; b0 += 16) {
            while (P.leaves[L[li]].s1 <= b0) ++li;
            int lj = li;
            const int last = std::min(b0 + 16, P.E_t) - 1;
            while (P.leaves[L[lj]].s1 <= last) ++lj;
            nlb = std::max(nlb, lj - li + 1);
        }
        const int lds = gemm_lds_bytes(U, std::min(nlb, per_ok));
        if (lds > 40960) continue;   // with 24 KB static: within 64 KB
        elig[g] = 1;
        const int nt = (nX + 15) / 16 - 1;
        int64_t stoff = -1;
        if (!equal) {
            stoff = (int64_t)lstart.size();
            for (int i = 0; i < nl; ++i) lstart.push_back(P.leaves[L[i]].s0);
            lstart.push_back(P.E_t);
        }
        gg[nt].push_back(NearGemmGroup{A.toff, (int64_t)ue[nt].size(), stoff, s, per_ok, nX, U, (A.dmax + 1) * U,
                                       A.tb});
        lds_max[nt] = std::max(lds_max[nt], lds);
        for (int u = 0; u < U; ++u) ue[nt].push_back(P.upos[A.uoff + u]);
        for (int ph = 0; ph < per_ok; ++ph)
            for (int u = 0; u < U; ++u)
                ue[nt].push_back(gemm_pack_range(ar[(size_t)ph * U + u], br[(size_t)ph * U + u]));
    }
    std::vector<NearGemmGroup> all;
    std::vector<int> uall;
    for (int nt = 0; nt < 4; ++nt) {
        t->ngg_start[nt] = (int)all.size();
        t->ngg_lds[nt] = lds_max[nt];
        for (NearGemmGroup G : gg[nt]) {
            G.eoff += (int64_t)uall.size();
            all.push_back(G);
        }
        uall.insert(uall.end(), ue[nt].begin(), ue[nt].end());
    }
    t->ngg_start[4] = (int)all.size();
    std::vector<int> sel;
    for (size_t rg = 0; rg < P.rows.size(); ++rg)
        if (!elig[P.leaves[P.rows[rg].leaf].group]) sel.push_back((int)rg);
    t->n_sel = (int64_t)sel.size();
    if (!all.empty()) {
        PF_TRY(upload(t, &t->ngg, all.data(), all.size()));
        PF_TRY(upload(t, &t->nue, uall.data(), uall.size()));
    }
    if (!lstart.empty()) PF_TRY(upload(t, &t->nlst, lstart.data(), lstart.size()));
    if (!sel.empty()) PF_TRY(upload(t, &t->nsel, sel.data(), sel.size()));
    return PFMM_OK;
}

pfmm_status setup_device(pfmm_tree* t, hipStream_t st, int ops_mask) {
    Plan& P = t->P;
    FarTables& F = t->F;
    const int64_t N = (int64_t)P.E_t * P.E_x;
    PF_TRY(upload(t, &t->sigma, P.sigma.data(), P.sigma.size()));
    PF_TRY(upload(t, &t->inv_sigma, P.inv_sigma.data(), P.inv_sigma.size()));
    PF_TRY(upload(t, &t->adj, P.adj.data(), P.adj.size()));
    PF_TRY(dalloc(t, &t->wd, (size_t)N));
    PF_TRY(dalloc(t, &t->fd, (size_t)N));
    PF_TRY(dalloc(t, &t->fn, (size_t)N));
    HIP_TRY(hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&t->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&t->ev_join, hipEventDisableTiming));
    {
        // p0 mass diagonal |gamma_kx| (t_{kt+1} - t_kt): areas and step lengths
        // (h itself on a uniform grid)
        std::vector<double> hs(P.E_t);
        for (int k = 0; k < P.E_t; ++k) hs[k] = P.uniform_steps ? P.h : P.tnodes[k + 1] - P.tnodes[k];
        PF_TRY(upload(t, &t->mass, P.area.data(), P.area.size()));
        PF_TRY(upload(t, &t->hstep, hs.data(), hs.size()));
    }
    // coefficient maps
    {
        const int nx1 = P.m_x + 1;
        std::vector<int> kpos(P.Nc), kposmap(nx1 * nx1 * nx1, -1), cidx((P.m_t + 1) * P.Nk, -1);
        for (int i = 0; i < P.Nk; ++i) kposmap[(P.kidx_k[3 * i] * nx1 + P.kidx_k[3 * i + 1]) * nx1 + P.kidx_k[3 * i + 2]] = i;
        for (int c = 0; c < P.Nc; ++c) {
            kpos[c] = kposmap[(P.coef_k[3 * c] * nx1 + P.coef_k[3 * c + 1]) * nx1 + P.coef_k[3 * c + 2]];
            cidx[P.coef_a[c] * P.Nk + kpos[c]] = c;
        }
        int *a, *deg, *k3, *kp, *ki, *kpm, *ci;
        PF_TRY(upload(t, &a, P.coef_a.data(), P.coef_a.size()));
        PF_TRY(upload(t, &deg, P.coef_deg.data(), P.coef_deg.size()));
        PF_TRY(upload(t, &k3, P.coef_k.data(), P.coef_k.size()));
        PF_TRY(upload(t, &kp, kpos.data(), kpos.size()));
        PF_TRY(upload(t, &ki, P.kidx_k.data(), P.kidx_k.size()));
        PF_TRY(upload(t, &kpm, kposmap.data(), kposmap.size()));
        PF_TRY(upload(t, &ci, cidx.data(), cidx.size()));
        t->cm = CoefMaps{a, deg, k3, kp, ki, kpm, ci, P.Nc, P.Nk, P.m_t, P.m_x};
        // separable re-expansions: position of multi-index p with component j set to t
        std::vector<int> ax((size_t)3 * P.Nk * nx1, -1);
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < P.Nk; ++i) {
                int k[3] = {P.kidx_k[3 * i], P.kidx_k[3 * i + 1], P.kidx_k[3 * i + 2]};
                for (int tt = 0; tt < nx1; ++tt) {
                    k[j] = tt;
                    if (k[0] + k[1] + k[2] <= P.m_x)
                        ax[((size_t)j * P.Nk + i) * nx1 + tt] = kposmap[(k[0] * nx1 + k[1]) * nx1 + k[2]];
                }
            }
        int* axd;
        PF_TRY(upload(t, &axd, ax.data(), ax.size()));
        t->sm = SepMaps{a, kp, ci, ki, axd, P.Nc, P.Nk, P.m_t, P.m_x};
        // intervals per block of k_m2m_sep / k_l2l_sep: the larger of 2, 1 whose LDS fits 64 KB
        // (4 intervals per block measured slower: fewer, larger blocks, 2 resident per CU at m = 6)
        const size_t tabs = (size_t)(3 * nx1 * nx1) * sizeof(double);
        const int nt1 = P.m_t + 1;
        t->ki_m2m = t->ki_l2l = 0;
        for (int KI = 2; KI >= 1 && !t->ki_m2m; KI /= 2)
            if ((3 * (size_t)P.Nc * KI + 2 * KI * nt1 * nt1) * sizeof(double) + tabs <= 65536) t->ki_m2m = KI;
        for (int KI = 2; KI >= 1 && !t->ki_l2l; KI /= 2)
            if ((2 * (size_t)P.Nc * KI + 2 * KI * nt1 * nt1) * sizeof(double) + tabs <= 65536) t->ki_l2l = KI;
        if (!t->ki_m2m || !t->ki_l2l) return fail(PFMM_EUNSUPPORTED, "expansion degrees too large for the re-expansion kernels");
        // S2M / L2T leaf blocks (leaves hold at most 64 triangles): stage A_x in
        // LDS when it fits, with the largest of 4, 2, 1 intervals per block
        for (int stage = 1; stage >= 0 && !t->ki_s2m; --stage)
            for (int KI = 4; KI >= 1 && !t->ki_s2m; KI /= 2)
                if (((size_t)nt1 * 64 * KI + (stage ? 64 * (size_t)P.Nk : 0)) * sizeof(double) <= 65536) {
                    t->ki_s2m = KI;
                    t->stage_s2m = stage;
                }
        for (int stage = 1; stage >= 0 && !t->ki_l2t; --stage)
            for (int KI = 4; KI >= 1 && !t->ki_l2t; KI /= 2)
                if (((size_t)P.Nc * KI + (size_t)nt1 * 64 * KI + (stage ? 64 * (size_t)P.Nk : 0)) * sizeof(double) <=
                    65536) {
                    t->ki_l2t = KI;
                    t->stage_l2t = stage;
                }
        if (!t->ki_s2m || !t->ki_l2t) return fail(PFMM_EUNSUPPORTED, "expansion degrees too large for the S2M/L2T kernels");
    }
    PF_TRY(upload(t, &t->At, F.At.data(), F.At.size()));
    PF_TRY(upload(t, &t->Ax, F.Ax.data(), F.Ax.size()));
    PF_TRY(upload(t, &t->AxK, F.AxK.data(), F.AxK.size()));
    if (ops_mask & PFMM_OP_K1) PF_TRY(upload(t, &t->AxK1, F.AxK1.data(), F.AxK1.size()));
    PF_TRY(upload(t, &t->qt, F.qt.data(), F.qt.size()));
    PF_TRY(upload(t, &t->qx, F.qx.data(), F.qx.size()));
    PF_TRY(upload(t, &t->chunk_cols, F.chunk_cols.data(), F.chunk_cols.size()));
    PF_TRY(upload(t, &t->chunk_off, F.chunk_off.data(), F.chunk_off.size()));
    PF_TRY(upload(t, &t->E1, F.E1.data(), F.E1.size()));
    PF_TRY(upload(t, &t->Cab, F.Cab.data(), F.Cab.size()));
    double* E1 = t->E1;
    double* Cab = t->Cab;
    // matrix-core M2L: 16-row tiles, their K-step counts, split-K segments over waves
    {
        const int Nc = P.Nc, ntile = (Nc + 15) / 16;
        std::vector<int> pk(Nc), ks(ntile);
        for (int c = 0; c < Nc; ++c)
            pk[c] = P.coef_a[c] | (P.coef_k[3 * c] << 4) | (P.coef_k[3 * c + 1] << 8) | (P.coef_k[3 * c + 2] << 12) |
                    (P.coef_deg[c] << 16);
        int64_t total = 0;
        for (int tt = 0; tt < ntile; ++tt) {
            const int dmin = P.coef_deg[16 * tt];
            const int cols = (P.m_t + 1) * binom(P.m_x - dmin + 3, 3);
            ks[tt] = (cols + 3) / 4;
            total += ks[tt];
        }
        // Split-K plan of one output block (all row tiles, one interval half).
        // For a block length T every tile's K-range is cut at multiples of T;
        // segments with the same start share the moment operands, so they are
        // grouped three at a time (sorted by length, so a group's lengths are
        // close) into waves.  Waves are then dealt to the 4 SIMDs of the CU
        // (wave w runs on SIMD w % 4) by longest-processing-time on their
        // slot-steps.  T minimises (busiest SIMD's slot-steps + longest wave),
        // i.e. MFMA balance plus the dependent chain of the slowest wave.
        std::vector<int> wmeta, segtab, redtile;
        bool ok = false;
        {
            struct Seg { int tile, start, end; };
            int best_cost = INT32_MAX;
            std::vector<std::vector<Seg>> best_waves;
            int maxks = 0;
            for (int k : ks) maxks = std::max(maxks, k);
            for (int T = 1; T <= maxks; ++T) {
                int nblk = (maxks + T - 1) / T;
                std::vector<std::vector<Seg>> waves;
                for (int b = 0; b < nblk; ++b) {
                    std::vector<Seg> sg;
                    for (int tt = 0; tt < ntile; ++tt)
                        if (ks[tt] > b * T) sg.push_back({tt, b * T, std::min((b + 1) * T, ks[tt])});
                    std::stable_sort(sg.begin(), sg.end(), [](const Seg& x, const Seg& y) { return x.end > y.end; });
                    for (size_t i = 0; i < sg.size(); i += kM2LSlots) {
                        std::vector<Seg> wv(sg.begin() + i, sg.begin() + std::min(sg.size(), i + kM2LSlots));
                        waves.push_back(wv);
                    }
                }
                if ((int)waves.size() > kM2LWaves) continue;
                // LPT over SIMDs, at most kM2LWaves / 4 waves each
                std::vector<int> order(waves.size());
                for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
                auto load = [&](int i) { int l = 0; for (auto& g : waves[i]) l += g.end - g.start; return l; };
                std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return load(x) > load(y); });
                int simd_load[4] = {0, 0, 0, 0}, simd_n[4] = {0, 0, 0, 0};
                std::vector<std::vector<Seg>> placed(kM2LWaves);
                int longest = 0;
                for (int i : order) {
                    int pick = -1;
                    for (int q = 0; q < 4; ++q)
                        if (simd_n[q] < kM2LWaves / 4 && (pick < 0 || simd_load[q] < simd_load[pick])) pick = q;
                    placed[simd_n[pick] * 4 + pick] = waves[i];
                    simd_n[pick] += 1;
                    simd_load[pick] += load(i);
                    longest = std::max(longest, waves[i][0].end - waves[i][0].start);
                }
                const int cost = *std::max_element(simd_load, simd_load + 4) + longest;
                if (cost < best_cost) { best_cost = cost; best_waves = placed; }
            }
            if (!best_waves.empty()) {
                ok = true;
                wmeta.assign(2 * kM2LWaves, 0);
                segtab.assign((size_t)kM2LWaves * kM2LSlots * 3, -1);
                for (int wv = 0; wv < kM2LWaves; ++wv) {
                    const auto& g = best_waves[wv];
                    wmeta[2 * wv] = g.empty() ? 0 : g[0].start;
                    wmeta[2 * wv + 1] = (int)g.size();
                    for (int i = 0; i < kM2LSlots; ++i) {
                        int* e = &segtab[((size_t)wv * kM2LSlots + i) * 3];
                        if (i < (int)g.size()) {
                            e[0] = g[i].tile;
                            e[1] = g[i].end;
                            e[2] = -1;
                            if (g[i].start > 0) { e[2] = (int)redtile.size(); redtile.push_back(e[0]); }
                        } else {
                            e[0] = -1; e[1] = 0; e[2] = -1;
                        }
                    }
                }
            }
        }
        // a wave's segments must be sorted by end (descending) for the phase loop; empty slots end at start
        int slots = ok ? kM2LSlots : 0;
        if (P.m_t > 15 || P.m_x > 15) slots = 0;
        const int TS = (P.m_t + 1) * (P.m_t + 1) * (P.m_x + 1) * (P.m_x + 1);
        t->TSp = (TS + 127) / 128 * 128;
        const size_t shm = std::max((size_t)6 * t->TSp * sizeof(double) + (size_t)2 * P.Nc * sizeof(int),
                                    redtile.size() * 8 * 64 * sizeof(double));
        int dev = 0, lds_max = 65536;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (shm > (size_t)lds_max) slots = 0;
        if (slots && shm > 65536)
            HIP_TRY(hipFuncSetAttribute((const void*)k_m2l_mfma<kM2LSlots>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        t->m2l_shm = shm;
        t->mfma_slots = slots;
        if (slots) {
            for (int wv = 0; wv < kM2LWaves; ++wv)
                for (int i = 0; i < kM2LSlots; ++i) {
                    int* e = &segtab[((size_t)wv * kM2LSlots + i) * 3];
                    if (e[0] < 0) e[1] = wmeta[2 * wv];
                }
            std::vector<int> segall(segtab);
            segall.insert(segall.end(), redtile.begin(), redtile.end());
            t->n_partial = (int)redtile.size();
            PF_TRY(upload(t, &t->packinfo, pk.data(), pk.size()));
            PF_TRY(upload(t, &t->slot_tile, segall.data(), segall.size()));
            PF_TRY(upload(t, &t->tile_ks, wmeta.data(), wmeta.size()));
        }
    }
    // wide matrix-core M2L: row groups for two and four interval blocks
    if (t->mfma_slots) {
        const int Nc = P.Nc, ntile = (Nc + 15) / 16;
        std::vector<int> ks(ntile);
        for (int tt = 0; tt < ntile; ++tt)
            ks[tt] = ((P.m_t + 1) * binom(P.m_x - P.coef_deg[16 * tt] + 3, 3) + 3) / 4;
        int dev = 0, lds_max = 65536;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        const int Nc4 = (Nc + 3) & ~3;
        // compact table length: (m_t+1)^2 time pairs of (m_x+1)(m_x+2)/2 entries,
        // plus m_x entries read (masked) past the last pair
        const int TSc = (P.m_t + 1) * (P.m_t + 1) * (P.m_x + 1) * (P.m_x + 2) / 2 + P.m_x;
        t->TSc64 = (TSc + 127) / 128 * 128;
        t->TSc32 = (TSc + 255) / 256 * 256;
        for (int q = 0; q < (t->has_f32 ? 3 : 1); ++q)
            for (int v = 0; v < 3; ++v) {
                auto& W = t->wide[q][v];
                const int maxs = kWideMaxs[q][v], waves = kWideWaves[q][v];
                const size_t es = q == 0 ? sizeof(double) : sizeof(float);
                const int tsp = q == 0 ? t->TSc64 : t->TSc32;
                std::vector<int> tab;
                int maxp = 0;
                if (!plan_wide(ks, maxs, waves, tab, W.G, W.stride, maxp)) continue;
                W.shm = std::max((size_t)12 * tsp * es + (size_t)(Nc4 + 16) * 4 * sizeof(int), (size_t)maxp * 8 * 64 * es);
                if (W.shm > (size_t)lds_max) continue;
                if (W.shm > 65536)
                    HIP_TRY(hipFuncSetAttribute(wide_fn(q, v), hipFuncAttributeMaxDynamicSharedMemorySize, (int)W.shm));
                PF_TRY(upload(t, &W.plan, tab.data(), tab.size()));
                W.ok = true;
            }
        // class-aware M2L for levels whose intervals differ
        bool any_cls = false;
        for (int l = 2; l <= P.depth; ++l) any_cls = any_cls || !P.lev[l].uniform;
        for (int q = 0; any_cls && q < (t->has_f32 ? 3 : 1); ++q) {
            auto& W = t->wcls[q];
            const size_t es = q == 0 ? sizeof(double) : sizeof(float);
            const int tsp = q == 0 ? t->TSc64 : t->TSc32;
            std::vector<int> tab;
            int maxp = 0;
            if (!plan_wide(ks, kClsMaxs[q], kClsWaves, tab, W.G, W.stride, maxp)) continue;
            W.shm = std::max((size_t)6 * tsp * es + (size_t)(Nc4 + 16) * 4 * sizeof(int), (size_t)maxp * 4 * 64 * es);
            if (W.shm > (size_t)lds_max) continue;
            if (W.shm > 65536) {
                HIP_TRY(hipFuncSetAttribute(cls_fn(q), hipFuncAttributeMaxDynamicSharedMemorySize, (int)W.shm));
                HIP_TRY(hipFuncSetAttribute(cls_batch_fn(q), hipFuncAttributeMaxDynamicSharedMemorySize, (int)W.shm));
            }
            PF_TRY(upload(t, &W.plan, tab.data(), tab.size()));
            W.ok = true;
        }
    }
    // staged 1D tables of the matrix-core M2L: per (level, time class, offset) the
    // x table with C_ab folded in and the plain table for y and z, each padded
    // to TSp doubles so that 1 KB pieces can be copied straight into LDS
    std::vector<int64_t> e1s_off(P.depth + 1, 0);
    if (t->mfma_slots) {
        const int nt1 = P.m_t + 1, nx1 = P.m_x + 1, TS = nt1 * nt1 * nx1 * nx1, TSp = t->TSp;
        std::vector<double> E1s;
        for (int l = 2; l <= P.depth; ++l) {
            const FarLevel& FL = F.lv[l];
            const int nR = 2 * FL.R + 1;
            e1s_off[l] = (int64_t)E1s.size();
            E1s.resize(E1s.size() + (size_t)FL.ncls * nR * 2 * TSp, 0.0);
            for (int D = 0; D < FL.ncls; ++D)   // time class (D = time offset - 2 on uniform levels)
                for (int oi = 0; oi < nR; ++oi) {
                    const double* e = &F.E1[FL.e1_off + ((size_t)D * nR + oi) * TS];
                    double* x = &E1s[e1s_off[l] + (((size_t)D * nR + oi) * 2 + 0) * TSp];
                    double* yz = x + TSp;
                    for (int i = 0; i < TS; ++i) {
                        x[i] = F.Cab[FL.cab_off + (size_t)D * nt1 * nt1 + i / (nx1 * nx1)] * e[i];
                        yz[i] = e[i];
                    }
                }
        }
        PF_TRY(upload(t, &t->E1s, E1s.data(), E1s.size()));
        // compact rows of the wide M2L: entry (a, b, kappa, nu) with kappa + nu <= m_x
        // at (a (m_t+1) + b) BS + T(kappa) + nu, T(kappa) = kappa (m_x+1) - kappa (kappa-1) / 2
        const int BS = nx1 * (nx1 + 1) / 2;
        const size_t nrows = E1s.size() / TSp;
        std::vector<double> E1c(nrows * t->TSc64, 0.0);
        for (size_t r = 0; r < nrows; ++r)
            for (int ab = 0; ab < nt1 * nt1; ++ab)
                for (int k = 0; k < nx1; ++k)
                    for (int n = 0; n + k < nx1; ++n)
                        E1c[r * t->TSc64 + (size_t)ab * BS + (k * nx1 - k * (k - 1) / 2) + n] =
                            E1s[r * TSp + (size_t)ab * nx1 * nx1 + k * nx1 + n];
        PF_TRY(upload(t, &t->E1c, E1c.data(), E1c.size()));
        if (t->has_f32) {
            std::vector<float> E1f(nrows * t->TSc32, 0.f);
            for (size_t r = 0; r < nrows; ++r)
                for (int i = 0; i < t->TSc64 && i < t->TSc32; ++i) E1f[r * t->TSc32 + i] = (float)E1c[r * t->TSc64 + i];
            PF_TRY(upload(t, &t->E1c32, E1f.data(), E1f.size()));
            for (float& x : E1f) {   // nearest bfloat16, ties to even
                uint32_t u;
                std::memcpy(&u, &x, 4);
                u += 0x7fffu + ((u >> 16) & 1u);
                u &= 0xffff0000u;
                std::memcpy(&x, &u, 4);
            }
            PF_TRY(upload(t, &t->E1c16, E1f.data(), E1f.size()));
        }
    }
    // levels
    t->lv.assign(P.depth + 1, DevLevel());
    for (int l = 0; l < 2 && l <= P.depth; ++l) {
        const Level& L = P.lev[l];
        for (size_t i = 0; i < L.leaf.size(); ++i)
            if (L.present[i] && L.leaf[i]) t->low_leaves = true;
    }
    for (int l = 2; l <= P.depth; ++l) {
        const Level& L = P.lev[l];
        const FarLevel& FL = F.lv[l];
        DevLevel& D = t->lv[l];
        D.l = l; D.nx = L.nx(); D.n_int = L.n_int;
        D.n_leafx = (int)FL.leaf_xs.size();
        D.uniform = L.uniform;
        for (int k = 0; k < L.n_int; ++k) D.maxlen = std::max(D.maxlen, FL.ilen[k]);
        PF_TRY(upload(t, &D.ist, FL.istart.data(), FL.istart.size()));
        PF_TRY(upload(t, &D.ilen, FL.ilen.data(), FL.ilen.size()));
        PF_TRY(upload(t, &D.lflag, FL.leaf.data(), FL.leaf.size()));
        {
            std::vector<int2> ch(FL.chunk_li.size());
            for (size_t i = 0; i < ch.size(); ++i) ch[i] = int2{FL.chunk_li[i], FL.chunk_r0[i]};
            D.n_lchunk = (int)ch.size();
            PF_TRY(upload(t, &D.lchunk, ch.data(), ch.size()));
        }
        PF_TRY(upload(t, &D.inner, FL.inner.data(), FL.inner.size()));
        if (!L.uniform) {
            if (!t->mfma_slots || !t->wcls[0].ok || (t->has_f32 && (!t->wcls[1].ok || !t->wcls[2].ok)))
                return fail(PFMM_EUNSUPPORTED, "levels with unequal intervals need the matrix-core M2L "
                                               "(degrees <= 15)");
            // columns of the class-aware M2L: the target intervals of each time
            // offset, sorted by class into sub-blocks of 16 of one class (the
            // last of a class padded with k = -1), NB sub-blocks to a column
            // block; a class's last block is filled up with empty sub-blocks
            // (class -1, no loads or products) so that every block holds one
            // class and a workgroup walks its sources once.  The moments are
            // gathered into this column order before each launch, so a
            // sub-block's B operand is one contiguous row
            const int per = 16 * kClsNB;
            for (int Dt = 2; Dt <= 3; ++Dt) {
                std::vector<std::pair<int, int>> cl;   // (class, k)
                for (int k = 0; k < L.n_int; ++k)
                    if (L.cls[Dt - 2][k] >= 0) cl.emplace_back(L.cls[Dt - 2][k], k);
                std::stable_sort(cl.begin(), cl.end());
                std::vector<int2> cols;
                auto close_class = [&](int c) {
                    while (cols.size() % 16) cols.push_back(int2{-1, c});
                    while (cols.size() % per) cols.push_back(int2{-1, -1});   // empty sub-blocks
                };
                for (size_t i = 0; i < cl.size(); ++i) {
                    if (i > 0 && cl[i].first != cl[i - 1].first) close_class(cl[i - 1].first);
                    cols.push_back(int2{cl[i].second, cl[i].first});
                }
                if (!cl.empty()) close_class(cl.back().first);
                const int nblk = (int)(cols.size() / per);
                std::vector<int2> br(nblk);
                std::vector<int> perm(cols.size());
                for (int b = 0; b < nblk; ++b) {
                    int lo = INT32_MAX, hi = -1;
                    for (int i = b * per; i < (b + 1) * per; ++i)
                        if (cols[i].y >= 0) { lo = std::min(lo, cols[i].y); hi = std::max(hi, cols[i].y); }
                    br[b] = int2{lo, hi};
                }
                for (size_t i = 0; i < cols.size(); ++i) perm[i] = cols[i].x >= 0 ? cols[i].x - Dt : -1;
                D.nccb[Dt - 2] = nblk;
                D.ncp[Dt - 2] = (int)cols.size();
                PF_TRY(upload(t, &D.ccols[Dt - 2], cols.data(), cols.size()));
                PF_TRY(upload(t, &D.cbr[Dt - 2], br.data(), br.size()));
                PF_TRY(upload(t, &D.cperm[Dt - 2], perm.data(), perm.size()));
            }
        }
        D.at_off = FL.at_off; D.qt_off = FL.qt_off; D.qx_off = FL.qx_off; D.n_off = FL.n_off;
        D.e1_off = FL.e1_off; D.cab_off = FL.cab_off; D.R = FL.R; D.e1s_off = e1s_off[l];
        PF_TRY(upload(t, &D.off3, FL.off3.data(), FL.off3.size()));
        // Two leading guard values (the wide M2L reads mu[-2], mu[-1] for target
        // interval 0, whose result it discards).  Zeroed once, so that every
        // moment a matrix-core M2L may multiply by a zero operator entry
        // (padding columns) is finite.
        PF_TRY(dalloc(t, &D.mu, (size_t)D.nx * P.Nc * D.n_int + 2));
        HIP_TRY(hipMemset(D.mu, 0, ((size_t)D.nx * P.Nc * D.n_int + 2) * sizeof(double)));
        D.mu += 2;
        PF_TRY(dalloc(t, &D.lam, (size_t)D.nx * P.Nc * D.n_int));
        {
            // enough workgroups to fill the chip several times: split source lists otherwise
            int dev = 0, ncu = 256;
            if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
            int nsplit_max = 1;
            for (int q = 0; q < 2; ++q) {
                int64_t wg = (int64_t)D.nx * ((D.n_int + 63) / 64) * (D.n_int > 32 ? 2 : 1);
                D.m2l_nb[q] = 0;
                if (!D.uniform) {   // class-aware M2L: whole source lists, no shares
                    D.nsplit_q[q] = 1;
                    continue;
                }
                if (t->mfma_slots && (q == 0 || t->has_f32)) {
                    for (int v = 2; v >= 0 && !D.m2l_nb[q]; --v)
                        if (t->wide[q][v].ok && (q == 0 || t->wide[2][v].ok) && D.n_int % (32 * kWideNB[v]) == 0 &&
                            (v > 0 || kWideUseNB1))
                            D.m2l_nb[q] = kWideNB[v];
                }
                int per_cu = std::max<int>(1, (int)(160 * 1024 / std::max<size_t>(1, t->m2l_shm)));   // resident per CU
                if (D.m2l_nb[q]) {
                    const int v = D.m2l_nb[q] == 4 ? 2 : (D.m2l_nb[q] == 2 ? 1 : 0);
                    D.ncb[q] = D.n_int / (32 * D.m2l_nb[q]);
                    wg = (int64_t)D.nx * t->wide[q][v].G * D.ncb[q];
                    per_cu = std::max<int>(1, (int)(160 * 1024 / std::max<size_t>(1, t->wide[q][v].shm)));
                }
                // Levels with fewer than 4 workgroups per CU split their source
                // lists into ns shares.  Wide kernels: enough shares for about
                // eight rounds of resident workgroups, ns = ceil(8 slots / wg) <= 8
                // (workgroup times vary with the list lengths, and finer shares
                // balance them; at 3072 x 256, levels 5 and 6: 26.0 ms at 3 shares,
                // 25.2 at 4, 25.4 at 6, 25.5 at 8).  Others (1..4): the share
                // minimising the rounds of resident workgroups per share,
                // ceil(wg ns / (ncu per_cu)) / ns, plus 2% per extra partial buffer.
                D.nsplit_q[q] = 1;
                if (wg < 4 * ncu && D.m2l_nb[q]) {
                    const int64_t slots = (int64_t)ncu * per_cu;
                    D.nsplit_q[q] = (int)std::min<int64_t>(8, std::max<int64_t>(1, (8 * slots + wg - 1) / wg));
                } else if (wg < 4 * ncu) {
                    double best = 1e30;
                    for (int ns = 1; ns <= 4; ++ns) {
                        const int64_t slots = (int64_t)ncu * per_cu;
                        const double c = (double)((wg * ns + slots - 1) / slots) / ns + 0.02 * (ns - 1);
                        if (c < best - 1e-9) { best = c; D.nsplit_q[q] = ns; }
                    }
                }
                nsplit_max = std::max(nsplit_max, D.nsplit_q[q]);
            }
            D.nsplit = D.nsplit_q[0];
            if (nsplit_max > 1) PF_TRY(dalloc(t, &D.lam_parts, (size_t)(nsplit_max - 1) * D.nx * P.Nc * D.n_int));
            D.parts_cap = nsplit_max;
            D.slot_pairs = (int64_t)FL.m2l_src.size();
            if (t->has_f32 && D.m2l_nb[1]) {
                PF_TRY(dalloc(t, &D.mu32, (size_t)D.nx * P.Nc * D.n_int + 2));
                HIP_TRY(hipMemset(D.mu32, 0, ((size_t)D.nx * P.Nc * D.n_int + 2) * sizeof(float)));
                D.mu32 += 2;
            }
            for (int Dt = 2; Dt <= 3 && !D.uniform; ++Dt) {
                const size_t np = (size_t)D.nx * P.Nc * D.ncp[Dt - 2];
                PF_TRY(dalloc(t, &D.mup[Dt - 2], np));
                if (t->has_f32) PF_TRY(dalloc(t, &D.mup32[Dt - 2], np));
            }
        }
        PF_TRY(upload(t, &D.leaf_xs, FL.leaf_xs.data(), FL.leaf_xs.size()));
        PF_TRY(upload(t, &D.ax_off, FL.ax_off.data(), FL.ax_off.size()));
        PF_TRY(upload(t, &D.tb, L.tb.data(), L.tb.size()));
        PF_TRY(upload(t, &D.te, L.te.data(), L.te.size()));
        if (ops_mask & PFMM_OP_K1) {
            std::vector<int> tb3(L.tb), te3(L.te);
            std::vector<int64_t> ao3(FL.ax_off);
            for (auto& x : tb3) x *= 3;
            for (auto& x : te3) x *= 3;
            for (auto& x : ao3) x *= 3;
            PF_TRY(upload(t, &D.tb3, tb3.data(), tb3.size()));
            PF_TRY(upload(t, &D.te3, te3.data(), te3.size()));
            PF_TRY(upload(t, &D.ax_off3, ao3.data(), ao3.size()));
        }
        PF_TRY(upload(t, &D.parent, L.parent.data(), L.parent.size()));
        std::vector<int> par;
        for (int xs = 0; xs < L.nx(); ++xs)
            if (FL.children_ptr[xs + 1] > FL.children_ptr[xs]) par.push_back(xs);
        D.n_par = (int)par.size();
        PF_TRY(upload(t, &D.par_xs, par.data(), par.size()));
        PF_TRY(upload(t, &D.ch_ptr, FL.children_ptr.data(), FL.children_ptr.size()));
        PF_TRY(upload(t, &D.ch, FL.children.data(), FL.children.size()));
        PF_TRY(upload(t, &D.m2l_ptr, FL.m2l_ptr.data(), FL.m2l_ptr.size()));
        PF_TRY(upload(t, &D.m2l_src, FL.m2l_src.data(), FL.m2l_src.size()));
        PF_TRY(upload(t, &D.m2l_cls, FL.m2l_cls.data(), FL.m2l_cls.size()));
        if (!L.uniform) {
            // target groups of the class-aware M2L: kClsKT consecutive slots
            // (Morton order: neighbours, with nearly the same offsets within
            // the truncation radius); per group, the union of the targets'
            // offset classes in increasing order with each target's source
            const int KT = kClsKT;
            const int ng = (L.nx() + KT - 1) / KT;
            std::vector<int> gx((size_t)ng * KT, -1), gptr(ng + 1, 0), gcls, gsrc;
            std::map<int, std::array<int, kClsKT>> merged;
            for (int gi = 0; gi < ng; ++gi) {
                merged.clear();
                for (int j = 0; j < KT; ++j) {
                    const int xs = gi * KT + j;
                    if (xs >= L.nx()) break;
                    gx[(size_t)gi * KT + j] = xs;
                    for (int e = FL.m2l_ptr[xs]; e < FL.m2l_ptr[xs + 1]; ++e) {
                        auto it = merged.find(FL.m2l_cls[e]);
                        if (it == merged.end()) {
                            std::array<int, kClsKT> none;
                            none.fill(-1);
                            it = merged.emplace(FL.m2l_cls[e], none).first;
                        }
                        it->second[j] = FL.m2l_src[e];
                    }
                }
                for (const auto& kv : merged) {
                    gcls.push_back(kv.first);
                    gsrc.insert(gsrc.end(), kv.second.begin(), kv.second.end());
                }
                gptr[gi + 1] = (int)gcls.size();
            }
            D.ntg = ng;
            PF_TRY(upload(t, &D.tg_x, gx.data(), gx.size()));
            PF_TRY(upload(t, &D.tg_ptr, gptr.data(), gptr.size()));
            if (!gcls.empty()) {
                PF_TRY(upload(t, &D.tg_cls, gcls.data(), gcls.size()));
                PF_TRY(upload(t, &D.tg_src, gsrc.data(), gsrc.size()));
            }
        }
        // explicit operators: only for the vector-unit M2L used above the matrix-core limits
        if (FL.n_off > 0 && t->mfma_slots == 0) {
            const int64_t total = (int64_t)FL.n_off * 2 * F.op_size;
            PF_TRY(dalloc(t, &D.ops, (size_t)total));
            hipLaunchKernelGGL(k_m2l_opgen, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, D.ops,
                               E1 + FL.e1_off, Cab + FL.cab_off, D.off3, t->chunk_cols, t->chunk_off, t->cm,
                               F.n_chunks, F.op_size, FL.R, total);
            HIP_TRY(hipGetLastError());
        }
    }
    // nearfield layout
    {
        const size_t nL = P.leaves.size();
        std::vector<int> rl(P.rows.size()), rk(P.rows.size());
        std::vector<int64_t> rb(P.rows.size());
        for (size_t i = 0; i < P.rows.size(); ++i) { rl[i] = P.rows[i].leaf; rk[i] = P.rows[i].kt; rb[i] = P.rows[i].boff; }
        std::vector<int> ltb(nL), lnx(nL), lr0(nL), lr1(nL), lg(nL);
        for (size_t i = 0; i < nL; ++i) {
            const LeafRec& R = P.leaves[i];
            ltb[i] = R.tb; lnx[i] = R.te - R.tb; lr0[i] = R.rect0; lr1[i] = R.rect1; lg[i] = R.group;
            if (lnx[i] > kWave) return fail(PFMM_EINVAL, "internal: a nearfield row chunk holds more than 64 triangles");
        }
        std::vector<int> j0(P.rects.size()), j1(P.rects.size()), rs(P.rects.size());
        for (size_t i = 0; i < P.rects.size(); ++i) {
            j0[i] = P.rects[i].j0; j1[i] = P.rects[i].j1; rs[i] = P.rects[i].set;
            // the nearfield kernels count a rectangle's columns in 32 bits
            if ((int64_t)(j1[i] - j0[i]) * P.set_size[rs[i]] > (int64_t)INT32_MAX)
                return fail(PFMM_EUNSUPPORTED, "a nearfield rectangle has more than 2^31 - 1 columns");
        }
        NearLayout& NL = t->nl;
        int *a1, *a2, *a4, *a5, *a6, *a7, *a8, *a9, *a10, *a11, *a12, *a13, *a14;
        int64_t* a3;
        PF_TRY(upload(t, &a1, rl.data(), rl.size()));
        PF_TRY(upload(t, &a2, rk.data(), rk.size()));
        PF_TRY(upload(t, &a3, rb.data(), rb.size()));
        PF_TRY(upload(t, &a4, ltb.data(), ltb.size()));
        PF_TRY(upload(t, &a5, lnx.data(), lnx.size()));
        PF_TRY(upload(t, &a6, lr0.data(), lr0.size()));
        PF_TRY(upload(t, &a7, lr1.data(), lr1.size()));
        PF_TRY(upload(t, &a8, lg.data(), lg.size()));
        PF_TRY(upload(t, &a9, j0.data(), j0.size()));
        PF_TRY(upload(t, &a10, j1.data(), j1.size()));
        PF_TRY(upload(t, &a11, rs.data(), rs.size()));
        PF_TRY(upload(t, &a12, P.set_off.data(), P.set_off.size()));
        PF_TRY(upload(t, &a13, P.set_size.data(), P.set_size.size()));
        PF_TRY(upload(t, &a14, P.set_pos.data(), P.set_pos.size()));
        NL = NearLayout{a1, a2, a3, a4, a5, a6, a7, a8, a9, a10, a11, a12, a13, a14, P.E_x, (int64_t)P.rows.size(), P.E_x};
        std::vector<GroupDev> gd(P.groups.size());
        for (size_t i = 0; i < P.groups.size(); ++i) {
            const AsmGroup& A = P.groups[i];
            gd[i] = GroupDev{A.tb, A.te, A.dmax, A.usize, A.uoff, A.toff, A.mapoff};
        }
        PF_TRY(upload(t, &t->groups, gd.data(), gd.size()));
        PF_TRY(upload(t, &t->umap, P.umap.data(), P.umap.size()));
        if (ops_mask & PFMM_OP_K1) {
            // the p1 double layer: the same row groups, leaves and rectangles
            // over expanded source sets (position 3 p + i: local vertex i)
            const Plan::P1Layout& L3 = P.p1;
            for (size_t i = 0; i < P.rects.size(); ++i)
                if ((int64_t)(j1[i] - j0[i]) * L3.set_size[rs[i]] > (int64_t)INT32_MAX)
                    return fail(PFMM_EUNSUPPORTED, "a nearfield rectangle has more than 2^31 - 1 columns");
            int64_t* b3;
            int *o3, *z3, *p3;
            PF_TRY(upload(t, &b3, L3.boff.data(), L3.boff.size()));
            PF_TRY(upload(t, &o3, L3.set_off.data(), L3.set_off.size()));
            PF_TRY(upload(t, &z3, L3.set_size.data(), L3.set_size.size()));
            PF_TRY(upload(t, &p3, L3.set_pos.data(), L3.set_pos.size()));
            t->nl3 = NL;
            t->nl3.rg_boff = b3;
            t->nl3.set_off = o3;
            t->nl3.set_size = z3;
            t->nl3.set_pos = p3;
            t->nl3.E_src = 3 * P.E_x;
            std::vector<GroupDev> g3(P.groups.size());
            for (size_t i = 0; i < P.groups.size(); ++i) {
                const AsmGroup& A = P.groups[i];
                g3[i] = GroupDev{A.tb, A.te, A.dmax, 3 * A.usize, A.uoff, L3.toff[i], (int64_t)i * 3 * P.E_x};
            }
            PF_TRY(upload(t, &t->groups3, g3.data(), g3.size()));
            PF_TRY(upload(t, &t->umap3, L3.umap.data(), L3.umap.size()));
            PF_TRY(dalloc(t, &t->wd3, (size_t)3 * N));
        }
        if (t->nf_mode == PFMM_NF_TOEPLITZ) {
            // per leaf rectangle: the table column u of every source triangle
            // (one list per distinct (group, set) pair)
            std::vector<int64_t> roff(P.rects.size(), 0);
            std::vector<int> ru;
            std::map<std::pair<int, int>, int64_t> seen;
            for (const LeafRec& R : P.leaves)
                for (int q = R.rect0; q < R.rect1; ++q) {
                    const int set = P.rects[q].set;
                    auto key = std::make_pair(R.group, set);
                    auto it = seen.find(key);
                    if (it == seen.end()) {
                        it = seen.emplace(key, (int64_t)ru.size()).first;
                        const AsmGroup& A = P.groups[R.group];
                        for (int i = 0; i < P.set_size[set]; ++i)
                            ru.push_back(P.umap[A.mapoff + P.set_pos[P.set_off[set] + i]]);
                    }
                    roff[q] = it->second;
                }
            PF_TRY(upload(t, &t->ru_off, roff.data(), roff.size()));
            PF_TRY(upload(t, &t->ru, ru.data(), ru.size()));
            PF_TRY(plan_near_gemm(t));
        }
    }
    if (ops_mask & PFMM_OP_V) { PF_TRY(assemble_near(t, 0, t->opV, st)); t->hasV = true; }
    if (ops_mask & PFMM_OP_K) { PF_TRY(assemble_near(t, 1, t->opK, st)); t->hasK = true; }
    if (ops_mask & PFMM_OP_K1) { PF_TRY(assemble_near(t, 2, t->opK1, st)); t->hasK1 = true; }
    HIP_TRY(hipStreamSynchronize(st));
    return PFMM_OK;
}

void prof_begin(pfmm_tree* t, int stage, hipStream_t st, int& idx) {
    idx = -1;
    if (!t->prof) return;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
    (void)hipEventRecord(a, st);
    t->ev.push_back(a);
    t->ev.push_back(b);
    idx = (int)t->ev.size() - 2;
    t->ev_used.emplace_back(stage, idx);
}

void prof_end(pfmm_tree* t, hipStream_t st, int idx) {
    if (idx >= 0) (void)hipEventRecord(t->ev[idx + 1], st);
}

// Precision index of the class-aware M2L (0 FP64, 1 FP32, 2 BF16 inputs)
// for the tree's current farfield precision; cls_prep also converts the
// level's moments for the reduced precisions and zeroes its locals (the
// class-aware kernel adds into them), stream-ordered on st.
int cls_q(const pfmm_tree* t) { return t->prec == PFMM_FP64 ? 0 : (t->prec == PFMM_MIXED_BF16 ? 2 : 1); }

int cls_prep(pfmm_tree* t, int l, hipStream_t st) {
    DevLevel& D = t->lv[l];
    const int64_t nl = (int64_t)D.nx * t->P.Nc * D.n_int;
    const int q = cls_q(t);
    for (int Dt = 2; Dt <= 3; ++Dt) {
        if (D.nccb[Dt - 2] == 0) continue;
        const int64_t np = (int64_t)D.nx * t->P.Nc * D.ncp[Dt - 2];
        const dim3 g((unsigned)((np + 255) / 256));
        if (q == 0)
            hipLaunchKernelGGL(k_gather_cols<double>, g, dim3(256), 0, st, D.mu, D.mup[Dt - 2], D.cperm[Dt - 2],
                               D.n_int, D.ncp[Dt - 2], np, 0);
        else
            hipLaunchKernelGGL(k_gather_cols<float>, g, dim3(256), 0, st, D.mu, D.mup32[Dt - 2], D.cperm[Dt - 2],
                               D.n_int, D.ncp[Dt - 2], np, q == 2 ? 1 : 0);
    }
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, st, D.lam, 0.0, nl);
    return q;
}

ClsUnit cls_unit(const pfmm_tree* t, int l, int Dt, int q) {
    const DevLevel& D = t->lv[l];
    const int64_t row0 = D.e1s_off / std::max(1, t->TSp);   // first table row of the level
    ClsUnit U{};
    U.mu = q ? (const void*)D.mup32[Dt - 2] : (const void*)D.mup[Dt - 2];
    U.ncp = D.ncp[Dt - 2];
    U.lam = D.lam;
    U.tgx = D.tg_x;
    U.tgptr = D.tg_ptr;
    U.tgcls = D.tg_cls;
    U.tgsrc = D.tg_src;
    U.off3 = D.off3;
    U.E1c = q == 0 ? (const void*)(t->E1c + row0 * t->TSc64)
                   : (const void*)((q == 2 ? t->E1c16 : t->E1c32) + row0 * t->TSc32);
    U.cols = D.ccols[Dt - 2];
    U.cbr = D.cbr[Dt - 2];
    U.n_int = D.n_int;
    U.R = D.R;
    U.ntg = D.ntg;
    U.nccb = D.nccb[Dt - 2];
    U.D = Dt;
    U.wg0 = 0;
    return U;
}

// M2L (eq. m2l) of level l in the tree's current farfield precision, with
// the level's kernel choice: the class-aware kernel for levels with unequal
// or missing intervals, else the wide matrix-core kernel (interval blocks and
// list shares per precision), the narrow one for levels with fewer than 32
// intervals, or the vector-unit kernel above the matrix-core limits.
void m2l_level(pfmm_tree* t, int l, hipStream_t st) {
    const Plan& P = t->P;
    DevLevel& D = t->lv[l];
    const int64_t nl = (int64_t)D.nx * P.Nc * D.n_int;
    const int64_t row0 = D.e1s_off / std::max(1, t->TSp);   // first table row of the level
    if (!D.uniform) {
        // class-aware M2L: zero the locals, then one launch per time offset
        const int q = cls_prep(t, l, st);
        const auto& W = t->wcls[q];
        for (int Dt = 2; Dt <= 3; ++Dt) {
            if (D.nccb[Dt - 2] == 0) continue;
            dim3 grid(W.G, D.ntg, D.nccb[Dt - 2]);
            cls_launcher(q)(grid, W.shm, st, cls_unit(t, l, Dt, q), q ? t->TSc32 : t->TSc64, t->packinfo, W.plan,
                            W.stride, P.Nc, P.m_t, P.m_x);
        }
        return;
    }
    // q: 0 FP64, 1 FP32, 2 BF16 inputs; the per-level choices of the two
    // reduced precisions coincide (same kernel shapes), stored at index 1
    const int q = (t->prec != PFMM_FP64 && D.m2l_nb[1]) ? (t->prec == PFMM_MIXED_BF16 ? 2 : 1) : 0;
    const int ql = q > 0 ? 1 : 0;
    if (D.m2l_nb[ql]) {
        const int v = D.m2l_nb[ql] == 4 ? 2 : (D.m2l_nb[ql] == 2 ? 1 : 0);
        const auto& W = t->wide[q][v];
        const int nsplit = D.nsplit_q[ql];
        dim3 grid(W.G, D.nx, D.ncb[ql] * nsplit);
        const void* m = D.mu;
        const void* e1 = t->E1c + row0 * t->TSc64;
        int tsp = t->TSc64;
        if (q >= 1) {
            hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, st, D.mu, D.mu32, nl,
                               q == 2 ? 1 : 0);
            m = D.mu32;
            e1 = (q == 2 ? t->E1c16 : t->E1c32) + row0 * t->TSc32;
            tsp = t->TSc32;
        }
        wide_launcher(q, v)(grid, W.shm, st, m, D.lam, D.m2l_ptr, D.m2l_src, D.m2l_cls, D.off3, e1, tsp, t->packinfo,
                            W.plan, W.stride, P.Nc, D.n_int, P.m_t, P.m_x, D.R, nsplit, D.ncb[ql], D.lam_parts);
        if (nsplit > 1)
            hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, st, D.lam, D.lam_parts,
                               nsplit - 1, nl);
    } else if (t->mfma_slots) {
        const size_t shm = t->m2l_shm;
        const int halves = D.n_int > 32 ? 2 : 1;
        dim3 grid(D.nx, (D.n_int + 63) / 64, halves * D.nsplit);
        dim3 block(64 * kM2LWaves);
        // share 0 writes lambda, share p >= 1 writes lam_parts + (p - 1) * (slots * Nc * n_int)
        hipLaunchKernelGGL(k_m2l_mfma<kM2LSlots>, grid, block, shm, st, D.mu, D.lam, D.m2l_ptr, D.m2l_src, D.m2l_cls,
                           D.off3, t->E1s + D.e1s_off, t->TSp, t->packinfo, t->tile_ks, t->slot_tile, t->n_partial,
                           P.Nc, D.n_int, P.m_t, P.m_x, D.R, D.nsplit, halves, D.lam_parts);
        if (D.nsplit > 1)
            hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, st, D.lam, D.lam_parts,
                               D.nsplit - 1, nl);
    } else {
        dim3 grid(D.nx, (D.n_int + kWave - 1) / kWave, t->F.n_chunks);
        hipLaunchKernelGGL(k_m2l, grid, dim3(kWave), 0, st, D.mu, D.lam, D.ops, D.m2l_ptr, D.m2l_src, D.m2l_cls,
                           t->chunk_cols, t->chunk_off, P.Nc, D.n_int, t->F.op_size);
    }
}

// phase 0: the whole apply; phase 1: permutation, nearfield, upward pass and
// the M2L of the levels with equal intervals (the others only prepared:
// moments converted, locals zeroed); phase 2: L2L, L2T and the final
// permutation.  Between phases 1 and 2 a batch runs the class-aware M2L of
// all its trees in one launch per time offset.
// kind: 0 V_h, 1 K_h, 2 K_h with p1 trial functions (w: vertex values,
// n_steps x n_vertices).
pfmm_status apply(pfmm_tree* t, int kind, const double* w, double* f, hipStream_t st, int phase = 0) {
    Plan& P = t->P;
    const bool K = kind >= 1, p1 = kind == 2;
    const int64_t N = (int64_t)P.E_t * P.E_x;
    const unsigned nb = (unsigned)((N + 255) / 256);
    int ev;
    if (phase != 2) {
        prof_begin(t, 0, st, ev);
        if (p1)
            hipLaunchKernelGGL(k_gather_p1, dim3((unsigned)((3 * N + 255) / 256)), dim3(256), 0, st, w, t->wd3,
                               t->inv_sigma, t->geom.tris, t->n_verts, P.E_x, 3 * N);
        else
            hipLaunchKernelGGL(k_permute_in, dim3(nb), dim3(256), 0, st, w, t->wd, t->inv_sigma, P.E_x, N);
        prof_end(t, st, ev);
    }
    // The nearfield product needs only the permuted densities: in Toeplitz
    // mode it runs on the side stream into fn while the farfield chain fills
    // fd, and the two meet in the final permutation.  The stored-block product
    // runs in order: it streams HBM at close to the read rate, and beside the
    // upward pass it slowed that pass by more than it hid (measured).  With
    // stage timing on, or while st is being captured into a graph (batched
    // applies, whose branches already run trees side by side), both run in
    // order on st: same kernels, same results.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cap));
    const bool fork = phase == 0 && !t->prof && cap == hipStreamCaptureStatusNone && t->nf_mode == PFMM_NF_TOEPLITZ;
    auto nearfield = [&](hipStream_t sn) {
        const int64_t nrg = (int64_t)P.rows.size();
        hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, sn, t->fn, 0.0, N);
        if (nrg > 0 && t->nf_mode == PFMM_NF_TOEPLITZ) {
            const double* tab = K ? t->opK.table : t->opV.table;
            const unsigned mt = (unsigned)((P.E_t + 15) / 16);
            for (int c = 0; c < 4; ++c) {
                const int g0 = t->ngg_start[c], g1 = t->ngg_start[c + 1];
                if (g1 <= g0) continue;
                const dim3 grid((unsigned)(g1 - g0), mt);
                const NearGemmGroup* gp = t->ngg + g0;
                // dynamic LDS: the largest group's quad ranges and records (at most 40 KB)
                const size_t shm = (size_t)t->ngg_lds[c];
                if (c == 0) hipLaunchKernelGGL(k_near_gemm<1>, grid, dim3(256), shm, sn, tab, gp, t->nue, t->nlst, t->wd, t->fn, P.E_x, P.E_t);
                if (c == 1) hipLaunchKernelGGL(k_near_gemm<2>, grid, dim3(256), shm, sn, tab, gp, t->nue, t->nlst, t->wd, t->fn, P.E_x, P.E_t);
                if (c == 2) hipLaunchKernelGGL(k_near_gemm<3>, grid, dim3(256), shm, sn, tab, gp, t->nue, t->nlst, t->wd, t->fn, P.E_x, P.E_t);
                if (c == 3) hipLaunchKernelGGL(k_near_gemm<4>, grid, dim3(256), shm, sn, tab, gp, t->nue, t->nlst, t->wd, t->fn, P.E_x, P.E_t);
            }
            if (t->n_sel > 0)
                hipLaunchKernelGGL(k_near_toep, dim3((unsigned)((t->n_sel + 3) / 4)), dim3(256), 0, sn, tab, t->groups,
                                   t->ru_off, t->ru, t->wd, t->fn, t->nl, (const int*)t->nsel, t->n_sel);
        }
        else if (nrg > 0 && p1)
            hipLaunchKernelGGL(k_near_apply, dim3((unsigned)((nrg + 3) / 4)), dim3(256), 0, sn, t->opK1.B, t->wd3,
                               t->fn, t->nl3);
        else if (nrg > 0)
            hipLaunchKernelGGL(k_near_apply, dim3((unsigned)((nrg + 3) / 4)), dim3(256), 0, sn,
                               K ? t->opK.B : t->opV.B, t->wd, t->fn, t->nl);
    };
    if (fork) {
        HIP_TRY(hipEventRecord(t->ev_fork, st));
        HIP_TRY(hipStreamWaitEvent(t->side, t->ev_fork, 0));
        nearfield(t->side);
        HIP_TRY(hipEventRecord(t->ev_join, t->side));
    }
    if (phase == 1) {
        prof_begin(t, 6, st, ev);
        nearfield(st);
        prof_end(t, st, ev);
    }
    if (phase != 2 && (t->low_leaves || !P.has_far))
        hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, st, t->fd, 0.0, N);
    if (P.has_far && phase != 2) {
        // S2M
        prof_begin(t, 1, st, ev);
        for (int l = 2; l <= P.depth; ++l) {
            DevLevel& D = t->lv[l];
            if (D.n_leafx == 0) continue;
            const int KI = t->ki_s2m, nt1 = P.m_t + 1;
            const size_t shm = ((size_t)nt1 * 64 * KI + (t->stage_s2m ? 64 * (size_t)P.Nk : 0)) * sizeof(double);
            if (p1)   // three rows per triangle: its local vertices
                hipLaunchKernelGGL(k_s2m_blk, dim3(D.n_leafx, (D.n_int + KI - 1) / KI), dim3(256), shm, st, t->wd3,
                                   D.mu, D.leaf_xs, D.ax_off3, D.tb3, D.te3, t->At + D.at_off, t->AxK1, t->sm,
                                   D.n_int, D.ist, D.ilen, D.lflag, 3 * P.E_x, KI, t->stage_s2m);
            else
                hipLaunchKernelGGL(k_s2m_blk, dim3(D.n_leafx, (D.n_int + KI - 1) / KI), dim3(256), shm, st, t->wd,
                                   D.mu, D.leaf_xs, D.ax_off, D.tb, D.te, t->At + D.at_off, K ? t->AxK : t->Ax,
                                   t->sm, D.n_int, D.ist, D.ilen, D.lflag, P.E_x, KI, t->stage_s2m);
        }
        prof_end(t, st, ev);
        // M2M, levels p-1 .. 2
        prof_begin(t, 2, st, ev);
        for (int l = P.depth - 1; l >= 2; --l) {
            DevLevel& D = t->lv[l];
            DevLevel& C = t->lv[l + 1];
            if (D.n_par == 0) continue;
            const int KI = t->ki_m2m, nt1 = P.m_t + 1, nx1 = P.m_x + 1;
            const size_t shm = (3 * (size_t)P.Nc * KI + 3 * nx1 * nx1 + 2 * KI * nt1 * nt1) * sizeof(double);
            hipLaunchKernelGGL(k_m2m_sep, dim3(D.n_par, (D.n_int + KI - 1) / KI), dim3(256), shm, st, C.mu, D.mu,
                               D.par_xs, D.ch_ptr, D.ch, t->qt + C.qt_off, t->qx + C.qx_off, t->sm, D.n_int, C.n_int,
                               KI, D.inner);
        }
        prof_end(t, st, ev);
        // M2L, levels 2 .. p
        prof_begin(t, 3, st, ev);
        for (int l = 2; l <= P.depth; ++l) {
            if (phase == 1 && !t->lv[l].uniform) cls_prep(t, l, st);
            else m2l_level(t, l, st);
        }
        prof_end(t, st, ev);
    }
    if (P.has_far && phase != 1) {
        // L2L, levels 3 .. p
        prof_begin(t, 4, st, ev);
        for (int l = 3; l <= P.depth; ++l) {
            DevLevel& D = t->lv[l];
            DevLevel& Pp = t->lv[l - 1];
            const int KI = t->ki_l2l, nt1 = P.m_t + 1, nx1 = P.m_x + 1;
            const size_t shm = (2 * (size_t)P.Nc * KI + 3 * nx1 * nx1 + 2 * KI * nt1 * nt1) * sizeof(double);
            hipLaunchKernelGGL(k_l2l_sep, dim3(D.nx, (Pp.n_int + KI - 1) / KI), dim3(256), shm, st, Pp.lam, D.lam,
                               D.parent, t->qt + D.qt_off, t->qx + D.qx_off, t->sm, D.n_int, Pp.n_int, KI);
        }
        prof_end(t, st, ev);
        // L2T
        prof_begin(t, 5, st, ev);
        for (int l = 2; l <= P.depth; ++l) {
            DevLevel& D = t->lv[l];
            if (D.n_leafx == 0) continue;
            const int KI = t->ki_l2t, nt1 = P.m_t + 1;
            const size_t shm = ((size_t)P.Nc * KI + (size_t)nt1 * 64 * KI + (t->stage_l2t ? 64 * (size_t)P.Nk : 0)) *
                               sizeof(double);
            hipLaunchKernelGGL(k_l2t_blk, dim3(D.n_lchunk, (D.n_int + KI - 1) / KI), dim3(256), shm, st, D.lam, t->fd,
                               D.leaf_xs, D.ax_off, D.tb, D.te, t->At + D.at_off, t->Ax, t->sm, D.n_int, D.ist,
                               D.ilen, D.lflag, D.lchunk, D.maxlen, P.E_x, KI, t->stage_l2t);
        }
        prof_end(t, st, ev);
    }
    if (phase == 1) {
        HIP_TRY(hipGetLastError());
        return PFMM_OK;
    }
    // nearfield
    if (fork) {
        HIP_TRY(hipStreamWaitEvent(st, t->ev_join, 0));
    } else if (phase == 0) {
        prof_begin(t, 6, st, ev);
        nearfield(st);
        prof_end(t, st, ev);
    }
    prof_begin(t, 7, st, ev);
    hipLaunchKernelGGL(k_permute_out, dim3(nb), dim3(256), 0, st, t->fd, t->fn, f, t->sigma, P.E_x, N);
    prof_end(t, st, ev);
    HIP_TRY(hipGetLastError());
    return PFMM_OK;
}

// ---------------------------------------------------------------- autotuner
// Launch configurations of the matrix-core M2L per (level, precision):
// interval blocks per workgroup of the wide kernel (variant v: 32, 64, 128
// intervals) and interaction-list shares.  Candidates are timed on the device
// (one warm-up, then three launches between HIP events); the fastest is kept
// and cached in a small JSON file keyed by the device and the level's shape.
struct TuneEntry { std::string kernel; int nb = 0, shares = 1; double ms = 0.0; };

std::map<std::string, TuneEntry> tune_read(const char* path) {
    std::map<std::string, TuneEntry> m;
    if (!path) return m;
    FILE* f = std::fopen(path, "r");
    if (!f) return m;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        // "key": {"kernel": "name", "nb": N, "shares": S, "ms": T}
        const char* a = std::strchr(line, '"');
        if (!a) continue;
        const char* b = std::strchr(a + 1, '"');
        if (!b) continue;
        std::string key(a + 1, b);
        const char* k = std::strstr(b, "\"kernel\": \"");
        if (!k) continue;
        k += 11;
        const char* ke = std::strchr(k, '"');
        if (!ke) continue;
        TuneEntry e;
        e.kernel.assign(k, ke);
        if (std::sscanf(ke, "\", \"nb\": %d, \"shares\": %d, \"ms\": %lf", &e.nb, &e.shares, &e.ms) != 3) continue;
        m[key] = e;
    }
    std::fclose(f);
    return m;
}

bool tune_write(const char* path, const std::map<std::string, TuneEntry>& m) {
    if (!path) return true;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m) {
        std::fprintf(f, "\"%s\": {\"kernel\": \"%s\", \"nb\": %d, \"shares\": %d, \"ms\": %.6f}%s\n", kv.first.c_str(),
                     kv.second.kernel.c_str(), kv.second.nb, kv.second.shares, kv.second.ms,
                     ++i < m.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

// room for `shares` list shares of level D's partial locals
pfmm_status ensure_parts(pfmm_tree* t, DevLevel& D, int shares) {
    if (shares <= D.parts_cap) return PFMM_OK;
    if (D.lam_parts) {
        auto it = std::find(t->allocs.begin(), t->allocs.end(), (void*)D.lam_parts);
        if (it != t->allocs.end()) t->allocs.erase(it);
        t->bytes -= (uint64_t)(D.parts_cap - 1) * D.nx * t->P.Nc * D.n_int * sizeof(double);
        HIP_TRY(hipFree(D.lam_parts));
        D.lam_parts = nullptr;
        D.parts_cap = 1;
    }
    PF_TRY(dalloc(t, &D.lam_parts, (size_t)(shares - 1) * D.nx * t->P.Nc * D.n_int));
    D.parts_cap = shares;
    return PFMM_OK;
}

pfmm_status autotune(pfmm_tree* t, const char* path, hipStream_t st, int* n_tuned, int* n_cached) {
    const Plan& P = t->P;
    *n_tuned = *n_cached = 0;
    if (!P.has_far || !t->mfma_slots) return PFMM_OK;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, t->device));
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    std::map<std::string, TuneEntry> cache = tune_read(path);
    const int saved = t->prec;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    pfmm_status status = PFMM_OK;
    bool dirty = false;
    for (int l = 2; l <= P.depth && status == PFMM_OK; ++l) {
        DevLevel& D = t->lv[l];
        if (!D.uniform) continue;
        for (int ql = 0; ql < (t->has_f32 ? 2 : 1) && status == PFMM_OK; ++ql) {
            // candidates of this (level, precision)
            std::vector<std::pair<int, int>> cand;   // (variant or -1 for the narrow kernel, shares)
            const bool wide = ql == 0 ? D.m2l_nb[0] != 0 : D.m2l_nb[1] != 0;
            if (ql == 1 && !wide) continue;          // reduced precisions use the wide kernel only
            if (wide) {
                for (int v = 0; v < 3; ++v) {
                    if (!t->wide[ql][v].ok || (ql == 1 && !t->wide[2][v].ok)) continue;
                    if (D.n_int % (32 * kWideNB[v])) continue;
                    for (int ns : {1, 2, 3, 4, 6, 8}) cand.emplace_back(v, ns);
                }
            } else {
                for (int ns : {1, 2, 3, 4}) cand.emplace_back(-1, ns);
            }
            if (cand.empty()) continue;
            char key[256];
            std::snprintf(key, sizeof(key), "%s:%dcu|Nc=%d|mt=%d|mx=%d|nint=%d|nx=%d|pairs=%lld|%s", arch.c_str(),
                          prop.multiProcessorCount, P.Nc, P.m_t, P.m_x, D.n_int, D.nx, (long long)D.slot_pairs,
                          ql ? "fp32" : "fp64");
            auto apply_choice = [&](int v, int ns) -> pfmm_status {
                PF_TRY(ensure_parts(t, D, ns));
                if (v >= 0) {
                    D.m2l_nb[ql] = kWideNB[v];
                    D.ncb[ql] = D.n_int / (32 * kWideNB[v]);
                    D.nsplit_q[ql] = ns;
                    if (ql == 0) D.nsplit = ns;
                } else {
                    D.nsplit_q[0] = D.nsplit = ns;
                }
                return PFMM_OK;
            };
            auto it = cache.find(key);
            if (it != cache.end()) {
                int v = -1;
                for (int q = 0; q < 3; ++q) if (kWideNB[q] == it->second.nb) v = q;
                const bool valid = (it->second.kernel == "k_m2l_wide") == wide &&
                                   std::find(cand.begin(), cand.end(), std::make_pair(wide ? v : -1, it->second.shares)) !=
                                       cand.end();
                if (valid) {
                    status = apply_choice(wide ? v : -1, it->second.shares);
                    ++*n_cached;
                    continue;
                }
            }
            t->prec = ql ? PFMM_MIXED_FP32 : PFMM_FP64;
            double best = 1e30;
            std::pair<int, int> pick = cand[0];
            for (const auto& c : cand) {
                status = apply_choice(c.first, c.second);
                if (status != PFMM_OK) break;
                m2l_level(t, l, st);
                hipError_t e = hipEventRecord(e0, st);
                for (int r = 0; r < 3 && e == hipSuccess; ++r) m2l_level(t, l, st);
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess) e = hipGetLastError();
                if (e != hipSuccess) { status = fail(PFMM_EDEVICE, std::string("autotune: ") + hipGetErrorString(e)); break; }
                if (ms / 3.0 < best) { best = ms / 3.0; pick = c; }
            }
            if (status != PFMM_OK) break;
            status = apply_choice(pick.first, pick.second);
            TuneEntry te;
            te.kernel = wide ? "k_m2l_wide" : "k_m2l_mfma";
            te.nb = pick.first >= 0 ? kWideNB[pick.first] : 0;
            te.shares = pick.second;
            te.ms = best;
            cache[key] = te;
            dirty = true;
            ++*n_tuned;
        }
    }
    t->prec = saved;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status == PFMM_OK && dirty && !tune_write(path, cache))
        return fail(PFMM_EINVAL, std::string("cannot write the autotune cache ") + path);
    return status;
}

void fill_stats(const Plan& P, uint64_t bytes, pfmm_stats* out, int m2l_mfma) {
    out->depth = P.depth;
    out->n_levels_far = P.depth >= 2 ? P.depth - 1 : 0;
    out->boxes = P.n_boxes;
    out->leaves = P.n_leaves;
    out->near_entries = P.near_entries;
    out->m2l_pairs = P.m2l_pairs;
    out->near_row_groups = (int64_t)P.rows.size();
    out->distinct_integrals = P.distinct;
    out->device_bytes = bytes;
    out->m2l_matrix_cores = m2l_mfma;
    out->near_gemm_groups = m2l_mfma < 0 ? -1 : 0;   // set by the caller once decided
    out->n_time_classes = P.max_time_classes;
    out->near_entries_V = 0;                          // set by the caller for a built tree
    out->near_entries_K = 0;
    out->near_nonzero_K = P.near_nonzero_K;
    out->near_entries_K1 = P.p1.built ? P.p1.near_entries : 0;
}

}  // namespace

// ====================================================================== internal accessors

namespace pfmm {

pfmm_status set_error(pfmm_status s, const std::string& msg) { return fail(s, msg); }
int tree_device(const pfmm_tree* t) { return t->device; }
int64_t tree_dofs(const pfmm_tree* t) { return (int64_t)t->P.E_t * t->P.E_x; }
int64_t tree_triangles(const pfmm_tree* t) { return t->P.E_x; }
bool tree_profiling(const pfmm_tree* t) { return t->prof; }
int tree_precision(const pfmm_tree* t) { return t->prec; }
const int* tree_sigma(const pfmm_tree* t) { return t->sigma; }
const int* tree_inv_sigma(const pfmm_tree* t) { return t->inv_sigma; }
const int* tree_adjacency(const pfmm_tree* t) { return t->adj; }

pfmm_status tree_near_diag(pfmm_tree* t, double* d_dev, hipStream_t st) {
    if (!t->hasV) return fail(PFMM_EINVAL, "V_h was not built for this tree");
    if (!t->P.uniform_steps)
        return fail(PFMM_EUNSUPPORTED, "the learned preconditioner needs uniform time steps");
    const int nl = (int)t->P.leaves.size();
    hipLaunchKernelGGL(k_near_diag, dim3((unsigned)((nl + 3) / 4)), dim3(256), 0, st, t->opV.table, t->groups,
                       t->umap, t->nl, (int)t->P.leaves.size(), t->inv_sigma, d_dev);
    HIP_TRY(hipGetLastError());
    return PFMM_OK;
}
bool tree_has(const pfmm_tree* t, int op) {
    return op == PFMM_OP_V ? t->hasV : (op == PFMM_OP_K ? t->hasK : (op == PFMM_OP_K1 ? t->hasK1 : false));
}
const double* tree_area(const pfmm_tree* t) { return t->mass; }
const double* tree_steps(const pfmm_tree* t) { return t->hstep; }
bool tree_uniform_steps(const pfmm_tree* t) { return t->P.uniform_steps; }
pfmm_status tree_apply(pfmm_tree* t, bool K, const double* x, double* y, hipStream_t st) { return apply(t, K, x, y, st); }
pfmm_status tree_apply_p1(pfmm_tree* t, const double* x, double* y, hipStream_t st) { return apply(t, 2, x, y, st); }
int tree_vertices(const pfmm_tree* t) { return t->n_verts; }
const int* tree_tris(const pfmm_tree* t) { return t->geom.tris; }
pfmm_status tree_apply_phase(pfmm_tree* t, bool K, const double* x, double* y, hipStream_t st, int phase) {
    return apply(t, K, x, y, st, phase);
}

// ---------------------------------------------------------------- cross-problem M2L
struct BatchM2L {
    int device = 0;
    std::vector<pfmm_tree*> trees;
    ClsUnit* dev = nullptr;       // units grouped by (precision, time offset)
    int cap = 0;
    struct Seg { int q, D, off, n, wg; const pfmm_tree* ref; };
    std::vector<Seg> segs;
};

pfmm_status batch_m2l_create(pfmm_tree* const* trees, int n, BatchM2L** out) {
    *out = nullptr;
    int units = 0;
    for (int i = 0; i < n; ++i) {
        const pfmm_tree* t = trees[i];
        // one launch needs one row-group plan: the same degrees on the matrix-core path
        if (!t->mfma_slots || t->P.m_t != trees[0]->P.m_t || t->P.m_x != trees[0]->P.m_x) return PFMM_OK;
        for (int l = 2; l <= t->P.depth && t->P.has_far; ++l)
            if (!t->lv[l].uniform) units += 2;
    }
    if (units == 0) return PFMM_OK;   // nothing to batch: every level has equal intervals
    BatchM2L* b = new (std::nothrow) BatchM2L();
    if (!b) return fail(PFMM_ENOMEM, "host allocation failed");
    b->device = trees[0]->device;
    b->trees.assign(trees, trees + n);
    b->cap = units;
    if (hipMalloc(&b->dev, (size_t)units * sizeof(ClsUnit)) != hipSuccess) {
        delete b;
        return fail(PFMM_ENOMEM, "hipMalloc failed for the batched M2L units");
    }
    *out = b;
    return PFMM_OK;
}

pfmm_status batch_m2l_prepare(BatchM2L* b) {
    std::vector<ClsUnit> host;
    b->segs.clear();
    for (int q = 0; q < 3; ++q)
        for (int D = 2; D <= 3; ++D) {
            BatchM2L::Seg sg{q, D, (int)host.size(), 0, 0, nullptr};
            for (pfmm_tree* t : b->trees) {
                if (cls_q(t) != q || !t->P.has_far) continue;
                for (int l = 2; l <= t->P.depth; ++l) {
                    const DevLevel& Dl = t->lv[l];
                    if (Dl.uniform || Dl.nccb[D - 2] == 0) continue;
                    if (!t->wcls[q].ok) return fail(PFMM_EDEVICE, "internal: class-aware M2L plan missing");
                    if (!sg.ref) sg.ref = t;
                    ClsUnit U = cls_unit(t, l, D, q);
                    U.wg0 = sg.wg;
                    sg.wg += t->wcls[q].G * U.ntg * U.nccb;
                    host.push_back(U);
                    ++sg.n;
                }
            }
            if (sg.n) b->segs.push_back(sg);
        }
    if ((int)host.size() > b->cap) return fail(PFMM_EINVAL, "internal: batched M2L units exceed their buffer");
    if (!host.empty())
        HIP_TRY(hipMemcpy(b->dev, host.data(), host.size() * sizeof(ClsUnit), hipMemcpyHostToDevice));
    return PFMM_OK;
}

pfmm_status batch_m2l_launch(BatchM2L* b, hipStream_t st) {
    for (const auto& sg : b->segs) {
        const pfmm_tree* r = sg.ref;
        const auto& W = r->wcls[sg.q];
        cls_batch_launcher(sg.q)((unsigned)sg.wg, W.shm, st, b->dev + sg.off, sg.n, W.G, sg.q ? r->TSc32 : r->TSc64,
                                 r->packinfo, W.plan, W.stride, r->P.Nc, r->P.m_t, r->P.m_x);
    }
    HIP_TRY(hipGetLastError());
    return PFMM_OK;
}

void batch_m2l_destroy(BatchM2L* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->dev) (void)hipFree(b->dev);
    delete b;
}
pfmm_status tree_geometry(pfmm_tree* t, TreeGeom* out) {
    PF_TRY(upload_geometry(t));
    out->verts = t->geom.verts;
    out->tris = t->geom.tris;
    out->area = t->geom.area;
    out->normal = t->geom.normal;
    out->tnodes = t->tnodes_dev;
    out->n_tri = t->P.E_x;
    out->n_steps = t->P.E_t;
    out->alpha = t->P.alpha;
    out->t_first = t->P.tnodes.front();
    out->t_last = t->P.tnodes.back();
    return PFMM_OK;
}

}  // namespace pfmm

// ====================================================================== C ABI

extern "C" {

pfmm_status pfmm_default_params(pfmm_params* out) {
    if (!out) return fail(PFMM_EINVAL, "NULL params");
    std::memset(out, 0, sizeof(*out));
    out->alpha = 1.0;
    out->m_t = 6;
    out->m_x = 6;
    out->n_max = 64;
    out->c_st = 0.9;
    out->n_tr = 5;
    out->q_reg = 4;
    out->q_sing = 5;
    out->precision = PFMM_FP64;
    out->operators = PFMM_OP_V | PFMM_OP_K;
    out->check_finite = 1;
    out->nearfield_gemm = 1;
    out->device_mem_budget = 0;
    return PFMM_OK;
}

pfmm_status pfmm_plan_stats(const double* vertices, int64_t n_vertices, const int32_t* triangles, int64_t n_triangles,
                            const double* time_nodes, int64_t n_steps, const pfmm_params* p, pfmm_stats* out) {
    if (!out) return fail(PFMM_EINVAL, "NULL stats");
    pfmm_params prm;
    if (p) prm = *p; else pfmm_default_params(&prm);
    try {
        Plan P;
        std::string msg;
        pfmm_status s = build_plan(vertices, n_vertices, triangles, n_triangles, time_nodes, n_steps, prm, P, msg);
        if (s != PFMM_OK) return fail(s, msg);
        FarTables F;
        const bool p1 = (prm.operators & PFMM_OP_K1) != 0;
        build_far_tables(P, F, p1);
        if (p1) build_p1_layout(P);
        fill_stats(P, estimate_bytes(P, F, prm.operators, prm.precision, prm.nearfield_mode), out, -1);
    } catch (const std::bad_alloc&) {
        return fail(PFMM_ENOMEM, "host allocation failed while planning");
    } catch (const std::exception& e) {
        return fail(PFMM_EINVAL, e.what());
    }
    return PFMM_OK;
}

pfmm_status pfmm_build_tree(const double* vertices, int64_t n_vertices, const int32_t* triangles, int64_t n_triangles,
                            const double* time_nodes, int64_t n_steps, const pfmm_params* p, int32_t device,
                            void* stream, pfmm_tree** out) {
    if (!out) return fail(PFMM_EINVAL, "NULL output pointer");
    *out = nullptr;
    pfmm_params prm;
    if (p) prm = *p; else pfmm_default_params(&prm);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(PFMM_EDEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(PFMM_EINVAL, "device ordinal out of range");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(PFMM_EDEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    HIP_TRY(hipSetDevice(device));
    std::unique_ptr<pfmm_tree> t(new (std::nothrow) pfmm_tree());
    if (!t) return fail(PFMM_ENOMEM, "host allocation failed");
    t->device = device;
    try {
        std::string msg;
        pfmm_status s = build_plan(vertices, n_vertices, triangles, n_triangles, time_nodes, n_steps, prm, t->P, msg);
        if (s != PFMM_OK) return fail(s, msg);
        const bool p1 = (prm.operators & PFMM_OP_K1) != 0;
        build_far_tables(t->P, t->F, p1);
        if (p1) build_p1_layout(t->P);
        t->n_verts = t->P.n_vert;
    } catch (const std::bad_alloc&) {
        return fail(PFMM_ENOMEM, "host allocation failed while planning");
    }
    if (t->P.Nc > 2048) return fail(PFMM_EUNSUPPORTED, "(m_t+1) * C(m_x+3,3) must be <= 2048");
    const uint64_t need = estimate_bytes(t->P, t->F, prm.operators, prm.precision, prm.nearfield_mode);
    size_t fr = 0, tot = 0;
    HIP_TRY(hipMemGetInfo(&fr, &tot));
    const uint64_t budget = prm.device_mem_budget ? prm.device_mem_budget : (uint64_t)(0.9 * (double)fr);
    if (need > budget)
        return fail(PFMM_ENOMEM, "tree needs " + std::to_string(need) + " device bytes, budget " + std::to_string(budget));
    hipStream_t st = as_stream(stream);
    t->prec = prm.precision;
    t->has_f32 = prm.precision == PFMM_MIXED_FP32 || prm.precision == PFMM_MIXED_BF16;
    t->nf_mode = prm.nearfield_mode;
    t->nf_gemm = prm.nearfield_gemm;
    pfmm_status s = setup_device(t.get(), st, prm.operators);
    if (s != PFMM_OK) {
        pfmm_destroy(t.release());
        return s;
    }
    *out = t.release();
    return PFMM_OK;
}

pfmm_status pfmm_apply_V(pfmm_tree* t, const double* w_dev, double* f_dev, void* stream) {
    if (!t || !w_dev || !f_dev) return fail(PFMM_EINVAL, "NULL argument");
    if (!t->hasV) return fail(PFMM_EINVAL, "V_h was not built for this tree");
    if (hipSetDevice(t->device) != hipSuccess) return fail(PFMM_EDEVICE, "hipSetDevice failed");
    return apply(t, false, w_dev, f_dev, as_stream(stream));
}

pfmm_status pfmm_apply_K(pfmm_tree* t, const double* u_dev, double* f_dev, void* stream) {
    if (!t || !u_dev || !f_dev) return fail(PFMM_EINVAL, "NULL argument");
    if (!t->hasK) return fail(PFMM_EINVAL, "K_h was not built for this tree");
    if (hipSetDevice(t->device) != hipSuccess) return fail(PFMM_EDEVICE, "hipSetDevice failed");
    return apply(t, true, u_dev, f_dev, as_stream(stream));
}

pfmm_status pfmm_apply_K1(pfmm_tree* t, const double* u_dev, double* f_dev, void* stream) {
    if (!t || !u_dev || !f_dev) return fail(PFMM_EINVAL, "NULL argument");
    if (!t->hasK1) return fail(PFMM_EINVAL, "the p1 double layer was not built for this tree");
    if (hipSetDevice(t->device) != hipSuccess) return fail(PFMM_EDEVICE, "hipSetDevice failed");
    return apply(t, 2, u_dev, f_dev, as_stream(stream));
}

pfmm_status pfmm_set_precision(pfmm_tree* t, int32_t precision) {
    if (!t) return fail(PFMM_EINVAL, "NULL tree");
    if (precision == PFMM_FP64) { t->prec = PFMM_FP64; return PFMM_OK; }
    if (precision == PFMM_MIXED_FP32 || precision == PFMM_MIXED_BF16) {
        if (!t->has_f32) return fail(PFMM_EINVAL, "tree was not built in a mixed precision");
        t->prec = precision;
        return PFMM_OK;
    }
    return fail(PFMM_EINVAL, "unknown precision");
}

pfmm_status pfmm_autotune(pfmm_tree* t, const char* cache_path, void* stream, int32_t* n_tuned, int32_t* n_cached) {
    if (!t) return fail(PFMM_EINVAL, "NULL tree");
    if (t->prof) return fail(PFMM_EINVAL, "stage profiling is on");
    if (hipSetDevice(t->device) != hipSuccess) return fail(PFMM_EDEVICE, "hipSetDevice failed");
    int a = 0, b = 0;
    const pfmm_status s = autotune(t, cache_path, as_stream(stream), &a, &b);
    if (n_tuned) *n_tuned = a;
    if (n_cached) *n_cached = b;
    return s;
}

pfmm_status pfmm_tree_stats(const pfmm_tree* t, pfmm_stats* out) {
    if (!t || !out) return fail(PFMM_EINVAL, "NULL argument");
    fill_stats(t->P, t->bytes, out, t->mfma_slots > 0 ? 1 : 0);
    out->near_gemm_groups = t->ngg_start[4];
    const bool stored = t->nf_mode == PFMM_NF_STORED;
    out->near_entries_V = t->hasV && stored ? t->P.near_entries : 0;
    out->near_entries_K = t->hasK && stored ? t->P.near_entries : 0;
    out->near_entries_K1 = t->hasK1 ? t->P.p1.near_entries : 0;
    return PFMM_OK;
}

pfmm_status pfmm_profile_enable(pfmm_tree* t, int32_t enable) {
    if (!t) return fail(PFMM_EINVAL, "NULL tree");
    t->prof = enable != 0;
    return PFMM_OK;
}

pfmm_status pfmm_profile_read(pfmm_tree* t, double* ms, int64_t* counts, int32_t* n_stages) {
    if (!t) return fail(PFMM_EINVAL, "NULL tree");
    for (auto& u : t->ev_used) {
        const int stage = u.first, i = u.second;
        if (hipEventSynchronize(t->ev[i + 1]) != hipSuccess) return fail(PFMM_EDEVICE, "event synchronize failed");
        float m = 0.f;
        if (hipEventElapsedTime(&m, t->ev[i], t->ev[i + 1]) == hipSuccess) {
            t->prof_ms[stage] += m;
            t->prof_cnt[stage] += 1;
        }
    }
    for (hipEvent_t e : t->ev) (void)hipEventDestroy(e);
    t->ev.clear();
    t->ev_used.clear();
    for (int s = 0; s < 8; ++s) {
        if (ms) ms[s] = t->prof_ms[s];
        if (counts) counts[s] = t->prof_cnt[s];
        t->prof_ms[s] = 0;
        t->prof_cnt[s] = 0;
    }
    if (n_stages) *n_stages = 8;
    return PFMM_OK;
}

void pfmm_destroy(pfmm_tree* t) {
    if (!t) return;
    (void)hipSetDevice(t->device);
    for (hipEvent_t e : t->ev) (void)hipEventDestroy(e);
    if (t->side) {
        (void)hipStreamSynchronize(t->side);
        (void)hipStreamDestroy(t->side);
    }
    for (hipEvent_t e : {t->ev_fork, t->ev_join})
        if (e) (void)hipEventDestroy(e);
    for (void* p : t->allocs) (void)hipFree(p);
    delete t;
}

const char* pfmm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
