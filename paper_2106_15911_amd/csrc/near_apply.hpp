// Stored-block nearfield product of the space-time FMM (Section 3.4, the
// nearfield part of Algorithm 2).  Included by pfmm.hip inside its anonymous
// namespace; relies on kWave and NearLayout declared there.
#pragma once

// Nearfield product f[kt, rows] += B * w over the causal columns.  One wave
// per row group; lane = (column slot, row); partial sums reduced in LDS.
__global__ void __launch_bounds__(256) k_near_apply(const double* __restrict__ B, const double* __restrict__ wd,
                                                    double* __restrict__ fd, NearLayout L) {
    __shared__ double red[256];
    const int wv = threadIdx.x / kWave;
    const int64_t rg = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv;
    const int lane = threadIdx.x % kWave;
    double acc = 0.0;
    int nX = 1, cpi = 64, r = 0, cs = 0, kt = 0, t0 = 0;
    if (rg < L.n_rows) {
        const int leaf = L.rg_leaf[rg];
        kt = L.rg_kt[rg];
        nX = L.lf_nx[leaf];
        t0 = L.lf_tb[leaf];
        cpi = kWave / nX;
        cs = lane / nX;
        r = lane % nX;
        if (cs < cpi) {
            const double* blk = B + L.rg_boff[rg];
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
                // four columns per trip with independent loads; the block stream
                // is read once (non-temporal), the densities stay in L2
                for (int64_t c = cs; c < total; c += 4 * cpi) {
                    double bv[4], xv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t cc = c + u * cpi;
                        const bool ok = cc < total;
                        const int64_t ce = ok ? cc : cs;
                        bv[u] = __builtin_nontemporal_load(&blk[(colbase + ce) * nX + r]);
                        xv[u] = wd[(int64_t)(ok ? jt : j0) * L.E_x + pos[ok ? i : 0]];
                        bv[u] = ok ? bv[u] : 0.0;
                        i += cpi;
                        while (i >= S) { i -= S; ++jt; }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc = fma(bv[u], xv[u], acc);
                }
                colbase += total;
            }
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (rg < L.n_rows && lane < nX) {
        double s = 0.0;
        for (int c = 0; c < cpi; ++c) s += red[wv * kWave + c * nX + lane];
        fd[(int64_t)kt * L.E_x + t0 + lane] += s;
    }
}

// Nearfield product without stored blocks, for uniform time steps: the block
// entry of target row r, target step kt and source (jt, triangle) depends on
// the triangles and d = kt - jt only (the time integrals of eq.
// eval_sl_nf_block see the steps through their difference), so every entry
// is read from the leaf group's distinct-integral table T[d][u][r] (rows
// innermost: the rows of one column are contiguous).  ru holds, per leaf
// rectangle, the table column u of each of its source triangles.  Same
// thread layout and summation order per lane as k_near_apply; the tables of
// one group are reused by all its row groups (consecutive in launch order).
__global__ void __launch_bounds__(256) k_near_toep(const double* __restrict__ table, const GroupDev* __restrict__ groups,
                                                   const int64_t* __restrict__ ru_off, const int* __restrict__ ru,
                                                   const double* __restrict__ wd, double* __restrict__ fd,
                                                   NearLayout L) {
    __shared__ double red[256];
    const int wv = threadIdx.x / kWave;
    const int64_t rg = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv;
    const int lane = threadIdx.x % kWave;
    double acc = 0.0;
    int nX = 1, cpi = 64, r = 0, cs = 0, kt = 0, t0 = 0;
    if (rg < L.n_rows) {
        const int leaf = L.rg_leaf[rg];
        kt = L.rg_kt[rg];
        nX = L.lf_nx[leaf];
        t0 = L.lf_tb[leaf];
        cpi = kWave / nX;
        cs = lane / nX;
        r = lane % nX;
        if (cs < cpi) {
            const GroupDev gr = groups[L.lf_group[leaf]];
            const double* T = table + gr.toff + r;
            const int64_t dstride = (int64_t)gr.usize * nX;
            for (int q = L.lf_rect0[leaf]; q < L.lf_rect1[leaf]; ++q) {
                const int j0 = L.rc_j0[q];
                const int ns = min(L.rc_j1[q], kt + 1) - j0;
                if (ns <= 0) continue;
                const int S = L.set_size[L.rc_set[q]];
                const int* pos = L.set_pos + L.set_off[L.rc_set[q]];
                const int* uq = ru + ru_off[q];
                const int64_t total = (int64_t)ns * S;
                int jt = j0, i = cs;
                while (i >= S) { i -= S; ++jt; }
                for (int64_t c = cs; c < total; c += 4 * cpi) {
                    double bv[4], xv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool ok = c + u * cpi < total;
                        const int jj = ok ? jt : j0, ii = ok ? i : 0;
                        bv[u] = T[(int64_t)(kt - jj) * dstride + (int64_t)uq[ii] * nX];
                        xv[u] = wd[(int64_t)jj * L.E_x + pos[ii]];
                        bv[u] = ok ? bv[u] : 0.0;
                        i += cpi;
                        while (i >= S) { i -= S; ++jt; }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc = fma(bv[u], xv[u], acc);
                }
            }
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (rg < L.n_rows && lane < nX) {
        double s = 0.0;
        for (int c = 0; c < cpi; ++c) s += red[wv * kWave + c * nX + lane];
        fd[(int64_t)kt * L.E_x + t0 + lane] += s;
    }
}
