// Stored-block nearfield product of the space-time FMM (Section 3.4, the
// nearfield part of Algorithm 2).  Included by pfmm.hip inside its anonymous
// namespace; relies on kWave and NearLayout declared there.
#pragma once

// Nearfield product f[kt, rows] += B * w over the causal columns.  One wave
// per row group; lane = (column slot cs, row r), cpi = 64 / nX column slots;
// partial sums reduced in LDS.  The source densities of a rectangle's columns
// are gathered into LDS CH = 4 cpi floor(64 / cpi) <= 256 columns at a time
// (one gather per column instead of one per column and lane group), so the
// vector memory path carries the block stream and little else.  When the
// workgroup's four row groups are steps of one leaf (consecutive in the row
// list), the workgroup stages each chunk once for all four (the longest
// row's columns); otherwise every wave stages its own.  A lane's columns run
// in trips of four (cs + 4 cpi t + u cpi); a trip never straddles a chunk,
// and the fma order per lane is the trip order either way.
__global__ void __launch_bounds__(256) k_near_apply(const double* __restrict__ B, const double* __restrict__ wd,
                                                    double* __restrict__ fd, NearLayout L) {
    __shared__ double red[256];
    __shared__ double xsh[256 / kWave][256];
    const int wv = threadIdx.x / kWave;
    const int64_t rg0 = (int64_t)blockIdx.x * (blockDim.x / kWave);
    const int64_t rg = rg0 + wv;
    const int lane = threadIdx.x % kWave;
    double acc = 0.0;
    int nX = 1, cpi = 64, r = 0, cs = 0, kt = 0, t0 = 0;
    // one leaf for the whole workgroup?  (same answer in every thread)
    bool one_leaf = rg0 + 3 < L.n_rows;
    int ktmax = 0;
    if (one_leaf) {
        const int l0 = L.rg_leaf[rg0];
        for (int k = 1; k < 4; ++k) one_leaf = one_leaf && L.rg_leaf[rg0 + k] == l0;
        for (int k = 0; k < 4; ++k) ktmax = max(ktmax, L.rg_kt[rg0 + k]);
    }
    if (rg < L.n_rows) {   // uniform per wave (and per workgroup when one_leaf)
        const int leaf = L.rg_leaf[rg];
        kt = L.rg_kt[rg];
        nX = L.lf_nx[leaf];
        t0 = L.lf_tb[leaf];
        cpi = kWave / nX;
        cs = lane / nX;
        r = lane % nX;
        const int CH = 4 * cpi * (kWave / cpi);   // columns per chunk, a whole number of trips
        const bool act = cs < cpi;
        const double* blk = B + L.rg_boff[rg];
        double* xs = one_leaf ? xsh[0] : xsh[wv];
        int64_t colbase = 0;
        for (int q = L.lf_rect0[leaf]; q < L.lf_rect1[leaf]; ++q) {
            const int j0 = L.rc_j0[q];
            const int S = L.set_size[L.rc_set[q]];
            const int* pos = L.set_pos + L.set_off[L.rc_set[q]];
            const int ns = min(L.rc_j1[q], kt + 1) - j0;
            const int total = ns > 0 ? ns * S : 0;   // this row group's columns (at most E_t * E_x)
            // columns staged: this row group's, or the workgroup's longest
            const int nsm = one_leaf ? min(L.rc_j1[q], ktmax + 1) - j0 : ns;
            if (nsm <= 0) continue;
            const int tstage = nsm * S;
            for (int base = 0; base < tstage; base += CH) {
                if (one_leaf) {
                    __syncthreads();   // every wave is done with the previous chunk
                    const int c = base + (int)threadIdx.x;
                    if ((int)threadIdx.x < CH && c < tstage) {
                        const int d = c / S;   // column c = (source step j0 + d, triangle pos[c - d S])
                        xs[threadIdx.x] = wd[(int64_t)(j0 + d) * L.E_src + pos[c - d * S]];
                    }
                    __syncthreads();
                } else {
                    // the previous chunk's reads are done before the buffer is refilled
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int cl = lane + kWave * k;
                        const int c = base + cl;
                        if (cl < CH && c < tstage) {
                            const int d = c / S;
                            xs[cl] = wd[(int64_t)(j0 + d) * L.E_src + pos[c - d * S]];
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
                if (act && base < total) {
                    // four columns per trip with independent loads; the block
                    // stream is read once (non-temporal)
                    const int cend = min(total, base + CH);
                    for (int c = base + cs; c < cend; c += 4 * cpi) {
                        double bv[4], xv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int cc = c + u * cpi;
                            const bool ok = cc < total;
                            bv[u] = __builtin_nontemporal_load(&blk[(colbase + (ok ? cc : cs)) * nX + r]);
                            xv[u] = ok ? xs[cc - base] : 0.0;
                            bv[u] = ok ? bv[u] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) acc = fma(bv[u], xv[u], acc);
                    }
                }
            }
            colbase += total;
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
                                                   NearLayout L, const int* __restrict__ sel, int64_t n_sel) {
    __shared__ double red[256];
    const int wv = threadIdx.x / kWave;
    // row group: the idx-th of the selection sel[0, n_sel), or of all when sel is null
    const int64_t idx = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv;
    const int64_t rg = sel ? (idx < n_sel ? sel[idx] : L.n_rows) : idx;
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

// Toeplitz nearfield of one assembly group (leaf spatial box, rows r < nX)
// on the FP64 matrix cores.  The group's leaves are time translates: one per
// interval [s0, s0 + s) over all steps, and source triangle u (table column)
// contributes the steps jt in [s0 + a_u, s0 + b_u) clipped at 0, with
// (a_u, b_u) depending on the leaf index modulo a period `per` (checked on
// the host).  With k = d U + u over the time offsets d and the columns u,
//   f[kt][r] += sum_k A[kt][k] T[k][r],
//   A[kt][k] = w[kt - d][pos_u] if kt - d lies in that range, else 0,
//   T[k][r]  = the distinct-integral table T[d][u][r] as stored (row k of
//              length nX),
// a dense GEMM: a wave owns 16 target steps and NT 16-column tiles of rows,
// v_mfma_f64_16x16x4f64 with A[i][k] from lane i + 16 k and B[k][j] from
// lane j + 16 k; D[i][j] in lane j + 16 (i % 4), register i / 4.
struct NearGemmGroup {
    int64_t toff, eoff;       // table offset (doubles), offset into the per-column records [phase][u]
    int s, per, nX, U, K, tb; // interval length, period, rows, columns, K = (dmax + 1) U, first row position
};

// One workgroup per 16 target steps of a group; its 4 waves take
// consecutive quarters of the K range and their partial tiles are added
// through LDS in wave order (fixed order: deterministic results).  The
// group's per-column records are copied to LDS first when they fit
// (lds_records: capacity in records, 0 = read them from global memory).
template <int NT>
__global__ void __launch_bounds__(256) k_near_gemm(const double* __restrict__ table,
                                                   const NearGemmGroup* __restrict__ gg, const int4* __restrict__ ue,
                                                   const double* __restrict__ wd, double* __restrict__ fd, int E_x,
                                                   int E_t, int lds_records) {
    __shared__ double red[3][NT][4][kWave];
    extern __shared__ int4 srec[];
    const NearGemmGroup G = gg[blockIdx.x];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int li = lane & 15, lk = lane >> 4;
    const int kt0 = blockIdx.y * 16;
    const int kt = kt0 + li;
    const int s0 = (kt / G.s) * G.s;
    const double* T = table + G.toff;
    const int nrec = G.per * G.U;
    const int4* Eg = ue + G.eoff;
    const bool in_lds = nrec <= lds_records;   // uniform over the workgroup
    if (in_lds) {
        for (int i = threadIdx.x; i < nrec; i += blockDim.x) srec[i] = Eg[i];
        __syncthreads();
    }
    const int4* E = (in_lds ? srec : Eg) + ((kt / G.s) % G.per) * G.U;   // this target step's phase
    d4_t acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = d4_t{0.0, 0.0, 0.0, 0.0};
    const int kq = ((G.K + 15) / 16) * 4;                 // K values per wave, a multiple of 4
    const int kb = wv * kq, ke = min(G.K, kb + kq);
    // Operands are fetched kPF K-steps ahead into a register ring (the
    // density gather and the table row of a K-step do not depend on the
    // products), so kPF gathers per lane are in flight while the matrix
    // cores work; the products run in the same K order as without the ring.
    constexpr int kPF = 4;
    int d = (kb + lk) / G.U, u = (kb + lk) - ((kb + lk) / G.U) * G.U;   // (d, u) of the next fetch
    auto fetch = [&](int k, double& a, double* b) {
        a = 0.0;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) b[nt] = 0.0;
        if (k < ke) {
            const int4 e = E[u];   // (position, a_u, b_u)
            const int jt = kt - d;
            if (kt < E_t && jt >= 0 && jt >= s0 + e.y && jt < s0 + e.z) a = wd[(int64_t)jt * E_x + e.x];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int r = nt * 16 + li;
                if (r < G.nX) b[nt] = T[(int64_t)k * G.nX + r];
            }
        }
        u += 4;
        while (u >= G.U) {
            u -= G.U;
            ++d;
        }
    };
    double ra[kPF], rb[kPF][NT];
#pragma unroll
    for (int p = 0; p < kPF; ++p) fetch(kb + lk + 4 * p, ra[p], rb[p]);
    for (int k0 = kb; k0 < ke; k0 += 4 * kPF) {
#pragma unroll
        for (int p = 0; p < kPF; ++p) {
            if (k0 + 4 * p < ke)   // uniform over the wave
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[p], rb[p][nt], acc[nt], 0, 0, 0);
            fetch(k0 + 4 * (p + kPF) + lk, ra[p], rb[p]);
        }
    }
    if (wv > 0)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[wv - 1][nt][q][lane] = acc[nt][q];
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double v = acc[nt][q] + red[0][nt][q][lane] + red[1][nt][q][lane] + red[2][nt][q][lane];
            const int kk = kt0 + lk + 4 * q, r = nt * 16 + li;
            if (kk < E_t && r < G.nX) fd[(int64_t)kk * E_x + G.tb + r] += v;
        }
}
