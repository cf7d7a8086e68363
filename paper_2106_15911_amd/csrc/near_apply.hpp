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
// on the FP64 matrix cores.  The group's leaves cover all steps in order,
// leaf i the steps [s0_i, s0_{i+1}), and source triangle u (table column)
// contributes the steps jt in [s0_i + a_u, s0_i + b_u) clipped at 0, with
// (a_u, b_u) depending on the leaf index modulo a period `per` (checked on
// the host; per is the number of leaves when every leaf has its own
// ranges).  Leaves of one length s start at i s; otherwise their starts are
// read from a list.  Over the time offsets d and the columns u,
//   f[kt][r] += sum_{u, d} A[kt][(u, d)] T[d][u][r],
//   A[kt][(u, d)] = w[kt - d][pos_u] if kt - d lies in u's range, else 0,
// with T the distinct-integral table as stored (row d U + u of length nX):
// a dense GEMM with M = 16 target steps, N = the rows (NT 16-column tiles)
// and K = the (u, d) pairs, on v_mfma_f64_16x16x4f64 (A[i][k] from lane
// i + 16 k, B[k][j] from lane j + 16 k; D[i][j] in lane j + 16 (i % 4),
// register i / 4).  A K-step takes four consecutive columns u (one per lane
// row k) at one offset d, and the offsets of a column quad are consecutive
// K-steps: the A operand of offset d + 1 is that of offset d moved one target
// step on, w[kt - d - 1] = w[(kt - 1) - d], i.e. one lane along each 16-lane
// row.  A DPP row shift does that move; the value entering lane 0 of a row
// comes from a second register that holds the next 16 such values, so a
// column quad costs two density gathers per 16 offsets instead of one per
// offset.  The mask of a lane's own range is applied after the shift.
struct NearGemmGroup {
    int64_t toff, eoff;       // table offset (doubles), offset into the per-column records [phase][u]
    int64_t stoff;            // offset of the leaf starts (per + 1 of them) in the start list; -1: i s
    int s, per, nX, U, K, tb; // leaf length (when equal), period, rows, columns, K = (dmax + 1) U, first row position
};

// Move the two 32-bit halves of a double by the DPP pattern CTRL; lanes
// whose source lies outside their 16-lane row keep `old`.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double old, double src) {
    const int2 o = __builtin_bit_cast(int2, old), s = __builtin_bit_cast(int2, src);
    int2 r;
    r.x = __builtin_amdgcn_update_dpp(o.x, s.x, CTRL, 0xf, 0xf, false);
    r.y = __builtin_amdgcn_update_dpp(o.y, s.y, CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, r);
}
constexpr int kDppRowShr1 = 0x111;   // lane i of a row takes lane i - 1
constexpr int kDppRowShl1 = 0x101;   // lane i of a row takes lane i + 1
constexpr int kXcdsNear = 8;         // accelerator complex dies of an MI355X (one L2 each)

// Per-column source range (a_u, b_u) of one phase as two 16-bit fields.
__host__ __device__ inline int gemm_pack_range(int a, int b) {
    return (int)((unsigned)(a + 32768) | ((unsigned)(b + 32768) << 16));
}
// Dynamic LDS of k_near_gemm for a group of U columns that stages nlb record
// rows (the group's period, or the most leaves one 16-step block meets if
// fewer): the d range of every column quad (int2), the columns' density
// positions and their packed ranges.
inline int gemm_lds_bytes(int U, int nlb) { return 8 * ((U + 3) / 4) + 4 * U + 4 * nlb * U; }

// One workgroup per 16 target steps of a group.  The workgroup copies the
// records of the leaves its steps meet to LDS and finds, for each column quad, the offsets d at
// which any of its 16 target steps has a source in range (offsets outside
// are skipped, not multiplied by zero); then its 4 waves take consecutive
// quarters of the column quads, run their (quad, offset) K-steps in order,
// and add their partial tiles through LDS in wave order (fixed order:
// deterministic results).  Operands are fetched kPF K-steps ahead into a
// register ring.  Every fetch issues the same buffer loads (table row,
// density for a quad's first offset, next 16 lane-0 values); a load that a
// K-step does not need gets an offset past the buffer's end, which returns
// zero without a memory access, so the number of loads in flight is the same
// on every path and the waits can count them.
template <int NT>
__global__ void __launch_bounds__(256) k_near_gemm(const double* __restrict__ table,
                                                   const NearGemmGroup* __restrict__ gg, const int* __restrict__ ue,
                                                   const int* __restrict__ lst, const double* __restrict__ wd,
                                                   double* __restrict__ fd, int E_x, int E_t) {
    __shared__ double red[3][NT][4][kWave];
    extern __shared__ int2 rng[];   // [quads], then positions [U], then packed ranges [block leaves][U]
    // Workgroups are dealt to the 8 XCDs round-robin by linear id; remap so
    // that XCD x runs all step blocks of group x, then of group x + 8, ...:
    // a group's table stays in that XCD's L2 while its blocks run, and
    // neighbouring groups (similar costs) go to different XCDs.
    int gi, bi;
    {
        const int ng = gridDim.x, nb = gridDim.y;
        const int lin = blockIdx.x + ng * blockIdx.y;
        const int full = (ng / kXcdsNear) * kXcdsNear * nb;
        if (lin < full) {
            const int k = lin / kXcdsNear;
            gi = (k / nb) * kXcdsNear + lin % kXcdsNear;
            bi = k % nb;
        } else {   // the last ng mod 8 groups, in order
            gi = (ng / kXcdsNear) * kXcdsNear + (lin - full) / nb;
            bi = (lin - full) % nb;
        }
    }
    const NearGemmGroup G = gg[gi];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
    const int li = lane & 15, lk = lane >> 4;
    const int kt0 = bi * 16;
    const int kt = kt0 + li;
    const int U = G.U, nX = G.nX;
    const int nq = (U + 3) / 4;
    const int dmax = G.K / U - 1;
    const int* ls = G.stoff >= 0 ? lst + G.stoff : nullptr;
    // leaf of step k (k < E_t) and start of leaf i (i <= number of leaves)
    auto leaf_of = [&](int k) {
        if (!ls) return k / G.s;
        int a = 0, b = G.per - 1;   // per = number of leaves here
        while (a < b) {
            const int m = (a + b + 1) / 2;
            if (ls[m] <= k) a = m; else b = m - 1;
        }
        return a;
    };
    auto start_of = [&](int i) { return ls ? ls[i] : i * G.s; };
    const int kend = min(kt0 + 16, E_t);
    const int li0 = leaf_of(kt0), nlb = leaf_of(kend - 1) - li0 + 1;
    // staged records: one set per phase when the period is no longer than
    // the run of leaves the block meets, else one per leaf of the run
    const bool by_phase = G.per <= nlb;   // uniform over the workgroup
    const int nrow = by_phase ? G.per : nlb;
    auto row_of = [&](int lf) { return by_phase ? lf % G.per : lf - li0; };
    int* spos = (int*)(rng + nq);
    int* srec = spos + U;   // [row][u]
    const int* Eg = ue + G.eoff;
    for (int i = threadIdx.x; i < U; i += blockDim.x) spos[i] = Eg[i];
    for (int i = threadIdx.x; i < nrow * U; i += blockDim.x) {
        const int r = i / U;
        srec[i] = Eg[U + (by_phase ? r : (li0 + r) % G.per) * U + (i - r * U)];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
        // union over the quad's columns and the block's target steps of the
        // offsets d with kt - d in range: per leaf met by the block,
        // [first target - last source, last target - first source]
        int lo = INT32_MAX, hi = -1;
        for (int u = 4 * q; u < min(4 * q + 4, U); ++u) {
            for (int k = kt0, lf = li0; k < kend; ++lf) {
                const int s0 = start_of(lf);
                const int kl = min(kend, start_of(lf + 1)) - 1;
                const int e = srec[row_of(lf) * U + u];
                const int jlo = max(0, s0 + (e & 0xffff) - 32768), jhi = s0 + (int)((unsigned)e >> 16) - 32768;
                const int dl = max(0, k - jhi + 1), dh = kl - jlo;
                if (jlo < jhi && dl <= dh) {
                    lo = min(lo, dl);
                    hi = max(hi, dh);
                }
                k = kl + 1;
            }
        }
        rng[q] = lo <= hi ? int2{lo, hi} : int2{1, 0};
    }
    __syncthreads();
    const int lfk = leaf_of(min(kt, E_t - 1));        // this target step's leaf (lanes past E_t: masked)
    const int s0k = start_of(lfk);
    const int* rec = srec + row_of(lfk) * U;
    // buffers: the group's table, and the density rows the workgroup can read
    // (offsets up to dmax + 16 steps back from its first target step)
    constexpr int kOut = 0x7ffffff8;   // past the end of either buffer: loads return zero
    const int r0 = max(0, kt0 - 16 - dmax), r1 = kend;
    const __amdgpu_buffer_rsrc_t rsT = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(table + G.toff), (short)0, G.K * nX * (int)sizeof(double), 0x00020000);
    const __amdgpu_buffer_rsrc_t rsW = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(wd + (int64_t)r0 * E_x), (short)0, (r1 - r0) * E_x * (int)sizeof(double), 0x00020000);
    auto bload = [](__amdgpu_buffer_rsrc_t rs, int off) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
    };
    const int qpw = (nq + 3) / 4;
    const int qb = wv * qpw, qe = min(nq, qb + qpw);
    int nsteps = 0;
    for (int q = qb; q < qe; ++q) {
        const int2 r = rng[q];
        nsteps += max(0, __builtin_amdgcn_readfirstlane(r.y) - __builtin_amdgcn_readfirstlane(r.x) + 1);
    }
    // (quad, offset) cursors: the fetch runs kPF K-steps ahead of the products
    struct Cursor {
        int q, d, lo, hi;
    };
    auto seek = [&](Cursor& c) {   // from quad c.q on, the first quad with offsets
        for (; c.q < qe; ++c.q) {
            const int2 r = rng[c.q];
            c.lo = __builtin_amdgcn_readfirstlane(r.x);
            c.hi = __builtin_amdgcn_readfirstlane(r.y);
            if (c.lo <= c.hi) break;
        }
        c.d = c.lo;
    };
    auto advance = [&](Cursor& c) {
        if (++c.d > c.hi) {
            ++c.q;
            seek(c);
        }
    };
    constexpr int kPF = 4;
    struct Slot {
        double a, q, b[NT];   // A at a quad's first offset; the next 16 lane-0 values; table row values
        int jlo, wid;         // this lane's source range [jlo, jlo + wid) for the quad's column
    };
    Slot ring[kPF];
    Cursor fc{qb, 0, 1, 0}, cc{qb, 0, 1, 0};
    seek(fc);
    seek(cc);
    int pos = 0;   // density position of the fetch cursor's column
    auto fetch = [&](Slot& S) {
        const bool live = fc.q < qe;   // uniform; past the wave's last K-step every load returns zero
        const int u = 4 * fc.q + lk;
        const bool uv = live && u < U;
        const int j = fc.d - fc.lo;    // uniform
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int r = nt * 16 + li;
            S.b[nt] = bload(rsT, (uv && r < nX) ? ((fc.d * U + u) * nX + r) * (int)sizeof(double) : kOut);
        }
        if (live && j == 0) {
            int jl = 0, wdt = 0;
            pos = 0;
            if (uv) {
                pos = spos[u];
                const int e = rec[u];
                if (kt < E_t) {
                    jl = max(0, s0k + (e & 0xffff) - 32768);
                    wdt = max(0, s0k + (int)((unsigned)e >> 16) - 32768 - jl);
                }
            }
            S.jlo = jl;
            S.wid = wdt;
        }
        const int ja = kt - fc.d, jq = kt0 - fc.d - 1 - li;
        const bool na = uv && j == 0 && ja >= r0 && ja < r1;
        const bool nq16 = uv && (j & 15) == 0 && jq >= r0 && jq < r1;
        S.a = bload(rsW, na ? ((ja - r0) * E_x + pos) * (int)sizeof(double) : kOut);
        S.q = bload(rsW, nq16 ? ((jq - r0) * E_x + pos) * (int)sizeof(double) : kOut);
        if (live) advance(fc);
    };
    d4_t acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = d4_t{0.0, 0.0, 0.0, 0.0};
    double A = 0.0, Q = 0.0;
    int jlo = 0, wid = 0;
    auto consume = [&](const Slot& S) {
        const int j = cc.d - cc.lo;   // uniform
        if (j == 0) {
            A = S.a;
            Q = S.q;
            jlo = S.jlo;
            wid = S.wid;
        } else {
            A = dpp_move<kDppRowShr1>(Q, A);
            Q = (j & 15) == 0 ? S.q : dpp_move<kDppRowShl1>(Q, Q);
        }
        const double am = (unsigned)(kt - cc.d - jlo) < (unsigned)wid ? A : 0.0;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(am, S.b[nt], acc[nt], 0, 0, 0);
        advance(cc);
    };
#pragma unroll
    for (int p = 0; p < kPF; ++p) fetch(ring[p]);
    int n0 = 0;
    for (; n0 + kPF <= nsteps; n0 += kPF) {
#pragma unroll
        for (int p = 0; p < kPF; ++p) {
            consume(ring[p]);
            fetch(ring[p]);
        }
    }
#pragma unroll
    for (int p = 0; p < kPF; ++p)
        if (n0 + p < nsteps) consume(ring[p]);   // uniform over the wave
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
            if (kk < E_t && r < nX) fd[(int64_t)kk * E_x + G.tb + r] += v;
        }
}
