// Matrix-core M2L kernels of the space-time FMM (eq. m2l with the
// coefficients of eqs. exp_coeffs_3d / exp_coeffs_1d) and their launch
// helpers.  Included by pfmm.hip inside its anonymous namespace; relies on
// kWave and the HIP runtime declared there.
#pragma once

// M2L on FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// A workgroup owns the locals of one target slot X for 64 consecutive
// intervals k0..k0+63 (all rows of eq. m2l).  Waves 0-3 take intervals
// k0..k0+31, waves 4-7 take k0+32..k0+63; within a half, the 16 even and the
// 16 odd intervals form two 16-column MFMA tiles, so the second source
// interval of odd targets (Delta = 3) costs no wasted columns.  The output
// rows (coefficient order: degree, time index, multi-index) are cut into
// 16-row tiles; tile t only needs the first tile_ks[t] 4-column K-steps
// (|kappa + nu| <= m_x), and the tiles are spread over the 4 waves of a
// half by their K-step counts (slot_tile, computed on the host).
// Operator tiles are generated on the fly from the 1D coefficient tables of
// eq. exp_coeffs_1d held in LDS: A = C_ab E_x E_y E_z.
// MFMA register layout (checked on gfx950): A[i][k] lane i+16k, B[k][j]
// lane j+16k, D[i][j] lane j+16(i%4), register i/4.
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int kM2LWaves = 16;   // waves per workgroup (one interval half)
constexpr int kXcds = 8;        // accelerator complex dies of an MI355X (one L2 each)
constexpr int kM2LSlots = 3;    // accumulator slots (row-tile segments) per wave

// Work split of one (X, interval half) output block.  Each 16-row tile's
// K-range (its staircase length) is cut at multiples of a target length;
// every wave owns up to kM2LSlots segments that start at the same K-step
// (so they share the moment operands), sorted by length.  Segments after the
// first of a tile are partial sums, added to the first segment through LDS
// at the end.  wave_meta[w] = (K-step start, number of segments);
// seg[w][i] = (tile, length, partial index or -1); red_slot gives, for each
// partial segment, the owner wave and slot that adds it.
template <int MAXS>
__global__ void __launch_bounds__(64 * kM2LWaves) k_m2l_mfma(
    const double* __restrict__ mu, double* __restrict__ lam, const int* __restrict__ ptr, const int* __restrict__ src,
    const int* __restrict__ cls, const int* __restrict__ off3, const double* __restrict__ E1s, int TSp,
    const int* __restrict__ packinfo, const int* __restrict__ wave_meta,
    const int* __restrict__ seg, int n_partial, int Nc, int n_int, int mt, int mx, int R, int nsplit,
    int halves, double* __restrict__ lam_parts) {
    extern __shared__ double smem[];
    const int nt1 = mt + 1, nx1 = mx + 1;
    const int nx2 = nx1 * nx1;
    // two buffers of the three 1D tables of one (source, Delta) phase: [buf][x | y | z][TSp]
    int* sCol = (int*)(smem + 6 * TSp);          // per coefficient: table column offsets (x | y<<16), (z | deg<<16)
    const int lane = threadIdx.x % kWave;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // Workgroups are dealt to the 8 XCDs round-robin by linear id.  Remap so
    // that each XCD walks a contiguous range of target slots (Morton order):
    // concurrently running neighbours share most of their interaction lists,
    // so the source moments they stream stay in that XCD's L2.
    int bx, by, bz;
    {
        const int nxg = gridDim.x, nyg = gridDim.y;
        const int total = nxg * nyg * gridDim.z;
        const int lin = blockIdx.x + nxg * (blockIdx.y + nyg * blockIdx.z);
        const int per = total / kXcds;
        const int lm = lin < per * kXcds ? (lin % kXcds) * per + lin / kXcds : lin;
        bx = lm % nxg;
        by = (lm / nxg) % nyg;
        bz = lm / (nxg * nyg);
    }
    const int half = bz % halves;
    const int split = bz / halves;             // which share of the source list this workgroup takes
    const int X = bx;
    if (split > 0) lam = lam_parts + (int64_t)(split - 1) * ((int64_t)gridDim.x * Nc * n_int);
    const int lr = lane & 15, lq = lane >> 4;
    const int kE = by * 64 + 32 * half + 2 * lr;
    const int kO = kE + 1;
    for (int c = threadIdx.x; c < Nc; c += blockDim.x) {
        const int ci = packinfo[c];
        const int cb = (ci & 15) * nt1 * nx2;
        sCol[2 * c] = (cb + ((ci >> 4) & 15) * nx1) | ((cb + ((ci >> 8) & 15) * nx1) << 16);
        sCol[2 * c + 1] = (cb + ((ci >> 12) & 15) * nx1) | (((ci >> 16) & 255) << 16);
    }
    const int sbeg = __builtin_amdgcn_readfirstlane(wave_meta[2 * w]);
    int tiles[MAXS], ks[MAXS], part[MAXS], rX[MAXS], rY[MAXS], rZ[MAXS], rD[MAXS];
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        tiles[i] = __builtin_amdgcn_readfirstlane(seg[(w * MAXS + i) * 3]);
        ks[i] = __builtin_amdgcn_readfirstlane(seg[(w * MAXS + i) * 3 + 1]);   // segment end (exclusive, absolute)
        part[i] = __builtin_amdgcn_readfirstlane(seg[(w * MAXS + i) * 3 + 2]);
        const int row = 16 * (tiles[i] >= 0 ? tiles[i] : 0) + lr;
        const bool rv = tiles[i] >= 0 && row < Nc;
        const int ri = rv ? packinfo[row] : 0;
        const int b = ri & 15;
        rX[i] = b * nx2 + ((ri >> 4) & 15);
        rY[i] = b * nx2 + ((ri >> 8) & 15);
        rZ[i] = b * nx2 + ((ri >> 12) & 15);
        rD[i] = mx - (rv ? ((ri >> 16) & 255) : 255);   // largest column degree this row accepts
    }
    d4_t accE[MAXS], accO[MAXS];
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        accE[i] = d4_t{0.0, 0.0, 0.0, 0.0};
        accO[i] = d4_t{0.0, 0.0, 0.0, 0.0};
    }
    const int nR = 2 * R + 1;
    const int sb = ptr[X], se = ptr[X + 1];
    const int s_lo = sb + (int)(((int64_t)(se - sb) * split) / nsplit);
    const int s_hi = sb + (int)(((int64_t)(se - sb) * (split + 1)) / nsplit);
    // Phase p = (source s_lo + p/2, Delta = 2 + p%2).  Its tables are copied
    // global -> LDS asynchronously (no registers) one phase ahead, into the
    // buffer the previous phase has released; each wave copies 1 KB pieces.
    const int n_phase = 2 * (s_hi - s_lo);
    const int pieces = TSp / 128;                    // 1 KB pieces per table
    auto stage = [&](int p) {
        const int si = s_lo + (p >> 1), D = 2 + (p & 1);
        const int c3 = cls[si];
        double* dst = smem + (p & 1) * 3 * TSp;
        for (int c = w; c < 3 * pieces; c += kM2LWaves) {
            const int tb = c / pieces, pc = c - tb * pieces;
            const int o = off3[3 * c3 + tb] + R;
            const double* g = E1s + (((int64_t)(D - 2) * nR + o) * 2 + (tb == 0 ? 0 : 1)) * TSp + pc * 128 + 2 * lane;
            __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)g,
                                             (void __attribute__((address_space(3)))*)(dst + tb * TSp + pc * 128),
                                             16, 0, 0);
        }
    };
    if (n_phase > 0) stage(0);
    for (int p = 0; p < n_phase; ++p) {
        const int si = s_lo + (p >> 1), D = 2 + (p & 1);
        const int Y = src[si];
        const double* muY = mu + (int64_t)Y * Nc * n_int;
        const double* sEx = smem + (p & 1) * 3 * TSp;
        const double* sEy = sEx + TSp;
        const double* sEz = sEx + 2 * TSp;
        __builtin_amdgcn_s_waitcnt(0);   // this wave's pieces of phase p have landed in LDS
        __syncthreads();                 // ... everyone's; and phase p-1 is done with the other buffer
        if (p + 1 < n_phase) stage(p + 1);
        {
            const bool vE = (D == 2) && (kE < n_int) && (kE >= D);
            const bool vO = (kO < n_int) && (kO >= D);
            if (D == 3 && !__any(vO)) continue;
            const int64_t oE = vE ? (kE - D) : 0, oO = vO ? (kO - D) : 0;
            const double mE = vE ? 1.0 : 0.0, mO = vO ? 1.0 : 0.0;
            int cxy0, czd0, cxy1, czd1;
            double e0, o0, e1, o1;
            auto fetch = [&](int step, int& cxy, int& czd, double& e, double& o) {
                const int cn = 4 * step + lq;
                const bool ok = cn < Nc;
                const int cc = ok ? cn : 0;
                cxy = sCol[2 * cc];
                czd = ok ? sCol[2 * cc + 1] : (sCol[2 * cc + 1] | (255 << 16));
                e = muY[(int64_t)cc * n_int + oE];
                o = muY[(int64_t)cc * n_int + oO];
            };
            // one K-step with n active slots, operands taken from (cxy, czd, e, o)
            auto step = [&](auto nc, int cxy, int czd, double e, double o) {
                constexpr int n = decltype(nc)::value;
                const int cdeg = czd >> 16;
                const double bE = e * mE, bO = o * mO;
                const int cX = cxy & 0xffff, cY = cxy >> 16, cZ = czd & 0xffff;
                double A[n];
#pragma unroll
                for (int i = 0; i < n; ++i) {
                    const double ex = sEx[cX + rX[i]];
                    const double ey = sEy[cY + rY[i]];
                    const double ez = sEz[cZ + rZ[i]];
                    const double msk = (cdeg <= rD[i]) ? 1.0 : 0.0;
                    A[i] = (ex * ey) * (ez * msk);
                }
#pragma unroll
                for (int i = 0; i < n; ++i) {
                    if (D == 2) accE[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[i], bE, accE[i], 0, 0, 0);
                    accO[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[i], bO, accO[i], 0, 0, 0);
                }
            };
            // two operand sets used alternately: the set consumed at step s is
            // refilled with step s+2, so a load has a full step of work to land
            fetch(sbeg, cxy0, czd0, e0, o0);
            fetch(sbeg + 1, cxy1, czd1, e1, o1);
            int s = sbeg;
            auto phase = [&](auto nc, int s_end) {
                for (; s + 1 < s_end; s += 2) {
                    {
                        const int a0 = cxy0, b0 = czd0;
                        const double f0 = e0, g0 = o0;
                        fetch(s + 2, cxy0, czd0, e0, o0);
                        step(nc, a0, b0, f0, g0);
                    }
                    {
                        const int a1 = cxy1, b1 = czd1;
                        const double f1 = e1, g1 = o1;
                        fetch(s + 3, cxy1, czd1, e1, o1);
                        step(nc, a1, b1, f1, g1);
                    }
                }
                if (s < s_end) {
                    const int a0 = cxy0, b0 = czd0;
                    const double f0 = e0, g0 = o0;
                    cxy0 = cxy1; czd0 = czd1; e0 = e1; o0 = o1;
                    fetch(s + 2, cxy1, czd1, e1, o1);
                    step(nc, a0, b0, f0, g0);
                    ++s;
                }
            };
            static_assert(MAXS == 3, "phase dispatch below is written for three slots");
            phase(std::integral_constant<int, 3>{}, ks[2]);
            phase(std::integral_constant<int, 2>{}, ks[1]);
            phase(std::integral_constant<int, 1>{}, ks[0]);
        }
    }
    // partial segments: park in LDS, owners add them in a fixed order
    __syncthreads();
    double* red = smem;   // [n_partial][8][64]
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        if (tiles[i] >= 0 && part[i] >= 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                red[((int64_t)part[i] * 8 + r) * kWave + lane] = accE[i][r];
                red[((int64_t)part[i] * 8 + 4 + r) * kWave + lane] = accO[i][r];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        if (tiles[i] < 0 || part[i] >= 0) continue;
        // add every partial segment of this tile (they follow in seg order)
        for (int q = 0; q < n_partial; ++q) {
            if (seg[(kM2LWaves * MAXS) * 3 + q] != tiles[i]) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                accE[i][r] += red[((int64_t)q * 8 + r) * kWave + lane];
                accO[i][r] += red[((int64_t)q * 8 + 4 + r) * kWave + lane];
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * tiles[i] + lq + 4 * r;
            if (row >= Nc) continue;
            if (kE < n_int) lam[((int64_t)X * Nc + row) * n_int + kE] = accE[i][r];
            if (kO < n_int) lam[((int64_t)X * Nc + row) * n_int + kO] = accO[i][r];
        }
    }
}

// M2L on matrix cores, wide form for levels with >= 32 intervals, in FP64
// (T = double, v_mfma_f64_16x16x4f64) or with FP32 moments and operator
// tables and FP32 accumulation (T = float, v_mfma_f32_16x16x4f32).  With
// RB = true (T = float) the moments and table entries are bfloat16 values and
// every generated operator entry is rounded to bfloat16 before its product:
// BF16 inputs with exact products and FP32 accumulation.
//
// The rows of eq. m2l (16-row tiles of the staircase) are partitioned into
// row groups; a workgroup of WAVES waves owns one target slot X, one row
// group and NB blocks of 32 consecutive intervals.  It walks X's interaction
// list one source slot Y at a time; both time offsets of the source
// (Delta = 2 for every target interval, Delta = 3 for the odd ones) are
// applied in the same phase, so each source moment is read once per
// workgroup.  An operator element a wave generates from the 1D tables feeds
// 2 NB products (Delta = 2, even and odd intervals of every block) or NB
// products (Delta = 3, odd intervals).  Within a group the tiles' K-ranges
// are cut into segments (up to MAXS per wave, sharing their first K-step);
// partial segments are added to their tile's first segment through LDS, one
// interval block at a time.
//
// The 1D coefficient tables E_{kappa,nu}(r, d_ab) (eq. exp_coeffs_1d) of a
// (level, Delta, offset) are stored compactly: for every time pair (a, b) the
// entries with kappa + nu <= m_x, kappa-major, so that entry (a, b, kappa,
// nu) sits at (a (m_t+1) + b) BS + T(kappa) + nu with BS = (m_x+1)(m_x+2)/2
// and T(kappa) = kappa (m_x+1) - kappa (kappa-1)/2: a column part plus a row
// part.  Entries with kappa + nu > m_x are never used unmasked (their total
// degree exceeds m_x); reading them stays inside the padded table.  The x
// table has C_ab folded in.
//
// Per group g the host table plan[g * plan_stride ...] holds
//   [0, 2 W)                  wave w: (first K-step, number of segments)
//   [2 W, 2 W + 3 W MAXS)     wave w, slot i: (tile, end K-step, partial index or -1)
//   [2 W + 3 W MAXS]          number of partial segments n_p
//   [.. + 1, .. + 1 + n_p)    the tile of every partial segment
// with W = WAVES.  A wave's slots are sorted by end; every end but the
// largest lies an even number of K-steps after the wave's first K-step (a
// tile's last segment may be extended by one K-step whose columns are all
// beyond the tile's degree limit), so the two operand sets below alternate
// without copies.  Source moments are read through a buffer descriptor
// spanning the source slot's moments: prefetches beyond a segment (and
// padding columns) return zero without touching other memory.
template <class T> struct M2LTraits;
template <> struct M2LTraits<double> {
    using acc_t = d4_t;
    using pair_t = double2;
    static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // D[i][j] of a 16x16 tile: lane j + 16 (i % 4), register i / 4
    static __device__ __forceinline__ int row(int lq, int r) { return lq + 4 * r; }
    static __device__ __forceinline__ pair_t load_pair(__amdgpu_buffer_rsrc_t rs, int off) {
        return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    }
};
template <> struct M2LTraits<float> {
    using acc_t = f4_t;
    using pair_t = float2;
    static __device__ __forceinline__ acc_t mfma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // D[i][j] of a 16x16 tile: lane j + 16 (i / 4), register i % 4
    static __device__ __forceinline__ int row(int lq, int r) { return 4 * lq + r; }
    static __device__ __forceinline__ pair_t load_pair(__amdgpu_buffer_rsrc_t rs, int off) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
    }
};

// Round to the nearest bfloat16 (ties to even), kept in an FP32 register.
__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

typedef short s4_t __attribute__((ext_vector_type(4)));

// The bfloat16 bits of an FP32 value that already holds a bfloat16 value.
__device__ __forceinline__ short bf16_bits(float x) { return (short)(__float_as_uint(x) >> 16); }

template <class T, int NB, int MAXS, int WAVES, bool RB = false>
__global__ void __launch_bounds__(64 * WAVES) k_m2l_wide(
    const T* __restrict__ mu, double* __restrict__ lam, const int* __restrict__ ptr, const int* __restrict__ src,
    const int* __restrict__ cls, const int* __restrict__ off3, const T* __restrict__ E1c, int TSp,
    const int* __restrict__ packinfo, const int* __restrict__ plan, int plan_stride, int Nc, int n_int, int mt,
    int mx, int R, int nsplit, int ncb, double* __restrict__ lam_parts) {
    static_assert(MAXS >= 1 && MAXS <= 4, "phase dispatch below is written for one to four slots");
    using Tr = M2LTraits<T>;
    using acc_t = typename Tr::acc_t;
    using pair_t = typename Tr::pair_t;
    constexpr int ES = sizeof(T);              // bytes per table entry / moment
    extern __shared__ double smem[];
    const int nt1 = mt + 1, nx1 = mx + 1;
    const int BS = nx1 * (nx1 + 1) / 2;        // compact entries per time pair (a, b)
    const int Nc4 = (Nc + 3) & ~3;
    // two buffers of the six 1D tables of one source phase:
    // [buf][Delta 2: x | y | z, Delta 3: x | y | z][TSp]; then per coefficient
    // column (padded): byte offsets of its x, y, z table columns and its
    // degree (255 for padding columns)
    int4* sCol = (int4*)((char*)smem + 12 * TSp * ES);
    const int lane = threadIdx.x % kWave;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // Workgroups are dealt to the 8 XCDs round-robin by linear id; remap so
    // that each XCD walks a contiguous range of (row group, target slot):
    // the groups of one slot and neighbouring slots read the same moments.
    int g, X, bz;
    {
        const int ng = gridDim.x, nxs = gridDim.y;
        const int total = ng * nxs * gridDim.z;
        const int lin = blockIdx.x + ng * (blockIdx.y + nxs * blockIdx.z);
        const int per = total / kXcds;
        const int lm = lin < per * kXcds ? (lin % kXcds) * per + lin / kXcds : lin;
        g = lm % ng;
        X = (lm / ng) % nxs;
        bz = lm / (ng * nxs);
    }
    const int cb = bz % ncb;
    const int split = bz / ncb;                // which share of the source list this workgroup takes
    if (split > 0) lam = lam_parts + (int64_t)(split - 1) * ((int64_t)gridDim.y * Nc * n_int);
    const int* gp = plan + (int64_t)g * plan_stride;
    const int lr = lane & 15, lq = lane >> 4;
    const int k0 = cb * (32 * NB) + 2 * lr;    // even target interval of block 0
    auto tri = [&](int k) { return k * nx1 - (k * (k - 1)) / 2; };
    for (int c = threadIdx.x; c < Nc4 + 16; c += blockDim.x) {
        int4 v = {0, 0, 0, 255};
        if (c < Nc) {
            const int ci = packinfo[c];
            const int cbase = (ci & 15) * nt1 * BS;
            v.x = ES * (cbase + tri((ci >> 4) & 15));
            v.y = ES * (cbase + tri((ci >> 8) & 15));
            v.z = ES * (cbase + tri((ci >> 12) & 15));
            v.w = (ci >> 16) & 255;
        }
        sCol[c] = v;
    }
    const int sbeg = __builtin_amdgcn_readfirstlane(gp[2 * w]);
    int tiles[MAXS], ks[MAXS], part[MAXS], rX[MAXS], rY[MAXS], rZ[MAXS], rD[MAXS];
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        const int* e = gp + 2 * WAVES + (w * MAXS + i) * 3;
        tiles[i] = __builtin_amdgcn_readfirstlane(e[0]);
        ks[i] = __builtin_amdgcn_readfirstlane(e[1]);   // segment end (exclusive, absolute)
        part[i] = __builtin_amdgcn_readfirstlane(e[2]);
        const int row = 16 * (tiles[i] >= 0 ? tiles[i] : 0) + lr;
        const bool rv = tiles[i] >= 0 && row < Nc;
        const int ri = rv ? packinfo[row] : 0;
        const int b = ri & 15;
        rX[i] = ES * (b * BS + ((ri >> 4) & 15));
        rY[i] = ES * (b * BS + ((ri >> 8) & 15) + TSp);
        rZ[i] = ES * (b * BS + ((ri >> 12) & 15) + 2 * TSp);
        rD[i] = mx - (rv ? ((ri >> 16) & 255) : 255);   // largest column degree this row accepts
    }
    acc_t accE[MAXS][NB], accO[MAXS][NB];
#pragma unroll
    for (int i = 0; i < MAXS; ++i)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            accE[i][nb] = acc_t{0, 0, 0, 0};
            accO[i][nb] = acc_t{0, 0, 0, 0};
        }
    const int nR = 2 * R + 1;
    const int sb = ptr[X], se = ptr[X + 1];
    const int s_lo = sb + (int)(((int64_t)(se - sb) * split) / nsplit);
    const int s_hi = sb + (int)(((int64_t)(se - sb) * (split + 1)) / nsplit);
    const int n_phase = s_hi - s_lo;
    const int pieces = TSp * ES / 1024;              // 1 KB pieces per table
    auto stage = [&](int p) {
        const int c3 = cls[s_lo + p];
        char* dst = (char*)smem + (p & 1) * 6 * TSp * ES;
        for (int c = w; c < 6 * pieces; c += WAVES) {
            const int tb = c / pieces, pc = c - tb * pieces;   // tb = 3 (Delta - 2) + axis
            const int D = tb / 3, axis = tb - 3 * D;
            const int o = off3[3 * c3 + axis] + R;
            const char* gsrc = (const char*)(E1c + (((int64_t)D * nR + o) * 2 + (axis == 0 ? 0 : 1)) * TSp) +
                               pc * 1024 + 16 * lane;
            __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)gsrc,
                                             (void __attribute__((address_space(3)))*)(dst + tb * TSp * ES + pc * 1024),
                                             16, 0, 0);
        }
    };
    // Lane (lr, lq) of K-step s reads, for every block nb, the pair
    // mu[Y][c][k - 2], mu[Y][c][k - 1] with c = 4 s + lq and k = its even
    // target interval: the Delta = 2 sources of the even and odd targets, and
    // (first value) the Delta = 3 source of the odd target.  Block nb is
    // 32 values further.  Targets k < 2 have no sources: their results are
    // written as zero at the end.  The descriptor starts two values before the
    // slot (mu has two leading guard values), so every offset is >= 0; reads
    // past the slot's last coefficient are out of its range and return zero.
    const int vbase = ((4 * sbeg + lq) * n_int + k0) * ES;   // byte offset of mu[Y][c][k - 2] from the descriptor base
    const int bstep = 4 * n_int * ES;                        // bytes between consecutive K-steps
    const int slot_bytes = (Nc * n_int + 2) * ES;
    const char* lds = (const char*)smem;
    const int d3 = 3 * TSp * ES;                             // Delta = 3 tables follow the Delta = 2 ones
    if (n_phase > 0) stage(0);
    for (int p = 0; p < n_phase; ++p) {
        const int Y = src[s_lo + p];
        const int boff = (p & 1) * 6 * TSp * ES;       // byte offset of this phase's table buffer
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(mu + (int64_t)Y * Nc * n_int - 2), (short)0, slot_bytes, 0x00020000);
        __builtin_amdgcn_s_waitcnt(0);   // this wave's pieces of phase p have landed in LDS
        __syncthreads();                 // ... everyone's; and phase p-1 is done with the other buffer
        if (p + 1 < n_phase) stage(p + 1);
        int pX[MAXS], pY[MAXS], pZ[MAXS];
#pragma unroll
        for (int i = 0; i < MAXS; ++i) {
            pX[i] = boff + rX[i];
            pY[i] = boff + rY[i];
            pZ[i] = boff + rZ[i];
        }
        auto load = [&](pair_t* bv, int s) {
            const int vo = vbase + (s - sbeg) * bstep;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) bv[nb] = Tr::load_pair(rs, vo + nb * 32 * ES);
        };
        // one K-step with n active slots
        auto step = [&](auto nc, int4 col, const pair_t* bv) {
            constexpr int n = decltype(nc)::value;
            T A2[n], A3[n];
#pragma unroll
            for (int i = 0; i < n; ++i) {
                const T msk = (col.w <= rD[i]) ? T(1) : T(0);
                const T x2 = *(const T*)(lds + (pX[i] + col.x));
                const T y2 = *(const T*)(lds + (pY[i] + col.y));
                const T z2 = *(const T*)(lds + (pZ[i] + col.z));
                const T x3 = *(const T*)(lds + (pX[i] + d3 + col.x));
                const T y3 = *(const T*)(lds + (pY[i] + d3 + col.y));
                const T z3 = *(const T*)(lds + (pZ[i] + d3 + col.z));
                A2[i] = (x2 * y2) * (z2 * msk);
                A3[i] = (x3 * y3) * (z3 * msk);
                if constexpr (RB) {
                    A2[i] = bf16_round(A2[i]);
                    A3[i] = bf16_round(A3[i]);
                }
            }
            // raised wave priority while this wave issues its products: the
            // arbiter then lets it issue them back to back instead of
            // interleaving other waves' operand generation (about 1% faster)
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int i = 0; i < n; ++i)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    accE[i][nb] = Tr::mfma(A2[i], bv[nb].x, accE[i][nb]);
                    accO[i][nb] = Tr::mfma(A2[i], bv[nb].y, accO[i][nb]);
                    accO[i][nb] = Tr::mfma(A3[i], bv[nb].x, accO[i][nb]);
                }
            __builtin_amdgcn_s_setprio(0);
        };
        if constexpr (RB) {
            // BF16 inputs on the BF16 matrix cores (v_mfma_f32_16x16x16bf16_1k):
            // four consecutive K-steps s..s+3 per product.  Lane (lr, lq)
            // supplies in element e the operator entry and the moment of K
            // index 4 (s + e) + lq, for A and B alike, so the product sums
            // the same 16 K indices as four 16x16x4 steps.  A slot's entries
            // past its segment end are zero (the moments there may belong to
            // another wave's segment).  Slots are sorted by descending end.
            for (int s = sbeg; s < ks[0]; s += 4) {
                int4 cq[4];
                s4_t bx[NB], by[NB];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    pair_t b[NB];
                    load(b, s + e);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        bx[nb][e] = bf16_bits(b[nb].x);
                        by[nb][e] = bf16_bits(b[nb].y);
                    }
                    cq[e] = sCol[4 * (s + e) + lq];
                }
#pragma unroll
                for (int i = 0; i < MAXS; ++i) {
                    if (ks[i] <= s) continue;   // uniform over the wave
                    s4_t a2, a3;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int4 col = cq[e];
                        const T msk = (col.w <= rD[i] && s + e < ks[i]) ? T(1) : T(0);
                        const T x2 = *(const T*)(lds + (pX[i] + col.x));
                        const T y2 = *(const T*)(lds + (pY[i] + col.y));
                        const T z2 = *(const T*)(lds + (pZ[i] + col.z));
                        const T x3 = *(const T*)(lds + (pX[i] + d3 + col.x));
                        const T y3 = *(const T*)(lds + (pY[i] + d3 + col.y));
                        const T z3 = *(const T*)(lds + (pZ[i] + d3 + col.z));
                        a2[e] = bf16_bits(bf16_round((x2 * y2) * (z2 * msk)));
                        a3[e] = bf16_bits(bf16_round((x3 * y3) * (z3 * msk)));
                    }
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        accE[i][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, bx[nb], accE[i][nb], 0, 0, 0);
                        accO[i][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, by[nb], accO[i][nb], 0, 0, 0);
                        accO[i][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3, bx[nb], accO[i][nb], 0, 0, 0);
                    }
                }
            }
            continue;
        }
        // two operand sets used alternately; the set consumed at step s is
        // refilled with step s + 2 right after its products are issued
        int s = sbeg;
        int4 cA = sCol[4 * s + lq], cB = sCol[4 * s + 4 + lq];
        pair_t bA[NB], bB[NB];
        load(bA, s);
        load(bB, s + 1);
        auto phase = [&](auto nc, int s_end) {
            for (; s + 1 < s_end; s += 2) {
                step(nc, cA, bA);
                cA = sCol[4 * s + 8 + lq];
                load(bA, s + 2);
                step(nc, cB, bB);
                cB = sCol[4 * s + 12 + lq];
                load(bB, s + 3);
            }
        };
        if constexpr (MAXS >= 4) phase(std::integral_constant<int, 4>{}, ks[3]);
        if constexpr (MAXS >= 3) phase(std::integral_constant<int, 3>{}, ks[2]);
        if constexpr (MAXS >= 2) phase(std::integral_constant<int, 2>{}, ks[1]);
        phase(std::integral_constant<int, 1>{}, ks[0]);
        if (s < ks[0]) {   // odd final step of the slots that end last
            int na = 1;
#pragma unroll
            for (int i = 1; i < MAXS; ++i) na += ks[i] > s ? 1 : 0;
            if (na == 1) step(std::integral_constant<int, 1>{}, cA, bA);
            if constexpr (MAXS >= 2) if (na == 2) step(std::integral_constant<int, 2>{}, cA, bA);
            if constexpr (MAXS >= 3) if (na == 3) step(std::integral_constant<int, 3>{}, cA, bA);
            if constexpr (MAXS >= 4) if (na == 4) step(std::integral_constant<int, 4>{}, cA, bA);
        }
    }
    // partial segments: one interval block at a time, park in LDS and let the
    // owners of the tiles' first segments add them in a fixed order
    const int n_partial = gp[2 * WAVES + 3 * WAVES * MAXS];
    const int* ptile = gp + 2 * WAVES + 3 * WAVES * MAXS + 1;
    T* red = (T*)smem;   // [n_partial][8][64]
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXS; ++i) {
            if (tiles[i] >= 0 && part[i] >= 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    red[((int64_t)part[i] * 8 + r) * kWave + lane] = accE[i][nb][r];
                    red[((int64_t)part[i] * 8 + 4 + r) * kWave + lane] = accO[i][nb][r];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXS; ++i) {
            if (tiles[i] < 0 || part[i] >= 0) continue;
            for (int q = 0; q < n_partial; ++q) {
                if (ptile[q] != tiles[i]) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    accE[i][nb][r] += red[((int64_t)q * 8 + r) * kWave + lane];
                    accO[i][nb][r] += red[((int64_t)q * 8 + 4 + r) * kWave + lane];
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        if (tiles[i] < 0 || part[i] >= 0) continue;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int kE = k0 + 32 * nb, kO = kE + 1;
            const bool has = kE >= 2;   // targets 0 and 1 have no interaction list in time
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * tiles[i] + Tr::row(lq, r);
                if (row >= Nc) continue;
                double* out = lam + ((int64_t)X * Nc + row) * n_int;
                out[kE] = has ? (double)accE[i][nb][r] : 0.0;
                out[kO] = has ? (double)accO[i][nb][r] : 0.0;
            }
        }
    }
}

// wide M2L variants (interval blocks, slots per wave, waves per workgroup):
// [0] for levels with 32 intervals, [1] with a multiple of 64, [2] of 128
// [precision: 0 FP64, 1 FP32, 2 BF16 inputs][variant]
constexpr int kWideNB[3] = {1, 2, 4};
constexpr int kWideMaxs[3][3] = {{2, 2, 1}, {2, 2, 2}, {2, 2, 1}};
constexpr int kWideWaves[3][3] = {{16, 16, 16}, {16, 16, 16}, {16, 16, 16}};
constexpr bool kWideUseNB1 = true;   // levels with 32 intervals: wide form instead of k_m2l_mfma

template <int Q, int V>
using WideT = std::conditional_t<Q == 0, double, float>;

template <int Q, int V>
const void* wide_fn() {
    return (const void*)k_m2l_wide<WideT<Q, V>, kWideNB[V], kWideMaxs[Q][V], kWideWaves[Q][V], Q == 2>;
}

const void* wide_fn(int q, int v) {
    if (q == 0) return v == 0 ? wide_fn<0, 0>() : (v == 1 ? wide_fn<0, 1>() : wide_fn<0, 2>());
    if (q == 1) return v == 0 ? wide_fn<1, 0>() : (v == 1 ? wide_fn<1, 1>() : wide_fn<1, 2>());
    return v == 0 ? wide_fn<2, 0>() : (v == 1 ? wide_fn<2, 1>() : wide_fn<2, 2>());
}

template <int Q, int V>
void launch_wide(dim3 grid, size_t shm, hipStream_t st, const void* mu, double* lam, const int* ptr, const int* src,
                 const int* cls, const int* off3, const void* E1s, int TSp, const int* packinfo, const int* plan,
                 int plan_stride, int Nc, int n_int, int mt, int mx, int R, int nsplit, int ncb, double* lam_parts) {
    using T = WideT<Q, V>;
    hipLaunchKernelGGL((k_m2l_wide<T, kWideNB[V], kWideMaxs[Q][V], kWideWaves[Q][V], Q == 2>), grid,
                       dim3(64 * kWideWaves[Q][V]), shm, st, (const T*)mu, lam, ptr, src, cls, off3, (const T*)E1s,
                       TSp, packinfo, plan, plan_stride, Nc, n_int, mt, mx, R, nsplit, ncb, lam_parts);
}

using WideLaunch = void (*)(dim3, size_t, hipStream_t, const void*, double*, const int*, const int*, const int*,
                            const int*, const void*, int, const int*, const int*, int, int, int, int, int, int, int,
                            int, double*);

WideLaunch wide_launcher(int q, int v) {
    if (q == 0) return v == 0 ? launch_wide<0, 0> : (v == 1 ? launch_wide<0, 1> : launch_wide<0, 2>);
    if (q == 1) return v == 0 ? launch_wide<1, 0> : (v == 1 ? launch_wide<1, 1> : launch_wide<1, 2>);
    return v == 0 ? launch_wide<2, 0> : (v == 1 ? launch_wide<2, 1> : launch_wide<2, 2>);
}

// FP32 copy of a level's moments for the mixed-precision M2L (rounded on to
// bfloat16 values when bf16 is set).
__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n, int bf16) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = bf16 ? bf16_round((float)a[i]) : (float)a[i];
}

// Sum the per-share partial locals of a level whose interaction lists were
// split over several workgroups (fixed order: share 0, 1, ...), with
// Neumaier's compensated summation in FP64: the partial sums (each the FP32
// matrix-core result of one share in the mixed modes) can cancel, and the
// compensation keeps the folded value within one rounding of the exact sum
// of the shares.
__global__ void k_sum_parts(double* __restrict__ lam, const double* __restrict__ parts, int nparts, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = lam[i], c = 0.0;
    for (int p = 0; p < nparts; ++p) {
        const double x = parts[(int64_t)p * n + i];
        const double u = s + x;
        c += fabs(s) >= fabs(x) ? (s - u) + x : (x - u) + s;
        s = u;
    }
    lam[i] = s + c;
}

// M2L on matrix cores for levels whose intervals differ in length or are
// missing (time split points at the nearest step, Algorithm 1; partial
// levels where leaves sit at several levels of one time range).  The
// operator of eq. m2l depends on the target and source intervals through
// their node differences only, so the pairs of a level fall into a few time
// classes, each with its own 1D tables (eq. exp_coeffs_1d, same compact rows
// as k_m2l_wide).  One launch handles one time offset D (2: every target
// interval k >= 2 with source k - 2; 3: odd k with source k - 3): its columns
// are the target intervals of the level, sorted by class on the host
// (cols[i] = (k, class), padded with k = -1), so that a workgroup's 16 NB
// columns span few classes.  A level has few columns per class (one time
// offset, a few of the 2^l intervals), so the operator tiles are shared
// across target slots instead: the operator of a pair depends on the source
// only through its spatial offset Y - X, and neighbouring target slots have
// nearly the same offsets within the truncation radius.  A workgroup owns a
// group of KT target slots (consecutive in the slots' Morton order), one row
// group and one block of 16 NB columns; it walks the union of the group's
// offsets (merged on the host: per offset, the source slot of each target
// or -1) and, per offset, the classes of its columns (cbr[cb] = first and
// last class of the block); the operator tile of (offset, class) is
// generated from LDS once and multiplies the columns of that class of every
// target that has a source at that offset.  The results are added to lam,
// which the caller zeroes before the first of the two launches (each
// (X, row, k) is owned by one workgroup per launch, and its products are
// summed in the group's offset order: deterministic).
// One level of one tree for the class-aware M2L (one time offset D).
struct ClsUnit {
    const void* mu;          // moments gathered into column order [slot][coef][column]
                             // (FP64, or FP32 / BF16 values)
    double* lam;             // locals of the level (added to)
    const int* tgx;          // target slots of each group [group][KT] (-1: none)
    const int* tgptr;        // merged offsets of each group: CSR over groups
    const int* tgcls;        //   spatial offset class
    const int* tgsrc;        //   source slot of each target [entry][KT] (-1: none)
    const int* off3;         // offsets per class
    const void* E1c;         // compact 1D tables of the level [class][offset][x | yz]
    const int2* cols;        // columns (k, class), padded with k = -1
    const int2* cbr;         // first and last class per column block
    int n_int, R, ntg, nccb, D;   // ntg: target groups
    int ncp;                 // columns of the gathered moments (16 NB nccb)
    int wg0;                 // first workgroup of this unit in a batched launch
};

// mup[slot][c][i] = mu[slot][c][perm[i]] (0 where perm[i] < 0), converted to
// T (rounded on to bfloat16 values when bf16 is set): the class-aware M2L's
// B operand in column order.
template <class T>
__global__ void k_gather_cols(const double* __restrict__ mu, T* __restrict__ mup, const int* __restrict__ perm,
                              int n_int, int ncp, int64_t n, int bf16) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t row = i / ncp;
    const int k = perm[i - row * ncp];
    const double v = k >= 0 ? mu[row * n_int + k] : 0.0;
    if constexpr (sizeof(T) == 8) mup[i] = v;
    else mup[i] = bf16 ? bf16_round((float)v) : (float)v;
}

template <class T, int NB, int MAXS, int WAVES, int KT, bool RB>
__device__ __forceinline__ void m2l_cls_body(
    double* smem, const ClsUnit& U, int g, int tg, int cb, int TSp, const int* __restrict__ packinfo,
    const int* __restrict__ plan, int plan_stride, int Nc, int mt, int mx) {
    static_assert(MAXS >= 1 && MAXS <= 4, "phase dispatch below is written for one to four slots");
    using Tr = M2LTraits<T>;
    using acc_t = typename Tr::acc_t;
    constexpr int ES = sizeof(T);
    const T* __restrict__ mu = (const T*)U.mu;
    double* __restrict__ lam = U.lam;
    const int* __restrict__ off3 = U.off3;
    const T* __restrict__ E1c = (const T*)U.E1c;
    const int2* __restrict__ cols = U.cols;
    const int2* __restrict__ cbr = U.cbr;
    const int R = U.R;
    const int nt1 = mt + 1, nx1 = mx + 1;
    const int BS = nx1 * (nx1 + 1) / 2;
    const int Nc4 = (Nc + 3) & ~3;
    // two buffers of the three 1D tables of one (offset, class) phase, then
    // the per-column table offsets and degrees
    int4* sCol = (int4*)((char*)smem + 6 * TSp * ES);
    const int lane = threadIdx.x % kWave;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int* gp = plan + (int64_t)g * plan_stride;
    const int lr = lane & 15, lq = lane >> 4;
    auto tri = [&](int k) { return k * nx1 - (k * (k - 1)) / 2; };
    for (int c = threadIdx.x; c < Nc4 + 16; c += blockDim.x) {
        int4 v = {0, 0, 0, 255};
        if (c < Nc) {
            const int ci = packinfo[c];
            const int cbase = (ci & 15) * nt1 * BS;
            v.x = ES * (cbase + tri((ci >> 4) & 15));
            v.y = ES * (cbase + tri((ci >> 8) & 15));
            v.z = ES * (cbase + tri((ci >> 12) & 15));
            v.w = (ci >> 16) & 255;
        }
        sCol[c] = v;
    }
    // this lane's target interval in every sub-block nb, and the sub-block's
    // class (one per sub-block, -1 for an empty one: uniform over the wave)
    int kcol[NB], ccol[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int2 e = cols[(cb * NB + nb) * 16 + lr];
        kcol[nb] = e.x;
        ccol[nb] = __builtin_amdgcn_readfirstlane(e.y);
    }
    int X[KT];
#pragma unroll
    for (int j = 0; j < KT; ++j) X[j] = __builtin_amdgcn_readfirstlane(U.tgx[tg * KT + j]);
    const int2 crange = cbr[cb];
    const int cmin = __builtin_amdgcn_readfirstlane(crange.x);
    const int ncr = __builtin_amdgcn_readfirstlane(crange.y - crange.x + 1);
    const int sbeg = __builtin_amdgcn_readfirstlane(gp[2 * w]);
    int tiles[MAXS], ks[MAXS], part[MAXS], rX[MAXS], rY[MAXS], rZ[MAXS], rD[MAXS];
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        const int* e = gp + 2 * WAVES + (w * MAXS + i) * 3;
        tiles[i] = __builtin_amdgcn_readfirstlane(e[0]);
        ks[i] = __builtin_amdgcn_readfirstlane(e[1]);
        part[i] = __builtin_amdgcn_readfirstlane(e[2]);
        const int row = 16 * (tiles[i] >= 0 ? tiles[i] : 0) + lr;
        const bool rv = tiles[i] >= 0 && row < Nc;
        const int ri = rv ? packinfo[row] : 0;
        const int b = ri & 15;
        rX[i] = ES * (b * BS + ((ri >> 4) & 15));
        rY[i] = ES * (b * BS + ((ri >> 8) & 15) + TSp);
        rZ[i] = ES * (b * BS + ((ri >> 12) & 15) + 2 * TSp);
        rD[i] = mx - (rv ? ((ri >> 16) & 255) : 255);
    }
    acc_t acc[KT][MAXS][NB];
#pragma unroll
    for (int j = 0; j < KT; ++j)
#pragma unroll
        for (int i = 0; i < MAXS; ++i)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[j][i][nb] = acc_t{0, 0, 0, 0};
    const int nR = 2 * R + 1;
    const int sb = U.tgptr[tg], se = U.tgptr[tg + 1];
    const int n_phase = (se - sb) * ncr;
    const int pieces = TSp * ES / 1024;
    auto stage = [&](int p) {
        const int si = sb + p / ncr, c = cmin + p % ncr;
        const int c3 = U.tgcls[si];
        char* dst = (char*)smem + (p & 1) * 3 * TSp * ES;
        for (int q = w; q < 3 * pieces; q += WAVES) {
            const int axis = q / pieces, pc = q - axis * pieces;
            const int o = off3[3 * c3 + axis] + R;
            const char* gsrc = (const char*)(E1c + (((int64_t)c * nR + o) * 2 + (axis == 0 ? 0 : 1)) * TSp) +
                               pc * 1024 + 16 * lane;
            __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)gsrc,
                                             (void __attribute__((address_space(3)))*)(dst + axis * TSp * ES + pc * 1024),
                                             16, 0, 0);
        }
    };
    // byte offsets of the gathered moments of column (cb NB + nb) 16 + lr
    // for K-step sbeg (padding columns hold zeros); loads past the slot
    // return zero
    const int ncp = U.ncp;
    int vb[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) vb[nb] = ((4 * sbeg + lq) * ncp + (cb * NB + nb) * 16 + lr) * ES;
    const int bstep = 4 * ncp * ES;
    const int slot_bytes = Nc * ncp * ES;
    const char* lds = (const char*)smem;
    if (n_phase > 0) stage(0);
    for (int p = 0; p < n_phase; ++p) {
        const int si = sb + p / ncr, c = cmin + p % ncr;
        const int boff = (p & 1) * 3 * TSp * ES;
        // the source slot of each target at this offset (-1: none; its
        // loads and products are skipped, a wave-uniform branch)
        int Y[KT];
        __amdgpu_buffer_rsrc_t rs[KT];
#pragma unroll
        for (int j = 0; j < KT; ++j) {
            Y[j] = __builtin_amdgcn_readfirstlane(U.tgsrc[(int64_t)si * KT + j]);
            rs[j] = __builtin_amdgcn_make_buffer_rsrc((void*)(mu + (int64_t)(Y[j] >= 0 ? Y[j] : 0) * Nc * ncp),
                                                      (short)0, slot_bytes, 0x00020000);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (p + 1 < n_phase) stage(p + 1);
        // sub-blocks of another class skip their loads and products (a
        // wave-uniform branch)
        bool on[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) on[nb] = ccol[nb] == c;
        int pX[MAXS], pY[MAXS], pZ[MAXS];
#pragma unroll
        for (int i = 0; i < MAXS; ++i) {
            pX[i] = boff + rX[i];
            pY[i] = boff + rY[i];
            pZ[i] = boff + rZ[i];
        }
        auto load = [&](T (*bv)[NB], int s) {
#pragma unroll
            for (int j = 0; j < KT; ++j)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int vo = vb[nb] + (s - sbeg) * bstep;
                    if (!on[nb] || Y[j] < 0) bv[j][nb] = T(0);
                    else if constexpr (ES == 8)
                        bv[j][nb] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs[j], vo, 0, 0));
                    else
                        bv[j][nb] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs[j], vo, 0, 0));
                }
        };
        auto step = [&](auto nc, int4 col, T (*bv)[NB]) {
            constexpr int n = decltype(nc)::value;
            T A[n];
#pragma unroll
            for (int i = 0; i < n; ++i) {
                const T m = (col.w <= rD[i]) ? T(1) : T(0);
                const T x = *(const T*)(lds + (pX[i] + col.x));
                const T y = *(const T*)(lds + (pY[i] + col.y));
                const T z = *(const T*)(lds + (pZ[i] + col.z));
                A[i] = (x * y) * (z * m);
                if constexpr (RB) A[i] = bf16_round(A[i]);
            }
#pragma unroll
            for (int j = 0; j < KT; ++j)
                if (Y[j] >= 0)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        if (on[nb])
#pragma unroll
                            for (int i = 0; i < n; ++i) acc[j][i][nb] = Tr::mfma(A[i], bv[j][nb], acc[j][i][nb]);
        };
        int s = sbeg;
        int4 cA = sCol[4 * s + lq], cB = sCol[4 * s + 4 + lq];
        T bA[KT][NB], bB[KT][NB];
        load(bA, s);
        load(bB, s + 1);
        auto phase = [&](auto nc, int s_end) {
            for (; s + 1 < s_end; s += 2) {
                step(nc, cA, bA);
                cA = sCol[4 * s + 8 + lq];
                load(bA, s + 2);
                step(nc, cB, bB);
                cB = sCol[4 * s + 12 + lq];
                load(bB, s + 3);
            }
        };
        if constexpr (MAXS >= 4) phase(std::integral_constant<int, 4>{}, ks[3]);
        if constexpr (MAXS >= 3) phase(std::integral_constant<int, 3>{}, ks[2]);
        if constexpr (MAXS >= 2) phase(std::integral_constant<int, 2>{}, ks[1]);
        phase(std::integral_constant<int, 1>{}, ks[0]);
        if (s < ks[0]) {
            int na = 1;
#pragma unroll
            for (int i = 1; i < MAXS; ++i) na += ks[i] > s ? 1 : 0;
            if (na == 1) step(std::integral_constant<int, 1>{}, cA, bA);
            if constexpr (MAXS >= 2) if (na == 2) step(std::integral_constant<int, 2>{}, cA, bA);
            if constexpr (MAXS >= 3) if (na == 3) step(std::integral_constant<int, 3>{}, cA, bA);
            if constexpr (MAXS >= 4) if (na == 4) step(std::integral_constant<int, 4>{}, cA, bA);
        }
    }
    // partial segments through LDS, added by the tiles' first segments in a fixed order
    const int n_partial = gp[2 * WAVES + 3 * WAVES * MAXS];
    const int* ptile = gp + 2 * WAVES + 3 * WAVES * MAXS + 1;
    T* red = (T*)smem;   // [n_partial][4][64]
#pragma unroll
    for (int j = 0; j < KT; ++j)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < MAXS; ++i)
                if (tiles[i] >= 0 && part[i] >= 0)
#pragma unroll
                    for (int r = 0; r < 4; ++r) red[((int64_t)part[i] * 4 + r) * kWave + lane] = acc[j][i][nb][r];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < MAXS; ++i) {
                if (tiles[i] < 0 || part[i] >= 0) continue;
                for (int q = 0; q < n_partial; ++q) {
                    if (ptile[q] != tiles[i]) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[j][i][nb][r] += red[((int64_t)q * 4 + r) * kWave + lane];
                }
            }
        }
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        if (X[j] < 0) continue;
#pragma unroll
        for (int i = 0; i < MAXS; ++i) {
            if (tiles[i] < 0 || part[i] >= 0) continue;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                if (kcol[nb] < 0) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * tiles[i] + Tr::row(lq, r);
                    if (row >= Nc) continue;
                    double* out = lam + ((int64_t)X[j] * Nc + row) * U.n_int + kcol[nb];
                    *out += (double)acc[j][i][nb][r];
                }
            }
        }
    }
}

template <class T, int NB, int MAXS, int WAVES, int KT, bool RB = false>
__global__ void __launch_bounds__(64 * WAVES) k_m2l_cls(ClsUnit U, int TSp, const int* __restrict__ packinfo,
                                                       const int* __restrict__ plan, int plan_stride, int Nc, int mt,
                                                       int mx) {
    extern __shared__ double smem[];
    // XCD-aware remap of the linear workgroup id (as k_m2l_wide)
    const int ng = gridDim.x, nxs = gridDim.y;
    const int total = ng * nxs * gridDim.z;
    const int lin = blockIdx.x + ng * (blockIdx.y + nxs * blockIdx.z);
    const int per = total / kXcds;
    const int lm = lin < per * kXcds ? (lin % kXcds) * per + lin / kXcds : lin;
    m2l_cls_body<T, NB, MAXS, WAVES, KT, RB>(smem, U, lm % ng, (lm / ng) % nxs, lm / (ng * nxs), TSp, packinfo,
                                             plan, plan_stride, Nc, mt, mx);
}

// The class-aware M2L of many (tree, level) units in one launch (trees of a
// batch with the same degrees share the row-group plan): a 1D grid over the
// units' workgroups, each finding its unit by binary search on wg0.
template <class T, int NB, int MAXS, int WAVES, int KT, bool RB = false>
__global__ void __launch_bounds__(64 * WAVES) k_m2l_cls_batch(const ClsUnit* __restrict__ units, int n_units, int G,
                                                             int TSp, const int* __restrict__ packinfo,
                                                             const int* __restrict__ plan, int plan_stride, int Nc,
                                                             int mt, int mx) {
    extern __shared__ double smem[];
    const int total = gridDim.x;
    const int lin = blockIdx.x;
    const int per = total / kXcds;
    const int lm = lin < per * kXcds ? (lin % kXcds) * per + lin / kXcds : lin;
    int lo = 0, hi = n_units - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (units[mid].wg0 <= lm) lo = mid; else hi = mid - 1;
    }
    const ClsUnit U = units[lo];
    const int loc = lm - U.wg0;
    m2l_cls_body<T, NB, MAXS, WAVES, KT, RB>(smem, U, loc % G, (loc / G) % U.ntg, loc / (G * U.ntg), TSp, packinfo,
                                             plan, plan_stride, Nc, mt, mx);
}

// class-aware M2L: one column block of 16 per workgroup, 16 waves, three
// target slots per workgroup, two slots per wave (per precision: FP64, FP32,
// BF16 inputs).  Measured on the 12,288 x 479 and 10,800 x 239 trees of the
// 48-problem batch (M2L stage, FP64): one target, two blocks of 16 columns
// 229 / 246 ms; two targets 223 / 218 ms; three 215 / 210 ms; four with one
// slot per wave (two would spill) 271 / 264 ms
constexpr int kClsNB = 1, kClsWaves = 16, kClsKT = 3;
constexpr int kClsMaxs[3] = {2, 2, 2};

template <int Q>
const void* cls_fn() {
    return (const void*)k_m2l_cls<std::conditional_t<Q == 0, double, float>, kClsNB, kClsMaxs[Q], kClsWaves, kClsKT, Q == 2>;
}

template <int Q>
const void* cls_batch_fn() {
    return (const void*)k_m2l_cls_batch<std::conditional_t<Q == 0, double, float>, kClsNB, kClsMaxs[Q], kClsWaves,
                                        kClsKT, Q == 2>;
}

const void* cls_fn(int q) { return q == 0 ? cls_fn<0>() : (q == 1 ? cls_fn<1>() : cls_fn<2>()); }
const void* cls_batch_fn(int q) { return q == 0 ? cls_batch_fn<0>() : (q == 1 ? cls_batch_fn<1>() : cls_batch_fn<2>()); }

template <int Q>
void launch_cls(dim3 grid, size_t shm, hipStream_t st, const ClsUnit& U, int TSp, const int* packinfo, const int* plan,
                int plan_stride, int Nc, int mt, int mx) {
    using T = std::conditional_t<Q == 0, double, float>;
    hipLaunchKernelGGL((k_m2l_cls<T, kClsNB, kClsMaxs[Q], kClsWaves, kClsKT, Q == 2>), grid, dim3(64 * kClsWaves), shm, st, U,
                       TSp, packinfo, plan, plan_stride, Nc, mt, mx);
}

template <int Q>
void launch_cls_batch(unsigned n_wg, size_t shm, hipStream_t st, const ClsUnit* units, int n_units, int G, int TSp,
                      const int* packinfo, const int* plan, int plan_stride, int Nc, int mt, int mx) {
    using T = std::conditional_t<Q == 0, double, float>;
    hipLaunchKernelGGL((k_m2l_cls_batch<T, kClsNB, kClsMaxs[Q], kClsWaves, kClsKT, Q == 2>), dim3(n_wg), dim3(64 * kClsWaves),
                       shm, st, units, n_units, G, TSp, packinfo, plan, plan_stride, Nc, mt, mx);
}

using ClsLaunch = void (*)(dim3, size_t, hipStream_t, const ClsUnit&, int, const int*, const int*, int, int, int, int);
using ClsBatchLaunch = void (*)(unsigned, size_t, hipStream_t, const ClsUnit*, int, int, int, const int*, const int*,
                                int, int, int, int);

ClsLaunch cls_launcher(int q) { return q == 0 ? launch_cls<0> : (q == 1 ? launch_cls<1> : launch_cls<2>); }
ClsBatchLaunch cls_batch_launcher(int q) {
    return q == 0 ? launch_cls_batch<0> : (q == 1 ? launch_cls_batch<1> : launch_cls_batch<2>);
}
