// Host-computed expansion tables of Section 3.1 / 3.4 for the device kernels.
#pragma once
#include <cstdint>
#include <vector>

#include "plan.hpp"

namespace pfmm {

struct FarLevel {
    int l = 0;
    int nx = 0, n_int = 0;              // slots, intervals
    std::vector<int> istart, ilen;      // steps of interval k (start, count; 0, 0 if absent)
    // leaves of this level: slots that are leaves in at least one interval;
    // leaf[li * n_int + k] = 1 if (leaf_xs[li], k) is a leaf box
    std::vector<int> leaf_xs;
    std::vector<uint8_t> leaf;
    // boxes with children: inner[xs * n_int + k] = 1 if (xs, k) is present and not a leaf
    std::vector<uint8_t> inner;
    std::vector<int64_t> ax_off;        // per leaf slot, offset into Ax / AxK
    // S2M / L2T blocks: (leaf slot index, first row) of row chunks of at most 64 triangles
    std::vector<int> chunk_li, chunk_r0;
    int64_t at_off = 0;                 // A_t block: [E_t][m_t+1] (row j: step j in its interval of this level)
    // q^(t) for this level as the CHILD level: [n_int][m_t+1 (a_c)][m_t+1 (a_p)]
    int64_t qt_off = -1;
    // q^(x) per slot of this level as CHILD: [nx][3][m_x+1 (kappa)][m_x+1 (nu)]
    int64_t qx_off = -1;
    // M2L: CSR over target slots of (source slot, offset class)
    std::vector<int> m2l_ptr, m2l_src, m2l_cls;
    int n_off = 0;                      // distinct offsets used
    std::vector<int> off3;              // per offset class: grid offset (target - source) per axis
    int R = 0;                          // largest |offset| per axis covered by E1
    int ncls = 0;                       // M2L time classes (Level::cls_rep)
    int64_t e1_off = 0;                 // E1 tables [ncls][2R+1][m_t+1][m_t+1][m_x+1][m_x+1]
    int64_t cab_off = 0;                // C_ab [ncls][m_t+1][m_t+1]
    std::vector<int> children_ptr, children;   // for M2M: child slots (level l+1) of slot xs
};

struct FarTables {
    std::vector<FarLevel> lv;           // indexed by level (entries < 2 unused)
    std::vector<double> At, Ax, AxK, qt, qx, E1, Cab;
    // S2M of the double layer with p1 trial functions: three rows per
    // triangle (local vertex i), alpha int lambda_i n.grad T_kappa; offsets
    // 3 ax_off (built when requested)
    std::vector<double> AxK1;
    // row chunks of the M2L operator (rows in coefficient order)
    int chunk = 32, n_chunks = 0;
    std::vector<int> chunk_cols;        // columns per chunk (staircase prefix)
    std::vector<int64_t> chunk_off;     // offset of chunk inside one operator
    int64_t op_size = 0;                // doubles per operator (one class)
};

void build_far_tables(const Plan& P, FarTables& F, bool with_p1 = false);

}  // namespace pfmm
