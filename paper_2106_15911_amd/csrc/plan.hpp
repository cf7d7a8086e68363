// Host planner of the space-time FMM: geometry, the box cluster tree of
// Algorithm 1, the temporal and space-time lists of Section 3.3, the
// nearfield row groups and the expansion tables of Section 3.1/3.4.
// Pure host C++; no GPU calls.
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "pfmm.h"

namespace pfmm {

// One level of the box cluster tree.  Every box of level l is a pair
// (spatial box slot xs, temporal interval k) with k the path index
// 2 * parent + child bit (0 <= k < 2^l).
struct Level {
    int lx = 0;                 // number of spatial refinements above this level
    double hx = 0.0;            // unpadded spatial half-size
    double pad = 0.0;           // padding of every box of this level
    double H = 0.0;             // padded half-size hx + pad
    int rtype = -1;             // refinement to l+1: 0 temporal, 1 space-time, -1 none
    int n_int = 1;              // 2^l
    std::vector<int> istart, iend;          // steps [istart, iend) of interval k; -1 absent
    std::vector<std::array<int, 3>> ix;     // grid index of spatial slot xs
    std::vector<int> tb, te;                // triangle range (sorted order) of slot xs
    std::vector<int> parent;                // slot of the parent spatial box at l-1
    std::vector<int> octant;                // child octant bits (x<<2|y<<1|z) in the parent
    std::vector<uint8_t> present, leaf;     // [xs * n_int + k]
    // M2L time classes (levels >= 2): the operator of eq. m2l depends on the
    // target and source intervals only through their node differences, i.e.
    // (start_k - start_J, len_k, len_J) (in steps on a uniform grid, as times
    // otherwise).  cls[D - 2][k] is the class
    // of target interval k with source J = k - D (D = 2, 3 for odd k; -1 if
    // there is none); cls_rep[c] = (k, J) a representative pair, cls_D[c] = D.
    std::vector<int> cls[2];
    std::vector<std::array<int, 2>> cls_rep;
    std::vector<int> cls_D;
    // every interval present with the same length, every slot in every
    // interval, leaf status independent of the interval: the classes are
    // exactly D = 2 (class 0) and D = 3 (class 1) and the batched-in-time
    // M2L kernels apply
    bool uniform = true;
    int nx() const { return (int)ix.size(); }
    bool box(int xs, int k) const { return present[(size_t)xs * n_int + k] != 0; }
    bool is_leaf(int xs, int k) const { return leaf[(size_t)xs * n_int + k] != 0; }
};

// Nearfield source rectangle of a leaf: source steps [j0, j1) and a set of
// source triangles (sorted positions).
struct Rect { int j0, j1, set; };

struct LeafRec {
    int l, xs, k;       // level, spatial slot, interval
    int s0, s1;         // steps
    int tb, te;         // triangle positions
    int rect0, rect1;   // range into rects
    int group;          // assembly group (level, spatial slot)
};

struct RowGroup {
    int leaf;           // index into leaves
    int kt;             // target time step
    int64_t boff;       // offset (doubles) of its column-major block
    int64_t ncols;      // columns (causal source elements)
};

struct AsmGroup {
    int l, xs;          // level, spatial slot (leaf spatial box)
    int tb, te;         // target triangle positions
    int dmax;           // largest time offset needed
    int64_t uoff;       // offset into upos (source positions, sorted)
    int usize;
    int64_t toff;       // offset of the table [d][u][r] (rows innermost)
    int64_t mapoff;     // offset of the position -> u map (size E_x)
};

struct TouchPair {      // touching panel pair inside an assembly group
    int group, r, u, nshared;
};

struct Plan {
    // inputs
    int E_x = 0, E_t = 0, n_vert = 0;
    double alpha = 1.0, T = 0.0, h = 0.0;
    int m_t = 6, m_x = 6, n_max = 64, n_tr = 5, q_reg = 4, q_sing = 5;
    double c_st = 0.9;
    std::vector<double> verts;          // n_vert x 3
    std::vector<int> tris;              // E_x x 3 (natural order)
    std::vector<int> adj;               // E_x x 3: triangle across edge (v_e, v_{e+1})
    std::vector<double> tnodes;         // E_t + 1
    bool uniform_steps = true;          // all steps of length h = T / E_t (to 1e-12 h)

    // geometry (natural triangle order)
    std::vector<double> area, normal, centroid, maxedge;
    double lo0[3] = {0, 0, 0}, h0 = 0.0;

    // triangle ordering: pos = sigma[natural], natural = inv_sigma[pos]
    std::vector<int> sigma, inv_sigma;

    std::vector<Level> lev;
    int depth = 0;

    // coefficient ordering (degree, time index, multi-index)
    int Nk = 0, Nc = 0;
    std::vector<int> coef_a, coef_deg, coef_k;   // coef_k: Nc x 3
    std::vector<int> kidx_k;                     // Nk x 3 (spatial multi-index order)

    // counts
    int64_t n_boxes = 0, n_leaves = 0, near_entries = 0, m2l_pairs = 0, distinct = 0;
    int64_t near_nonzero_K = 0;   // causal nearfield entries between panels that are not coplanar

    // nearfield
    std::vector<LeafRec> leaves;
    std::vector<Rect> rects;
    std::vector<int> set_off, set_size, set_pos;
    std::vector<RowGroup> rows;
    std::vector<AsmGroup> groups;
    std::vector<int> upos;                       // source positions per group
    std::vector<int> umap;                       // per group E_x map pos -> u (-1 absent)
    std::vector<TouchPair> touch;
    int64_t table_size = 0;                      // doubles of all distinct tables

    // nearfield of the double layer with p1 trial functions (Section 2):
    // every source triangle position p contributes three columns 3 p + i
    // (its local vertices i); expanded source sets, block offsets per row
    // group, and per assembly group the expanded table (usize3 = 3 usize
    // columns) and position map (3 E_x entries per group)
    struct P1Layout {
        bool built = false;
        std::vector<int> set_off, set_size, set_pos;   // expanded sets
        std::vector<int64_t> boff;                     // per row group
        int64_t near_entries = 0;
        std::vector<int64_t> toff;                     // per assembly group
        int64_t table_size = 0;
        std::vector<int> umap;                         // groups x 3 E_x
    } p1;

    // farfield levels (>= 2 and <= depth)
    int far_lo = 2;
    bool has_far = false;
    int max_time_classes = 0;   // most M2L time classes on one level >= 2
};

// Build everything host-side.  Returns PFMM_OK or an error status with msg.
pfmm_status build_plan(const double* V, int64_t nv, const int32_t* T, int64_t nt,
                       const double* tn, int64_t E_t, const pfmm_params& p,
                       Plan& P, std::string& msg);

// Fill P.p1 from the p0 nearfield layout (call after build_plan).
void build_p1_layout(Plan& P);

// Gauss-Legendre nodes/weights on [0, 1] (Newton iteration on P_n).
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);

// Chebyshev nodes cos((2k+1) pi / (2(m+1))), k = 0..m.
std::vector<double> cheb_nodes(int m);

int binom(int n, int k);

}  // namespace pfmm
