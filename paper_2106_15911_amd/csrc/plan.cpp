// Host planner: Algorithm 1 (box cluster tree), Section 3.3 lists and the
// nearfield layout.  See plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <unordered_map>

namespace pfmm {

int binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    long long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return (int)r;
}

void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
    // Newton iteration on the Legendre polynomial P_n; nodes mapped to [0, 1].
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    auto legendre = [n](double z, double& pn, double& pm) {
        pm = 1.0;
        pn = z;
        for (int k = 1; k < n; ++k) {
            double pk = ((2.0 * k + 1.0) * z * pn - k * pm) / (k + 1.0);
            pm = pn;
            pn = pk;
        }
    };
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pn, pm;
        for (int it = 0; it < 100; ++it) {
            legendre(z, pn, pm);
            double dp = n * (z * pn - pm) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) <= 1e-16) break;
        }
        legendre(z, pn, pm);
        double dp = n * (z * pn - pm) / (z * z - 1.0);
        x[i] = 0.5 * (1.0 + z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
    std::vector<double> xs(n), ws(n);
    for (int i = 0; i < n; ++i) { xs[i] = x[idx[i]]; ws[i] = w[idx[i]]; }
    x.swap(xs);
    w.swap(ws);
}

std::vector<double> cheb_nodes(int m) {
    std::vector<double> r(m + 1);
    for (int k = 0; k <= m; ++k) r[k] = std::cos((2.0 * k + 1.0) * M_PI / (2.0 * (m + 1)));
    return r;
}

namespace {

inline bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Algorithm 1 halves a time interval at its midpoint; on a grid of steps the
// split falls on the node nearest to the midpoint of [t_s0, t_s1] (the
// earlier of two nodes equally near, within 1e-12 T), which for uniform
// steps is the middle step, the earlier one for an odd count.
int split_node(const double* tn, int s0, int s1, double T) {
    const double tm = 0.5 * (tn[s0] + tn[s1]);
    double best = INFINITY;
    for (int j = s0 + 1; j < s1; ++j) best = std::min(best, std::fabs(tn[j] - tm));
    for (int j = s0 + 1; j < s1; ++j)
        if (std::fabs(tn[j] - tm) <= best + 1e-12 * T) return j;
    return (s0 + s1) / 2;
}

struct SlotBuild {
    std::array<int, 3> ix;
    std::vector<int> tris;   // natural indices
    int parent;
    int octant;
};

}  // namespace

pfmm_status build_plan(const double* V, int64_t nv, const int32_t* Tr, int64_t nt,
                       const double* tn, int64_t E_t, const pfmm_params& p,
                       Plan& P, std::string& msg) {
    // ------------------------------------------------------------ validation
    if (!V || !Tr || !tn) { msg = "NULL mesh or time array"; return PFMM_EINVAL; }
    if (nv < 3 || nt < 1 || E_t < 1) { msg = "empty mesh or time grid"; return PFMM_EINVAL; }
    if (nt > (1 << 26) || E_t > (1 << 24)) { msg = "mesh or time grid too large"; return PFMM_EUNSUPPORTED; }
    if (!(p.alpha > 0) || !std::isfinite(p.alpha)) { msg = "alpha must be > 0"; return PFMM_EINVAL; }
    if (p.m_t < 0 || p.m_t > 16 || p.m_x < 0 || p.m_x > 16) { msg = "degrees must be in [0,16]"; return PFMM_EINVAL; }
    if (p.n_max < 1) { msg = "n_max must be >= 1"; return PFMM_EINVAL; }
    if (!(p.c_st > 0) || !std::isfinite(p.c_st)) { msg = "c_st must be > 0"; return PFMM_EINVAL; }
    if (p.n_tr < -1) { msg = "n_tr must be >= -1"; return PFMM_EINVAL; }
    if (p.q_reg < 1 || p.q_reg > 16 || p.q_sing < 1 || p.q_sing > 16) { msg = "quadrature orders must be in [1,16]"; return PFMM_EINVAL; }
    if (p.precision != PFMM_FP64 && p.precision != PFMM_MIXED_FP32 && p.precision != PFMM_MIXED_BF16) {
        msg = "unknown precision";
        return PFMM_EINVAL;
    }
    if (p.operators & ~(PFMM_OP_V | PFMM_OP_K | PFMM_OP_K1)) { msg = "unknown operator bits"; return PFMM_EINVAL; }
    if ((p.operators & PFMM_OP_K1) && p.nearfield_mode == PFMM_NF_TOEPLITZ) {
        msg = "the p1 double layer needs the stored nearfield";
        return PFMM_EUNSUPPORTED;
    }
    if (p.nearfield_mode != PFMM_NF_STORED && p.nearfield_mode != PFMM_NF_TOEPLITZ) {
        msg = "unknown nearfield mode";
        return PFMM_EINVAL;
    }
    if (p.nearfield_gemm != 0 && p.nearfield_gemm != 1) { msg = "nearfield_gemm must be 0 or 1"; return PFMM_EINVAL; }
    for (int64_t i = 0; i < nv && p.check_finite; ++i)
        if (!finite3(V + 3 * i)) { msg = "non-finite vertex"; return PFMM_ENONFINITE; }
    for (int64_t i = 0; i <= E_t && p.check_finite; ++i)
        if (!std::isfinite(tn[i])) { msg = "non-finite time node"; return PFMM_ENONFINITE; }
    for (int64_t i = 0; i < 3 * nt; ++i)
        if (Tr[i] < 0 || Tr[i] >= nv) { msg = "triangle vertex index out of range"; return PFMM_EINVAL; }
    for (int64_t i = 0; i < E_t; ++i)
        if (!(tn[i + 1] > tn[i])) { msg = "time nodes must be strictly increasing"; return PFMM_EINVAL; }
    const double Ttot = tn[E_t] - tn[0];
    const double h = Ttot / (double)E_t;
    bool uniform_steps = true;
    for (int64_t i = 0; i < E_t; ++i)
        if (std::fabs((tn[i + 1] - tn[i]) - h) > 1e-12 * h) uniform_steps = false;
    if (!uniform_steps && p.nearfield_mode == PFMM_NF_TOEPLITZ) {
        msg = "the Toeplitz nearfield needs uniform time steps";
        return PFMM_EUNSUPPORTED;
    }

    P = Plan();
    P.uniform_steps = uniform_steps;
    P.E_x = (int)nt; P.E_t = (int)E_t; P.n_vert = (int)nv;
    P.alpha = p.alpha; P.T = Ttot; P.h = h;
    P.m_t = p.m_t; P.m_x = p.m_x; P.n_max = p.n_max; P.n_tr = p.n_tr;
    P.q_reg = p.q_reg; P.q_sing = p.q_sing; P.c_st = p.c_st;
    P.verts.assign(V, V + 3 * nv);
    P.tris.assign(Tr, Tr + 3 * nt);
    P.tnodes.assign(tn, tn + E_t + 1);

    // ------------------------------------------------------------ geometry
    const int E_x = P.E_x;
    P.area.resize(E_x); P.normal.resize(3 * E_x); P.centroid.resize(3 * E_x); P.maxedge.resize(E_x);
    for (int i = 0; i < E_x; ++i) {
        const double* a = &P.verts[3 * P.tris[3 * i]];
        const double* b = &P.verts[3 * P.tris[3 * i + 1]];
        const double* c = &P.verts[3 * P.tris[3 * i + 2]];
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        double a2 = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(a2 > 0)) { msg = "degenerate triangle " + std::to_string(i); return PFMM_EINVAL; }
        P.area[i] = 0.5 * a2;
        for (int j = 0; j < 3; ++j) {
            P.normal[3 * i + j] = n[j] / a2;
            P.centroid[3 * i + j] = (a[j] + b[j] + c[j]) / 3.0;
        }
        double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        double l2 = std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
        double e3[3] = {c[0] - b[0], c[1] - b[1], c[2] - b[2]};
        double l3 = std::sqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]);
        P.maxedge[i] = std::max(l1, std::max(l2, l3));
    }
    // closed, consistently oriented surface: every directed edge appears once
    // and its reverse appears once
    // (the triangle across each edge gives the edge adjacency)
    {
        std::unordered_map<uint64_t, int> dir;   // directed edge -> triangle
        dir.reserve(6 * nt);
        for (int i = 0; i < E_x; ++i)
            for (int e = 0; e < 3; ++e) {
                uint64_t a = (uint32_t)P.tris[3 * i + e], b = (uint32_t)P.tris[3 * i + (e + 1) % 3];
                if (!dir.emplace((a << 32) | b, i).second) { msg = "mesh is not consistently oriented (repeated directed edge)"; return PFMM_EINVAL; }
            }
        P.adj.assign(3 * (size_t)E_x, -1);
        for (int i = 0; i < E_x; ++i)
            for (int e = 0; e < 3; ++e) {
                uint64_t a = (uint32_t)P.tris[3 * i + e], b = (uint32_t)P.tris[3 * i + (e + 1) % 3];
                auto it = dir.find((b << 32) | a);
                if (it == dir.end()) { msg = "mesh is not closed (boundary edge)"; return PFMM_EINVAL; }
                P.adj[3 * i + e] = it->second;
            }
    }
    double lo[3], hi[3];
    for (int j = 0; j < 3; ++j) { lo[j] = P.verts[j]; hi[j] = P.verts[j]; }
    for (int i = 1; i < P.n_vert; ++i)
        for (int j = 0; j < 3; ++j) { lo[j] = std::min(lo[j], P.verts[3 * i + j]); hi[j] = std::max(hi[j], P.verts[3 * i + j]); }
    double ext = 0.0;
    for (int j = 0; j < 3; ++j) ext = std::max(ext, hi[j] - lo[j]);
    P.h0 = 0.5 * ext;
    for (int j = 0; j < 3; ++j) P.lo0[j] = 0.5 * (lo[j] + hi[j]) - P.h0;

    // ------------------------------------------------------------ Algorithm 1
    std::vector<std::vector<SlotBuild>> slots(1);
    slots[0].push_back(SlotBuild{{0, 0, 0}, {}, -1, 0});
    slots[0][0].tris.resize(E_x);
    std::iota(slots[0][0].tris.begin(), slots[0][0].tris.end(), 0);
    P.lev.emplace_back();
    {
        Level& L0 = P.lev[0];
        L0.lx = 0; L0.n_int = 1;
        L0.istart = {0}; L0.iend = {(int)E_t};
        L0.present = {1}; L0.leaf = {1};
    }
    for (int l = 0;; ++l) {
        if (l >= 40) { msg = "tree deeper than 40 levels"; return PFMM_EUNSUPPORTED; }
        Level& L = P.lev[l];
        const double hx = P.h0 / std::ldexp(1.0, L.lx);
        const double ht_next = Ttot / std::ldexp(1.0, l + 2);
        const bool temporal = hx * hx / (4.0 * P.alpha * ht_next) <= P.c_st;
        const int nxs = (int)slots[l].size();
        // refine decisions
        bool any = false;
        std::vector<uint8_t> slot_ref(nxs, 0), int_ref(L.n_int, 0);
        for (int xs = 0; xs < nxs; ++xs)
            for (int k = 0; k < L.n_int; ++k) {
                size_t id = (size_t)xs * L.n_int + k;
                if (!L.present[id]) continue;
                int steps = L.iend[k] - L.istart[k];
                int64_t nel = (int64_t)steps * (int64_t)slots[l][xs].tris.size();
                if (nel >= P.n_max && steps > 1) {
                    L.leaf[id] = 0;
                    slot_ref[xs] = 1;
                    int_ref[k] = 1;
                    any = true;
                }
            }
        if (!any) break;
        if (!temporal && L.lx >= 20) { msg = "spatial refinement deeper than 20"; return PFMM_EUNSUPPORTED; }
        L.rtype = temporal ? 0 : 1;
        Level C;
        C.lx = L.lx + (temporal ? 0 : 1);
        C.n_int = 2 * L.n_int;
        C.istart.assign(C.n_int, -1);
        C.iend.assign(C.n_int, -1);
        for (int k = 0; k < L.n_int; ++k) {
            if (!int_ref[k]) continue;
            int s0 = L.istart[k], s1 = L.iend[k], mid = split_node(tn, s0, s1, Ttot);
            C.istart[2 * k] = s0; C.iend[2 * k] = mid;
            C.istart[2 * k + 1] = mid; C.iend[2 * k + 1] = s1;
        }
        std::vector<SlotBuild> cs;
        std::vector<std::vector<int>> child_of(nxs);   // child slots of each parent slot
        for (int xs = 0; xs < nxs; ++xs) {
            if (!slot_ref[xs]) continue;
            const SlotBuild& S = slots[l][xs];
            if (temporal) {
                child_of[xs].push_back((int)cs.size());
                cs.push_back(SlotBuild{S.ix, S.tris, xs, 0});
            } else {
                double lox[3], mid[3];
                for (int j = 0; j < 3; ++j) { lox[j] = P.lo0[j] + S.ix[j] * (2.0 * hx); mid[j] = lox[j] + hx; }
                std::vector<int> part[8];
                for (int t : S.tris) {
                    const double* c = &P.centroid[3 * t];
                    int code = ((c[0] > mid[0]) << 2) | ((c[1] > mid[1]) << 1) | (c[2] > mid[2]);
                    part[code].push_back(t);
                }
                for (int oc = 0; oc < 8; ++oc) {
                    if (part[oc].empty()) continue;
                    std::array<int, 3> ix = {2 * S.ix[0] + ((oc >> 2) & 1), 2 * S.ix[1] + ((oc >> 1) & 1), 2 * S.ix[2] + (oc & 1)};
                    child_of[xs].push_back((int)cs.size());
                    cs.push_back(SlotBuild{ix, std::move(part[oc]), xs, oc});
                }
            }
        }
        C.present.assign(cs.size() * (size_t)C.n_int, 0);
        C.leaf.assign(cs.size() * (size_t)C.n_int, 1);
        for (int xs = 0; xs < nxs; ++xs)
            for (int k = 0; k < L.n_int; ++k) {
                size_t id = (size_t)xs * L.n_int + k;
                if (!L.present[id] || L.leaf[id]) continue;
                for (int c : child_of[xs])
                    for (int b = 0; b < 2; ++b) C.present[(size_t)c * C.n_int + 2 * k + b] = 1;
            }
        slots.push_back(std::move(cs));
        P.lev.push_back(std::move(C));
    }
    P.depth = (int)P.lev.size() - 1;

    // ------------------------------------------------------------ triangle order
    {
        const int Ltot = P.lev[P.depth].lx;
        std::vector<uint64_t> key(E_x, 0);
        for (int t = 0; t < E_x; ++t) {
            int ix[3] = {0, 0, 0}, lx = 0;
            uint64_t k = 0;
            const double* c = &P.centroid[3 * t];
            for (int l = 0; l < P.depth; ++l) {
                if (P.lev[l].rtype != 1) continue;
                double hx = P.h0 / std::ldexp(1.0, lx);
                int code = 0;
                for (int j = 0; j < 3; ++j) {
                    double lox = P.lo0[j] + ix[j] * (2.0 * hx);
                    int bit = c[j] > lox + hx;
                    ix[j] = 2 * ix[j] + bit;
                    code |= bit << (2 - j);
                }
                k = (k << 3) | (uint64_t)code;
                ++lx;
            }
            (void)Ltot;
            key[t] = k;
        }
        P.inv_sigma.resize(E_x);
        std::iota(P.inv_sigma.begin(), P.inv_sigma.end(), 0);
        std::stable_sort(P.inv_sigma.begin(), P.inv_sigma.end(), [&](int a, int b) { return key[a] < key[b]; });
        P.sigma.resize(E_x);
        for (int i = 0; i < E_x; ++i) P.sigma[P.inv_sigma[i]] = i;
        // slot ranges
        for (int l = 0; l <= P.depth; ++l) {
            Level& L = P.lev[l];
            const int nxs = (int)slots[l].size();
            L.ix.resize(nxs); L.tb.resize(nxs); L.te.resize(nxs); L.parent.resize(nxs); L.octant.resize(nxs);
            for (int xs = 0; xs < nxs; ++xs) {
                const SlotBuild& S = slots[l][xs];
                L.ix[xs] = S.ix; L.parent[xs] = S.parent; L.octant[xs] = S.octant;
                int mn = E_x, mx = -1;
                for (int t : S.tris) { mn = std::min(mn, P.sigma[t]); mx = std::max(mx, P.sigma[t]); }
                if (mx - mn + 1 != (int)S.tris.size()) { msg = "internal: spatial box not contiguous in sorted order"; return PFMM_EINVAL; }
                L.tb[xs] = mn; L.te[xs] = mx + 1;
            }
        }
    }

    // ------------------------------------------------------------ padding
    {
        std::vector<double> pad(P.depth + 1, 0.0);
        for (int l = 0; l <= P.depth; ++l) {
            Level& L = P.lev[l];
            const double hx = P.h0 / std::ldexp(1.0, L.lx);
            double pm = 0.0;
            for (int xs = 0; xs < L.nx(); ++xs) {
                double lox[3], hix[3];
                for (int j = 0; j < 3; ++j) { lox[j] = P.lo0[j] + L.ix[xs][j] * (2.0 * hx); hix[j] = lox[j] + 2.0 * hx; }
                for (int q = L.tb[xs]; q < L.te[xs]; ++q) {
                    int t = P.inv_sigma[q];
                    for (int v = 0; v < 3; ++v) {
                        const double* x = &P.verts[3 * P.tris[3 * t + v]];
                        for (int j = 0; j < 3; ++j) pm = std::max(pm, std::max(lox[j] - x[j], x[j] - hix[j]));
                    }
                }
            }
            pad[l] = (pm >= 1e-12 * P.h0) ? pm : 0.0;
        }
        for (int l = P.depth - 1; l >= 0; --l) pad[l] = std::max(pad[l], pad[l + 1]);
        for (int l = 0; l <= P.depth; ++l) {
            Level& L = P.lev[l];
            L.hx = P.h0 / std::ldexp(1.0, L.lx);
            L.pad = pad[l];
            L.H = L.hx + L.pad;
        }
    }

    // ------------------------------------------------------------ counts, uniformity
    for (int l = 0; l <= P.depth; ++l) {
        const Level& L = P.lev[l];
        for (size_t i = 0; i < L.present.size(); ++i)
            if (L.present[i]) { ++P.n_boxes; if (L.leaf[i]) ++P.n_leaves; }
    }
    // M2L time classes per level >= 2, and whether the level is uniform
    // (every interval present with one length, every slot in every interval,
    // leaf status independent of the interval)
    for (int l = 2; l <= P.depth; ++l) {
        Level& L = P.lev[l];
        const int len = L.iend[0] - L.istart[0];
        L.uniform = P.uniform_steps;
        for (int k = 0; k < L.n_int; ++k)
            if (L.istart[k] < 0 || L.iend[k] - L.istart[k] != len) L.uniform = false;
        for (size_t i = 0; i < L.present.size(); ++i)
            if (!L.present[i]) L.uniform = false;
        for (int xs = 0; xs < L.nx() && L.uniform; ++xs)
            for (int k = 1; k < L.n_int; ++k)
                if (L.leaf[(size_t)xs * L.n_int + k] != L.leaf[(size_t)xs * L.n_int]) L.uniform = false;
        // class key: (D, start_k - start_J, len_k, len_J), in steps for a
        // uniform grid, else as times rounded to 2^-40 T
        std::map<std::array<int64_t, 4>, int> ids;
        auto tq = [&](int a, int b) { return (int64_t)std::llround((tn[b] - tn[a]) / Ttot * 1099511627776.0); };
        for (int D = 2; D <= 3; ++D) {
            L.cls[D - 2].assign(L.n_int, -1);
            if (L.uniform && L.n_int > D) {
                // classes 0 and 1 are D = 2 and D = 3 (representatives k = D, J = 0)
                L.cls_rep.push_back({D, 0});
                L.cls_D.push_back(D);
            }
        }
        for (int k = 2; k < L.n_int; ++k)
            for (int D = 2; D <= 3; ++D) {
                const int J = k - D;
                if ((D == 3 && !(k & 1)) || J < 0 || L.istart[k] < 0 || L.istart[J] < 0) continue;
                if (L.uniform) { L.cls[D - 2][k] = D - 2; continue; }
                const std::array<int64_t, 4> key =
                    P.uniform_steps ? std::array<int64_t, 4>{D, L.istart[k] - L.istart[J], L.iend[k] - L.istart[k],
                                                             L.iend[J] - L.istart[J]}
                                    : std::array<int64_t, 4>{D, tq(L.istart[J], L.istart[k]), tq(L.istart[k], L.iend[k]),
                                                             tq(L.istart[J], L.iend[J])};
                auto it = ids.find(key);
                if (it == ids.end()) {
                    it = ids.emplace(key, (int)L.cls_rep.size()).first;
                    L.cls_rep.push_back({k, J});
                    L.cls_D.push_back(D);
                }
                L.cls[D - 2][k] = it->second;
            }
        P.max_time_classes = std::max(P.max_time_classes, (int)L.cls_rep.size());
    }
    P.has_far = P.depth >= 2;

    // ------------------------------------------------------------ coefficient order
    {
        const int m = P.m_x;
        P.Nk = binom(m + 3, 3);
        P.Nc = (P.m_t + 1) * P.Nk;
        std::vector<std::array<int, 3>> bydeg;
        for (int n = 0; n <= m; ++n)
            for (int k1 = n; k1 >= 0; --k1)
                for (int k2 = n - k1; k2 >= 0; --k2) bydeg.push_back({k1, k2, n - k1 - k2});
        P.kidx_k.resize(3 * P.Nk);
        for (int i = 0; i < P.Nk; ++i)
            for (int j = 0; j < 3; ++j) P.kidx_k[3 * i + j] = bydeg[i][j];
        P.coef_a.resize(P.Nc); P.coef_deg.resize(P.Nc); P.coef_k.resize(3 * P.Nc);
        int c = 0;
        for (int n = 0; n <= m; ++n) {
            int k0 = binom(n + 2, 3), ks = binom(n + 2, 2);
            for (int a = 0; a <= P.m_t; ++a)
                for (int i = 0; i < ks; ++i, ++c) {
                    P.coef_a[c] = a;
                    P.coef_deg[c] = n;
                    for (int j = 0; j < 3; ++j) P.coef_k[3 * c + j] = bydeg[k0 + i][j];
                }
        }
    }

    // ------------------------------------------------------------ neighbours per level
    auto close = [&](const std::array<int, 3>& a, const std::array<int, 3>& b) {
        if (P.n_tr < 0) return true;
        int d = std::max(std::abs(a[0] - b[0]), std::max(std::abs(a[1] - b[1]), std::abs(a[2] - b[2])));
        return d <= P.n_tr;
    };
    std::vector<std::vector<std::vector<int>>> nbr(P.depth + 1);
    for (int l = 0; l <= P.depth; ++l) {
        const Level& L = P.lev[l];
        nbr[l].resize(L.nx());
        for (int a = 0; a < L.nx(); ++a)
            for (int b = 0; b < L.nx(); ++b)
                if (close(L.ix[a], L.ix[b])) nbr[l][a].push_back(b);
    }

    // ------------------------------------------------------------ M2L pair count
    for (int l = 2; l <= P.depth; ++l) {
        const Level& L = P.lev[l];
        for (int xs = 0; xs < L.nx(); ++xs)
            for (int k = 0; k < L.n_int; ++k) {
                if (!L.box(xs, k) || k < 2) continue;
                int cand[2] = {k - 2, (k % 2) ? k - 3 : -1};
                for (int J : cand) {
                    if (J < 0 || L.istart[J] < 0) continue;
                    for (int ys : nbr[l][xs])
                        if (L.box(ys, J)) ++P.m2l_pairs;
                }
            }
    }

    // ------------------------------------------------------------ nearfield lists
    // NL(Z): leaf boxes of N(Z), needed for the children of non-leaf boxes.
    // A box is encoded as (l << 56) | (k << 28) | xs.
    auto enc = [](int l, int k, int xs) { return ((uint64_t)l << 56) | ((uint64_t)k << 28) | (uint64_t)xs; };
    std::vector<std::unordered_map<uint64_t, std::vector<uint64_t>>> NL(P.depth + 1);
    std::map<std::pair<int, std::vector<int>>, int> set_ids;   // (level, sorted slots) -> set
    auto make_set = [&](int l, std::vector<int> xsl) {
        std::sort(xsl.begin(), xsl.end());
        auto key = std::make_pair(l, xsl);
        auto it = set_ids.find(key);
        if (it != set_ids.end()) return it->second;
        std::vector<int> pos;
        const Level& L = P.lev[l];
        for (int xs : xsl)
            for (int q = L.tb[xs]; q < L.te[xs]; ++q) pos.push_back(q);
        std::sort(pos.begin(), pos.end());
        int id = (int)P.set_off.size();
        P.set_off.push_back((int)P.set_pos.size());
        P.set_size.push_back((int)pos.size());
        P.set_pos.insert(P.set_pos.end(), pos.begin(), pos.end());
        set_ids.emplace(std::move(key), id);
        return id;
    };
    std::map<std::array<int, 3>, int> group_of;   // (l, xs, row chunk) -> group
    for (int l = 0; l <= P.depth; ++l) {
        const Level& L = P.lev[l];
        for (int xs = 0; xs < L.nx(); ++xs)
            for (int k = 0; k < L.n_int; ++k) {
                if (!L.box(xs, k)) continue;
                const bool lf = L.is_leaf(xs, k);
                // same-level part of N(Z), grouped by source interval
                std::vector<std::pair<int, std::vector<int>>> same;   // (J, slots)
                int Js[2] = {k == 0 ? 0 : k - 1, k == 0 ? -1 : k};
                for (int J : Js) {
                    if (J < 0 || L.istart[J] < 0) continue;
                    std::vector<int> ys;
                    for (int y : nbr[l][xs])
                        if (L.box(y, J)) ys.push_back(y);
                    if (!ys.empty()) same.emplace_back(J, std::move(ys));
                }
                const std::vector<uint64_t>* pnl = nullptr;
                if (l > 0) {
                    const Level& Lp = P.lev[l - 1];
                    auto it = NL[l - 1].find(enc(l - 1, k >> 1, L.parent[xs]));
                    if (it != NL[l - 1].end()) pnl = &it->second;
                    (void)Lp;
                }
                if (!lf) {
                    std::vector<uint64_t> nl;
                    for (auto& s : same)
                        for (int y : s.second)
                            if (L.is_leaf(y, s.first)) nl.push_back(enc(l, s.first, y));
                    if (pnl) nl.insert(nl.end(), pnl->begin(), pnl->end());
                    NL[l][enc(l, k, xs)] = std::move(nl);
                    continue;
                }
                // leaf: build its rects
                LeafRec R;
                R.l = l; R.xs = xs; R.k = k;
                R.s0 = L.istart[k]; R.s1 = L.iend[k];
                R.tb = L.tb[xs]; R.te = L.te[xs];
                R.rect0 = (int)P.rects.size();
                for (auto& s : same) {
                    int set = make_set(l, s.second);
                    P.rects.push_back(Rect{L.istart[s.first], L.iend[s.first], set});
                }
                if (pnl) {
                    std::map<std::pair<int, int>, std::vector<int>> byint;   // (level, k) -> slots
                    for (uint64_t b : *pnl) {
                        int bl = (int)(b >> 56), bk = (int)((b >> 28) & 0xfffffff), bx = (int)(b & 0xfffffff);
                        byint[{bl, bk}].push_back(bx);
                    }
                    for (auto& kv : byint) {
                        const Level& Lb = P.lev[kv.first.first];
                        int set = make_set(kv.first.first, kv.second);
                        P.rects.push_back(Rect{Lb.istart[kv.first.second], Lb.iend[kv.first.second], set});
                    }
                }
                R.rect1 = (int)P.rects.size();
                // The nearfield kernels give each row of a leaf one lane of a
                // wave: a leaf with more than 64 triangles (one whose interval
                // has a single step, where Algorithm 1 stops refining) becomes
                // several row chunks of at most 64 triangles, each with its own
                // assembly group (same sources, its own rows of the table).
                const int nch = (R.te - R.tb + 63) / 64;
                for (int ch = 0; ch < nch; ++ch) {
                    LeafRec Rc = R;
                    Rc.tb = R.tb + (int)((int64_t)(R.te - R.tb) * ch / nch);
                    Rc.te = R.tb + (int)((int64_t)(R.te - R.tb) * (ch + 1) / nch);
                    auto g = group_of.find({l, xs, ch});
                    if (g == group_of.end()) {
                        AsmGroup G;
                        G.l = l; G.xs = xs; G.tb = Rc.tb; G.te = Rc.te; G.dmax = 0;
                        G.uoff = 0; G.usize = 0; G.toff = 0; G.mapoff = 0;
                        int id = (int)P.groups.size();
                        P.groups.push_back(G);
                        g = group_of.emplace(std::array<int, 3>{l, xs, ch}, id).first;
                    }
                    Rc.group = g->second;
                    P.leaves.push_back(Rc);
                }
            }
    }

    // ------------------------------------------------------------ row groups
    int64_t boff = 0;
    for (size_t li = 0; li < P.leaves.size(); ++li) {
        const LeafRec& R = P.leaves[li];
        const int nX = R.te - R.tb;
        for (int kt = R.s0; kt < R.s1; ++kt) {
            int64_t nc = 0;
            for (int r = R.rect0; r < R.rect1; ++r) {
                const Rect& q = P.rects[r];
                int ns = std::min(q.j1, kt + 1) - q.j0;
                if (ns > 0) nc += (int64_t)ns * P.set_size[q.set];
            }
            P.rows.push_back(RowGroup{(int)li, kt, boff, nc});
            boff += nc * nX;
        }
    }
    P.near_entries = boff;
    // K_h entries between coplanar panels vanish ((x - y) . n_y = 0): count
    // the others.  Panels are grouped by their plane (unit normal and offset,
    // rounded); per source set, a histogram of its planes.
    {
        std::map<std::array<int64_t, 4>, int> plane_ids;
        std::vector<int> plane(E_x);
        for (int q = 0; q < E_x; ++q) {
            const int t = P.inv_sigma[q];
            const double* n = &P.normal[3 * t];
            const double* c = &P.centroid[3 * t];
            const double d = n[0] * c[0] + n[1] * c[1] + n[2] * c[2];
            std::array<int64_t, 4> key = {std::llround(n[0] * 1e9), std::llround(n[1] * 1e9), std::llround(n[2] * 1e9),
                                          std::llround(d / P.h0 * 1e9)};
            plane[q] = plane_ids.emplace(key, (int)plane_ids.size()).first->second;
        }
        std::vector<std::map<int, int>> set_planes(P.set_off.size());
        for (size_t st = 0; st < P.set_off.size(); ++st)
            for (int i = 0; i < P.set_size[st]; ++i) ++set_planes[st][plane[P.set_pos[P.set_off[st] + i]]];
        int64_t nz = 0;
        for (const LeafRec& R : P.leaves) {
            for (int r = R.rect0; r < R.rect1; ++r) {
                const Rect& q = P.rects[r];
                // non-coplanar (target, source) panel pairs of this rectangle
                int64_t pairs = 0;
                for (int tq = R.tb; tq < R.te; ++tq) {
                    auto it = set_planes[q.set].find(plane[tq]);
                    pairs += P.set_size[q.set] - (it == set_planes[q.set].end() ? 0 : it->second);
                }
                // causal step pairs (k_t >= j_t) of the leaf's steps and the rectangle's
                int64_t steps = 0;
                for (int kt = R.s0; kt < R.s1; ++kt) steps += std::max(0, std::min(q.j1, kt + 1) - q.j0);
                nz += pairs * steps;
            }
        }
        P.near_nonzero_K = nz;
    }

    // ------------------------------------------------------------ assembly groups
    {
        std::vector<std::vector<int>> gsets(P.groups.size());
        for (const LeafRec& R : P.leaves) {
            AsmGroup& G = P.groups[R.group];
            for (int r = R.rect0; r < R.rect1; ++r) {
                const Rect& q = P.rects[r];
                if (q.j0 > R.s1 - 1) continue;
                G.dmax = std::max(G.dmax, R.s1 - 1 - q.j0);
                gsets[R.group].push_back(q.set);
            }
        }
        int64_t toff = 0;
        for (size_t g = 0; g < P.groups.size(); ++g) {
            AsmGroup& G = P.groups[g];
            std::vector<int>& ss = gsets[g];
            std::sort(ss.begin(), ss.end());
            ss.erase(std::unique(ss.begin(), ss.end()), ss.end());
            std::vector<int> u;
            for (int s : ss) u.insert(u.end(), P.set_pos.begin() + P.set_off[s], P.set_pos.begin() + P.set_off[s] + P.set_size[s]);
            std::sort(u.begin(), u.end());
            u.erase(std::unique(u.begin(), u.end()), u.end());
            G.uoff = (int64_t)P.upos.size();
            G.usize = (int)u.size();
            P.upos.insert(P.upos.end(), u.begin(), u.end());
            G.toff = toff;
            toff += (int64_t)(G.dmax + 1) * (G.te - G.tb) * G.usize;
            G.mapoff = (int64_t)g * E_x;
        }
        // steps of different lengths: no Toeplitz reuse, every stored entry
        // is integrated on its own (no distinct-integral table)
        P.table_size = P.uniform_steps ? toff : 0;
        P.distinct = P.uniform_steps ? toff : P.near_entries;
        P.umap.assign(P.groups.size() * (size_t)E_x, -1);
        for (size_t g = 0; g < P.groups.size(); ++g) {
            const AsmGroup& G = P.groups[g];
            for (int i = 0; i < G.usize; ++i) P.umap[G.mapoff + P.upos[G.uoff + i]] = i;
        }
    }

    // ------------------------------------------------------------ touching pairs
    {
        std::vector<std::vector<int>> vt(P.n_vert);
        for (int t = 0; t < E_x; ++t)
            for (int v = 0; v < 3; ++v) vt[P.tris[3 * t + v]].push_back(t);
        for (size_t g = 0; g < P.groups.size(); ++g) {
            const AsmGroup& G = P.groups[g];
            for (int q = G.tb; q < G.te; ++q) {
                int kx = P.inv_sigma[q];
                std::vector<int> nb;
                for (int v = 0; v < 3; ++v)
                    for (int j : vt[P.tris[3 * kx + v]]) nb.push_back(j);
                std::sort(nb.begin(), nb.end());
                nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
                for (int j : nb) {
                    int u = P.umap[G.mapoff + P.sigma[j]];
                    if (u < 0) continue;
                    int ns = 0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) ns += P.tris[3 * kx + a] == P.tris[3 * j + b];
                    P.touch.push_back(TouchPair{(int)g, q - G.tb, u, ns});
                }
            }
        }
        std::stable_sort(P.touch.begin(), P.touch.end(), [](const TouchPair& a, const TouchPair& b) { return a.nshared > b.nshared; });
    }
    return PFMM_OK;
}

void build_p1_layout(Plan& P) {
    Plan::P1Layout& L = P.p1;
    L = Plan::P1Layout();
    L.built = true;
    for (size_t st = 0; st < P.set_off.size(); ++st) {
        L.set_off.push_back((int)L.set_pos.size());
        L.set_size.push_back(3 * P.set_size[st]);
        for (int i = 0; i < P.set_size[st]; ++i)
            for (int c = 0; c < 3; ++c) L.set_pos.push_back(3 * P.set_pos[P.set_off[st] + i] + c);
    }
    int64_t boff = 0;
    for (const RowGroup& R : P.rows) {
        L.boff.push_back(boff);
        boff += 3 * R.ncols * (P.leaves[R.leaf].te - P.leaves[R.leaf].tb);
    }
    L.near_entries = boff;
    int64_t toff = 0;
    for (const AsmGroup& G : P.groups) {
        L.toff.push_back(toff);
        if (P.uniform_steps) toff += (int64_t)(G.dmax + 1) * (G.te - G.tb) * 3 * G.usize;
    }
    L.table_size = toff;
    L.umap.assign(P.groups.size() * (size_t)3 * P.E_x, -1);
    for (size_t g = 0; g < P.groups.size(); ++g) {
        const AsmGroup& G = P.groups[g];
        for (int i = 0; i < G.usize; ++i)
            for (int c = 0; c < 3; ++c)
                L.umap[g * (size_t)3 * P.E_x + 3 * P.upos[G.uoff + i] + c] = 3 * i + c;
    }
}

}  // namespace pfmm
