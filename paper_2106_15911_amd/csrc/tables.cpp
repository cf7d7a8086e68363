// Expansion tables (Section 3.1 and 3.4) computed on the host from the plan.
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <map>

namespace pfmm {

namespace {

void cheb_T(int kmax, double x, double* out) {
    out[0] = 1.0;
    if (kmax >= 1) out[1] = x;
    for (int k = 2; k <= kmax; ++k) out[k] = 2.0 * x * out[k - 1] - out[k - 2];
}

void cheb_dT(int kmax, double x, double* out) {
    // T_k' = k U_{k-1}
    double U[40];
    U[0] = 1.0;
    if (kmax >= 1) U[1] = 2.0 * x;
    for (int k = 2; k <= kmax; ++k) U[k] = 2.0 * x * U[k - 1] - U[k - 2];
    out[0] = 0.0;
    for (int k = 1; k <= kmax; ++k) out[k] = k * U[k - 1];
}

// Lagrange basis at transformed Chebyshev nodes of the interval [ta, tb].
void lagrange(const std::vector<double>& xi, double ta, double tb, double t, double* L) {
    const int m = (int)xi.size();
    std::vector<double> nodes(m);
    for (int k = 0; k < m; ++k) nodes[k] = 0.5 * (ta + tb) + 0.5 * (tb - ta) * xi[k];
    for (int b = 0; b < m; ++b) {
        double v = 1.0;
        for (int k = 0; k < m; ++k)
            if (k != b) v = v * (t - nodes[k]) / (nodes[b] - nodes[k]);
        L[b] = v;
    }
}

double lam(int k) { return k == 0 ? 1.0 : 2.0; }

}  // namespace

void build_far_tables(const Plan& P, FarTables& F, bool with_p1) {
    F = FarTables();
    const int mt = P.m_t, mx = P.m_x, nt1 = mt + 1, nx1 = mx + 1, Nk = P.Nk;
    const std::vector<double> xt = cheb_nodes(mt), xx = cheb_nodes(mx);
    F.lv.resize(P.depth + 1);

    // temporal quadrature for A_t: same point count as needed for exactness
    std::vector<double> gt, wt;
    gauss_legendre01(mt / 2 + 2, gt, wt);
    // triangle rule for A_x: collapsed Gauss, exact to degree >= m_x
    std::vector<double> gx, wx;
    gauss_legendre01(mx / 2 + 2, gx, wx);
    const int qx = (int)gx.size();

    for (int l = 2; l <= P.depth; ++l) {
        const Level& L = P.lev[l];
        FarLevel& FL = F.lv[l];
        FL.l = l;
        FL.nx = L.nx();
        FL.n_int = L.n_int;
        FL.istart.assign(L.n_int, 0);
        FL.ilen.assign(L.n_int, 0);
        for (int k = 0; k < L.n_int; ++k)
            if (L.istart[k] >= 0) { FL.istart[k] = L.istart[k]; FL.ilen[k] = L.iend[k] - L.istart[k]; }
        FL.inner.assign((size_t)L.nx() * L.n_int, 0);
        for (size_t i = 0; i < L.present.size(); ++i) FL.inner[i] = L.present[i] && !L.leaf[i];
        // ---------------- leaves, A_t, A_x
        for (int xs = 0; xs < L.nx(); ++xs) {
            bool any = false;
            for (int k = 0; k < L.n_int; ++k) any = any || (L.box(xs, k) && L.is_leaf(xs, k));
            if (!any) continue;
            FL.leaf_xs.push_back(xs);
            for (int k = 0; k < L.n_int; ++k) FL.leaf.push_back(L.box(xs, k) && L.is_leaf(xs, k) ? 1 : 0);
        }
        if (!FL.leaf_xs.empty()) {
            // one row per time step (E_t rows): the integrals of the Lagrange
            // basis of the step's interval on this level (zero where the
            // interval is absent)
            FL.at_off = (int64_t)F.At.size();
            F.At.resize(F.At.size() + (size_t)P.E_t * nt1, 0.0);
            for (int k = 0; k < L.n_int; ++k) {
                if (L.istart[k] < 0) continue;
                const double ta = P.tnodes[L.istart[k]], tb = P.tnodes[L.iend[k]];
                for (int j = L.istart[k]; j < L.iend[k]; ++j) {
                    const double t0 = P.tnodes[j], t1 = P.tnodes[j + 1];
                    std::vector<double> row(nt1, 0.0), Lb(nt1);
                    for (size_t q = 0; q < gt.size(); ++q) {
                        lagrange(xt, ta, tb, t0 + (t1 - t0) * gt[q], Lb.data());
                        for (int a = 0; a < nt1; ++a) row[a] += Lb[a] * (wt[q] * (t1 - t0));
                    }
                    std::copy(row.begin(), row.end(), F.At.begin() + FL.at_off + (int64_t)j * nt1);
                }
            }
            for (size_t li = 0; li < FL.leaf_xs.size(); ++li)
                for (int r0 = 0; r0 < L.te[FL.leaf_xs[li]] - L.tb[FL.leaf_xs[li]]; r0 += 64) {
                    FL.chunk_li.push_back((int)li);
                    FL.chunk_r0.push_back(r0);
                }
            for (int xs : FL.leaf_xs) {
                FL.ax_off.push_back((int64_t)F.Ax.size());
                double lo[3];
                for (int j = 0; j < 3; ++j) lo[j] = P.lo0[j] + L.ix[xs][j] * (2.0 * L.hx) - L.pad;
                const double H = L.H;
                for (int q = L.tb[xs]; q < L.te[xs]; ++q) {
                    const int t = P.inv_sigma[q];
                    const double* A = &P.verts[3 * P.tris[3 * t]];
                    const double* B = &P.verts[3 * P.tris[3 * t + 1]];
                    const double* C = &P.verts[3 * P.tris[3 * t + 2]];
                    const double* n = &P.normal[3 * t];
                    std::vector<double> rowV(Nk, 0.0), rowK(Nk, 0.0), rowK1(3 * Nk, 0.0);
                    for (int i = 0; i < qx; ++i)
                        for (int jq = 0; jq < qx; ++jq) {
                            const double s = gx[i], tt = gx[i] * gx[jq];
                            const double wq = wx[i] * wx[jq] * gx[i] * 2.0 * P.area[t];
                            const double lam[3] = {1.0 - s, s - tt, tt};   // barycentric coordinates
                            double Tj[3][40], dTj[3][40];
                            for (int d = 0; d < 3; ++d) {
                                double y = A[d] + s * (B[d] - A[d]) + tt * (C[d] - B[d]);
                                double yh = (y - lo[d]) / H - 1.0;
                                cheb_T(mx, yh, Tj[d]);
                                cheb_dT(mx, yh, dTj[d]);
                                for (int k = 0; k <= mx; ++k) dTj[d][k] /= H;
                            }
                            for (int c = 0; c < Nk; ++c) {
                                const int k1 = P.kidx_k[3 * c], k2 = P.kidx_k[3 * c + 1], k3 = P.kidx_k[3 * c + 2];
                                rowV[c] += wq * Tj[0][k1] * Tj[1][k2] * Tj[2][k3];
                                const double dk = wq * P.alpha * (n[0] * dTj[0][k1] * Tj[1][k2] * Tj[2][k3]
                                                                  + n[1] * Tj[0][k1] * dTj[1][k2] * Tj[2][k3]
                                                                  + n[2] * Tj[0][k1] * Tj[1][k2] * dTj[2][k3]);
                                rowK[c] += dk;
                                if (with_p1)
                                    for (int v = 0; v < 3; ++v) rowK1[v * Nk + c] += lam[v] * dk;
                            }
                        }
                    F.Ax.insert(F.Ax.end(), rowV.begin(), rowV.end());
                    F.AxK.insert(F.AxK.end(), rowK.begin(), rowK.end());
                    if (with_p1) F.AxK1.insert(F.AxK1.end(), rowK1.begin(), rowK1.end());
                }
            }
        }
        // ---------------- q^(t), q^(x) with this level as the child level
        if (l >= 3) {
            const Level& Lp = P.lev[l - 1];
            FL.qt_off = (int64_t)F.qt.size();
            for (int k = 0; k < L.n_int; ++k) {
                const int kp = k >> 1;
                if (L.istart[k] < 0 || Lp.istart[kp] < 0) {   // absent interval: no re-expansion
                    F.qt.insert(F.qt.end(), (size_t)nt1 * nt1, 0.0);
                    continue;
                }
                const double ca = P.tnodes[L.istart[k]], cb = P.tnodes[L.iend[k]];
                const double pa = P.tnodes[Lp.istart[kp]], pb = P.tnodes[Lp.iend[kp]];
                std::vector<double> Lb(nt1);
                for (int ac = 0; ac < nt1; ++ac) {
                    const double tc = 0.5 * (ca + cb) + 0.5 * (cb - ca) * xt[ac];
                    lagrange(xt, pa, pb, tc, Lb.data());
                    for (int ap = 0; ap < nt1; ++ap) F.qt.push_back(Lb[ap]);
                }
            }
            FL.qx_off = (int64_t)F.qx.size();
            double Tn[40][40];
            for (int n = 0; n <= mx; ++n) cheb_T(mx, xx[n], Tn[n]);     // Tn[n][kappa]
            for (int xs = 0; xs < L.nx(); ++xs) {
                const int ps = L.parent[xs];
                for (int d = 0; d < 3; ++d) {
                    const double lc = P.lo0[d] + L.ix[xs][d] * (2.0 * L.hx) - L.pad;
                    const double lp = P.lo0[d] + Lp.ix[ps][d] * (2.0 * Lp.hx) - Lp.pad;
                    double Tp[40][40];
                    for (int n = 0; n <= mx; ++n) {
                        const double yc = lc + L.H * (1.0 + xx[n]);
                        cheb_T(mx, (yc - lp) / Lp.H - 1.0, Tp[n]);
                    }
                    for (int ka = 0; ka <= mx; ++ka)
                        for (int nu = 0; nu <= mx; ++nu) {
                            double s = 0.0;
                            for (int n = 0; n <= mx; ++n) s += Tn[n][ka] * Tp[n][nu];
                            F.qx.push_back(lam(ka) / (mx + 1) * s);
                        }
                }
            }
        }
        // ---------------- children (level l+1) of each slot, for M2M
        FL.children_ptr.assign(L.nx() + 1, 0);
        if (l < P.depth) {
            const Level& Lc = P.lev[l + 1];
            std::vector<std::vector<int>> ch(L.nx());
            for (int xs = 0; xs < Lc.nx(); ++xs) ch[Lc.parent[xs]].push_back(xs);
            for (int xs = 0; xs < L.nx(); ++xs) {
                FL.children_ptr[xs + 1] = FL.children_ptr[xs] + (int)ch[xs].size();
                FL.children.insert(FL.children.end(), ch[xs].begin(), ch[xs].end());
            }
        }
        // ---------------- M2L interaction structure and 1D coefficient tables
        std::map<std::array<int, 3>, int> offid;
        std::vector<std::array<int, 3>> offs;
        FL.m2l_ptr.assign(L.nx() + 1, 0);
        for (int xs = 0; xs < L.nx(); ++xs) {
            for (int ys = 0; ys < L.nx(); ++ys) {
                std::array<int, 3> o = {L.ix[xs][0] - L.ix[ys][0], L.ix[xs][1] - L.ix[ys][1], L.ix[xs][2] - L.ix[ys][2]};
                if (P.n_tr >= 0 && std::max(std::abs(o[0]), std::max(std::abs(o[1]), std::abs(o[2]))) > P.n_tr) continue;
                auto it = offid.find(o);
                int id;
                if (it == offid.end()) { id = (int)offs.size(); offid.emplace(o, id); offs.push_back(o); }
                else id = it->second;
                FL.m2l_src.push_back(ys);
                FL.m2l_cls.push_back(id);
            }
            FL.m2l_ptr[xs + 1] = (int)FL.m2l_src.size();
        }
        FL.n_off = (int)offs.size();
        const int R = (P.n_tr >= 0) ? P.n_tr : (1 << L.lx) - 1;
        const int nR = 2 * R + 1;
        // one set of tables per time class (for uniform levels: class c is the
        // time offset D = c + 2, representative pair (D, 0)); at least two
        // classes are reserved so that uniform levels with fewer intervals keep
        // the [D - 2] layout of the batched-in-time kernels
        FL.ncls = std::max(2, (int)L.cls_rep.size());
        FL.e1_off = (int64_t)F.E1.size();
        FL.cab_off = (int64_t)F.Cab.size();
        F.E1.resize(F.E1.size() + (size_t)FL.ncls * nR * nt1 * nt1 * nx1 * nx1, 0.0);
        F.Cab.resize(F.Cab.size() + (size_t)FL.ncls * nt1 * nt1, 0.0);
        double Tn[40][40];
        for (int n = 0; n <= mx; ++n) cheb_T(mx, xx[n], Tn[n]);
        for (int cl = 0; cl < (int)L.cls_rep.size(); ++cl) {
            const int k = L.cls_rep[cl][0], J = L.cls_rep[cl][1];   // representative interval pair
            const int D = cl + 2;   // table slot: (D - 2) = class
            const double ia = P.tnodes[L.istart[k]], ib = P.tnodes[L.iend[k]];
            const double ja = P.tnodes[L.istart[J]], jb = P.tnodes[L.iend[J]];
            for (int a = 0; a < nt1; ++a)
                for (int b = 0; b < nt1; ++b) {
                    const double tI = 0.5 * (ia + ib) + 0.5 * (ib - ia) * xt[b];
                    const double tJ = 0.5 * (ja + jb) + 0.5 * (jb - ja) * xt[a];
                    const double dt = tI - tJ;
                    F.Cab[FL.cab_off + ((size_t)(D - 2) * nt1 + a) * nt1 + b] = std::pow(4.0 * M_PI * P.alpha * dt, -1.5);
                    const double dab = 4.0 * P.alpha * dt / (L.H * L.H);
                    for (int oi = 0; oi < nR; ++oi) {
                        const int o = oi - R;
                        // r = (lower corner of target - lower corner of source) / H
                        const double cX = P.lo0[0] + o * (2.0 * L.hx) - L.pad;
                        const double cY = P.lo0[0] + 0 * (2.0 * L.hx) - L.pad;
                        const double r = (cX - cY) / L.H;
                        double* E = &F.E1[FL.e1_off + ((((size_t)(D - 2) * nR + oi) * nt1 + a) * nt1 + b) * nx1 * nx1];
                        for (int ka = 0; ka <= mx; ++ka)
                            for (int nu = 0; nu <= mx; ++nu) {
                                double s = 0.0;
                                for (int n = 0; n <= mx; ++n)
                                    for (int m = 0; m <= mx; ++m) {
                                        const double z = r + xx[n] - xx[m];
                                        s += std::exp(-z * z / dab) * Tn[n][nu] * Tn[m][ka];
                                    }
                                E[ka * nx1 + nu] = lam(ka) * lam(nu) / ((mx + 1.0) * (mx + 1.0)) * s;
                            }
                    }
                }
        }
        for (auto& o : offs) { FL.off3.push_back(o[0]); FL.off3.push_back(o[1]); FL.off3.push_back(o[2]); }
        FL.R = R;
    }
    // ---------------- operator chunking (rows in coefficient order)
    const int Nc = P.Nc;
    F.n_chunks = (Nc + F.chunk - 1) / F.chunk;
    F.chunk_cols.resize(F.n_chunks);
    F.chunk_off.resize(F.n_chunks + 1);
    F.chunk_off[0] = 0;
    for (int j = 0; j < F.n_chunks; ++j) {
        const int dmin = P.coef_deg[j * F.chunk];
        F.chunk_cols[j] = nt1 * binom(mx - dmin + 3, 3);
        F.chunk_off[j + 1] = F.chunk_off[j] + (int64_t)F.chunk_cols[j] * F.chunk;
    }
    F.op_size = F.chunk_off[F.n_chunks];
}

}  // namespace pfmm
