// Library-internal accessors shared between the translation units of
// libpfmm.so (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "pfmm.h"

namespace pfmm {

// Record `msg` as the thread's last error and return `s`.
pfmm_status set_error(pfmm_status s, const std::string& msg);

int tree_device(const pfmm_tree* t);
int64_t tree_dofs(const pfmm_tree* t);            // E_t * E_x
int64_t tree_triangles(const pfmm_tree* t);       // E_x
bool tree_has(const pfmm_tree* t, int op);        // PFMM_OP_V / PFMM_OP_K built
// The p0 x p0 mass matrix is diagonal, |gamma_kx| (t_{kt+1} - t_kt): the
// triangle areas (device, E_x doubles, natural order) and the step lengths
// (device, E_t doubles).
const double* tree_area(const pfmm_tree* t);
const double* tree_steps(const pfmm_tree* t);
bool tree_uniform_steps(const pfmm_tree* t);

// Stage profiling (pfmm_profile_enable) switched on.
bool tree_profiling(const pfmm_tree* t);

// Farfield precision of the next applies (pfmm_precision).
int tree_precision(const pfmm_tree* t);

// Diagonal of V_h per triangle (same triangle, same step; natural order,
// device, E_x doubles) read from the nearfield's distinct integrals.
pfmm_status tree_near_diag(pfmm_tree* t, double* d_dev, hipStream_t st);

// Learned preconditioner (precond.hip): z = s N(x(v)) over a whole vector,
// and training on pairs (R[p], E[p]) with V_h E[p] = R[p].  part: device
// scratch of precond_scratch_doubles(n) doubles for precond_apply.
size_t precond_scratch_doubles(int64_t n);
pfmm_status precond_apply(const pfmm_precond* pc, const double* v, double* z, const double* D, const int* adj,
                          int64_t ex, int64_t n, double* part, hipStream_t st);
pfmm_status precond_fit(pfmm_precond* pc, const double* R, const double* E, int npair, const double* D,
                        const int* adj, int64_t ex, int64_t n, int steps, int batch, float lr, uint64_t seed,
                        hipStream_t st);

// Device triangle orderings: sigma[natural] = sorted position, inv_sigma[position] = natural.
const int* tree_sigma(const pfmm_tree* t);
const int* tree_inv_sigma(const pfmm_tree* t);
// Device edge adjacency: adj[3 k + e] = triangle across edge e of triangle k (natural order).
const int* tree_adjacency(const pfmm_tree* t);
float precond_last_loss(const pfmm_precond* pc);

// Stream-ordered applies without argument checks (natural order in and out).
pfmm_status tree_apply(pfmm_tree* t, bool K, const double* x, double* y, hipStream_t st);
// The p1 double layer (x: n_steps x n_vertices) and the mesh it needs.
pfmm_status tree_apply_p1(pfmm_tree* t, const double* x, double* y, hipStream_t st);
int tree_vertices(const pfmm_tree* t);
const int* tree_tris(const pfmm_tree* t);   // device, natural order, n_triangles x 3

// The apply in two phases around a batched M2L: phase 1 permutes, runs the
// nearfield, the upward pass and the M2L of the levels with equal intervals
// (the others prepared); phase 2 runs L2L, L2T and the final permutation.
pfmm_status tree_apply_phase(pfmm_tree* t, bool K, const double* x, double* y, hipStream_t st, int phase);

// Cross-problem M2L: the class-aware M2L of the levels with unequal or
// missing intervals of all trees of a batch in one launch per (precision,
// time offset).  create returns *out = NULL when the trees cannot share a
// launch (different degrees, no matrix-core path) or have no such level;
// prepare fills the unit descriptors for the trees' current precisions
// (synchronous; outside graph capture); launch enqueues the launches.
struct BatchM2L;
pfmm_status batch_m2l_create(pfmm_tree* const* trees, int n, BatchM2L** out);
pfmm_status batch_m2l_prepare(BatchM2L* b);
pfmm_status batch_m2l_launch(BatchM2L* b, hipStream_t st);
void batch_m2l_destroy(BatchM2L* b);

// The tree's mesh and time grid on the device (natural triangle order).
struct TreeGeom {
    const double* verts;     // n_vertices x 3
    const int* tris;         // n_tri x 3
    const double* area;      // n_tri
    const double* normal;    // n_tri x 3 (unit, outward)
    const double* tnodes;    // n_steps + 1
    int n_tri, n_steps;
    double alpha, t_first, t_last;
};
pfmm_status tree_geometry(pfmm_tree* t, TreeGeom* out);

}  // namespace pfmm
