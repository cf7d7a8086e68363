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
// Diagonal of the p0 x p0 mass matrix per triangle, |gamma_k| h_t (device, E_x doubles).
const double* tree_mass(const pfmm_tree* t);

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

}  // namespace pfmm
