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

// Stream-ordered applies without argument checks (natural order in and out).
pfmm_status tree_apply(pfmm_tree* t, bool K, const double* x, double* y, hipStream_t st);

}  // namespace pfmm
