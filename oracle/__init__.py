"""CPU FP64 oracle for the space-time FMM of the heat equation.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately simple
implementation of what the GPU library computes, used to check it.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never does.

Sources (Watschinger, Merta, Of, Zapletal, "A parallel fast multipole method
for a space-time boundary element method for the heat equation"):

* Section 2 — heat kernel (eq. heat_kernel), p0 x p0 Galerkin matrix V_h and
  its block lower-triangular structure; the double-layer operator K; the
  representation formula u = V~w - Wu at interior points.
* Section 3.1 — kernel expansion (eqs. kernel_approx, exp_coeffs_3d,
  def_r_j, def_d_ab, exp_coeffs_1d), box-size coupling (eq. rel_h_t_h_x).
* Section 3.2 — Algorithm 1 (box cluster tree), split points and padding.
* Section 3.3 — temporal and space-time nearfield / interaction lists
  (eqs. 03:ILtemp, 03:Iarea, def_st_nearfield, def_st_interaction_list).
* Section 3.4 — S2M, M2L, L2T, temporal and space-time M2M (and their
  transposes, L2L), Algorithm 2.

Modules: quadrature (Gauss rules and the singular panel-pair rules),
timeint (analytic time integrals), dense (dense Galerkin assembly for tiny
meshes), tree (Algorithm 1 and the lists), fmm (expansions and the apply),
solve (unpreconditioned GMRES), represent (single- and double-layer
potentials at interior points).

Module p1: the double layer with p1-continuous trial functions in space,
the mixed mass matrix and the FMM for it (Section 2).

Parity status per function is listed in the module headers; every function
here is pinned by a ``-m "not gpu"`` test against a value fixed by the paper
or by mathematics other than this code.
"""
