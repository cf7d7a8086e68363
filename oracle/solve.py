"""Dirichlet solve of the Galerkin system (oracle, test-only).

Section 2, linear system 02:linear:system: find w with
    V_h w = (1/2 M_h + K_h) g,
where M_h is the mass matrix of the p0 x p0 pairing (diagonal, |gamma_k| h_t
for uniform steps) and g the coefficients of the projected Dirichlet datum.
Section 5 solves it with unpreconditioned GMRES to a relative precision of
1e-8; the paper states neither restart nor orthogonalisation, read here as
GMRES (Saad and Schultz, 1986) from x0 = 0 without restart, modified
Gram-Schmidt Arnoldi and Givens rotations, stopped when the least-squares
residual estimate ||b - A x_k||_2 / ||b||_2 reaches rtol.

Parity: pinned in tests/test_oracle_solve.py against numpy.linalg.solve, the
finite termination of GMRES on a matrix with few distinct eigenvalues, the
true residual of every reported iterate, and a manufactured Neumann datum of a
heat source outside the domain.
"""
import numpy as np


def gmres(matvec, b, rtol=1e-8, max_iter=200):
    """Solve A x = b; returns (x, iterations, relative residual estimates per iteration)."""
    b = np.asarray(b, dtype=np.float64)
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros_like(b), 0, [0.0]
    n = b.size
    V = np.zeros((max_iter + 1, n))
    H = np.zeros((max_iter + 1, max_iter))
    cs = np.zeros(max_iter)
    sn = np.zeros(max_iter)
    e = np.zeros(max_iter + 1)          # right-hand side of the rotated least-squares problem
    e[0] = beta
    V[0] = b / beta
    hist = [1.0]
    k = 0
    for j in range(max_iter):
        w = matvec(V[j])
        for i in range(j + 1):          # modified Gram-Schmidt
            H[i, j] = float(np.dot(w, V[i]))
            w = w - H[i, j] * V[i]
        H[j + 1, j] = float(np.linalg.norm(w))
        if H[j + 1, j] > 0.0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):              # earlier rotations on the new column
            a, c = H[i, j], H[i + 1, j]
            H[i, j] = cs[i] * a + sn[i] * c
            H[i + 1, j] = -sn[i] * a + cs[i] * c
        r = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / r, H[j + 1, j] / r
        H[j, j] = r
        H[j + 1, j] = 0.0
        e[j + 1] = -sn[j] * e[j]
        e[j] = cs[j] * e[j]
        k = j + 1
        hist.append(abs(e[j + 1]) / beta)
        if hist[-1] <= rtol or H[j, j] == 0.0:
            break
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):      # back substitution with the triangular factor
        y[i] = (e[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    return V[:k].T @ y, k, hist


def dirichlet_rhs(g, mass, apply_K):
    """(1/2 M_h + K_h) g for the diagonal mass matrix `mass` (system 02:linear:system)."""
    return 0.5 * mass * g + apply_K(g)
