"""Pins of the oracle's representation formula (CPU only).

* G1 and K1, the closed-form time antiderivatives of G and G / (2 s), against
  adaptive quadrature of the kernel in time.
* The single-layer potential of the constant density 1 on the cube surface
  at interior points against the face-wise formula: the surface integral of
  G factorises per face into a one-dimensional Gaussian times erf products,
  leaving a one-dimensional integral over the time lag.
* The double-layer potential of the constant 1 at interior points against
  the volume heat potential of the constant minus one (divergence theorem:
  d/ds of the volume integral of G is the flux of alpha grad G through the
  surface, and the volume integral tends to 1 as s -> 0 inside the domain).
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import erf

from oracle.represent import G1, K1, potentials, representation
from oracle.timeint import G
from workloads import cube_surface_mesh, uniform_time_nodes

ALPHA = 0.7


@pytest.mark.parametrize("r", [0.05, 0.3, 1.2])
@pytest.mark.parametrize("s", [0.01, 0.2, 1.5])
def test_time_antiderivatives(r, s):
    g = quad(lambda x: G(r, x, ALPHA), 0.0, s, epsabs=0, epsrel=1e-13, limit=200)[0]
    k = quad(lambda x: G(r, x, ALPHA) / (2 * x), 0.0, s, epsabs=0, epsrel=1e-13, limit=200)[0]
    assert abs(G1(r, s, ALPHA) - g) <= 1e-11 * abs(g) + 1e-300
    assert abs(K1(r, s, ALPHA) - k) <= 1e-10 * abs(k) + 1e-300
    assert G1(r, 0.0, ALPHA) == 0.0 and K1(r, -1.0, ALPHA) == 0.0


def _single_layer_of_one(x, t, alpha):
    """int_0^t int_{surface of (-1,1)^3} G(x - y, s) ds_y ds."""
    def integrand(s):
        c = 2.0 * np.sqrt(alpha * s)
        I1 = lambda xi: 0.5 * (erf((xi + 1) / c) - erf((xi - 1) / c))
        g1 = lambda z: np.exp(-z * z / (4 * alpha * s)) / np.sqrt(4 * np.pi * alpha * s)
        tot = 0.0
        for a in range(3):
            others = [j for j in range(3) if j != a]
            prod = I1(x[others[0]]) * I1(x[others[1]])
            tot += (g1(x[a] - 1.0) + g1(x[a] + 1.0)) * prod
        return tot
    return quad(integrand, 0.0, t, epsabs=0, epsrel=1e-12, limit=400)[0]


def _volume_potential_of_one(x, t, alpha):
    c = 2.0 * np.sqrt(alpha * t)
    return np.prod([0.5 * (erf((1 - xj) / c) + erf((1 + xj) / c)) for xj in x])


def test_potentials_of_constant_densities():
    v, tri = cube_surface_mesh(4)
    tn = uniform_time_nodes(10, 1.0)
    pts = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.4], [-0.45, 0.1, 0.05]])
    times = np.array([0.37, 1.0, 0.8])
    one = np.ones(10 * len(tri))
    sl, dl = potentials(v, tri, tn, one, one, pts, times, ALPHA, q=12)
    for i, (x, t) in enumerate(zip(pts, times)):
        ref_s = _single_layer_of_one(x, t, ALPHA)
        ref_d = _volume_potential_of_one(x, t, ALPHA) - 1.0
        assert abs(sl[i] - ref_s) <= 1e-8 * abs(ref_s), (i, sl[i], ref_s)
        assert abs(dl[i] - ref_d) <= 1e-8 * abs(ref_d), (i, dl[i], ref_d)
    # the formula's two terms: u = V~ w - W g
    u = representation(v, tri, tn, one, one, pts, times, ALPHA, q=12)
    assert np.allclose(u, sl - dl, rtol=0, atol=1e-15 * np.abs(sl).max())


def test_causality_and_linearity():
    """Densities on steps after the target time do not contribute; the
    potentials are linear in the densities."""
    v, tri = cube_surface_mesh(2)
    tn = uniform_time_nodes(8, 1.0)
    rng = np.random.default_rng(5)
    w = rng.uniform(-1, 1, 8 * len(tri))
    u = rng.uniform(-1, 1, 8 * len(tri))
    pts = np.array([[0.1, 0.2, -0.3]])
    t = np.array([0.4])                      # inside step 3 (0.375 .. 0.5)
    a = potentials(v, tri, tn, w, u, pts, t, ALPHA)
    w2, u2 = w.copy(), u.copy()
    w2[4 * len(tri):] = 5.0                  # steps 4.. start after t
    u2[4 * len(tri):] = -3.0
    b = potentials(v, tri, tn, w2, u2, pts, t, ALPHA)
    assert a[0][0] == b[0][0] and a[1][0] == b[1][0]
    c = potentials(v, tri, tn, 2 * w, 3 * u, pts, t, ALPHA)
    assert np.isclose(c[0][0], 2 * a[0][0], rtol=1e-14) and np.isclose(c[1][0], 3 * a[1][0], rtol=1e-14)
