"""Pins of the oracle's time integrals and panel quadrature (CPU only).

* Closed-form time integrals vs brute-force 2D quadrature of the heat kernel
  over the time rectangle (Section 2, eq. heat_kernel) and vs mpmath.
* Singular panel-pair rules vs the analytic in-plane potential of a triangle,
  integrated over the target triangle by adaptive quadrature.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import quadrature as Q
from oracle.timeint import G, G2, K2, time_factor, use_hat


@pytest.mark.parametrize("r", [0.01, 0.1, 0.3])
@pytest.mark.parametrize("d", [0, 1, 4])
def test_time_integrals_vs_bruteforce(r, d):
    alpha, h = 0.7, 0.05

    def fv(tau, t):
        return float(G(r, t - tau, alpha))

    def fk(tau, t):
        s = t - tau
        return float(G(r, s, alpha)) / (2 * s) if s > 0 else 0.0

    if d == 0:
        lim = dict(a=0, b=h, gfun=lambda t: 0, hfun=lambda t: t)
    else:
        lim = dict(a=d * h, b=(d + 1) * h, gfun=lambda t: 0, hfun=lambda t: h)
    ref_v = integrate.dblquad(fv, epsabs=1e-17, epsrel=1e-13, **lim)[0]
    ref_k = integrate.dblquad(fk, epsabs=1e-19, epsrel=1e-13, **lim)[0]
    v = time_factor(np.array([r]), d, h, alpha, "V")[0]
    k = time_factor(np.array([r]), d, h, alpha, "K")[0]
    assert abs(v - ref_v) <= 1e-11 * abs(ref_v)
    assert abs(k - ref_k) <= 2e-11 * abs(ref_k)


def test_antiderivatives_mpmath():
    """G2'' = G and K2'' = G/(2s) in s, checked at 50 digits; G2(r,0+) -> 0."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    alpha = mp.mpf("0.7")

    def g2(r, s):
        z = r / (2 * mp.sqrt(alpha * s))
        return ((s + r * r / (2 * alpha)) * mp.erfc(z) - r * mp.sqrt(s / (mp.pi * alpha)) * mp.exp(-z * z)) / (4 * mp.pi * alpha * r)

    def k2(r, s):
        z = r / (2 * mp.sqrt(alpha * s))
        return ((s - r * r / (2 * alpha)) * mp.erfc(z) + r * mp.sqrt(s / (mp.pi * alpha)) * mp.exp(-z * z)) / (4 * mp.pi * r ** 3)

    def g(r, s):
        return (4 * mp.pi * alpha * s) ** mp.mpf(-1.5) * mp.exp(-r * r / (4 * alpha * s))

    for r, s in [(mp.mpf("0.05"), mp.mpf("0.01")), (mp.mpf("0.3"), mp.mpf("0.2"))]:
        assert abs(mp.diff(lambda x: g2(r, x), s, 2) - g(r, s)) < mp.mpf("1e-30") * g(r, s)
        assert abs(mp.diff(lambda x: k2(r, x), s, 2) - g(r, s) / (2 * s)) < mp.mpf("1e-30") * g(r, s) / s
        # the float implementation agrees with the 50-digit one
        assert abs(float(G2(float(r), float(s), 0.7)) - float(g2(r, s))) < 1e-14 * abs(float(g2(r, s)))
        assert abs(float(K2(float(r), float(s), 0.7)) - float(k2(r, s))) < 1e-14 * abs(float(k2(r, s)))
    # near-cancelling point: closed form and hat rule both match 50-digit value
    r, d, h = mp.mpf("0.01"), 6, mp.mpf("0.01")
    ex = g2(r, (d + 1) * h) - 2 * g2(r, d * h) + g2(r, (d - 1) * h)
    v = time_factor(np.array([float(r)]), d, float(h), 0.7, "V")[0]
    assert bool(use_hat(np.array([float(r)]), d, float(h), 0.7, "V")[0]) is False
    assert abs(v - float(ex)) < 1e-11 * abs(float(ex))
    r = mp.mpf("1e-7")
    ex = g2(r, (d + 1) * h) - 2 * g2(r, d * h) + g2(r, (d - 1) * h)
    assert bool(use_hat(np.array([float(r)]), d, float(h), 0.7, "V")[0]) is True
    v = time_factor(np.array([float(r)]), d, float(h), 0.7, "V")[0]
    assert abs(v - float(ex)) < 1e-12 * abs(float(ex))


# ---------------------------------------------------------------- quadrature

def test_gauss_legendre_exact():
    g, w = Q.gauss_legendre01(5)
    for p in range(10):
        assert abs(np.sum(w * g ** p) - 1.0 / (p + 1)) < 1e-15


def _tris():
    V = np.array([[0, 0, 0], [1, 0, 0], [0.3, 0.9, 0], [1.2, 0.8, 0], [-0.6, 0.4, 0],
                  [0.2, 0.1, 0.8], [1.0, -0.7, 0.0], [1.7, 0.1, 0.0]], dtype=float)
    return V


@pytest.mark.parametrize("case", ["identical", "edge", "vertex", "edge90", "vertex90"])
def test_singular_rules_polynomials(case):
    """Constant and polynomial integrands are integrated exactly."""
    V = _tris()
    T = {"identical": ([0, 1, 2], [0, 1, 2]), "edge": ([0, 1, 2], [1, 0, 6]),
         "vertex": ([0, 1, 2], [1, 3, 7]), "edge90": ([0, 1, 2], [1, 0, 5]),
         "vertex90": ([0, 1, 2], [0, 5, 4])}[case]
    tris = np.array(T)
    d, W = Q.pair_rule(V, tris, 0, 1, True, 4, 6)
    d2, W2 = Q.regular_rule(V[tris[0]], V[tris[1]], 8)   # exact for these polynomials
    for f in (lambda x: np.ones(len(x)), lambda x: (x ** 2).sum(1), lambda x: (x ** 4).sum(1) + x[:, 0] * x[:, 1] ** 2):
        assert abs(np.sum(W * f(d)) - np.sum(W2 * f(d2))) < 1e-13


def _inplane_potential(T, x):
    """int_T dy / |x - y| for x in the plane of the 2D triangle T (ccw)."""
    tot = 0.0
    for e in range(3):
        A, B = T[e], T[(e + 1) % 3]
        L = np.linalg.norm(B - A)
        t = (B - A) / L
        n = np.array([t[1], -t[0]])          # outward for ccw
        de = np.dot(A - x, n)
        lm, lp = np.dot(A - x, t), np.dot(B - x, t)
        Rm, Rp = np.linalg.norm(A - x), np.linalg.norm(B - x)
        if abs(de) < 1e-14:
            continue
        tot += de * np.log((lp + Rp) / (lm + Rm))
    return tot


def _tri_integral(T, f):
    """Adaptive 2D integral of f over a 2D triangle."""
    A, B, C = T

    def g(v, u):
        x = A + u * (B - A) + v * (C - A)
        return f(x)
    area2 = abs(np.cross(B - A, C - A))
    return area2 * integrate.dblquad(g, 0, 1, lambda u: 0, lambda u: 1 - u, epsabs=1e-13, epsrel=1e-11)[0]


def test_inplane_potential_formula():
    T = np.array([[0.0, 0.0], [1.0, 0.0], [0.3, 0.9]])
    x = np.array([1.5, 1.2])
    ref = _tri_integral(T, lambda y: 1.0 / np.linalg.norm(x - y))
    assert abs(_inplane_potential(T, x) - ref) < 1e-10 * ref


@pytest.mark.parametrize("case", ["identical", "edge", "vertex"])
def test_singular_rules_one_over_r(case):
    """Coplanar touching pairs: rule vs int_{T1} (analytic potential of T2)."""
    V = _tris()
    T = {"identical": ([0, 1, 2], [0, 1, 2]), "edge": ([0, 1, 2], [1, 0, 6]),
         "vertex": ([0, 1, 2], [1, 3, 7])}[case]
    tris = np.array(T)
    P1, P2 = V[tris[0]][:, :2], V[tris[1]][:, :2]
    ccw = lambda P: P if np.cross(P[1] - P[0], P[2] - P[0]) > 0 else P[[0, 2, 1]]
    ref = _tri_integral(ccw(P1), lambda x: _inplane_potential(ccw(P2), x))
    d, W = Q.pair_rule(V, tris, 0, 1, True, 4, 12)
    val = np.sum(W / np.linalg.norm(d, axis=1))
    assert abs(val - ref) < 1e-8 * ref
    # the default order is already accurate to a few 1e-5 for this kernel
    d, W = Q.pair_rule(V, tris, 0, 1, True, 4, 5)
    assert abs(np.sum(W / np.linalg.norm(d, axis=1)) - ref) < 1e-3 * ref
