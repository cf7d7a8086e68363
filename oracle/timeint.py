"""Analytic time integrals of the heat kernel for p0-in-time Galerkin entries.

Heat kernel (Section 2, eq. heat_kernel):
    G(r, s) = (4 pi alpha s)^(-3/2) exp(-r^2 / (4 alpha s)) for s > 0, else 0.

A p0 x p0 entry of V_h (Section 2, matrix V) integrates G over a pair of
time steps.  With G2 the second antiderivative of G in s that vanishes with
its first derivative at s = 0,

    G2(r, s) = [(s + r^2/(2 alpha)) erfc(z) - r sqrt(s/(pi alpha)) e^{-z^2}]
               / (4 pi alpha r),   z = r / (2 sqrt(alpha s)),

the time double integral over steps k and j of length h with d = k - j >= 0
equals the second difference
    D2G2(r, d) = G2(r, (d+1)h) - 2 G2(r, d h) + G2(r, (d-1)h),  G2(., s<=0) = 0.

For the double layer K (Section 2, operator K) the kernel is
alpha dG/dn_y = ((x - y).n_y / (2 s)) G, and the analogous antiderivative is
    K2(r, s) = [(s - r^2/(2 alpha)) erfc(z) + r sqrt(s/(pi alpha)) e^{-z^2}]
               / (4 pi r^3)  ( = -(alpha/r) dG2/dr ),
so an entry is (x - y).n_y times D2K2.

For d >= 2 the leading s/r and s/r^3 terms cancel in the second difference.
When the estimated cancellation ratio exceeds 1e4 (or r = 0) the second
difference is evaluated instead as the hat-function integral
    int_{(d-1)h}^{(d+1)h} (h - |s - d h|) g(s) ds,  g = G  or  G/(2 s),
with 16-point Gauss-Legendre on each half.

Parity: pinned by tests against brute-force two-dimensional quadrature of the
kernel over the time rectangle and against mpmath at 50 digits.
"""
import numpy as np
from scipy.special import erfc

from .quadrature import gauss_legendre01

HAT_POINTS = 16
CANCEL_LIMIT = 1.0e4


def G(r, s, alpha):
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros(np.broadcast(r, s).shape)
    pos = np.broadcast_to(s > 0, out.shape)
    rb = np.broadcast_to(r, out.shape)[pos]
    sb = np.broadcast_to(s, out.shape)[pos]
    out[pos] = (4.0 * np.pi * alpha * sb) ** -1.5 * np.exp(-rb * rb / (4.0 * alpha * sb))
    return out


def G2(r, s, alpha):
    """Second s-antiderivative of G (r > 0); zero for s <= 0."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    shape = np.broadcast(r, s).shape
    rb = np.broadcast_to(r, shape)
    sb = np.broadcast_to(s, shape)
    out = np.zeros(shape)
    pos = sb > 0
    rr, ss = rb[pos], sb[pos]
    z = rr / (2.0 * np.sqrt(alpha * ss))
    out[pos] = ((ss + rr * rr / (2.0 * alpha)) * erfc(z)
                - rr * np.sqrt(ss / (np.pi * alpha)) * np.exp(-z * z)) / (4.0 * np.pi * alpha * rr)
    return out


def K2(r, s, alpha):
    """Second s-antiderivative of G/(2s) (r > 0); zero for s <= 0."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    shape = np.broadcast(r, s).shape
    rb = np.broadcast_to(r, shape)
    sb = np.broadcast_to(s, shape)
    out = np.zeros(shape)
    pos = sb > 0
    rr, ss = rb[pos], sb[pos]
    z = rr / (2.0 * np.sqrt(alpha * ss))
    out[pos] = ((ss - rr * rr / (2.0 * alpha)) * erfc(z)
                + rr * np.sqrt(ss / (np.pi * alpha)) * np.exp(-z * z)) / (4.0 * np.pi * rr ** 3)
    return out


def _hat(r, d, h, alpha, kind):
    """int (h - |s - d h|) g(s) ds over [(d-1)h, (d+1)h], g = G or G/(2s)."""
    g, w = gauss_legendre01(HAT_POINTS)
    r = np.asarray(r, dtype=np.float64)[..., None]
    tot = 0.0
    # left half: s = (d-1)h + h g, weight (s - (d-1)h) = h g
    sl = (d - 1) * h + h * g
    sr = d * h + h * g          # right half: weight ((d+1)h - s) = h (1 - g)
    fl = G(r, sl, alpha)
    fr = G(r, sr, alpha)
    if kind == "K":
        fl = fl / (2.0 * sl)
        fr = fr / (2.0 * sr)
    tot = (h * h) * (np.sum(w * g * fl, axis=-1) + np.sum(w * (1.0 - g) * fr, axis=-1))
    return tot


def use_hat(r, d, h, alpha, kind):
    """Branch test: True where the closed-form second difference cancels badly."""
    r = np.asarray(r, dtype=np.float64)
    if d < 2:
        return np.zeros(r.shape, dtype=bool)
    big = (d + 1.0) * (4.0 * np.pi * alpha * d * h) ** 1.5
    if kind == "V":
        lhs = CANCEL_LIMIT * (4.0 * np.pi * alpha) * r * h
    else:
        big = 2.0 * d * big
        lhs = CANCEL_LIMIT * (4.0 * np.pi) * r * r * r
    return lhs < big


def time_factor(r, d, h, alpha, kind):
    """D2G2 (kind 'V') or D2K2 (kind 'K') at distance r for offset d >= 0."""
    r = np.asarray(r, dtype=np.float64)
    F = G2 if kind == "V" else K2
    out = F(r, (d + 1) * h, alpha) - 2.0 * F(r, d * h, alpha) + F(r, (d - 1) * h, alpha)
    if d >= 2:
        m = use_hat(r, d, h, alpha, kind)
        if np.any(m):
            out = np.where(m, 0.0, out)
            out[m] = _hat(r[m], d, h, alpha, kind)
    return out


def time_factors_all(r, dmax, h, alpha, kind):
    """time_factor for d = 0..dmax; returns (dmax+1,) + r.shape.

    The closed forms are evaluated once per node s = m h (m = 0..dmax+1) and
    differenced; the hat branch replaces the entries it selects.
    """
    r = np.asarray(r, dtype=np.float64)
    F = G2 if kind == "V" else K2
    vals = np.stack([F(r, m * h, alpha) for m in range(dmax + 2)])
    out = np.empty((dmax + 1,) + r.shape)
    out[0] = vals[1]
    for d in range(1, dmax + 1):
        out[d] = vals[d + 1] - 2.0 * vals[d] + vals[d - 1]
        if d >= 2:
            m = use_hat(r, d, h, alpha, kind)
            if np.any(m):
                out[d][m] = _hat(r[m], d, h, alpha, kind)
    return out


def needs_singular_rule(d):
    """Touching panel pairs use the singular spatial rules for d in {0, 1}."""
    return d <= 1


# ---------------------------------------------------------------- steps of any length
# For a time grid with steps of different lengths the double time integral
# over target step k = [tk0, tk1] and source step j = [tj0, tj1] is the
# four-term combination of the second antiderivative at the node differences,
#     F(tk1 - tj0) - F(tk1 - tj1) - F(tk0 - tj0) + F(tk0 - tj1),   F(., s <= 0) = 0,
# (with equal steps h and d = k - j this is the second difference above).
# When the steps are separated (d >= 2 in step indices) and the same
# cancellation test flags the closed form -- with h the longer of the two
# steps and d the lag tk0 - tj0 in units of h -- the integral is evaluated
# instead as int phi(s) g(s) ds over s in [tk0 - tj1, tk1 - tj0], phi the
# overlap length of the two steps at lag s: a trapezoid (a hat for equal
# steps) rising over the shorter step length, flat over the difference of the
# lengths, falling over the shorter length; 16-point Gauss-Legendre per piece.

def _trapezoid(r, tk0, tk1, tj0, tj1, alpha, kind):
    g, w = gauss_legendre01(HAT_POINTS)
    r = np.asarray(r, dtype=np.float64)[..., None]
    hk, hj = tk1 - tk0, tj1 - tj0
    hm = min(hk, hj)
    a = tk0 - tj1
    b = a + hm
    c = b + abs(hk - hj)
    e = tk1 - tj0

    def f(s):
        v = G(r, s, alpha)
        return v / (2.0 * s) if kind == "K" else v

    tot = hm * np.sum(w * (hm * g) * f(a + hm * g), axis=-1)            # rising piece
    if c > b:
        tot = tot + (c - b) * np.sum(w * hm * f(b + (c - b) * g), axis=-1)   # plateau
    tot = tot + hm * np.sum(w * (hm * (1.0 - g)) * f(c + hm * g), axis=-1)   # falling piece
    return tot


def use_trapezoid(r, tk0, tk1, tj0, tj1, d, alpha, kind):
    """Branch test for steps of any length (the test of use_hat with h the
    longer step and d the lag in units of h); only for separated steps."""
    r = np.asarray(r, dtype=np.float64)
    if d < 2:
        return np.zeros(r.shape, dtype=bool)
    h = max(tk1 - tk0, tj1 - tj0)
    lag = tk0 - tj0
    big = (lag / h + 1.0) * (4.0 * np.pi * alpha * lag) ** 1.5
    if kind == "V":
        lhs = CANCEL_LIMIT * (4.0 * np.pi * alpha) * r * h
    else:
        big = 2.0 * (lag / h) * big
        lhs = CANCEL_LIMIT * (4.0 * np.pi) * r * r * r
    return lhs < big


def time_factor_steps(r, tk0, tk1, tj0, tj1, d, alpha, kind):
    """Double time integral of G (V) or G/(2s) (K, without the (x-y).n_y
    factor) over target step [tk0, tk1] and source step [tj0, tj1] at
    distance r; d = k - j >= 0 is the step-index offset (d >= 2: separated)."""
    r = np.asarray(r, dtype=np.float64)
    F = G2 if kind == "V" else K2
    out = F(r, tk1 - tj0, alpha) - F(r, tk1 - tj1, alpha) - F(r, tk0 - tj0, alpha) + F(r, tk0 - tj1, alpha)
    if d >= 2:
        m = use_trapezoid(r, tk0, tk1, tj0, tj1, d, alpha, kind)
        if np.any(m):
            out = np.where(m, 0.0, out)
            out[m] = _trapezoid(r[m], tk0, tk1, tj0, tj1, alpha, kind)
    return out
