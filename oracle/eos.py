"""Equation-of-state loop analysis (Sec. IV.A) in numpy — TEST
INFRASTRUCTURE ONLY (imported by tests and nothing in the product path).

In a finite box the equation of state P*(eta) near a first-order transition
shows a Mayer-Wood loop: a local maximum at the lower density and a local
minimum at the higher one.  The interface free energy per disk follows from
integrating the equation of state: with v = pi / eta the area per disk (sigma
the disk radius) and beta P sigma^2 = P* / 4 (P* being beta P (2 sigma)^2,
Eq. (1)), the Maxwell pressure P_c gives equal areas,
    integral from v1 to v3 of (P*(v) - P_c) dv = 0,
over the outer roots v1 < v2 < v3 of P*(v) = P_c, and the free energy per
disk above the common tangent is largest at the middle root:
    beta Delta f = (1/4) |integral from v1 to v2 of (P*(v) - P_c) dv|.
In two dimensions Delta f scales as N^(-1/2) for a first-order transition and
as N^(-1) for a continuous one (Sec. IV.A).

The smooth P*(v) is an (optionally weighted) least-squares polynomial in
v - mean(v) from numpy.polyfit; its stationary points and the roots of
P*(v) = P_c come from numpy.roots (companion-matrix eigenvalues); P_c from
scipy's brentq; the integrals are exact antiderivatives of the polynomial.
"""
import numpy as np
from scipy.optimize import brentq


def _fit(eta, P, order, se):
    v = np.pi / np.asarray(eta, np.float64)
    c = v.mean()
    w = None if se is None else 1.0 / np.asarray(se, np.float64)
    coef = np.polyfit(v - c, np.asarray(P, np.float64), order, w=w)
    return np.poly1d(coef), c, v.min() - c, v.max() - c


def _real_roots_in(poly, lo, hi):
    r = np.roots(poly.coeffs) if poly.order > 0 else np.array([])
    r = np.sort(r[np.abs(r.imag) < 1e-9 * max(1.0, np.abs(r).max(initial=0.0))].real)
    return r[(r >= lo) & (r <= hi)]


def loop(eta, P, order=3, se=None):
    """Mayer-Wood loop of P*(eta): its extrema, the Maxwell pressure, the
    coexisting densities and beta Delta f (dict), or None without a loop."""
    p, c, lo, hi = _fit(eta, P, order, se)
    dp, d2p = p.deriv(), p.deriv(2)
    st = _real_roots_in(dp, lo, hi)
    mx = [u for u in st if d2p(u) < 0]
    mn = [u for u in st if d2p(u) > 0]
    if len(mx) != 1 or len(mn) != 1 or not mn[0] < mx[0]:
        return None
    u_max, u_min = mx[0], mn[0]          # P local max at larger v (lower eta)
    P_max, P_min = p(u_max), p(u_min)
    ip = p.integ()

    def roots(Pc):
        r = _real_roots_in(p - np.poly1d([Pc]), lo, hi)
        return r if len(r) == 3 else None

    def g(Pc):
        r = roots(Pc)
        if r is None:
            raise ValueError("the Maxwell construction leaves the data range")
        return (ip(r[2]) - ip(r[0])) - Pc * (r[2] - r[0])

    span = P_max - P_min
    Pc = brentq(g, P_min + 1e-12 * span, P_max - 1e-12 * span, xtol=1e-14, rtol=1e-15)
    r = roots(Pc)
    df = 0.25 * abs((ip(r[1]) - ip(r[0])) - Pc * (r[1] - r[0]))
    return dict(eta_max=np.pi / (u_max + c), P_max=P_max, eta_min=np.pi / (u_min + c),
                P_min=P_min, P_coex=Pc, eta_liquid=np.pi / (r[2] + c),
                eta_solid=np.pi / (r[0] + c), delta_f=df)


def power_law(x, y):
    """y = a x^b by least squares on (ln x, ln y): returns (b, a)."""
    b, ln_a = np.polyfit(np.log(np.asarray(x, np.float64)), np.log(np.asarray(y, np.float64)), 1)
    return b, np.exp(ln_a)
