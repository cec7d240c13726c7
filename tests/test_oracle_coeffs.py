"""Pins of the oracle's printed coefficients against independent derivations.

Each printed closed form in section 2 of the paper is re-derived here from its
definition (a Hermite interpolation problem solved numerically, an exact
polynomial integral, a complex-step Jacobian) rather than retyped, so a wrong
coefficient, sign or index in the oracle fails one of these tests.
"""
import numpy as np
import numpy.polynomial.polynomial as P
import pytest

from oracle import hweno as O

RNG = np.random.default_rng(12345)


def hermite_fit(conds, deg):
    """Polynomial in xi (coefficients low->high) meeting value/derivative
    conditions [(xi, order, value)], solved as a square linear system."""
    A = np.zeros((len(conds), deg + 1))
    b = np.zeros(len(conds))
    for r, (xi, order, val) in enumerate(conds):
        for k in range(deg + 1):
            if k >= order:
                A[r, k] = np.prod(np.arange(k - order + 1, k + 1)) * xi ** (k - order)
        b[r] = val
    return np.linalg.solve(A, b)


def deriv_at(c, order, xi):
    return P.polyval(xi, P.polyder(c, order)) if order else P.polyval(xi, c)


def quartic_p0(um, u0, up, vm, vp, dx):
    # (HWEp0): p0(x_{i+l}) = u_{i+l} (l=-1,0,1), p0'(x_{i+-1}) = v_{i+-1}; xi=(x-x_i)/dx
    return hermite_fit([(-1, 0, um), (0, 0, u0), (1, 0, up), (-1, 1, dx * vm), (1, 1, dx * vp)], 4)


@pytest.mark.parametrize("trial", range(5))
def test_candidate_values_and_derivatives(trial):
    um, u0, up, vm, vp = RNG.normal(size=5)
    dx = RNG.uniform(0.01, 2.0)
    c = quartic_p0(um, u0, up, vm, vp, dx)
    p0, p1, p2, dp0 = O.candidates_at_right_face(um, u0, up, vm, vp, dx)
    assert p0 == pytest.approx(deriv_at(c, 0, 0.5), rel=1e-12, abs=1e-12)
    assert dp0 == pytest.approx(deriv_at(c, 1, 0.5) / dx, rel=1e-12, abs=1e-12)
    # p1 through (x_{i-1}, x_i), p2 through (x_i, x_{i+1}), evaluated at xi = 1/2
    assert p1 == pytest.approx(u0 + 0.5 * (u0 - um), rel=1e-14, abs=0)
    assert p2 == pytest.approx(0.5 * (u0 + up), rel=1e-14, abs=0)
    d0, d1, d2 = O.candidate_derivatives_at_centre(um, u0, up, vm, vp, dx)
    assert d0 == pytest.approx(deriv_at(c, 1, 0.0) / dx, rel=1e-12, abs=1e-12)
    assert d1 == pytest.approx((u0 - um) / dx, rel=1e-14, abs=0)
    assert d2 == pytest.approx((up - u0) / dx, rel=1e-14, abs=0)


@pytest.mark.parametrize("trial", range(5))
def test_smoothness_indicator_closed_form_equals_definition(trial):
    """(GHYZ): beta = sum_a int_{I_i} dx^{2a-1} (p^{(a)})^2 dx, which in xi is
    sum_a int_{-1/2}^{1/2} (d^a p/dxi^a)^2 dxi, integrated exactly."""
    um, u0, up, vm, vp = RNG.normal(size=5)
    dx = RNG.uniform(0.01, 2.0)
    c = quartic_p0(um, u0, up, vm, vp, dx)
    beta0 = 0.0
    for a in range(1, 5):
        sq = P.polypow(P.polyder(c, a), 2)
        integ = P.polyint(sq)
        beta0 += P.polyval(0.5, integ) - P.polyval(-0.5, integ)
    b0, b1, b2 = O.smoothness_indicators(um, u0, up, vm, vp, dx)
    assert b0 == pytest.approx(beta0, rel=1e-11, abs=0)
    assert b1 == pytest.approx((u0 - um) ** 2, rel=1e-14, abs=0)
    assert b2 == pytest.approx((up - u0) ** 2, rel=1e-14, abs=0)


def quintic_P(fm1, f0, fp1, fp2, hm1, hp2, dx):
    # (Pc): P(x_{i+l}) = f_{i+l} (l=-1..2), P'(x_{i+l}) = h_{i+l} (l=-1,2)
    return hermite_fit([(-1, 0, fm1), (0, 0, f0), (1, 0, fp1), (2, 0, fp2),
                        (-1, 1, dx * hm1), (2, 1, dx * hp2)], 5)


@pytest.mark.parametrize("trial", range(5))
def test_central_D_from_hermite_quintic(trial):
    """(Cd-1)-(DfDh): derivatives of the quintic Hermite interpolant at
    x_{i+1/2}, with dx^2 P'' = P_xixi, dx^2 P''' = P_xixixi/dx, etc."""
    f = RNG.normal(size=4)
    hm1, hp2 = RNG.normal(size=2)
    dx = RNG.uniform(0.01, 2.0)
    c = quintic_P(*f, hm1, hp2, dx)
    d2 = deriv_at(c, 2, 0.5)
    d3 = deriv_at(c, 3, 0.5) / dx
    d4 = deriv_at(c, 4, 0.5)
    d5 = deriv_at(c, 5, 0.5) / dx
    Df, Dh = O.central_D(*f, hm1, hp2, dx)
    scale = 1 + abs(d2) + abs(d4) + abs(d3) + abs(d5)
    assert Df == pytest.approx(-d2 / 24 + 7 * d4 / 5760, abs=1e-12 * scale)
    assert Dh == pytest.approx(-d3 / 24 + 7 * d5 / 5760, abs=1e-12 * scale)


@pytest.mark.parametrize("trial", range(4))
def test_conservative_flux_difference_exact_for_quintics(trial):
    """(flux-high)/(D6): with f a quintic polynomial and h = f', the flux
    f(x_{i+1/2}) + D(f) has difference quotient exactly f'(x_i), and
    h(x_{i+1/2}) + D(h) has difference quotient exactly h'(x_i) = f''(x_i)."""
    cf = RNG.normal(size=6)
    dx = RNG.uniform(0.05, 1.0)
    xi = RNG.uniform(-1, 1)
    F = lambda x: P.polyval(x, cf)
    dF = lambda x, k=1: P.polyval(x, P.polyder(cf, k))
    xs = xi + dx * np.arange(-2, 3)            # cells i-2..i+2
    fv, hv = F(xs), dF(xs)
    Df_p, Dh_p = O.central_D(fv[1], fv[2], fv[3], fv[4], hv[1], hv[4], dx)   # x_{i+1/2}
    Df_m, Dh_m = O.central_D(fv[0], fv[1], fv[2], fv[3], hv[0], hv[3], dx)   # x_{i-1/2}
    fl = lambda x, D: F(x) + D
    hl = lambda x, D: dF(x) + D
    q1 = (fl(xi + dx / 2, Df_p) - fl(xi - dx / 2, Df_m)) / dx
    q2 = (hl(xi + dx / 2, Dh_p) - hl(xi - dx / 2, Dh_m)) / dx
    assert q1 == pytest.approx(dF(xi), rel=1e-9, abs=1e-9)
    assert q2 == pytest.approx(dF(xi, 2), rel=1e-9, abs=1e-9)


def test_mixed_flux_difference_is_fourth_order_central():
    """(mixed): difference quotient of the interface values is exact for
    quartic data (it equals the five-point central first derivative)."""
    for _ in range(4):
        ce = RNG.normal(size=5)
        dx = RNG.uniform(0.05, 1.0)
        xi = RNG.uniform(-1, 1)
        e = P.polyval(xi + dx * np.arange(-2, 3), ce)
        q = (O.mixed_flux(e[1], e[2], e[3], e[4]) - O.mixed_flux(e[0], e[1], e[2], e[3])) / dx
        assert q == pytest.approx(P.polyval(xi, P.polyder(ce)), rel=1e-10, abs=1e-10)


def _euler_state(dim, n=7):
    rho = RNG.uniform(0.2, 3.0, n)
    u = RNG.uniform(-2, 2, n)
    v = RNG.uniform(-2, 2, n)
    p = RNG.uniform(0.2, 5.0, n)
    g = 1.4
    if dim == 1:
        return np.stack([rho, rho * u, p / (g - 1) + 0.5 * rho * u * u])
    return np.stack([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])


@pytest.mark.parametrize("dim,d", [(1, 0), (2, 0), (2, 1)])
def test_euler_jacobian_against_complex_step(dim, d):
    sys = O.Euler(1.4, dim)
    U = _euler_state(dim)
    J = sys.jacobian(U, d)
    nc = U.shape[0]
    hstep = 1e-30
    for j in range(nc):
        Uc = U.astype(complex)
        Uc[j] += 1j * hstep
        col = np.imag(sys.flux(Uc, d)) / hstep
        np.testing.assert_allclose(J[..., :, j], col.T, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim,d", [(1, 0), (2, 0), (2, 1)])
def test_euler_eigenvectors_diagonalise_jacobian(dim, d):
    sys = O.Euler(1.4, dim)
    U = _euler_state(dim)
    L, R = sys.eig(U, d)
    rho, mu, nu, Pp, c, H = sys.primitives(U)
    vel = mu if d == 0 else nu
    lam = [vel - c, vel, vel + c] if dim == 1 else [vel - c, vel, vel, vel + c]
    A = sys.jacobian(U, d)
    for k in range(U.shape[1]):
        np.testing.assert_allclose(R[k] @ np.diag([l[k] for l in lam]) @ L[k], A[k],
                                   rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(L[k] @ R[k], np.eye(U.shape[0]), atol=1e-12)
