"""Pins of the oracle's gravity source (euler2d-s) and fixed-state (Dirichlet)
boundaries, as used by Example 4.11 (Rayleigh-Taylor).

* Hydrostatic layers: constant density, zero velocity and a pressure linear
  in y with P_y = g rho is a steady state of (euler2d-s). Every candidate
  interpolant is exact on linear data and D(f) vanishes on it, so the
  operator must vanish to round-off in the rows whose stencils stay inside
  one layer, for all three equations.
* A uniform state inside fixed-state boundaries holding the same state: no
  flux varies, so L^1 = S(U) = g (0, 0, rho, rho v) exactly, L^2 = L^3 = 0.
* Fixed states equal to the edge cells (with zero derivatives) give the
  transmissive operator.
* Example 4.11's data is symmetric about x = 1/8 and the walls keep it so.
"""
import numpy as np
import pytest

from oracle import hweno as O
from paper_2411_11229_amd import workloads as WL

G = 5.0 / 3.0


def cons(r, u, v, p, g=G):
    return (r, r * u, r * v, p / (g - 1.0) + 0.5 * r * (u * u + v * v))


def hydrostatic(nx, ny):
    w = WL.rayleigh_taylor(nx)
    X, Y = np.meshgrid(w.x, w.y)
    low = Y < 0.5
    rho = np.where(low, 2.0, 1.0)
    P = np.where(low, 2.0 * Y + 1.0, Y + 1.5)
    z = np.zeros_like(X)
    w.U = np.stack(cons(rho, z, z, P))
    w.V = np.zeros_like(w.U)
    w.W = np.stack([z, z, z, np.where(low, 2.0, 1.0) / (G - 1.0)])
    return w


def test_hydrostatic_layers_are_steady():
    w = hydrostatic(8, 32)
    p = O.Problem(**w.problem_kwargs())
    L1, L2, L3, vt, wt = O.rhs(p, w.U, w.V, w.W)
    ny = w.ny
    rows = np.r_[3:ny // 2 - 3, ny // 2 + 3:ny - 3]
    scale = 2.0 * p.gravity          # g rho, the size of each balanced term
    assert np.max(np.abs(L1[:, rows, :])) <= 1e-12 * scale
    assert np.max(np.abs(L2[:, rows, :])) <= 1e-12 * scale
    assert np.max(np.abs(L3[:, rows, :])) <= 1e-12 * scale / w.dy
    # the interface and the fixed-state rows are not in balance
    assert np.max(np.abs(L1[:, ny // 2 - 1:ny // 2 + 1, :])) > 1.0


def test_uniform_state_source_exact():
    nx, ny = 10, 12
    st = cons(1.3, 0.4, -0.7, 2.1)
    U = np.stack([np.full((ny, nx), v) for v in st])
    z = np.zeros_like(U)
    p = O.Problem(dim=2, nx=nx, ny=ny, dx=0.1, dy=0.07, system='euler', gas_gamma=G,
                  bc=('dirichlet',) * 4, bc_state=(st,) * 4, gravity=0.8)
    L1, L2, L3, vt, wt = O.rhs(p, U, z, z)
    S = np.array([0.0, 0.0, 0.8 * st[0], 0.8 * st[2]])
    np.testing.assert_allclose(L1, np.broadcast_to(S[:, None, None], L1.shape), rtol=0, atol=1e-13)
    for a in (L2, L3, vt, wt):
        assert np.max(np.abs(a)) <= 1e-13


def test_fixed_states_equal_to_edges_act_as_transmissive():
    w = WL.euler2d_quadrants(14, seed=4401, ny=12)   # V = W = 0
    # make the bottom and top rows constant along x so one state matches them
    half = w.ny // 2
    w.U[:, :half, :] = w.U[:, :1, :1]
    w.U[:, half:, :] = w.U[:, -1:, -1:]
    lo, hi = tuple(w.U[:, 0, 0]), tuple(w.U[:, -1, 0])
    pt = O.Problem(**w.problem_kwargs())
    pd = O.Problem(**dict(w.problem_kwargs(), bc=('transmissive', 'transmissive', 'dirichlet', 'dirichlet'),
                          bc_state=(None, None, lo, hi)))
    a = O.rhs(pt, w.U, w.V, w.W)
    b = O.rhs(pd, w.U, w.V, w.W, O.max_speed(pt, w.U))
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-13 * max(1.0, np.max(np.abs(x))))


def test_rayleigh_taylor_stays_mirror_symmetric():
    w = WL.rayleigh_taylor(16)
    p = O.Problem(**w.problem_kwargs())
    U, V, W, log = O.run(p, w.U, w.V, w.W, 1e9, max_steps=8)
    flip = lambda a: a[..., ::-1]
    sign = np.array([1.0, -1.0, 1.0, 1.0])[:, None, None]
    np.testing.assert_allclose(U, sign * flip(U), rtol=0, atol=1e-12 * np.max(np.abs(U)))
    np.testing.assert_allclose(W, sign * flip(W), rtol=0, atol=1e-12 * np.max(np.abs(W)))
    np.testing.assert_allclose(V, -sign * flip(V), rtol=0, atol=1e-12 * np.max(np.abs(V)))


def test_source_rejected_outside_2d_euler():
    w = WL.paper_burgers2d(8)
    p = O.Problem(**w.problem_kwargs(), gravity=1.0)
    with pytest.raises(ValueError):
        O.rhs(p, w.U, w.V, w.W)
