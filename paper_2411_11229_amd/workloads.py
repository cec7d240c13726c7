"""Seeded synthetic inputs (initial states) for tests and benchmarks.

This module builds initial data only: cell-centre grids, initial states U and
their exact spatial derivatives V = U_x, W = U_y, and the problem parameters.
It contains none of the scheme's arithmetic, and both the HIP path and the
CPU oracle consume what it returns. Every array is float64 NumPy,
component-major: ``[comp, x]`` in 1D, ``[comp, y, x]`` in 2D.

Workloads (the paper measures on analytic problems only; these are seeded
stand-ins with the shapes and value ranges of its examples):
  * ``paper_burgers1d``  Example 4.1 (u0 = 0.5 + sin x on [-pi, pi]).
  * ``paper_euler1d``    Example 4.2 (rho = 1 + 0.2 sin(pi x), u = 1, P = 1).
  * ``paper_burgers2d``  Example 4.5.
  * ``paper_euler2d``    Example 4.6.
  * ``advection1d_modes``   1D advection, sine plus seeded small Fourier modes.
  * ``euler1d_riemann_sine`` 1D Euler, seeded piecewise-constant states with
    a sinusoidal density perturbation (Shu-Osher-like, Example 4.3 ranges).
  * ``euler2d_smooth``   2D Euler, seeded smooth Fourier-mode perturbations.
  * ``euler2d_quadrants`` 2D Euler, seeded four-quadrant Riemann data.
  * ``mach2000_initial`` the initial state of Example 4.10 (time-step pin).
  * ``blast_wave_1d``    Example 4.4 (Woodward-Colella blast waves between
    two reflective walls).
  * ``rayleigh_taylor``  Example 4.11 (gravity source, walls, fixed states).
  * ``double_mach``      Example 4.7 (double Mach reflection).
  * ``with_bc``          any of the above with other boundary conditions.
"""
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    """An initial state plus the parameters that describe its problem."""
    name: str
    dim: int
    system: str                 # 'advection' | 'burgers' | 'euler'
    nx: int
    ny: int
    dx: float
    dy: float
    U: np.ndarray
    V: np.ndarray
    W: object                   # np.ndarray in 2D, None in 1D
    bc: tuple = ('periodic',) * 4
    gas_gamma: float = 1.4
    adv_a: float = 1.0
    adv_b: float = 1.0
    t_end: float = None
    x: np.ndarray = None
    y: np.ndarray = None
    extra: dict = field(default_factory=dict)
    bc_state: tuple = (None, None, None, None)   # conserved states of 'dirichlet' sides
    gravity: float = 0.0

    def problem_kwargs(self):
        """Keyword arguments shared by the oracle's Problem and the binding."""
        kw = dict(dim=self.dim, nx=self.nx, ny=self.ny, dx=self.dx, dy=self.dy,
                  system=self.system, adv_a=self.adv_a, adv_b=self.adv_b,
                  gas_gamma=self.gas_gamma, bc=tuple(self.bc))
        if any(b is not None for b in self.bc_state):
            kw['bc_state'] = tuple(self.bc_state)
        if self.gravity != 0.0:
            kw['gravity'] = self.gravity
        if 'split' in self.extra:
            kw['split'] = tuple(self.extra['split'])
        return kw


def centres(n, lo, hi):
    h = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * h, h


def conserved_1d(rho, u, p, rx, ux, px, g):
    """(rho, rho u, E) and their x-derivatives from primitives, E = p/(g-1) + rho u^2/2."""
    U = np.stack([rho, rho * u, p / (g - 1.0) + 0.5 * rho * u * u])
    V = np.stack([rx, rx * u + rho * ux, px / (g - 1.0) + 0.5 * rx * u * u + rho * u * ux])
    return U, V


def conserved_2d(rho, u, v, p, dr, du, dv, dp, g):
    """(rho, rho u, rho v, E) and one directional derivative of it."""
    U = np.stack([rho, rho * u, rho * v, p / (g - 1.0) + 0.5 * rho * (u * u + v * v)])
    D = np.stack([dr, dr * u + rho * du, dr * v + rho * dv,
                  dp / (g - 1.0) + 0.5 * dr * (u * u + v * v) + rho * (u * du + v * dv)])
    return U, D


# ---------------------------------------------------------------- paper examples
def paper_burgers1d(n):
    x, h = centres(n, -math.pi, math.pi)
    U = (0.5 + np.sin(x))[None]
    V = np.cos(x)[None]
    return Workload('burgers1d', 1, 'burgers', n, 1, h, 1.0, U, V, None, t_end=0.5, x=x)


def paper_euler1d(n, g=1.4):
    x, h = centres(n, 0.0, 2.0)
    rho = 1.0 + 0.2 * np.sin(math.pi * x)
    rx = 0.2 * math.pi * np.cos(math.pi * x)
    one, zero = np.ones_like(x), np.zeros_like(x)
    U, V = conserved_1d(rho, one, one, rx, zero, zero, g)
    return Workload('euler1d', 1, 'euler', n, 1, h, 1.0, U, V, None, gas_gamma=g, t_end=2.0, x=x)


def paper_burgers2d(n):
    x, h = centres(n, -2 * math.pi, 2 * math.pi)
    X, Y = np.meshgrid(x, x)           # [y, x]
    s = 0.5 * (X + Y)
    U = (0.5 + np.sin(s))[None]
    V = (0.5 * np.cos(s))[None]
    return Workload('burgers2d', 2, 'burgers', n, n, h, h, U, V, V.copy(), t_end=0.5, x=x, y=x)


def paper_euler2d(n, g=1.4):
    x, h = centres(n, 0.0, 2.0)
    X, Y = np.meshgrid(x, x)
    rho = 1.0 + 0.2 * np.sin(math.pi * (X + Y))
    dr = 0.2 * math.pi * np.cos(math.pi * (X + Y))
    one, zero = np.ones_like(X), np.zeros_like(X)
    U, V = conserved_2d(rho, one, one, one, dr, zero, zero, zero, g)
    _, W = conserved_2d(rho, one, one, one, dr, zero, zero, zero, g)
    return Workload('euler2d', 2, 'euler', n, n, h, h, U, V, W, gas_gamma=g, t_end=2.0, x=x, y=x)


def mach2000_initial(nx=640, ny=320, g=5.0 / 3.0):
    """Example 4.10: (rho, u, v, P) = (0.5, 0, 0, 0.4127) on [0,1]x[-0.25,0.25]."""
    x, hx = centres(nx, 0.0, 1.0)
    y, hy = centres(ny, -0.25, 0.25)
    X, Y = np.meshgrid(x, y)
    rho = 0.5 + 0 * X
    zero = 0 * X
    U, V = conserved_2d(rho, zero, zero, 0.4127 + zero, zero, zero, zero, zero, g)
    return Workload('mach2000', 2, 'euler', nx, ny, hx, hy, U, V, V.copy(),
                    bc=('transmissive',) * 4, gas_gamma=g, x=x, y=y)


def blast_wave_1d(n=800, g=1.4):
    """Example 4.4: (rho, u, P) = (1, 0, 1000) on [0, 0.1), (1, 0, 0.01) on
    [0.1, 0.9), (1, 0, 100) on [0.9, 1]; reflective walls at both ends;
    T = 0.038. Piecewise constant, so V = 0."""
    x, h = centres(n, 0.0, 1.0)
    p = np.where(x < 0.1, 1000.0, np.where(x < 0.9, 0.01, 100.0))
    one, zero = np.ones_like(x), np.zeros_like(x)
    U, V = conserved_1d(one, zero, p, zero, zero, zero, g)
    return Workload('blast_wave_1d', 1, 'euler', n, 1, h, 1.0, U, V, None,
                    bc=('reflective', 'reflective', 'periodic', 'periodic'), gas_gamma=g,
                    t_end=0.038, x=x)


def rayleigh_taylor(nx=60, g=5.0 / 3.0):
    """Example 4.11 on [0, 0.25] x [0, 1] with nx x 4nx cells: heavy fluid
    (rho = 2, P = 2y + 1) below y = 1/2, light fluid (rho = 1, P = y + 3/2)
    above, v = -0.025 c cos(8 pi x) with c = sqrt(g P / rho); gravity 1 in +y
    (the source of (euler2d-s)); reflective walls left and right, the fixed
    states (2, 0, 0, 1) below and (1, 0, 0, 2.5) above; T = 1.95. V, W are the
    exact derivatives away from the interface (zero jump contribution)."""
    ny = 4 * nx
    x, hx = centres(nx, 0.0, 0.25)
    y, hy = centres(ny, 0.0, 1.0)
    X, Y = np.meshgrid(x, y)
    low = Y < 0.5
    rho = np.where(low, 2.0, 1.0)
    p = np.where(low, 2.0 * Y + 1.0, Y + 1.5)
    py = np.where(low, 2.0, 1.0)
    c = np.sqrt(g * p / rho)
    cy = g * py / (2.0 * rho * c)
    cosx, sinx = np.cos(8 * math.pi * X), np.sin(8 * math.pi * X)
    v = -0.025 * c * cosx
    vx = 0.025 * c * 8 * math.pi * sinx
    vy = -0.025 * cy * cosx
    zero = np.zeros_like(X)
    U, V = conserved_2d(rho, zero, v, p, zero, zero, vx, zero, g)
    _, W = conserved_2d(rho, zero, v, p, zero, zero, vy, py, g)
    cons = lambda r, pp: (r, 0.0, 0.0, pp / (g - 1.0))
    return Workload('rayleigh_taylor', 2, 'euler', nx, ny, hx, hy, U, V, W,
                    bc=('reflective', 'reflective', 'dirichlet', 'dirichlet'), gas_gamma=g,
                    t_end=1.95, x=x, y=y, bc_state=(None, None, cons(2.0, 1.0), cons(1.0, 2.5)),
                    gravity=1.0)


def double_mach(nx=1600, g=1.4):
    """Example 4.7 on [0, 4] x [0, 1] with nx x nx/4 cells: a Mach 10 shock at
    60 degrees to the x-axis through (1/6, 0); post-shock (rho, u, v, P) =
    (8, 8.25 cos(pi/6), -8.25 sin(pi/6), 116.5) left of x = 1/6 + y/sqrt(3),
    (1.4, 0, 0, 1) right of it; V = W = 0. Boundaries: the post-shock state on
    the left (inflow), transmissive on the right (outflow), on the bottom the
    post-shock state for x < 1/6 and a reflective wall beyond, on the top the
    exact motion of the shock along the line y = 1, x_s = 1/6 + (1 + 20 t)/
    sqrt(3) (post-shock state to its left, pre-shock to its right); T = 0.2.
    The split boundaries are given as dicts (x0, slope, speed, kinds, states)
    for the problem's ``split``."""
    ny = nx // 4
    x, hx = centres(nx, 0.0, 4.0)
    y, hy = centres(ny, 0.0, 1.0)
    X, Y = np.meshgrid(x, y)
    r3 = math.sqrt(3.0)
    post = (8.0, 8.25 * math.cos(math.pi / 6), -8.25 * math.sin(math.pi / 6), 116.5)
    pre = (1.4, 0.0, 0.0, 1.0)
    left = X < 1.0 / 6.0 + Y / r3
    rho, u, v, p = (np.where(left, a, b) for a, b in zip(post, pre))
    zero = np.zeros_like(X)
    U, V = conserved_2d(rho, u, v, p, zero, zero, zero, zero, g)
    cons = lambda q: (q[0], q[0] * q[1], q[0] * q[2], q[3] / (g - 1.0) + 0.5 * q[0] * (q[1] ** 2 + q[2] ** 2))
    bottom = dict(x0=1.0 / 6.0, slope=0.0, speed=0.0, kinds=('dirichlet', 'reflective'),
                  states=(cons(post), None))
    top = dict(x0=1.0 / 6.0 + 1.0 / r3, slope=0.0, speed=20.0 / r3, kinds=('dirichlet', 'dirichlet'),
               states=(cons(post), cons(pre)))
    return Workload('double_mach', 2, 'euler', nx, ny, hx, hy, U, V, V.copy(),
                    bc=('dirichlet', 'transmissive', 'split', 'split'), gas_gamma=g, t_end=0.2,
                    x=x, y=y, bc_state=(cons(post), None, None, None),
                    extra=dict(split=(bottom, top), post=post, pre=pre))


def with_bc(w, bc):
    """A copy of workload ``w`` with boundary conditions ``bc`` (x_lo, x_hi,
    y_lo, y_hi); the data are unchanged."""
    import dataclasses
    return dataclasses.replace(w, bc=tuple(bc), name=f'{w.name}[{",".join(b[0] for b in bc)}]')


# ---------------------------------------------------------------- seeded configs
def advection1d_modes(n, seed=1000, a=1.0):
    """u0 = 0.5 + sin(pi x) + sum_{k=1..4} 1e-3 sin(k pi x + phi_k) on [0, 2],
    periodic, f = a u; exact solution at T = 2/|a| equals u0."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=4)
    x, h = centres(n, 0.0, 2.0)
    u = 0.5 + np.sin(math.pi * x)
    ux = math.pi * np.cos(math.pi * x)
    for k in range(1, 5):
        u = u + 1e-3 * np.sin(k * math.pi * x + phi[k - 1])
        ux = ux + 1e-3 * k * math.pi * np.cos(k * math.pi * x + phi[k - 1])
    return Workload('advection1d', 1, 'advection', n, 1, h, 1.0, u[None], ux[None], None,
                    adv_a=a, t_end=2.0, x=x)


def euler1d_riemann_sine(n=2000, seed=2000, g=1.4):
    """Seeded 1D Riemann data on [-5, 5], transmissive: 2-4 jumps (min gap
    0.5), per segment rho ~ U[0.1,5], u ~ U[-2,2], p ~ U[0.1,10]; density times
    (1 + A sin(m x)), A ~ U[0.1,0.3], m ~ U[3,8]; V from the smooth part
    (jumps contribute zero); end time T ~ U[0.2, 1.8]."""
    rng = np.random.default_rng(seed)
    J = int(rng.integers(2, 5))
    while True:
        pos = np.sort(rng.uniform(-4.5, 4.5, size=J))
        if J == 1 or np.min(np.diff(pos)) >= 0.5:
            break
    seg_rho = rng.uniform(0.1, 5.0, size=J + 1)
    seg_u = rng.uniform(-2.0, 2.0, size=J + 1)
    seg_p = rng.uniform(0.1, 10.0, size=J + 1)
    A = rng.uniform(0.1, 0.3)
    m = rng.uniform(3.0, 8.0)
    T = rng.uniform(0.2, 1.8)
    x, h = centres(n, -5.0, 5.0)
    seg = np.searchsorted(pos, x)
    base = seg_rho[seg]
    rho = base * (1.0 + A * np.sin(m * x))
    rx = base * A * m * np.cos(m * x)
    u, p = seg_u[seg], seg_p[seg]
    zero = np.zeros_like(x)
    U, V = conserved_1d(rho, u, p, rx, zero, zero, g)
    return Workload('euler1d_riemann', 1, 'euler', n, 1, h, 1.0, U, V, None,
                    bc=('transmissive',) * 4, gas_gamma=g, t_end=T, x=x,
                    extra=dict(jumps=pos, A=A, m=m))


def _fourier_field(rng, X, Y, modes=16, kmax=8, yscale=1.0):
    """Sum of ``modes`` waves sin(pi (kx x + ky y) + theta), 1 <= max|k| <=
    kmax, normalised to max |value| = 1 over the grid; returns the field and
    its exact x- and y-derivatives (same normalisation). kx is an integer;
    ky = j yscale with an integer j (yscale = 1: integers), which makes every
    wave periodic on a y-period of 2 / yscale."""
    f = np.zeros_like(X)
    fx = np.zeros_like(X)
    fy = np.zeros_like(X)
    jmax = int(math.floor(kmax / yscale + 1e-12))
    for _ in range(modes):
        while True:
            if yscale == 1.0:
                kx, ky = rng.integers(-kmax, kmax + 1, size=2)
            else:
                kx, j = rng.integers(-kmax, kmax + 1), rng.integers(-jmax, jmax + 1)
                ky = j * yscale
            if max(abs(kx), abs(ky)) >= 1:
                break
        th = rng.uniform(0.0, 2.0 * math.pi)
        arg = math.pi * (kx * X + ky * Y) + th
        f += np.sin(arg)
        c = np.cos(arg)
        fx += math.pi * kx * c
        fy += math.pi * ky * c
    s = np.max(np.abs(f))
    return f / s, fx / s, fy / s


def euler2d_smooth(n, seed=3000, g=1.4, amp=0.2, ny=None):
    """[0,2]^2 periodic; rho = 1 + amp phi_r, u = amp phi_u, v = amp phi_v,
    p = 1; each phi a seeded sum of 16 Fourier modes with max|k| <= 8.
    With ny != n the domain is [0,2] x [0, 2 ny/n] (dy = dx) and the
    y-wavenumbers are multiples of n/ny, so every mode is periodic on it."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    x, hx = centres(n, 0.0, 2.0)
    y, hy = centres(ny, 0.0, 2.0 * ny / n)
    X, Y = np.meshgrid(x, y)
    ys = n / ny
    fr, frx, fry = _fourier_field(rng, X, Y, yscale=ys)
    fu, fux, fuy = _fourier_field(rng, X, Y, yscale=ys)
    fv, fvx, fvy = _fourier_field(rng, X, Y, yscale=ys)
    rho, u, v = 1.0 + amp * fr, amp * fu, amp * fv
    p = np.ones_like(X)
    zero = np.zeros_like(X)
    U, V = conserved_2d(rho, u, v, p, amp * frx, amp * fux, amp * fvx, zero, g)
    _, W = conserved_2d(rho, u, v, p, amp * fry, amp * fuy, amp * fvy, zero, g)
    return Workload('euler2d_smooth', 2, 'euler', n, ny, hx, hy, U, V, W, gas_gamma=g,
                    x=x, y=y)


def euler2d_quadrants(n, seed=4000, g=1.4, ny=None):
    """[0,1]^2, transmissive, quadrants split at (0.5, 0.5); per quadrant rho ~
    U[0.1,5], u, v ~ U[-2,2], p ~ U[0.1,10]; V = W = 0; T = 0.25."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    q = rng.uniform([0.1, -2.0, -2.0, 0.1], [5.0, 2.0, 2.0, 10.0], size=(4, 4))
    x, hx = centres(n, 0.0, 1.0)
    y, hy = centres(ny, 0.0, 1.0)
    X, Y = np.meshgrid(x, y)
    quad = (X >= 0.5).astype(int) + 2 * (Y >= 0.5).astype(int)
    rho, u, v, p = (q[quad, j] for j in range(4))
    zero = np.zeros_like(X)
    U, V = conserved_2d(rho, u, v, p, zero, zero, zero, zero, g)
    return Workload('euler2d_quadrants', 2, 'euler', n, ny, hx, hy, U, V, V.copy(),
                    bc=('transmissive',) * 4, gas_gamma=g, t_end=0.25, x=x, y=y,
                    extra=dict(states=q))


def random_smooth_1d(n, system='burgers', seed=0, g=1.4, bc='periodic'):
    """Small smooth periodic 1D data for parity tests (any system)."""
    rng = np.random.default_rng(seed)
    x, h = centres(n, 0.0, 2.0)
    ph = rng.uniform(0, 2 * math.pi, size=3)
    a = rng.uniform(0.1, 0.3, size=3)
    s = sum(a[k] * np.sin((k + 1) * math.pi * x + ph[k]) for k in range(3))
    sx = sum(a[k] * (k + 1) * math.pi * np.cos((k + 1) * math.pi * x + ph[k]) for k in range(3))
    if system == 'euler':
        one, zero = np.ones_like(x), np.zeros_like(x)
        U, V = conserved_1d(1.0 + 0.5 * s, 0.5 + s, 1.0 + 0.3 * s, 0.5 * sx, sx, 0.3 * sx, g)
    else:
        U, V = (0.5 + s)[None], sx[None]
    return Workload('smooth1d', 1, system, n, 1, h, 1.0, U, V, None,
                    bc=(bc, bc, bc, bc), gas_gamma=g, x=x,
                    adv_a=float(rng.uniform(-1.5, 1.5)) if system == 'advection' else 1.0)
