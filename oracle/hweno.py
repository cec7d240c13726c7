"""Plain FP64 CPU oracle of the fifth-order finite-difference HWENO-I scheme.

TEST INFRASTRUCTURE ONLY. This module is the independent reference that the
HIP path is checked against. Only the test-suite, the package smoke check and
the CPU-baseline leg of the benchmark may import it; the product path never
does, and this module imports nothing from the product package.

Source: Xie, Tao, Jiao, Zhang, "An efficient fifth-order interpolation-based
Hermite WENO scheme for hyperbolic conservation laws" (arXiv 2411.11229).
Every function names the passage it follows (section / equation label).

Style: whole-array operations, one paper step per function, no fusion or
reordering beyond what the equations state. It runs on NumPy float64 arrays
(fast pins) and, unchanged, on torch-CPU float64 tensors (reverse-mode
gradients for the adjoint pins). Array layout: ``U[comp, ..., x]`` with the
sweep axis last; 2D arrays are ``[comp, y, x]``.

Readings of points the paper leaves open (each also listed in the design
notes of the repository):
  * p0 is the quartic through 5 Hermite conditions (the text calls it quintic).
  * u^+ at x_{i-1/2} is the mirror image (about x_i) of the u^- procedure,
    evaluated with the same cell's smoothness indicators.
  * v^{+-} are the linear values p0'(face); nonlinear weights act on u^{+-}
    and on the modified derivative only.
  * The spatial operator sees the unmodified stage derivative; the modified
    derivative only enters as the Runge-Kutta base.
  * LF alpha: global max of the spectral radius over the interior cells of the
    current stage state, per direction.
  * Systems: characteristic variables from the eigenvectors of the flux
    Jacobian at the cell centre U_i, shared by both faces and the centre of
    that cell; R has the textbook columns listed in ``Euler.right_eigvecs``
    and L = R^{-1}. D(f), D(h), LF and the mixed fluxes act component-wise.
  * Transmissive boundary: zero-order extrapolation of U, V and W into the two
    ghost cells.
  * Characteristic basis switch ('interface'): u^-_{i+1/2} and u^+_{i+1/2}
    in the eigenvectors of Roe's average of U_i, U_{i+1} (Jiang and Shu);
    v~ keeps the cell basis.
  * Dirichlet boundary ('dirichlet', the fixed top and bottom states of
    Example 4.11): both ghost cells hold the given state, the derivatives 0.
  * Split y-side ('split', Example 4.7's bottom and top): the rule of a ghost
    cell changes at x = x0 + slope y + speed t, with the stage times
    t, t + dt, t + dt/2 of SSP-RK3.
  * Source term (euler2d-s): S(u) added to L^1, S(v) and S(w) to the
    derivative equations (S is linear in u).
  * Reflective boundary (Euler only): mirror cells with the sign rules of
    (RBC-1d), (RBC-2d-x), (RBC-2d-y); ghost -1-k is the image of cell k.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import _array

NG = 2  # ghost cells per side: the interface x_{i+1/2} reads cells i-1..i+2 (Cd-1)


# ----------------------------------------------------------------------------
# Problem description
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    """Mesh, system and scheme parameters (section 2 and the parameter
    choices at the start of section 4: CFL 0.6, gamma0 0.95 in 1D and 0.99 in
    2D, d0 0.9, epsilon 1e-10 from (nonlinear))."""
    dim: int
    nx: int
    dx: float
    system: str                     # 'advection' | 'burgers' | 'euler'
    ny: int = 1
    dy: float = 1.0
    adv_a: float = 1.0              # advection: f = a u
    adv_b: float = 1.0              # advection: g = b u
    gas_gamma: float = 1.4
    gamma0: float = None            # default 0.95 (1D) / 0.99 (2D)
    d0: float = 0.9
    eps: float = 1e-10
    bc: tuple = ('periodic', 'periodic', 'periodic', 'periodic')  # x_lo x_hi y_lo y_hi
    basis: str = 'cell'             # characteristic basis: 'cell' | 'interface'
    bc_state: tuple = (None, None, None, None)   # conserved ghost state of 'dirichlet' sides
    gravity: float = 0.0            # g of the source term (euler2d-s), 2D Euler only
    split: tuple = (None, None)     # Split rules of 'split' y-sides (y_lo, y_hi)

    def __post_init__(self):
        if self.gamma0 is None:
            self.gamma0 = 0.95 if self.dim == 1 else 0.99
        self.split = tuple(Split(**sp) if isinstance(sp, dict) else sp for sp in self.split)

    @property
    def linear_gamma(self):
        g1 = (1.0 - self.gamma0) / 2.0
        return (self.gamma0, g1, g1)

    @property
    def linear_d(self):
        d1 = (1.0 - self.d0) / 2.0
        return (self.d0, d1, d1)

    @property
    def ncomp(self):
        if self.system == 'euler':
            return 3 if self.dim == 1 else 4
        return 1


# ----------------------------------------------------------------------------
# Flux functions (scalar laws of sections 2-3 and the Euler systems (euler1d),
# (euler2d)); d = 0 is the x-direction, d = 1 the y-direction.
# ----------------------------------------------------------------------------
class Advection:
    """Linear advection, f = a u, g = b u."""
    def __init__(self, a, b):
        self.speed = (a, b)

    def flux(self, U, d):
        return self.speed[d] * U

    def jac_apply(self, U, V, d):
        """f'(u) v: the flux h of (EQ1) / h, xi, eta, theta of (EQ3)."""
        return self.speed[d] * V

    def eig(self, U, d):
        return None

    def max_speed(self, U, d):
        return abs(self.speed[d])


class Burgers:
    """Burgers' equation, f = g = u^2/2 (Examples 4.1 and 4.5)."""
    def flux(self, U, d):
        return 0.5 * U * U

    def jac_apply(self, U, V, d):
        return U * V

    def eig(self, U, d):
        return None

    def max_speed(self, U, d):
        return _array.ns(U).amax(abs(U))


class Euler:
    """Compressible Euler equations with the ideal-gas EOS
    E = P/(gamma-1) + rho |vel|^2 / 2, in 1D (euler1d) and 2D (euler2d)."""
    def __init__(self, gas_gamma, dim):
        self.g = gas_gamma
        self.dim = dim

    def state(self, U):
        """rho, u, v, P and H = (E + P)/rho from U (EOS of (euler1d)/(euler2d))."""
        rho = U[0]
        mu = U[1] / rho
        nu = U[2] / rho if self.dim == 2 else 0.0 * rho
        E = U[-1]
        P = (self.g - 1.0) * (E - 0.5 * rho * (mu * mu + nu * nu))
        H = (E + P) / rho
        return rho, mu, nu, P, H

    def primitives(self, U):
        """state() plus the sound speed c = sqrt(gamma P / rho)."""
        rho, mu, nu, P, H = self.state(U)
        c = _array.ns(U).sqrt(self.g * P / rho)
        return rho, mu, nu, P, c, H

    def flux(self, U, d):
        xp = _array.ns(U)
        rho, mu, nu, P, H = self.state(U)
        E = U[-1]
        if self.dim == 1:
            return xp.stack([rho * mu, rho * mu * mu + P, mu * (E + P)])
        if d == 0:
            return xp.stack([rho * mu, rho * mu * mu + P, rho * mu * nu, mu * (E + P)])
        return xp.stack([rho * nu, rho * mu * nu, rho * nu * nu + P, nu * (E + P)])

    def jacobian(self, U, d):
        """Textbook flux Jacobian dF/dU, shape (..., nc, nc)."""
        xp = _array.ns(U)
        g = self.g
        rho, mu, nu, P, H = self.state(U)
        zero = 0.0 * rho
        one = zero + 1.0
        if self.dim == 1:
            rows = [[zero, one, zero],
                    [0.5 * (g - 3.0) * mu * mu, (3.0 - g) * mu, zero + (g - 1.0)],
                    [mu * (0.5 * (g - 1.0) * mu * mu - H), H - (g - 1.0) * mu * mu, g * mu]]
        else:
            k = 0.5 * (mu * mu + nu * nu)
            if d == 0:
                rows = [[zero, one, zero, zero],
                        [(g - 1.0) * k - mu * mu, (3.0 - g) * mu, -(g - 1.0) * nu, zero + (g - 1.0)],
                        [-mu * nu, nu, mu, zero],
                        [mu * ((g - 1.0) * k - H), H - (g - 1.0) * mu * mu, -(g - 1.0) * mu * nu, g * mu]]
            else:
                rows = [[zero, zero, one, zero],
                        [-mu * nu, nu, mu, zero],
                        [(g - 1.0) * k - nu * nu, -(g - 1.0) * mu, (3.0 - g) * nu, zero + (g - 1.0)],
                        [nu * ((g - 1.0) * k - H), -(g - 1.0) * mu * nu, H - (g - 1.0) * nu * nu, g * nu]]
        return xp.stack([xp.stack(r, axis=-1) for r in rows], axis=-2)

    def jac_apply(self, U, V, d):
        """A(U) V, i.e. h = f'(u) v for the system (EQ1)/(EQ3)."""
        return _array.ns(U).matvec(self.jacobian(U, d), V)

    def right_eigvecs(self, U, d):
        """Columns are right eigenvectors of A(U) for the eigenvalues
        (vel-c, vel, [vel,] vel+c), in the textbook normalisation."""
        xp = _array.ns(U)
        rho, mu, nu, P, c, H = self.primitives(U)
        zero = 0.0 * rho
        one = zero + 1.0
        if self.dim == 1:
            cols = [[one, mu - c, H - mu * c],
                    [one, mu, 0.5 * mu * mu],
                    [one, mu + c, H + mu * c]]
        else:
            k = 0.5 * (mu * mu + nu * nu)
            if d == 0:
                cols = [[one, mu - c, nu, H - mu * c],
                        [one, mu, nu, k],
                        [zero, zero, one, nu],
                        [one, mu + c, nu, H + mu * c]]
            else:
                cols = [[one, mu, nu - c, H - nu * c],
                        [one, mu, nu, k],
                        [zero, one, zero, mu],
                        [one, mu, nu + c, H + nu * c]]
        # R[..., row, col]
        return xp.stack([xp.stack(col, axis=-1) for col in cols], axis=-1)

    def eig(self, U, d):
        """(L, R) at every point, L = R^{-1} (local characteristic
        decomposition, remarks after Step 4 of section 2 and of section 3)."""
        xp = _array.ns(U)
        R = self.right_eigvecs(U, d)
        return xp.inv(R), R

    def max_speed(self, U, d):
        xp = _array.ns(U)
        rho, mu, nu, P, c, H = self.primitives(U)
        vel = mu if d == 0 else nu
        return xp.amax(abs(vel) + c)


def roe_state(sys, UL, UR):
    """A state whose flux Jacobian is Roe's average matrix of UL and UR (the
    interface basis of Jiang and Shu's characteristic decomposition, cited by
    the remark on systems in section 2): the sqrt(rho)-weighted averages of the
    velocities and of the total enthalpy H, the density sqrt(rho_L rho_R), and
    the pressure that gives the averaged sound speed
    c^2 = (gamma-1)(H - |vel|^2/2). The Jacobian depends on the velocities and
    H only, so its eigenvectors are Roe's."""
    rl, ul, vl, _, hl = sys.state(UL)
    rr, ur, vr, _, hr = sys.state(UR)
    xp = _array.ns(UL)
    wl, wr = xp.sqrt(rl), xp.sqrt(rr)
    u = (wl * ul + wr * ur) / (wl + wr)
    v = (wl * vl + wr * vr) / (wl + wr)
    H = (wl * hl + wr * hr) / (wl + wr)
    rho = wl * wr
    k = 0.5 * (u * u + v * v)
    c2 = (sys.g - 1.0) * (H - k)
    P = rho * c2 / sys.g
    E = P / (sys.g - 1.0) + rho * k
    if sys.dim == 1:
        return xp.stack([rho, rho * u, E])
    return xp.stack([rho, rho * u, rho * v, E])


def make_system(prob):
    if prob.system == 'advection':
        return Advection(prob.adv_a, prob.adv_b)
    if prob.system == 'burgers':
        return Burgers()
    if prob.system == 'euler':
        return Euler(prob.gas_gamma, prob.dim)
    raise ValueError(prob.system)


# ----------------------------------------------------------------------------
# Boundary: ghost cells by index map
# ----------------------------------------------------------------------------
# Reflective walls, remarks of sections 2 and 3 (RBC-1d), (RBC-2d-x),
# (RBC-2d-y): the ghost state is the mirror image of the interior about the
# wall, with the normal momentum negated; a derivative along the wall normal
# changes sign once more, a derivative along the wall does not. Per-component
# signs of (U, V = U_x, W = U_y) for a wall normal to direction d (Euler only;
# the paper states no reflective rule for the scalar laws).
REFLECT_SIGNS = {
    (1, 0): ((1.0, -1.0, 1.0), (-1.0, 1.0, -1.0), None),                    # (RBC-1d)
    (2, 0): ((1.0, -1.0, 1.0, 1.0), (-1.0, 1.0, -1.0, -1.0), (1.0, -1.0, 1.0, 1.0)),   # (RBC-2d-x)
    (2, 1): ((1.0, 1.0, -1.0, 1.0), (1.0, 1.0, -1.0, 1.0), (-1.0, -1.0, 1.0, -1.0)),  # (RBC-2d-y)
}


def reflect_signs(sys, d):
    """Signs of (U, along-derivative, other derivative) at a wall normal to
    direction d, in the order ``sweep`` receives its arrays: the along
    derivative is V for x-walls and W for y-walls. None for scalar laws."""
    if not isinstance(sys, Euler):
        return None, None, None
    sU, sV, sW = REFLECT_SIGNS[(sys.dim, d)]
    return (sU, sV, sW) if d == 0 else (sU, sW, sV)


def pad(a, bc_lo, bc_hi, axis=-1, sign=None, fixed=(None, None)):
    """Add NG ghost cells on both ends of ``axis`` (the last one for the
    reflective and fixed rules). 'periodic' wraps; 'transmissive' copies the
    nearest interior cell (zero-order extrapolation of U and of its
    derivatives); 'reflective' takes the mirror cell (ghost -1-k is the image
    of cell k, ghost n+k of cell n-1-k) with component c multiplied by
    sign[c]; 'dirichlet' puts the side's given value (fixed[0] below,
    fixed[1] above: a per-component sequence) in both ghost cells."""
    xp = _array.ns(a)
    n = a.shape[axis]
    idx, flip, fix = [], [], []
    for i in range(-NG, n + NG):
        fix.append(None)
        if 0 <= i < n:
            idx.append(i)
            flip.append(False)
            continue
        side = bc_lo if i < 0 else bc_hi
        if side == 'periodic':
            idx.append(i % n)
        elif side == 'transmissive':
            idx.append(min(max(i, 0), n - 1))
        elif side == 'reflective':
            if sign is None:
                raise ValueError('reflective walls are defined for the Euler equations only')
            idx.append(-1 - i if i < 0 else 2 * n - 1 - i)
        elif side == 'dirichlet':
            idx.append(0)
            fix[-1] = fixed[0] if i < 0 else fixed[1]
            if fix[-1] is None:
                raise ValueError('dirichlet side without a state')
        else:
            raise ValueError(side)
        flip.append(side == 'reflective')
    out = xp.take(a, idx, axis)
    if any(f is not None for f in fix):
        assert axis in (-1, a.ndim - 1)
        keep = np.ones((a.shape[0], len(idx)))
        add = np.zeros((a.shape[0], len(idx)))
        for j, f in enumerate(fix):
            if f is not None:
                keep[:, j] = 0.0
                add[:, j] = f
        shape = (a.shape[0],) + (1,) * (a.ndim - 2) + (len(idx),)
        out = out * xp.const(keep.reshape(shape), a) + xp.const(add.reshape(shape), a)
    if not any(flip):
        return out
    assert axis in (-1, a.ndim - 1)
    fac = np.ones((a.shape[0], len(idx)))
    for j, f in enumerate(flip):
        if f:
            fac[:, j] = sign
    fac = fac.reshape((a.shape[0],) + (1,) * (a.ndim - 2) + (len(idx),))
    return out * xp.const(fac, a)


@dataclass
class Split:
    """A y-side whose rule changes along x and in time (Example 4.7's bottom
    and top): ghost cell (x, y) at time t follows rule kinds[0] where
    x < x0 + slope y + speed t, else kinds[1]; a 'dirichlet' kind holds
    states[k] (conserved), with zero derivatives. Coordinates: cell centres
    with the domain's lower-left corner at (0, 0)."""
    x0: float
    slope: float
    speed: float
    kinds: tuple
    states: tuple = (None, None)


def pad_lines(a, lo, hi, sign, fixed, deriv=False, xc=None, yg=None, t=0.0):
    """``pad`` along the last axis where an end may be a ``Split`` (y-sides
    only, arrays transposed to [comp, x, y]): each split end is padded under
    both of its kinds and every ghost cell takes the kind its position
    selects. deriv: ``a`` is a derivative field (zero in fixed-state
    ghosts); xc: cell-centre x; yg: the ghost-row centres y (low pair, high
    pair) in padded order; t: the stage time."""
    xp = _array.ns(a)
    plain = lambda e: 'transmissive' if isinstance(e, Split) else e
    base = pad(a, plain(lo), plain(hi), sign=sign, fixed=fixed)
    if not isinstance(lo, Split) and not isinstance(hi, Split):
        return base
    n = a.shape[-1]
    npad = n + 2 * NG
    out = base
    for end, sp in ((0, lo), (1, hi)):
        if not isinstance(sp, Split):
            continue
        cols = [0, 1] if end == 0 else [n + NG, n + NG + 1]
        ys = yg[:2] if end == 0 else yg[2:]
        pads = []
        for k in range(2):
            kind = sp.kinds[k]
            st = None
            if kind == 'dirichlet':
                st = [0.0] * a.shape[0] if deriv else sp.states[k]
            ends = [plain(lo), plain(hi)]
            ends[end] = kind
            fx = list(fixed)
            fx[end] = st
            pads.append(pad(a, ends[0], ends[1], sign=sign, fixed=tuple(fx)))
        m = np.zeros((len(xc), npad))
        own = np.zeros((len(xc), npad))
        for j, y in zip(cols, ys):
            m[:, j] = (np.asarray(xc) < sp.x0 + sp.slope * y + sp.speed * t).astype(float)
            own[:, j] = 1.0
        shape = (1, len(xc), npad)
        m, own = m.reshape(shape), own.reshape(shape)
        out = (out * xp.const(1.0 - own, a) + pads[0] * xp.const(own * m, a)
               + pads[1] * xp.const(own * (1.0 - m), a))
    return out


# ----------------------------------------------------------------------------
# Section 2.1: HWENO interpolation on one cell (scalar data, vectorised)
# ----------------------------------------------------------------------------
def candidates_at_right_face(um, u0, up, vm, vp, dx):
    """(Pxi) and (P'xi): p0, p1, p2 and p0' at x_{i+1/2}."""
    p0 = -um / 8.0 + 9.0 / 16.0 * u0 + 9.0 / 16.0 * up - dx * (3.0 / 64.0 * vm + 9.0 / 64.0 * vp)
    p1 = -0.5 * um + 1.5 * u0
    p2 = 0.5 * u0 + 0.5 * up
    dp0 = (3.0 / 16.0 * um - 1.5 * u0 + 21.0 / 16.0 * up) / dx + vm / 16.0 - 3.0 / 16.0 * vp
    return p0, p1, p2, dp0


def candidate_derivatives_at_centre(um, u0, up, vm, vp, dx):
    """(limiter-p): p0', p1', p2' at x_i."""
    dp0 = 3.0 / (4.0 * dx) * (up - um) - 0.25 * (vm + vp)
    dp1 = (u0 - um) / dx
    dp2 = (up - u0) / dx
    return dp0, dp1, dp2


def smoothness_indicators(um, u0, up, vm, vp, dx):
    """(GHYZ) in the closed form printed after it: beta0 via a1..a4, beta1,
    beta2."""
    a1 = -dx / 4.0 * (vm + vp) + 0.75 * (up - um)
    a2 = dx / 4.0 * (vm - vp) + (um - 2.0 * u0 + up)
    a3 = dx / 4.0 * (vm + vp) + 0.25 * (um - up)
    a4 = dx / 4.0 * (vp - vm) - 0.5 * (um - 2.0 * u0 + up)
    b0 = ((a1 + a3 / 4.0) ** 2 + 13.0 / 3.0 * (a2 + 63.0 / 130.0 * a4) ** 2
          + 781.0 / 20.0 * a3 ** 2 + 1421461.0 / 2275.0 * a4 ** 2)
    b1 = (u0 - um) ** 2
    b2 = (u0 - up) ** 2
    return b0, b1, b2


def nonlinear_weights(b0, b1, b2, lin, eps):
    """(nonlinear): omega_l = wbar_l / sum, wbar_l = lin_l (1 + tau/(beta_l+eps)),
    tau = (|beta0-beta1| + |beta0-beta2|)^2 / 4."""
    tau = 0.25 * (abs(b0 - b1) + abs(b0 - b2)) ** 2
    w0 = lin[0] * (1.0 + tau / (b0 + eps))
    w1 = lin[1] * (1.0 + tau / (b1 + eps))
    w2 = lin[2] * (1.0 + tau / (b2 + eps))
    s = w0 + w1 + w2
    return w0 / s, w1 / s, w2 / s


def hweno_combine(w, lin, q0, q1, q2):
    """The combination of (interp) / (limiter):
    w0 (q0/lin0 - lin1/lin0 q1 - lin2/lin0 q2) + w1 q1 + w2 q2."""
    return (w[0] * (q0 / lin[0] - lin[1] / lin[0] * q1 - lin[2] / lin[0] * q2)
            + w[1] * q1 + w[2] * q2)


def hweno_cell(um, u0, up, vm, vp, dx, lin_gamma, lin_d, eps):
    """One HWENO-I application on cell i (section 2.1), from u_{i-1}, u_i,
    u_{i+1}, v_{i-1}, v_{i+1}. Returns

        uR = u^-_{i+1/2}, uL = u^+_{i-1/2}   (interp), nonlinear
        vR = v^-_{i+1/2}, vL = v^+_{i-1/2}   (interp), = p0' (linear)
        vt = modified derivative at x_i      (limiter)

    The left face is the mirror image of the right-face procedure about x_i
    (u_{i-1} <-> u_{i+1}, v -> -v), as the text prescribes; the mirrored
    stencils swap beta1 and beta2.
    """
    b0, b1, b2 = smoothness_indicators(um, u0, up, vm, vp, dx)
    # right face x_{i+1/2}
    wg = nonlinear_weights(b0, b1, b2, lin_gamma, eps)
    p0, p1, p2, dp0 = candidates_at_right_face(um, u0, up, vm, vp, dx)
    uR = hweno_combine(wg, lin_gamma, p0, p1, p2)
    vR = dp0
    # left face x_{i-1/2}: the same procedure on the mirrored data
    wg_m = nonlinear_weights(b0, b2, b1, lin_gamma, eps)
    q0, q1, q2, dq0 = candidates_at_right_face(up, u0, um, -vp, -vm, dx)
    uL = hweno_combine(wg_m, lin_gamma, q0, q1, q2)
    vL = -dq0
    # modified derivative at x_i (limiter), weights with the linear weights d
    wd = nonlinear_weights(b0, b1, b2, lin_d, eps)
    d0, d1, d2 = candidate_derivatives_at_centre(um, u0, up, vm, vp, dx)
    vt = hweno_combine(wd, lin_d, d0, d1, d2)
    return uR, uL, vR, vL, vt


# ----------------------------------------------------------------------------
# Section 2.2: central Hermite approximation of D(f), D(h)
# ----------------------------------------------------------------------------
def central_D(fm1, f0, fp1, fp2, hm1, hp2, dx):
    """(Pc)-(Cd-1)-(DfDh) at x_{i+1/2} from f_{i-1..i+2}, h_{i-1}, h_{i+2}."""
    s = fm1 - f0 - fp1 + fp2
    d2P = 9.0 / 8.0 * s + 5.0 / 12.0 * dx * (hm1 - hp2)
    d3P = (-(101.0 / 36.0 * fm1 - 27.0 / 4.0 * f0 + 27.0 / 4.0 * fp1 - 101.0 / 36.0 * fp2) / dx
           - 5.0 / 6.0 * (hm1 + hp2))
    d4P = -3.0 * s - 2.0 * dx * (hm1 - hp2)
    d5P = ((130.0 / 9.0 * fm1 - 30.0 * f0 + 30.0 * fp1 - 130.0 / 9.0 * fp2) / dx
           + 20.0 / 3.0 * (hm1 + hp2))
    Df = -d2P / 24.0 + 7.0 / 5760.0 * d4P
    Dh = -d3P / 24.0 + 7.0 / 5760.0 * d5P
    return Df, Dh


def mixed_flux(e_m1, e0, e_p1, e_p2):
    """(mixed): fourth-order linear interface value of a mixed-derivative flux."""
    return (-e_m1 + 7.0 * e0 + 7.0 * e_p1 - e_p2) / 12.0


def lax_friedrichs(fm, fp, um, up, alpha):
    """(flux-LF): 1/2 (f(u^-) + f(u^+) - alpha (u^+ - u^-))."""
    return 0.5 * (fm + fp - alpha * (up - um))


# ----------------------------------------------------------------------------
# One directional sweep: Steps 1-3 of section 2 (and Steps 1/2 of section 3)
# ----------------------------------------------------------------------------
def sweep(sys, d, U, A, B, h, alpha, bc_lo, bc_hi, lin_gamma, lin_d, eps, basis='cell',
          state=(None, None), geo=None):
    """HWENO-I procedure along the last axis for direction ``d``.

    U: state; A: derivative along the sweep (v for x, w for y); B: the other
    derivative (w for x, v for y) or None in 1D. Returns the residual
    contributions -(F_{i+1/2} - F_{i-1/2})/h of the three equations
    (u-equation, A-equation, B-equation via the mixed flux) and the modified
    derivative A~ at the interior cells. ``geo`` (y-sweep with split sides):
    dict(xc=..., yg=..., t=...) for ``pad_lines``.
    """
    xp = _array.ns(U)
    n = U.shape[-1]
    sU, sA, sB = reflect_signs(sys, d)
    zero = [0.0] * U.shape[0]
    geo = geo or {}
    Up = pad_lines(U, bc_lo, bc_hi, sU, state, False, **geo)
    Ap = pad_lines(A, bc_lo, bc_hi, sA, (zero, zero), True, **geo)
    # HWENO on cells -1..n (padded 1..n+2): interfaces -1/2..n-1/2 need them
    m, c, p = (slice(0, n + 2), slice(1, n + 3), slice(2, n + 4))
    Um, U0, Upl = Up[..., m], Up[..., c], Up[..., p]
    Am, Apl = Ap[..., m], Ap[..., p]
    eig = sys.eig(U0, d)
    if eig is None:
        wm, w0, wp, am, ap = Um, U0, Upl, Am, Apl
    else:  # local characteristic decomposition with the cell-centre basis
        Lc, Rc = eig
        wm, w0, wp = xp.matvec(Lc, Um), xp.matvec(Lc, U0), xp.matvec(Lc, Upl)
        am, ap = xp.matvec(Lc, Am), xp.matvec(Lc, Apl)
    uR, uL, _, _, vt = hweno_cell(wm, w0, wp, am, ap, h, lin_gamma, lin_d, eps)
    if eig is not None:
        uR, uL, vt = xp.matvec(Rc, uR), xp.matvec(Rc, uL), xp.matvec(Rc, vt)
    if eig is not None and basis == 'interface':
        # Jiang-Shu: the face values of cell j in the basis of that face (Roe
        # average of the two cells sharing it); v~ stays in the cell basis.
        # Interfaces between padded cells m and m+1, m = 0..n+2.
        Lh, Rh = sys.eig(roe_state(sys, Up[..., :-1], Up[..., 1:]), d)
        def in_basis(Lb):
            pr = lambda X: xp.matvec(Lb, X)
            return hweno_cell(pr(Um), pr(U0), pr(Upl), pr(Am), pr(Apl), h, lin_gamma, lin_d, eps)
        uR = xp.matvec(Rh[..., 1:n + 3, :, :], in_basis(Lh[..., 1:n + 3, :, :])[0])
        uL = xp.matvec(Rh[..., 0:n + 2, :, :], in_basis(Lh[..., 0:n + 2, :, :])[1])
    elif basis != 'cell':
        if eig is not None:
            raise ValueError(basis)
    # v^{+-} = p0'(faces): linear in the data, so taken component-wise
    _, _, vR, vL, _ = hweno_cell(Um, U0, Upl, Am, Apl, h, lin_gamma, lin_d, eps)
    # interface k+1/2 for k=-1..n-1: minus side from cell k, plus side from k+1
    u_minus, u_plus = uR[..., 0:n + 1], uL[..., 1:n + 2]
    v_minus, v_plus = vR[..., 0:n + 1], vL[..., 1:n + 2]
    # pointwise fluxes at all padded cells, from the unmodified stage data
    f = sys.flux(Up, d)
    hf = sys.jac_apply(Up, Ap, d)
    q = [slice(j, j + n + 1) for j in range(4)]     # cells k-1, k, k+1, k+2
    Df, Dh = central_D(f[..., q[0]], f[..., q[1]], f[..., q[2]], f[..., q[3]],
                       hf[..., q[0]], hf[..., q[3]], h)
    F = lax_friedrichs(sys.flux(u_minus, d), sys.flux(u_plus, d), u_minus, u_plus, alpha) + Df
    Hh = lax_friedrichs(sys.jac_apply(u_minus, v_minus, d), sys.jac_apply(u_plus, v_plus, d),
                        v_minus, v_plus, alpha) + Dh
    RU = -(F[..., 1:] - F[..., :-1]) / h
    RA = -(Hh[..., 1:] - Hh[..., :-1]) / h
    RB = None
    if B is not None:
        Bp = pad_lines(B, bc_lo, bc_hi, sB, (zero, zero), True, **geo)
        e = sys.jac_apply(Up, Bp, d)
        Eh = mixed_flux(e[..., q[0]], e[..., q[1]], e[..., q[2]], e[..., q[3]])
        RB = -(Eh[..., 1:] - Eh[..., :-1]) / h
    return RU, RA, RB, vt[..., 1:n + 1]


# ----------------------------------------------------------------------------
# Semi-discrete operator (odeH) / (ode2H)
# ----------------------------------------------------------------------------
def max_speed(prob, U):
    """alpha = max |f'(u)| per direction over the interior cells (flux-LF)."""
    sys = make_system(prob)
    ax = sys.max_speed(U, 0)
    ay = sys.max_speed(U, 1) if prob.dim == 2 else 0.0
    return (ax, ay)


def rhs(prob, U, V, W=None, alpha=None, t=0.0):
    """L^1, L^2 (, L^3) of (odeH)/(ode2H) and the modified derivatives
    v~ (, w~) of (limiter), for one stage state at time t (which only
    time-dependent boundaries see). Returns (L1, L2, L3, vt, wt); L3, wt are
    None in 1D."""
    sys = make_system(prob)
    if alpha is None:
        alpha = max_speed(prob, U)
    g, dl, eps, bs = prob.linear_gamma, prob.linear_d, prob.eps, prob.basis
    bx0, bx1, by0, by1 = prob.bc
    st = prob.bc_state
    if prob.dim == 1:
        L1, L2, _, vt = sweep(sys, 0, U, V, None, prob.dx, alpha[0], bx0, bx1, g, dl, eps, bs,
                              (st[0], st[1]))
        return L1, L2, None, vt, None
    xp = _array.ns(U)
    time = t
    # Step 1: x-direction on (u, v); mixed flux eta = f'(u) w
    Lx1, Lx2, Lx3, vt = sweep(sys, 0, U, V, W, prob.dx, alpha[0], bx0, bx1, g, dl, eps, bs,
                              (st[0], st[1]))
    # Step 2: y-direction on (u, w); mixed flux xi = g'(u) v
    t = lambda a: xp.moveaxis(a, -1, -2)
    geo = None
    if prob.split[0] is not None or prob.split[1] is not None:
        by0 = prob.split[0] if by0 == 'split' else by0
        by1 = prob.split[1] if by1 == 'split' else by1
        hy = prob.dy
        geo = dict(xc=(np.arange(prob.nx) + 0.5) * prob.dx,
                   yg=[-1.5 * hy, -0.5 * hy, (prob.ny + 0.5) * hy, (prob.ny + 1.5) * hy], t=time)
    Ly1, Ly3, Ly2, wt = sweep(sys, 1, t(U), t(W), t(V), prob.dy, alpha[1], by0, by1, g, dl, eps, bs,
                              (st[2], st[3]), geo)
    # Step 4
    L1, L2, L3 = Lx1 + t(Ly1), Lx2 + t(Ly2), Lx3 + t(Ly3)
    if prob.gravity != 0.0:
        L1, L2, L3 = L1 + gravity_source(prob, U), L2 + gravity_source(prob, V), L3 + gravity_source(prob, W)
    return L1, L2, L3, vt, t(wt)


def gravity_source(prob, X):
    """The source of (euler2d-s), S(U) = g (0, 0, rho, rho v). It is linear in
    U, so the equations of the derivatives v = u_x, w = u_y (obtained by
    differentiating (euler2d-s)) carry S(v) and S(w)."""
    if prob.system != 'euler' or prob.dim != 2:
        raise ValueError('the gravity source is defined for the 2D Euler equations')
    xp = _array.ns(X)
    z = 0.0 * X[0]
    return xp.stack([z, z, prob.gravity * X[0], prob.gravity * X[2]])


# ----------------------------------------------------------------------------
# Time stepping: (fully-hweno) / (2Dfully-hweno)
# ----------------------------------------------------------------------------
def time_step(prob, alpha, rule='production', cfl=0.6):
    """Delta t from the stage-1 alphas. 'production': cfl/(ax/dx + ay/dy).
    'accuracy': cfl/(ax/dx^{5/3} + ay/dy^{5/3}), the usual choice that makes
    the third-order time error O(dx^5) in the accuracy tests."""
    ax, ay = alpha
    if rule == 'production':
        den = ax / prob.dx + (ay / prob.dy if prob.dim == 2 else 0.0)
    elif rule == 'accuracy':
        den = ax / prob.dx ** (5.0 / 3.0) + (ay / prob.dy ** (5.0 / 3.0) if prob.dim == 2 else 0.0)
    else:
        raise ValueError(rule)
    return cfl / den


def step(prob, U, V, W, dt, alphas=None, t=0.0):
    """One SSP-RK3 step from time t with the modified derivatives as the RK
    base; the stages see the times t, t + dt, t + dt/2 (SSP-RK3's abscissae,
    for time-dependent boundaries). ``alphas``: optional fixed LF alphas for
    the three stages (frozen-alpha mode used for the adjoint); otherwise each
    stage takes alpha from its own state. Returns (U, V, W, alphas_used)."""
    a = [None, None, None] if alphas is None else list(alphas)
    two = prob.dim == 2
    a[0] = a[0] if a[0] is not None else max_speed(prob, U)
    L1, L2, L3, vt0, wt0 = rhs(prob, U, V, W, a[0], t)
    U1 = U + dt * L1
    V1 = vt0 + dt * L2
    W1 = wt0 + dt * L3 if two else None
    a[1] = a[1] if a[1] is not None else max_speed(prob, U1)
    L1, L2, L3, vt1, wt1 = rhs(prob, U1, V1, W1, a[1], t + dt)
    U2 = 0.75 * U + 0.25 * (U1 + dt * L1)
    V2 = 0.75 * vt0 + 0.25 * (vt1 + dt * L2)
    W2 = 0.75 * wt0 + 0.25 * (wt1 + dt * L3) if two else None
    a[2] = a[2] if a[2] is not None else max_speed(prob, U2)
    L1, L2, L3, vt2, wt2 = rhs(prob, U2, V2, W2, a[2], t + 0.5 * dt)
    U3 = U / 3.0 + 2.0 / 3.0 * (U2 + dt * L1)
    V3 = vt0 / 3.0 + 2.0 / 3.0 * (vt2 + dt * L2)
    W3 = wt0 / 3.0 + 2.0 / 3.0 * (wt2 + dt * L3) if two else None
    return U3, V3, W3, tuple(a)


@dataclass
class RunLog:
    steps: int = 0
    t: float = 0.0
    dts: list = field(default_factory=list)
    alphas: list = field(default_factory=list)


def run(prob, U, V, W, t_end, rule='production', cfl=0.6, max_steps=None, log=None):
    """Advance to t_end (the last step is clipped to land on t_end), or for
    ``max_steps`` steps if that comes first. Delta t from the alphas of the
    step's initial state."""
    log = log if log is not None else RunLog()
    t = log.t
    while t < t_end and (max_steps is None or log.steps < max_steps):
        alpha = max_speed(prob, U)
        dt = time_step(prob, alpha, rule, cfl)
        last = t + dt >= t_end
        if last:
            dt = t_end - t
        U, V, W, al = step(prob, U, V, W, dt, (alpha, None, None), t)
        t = t_end if last else t + dt
        log.steps += 1
        log.dts.append(dt)
        log.alphas.append(al)
    log.t = t
    return U, V, W, log


def run_fixed(prob, U, V, W, dts, alphas):
    """Frozen-alpha rollout: the recorded dt per step and alphas per stage.
    Differentiable end to end when given torch tensors."""
    for dt, al in zip(dts, alphas):
        U, V, W, _ = step(prob, U, V, W, dt, al)
    return U, V, W
