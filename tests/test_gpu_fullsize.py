"""The 2D Euler smooth periodic workload at full size (1024^2, smooth seeded
Fourier-mode perturbations of rho = 1, p = 1; 100 SSP-RK3 steps), FP64 and
FP32, where the oracle cannot follow a whole run:

* the operator and the first stage at sampled cells against the oracle
  evaluated one cell at a time (FP64: 1e-12 relative; FP32: the bounds of the
  FP32 parity tests);
* over 100 production steps: sum(u) of every component invariant (periodic
  domain, conservative update), and translation covariance (data rolled by
  a whole number of cells gives the rolled result: every cell runs the same
  arithmetic on the same values);
* the FP32 run against the FP64 run (the FP64 path matches the oracle at
  1e-12 on every smaller run), per field, reported and bounded;
and the largest grid one FP64 state array allows (11584^2): the operator
sampled, and the adjoint step by a dot-product test near the array ends.
"""
import numpy as np
import pytest
import torch

from oracle import hweno as O
from paper_2411_11229_amd import workloads as WL

from test_gpu_parity import (RTOL64, dev, f32_bounds, host, oprob, oracle_rhs_at, sample_cells,
                             solver)

pytestmark = pytest.mark.gpu

N, STEPS, SEED = 1024, 100, 3000


def _run(w, precision, roll=(0, 0)):
    dt_ = torch.float64 if precision == 'f64' else torch.float32
    r = lambda a: np.roll(a, roll, axis=(-2, -1))
    s = solver(w, precision=precision)
    U, V, W = dev(r(w.U), dt_), dev(r(w.V), dt_), dev(r(w.W), dt_)
    sums0 = U.double().sum(dim=(1, 2))
    steps, t, dts = s.run(U, V, W, t_end=1e9, max_steps=STEPS)
    s.health()
    return (U, V, W), sums0, U.double().sum(dim=(1, 2)), U.double().abs().sum(dim=(1, 2)), host(dts)


def extended(w):
    """The workload's arrays in x86 extended precision: the oracle then runs
    in it (its FP64 rounding in the derivative equations' residuals reaches
    1e-12 of their scale at 1024^2, where the flux differences cancel)."""
    return WL.Workload(**{**w.__dict__, **{k: getattr(w, k).astype(np.longdouble)
                                           for k in ('U', 'V', 'W')}})


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_smooth_1024_sampled_first_stage(precision):
    """FP64 against the oracle evaluated in extended precision at the sampled
    cells, FP32 against the FP64 oracle with the derived bounds."""
    w = WL.euler2d_smooth(N, seed=SEED)
    if precision == 'f32':
        for k in ('U', 'V', 'W'):
            setattr(w, k, getattr(w, k).astype(np.float32).astype(np.float64))
    p = oprob(w)
    alpha = O.max_speed(p, w.U)
    s = solver(w, precision=precision)
    dt_ = torch.float64 if precision == 'f64' else torch.float32
    U, V, W = dev(w.U, dt_), dev(w.V, dt_), dev(w.W, dt_)
    got = [host(x) for x in s.rhs(U, V, W, dev(np.array(alpha)))]
    cells = sample_cells(w.nx, w.ny, seed=11)
    ref = oracle_rhs_at(extended(w) if precision == 'f64' else w, p, alpha, cells)
    ref = [tuple(np.asarray(x, dtype=np.float64) for x in r) for r in ref]
    tol = f32_bounds(w, alpha) if precision == 'f32' else None
    scale = [max(np.max(np.abs(r[k])) for r in ref) for k in range(5)]
    worst = [0.0] * 5
    for (j, i), r in zip(cells, ref):
        for k in range(5):
            e = np.max(np.abs(got[k][:, j, i] - r[k]))
            lim = RTOL64 * max(scale[k], 1.0) if precision == 'f64' else tol[k]
            worst[k] = max(worst[k], e / max(scale[k], 1.0))
            assert e <= lim, f'cell {(j, i)} output {k}: err {e:.3e} > {lim:.3e}'
    print(f'  {precision}: worst sampled error per output (relative to the output scale) '
          + ' '.join(f'{x:.2e}' for x in worst))


def test_smooth_1024_run_invariants_f64():
    w = WL.euler2d_smooth(N, seed=SEED)
    (U, V, W), s0, s1, scale, dts = _run(w, 'f64')
    drift = ((s1 - s0).abs() / scale).max().item()
    print(f'  conservation: max |sum change| / sum|u| over {STEPS} steps: {drift:.2e}')
    assert drift <= 1e-13
    shift = (301, 17)
    (Ur, Vr, Wr), _, _, _, dts_r = _run(w, 'f64', roll=shift)
    np.testing.assert_array_equal(dts_r, dts)
    for k, (a, b) in enumerate(zip((U, V, W), (Ur, Vr, Wr))):
        ref = np.roll(host(a), shift, axis=(-2, -1))
        e = np.max(np.abs(host(b) - ref)) / np.max(np.abs(ref))
        print(f'  translation by {shift}: field {k} max rel diff {e:.2e}')
        assert e <= 1e-13


def test_smooth_1024_run_f32_against_f64():
    w = WL.euler2d_smooth(N, seed=SEED)
    (U, V, W), _, _, _, dts64 = _run(w, 'f64')
    w32 = WL.euler2d_smooth(N, seed=SEED)
    for k in ('U', 'V', 'W'):
        setattr(w32, k, getattr(w32, k).astype(np.float32).astype(np.float64))
    (U3, V3, W3), s0, s1, scale, dts32 = _run(w32, 'f32')
    # the FP32 fields are stored rounded: sums drift at the FP32 rounding level
    drift = ((s1 - s0).abs() / scale).max().item()
    print(f'  f32 conservation drift over {STEPS} steps: {drift:.2e}')
    assert drift <= 1e-5
    assert np.max(np.abs(dts32 - dts64) / dts64) <= 1e-5
    # per field: max error over the field's max. Measured on MI355X: u 8.2e-7,
    # v~ 1.9e-4, w~ 2.1e-4 (the derivative fields carry the FP32 rounding of
    # the stored fields through 1/dx-scaled differences). Bounds: about 10x.
    bounds = (1e-5, 2e-3, 2e-3)
    for k, (a, b, lim) in enumerate(zip((U, V, W), (U3, V3, W3), bounds)):
        ref = host(a)
        e = np.max(np.abs(host(b).astype(np.float64) - ref)) / np.max(np.abs(ref))
        print(f'  f32 vs f64 after {STEPS} steps: field {k} max rel err {e:.2e} (bound {lim:.0e})')
        assert e <= lim


def _oracle_at_device(p, alpha, U, V, W, cells):
    """The oracle operator at isolated cells, its two 5-cell lines per cell
    read from device arrays (the arrays are too large to copy whole)."""
    from test_gpu_parity import _mapidx
    sy = O.make_system(p)
    g, dl, eps = p.linear_gamma, p.linear_d, p.eps
    out = []
    for (j, i) in cells:
        cols = torch.tensor([_mapidx(i + k, p.nx, p.bc[0], p.bc[1]) for k in range(-2, 3)], device='cuda')
        rows = torch.tensor([_mapidx(j + k, p.ny, p.bc[2], p.bc[3]) for k in range(-2, 3)], device='cuda')
        xl = lambda F: F[:, j, :].index_select(1, cols).double().cpu().numpy()
        yl = lambda F: F[:, :, i].index_select(1, rows).double().cpu().numpy()
        RUx, RVx, RWx, vt = O.sweep(sy, 0, xl(U), xl(V), xl(W), p.dx, alpha[0],
                                    'transmissive', 'transmissive', g, dl, eps)
        RUy, RWy, RVy, wt = O.sweep(sy, 1, yl(U), yl(W), yl(V), p.dy, alpha[1],
                                    'transmissive', 'transmissive', g, dl, eps)
        out.append((RUx[:, 2] + RUy[:, 2], RVx[:, 2] + RVy[:, 2], RWx[:, 2] + RWy[:, 2],
                    vt[:, 2], wt[:, 2]))
    return out


def test_largest_state_array_sampled():
    """The largest 2D Euler FP64 grid one state array allows (4 x 11584^2
    doubles, 4.294e9 bytes, just under the 4 GiB the kernels address with
    32-bit byte offsets), four-quadrant data built on the device: the
    operator and the first stage at sampled cells (corners, the quadrant
    junction, random cells, and the last rows and columns, whose offsets are
    the largest) against the oracle evaluated cell by cell."""
    n = 11584
    assert 4 * n * n * 8 < 2 ** 32
    print(f'case 2D Euler quadrants {n}x{n} FP64', flush=True)
    small = WL.euler2d_quadrants(16, seed=4000)
    kw = dict(small.problem_kwargs(), nx=n, ny=n, dx=1.0 / n, dy=1.0 / n)
    p = O.Problem(**kw)
    alpha = O.max_speed(O.Problem(**small.problem_kwargs()), small.U)   # the same four states
    q = [torch.tensor(small.U[:, a, b], dtype=torch.float64, device='cuda')
         for a, b in ((0, 0), (0, -1), (-1, 0), (-1, -1))]
    xs = (torch.arange(n, device='cuda', dtype=torch.float64) + 0.5) / n
    right = (xs >= 0.5).view(1, 1, n)
    top = (xs >= 0.5).view(1, n, 1)
    col = lambda k: q[k].view(4, 1, 1)
    U = torch.where(top, torch.where(right, col(3), col(2)), torch.where(right, col(1), col(0))).contiguous()
    V = torch.zeros_like(U)
    W = torch.zeros_like(U)
    from paper_2411_11229_amd import hweno
    s = hweno.Solver(hweno.Problem(**kw))
    cells = sample_cells(n, n, k=24, seed=13) + [(n - 1, n - 3), (n - 2, n - 1), (n - 3, 7), (n // 2, n - 2)]
    ref = _oracle_at_device(p, alpha, U, V, W, cells)
    got = s.rhs(U, V, W, dev(np.array(alpha)))
    scale = [max(np.max(np.abs(r[k])) for r in ref) for k in range(5)]
    for (j, i), r in zip(cells, ref):
        for k in range(5):
            e = np.max(np.abs(host(got[k][:, j, i]) - r[k]))
            assert e <= RTOL64 * max(scale[k], 1.0), f'cell {(j, i)} output {k}: err {e:.3e}'
    del got
    torch.cuda.empty_cache()
    stages = torch.empty(2 * 3 * 4 * n * n, dtype=torch.float64, device='cuda')
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    dt_used = torch.zeros(1, dtype=torch.float64, device='cuda')
    U0 = {c: host(U[:, j, i]) for c, (j, i) in enumerate(cells)}
    s.step(U, V, W, t, 1e9, dt_used=dt_used, stages=stages)
    dt = O.time_step(p, alpha, 'production', 0.6)
    assert host(dt_used)[0] == pytest.approx(dt, rel=1e-12, abs=0)
    X1 = stages[:3 * 4 * n * n].view(3, 4, n, n)
    for c, ((j, i), r) in enumerate(zip(cells, ref)):
        exp = (U0[c] + dt * r[0], r[3] + dt * r[1], r[4] + dt * r[2])
        for k in range(3):
            e = np.max(np.abs(host(X1[k][:, j, i]) - exp[k]))
            assert e <= RTOL64 * max(np.max(np.abs(exp[k])), 1.0), f'stage 1 cell {(j, i)} field {k}: {e:.3e}'
    s.health()
    print(f'  {len(cells)} cells within 1e-12; dt {dt:.6e}')
    del stages, U, V, W, s
    torch.cuda.empty_cache()


def test_largest_state_array_adjoint_dot_product():
    """The adjoint step at the largest FP64 grid (11584^2, periodic smooth
    data built on the device) on cotangents and directions supported in the
    last 48 rows only, where the byte offsets are the largest:
    <(dX_{n+1}/dX_n)^T lam, delta> against Richardson central differences
    <lam, (step(X + e delta) - step(X - e delta)) / 2e> of the frozen step."""
    n = 11584
    print(f'case 2D Euler smooth {n}x{n} FP64 adjoint', flush=True)
    from paper_2411_11229_amd import hweno
    g_, h = 1.4, 2.0 / n
    kw = dict(dim=2, nx=n, ny=n, dx=h, dy=h, system='euler', gas_gamma=g_,
              bc=('periodic',) * 4)
    s = hweno.Solver(hweno.Problem(**kw))
    x = (torch.arange(n, device='cuda', dtype=torch.float64) + 0.5) * h
    X_, Y_ = x.view(1, n), x.view(n, 1)
    pi = np.pi
    sx, cx, sy_, cy = torch.sin(pi * X_), torch.cos(pi * X_), torch.sin(pi * Y_), torch.cos(pi * Y_)
    rho = 1 + 0.2 * sx * sy_
    u = 0.2 * cx * sy_
    v = 0.2 * sx * cy
    rx, ry = 0.2 * pi * cx * sy_, 0.2 * pi * sx * cy          # d rho / dx, dy
    ux, uy = -0.2 * pi * sx * sy_, 0.2 * pi * cx * cy
    vx, vy = 0.2 * pi * cx * cy, -0.2 * pi * sx * sy_
    E = 1.0 / (g_ - 1) + 0.5 * rho * (u * u + v * v)

    def cons_d(d_r, d_u, d_v):   # derivative of (rho, rho u, rho v, E) at p = 1
        return torch.stack([d_r, d_r * u + rho * d_u, d_r * v + rho * d_v,
                            0.5 * d_r * (u * u + v * v) + rho * (u * d_u + v * d_v)])
    U = torch.stack([rho, rho * u, rho * v, E]).contiguous()
    V = cons_d(rx, ux, vx).contiguous()
    W = cons_d(ry, uy, vy).contiguous()
    X = [U, V, W]
    del sx, cx, sy_, cy, rho, u, v, rx, ry, ux, uy, vx, vy, E
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    dt = torch.zeros(1, dtype=torch.float64, device='cuda')
    rec = torch.zeros(6, dtype=torch.float64, device='cuda')
    Y = [a.clone() for a in X]
    s.step(Y[0], Y[1], Y[2], t, 1e9, dt_used=dt, alpha_rec=rec)
    del Y
    gen = torch.Generator(device='cuda').manual_seed(17)

    def tail(a):   # random values in the last 48 rows, zero elsewhere
        z = torch.zeros_like(a)
        z[:, -48:, :] = torch.randn(z[:, -48:, :].shape, dtype=a.dtype, device='cuda', generator=gen)
        return z
    lam = [tail(a) for a in X]
    delta = [tail(a) for a in X]
    out = [torch.empty_like(a) for a in X]
    s.adjoint_step(X[0], X[1], X[2], dt, rec, lam, out)
    adj = sum(float((o * d).sum()) for o, d in zip(out, delta))
    del out

    def D(e):
        acc = 0.0
        for sign in (1.0, -1.0):
            Z = [a + sign * e * d for a, d in zip(X, delta)]
            s.step_frozen(Z[0], Z[1], Z[2], dt, rec)
            acc += sign * sum(float((l * z).sum()) for l, z in zip(lam, Z))
            del Z
        return acc / (2 * e)
    e = 1e-7
    fd = (4 * D(e) - D(2 * e)) / 3
    print(f'  adjoint {adj:.12e}  fd {fd:.12e}')
    assert adj == pytest.approx(fd, rel=1e-6, abs=0)
    del X, lam, delta, s
    torch.cuda.empty_cache()
