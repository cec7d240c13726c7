"""Split (position- and time-dependent) y-sides on the HIP path against the
FP64 oracle, and Example 4.7 (double Mach reflection) on the GPU.

Stage times: the top side of Example 4.7 moves with t, so one step compares
the three stage times t, t + dt, t + dt/2 of both implementations. The start:
five steps at CFL 0.1 (a Mach 10 shock with V = W = 0 overshoots to negative
pressure in the first stage at CFL 0.6, as Example 4.4's blast waves do),
then 0.6.
"""
import math

import numpy as np
import pytest
import torch

from oracle import hweno as O
from paper_2411_11229_amd import workloads as WL

from test_gpu_parity import (RTOL64, check_run, dev, f32_bounds, host, oprob, oracle_sensitivity,
                             solver)

pytestmark = pytest.mark.gpu
R3 = math.sqrt(3.0)


def _scale(w, k, r):
    scale = np.max(np.abs(r))
    if k >= 3:
        ax, h, D = (-1, w.dx, w.V) if k == 3 else (-2, w.dy, w.W)
        scale = max(scale, np.max(np.abs(np.diff(w.U, axis=ax))) / h, np.max(np.abs(D)))
    return scale


def cases():
    s = WL.euler2d_smooth(121, seed=3701, ny=45)
    s.bc = ('periodic', 'periodic', 'split', 'split')
    st = tuple(s.U[:, 0, 0])
    s.extra = dict(split=(dict(x0=0.9, slope=0.0, speed=0.0, kinds=('reflective', 'transmissive'),
                               states=(None, None)),
                          dict(x0=1.3, slope=-0.5, speed=0.0, kinds=('transmissive', 'dirichlet'),
                               states=(None, st))))
    return [('dmr-96x24', WL.double_mach(96)), ('dmr-160x40', WL.double_mach(160)),
            ('smooth-121x45-split', s)]


@pytest.mark.parametrize("name,w", cases(), ids=[c[0] for c in cases()])
def test_split_rhs_matches_oracle_f64(name, w):
    print(f'case {name}', flush=True)
    s = solver(w)
    p = oprob(w)
    alpha = O.max_speed(p, w.U)
    ref = O.rhs(p, w.U, w.V, w.W, alpha)
    got = s.rhs(dev(w.U), dev(w.V), dev(w.W), dev(np.array(alpha)))
    for k, (g, r) in enumerate(zip(got, ref)):
        e = np.max(np.abs(host(g) - r)) / _scale(w, k, r)
        print(f'  output {k}: rel err {e:.3e}')
        assert e <= RTOL64, f'{name} output {k}: {e:.3e}'


@pytest.mark.parametrize("name,w", [cases()[0], cases()[2]], ids=[cases()[k][0] for k in (0, 2)])
def test_split_rhs_f32(name, w):
    """The FP32 form with split sides against the FP64 oracle on the same
    (FP32-rounded) data, within the derived FP32 bounds."""
    print(f'case {name} f32', flush=True)
    for k in ('U', 'V', 'W'):
        setattr(w, k, getattr(w, k).astype(np.float32).astype(np.float64))
    s = solver(w, precision='f32')
    p = oprob(w)
    alpha = O.max_speed(p, w.U)
    f32 = lambda a: dev(a, torch.float32)
    got = s.rhs(f32(w.U), f32(w.V), f32(w.W), dev(np.array(alpha)))
    ref = O.rhs(p, w.U, w.V, w.W, alpha)
    tol = f32_bounds(w, alpha)
    for k, (g, r) in enumerate(zip(got, ref)):
        err = np.max(np.abs(host(g) - r))
        print(f'  output {k}: abs err {err:.3e}  bound {tol[k]:.3e}')
        assert err <= tol[k], f'output {k}: abs err {err:.3e} > bound {tol[k]:.3e}'


def _steps(s, U, V, W, n, t_end=1e9):
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    for k in range(n):
        s.step(U, V, W, t, t_end, cfl=0.1 if k < 5 else 0.6)
    return float(t.item())


def _oracle_steps(p, U, V, W, n):
    t = 0.0
    for k in range(n):
        alpha = O.max_speed(p, U)
        dt = O.time_step(p, alpha, 'production', 0.1 if k < 5 else 0.6)
        U, V, W, _ = O.step(p, U, V, W, dt, (alpha, None, None), t)
        t += dt
    return U, V, W, t


def test_split_step_with_moving_side_matches_oracle():
    w = WL.double_mach(96)
    s = solver(w)
    U, V, W = dev(w.U), dev(w.V), dev(w.W)
    _steps(s, U, V, W, 1)
    p = oprob(w)
    Uo, Vo, Wo, _ = _oracle_steps(p, w.U, w.V, w.W, 1)
    for k, (g, r) in enumerate(zip((U, V, W), (Uo, Vo, Wo))):
        e = np.max(np.abs(host(g) - r)) / np.max(np.abs(r))
        print(f'  field {k}: rel err {e:.3e}')
        assert e <= RTOL64


def test_double_mach_run_matches_oracle():
    w = WL.double_mach(96)
    s = solver(w)
    U, V, W = dev(w.U), dev(w.V), dev(w.W)
    _steps(s, U, V, W, 30)
    p = oprob(w)
    run = lambda a, b, c: _oracle_steps(p, a, b, c, 30)[:3]
    base, worst = oracle_sensitivity(p, w, run)
    check_run(w, (U, V, W), base, worst, 'double-mach-96x24')
    s.health()


def test_oblique_shock_moves_at_the_exact_speed_on_gpu():
    w = WL.double_mach(192)
    post, pre = w.extra['split'][1]['states']
    sp = lambda x0: dict(x0=x0, slope=0.0, speed=20.0 / R3, kinds=('dirichlet', 'dirichlet'),
                         states=(post, pre))
    w.extra = dict(w.extra, split=(sp(1.0 / 6.0), sp(1.0 / 6.0 + 1.0 / R3)))
    s = solver(w)
    U, V, W = dev(w.U), dev(w.V), dev(w.W)
    t = _steps(s, U, V, W, 80)
    s.health()
    assert t < 0.1
    r = host(U)[0]
    mid = 0.5 * (post[0] + pre[0])
    worst = 0.0
    for j, y in enumerate(w.y):
        i = int(np.argmax(r[j] < mid))
        xc = w.x[i - 1] + (mid - r[j, i - 1]) * (w.x[i] - w.x[i - 1]) / (r[j, i] - r[j, i - 1])
        worst = max(worst, abs(xc - (1.0 / 6.0 + (y + 20.0 * t) / R3)) / w.dx)
    print(f't = {t:.4f}: worst shock offset {worst:.2f} cells')
    assert np.isfinite(worst) and worst <= 1.5


def test_double_mach_to_final_time():
    """Example 4.7 at 480 x 120 to t = 0.2: completes with an admissible state;
    the Mach stem and the reflected shock raise the density well above the
    post-shock 8."""
    w = WL.double_mach(480)
    s = solver(w)
    U, V, W = dev(w.U), dev(w.V), dev(w.W)
    tt = torch.zeros(1, dtype=torch.float64, device='cuda')
    for _ in range(5):
        s.step(U, V, W, tt, w.t_end, cfl=0.1)
    k = 5
    while float(tt.item()) < w.t_end and k < 20000:
        for _ in range(64):
            s.step(U, V, W, tt, w.t_end)
        k += 64
    s.health()
    assert float(tt.item()) == pytest.approx(w.t_end, abs=1e-14)
    assert float(U[0].max()) > 12.0


def test_split_refused_by_frozen_step_and_adjoint():
    from paper_2411_11229_amd import hweno
    w = WL.double_mach(64)
    s = solver(w)
    X = [dev(w.U), dev(w.V), dev(w.W)]
    dt = torch.full((1,), 1e-4, dtype=torch.float64, device='cuda')
    rec = torch.ones(6, dtype=torch.float64, device='cuda')
    with pytest.raises(hweno.HwenoError) as ei:
        s.step_frozen(X[0], X[1], X[2], dt, rec)
    assert ei.value.code == -2
    out = [torch.empty_like(x) for x in X]
    with pytest.raises(hweno.HwenoError) as ei:
        s.adjoint_step(X[0], X[1], X[2], dt, rec, [x.clone() for x in X], out)
    assert ei.value.code == -2
