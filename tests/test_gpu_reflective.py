"""Reflective walls on the HIP path against the FP64 oracle (remarks on
boundary conditions in sections 2 and 3; Example 4.4).

* One operator evaluation and one step, FP64: max |gpu - oracle| <= 1e-12 *
  max |oracle| per field, for walls on every side and mixed with the other
  boundary types, at sizes whose last 60-column tile is ragged (nx = 61, 121:
  the next-to-last tile then holds a ghost column too) and whose rows span
  several strips. For the modified derivatives the scale also includes the
  size of the candidate derivatives they combine (max |u_{i+1} - u_i| / h and
  max |v|): next to a wall with piecewise-constant data they come out of
  order eps (1e-10) weights, about 1e-8, and the oracle's numerically
  inverted left eigenvectors (round-off where the closed form has zeros) then
  move them by about 1e-13, a rounding difference of the inputs' scale.
* Multi-step runs: within 10x the oracle's own 1-ulp divergence, as the other
  shock runs; mass and energy conserved between walls.
* Example 4.4 at N = 800 to t = 0.038: the density range over all steps
  against the paper's contour range (as the oracle's pin does), and parity
  with the oracle over the first 150 steps.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import hweno as O
from paper_2411_11229_amd import workloads as WL

from test_gpu_parity import (RTOL64, check_run, dev, f32_bounds, host, oprob, oracle_sensitivity,
                             rel_err, solver)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden', 'paper_tables.json')
R4 = ('reflective',) * 4


def cases():
    return [
        ('euler1d-smooth-61-rr', WL.random_smooth_1d(61, 'euler', seed=71, bc='reflective')),
        ('euler1d-riemann-121-rt', WL.with_bc(WL.euler1d_riemann_sine(121, seed=2012),
                                              ('reflective', 'transmissive', 'periodic', 'periodic'))),
        ('euler1d-riemann-97-tr', WL.with_bc(WL.euler1d_riemann_sine(97, seed=2013),
                                             ('transmissive', 'reflective', 'periodic', 'periodic'))),
        ('euler1d-blast-800', WL.blast_wave_1d(800)),
        ('euler1d-min-5', WL.random_smooth_1d(5, 'euler', seed=72, bc='reflective')),
        ('euler2d-smooth-130x70-rrrr', WL.with_bc(WL.euler2d_smooth(130, seed=3202, ny=70), R4)),
        ('euler2d-smooth-121x45-rttr', WL.with_bc(WL.euler2d_smooth(121, seed=3203, ny=45),
                                                  ('reflective', 'transmissive', 'transmissive',
                                                   'reflective'))),
        ('euler2d-smooth-61x66-pprr', WL.with_bc(WL.euler2d_smooth(61, seed=3204, ny=66),
                                                 ('periodic', 'periodic', 'reflective', 'reflective'))),
        ('euler2d-quadrants-96x80-rrpp', WL.with_bc(WL.euler2d_quadrants(96, seed=4202, ny=80),
                                                    ('reflective', 'reflective', 'periodic', 'periodic'))),
        ('euler2d-quadrants-64x48-rrrr', WL.with_bc(WL.euler2d_quadrants(64, seed=4203, ny=48), R4)),
        ('euler2d-min-5x5', WL.with_bc(WL.euler2d_smooth(5, seed=3205), R4)),
    ]


@pytest.mark.parametrize("name,w", cases(), ids=[c[0] for c in cases()])
def test_reflective_rhs_matches_oracle_f64(name, w):
    print(f'case {name}', flush=True)
    s = solver(w)
    p = oprob(w)
    alpha = O.max_speed(p, w.U)
    ref = O.rhs(p, w.U, w.V, w.W, alpha)
    two = w.dim == 2
    U, V = dev(w.U), dev(w.V)
    W = dev(w.W) if two else None
    al = torch.tensor(alpha, dtype=torch.float64, device='cuda')
    got = s.rhs(U, V, W, al)
    for k, (g, r) in enumerate(zip(got, ref)):
        if r is None:
            continue
        scale = np.max(np.abs(r))
        if k >= 3:   # v~ (x), w~ (y): also the scale of the candidate derivatives
            ax, h, D = (-1, w.dx, w.V) if k == 3 else (-2, w.dy, w.W)
            scale = max(scale, np.max(np.abs(np.diff(w.U, axis=ax))) / h, np.max(np.abs(D)))
        e = np.max(np.abs(host(g) - r)) / scale
        print(f'  output {k}: rel err {e:.3e}')
        assert e <= RTOL64, f'{name} output {k}: {e:.3e}'


@pytest.mark.parametrize("name,w", [cases()[1], cases()[5], cases()[9]],
                         ids=[cases()[k][0] for k in (1, 5, 9)])
def test_reflective_rhs_f32_against_f64_oracle(name, w):
    """FP32 path with walls, to the bound of the periodic FP32 parity test."""
    print(f'case {name}', flush=True)
    two = w.dim == 2
    w.U = w.U.astype(np.float32).astype(np.float64)
    w.V = w.V.astype(np.float32).astype(np.float64)
    w.W = w.W.astype(np.float32).astype(np.float64) if two else None
    s = solver(w, precision='f32')
    p = oprob(w)
    alpha = O.max_speed(p, w.U)
    f32 = lambda a: dev(a, torch.float32)
    got = s.rhs(f32(w.U), f32(w.V), f32(w.W) if two else None, dev(np.array(alpha)))
    ref = O.rhs(p, w.U, w.V, w.W, alpha)
    tol = f32_bounds(w, alpha)
    for k, (g, r) in enumerate(zip(got, ref)):
        if r is None:
            continue
        err = np.max(np.abs(host(g) - r))
        print(f'  output {k}: abs err {err:.3e}  bound {tol[k]:.3e}')
        assert err <= tol[k], f'output {k}: abs err {err:.3e} > bound {tol[k]:.3e}'


@pytest.mark.parametrize("name,w", cases()[:4] + cases()[5:], ids=[c[0] for c in cases()[:4] + cases()[5:]])
def test_reflective_step_matches_oracle_f64(name, w):
    print(f'case {name}', flush=True)
    s = solver(w)
    p = oprob(w)
    two = w.dim == 2
    U, V = dev(w.U), dev(w.V)
    W = dev(w.W) if two else None
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    dt = torch.zeros(1, dtype=torch.float64, device='cuda')
    cfl = 0.1 if 'blast' in name else 0.6
    s.step(U, V, W, t, 1e9, cfl=cfl, dt_used=dt)
    alpha = O.max_speed(p, w.U)
    dto = O.time_step(p, alpha, 'production', cfl)
    assert float(dt.item()) == pytest.approx(dto, rel=1e-14, abs=0)
    Uo, Vo, Wo, _ = O.step(p, w.U, w.V, w.W, dto, (alpha, None, None))
    for k, (g, r) in enumerate(zip((U, V, W), (Uo, Vo, Wo))):
        if r is None:
            continue
        e = rel_err(host(g), r)
        print(f'  field {k}: rel err {e:.3e}')
        assert e <= RTOL64, f'{name} field {k}: {e:.3e}'


def test_reflective_2d_run_matches_oracle_and_conserves():
    """20 production steps of seeded quadrant data in a box of four walls."""
    w = WL.with_bc(WL.euler2d_quadrants(64, seed=4204, ny=48), R4)
    s = solver(w)
    U, V, W = dev(w.U), dev(w.V), dev(w.W)
    m0 = U.sum(dim=(1, 2))
    steps, t, dts = s.run(U, V, W, t_end=1e9, max_steps=20)
    p = oprob(w)
    Uo, Vo, Wo, log = O.run(p, w.U, w.V, w.W, 1e9, max_steps=20)
    np.testing.assert_allclose(host(dts), np.array(log.dts), rtol=1e-12)
    run = lambda a, b, c: O.run(p, a, b, c, 1e9, max_steps=20)[:3]
    base, worst = oracle_sensitivity(p, w, run, base=(Uo, Vo, Wo))
    check_run(w, (U, V, W), base, worst, 'euler2d-quadrants-walls')
    m1 = U.sum(dim=(1, 2))
    scale = U.abs().sum(dim=(1, 2))
    for c in (0, 3):
        assert abs(float(m1[c] - m0[c])) <= 1e-13 * float(scale[c])
    s.health()


def _blast_steps(s, U, V, t_end, n_steps=None):
    """Example 4.4's stepping: first step at CFL 0.1, the rest at 0.6; the
    density range over all step states is kept on the device."""
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    lo = torch.ones(1, dtype=torch.float64, device='cuda')
    hi = torch.ones(1, dtype=torch.float64, device='cuda')
    k = 0
    while (n_steps is None or k < n_steps):
        for _ in range(64):
            s.step(U, V, None, t, t_end, cfl=0.1 if k == 0 else 0.6)
            lo = torch.minimum(lo, U[0].min())
            hi = torch.maximum(hi, U[0].max())
            k += 1
            if n_steps is not None and k >= n_steps:
                break
        if float(t.item()) >= t_end:
            break
    return float(t.item()), float(lo.item()), float(hi.item())


def test_blast_wave_first_steps_match_oracle():
    w = WL.blast_wave_1d(800)
    s = solver(w)
    U, V = dev(w.U), dev(w.V)
    _blast_steps(s, U, V, w.t_end, n_steps=150)
    p = oprob(w)

    def run(a, b, c):
        for k in range(150):
            al = O.max_speed(p, a)
            dt = O.time_step(p, al, 'production', 0.1 if k == 0 else 0.6)
            a, b, _, _ = O.step(p, a, b, None, dt, (al, None, None))
        return a, b
    base, worst = oracle_sensitivity(p, w, run)
    check_run(w, (U, V), base, worst, 'blast-150')


def test_blast_wave_density_range_matches_paper_on_gpu():
    ref = json.load(open(GOLDEN))['blast_wave_density_range']
    w = WL.blast_wave_1d(800)
    s = solver(w)
    U, V = dev(w.U), dev(w.V)
    t, lo, hi = _blast_steps(s, U, V, w.t_end)
    print(f't = {t}: rho in [{lo:.5f}, {hi:.5f}]')
    assert t == pytest.approx(w.t_end, abs=1e-15)
    assert abs(lo - ref['min']) <= 5e-4
    assert abs(hi - ref['max']) <= 2e-3 * ref['max']
    assert abs(float(U[0].sum()) * w.dx - 1.0) <= 1e-12
    s.health()


def test_reflective_rejected_for_scalar_laws():
    from paper_2411_11229_amd import hweno
    w = WL.random_smooth_1d(12, 'burgers', seed=3, bc='reflective')
    with pytest.raises(hweno.HwenoError):
        solver(w)


def _blast_final_gpu(gamma0, d0, n=800):
    w = WL.blast_wave_1d(n)
    s = solver(w, gamma0=gamma0, d0=d0)
    U, V = dev(w.U), dev(w.V)
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    k = 0
    while True:
        for _ in range(64):
            s.step(U, V, None, t, w.t_end, cfl=0.1 if k == 0 else 0.6)
            k += 1
        if float(t.item()) >= w.t_end:
            break
    s.health()
    return w.x, host(U)


G0_SWEEP = (0.95, 0.7, 0.5, 1.0 / 3.0, 0.1)
D0_SWEEP = (0.95, 0.9, 0.7, 0.5, 1.0 / 3.0, 0.1)


def test_blast_wave_linear_weight_sweeps_on_gpu():
    """The paper's sweeps of Example 4.4 at N = 800: gamma0 over
    (0.95, 0.7, 0.5, 1/3, 0.1) with d0 = 0.9 lowers the density peak in
    (0.7, 0.8) step by step; d0 over (0.95, ..., 0.1) with gamma0 = 0.95 raises
    the total variation of the density step by step."""
    peak = []
    for g0 in G0_SWEEP:
        x, U = _blast_final_gpu(g0, 0.9)
        peak.append(U[0][(x > 0.7) & (x < 0.8)].max())
    tv = []
    for d0 in D0_SWEEP:
        x, U = _blast_final_gpu(0.95, d0)
        tv.append(np.abs(np.diff(U[0])).sum())
    print('peaks', peak, 'TV', tv)
    assert all(a > b for a, b in zip(peak, peak[1:])), peak
    assert all(a < b for a, b in zip(tv, tv[1:])), tv


@pytest.mark.parametrize("g0,d0", [(1.0 / 3.0, 0.9), (0.95, 0.1)])
def test_blast_wave_sweep_settings_match_oracle(g0, d0):
    """Parity with the oracle over the first 120 steps at swept weights."""
    w = WL.blast_wave_1d(800)
    s = solver(w, gamma0=g0, d0=d0)
    U, V = dev(w.U), dev(w.V)
    _blast_steps(s, U, V, w.t_end, n_steps=120)
    p = oprob(w, gamma0=g0, d0=d0)

    def run(a, b, c):
        for k in range(120):
            al = O.max_speed(p, a)
            dt = O.time_step(p, al, 'production', 0.1 if k == 0 else 0.6)
            a, b, _, _ = O.step(p, a, b, None, dt, (al, None, None))
        return a, b
    base, worst = oracle_sensitivity(p, w, run)
    check_run(w, (U, V), base, worst, f'blast-g0={g0:.3f}-d0={d0:.3f}')
