"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances.
* FP64, one operator evaluation or one step: max |gpu - oracle| <= 1e-12 *
  max |oracle| per field (the two differ only in rounding order: FMA
  contraction, re-associated weight formulas, closed-form vs numerical L).
* FP64, multi-step runs: the nonlinear weights amplify round-off, so the
  bound is 10x the oracle's own divergence when its initial data are
  perturbed by one ulp (measured in the test, per field).
* FP32: absolute bound derived from the arithmetic: interface fluxes are
  evaluated in float (error <= c eps32 S with S the magnitude of the summed
  terms, c = 16 roundings), the flux difference in double, so
  |dL| <= 2 c eps32 S / h per direction; v~ errs by <= c eps32 (|V| + |U|/h).
Sizes span several 60-column tiles and 32-row strips with ragged tails.
"""
import math

import numpy as np
import pytest
import torch

from oracle import hweno as O
from paper_2411_11229_amd import workloads as WL

pytestmark = pytest.mark.gpu

RTOL64 = 1e-12


def H():
    from paper_2411_11229_amd import hweno
    return hweno


def solver(w, precision='f64', **kw):
    h = H()
    return h.Solver(h.Problem(**w.problem_kwargs(), precision=precision, **kw))


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device='cuda')


def host(t):
    return t.detach().double().cpu().numpy()


def rel_err(got, ref):
    scale = max(np.max(np.abs(ref)), 1e-300)
    return np.max(np.abs(got - ref)) / scale


def oprob(w, **kw):
    return O.Problem(**w.problem_kwargs(), **kw)


def rhs_cases():
    cs = [
        ('adv1d-periodic-150', WL.random_smooth_1d(150, 'advection', seed=21)),
        ('burgers1d-periodic-61', WL.random_smooth_1d(61, 'burgers', seed=22)),
        ('burgers1d-transmissive-121', WL.random_smooth_1d(121, 'burgers', seed=23, bc='transmissive')),
        ('burgers1d-min-5', WL.random_smooth_1d(5, 'burgers', seed=24)),
        ('euler1d-smooth-200', WL.random_smooth_1d(200, 'euler', seed=25)),
        ('euler1d-riemann-2000', WL.euler1d_riemann_sine(2000, seed=2000)),
        ('euler1d-riemann-97', WL.euler1d_riemann_sine(97, seed=2001)),
        ('burgers2d-64', WL.paper_burgers2d(64)),
        ('euler2d-smooth-130x70', WL.euler2d_smooth(130, seed=3002, ny=70)),
        ('euler2d-quadrants-96x80', WL.euler2d_quadrants(96, seed=4002, ny=80)),
        ('euler2d-paper-40', WL.paper_euler2d(40)),
        ('euler2d-min-5x5', WL.euler2d_smooth(5, seed=3003)),
    ]
    w = WL.paper_burgers2d(45)
    w.system, w.adv_a, w.adv_b = 'advection', 0.8, -1.7
    w.W = w.W * 0.3 + 0.2
    cs.append(('adv2d-45', w))
    return cs


@pytest.mark.parametrize("name,w", rhs_cases(), ids=[c[0] for c in rhs_cases()])
def test_rhs_matches_oracle_f64(name, w):
    print(f'case {name}', flush=True)
    s = solver(w)
    two = w.dim == 2
    U, V = dev(w.U), dev(w.V)
    W = dev(w.W) if two else None
    p = oprob(w)
    alpha = O.max_speed(p, w.U)
    a_dev = s.max_wavespeed(U)
    np.testing.assert_allclose(host(a_dev)[:w.dim], alpha[:w.dim], rtol=1e-14)
    got = s.rhs(U, V, W, dev(np.array(alpha)))
    ref = O.rhs(p, w.U, w.V, w.W, alpha)
    for k, (g, r) in enumerate(zip(got, ref)):
        if r is None:
            assert g is None
            continue
        e = rel_err(host(g), r)
        assert e <= RTOL64, f'output {k}: rel err {e:.3e}'


def f32_bounds(w, alpha):
    """Absolute error bounds of the FP32 operator, per output (see module
    docstring). Scales come from the oracle's pointwise fluxes; for systems,
    values that pass through the characteristic projection (u at the faces,
    v~) carry the condition number kappa = max |R| |L| (infinity norms) of
    the eigenvector matrices."""
    eps, c = 2.0 ** -24, 16.0
    p = oprob(w)
    sy = O.make_system(p)
    mx = lambda a: float(np.max(np.abs(a)))
    two = w.dim == 2
    tol = [0.0, 0.0, 0.0, 0.0, 0.0]
    lines = [(0, w.dx, w.V, w.W, 1, 2, 3)]
    if two:
        lines.append((1, w.dy, w.W, w.V, 2, 1, 4))
    for d, h, A, B, ia, ib, it in lines:
        kappa = 1.0
        eig = sy.eig(w.U, d)
        if eig is not None:
            L, R = eig
            kappa = float(np.max(np.abs(R).sum(axis=-1).max(axis=-1) * np.abs(L).sum(axis=-1).max(axis=-1)))
        f = sy.flux(w.U, d)
        ha = sy.jac_apply(w.U, A, d)
        SF = kappa * (mx(f) + alpha[d] * mx(w.U))
        SH = kappa * (mx(ha) + alpha[d] * mx(A)) + mx(f) / h
        tol[0] += 2 * c * eps * SF / h
        tol[ia] += 2 * c * eps * SH / h
        if two:
            tol[ib] += 2 * c * eps * mx(sy.jac_apply(w.U, B, d)) / h
        tol[it] = c * eps * kappa * (mx(A) + mx(w.U) / h)
    return tol


@pytest.mark.parametrize("name,w", rhs_cases()[:12:2], ids=[c[0] for c in rhs_cases()[:12:2]])
def test_rhs_f32_against_f64_oracle(name, w):
    """FP32 storage and arithmetic (FP64 smoothness indicators, weights and
    flux differences) against the FP64 oracle on float32-rounded inputs."""
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
        print(f'  output {k}: abs err {err:.3e}  bound {tol[k]:.3e}  rel {err / np.max(np.abs(r)):.2e}')
        assert err <= tol[k], f'output {k}: abs err {err:.3e} > bound {tol[k]:.3e}'


STEP_CASES = [
    ('burgers1d-121', lambda: WL.random_smooth_1d(121, 'burgers', seed=31), 'production'),
    ('euler1d-riemann-300', lambda: WL.euler1d_riemann_sine(300, seed=2002), 'production'),
    ('adv1d-80-accuracy', lambda: WL.advection1d_modes(80), 'accuracy'),
    ('euler2d-smooth-70x66', lambda: WL.euler2d_smooth(70, seed=3004, ny=66), 'production'),
    ('euler2d-quadrants-64', lambda: WL.euler2d_quadrants(64, seed=4003), 'production'),
    ('burgers2d-50-accuracy', lambda: WL.paper_burgers2d(50), 'accuracy'),
]


@pytest.mark.parametrize("name,mk,rule", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_step_matches_oracle_f64(name, mk, rule):
    print(f'case {name}', flush=True)
    w = mk()
    s = solver(w)
    two = w.dim == 2
    U, V = dev(w.U), dev(w.V)
    W = dev(w.W) if two else None
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    dt_used = torch.zeros(1, dtype=torch.float64, device='cuda')
    rec = torch.zeros(6, dtype=torch.float64, device='cuda')
    nf = 3 if two else 2
    stages = torch.empty(2 * nf * w.U.size, dtype=torch.float64, device='cuda')
    s.step(U, V, W, t, 10.0, rule, 0.6, dt_used=dt_used, alpha_rec=rec, stages=stages)
    p = oprob(w)
    a1 = O.max_speed(p, w.U)
    dt = O.time_step(p, a1, rule, 0.6)
    U3, V3, W3, als = O.step(p, w.U, w.V, w.W, dt)
    assert host(dt_used)[0] == pytest.approx(dt, rel=1e-14, abs=0)
    assert host(t)[0] == pytest.approx(dt, rel=1e-14, abs=0)
    r = host(rec).reshape(3, 2)
    for k in range(3):
        np.testing.assert_allclose(r[k, :w.dim], np.array(als[k])[:w.dim], rtol=1e-12)
    for g, ref in ((U, U3), (V, V3)) + (((W, W3),) if two else ()):
        e = rel_err(host(g), ref)
        assert e <= RTOL64, f'rel err {e:.3e}'
    # the saved stage-1 state equals the oracle's first stage
    L1, L2, L3, vt, wt = O.rhs(p, w.U, w.V, w.W, a1)
    n = w.U.size
    X1 = host(stages)
    assert rel_err(X1[:n].reshape(w.U.shape), w.U + dt * L1) <= RTOL64
    assert rel_err(X1[n:2 * n].reshape(w.U.shape), vt + dt * L2) <= RTOL64


def test_step_skipped_at_end_time():
    w = WL.random_smooth_1d(64, 'burgers', seed=41)
    s = solver(w)
    U, V = dev(w.U), dev(w.V)
    U0, V0 = U.clone(), V.clone()
    t = torch.full((1,), 0.5, dtype=torch.float64, device='cuda')
    dt_used = torch.full((1,), -1.0, dtype=torch.float64, device='cuda')
    s.step(U, V, None, t, 0.5, dt_used=dt_used)
    torch.cuda.synchronize()
    assert torch.equal(U, U0) and torch.equal(V, V0)
    assert float(dt_used.item()) == 0.0 and float(t.item()) == 0.5


def test_last_step_clipped_to_end_time():
    w = WL.random_smooth_1d(64, 'burgers', seed=42)
    s = solver(w)
    U, V = dev(w.U), dev(w.V)
    t = torch.full((1,), 0.3, dtype=torch.float64, device='cuda')
    dt_used = torch.zeros(1, dtype=torch.float64, device='cuda')
    s.step(U, V, None, t, 0.3 + 1e-5, dt_used=dt_used)
    assert float(t.item()) == 0.3 + 1e-5
    assert float(dt_used.item()) == pytest.approx(1e-5, rel=1e-9, abs=0)


def test_table1_burgers_run_reproduces_paper_on_gpu():
    """Full run of Example 4.1 (N = 80, t = 0.5, accuracy time step) on the
    GPU: same steps as the oracle, state within 1e-12, and the printed Table 1
    L-infinity error 1.255e-5."""
    w = WL.paper_burgers1d(80)
    s = solver(w)
    U, V = dev(w.U), dev(w.V)
    steps, t, dts = s.run(U, V, None, w.t_end, rule='accuracy')
    p = oprob(w)
    Uo, Vo, _, log = O.run(p, w.U, w.V, None, w.t_end, rule='accuracy')
    assert steps == log.steps and t == pytest.approx(0.5, abs=1e-15)
    np.testing.assert_allclose(host(dts), np.array(log.dts), rtol=1e-12)
    assert rel_err(host(U), Uo) <= 1e-12 and rel_err(host(V), Vo) <= 1e-11
    ex = w.x.copy()
    u = 0.5 + np.sin(ex)
    for _ in range(60):
        u = u - (u - 0.5 - np.sin(ex - u * 0.5)) / (1.0 + np.cos(ex - u * 0.5) * 0.5)
    assert np.max(np.abs(host(U)[0] - u)) == pytest.approx(1.255e-5, rel=2e-3, abs=0)


def test_periodic_conservation_on_gpu():
    """sum(u) of every component is invariant over steps (periodic, FP64)."""
    w = WL.euler2d_smooth(128, seed=3005, ny=96)
    s = solver(w)
    U, V, W = dev(w.U), dev(w.V), dev(w.W)
    s0 = U.sum(dim=(1, 2))
    s.run(U, V, W, t_end=1e9, max_steps=10)
    s1 = U.sum(dim=(1, 2))
    scale = U.abs().sum(dim=(1, 2))
    assert torch.all((s1 - s0).abs() <= 1e-13 * scale), (s0, s1)


def oracle_sensitivity(p, w, run, trials=2, seed=0, base=None):
    """Per-field max divergence of the oracle from itself when every input
    value is perturbed by one ulp (relative 2^-52, random sign)."""
    rng = np.random.default_rng(seed)
    base = run(w.U, w.V, w.W) if base is None else base
    worst = [0.0] * len(base)
    for _ in range(trials):
        pert = lambda a: None if a is None else a * (1 + rng.choice([-1.0, 1.0], size=a.shape) * 2.0 ** -52)
        other = run(pert(w.U), pert(w.V), pert(w.W))
        for k, (a, b) in enumerate(zip(base, other)):
            worst[k] = max(worst[k], rel_err(b, a))
    return base, worst


def check_run(w, gpu_fields, base, worst, label):
    for k, (g, r) in enumerate(zip(gpu_fields, base)):
        e = rel_err(host(g), r)
        bound = max(10.0 * worst[k], 1e-12)
        print(f'  {label} field {k}: rel err {e:.3e}  oracle 1-ulp divergence {worst[k]:.3e}')
        assert e <= bound, f'{label} field {k}: rel err {e:.3e} > {bound:.3e}'


def test_euler2d_smooth_run_matches_oracle():
    """20 production steps of the smooth-Fourier generator at 96x72 (periodic)."""
    w = WL.euler2d_smooth(96, seed=3006, ny=72)
    s = solver(w)
    U, V, W = dev(w.U), dev(w.V), dev(w.W)
    steps, t, dts = s.run(U, V, W, t_end=1e9, max_steps=20)
    p = oprob(w)
    Uo, Vo, Wo, log = O.run(p, w.U, w.V, w.W, 1e9, max_steps=20)
    np.testing.assert_allclose(host(dts), np.array(log.dts), rtol=1e-12)
    run = lambda a, b, c: O.run(p, a, b, c, 1e9, max_steps=20)[:3]
    base, worst = oracle_sensitivity(p, w, run, base=(Uo, Vo, Wo))
    check_run(w, (U, V, W), base, worst, 'euler2d-smooth')


@pytest.mark.parametrize("seed", [2000, 2003])
def test_euler1d_riemann_full_run(seed):
    """Seeded 1D Euler Riemann + sine data, N = 2000, transmissive, to its end
    time T (production dt): same number of steps and final time, fields
    within 10x the oracle's 1-ulp divergence."""
    w = WL.euler1d_riemann_sine(2000, seed=seed)
    print(f'seed {seed} T={w.t_end:.4f}', flush=True)
    s = solver(w)
    U, V = dev(w.U), dev(w.V)
    steps, t, dts = s.run(U, V, None, w.t_end)
    p = oprob(w)
    run = lambda a, b, c: O.run(p, a, b, None, w.t_end)[:2]
    Uo, Vo, _, log = O.run(p, w.U, w.V, None, w.t_end)
    assert steps == log.steps and t == pytest.approx(w.t_end, abs=1e-14)
    base, worst = oracle_sensitivity(p, w, run, base=(Uo, Vo))
    check_run(w, (U, V), base, worst, f'euler1d-riemann-{seed}')
    s.health()


def _mapidx(i, n, lo, hi):
    """Ghost index map of the boundary conditions (periodic wrap, transmissive clamp)."""
    if 0 <= i < n:
        return i
    side = lo if i < 0 else hi
    return i % n if side == 'periodic' else min(max(i, 0), n - 1)


def oracle_rhs_at(w, p, alpha, cells):
    """Oracle operator at isolated cells of a 2D grid: one 5-cell x-line and
    one 5-cell y-line per cell (ghosts by the problem's index map) through
    the oracle's own sweep; the centre cell of each line depends on nothing
    else."""
    sy = O.make_system(p)
    g, dl, eps = p.linear_gamma, p.linear_d, p.eps
    out = []
    for (j, i) in cells:
        cols = [_mapidx(i + k, w.nx, p.bc[0], p.bc[1]) for k in range(-2, 3)]
        rows = [_mapidx(j + k, w.ny, p.bc[2], p.bc[3]) for k in range(-2, 3)]
        xl = lambda F: F[:, j, :][:, cols]
        yl = lambda F: F[:, :, i][:, rows]
        RUx, RVx, RWx, vt = O.sweep(sy, 0, xl(w.U), xl(w.V), xl(w.W), p.dx, alpha[0],
                                    'transmissive', 'transmissive', g, dl, eps)
        RUy, RWy, RVy, wt = O.sweep(sy, 1, yl(w.U), yl(w.W), yl(w.V), p.dy, alpha[1],
                                    'transmissive', 'transmissive', g, dl, eps)
        out.append((RUx[:, 2] + RUy[:, 2], RVx[:, 2] + RVy[:, 2], RWx[:, 2] + RWy[:, 2],
                    vt[:, 2], wt[:, 2]))
    return out


def sample_cells(nx, ny, k=48, seed=7):
    rng = np.random.default_rng(seed)
    cells = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1), (1, nx // 2), (ny // 2, 1),
             (ny // 2, nx // 2), (ny // 2 - 1, nx // 2 - 1)]
    cells += [tuple(x) for x in zip(rng.integers(0, ny, k), rng.integers(0, nx, k))]
    return cells


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_full_size_quadrants_2048_sampled(precision):
    """The benchmark workload at full size (2048^2 four-quadrant Riemann,
    transmissive) in the benchmark's launch configuration: the operator and
    the first stage of a step at sampled cells (corners, edges, the quadrant
    junction, random cells) against the oracle evaluated one cell at a time;
    alphas from the oracle over the whole grid."""
    w = WL.euler2d_quadrants(2048, seed=4000)
    if precision == 'f32':
        w.U = w.U.astype(np.float32).astype(np.float64)
    p = oprob(w)
    alpha = O.max_speed(p, w.U)
    s = solver(w, precision=precision)
    dt_ = torch.float64 if precision == 'f64' else torch.float32
    U, V, W = dev(w.U, dt_), dev(w.V, dt_), dev(w.W, dt_)
    got = [host(x) for x in s.rhs(U, V, W, dev(np.array(alpha)))]
    cells = sample_cells(w.nx, w.ny)
    ref = oracle_rhs_at(w, p, alpha, cells)
    tol = f32_bounds(w, alpha) if precision == 'f32' else None
    scale = [max(np.max(np.abs(r[k])) for r in ref) for k in range(5)]
    for (j, i), r in zip(cells, ref):
        for k in range(5):
            e = np.max(np.abs(got[k][:, j, i] - r[k]))
            lim = RTOL64 * max(scale[k], 1.0) if precision == 'f64' else tol[k]
            assert e <= lim, f'cell {(j, i)} output {k}: err {e:.3e} > {lim:.3e}'
    # first stage of a step: X1 = (U + dt L1, v~ + dt L2, w~ + dt L3)
    nf = 3
    stages = torch.empty(2 * nf * w.U.size, dtype=dt_, device='cuda')
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    dt_used = torch.zeros(1, dtype=torch.float64, device='cuda')
    s.step(U, V, W, t, w.t_end, dt_used=dt_used, stages=stages)
    dt = O.time_step(p, alpha, 'production', 0.6)
    assert host(dt_used)[0] == pytest.approx(dt, rel=1e-12, abs=0)
    X1 = host(stages)[:3 * w.U.size].reshape((3,) + w.U.shape)
    for (j, i), r in zip(cells, ref):
        exp = (w.U[:, j, i] + dt * r[0], r[3] + dt * r[1], r[4] + dt * r[2])
        for k in range(3):
            e = np.max(np.abs(X1[k][:, j, i] - exp[k]))
            base_tol = (0.0, tol[3], tol[4])[k] if precision == 'f32' else 0.0
            lim = (RTOL64 * max(np.max(np.abs(exp[k])), 1.0) if precision == 'f64'
                   else base_tol + dt * tol[k] + 4 * 2.0 ** -24 * np.max(np.abs(exp[k])))
            assert e <= lim, f'stage 1 cell {(j, i)} field {k}: err {e:.3e} > {lim:.3e}'
    s.health()


def test_health_flags_nonphysical_state():
    w = WL.euler2d_quadrants(32, seed=4004)
    U = w.U.copy()
    U[3, 5, 7] = -1.0    # negative energy -> negative pressure
    s = solver(w)
    s.max_wavespeed(dev(U))
    with pytest.raises(H().HwenoError) as ei:
        s.health(clear=True)
    assert ei.value.code == -5
    s.max_wavespeed(dev(w.U))
    s.health()


def test_rhs_rejects_mismatched_tensors():
    w = WL.euler2d_smooth(20, seed=3007)
    s = solver(w)
    with pytest.raises(ValueError):
        s.rhs(dev(w.U).float(), dev(w.V), dev(w.W))
    with pytest.raises(ValueError):
        s.rhs(dev(w.U)[:, :10], dev(w.V), dev(w.W))
    with pytest.raises(ValueError):
        s.rhs(dev(w.U).transpose(1, 2), dev(w.V), dev(w.W))
