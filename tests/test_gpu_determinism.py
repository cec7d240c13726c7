"""Determinism of the HIP path across launch configurations.

* The strip height of the 2D marcher (rows one wavefront marches; chosen by
  an occupancy model, 71 rows at 2048^2 in FP64 and 36 in FP32) does not
  change a single bit of the operator or of a step: every output cell is the
  same function of its stencil, and the only cross-block reduction (the
  Lax-Friedrichs alphas) is a max, which is order independent. With 1-row
  strips every cell is computed by the code path the whole-field oracle
  comparisons at small sizes exercise, so these tests tie the production
  launch configuration to them.
* hweno_steps (stage-1 alphas from the previous step's last stage) equals
  the same number of hweno_step calls (alphas by a separate reduction), bit
  for bit, including the clipped last step and skipped steps past t_end.
"""
import numpy as np
import pytest
import torch

from paper_2411_11229_amd import workloads as WL

pytestmark = pytest.mark.gpu


def H():
    from paper_2411_11229_amd import hweno
    return hweno


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device='cuda')


@pytest.fixture
def strip_reset():
    yield
    H().set_strip_rows(0)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_strip_height_leaves_results_bit_identical_2048(precision, strip_reset):
    """The bench workload (2048^2 four-quadrant data) in the bench's launch
    configuration against 1-row and 5-row strips: hweno_rhs outputs and one
    hweno_step (fields, stage states, dt, alphas) agree bit for bit."""
    h = H()
    w = WL.euler2d_quadrants(2048, seed=4000)
    dtype = torch.float64 if precision == 'f64' else torch.float32
    s = h.Solver(h.Problem(**w.problem_kwargs(), precision=precision))
    U0, V0, W0 = dev(w.U, dtype), dev(w.V, dtype), dev(w.W, dtype)
    alpha = s.max_wavespeed(U0)
    results = {}
    for rows in (0, 1, 5):
        print(f'{precision} strip rows {rows or "auto"}', flush=True)
        h.set_strip_rows(rows)
        rhs = s.rhs(U0, V0, W0, alpha)
        U, V, W = U0.clone(), V0.clone(), W0.clone()
        t = torch.zeros(1, dtype=torch.float64, device='cuda')
        dt = torch.zeros(1, dtype=torch.float64, device='cuda')
        rec = torch.zeros(6, dtype=torch.float64, device='cuda')
        stages = torch.empty(2 * 3 * w.U.size, dtype=dtype, device='cuda')
        s.step(U, V, W, t, w.t_end, dt_used=dt, alpha_rec=rec, stages=stages)
        # one more step from a state with non-zero derivatives
        s.step(U, V, W, t, w.t_end)
        torch.cuda.synchronize()
        results[rows] = [x.clone() for x in rhs] + [U, V, W, t, dt, rec, stages]
        s.health()
    names = ['L1', 'L2', 'L3', 'vtilde', 'wtilde', 'U', 'V', 'W', 't', 'dt', 'alpha_rec', 'stages']
    for rows in (1, 5):
        for name, a, b in zip(names, results[0], results[rows]):
            assert torch.equal(a, b), f'{precision}: {name} differs between strip heights auto and {rows}'


CASES = [
    ('euler2d-quadrants-256', lambda: WL.euler2d_quadrants(256, seed=4001), 0.004, 'production'),
    ('euler2d-smooth-130x70', lambda: WL.euler2d_smooth(130, seed=3010, ny=70), 0.01, 'production'),
    ('euler1d-riemann-2000', lambda: WL.euler1d_riemann_sine(2000, seed=2004), 0.004, 'production'),
    ('burgers1d-accuracy-64', lambda: WL.paper_burgers1d(64), 0.03, 'accuracy'),
]


@pytest.mark.parametrize("name,mk,t_end,rule", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_alpha_steps_equal_single_steps(name, mk, t_end, rule, precision):
    """hweno_steps(k) against k hweno_step calls: same fields, times, time
    steps and recorded alphas, bit for bit; k runs past t_end, so the run
    contains a clipped step and skipped ones."""
    print(f'case {name} {precision}', flush=True)
    h = H()
    w = mk()
    dtype = torch.float64 if precision == 'f64' else torch.float32
    two = w.dim == 2
    s = h.Solver(h.Problem(**w.problem_kwargs(), precision=precision))
    k = 40
    outs = []
    for multi in (False, True):
        U, V = dev(w.U, dtype), dev(w.V, dtype)
        W = dev(w.W, dtype) if two else None
        t = torch.zeros(1, dtype=torch.float64, device='cuda')
        dts = torch.zeros(k, dtype=torch.float64, device='cuda')
        rec = torch.zeros(k, 6, dtype=torch.float64, device='cuda')
        if multi:
            s.steps(U, V, W, t, k, t_end, rule, dt_used=dts, alpha_rec=rec)
        else:
            for j in range(k):
                s.step(U, V, W, t, t_end, rule, dt_used=dts[j:j + 1], alpha_rec=rec[j])
        torch.cuda.synchronize()
        outs.append((U, V, W, t, dts, rec))
    a, b = outs
    n = int((a[4] > 0).sum())
    assert 0 < n < k, f'the run should end before {k} steps (took {n})'
    assert float(a[3]) == t_end
    for name_, x, y in zip(('U', 'V', 'W', 't', 'dt_used'), a[:5], b[:5]):
        if x is None:
            continue
        assert torch.equal(x, y), f'{name_} differs between hweno_steps and hweno_step'
    # alphas of the active steps (skipped steps record only stage 1)
    assert torch.equal(a[5][:n], b[5][:n])
    s.health()


def test_graph_replay_of_multi_steps_equals_eager():
    """Solver.run with HIP graphs (a captured hweno_steps chunk, replayed)
    against eager chunks: fields, step count, time steps bit for bit."""
    h = H()
    w = WL.euler2d_quadrants(96, seed=4005, ny=80)
    s = h.Solver(h.Problem(**w.problem_kwargs()))
    res = []
    for graph in (False, True):
        U, V, W = dev(w.U, torch.float64), dev(w.V, torch.float64), dev(w.W, torch.float64)
        n, t, dts = s.run(U, V, W, t_end=0.02, graph=graph, chunk=16)
        torch.cuda.synchronize()
        res.append((n, t, dts.clone(), U, V, W))
    assert res[0][0] == res[1][0] and res[0][1] == res[1][1]
    for x, y in zip(res[0][2:], res[1][2:]):
        assert torch.equal(x, y)
