"""Writes ``long_runs.npz``: FP64 oracle results of two long 2D Euler runs,
the expected values of the long-run parity tests (tests/test_gpu_longruns.py).

    python tests/golden/make_long_runs.py        # about 10 minutes, 8 processes

Only ``oracle/`` computes here (plus the seeded input generators, which hold
none of the scheme's arithmetic). For each run it stores the oracle's step
count, end time, time steps and final fields, and the oracle's own
sensitivity: the largest per-field relative divergence (max |a - b| / max |a|)
of runs whose every input value was perturbed by one ulp (relative 2^-52,
random sign, generator seed 0, two trials), the scale of the tests'
10x-one-ulp bound for runs whose nonlinear weights amplify round-off; and the
same divergence under a perturbation of one FP32 ulp (relative 2^-24, one
trial), the scale of the FP32 run's error.

Runs:
  quadrants_128   four-quadrant Riemann data (seed 4000) at 128^2,
                  transmissive, production dt (CFL 0.6) to T = 0.25;
  smooth_256      the smooth periodic Fourier-mode data (seed 3000) at
                  256^2, 100 production steps.
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import hweno as O                    # noqa: E402
from paper_2411_11229_amd import workloads as WL  # noqa: E402

OUT = os.path.join(HERE, 'long_runs.npz')
TRIALS = 2


def cases():
    return {
        'quadrants_128': (lambda: WL.euler2d_quadrants(128, seed=4000), 0.25, None),
        'smooth_256': (lambda: WL.euler2d_smooth(256, seed=3000), 1e9, 100),
    }


def perturbations(w):
    """Input sets: the data itself, TRIALS one-ulp perturbations, then one
    FP32-ulp perturbation."""
    rng = np.random.default_rng(0)
    sets = [(w.U, w.V, w.W)]
    for rel in [2.0 ** -52] * TRIALS + [2.0 ** -24]:
        pert = lambda a: a * (1 + rng.choice([-1.0, 1.0], size=a.shape) * rel)
        sets.append((pert(w.U), pert(w.V), pert(w.W)))
    return sets


def one_run(job):
    name, k = job
    mk, t_end, max_steps = cases()[name]
    w = mk()
    U, V, W = perturbations(w)[k]
    p = O.Problem(**w.problem_kwargs())
    Uo, Vo, Wo, log = O.run(p, U, V, W, t_end, max_steps=max_steps)
    return name, k, Uo, Vo, Wo, log.steps, log.t, np.array(log.dts)


def main():
    jobs = [(name, k) for name in cases() for k in range(TRIALS + 2)]
    with Pool(len(jobs)) as pool:
        res = pool.map(one_run, jobs)
    out = {}
    for name in cases():
        runs = {k: r for r in res if r[0] == name for k in [r[1]]}
        base = runs[0]
        fields = base[2:5]
        worst = np.zeros(3)
        for k in range(1, TRIALS + 1):
            for f in range(3):
                a, b = fields[f], runs[k][2 + f]
                worst[f] = max(worst[f], np.max(np.abs(a - b)) / np.max(np.abs(a)))
        out[f'{name}_U'], out[f'{name}_V'], out[f'{name}_W'] = fields
        out[f'{name}_steps'] = np.array(base[5])
        out[f'{name}_t'] = np.array(base[6])
        out[f'{name}_dts'] = base[7]
        out[f'{name}_ulp_divergence'] = worst
        f32 = runs[TRIALS + 1][2:5]
        out[f'{name}_f32ulp_divergence'] = np.array(
            [np.max(np.abs(fields[f] - f32[f])) / np.max(np.abs(fields[f])) for f in range(3)])
        print(f'{name}: {base[5]} steps to t = {base[6]:.6f}; one-ulp divergence '
              f'U {worst[0]:.3e} V {worst[1]:.3e} W {worst[2]:.3e}; FP32-ulp divergence '
              f'{out[f"{name}_f32ulp_divergence"]}', flush=True)
    np.savez_compressed(OUT, **out)
    print(OUT, os.path.getsize(OUT), 'bytes')


if __name__ == '__main__':
    main()
