"""Writes ``euler1d_runs.npz``: FP64 oracle results of the eight seeded 1D
Euler Riemann + sine runs (N = 2000, transmissive, production dt, each to
its own end time T), the expected values of the full-run parity tests in
tests/test_gpu_longruns.py.

    python tests/golden/make_euler1d_runs.py     # about 10 minutes, 8 processes

Only ``oracle/`` computes here (plus the seeded input generators, which hold
none of the scheme's arithmetic). For each seed it stores the oracle's step
count, end time, time steps and final fields (u, v), and the oracle's own
sensitivity: the largest per-field relative divergence (max |a - b| / max |a|)
of runs whose every input value was perturbed by one ulp (relative 2^-52,
random sign, generator seed 0, two trials), the scale of the tests'
10x-one-ulp bound; and the same divergence under a perturbation of one FP32
ulp (relative 2^-24, one trial), the scale of the FP32 run's error.
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

OUT = os.path.join(HERE, 'euler1d_runs.npz')
SEEDS = list(range(2000, 2008))
TRIALS = 2


def perturbations(w):
    """Input sets: the data itself, TRIALS one-ulp perturbations, then one
    FP32-ulp perturbation."""
    rng = np.random.default_rng(0)
    sets = [(w.U, w.V)]
    for rel in [2.0 ** -52] * TRIALS + [2.0 ** -24]:
        pert = lambda a: a * (1 + rng.choice([-1.0, 1.0], size=a.shape) * rel)
        sets.append((pert(w.U), pert(w.V)))
    return sets


def one_run(job):
    seed, k = job
    w = WL.euler1d_riemann_sine(2000, seed=seed)
    U, V = perturbations(w)[k]
    p = O.Problem(**w.problem_kwargs())
    Uo, Vo, _, log = O.run(p, U, V, None, w.t_end)
    return seed, k, Uo, Vo, log.steps, log.t, np.array(log.dts)


def main():
    jobs = [(seed, k) for seed in SEEDS for k in range(TRIALS + 2)]
    # longest runs first, so that the pool ends together
    jobs.sort(key=lambda j: -WL.euler1d_riemann_sine(2000, seed=j[0]).t_end)
    with Pool(8) as pool:
        res = pool.map(one_run, jobs, chunksize=1)
    out = {}
    for seed in SEEDS:
        runs = {r[1]: r for r in res if r[0] == seed}
        base = runs[0]
        fields = base[2:4]
        worst = np.zeros(2)
        for k in range(1, TRIALS + 1):
            for f in range(2):
                a, b = fields[f], runs[k][2 + f]
                worst[f] = max(worst[f], np.max(np.abs(a - b)) / np.max(np.abs(a)))
        name = f'seed{seed}'
        out[f'{name}_U'], out[f'{name}_V'] = fields
        out[f'{name}_steps'] = np.array(base[4])
        out[f'{name}_t'] = np.array(base[5])
        out[f'{name}_dts'] = base[6]
        out[f'{name}_ulp_divergence'] = worst
        f32 = runs[TRIALS + 1][2:4]
        out[f'{name}_f32ulp_divergence'] = np.array(
            [np.max(np.abs(fields[f] - f32[f])) / np.max(np.abs(fields[f])) for f in range(2)])
        print(f'{name}: {base[4]} steps to t = {base[5]:.6f}; one-ulp divergence '
              f'U {worst[0]:.3e} V {worst[1]:.3e}; FP32-ulp divergence '
              f'{out[f"{name}_f32ulp_divergence"]}', flush=True)
    np.savez_compressed(OUT, **out)
    print(OUT, os.path.getsize(OUT), 'bytes')


if __name__ == '__main__':
    main()
