"""Writes ``quadrant_runs.npz``: FP64 oracle results of more four-quadrant
Riemann runs (seeds 4001-4005, 128^2, transmissive, production dt, to
T = 0.25), the expected values of the multi-seed long-run parity tests in
tests/test_gpu_longruns.py. Seeds whose oracle run loses positivity (a
non-finite or non-physical state) are left out, so that the file holds the
first three seeds that reach T.

    python tests/golden/make_quadrant_runs.py    # about 30 minutes, 8 processes

Only ``oracle/`` computes here (plus the seeded input generators, which hold
none of the scheme's arithmetic). For each run it stores the oracle's step
count, end time, time steps and final fields, its largest per-field relative
divergence under one-ulp perturbations of every input value (relative
2^-52, random sign, generator seed 0, two trials) and the same under one
FP32 ulp (relative 2^-24, one trial).
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

OUT = os.path.join(HERE, 'quadrant_runs.npz')
SEEDS = [4001, 4002, 4003, 4004, 4005]
KEEP = 3
TRIALS = 2
N = 128


def perturbations(w):
    rng = np.random.default_rng(0)
    sets = [(w.U, w.V, w.W)]
    for rel in [2.0 ** -52] * TRIALS + [2.0 ** -24]:
        pert = lambda a: a * (1 + rng.choice([-1.0, 1.0], size=a.shape) * rel)
        sets.append((pert(w.U), pert(w.V), pert(w.W)))
    return sets


def admissible(U, g=1.4):
    rho = U[0]
    p = (g - 1.0) * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / rho)
    return bool(np.all(np.isfinite(U)) and np.all(rho > 0) and np.all(p > 0))


def one_run(job):
    seed, k = job
    w = WL.euler2d_quadrants(N, seed=seed)
    U, V, W = perturbations(w)[k]
    p = O.Problem(**w.problem_kwargs())
    try:
        with np.errstate(all='ignore'):
            Uo, Vo, Wo, log = O.run(p, U, V, W, w.t_end)
    except np.linalg.LinAlgError:    # a non-physical state: no eigenvectors
        return seed, k, None, None, None, 0, 0.0, None, False
    ok = admissible(Uo) and abs(log.t - w.t_end) <= 1e-12
    return seed, k, Uo, Vo, Wo, log.steps, log.t, np.array(log.dts), ok


def main():
    jobs = [(seed, k) for seed in SEEDS for k in range(TRIALS + 2)]
    with Pool(8) as pool:
        res = pool.map(one_run, jobs, chunksize=1)
    out = {}
    kept = []
    for seed in SEEDS:
        runs = {r[1]: r for r in res if r[0] == seed}
        if not all(runs[k][8] for k in runs) or len(kept) == KEEP:
            print(f'seed {seed}: left out (reached T with admissible states: '
                  f'{[runs[k][8] for k in sorted(runs)]})', flush=True)
            continue
        kept.append(seed)
        base = runs[0]
        fields = base[2:5]
        worst = np.zeros(3)
        for k in range(1, TRIALS + 1):
            for f in range(3):
                a, b = fields[f], runs[k][2 + f]
                worst[f] = max(worst[f], np.max(np.abs(a - b)) / np.max(np.abs(a)))
        name = f'seed{seed}'
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
    out['seeds'] = np.array(kept)
    np.savez_compressed(OUT, **out)
    print(OUT, os.path.getsize(OUT), 'bytes')


if __name__ == '__main__':
    main()
