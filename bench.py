#!/usr/bin/env python3
"""Benchmark of the HWENO-I hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): 2D Euler,
2048 x 2048 cells on [0,1]^2, seeded four-quadrant Riemann data, transmissive
boundaries, production time step (CFL 0.6) from the fused max-wave-speed
reduction every step. A "step" is one full SSP-RK3 step: wave-speed
reduction and time step (fused into the stage kernels: stage 1 takes dt from
its alphas, stage 3 reduces the next step's alphas), three fused stage
kernels; the timed steps are one hweno_steps call. Inputs are resident in
HBM before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

The default warm-up (30 steps) takes the GPU past its ramp: the first ten
steps of a fresh process run about 15% slower than the steady state, which
is reached after about twenty.

Prints ONE JSON line. ``value`` = cell-stage updates per second (cells x 3 x
steps / wall time) in FP64. The FP32 form of the same workload is reported in
``fp32``. ``roofline`` covers the dominant kernel (the fused 2D Euler stage
kernel), timed with HIP events recorded around each stage launch inside the
timed region. ``cpu_baseline`` times the FP64 CPU oracle on a bounded sample
on this host.
"""
import argparse
import ctypes
import hashlib
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
VALUES_PER_CELL_STEP = 104      # 2D Euler: algorithmic values moved per cell and step
KERNEL_SOURCES = ('paper_2411_11229_amd/csrc/hweno_kernels.hip',
                  'paper_2411_11229_amd/csrc/hweno_device.h')
PROFILE_JSON = os.path.join(ROOT, 'profiles', 'stage2d_euler_2048_traffic.json')


def kernel_hash():
    """sha256 of the stage kernels' sources with comments and blank space
    removed (the sources hold no string literal with comment markers), so
    that edits of comments alone keep the committed traffic record."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, p)).read()
        text = re.sub(r'/\*.*?\*/', ' ', text, flags=re.S)
        text = re.sub(r'//[^\n]*', ' ', text)
        # blank space matters only between two word characters
        text = re.sub(r'(?<=\w)\s+(?=\w)', ' ', text)
        h.update(re.sub(r'(?<!\w)\s+|\s+(?!\w)', '', text).encode())
    return h.hexdigest()


class HipEvents:
    """hipEvent_t handles through the HIP runtime already loaded by torch."""

    def __init__(self, n):
        self.hip = ctypes.CDLL('libamdhip64.so')
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float),
                                                 ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.ev = (ctypes.c_void_p * n)()
        for i in range(n):
            h = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(h)) != 0:
                raise RuntimeError('hipEventCreate failed')
            self.ev[i] = h
        self.n = n

    def group(self, k, size=4):
        """ctypes array view of events [k*size, (k+1)*size)."""
        arr = (ctypes.c_void_p * size)()
        for j in range(size):
            arr[j] = self.ev[k * size + j]
        return arr

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(ms), self.ev[a], self.ev[b]) != 0:
            raise RuntimeError('hipEventElapsedTime failed')
        return float(ms.value)

    def close(self):
        for i in range(self.n):
            self.hip.hipEventDestroy(self.ev[i])


def time_forward(n, precision, steps, warmup, seed=4000, basis='cell', ny=None):
    import torch
    from paper_2411_11229_amd import hweno, workloads
    ny = n if ny is None else ny
    w = workloads.euler2d_quadrants(n, seed=seed, ny=ny)
    prob = hweno.Problem(**w.problem_kwargs(), precision=precision, basis=basis)
    s = hweno.Solver(prob)
    dt_ = prob.dtype
    U = torch.tensor(w.U, dtype=dt_, device='cuda')
    V = torch.tensor(w.V, dtype=dt_, device='cuda')
    W = torch.tensor(w.W, dtype=dt_, device='cuda')
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    T_END = w.t_end
    if warmup:
        s.steps(U, V, W, t, warmup, T_END)
    ev = HipEvents(4 * steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.steps(U, V, W, t, steps, T_END, events=ev.ev)     # one call: K steps, fused alphas
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = [[ev.elapsed_ms(4 * k + j, 4 * k + j + 1) for j in range(3)] for k in range(steps)]
    ev.close()
    s.health()
    sim_t = float(t.item())
    cells = n * ny
    flat = [x for row in stage_ms for x in row]
    avg_stage = sum(flat) / len(flat)
    esize = 8 if precision == 'f64' else 4
    bytes_per_launch = VALUES_PER_CELL_STEP / 3.0 * esize * cells
    return dict(
        wall=wall, ms_per_step=1e3 * wall / steps, value=cells * 3 * steps / wall,
        avg_stage_ms=avg_stage, stage_ms_mean=[sum(r[j] for r in stage_ms) / steps for j in range(3)],
        bytes_per_launch=bytes_per_launch, achieved_gbs=bytes_per_launch / (avg_stage * 1e-3) / 1e9,
        sim_time=sim_t, state_finite=bool(torch.isfinite(U).all().item()))


def time_adjoint(precision, n=512, steps=200, every=20, basis='cell'):
    """Adjoint workload: 2D Euler n x n periodic smooth data (seed 5000),
    `steps` SSP-RK3 steps at the production dt of t = 0, checkpoints every
    `every` steps (None: segments sized from device memory, here one segment,
    nothing recomputed); J = dx dy/2 sum (U_T - U*)^2 with U* the seed-5001
    field. Returns forward and backward (segment recompute + adjoint steps)
    wall times of HwenoRollout, with the given characteristic basis."""
    import torch
    from paper_2411_11229_amd import hweno, rollout, workloads
    w = workloads.euler2d_smooth(n, seed=5000)
    tw = workloads.euler2d_smooth(n, seed=5001)
    prob = hweno.Problem(**w.problem_kwargs(), precision=precision, basis=basis)
    s = hweno.Solver(prob)
    dt_ = prob.dtype
    mk = lambda a: torch.tensor(a, dtype=dt_, device='cuda')
    a0 = s.max_wavespeed(mk(w.U)).cpu()
    dt_fixed = 0.6 / (float(a0[0]) / w.dx + float(a0[1]) / w.dy)
    target = mk(tw.U)

    def once(k):
        X = [mk(a).requires_grad_(True) for a in (w.U, w.V, w.W)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = rollout.rollout(s, X[0], X[1], X[2], steps=k, rule='fixed', dt_fixed=dt_fixed,
                              checkpoint_every=every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J = 0.5 * ((out[0] - target) ** 2).sum() * w.dx * w.dy
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ok = all(bool(torch.isfinite(x.grad).all()) for x in X)
        return t1 - t0, t2 - t1, ok

    seg = every if every is not None else rollout.segment_length(s, steps)
    once(min(seg, steps))             # warm-up
    fwd, bwd, ok = once(steps)
    kept = rollout.state_bytes_per_step(s) * (min(seg, steps) + 1)
    return dict(forward_s=fwd, backward_s=bwd, ratio=bwd / fwd, grads_finite=ok,
                segment_steps=seg, kept_state_gb=kept / 1e9)


def host_cpu():
    """Model name and logical CPU count of this host (/proc/cpuinfo)."""
    model = 'unknown'
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                model = line.split(':', 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return dict(model=model, logical_cpus=os.cpu_count(), usable_cpus=usable)


def cpu_baseline(n=1024, steps=2, seed=4000):
    """The FP64 oracle (unchanged) on a bounded sample: the same four-quadrant
    generator at n x n, `steps` SSP-RK3 steps; NumPy on one thread (about
    20 s), and the same oracle source on torch-CPU float64 with the host's
    threads (at most 16, the host's share of one GPU's cores)."""
    import numpy as np
    import torch
    from oracle import hweno as O
    from paper_2411_11229_amd import workloads
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:  # pragma: no cover
        lim = None
    w = workloads.euler2d_quadrants(n, seed=seed)
    p = O.Problem(**w.problem_kwargs())
    t0 = time.perf_counter()
    O.run(p, w.U, w.V, w.W, w.t_end, max_steps=steps)
    el = time.perf_counter() - t0
    if lim is not None:
        lim.unregister() if hasattr(lim, 'unregister') else None
    host = host_cpu()
    threads = max(1, min(16, host['usable_cpus'] or 1))
    old = torch.get_num_threads()
    torch.set_num_threads(threads)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    t0 = time.perf_counter()
    O.run(p, T(w.U), T(w.V), T(w.W), w.t_end, max_steps=steps)
    el_t = time.perf_counter() - t0
    torch.set_num_threads(old)
    return dict(value=n * n * 3 * steps / el, unit='cell-stage updates/s', cores=1,
                kind='oracle', sample=f'2D Euler four-quadrant {n}x{n}, {steps} SSP-RK3 steps, '
                                      f'NumPy FP64, 1 thread ({el:.1f} s)',
                host_cpu=host,
                torch_cpu=dict(value=n * n * 3 * steps / el_t, unit='cell-stage updates/s',
                               threads=threads,
                               sample=f'the same sample on torch-CPU float64 ({el_t:.1f} s)'))


def copy_bandwidth(gib=1.0, reps=20):
    """Achievable HBM bandwidth on this GPU (context for the roofline): a
    plain device-to-device copy of `gib` GiB, bytes read + written per
    second, timed with HIP events over `reps` copies after a warm-up."""
    import torch
    n = int(gib * (1 << 30) // 8)
    a = torch.ones(n, dtype=torch.float64, device='cuda')
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * n * 8 / (ms * 1e-3) / 1e9
    del a, b
    return dict(achieved=gbs, unit='GB/s', frac_of_peak=gbs / HBM_PEAK_GBS,
                kind=f'device copy of {gib:g} GiB (read + write), mean of {reps}')


def profile_record(precision='f64'):
    """The committed rocprofv3 counter summary of the FP64 or FP32 stage
    kernel (HBM traffic, VALU issue), if it was taken on the current kernel
    sources, else None."""
    if not os.path.exists(PROFILE_JSON):
        return None
    try:
        rec = json.load(open(PROFILE_JSON))
    except ValueError:
        return None
    if rec.get('kernel_source_sha256') != kernel_hash():
        return None
    return rec.get('f32', {}) if precision == 'f32' else rec


def traffic_record(precision='f64'):
    """HBM bytes per stage launch from the committed counter runs, or None."""
    rec = profile_record(precision)
    return None if rec is None else rec.get('traffic_bytes_per_launch')


def valu_record(precision='f64'):
    """VALU issue of the stage kernel from the committed counter runs
    (instructions per launch, the shares of wavefront and SIMD cycles issuing
    VALU, and the cycles the VALU work alone needs), or None."""
    rec = profile_record(precision)
    return None if rec is None else rec.get('valu')


def copy_probe(gib=1.0, reps=10):
    """Plain device copy of known size (for rocprofv3 counter calibration)."""
    import torch
    n = int(gib * (1 << 30) // 8)
    a = torch.ones(n, dtype=torch.float64, device='cuda')
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({'probe': 'copy', 'bytes_read_per_dispatch': n * 8,
                      'bytes_written_per_dispatch': n * 8, 'reps': reps}))


def _run_until(s, U, V, W, t_end, max_steps):
    """Steps to t_end in chunks; stops at the first chunk after which the
    state flags report a non-finite or non-physical state (or t is not
    finite). Returns (steps, t, status)."""
    import torch
    from paper_2411_11229_amd import hweno
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    k = 0
    while k < max_steps:
        s.steps(U, V, W, t, 32, t_end)
        k += 32
        try:
            s.health()
        except hweno.HwenoError as e:
            return k, float(t.item()), STATUS_NAMES.get(e.code, str(e.code))
        tv = float(t.item())
        if not tv == tv:
            return k, tv, 'non-finite time'
        if tv >= t_end:
            break
    return k, float(t.item()), 'ok' if float(t.item()) >= t_end else 'step limit'


STATUS_NAMES = {-4: 'non-finite state', -5: 'non-physical state'}


def basis_robustness():
    """Cell vs interface characteristic basis on the 1D Riemann + sine data
    (N = 2000, seeds 2000-2007, to each seed's T) and the 2D four-quadrant
    data (256^2, seeds 4000-4007, to T = 0.25), FP64: whether each run
    reaches T; and the 2048^2 stage-kernel time of both bases."""
    import torch
    from paper_2411_11229_amd import hweno, workloads
    out = {'c2_euler1d_riemann_2000': {}, 'c4_euler2d_quadrants_256': {}}
    for key, mk, seeds in (('c2_euler1d_riemann_2000', lambda sd: workloads.euler1d_riemann_sine(2000, seed=sd),
                            range(2000, 2008)),
                           ('c4_euler2d_quadrants_256', lambda sd: workloads.euler2d_quadrants(256, seed=sd),
                            range(4000, 4008))):
        for sd in seeds:
            w = mk(sd)
            row = {}
            for basis in ('cell', 'interface'):
                s = hweno.Solver(hweno.Problem(**w.problem_kwargs(), basis=basis))
                d = lambda a: None if a is None else torch.tensor(a, dtype=torch.float64, device='cuda')
                U, V, W = d(w.U), d(w.V), d(w.W)
                t0 = time.perf_counter()
                k, t, st = _run_until(s, U, V, W, w.t_end, 200000)
                torch.cuda.synchronize()
                row[basis] = dict(status=st, t=t, steps_le=k, s=round(time.perf_counter() - t0, 3))
            row['t_end'] = w.t_end
            out[key][str(sd)] = row
            print(json.dumps({key: {str(sd): row}}), file=sys.stderr, flush=True)
    cost = {}
    for basis in ('cell', 'interface'):
        r = time_forward(2048, 'f64', 5, 2, basis=basis)
        cost[basis] = r['avg_stage_ms']
    out['stage_ms_2048_f64'] = cost
    return out


def rayleigh_taylor_times():
    """Example 4.11 (gravity source, walls, fixed states) to t = 1.95 at the
    paper's three meshes, FP64, wall time per run (inputs resident; one
    warm-up run of 20 steps first)."""
    import torch
    from paper_2411_11229_amd import hweno, workloads
    out = {}
    for nx in (60, 120, 240):
        w = workloads.rayleigh_taylor(nx)
        s = hweno.Solver(hweno.Problem(**w.problem_kwargs()))
        d = lambda a: torch.tensor(a, dtype=torch.float64, device='cuda')
        U, V, W = d(w.U), d(w.V), d(w.W)
        s.run(U.clone(), V.clone(), W.clone(), t_end=w.t_end, max_steps=20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n, t, _ = s.run(U, V, W, t_end=w.t_end)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.health()
        out[f'{nx}x{4 * nx}'] = dict(steps=n, t=t, wall_s=wall,
                                     cell_stage_updates_per_s=nx * 4 * nx * 3 * n / wall)
        print(json.dumps({f'{nx}x{4 * nx}': out[f'{nx}x{4 * nx}']}), file=sys.stderr, flush=True)
    return out


def launch_bound_times():
    """Sizes where launch overhead sets the pace: the 1D Euler Riemann + sine
    data (N = 2000, seeds 2000-2007, each to its T) and Example 4.11 at
    60x240 to t = 1.95, FP64, stepped eagerly (five kernel launches per step)
    and through HIP graphs of 32 steps (Solver.run(graph=True)); wall time
    with inputs resident, after one warm-up run of each kind."""
    import torch
    from paper_2411_11229_amd import hweno, workloads
    out = {}
    cases = [(f'euler1d_riemann_2000_seed{sd}', workloads.euler1d_riemann_sine(2000, seed=sd))
             for sd in range(2000, 2008)]
    cases.append(('rayleigh_taylor_60x240', workloads.rayleigh_taylor(60)))
    for name, w in cases:
        s = hweno.Solver(hweno.Problem(**w.problem_kwargs()))
        d = lambda a: None if a is None else torch.tensor(a, dtype=torch.float64, device='cuda')
        row = {}
        for graph in (False, True):
            s.run(d(w.U), d(w.V), d(w.W), t_end=w.t_end, max_steps=64, graph=graph)
            U, V, W = d(w.U), d(w.V), d(w.W)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n, t, _ = s.run(U, V, W, t_end=w.t_end, graph=graph)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            s.health()
            row['graph' if graph else 'eager'] = dict(steps=n, t=t, wall_s=round(wall, 4),
                                                      us_per_step=round(1e6 * wall / n, 2))
        out[name] = row
        print(json.dumps({name: row}), file=sys.stderr, flush=True)
    return out


def double_mach_time(nx=1600):
    """Example 4.7 at nx x nx/4 to t = 0.2, FP64 (five start-up steps at CFL
    0.1, then 0.6): wall time with inputs resident."""
    import torch
    from paper_2411_11229_amd import hweno, workloads
    w = workloads.double_mach(nx)
    s = hweno.Solver(hweno.Problem(**w.problem_kwargs()))
    d = lambda a: torch.tensor(a, dtype=torch.float64, device='cuda')
    U, V, W = d(w.U), d(w.V), d(w.W)
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    for _ in range(5):
        s.step(U, V, W, t, w.t_end, cfl=0.1)
        n += 1
    while float(t.item()) < w.t_end and n < 100000:
        s.steps(U, V, W, t, 64, w.t_end)
        n += 64
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.health()
    return dict(cells=f'{nx}x{nx // 4}', t=float(t.item()), wall_s=wall, steps_upper_bound=n,
                rho_max=float(U[0].max()), rho_min=float(U[0].min()))


def share_times(n, g, steps, warmup):
    """Stage kernels on the per-GPU shape of a g-way y-slab decomposition of
    the n x n four-quadrant workload (n x n/g cells, transmissive y sides
    standing in for the halo rows a neighbour would send), FP64 and FP32,
    against the full n x n grid."""
    out = dict(shape=f'{n}x{n // g}', slabs=g)
    for prec in ('f64', 'f32'):
        r = time_forward(n, prec, steps, warmup, ny=n // g)
        out[prec] = dict(value=r['value'], avg_stage_ms=r['avg_stage_ms'],
                         frac=r['achieved_gbs'] / HBM_PEAK_GBS, ms_per_step=r['ms_per_step'])
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=30)
    ap.add_argument('--warmup', type=int, default=30)
    ap.add_argument('--n', type=int, default=2048)
    ap.add_argument('--no-cpu', action='store_true', help='skip the CPU oracle baseline')
    ap.add_argument('--no-fp32', action='store_true', help='skip the FP32 form')
    ap.add_argument('--no-adjoint', action='store_true', help='skip the adjoint/forward ratio')
    ap.add_argument('--adjoint-only', action='store_true',
                    help='time only the adjoint workload (for profiling)')
    ap.add_argument('--probe', choices=['copy'], help='run a calibration probe instead')
    ap.add_argument('--basis-robustness', action='store_true',
                    help='compare the cell and interface characteristic bases instead')
    ap.add_argument('--double-mach', action='store_true',
                    help='time the double Mach reflection example at 1600x400 instead')
    ap.add_argument('--launch-bound', action='store_true',
                    help='eager vs HIP-graph stepping on launch-bound sizes (1D Euler, Example 4.11)')
    ap.add_argument('--rayleigh-taylor', action='store_true',
                    help='time the Rayleigh-Taylor example at the paper\'s meshes instead')
    ap.add_argument('--share', type=int, metavar='G',
                    help='time the stage kernels on one of G y-slabs of the n x n grid instead '
                         '(the per-GPU shape of a G-way domain decomposition)')
    ap.add_argument('--precision', choices=['f64', 'f32'], default='f64',
                    help='precision of the headline run (and of --adjoint-only)')
    ap.add_argument('--basis', choices=['cell', 'interface'], default='cell',
                    help='characteristic basis of --adjoint-only')
    ap.add_argument('--checkpoint-every', type=int, default=20,
                    help='checkpoint segment of --adjoint-only (0: sized from device memory)')
    args = ap.parse_args()

    if args.gpus != 1:
        print(f'bench.py: the solver runs on one GPU (got --gpus {args.gpus}); '
              'there is no multi-GPU decomposition to measure.', file=sys.stderr)
        sys.exit(2)
    if args.probe == 'copy':
        copy_probe()
        return

    import torch
    if not torch.cuda.is_available():
        print('bench.py: no HIP device visible', file=sys.stderr)
        sys.exit(1)
    if args.adjoint_only:
        every = None if args.checkpoint_every == 0 else args.checkpoint_every
        print(json.dumps({f'adjoint_{args.precision}_{args.basis}':
                          time_adjoint(args.precision, basis=args.basis, every=every)}))
        return
    if args.basis_robustness:
        print(json.dumps({'basis_robustness': basis_robustness()}))
        return
    if args.double_mach:
        print(json.dumps({'double_mach': double_mach_time()}))
        return
    if args.rayleigh_taylor:
        print(json.dumps({'rayleigh_taylor': rayleigh_taylor_times()}))
        return
    if args.launch_bound:
        print(json.dumps({'launch_bound': launch_bound_times()}))
        return
    if args.share:
        print(json.dumps({'share': share_times(args.n, args.share, args.steps, args.warmup)}))
        return

    main_run = time_forward(args.n, args.precision, args.steps, args.warmup)
    fp32 = None
    if not args.no_fp32 and args.precision == 'f64':
        r = time_forward(args.n, 'f32', args.steps, args.warmup)
        fp32 = dict(value=r['value'], ms_per_step=r['ms_per_step'],
                    avg_stage_kernel_ms=r['avg_stage_ms'], achieved_gbs=r['achieved_gbs'],
                    frac=r['achieved_gbs'] / HBM_PEAK_GBS,
                    algorithmic_bytes_per_launch=r['bytes_per_launch'],
                    traffic=traffic_record('f32'), valu=valu_record('f32'))
    adjoint = None
    if not args.no_adjoint:
        a64 = time_adjoint('f64')
        a32 = time_adjoint('f32') if not args.no_fp32 else None
        adjoint = dict(workload='2D Euler 512x512 periodic smooth (seed 5000), 200 SSP-RK3 steps at '
                                'the t=0 production dt, checkpoints every 20, stage states stored '
                                'during segment recompute',
                       forward_s_f64=a64['forward_s'], backward_s_f64=a64['backward_s'],
                       ratio_f64=a64['ratio'], grads_finite=a64['grads_finite'])
        if a32:
            adjoint.update(forward_s_f32=a32['forward_s'], backward_s_f32=a32['backward_s'],
                           ratio_f32=a32['ratio'])
        # the interface (Roe) basis, and both bases with every step kept in
        # HBM (segments sized from device memory: no recomputation)
        ai = time_adjoint('f64', basis='interface')
        adjoint['ratio_f64_interface'] = ai['ratio']
        kept = {}
        for prec, basis in (('f64', 'cell'), ('f64', 'interface'), ('f32', 'cell'),
                            ('f32', 'interface')):
            if prec == 'f32' and args.no_fp32:
                continue
            a = time_adjoint(prec, basis=basis, every=None)
            kept[f'ratio_{prec}_{basis}'] = a['ratio']
            kept[f'kept_state_gb_{prec}'] = a['kept_state_gb']
            kept[f'segment_steps_{prec}'] = a['segment_steps']
        adjoint['all_steps_kept'] = kept
    cpu = None if args.no_cpu else cpu_baseline()
    copy = copy_bandwidth()

    traffic = traffic_record(args.precision)
    roof = dict(bound='hbm', achieved=main_run['achieved_gbs'], peak=HBM_PEAK_GBS, unit='GB/s',
                frac=main_run['achieved_gbs'] / HBM_PEAK_GBS,
                traffic=traffic,
                kernel=f'stage2d_kernel<Euler<2>, {"double" if args.precision == "f64" else "float"}>',
                algorithmic_bytes_per_launch=main_run['bytes_per_launch'],
                avg_launch_ms=main_run['avg_stage_ms'],
                stage_launch_ms=main_run['stage_ms_mean'],
                achievable_copy_gbs=copy['achieved'],
                valu=valu_record(args.precision))
    out = {
        'metric': '2D Euler cell-updates/s per RK stage',
        'value': main_run['value'],
        'unit': 'cell-stage updates/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': main_run['ms_per_step'],
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': args.precision,
        'data': 'synthetic',
        'config': {'workload': f'2D Euler {args.n}x{args.n} four-quadrant Riemann, transmissive, '
                               'production dt (CFL 0.6), seed 4000',
                   'cells': args.n * args.n, 'gas_gamma': 1.4, 'gamma0': 0.99, 'd0': 0.9,
                   'eps': 1e-10},
        'roofline': roof,
        'cpu_baseline': cpu,
        'hbm_copy': copy,
        'fp32': fp32,
        'adjoint_over_forward': adjoint,
        'sim_time_reached': main_run['sim_time'],
        'state_finite': main_run['state_finite'],
    }
    print(json.dumps(out))


if __name__ == '__main__':
    main()
