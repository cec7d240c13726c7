"""Graph-captured stepping, Solver.run(graph=True): one chunk of SSP-RK3
steps is captured as a HIP graph and replayed. Against eager stepping on the
same data it must give the same number of steps, the same final time, the
same per-step dt and stage alphas and the same fields, bit for bit: over many
replays (with the run's own syncs and eager copies between them), past the
end time (device-skipped steps inside a replay) and with an eager tail when
the step limit is not a multiple of the chunk."""
import pytest
import torch

from paper_2411_11229_amd import workloads as WL

from test_gpu_parity import dev, solver

pytestmark = pytest.mark.gpu


def _run(w, graph, basis='cell', **kw):
    s = solver(w, basis=basis)
    two = w.dim == 2
    U, V = dev(w.U), dev(w.V)
    W = dev(w.W) if two else None
    out = s.run(U, V, W, t_end=w.t_end, record=True, graph=graph, **kw)
    s.health()
    return out, (U, V, W)


@pytest.mark.parametrize("name,mk,kw", [
    ('euler1d-riemann-2000-to-T', lambda: WL.euler1d_riemann_sine(2000, seed=2000), {}),
    ('euler1d-riemann-97-limit-70', lambda: WL.euler1d_riemann_sine(97, seed=2001), dict(max_steps=70)),
    ('rayleigh-taylor-16x64-limit-100', lambda: WL.rayleigh_taylor(16), dict(max_steps=100, chunk=16)),
    ('double-mach-64x16-limit-40', lambda: WL.double_mach(64), dict(max_steps=40, cfl=0.1)),
    ('euler2d-quadrants-96x80-limit-50', lambda: WL.euler2d_quadrants(96, seed=4302, ny=80),
     dict(max_steps=50)),
    ('euler2d-quadrants-96x80-interface-limit-30',
     lambda: WL.euler2d_quadrants(96, seed=4304, ny=80), dict(max_steps=30, basis='interface')),
], ids=lambda x: x if isinstance(x, str) else '')
def test_graph_run_equals_eager_run(name, mk, kw):
    print(f'case {name}', flush=True)
    w = mk()
    (n0, t0, dts0, rec0), X0 = _run(w, False, **kw)
    (n1, t1, dts1, rec1), X1 = _run(w, True, **kw)
    print(f'  steps {n0} / {n1}, t {t0!r} / {t1!r}')
    assert n1 == n0 and t1 == t0
    assert torch.equal(dts1, dts0) and torch.equal(rec1, rec0)
    for a, b in zip(X1, X0):
        if a is not None:
            assert torch.equal(a, b)
