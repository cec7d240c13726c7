"""The oracle on torch-CPU float64 (the gradient reference of the adjoint):
same values as on NumPy, and its reverse-mode gradient of a final-state loss
agrees with finite differences (frozen alphas and time steps). The nonlinear
weights make the map strongly curved (epsilon = 1e-10 in their denominators),
so the difference quotients are Richardson-extrapolated central differences
at small steps: (4 D(e) - D(2e)) / 3 removes the e^2 term."""
import numpy as np
import pytest
import torch

from oracle import hweno as O
from paper_2411_11229_amd import workloads as WL


def _setup(kind):
    if kind == 'euler2d':
        w = WL.euler2d_smooth(10, seed=3100, ny=9)
    elif kind == 'euler2d-reflective':
        w = WL.with_bc(WL.euler2d_smooth(10, seed=3102, ny=9),
                       ('reflective', 'transmissive', 'reflective', 'reflective'))
    elif kind == 'rayleigh-taylor':
        w = WL.rayleigh_taylor(6)
    elif kind == 'euler1d':
        w = WL.euler1d_riemann_sine(24, seed=2010)
    elif kind == 'euler1d-reflective':
        w = WL.with_bc(WL.euler1d_riemann_sine(24, seed=2011),
                       ('reflective', 'reflective', 'periodic', 'periodic'))
    else:
        w = WL.paper_burgers2d(8)
    p = O.Problem(**w.problem_kwargs())
    _, _, _, log = O.run(p, w.U, w.V, w.W, 1e9, max_steps=3)
    return w, p, log


def _loss(p, w, log, U, V, W, target):
    Ue, _, _ = O.run_fixed(p, U, V, W, log.dts, log.alphas)
    return 0.5 * ((Ue - target) ** 2).sum() * p.dx * (p.dy if p.dim == 2 else 1.0)


@pytest.mark.parametrize("kind", ["euler1d", "euler1d-reflective", "euler2d",
                                  "euler2d-reflective", "rayleigh-taylor", "burgers2d"])
def test_torch_oracle_gradient_matches_finite_differences(kind):
    w, p, log = _setup(kind)
    rng = np.random.default_rng(5)
    target = w.U + 0.05 * rng.standard_normal(w.U.shape)
    t = lambda a: None if a is None else torch.tensor(a, dtype=torch.float64, requires_grad=True)
    U, V, W = t(w.U), t(w.V), t(w.W)
    tt = torch.tensor(target, dtype=torch.float64)
    J = _loss(p, w, log, U, V, W, tt)
    J.backward()
    # torch and NumPy oracles agree on the forward
    Un, _, _ = O.run_fixed(p, w.U, w.V, w.W, log.dts, log.alphas)
    Ut, _, _ = O.run_fixed(p, *(None if a is None else torch.tensor(a) for a in (w.U, w.V, w.W)),
                           log.dts, log.alphas)
    np.testing.assert_allclose(Ut.numpy(), Un, rtol=1e-13, atol=1e-13)
    for k in range(4):
        d = [rng.standard_normal(a.shape) if a is not None else None for a in (w.U, w.V, w.W)]
        eps = 1e-7
        def J_at(s):
            args = [None if a is None else torch.tensor(a + s * da) for a, da in zip((w.U, w.V, w.W), d)]
            return float(_loss(p, w, log, *args, tt))
        D = lambda e: (J_at(e) - J_at(-e)) / (2 * e)
        fd = (4 * D(eps) - D(2 * eps)) / 3
        ad = sum(float((g.grad * torch.tensor(da)).sum()) for g, da in zip((U, V, W), d) if g is not None)
        assert ad == pytest.approx(fd, rel=1e-6, abs=1e-10), (k, ad, fd)
