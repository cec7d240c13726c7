"""Host logic of the differentiable rollout: the memory-sized checkpoint
segments (no GPU needed)."""
import types

import torch

from paper_2411_11229_amd import rollout


def fake_solver(dim, ncomp, nx, ny, dtype):
    return types.SimpleNamespace(prob=types.SimpleNamespace(dim=dim, ncomp=ncomp, nx=nx, ny=ny,
                                                            dtype=dtype))


def test_state_bytes_per_step():
    s = fake_solver(2, 4, 512, 512, torch.float64)
    # u, v, w of 4 components at 512^2 in FP64, plus two stage states
    assert rollout.state_bytes_per_step(s) == 3 * 4 * 512 * 512 * 8 * 3
    assert rollout.state_bytes_per_step(s, store_stages=False) == 3 * 4 * 512 * 512 * 8
    s1 = fake_solver(1, 3, 1000, 1, torch.float32)
    assert rollout.state_bytes_per_step(s1) == 2 * 3 * 1000 * 4 * 3


def test_segment_length_from_budget():
    s = fake_solver(2, 4, 512, 512, torch.float64)
    per = rollout.state_bytes_per_step(s)
    # everything fits: one segment of all steps
    assert rollout.segment_length(s, 200, budget_bytes=201 * per) == 200
    assert rollout.segment_length(s, 200, budget_bytes=10 ** 15) == 200
    # the segment keeps k + 1 step-start states: the longest k that fits
    assert rollout.segment_length(s, 200, budget_bytes=21 * per) == 20
    assert rollout.segment_length(s, 200, budget_bytes=21 * per + per - 1) == 20
    # never below one step
    assert rollout.segment_length(s, 200, budget_bytes=0) == 1
