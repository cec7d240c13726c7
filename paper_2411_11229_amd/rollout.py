"""Differentiable rollout of the HWENO-I time stepping (torch.autograd).

``HwenoRollout.apply(U0, V0, W0, solver, steps, ...)`` runs ``steps``
SSP-RK3 steps on the GPU and returns the final (U, V, W) (or (U, V) in 1D).
Its backward applies the hand-written discrete adjoint of each step
(``hweno_adjoint_step``) in reverse order, with the Lax-Friedrichs alphas and
time steps recorded by the forward held fixed. Memory: the forward keeps a
checkpoint of the state every ``checkpoint_every`` steps; the backward re-runs
one segment at a time from its checkpoint with the recorded dt and alphas
(``hweno_step_frozen``), keeping that segment's step-start states and, by
default, its stage states X^(1), X^(2), so the adjoint of a step needs no
forward recomputation. The last segment, which the backward needs first, is
kept by the forward itself (step-start and stage states, written by the
steps it takes anyway), so only the earlier segments are recomputed.

``checkpoint_every=None`` sizes the segments from device memory: the whole
rollout is one segment (nothing recomputed) when its step-start and stage
states fit in half of the free device memory, else the longest segment that
does. A 512^2 FP64 Euler rollout of 200 steps keeps 15 GB that way.
"""
import torch

from . import hweno


def state_bytes_per_step(solver, store_stages=True):
    """Device bytes one kept step costs: its step-start state (u, v[, w])
    and, with store_stages, its two stage states."""
    nf = 3 if solver.prob.dim == 2 else 2
    plane = solver.prob.ncomp * solver.prob.nx * solver.prob.ny
    item = torch.empty((), dtype=solver.prob.dtype).element_size()
    return nf * plane * item * (3 if store_stages else 1)


def segment_length(solver, steps, store_stages=True, budget_bytes=None):
    """Steps per checkpoint segment for a rollout of `steps` steps: all of
    them when the kept states fit in budget_bytes (default: half of the free
    device memory), else the longest segment that fits (at least 1)."""
    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info(solver.device)
        budget_bytes = free // 2
    per = state_bytes_per_step(solver, store_stages)
    return max(1, min(steps, budget_bytes // per - 1))


class HwenoRollout(torch.autograd.Function):

    @staticmethod
    def forward(ctx, U0, V0, W0, solver, steps, rule='production', cfl=0.6, dt_fixed=0.0,
                checkpoint_every=20, store_stages=True):
        two = solver.prob.dim == 2
        dev = solver.device
        if checkpoint_every is None:
            checkpoint_every = segment_length(solver, steps, store_stages)
        U = U0.detach().clone().contiguous()
        V = V0.detach().clone().contiguous()
        W = W0.detach().clone().contiguous() if two else None
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        dts = torch.zeros(steps, dtype=torch.float64, device=dev)
        recs = torch.zeros(steps, 6, dtype=torch.float64, device=dev)
        ckpts = []
        nf = 3 if two else 2
        plane = solver.prob.ncomp * solver.prob.nx * solver.prob.ny
        last = ((steps - 1) // checkpoint_every) * checkpoint_every if steps > 0 else 0
        n_last = steps - last
        # the last segment's step-start states and (optionally) stage states
        seg_states = torch.empty(checkpoint_every + 1, nf * plane, dtype=solver.prob.dtype, device=dev)
        seg_stages = (torch.empty(checkpoint_every, 2 * nf * plane, dtype=solver.prob.dtype,
                                  device=dev) if store_stages else None)
        for k in range(steps):
            if k % checkpoint_every == 0:
                ckpts.append((U.clone(), V.clone(), W.clone() if two else None))
            st = None
            if k >= last:
                j = k - last
                for f, x in enumerate((U, V, W)[:nf]):
                    seg_states[j, f * plane:(f + 1) * plane].copy_(x.reshape(-1))
                st = seg_stages[j] if seg_stages is not None else None
            solver.step(U, V, W, t, float('inf'), rule, cfl, dt_fixed,
                        dt_used=dts[k:k + 1], alpha_rec=recs[k], stages=st)
        ctx.solver, ctx.steps, ctx.every = solver, steps, checkpoint_every
        ctx.ckpts, ctx.dts, ctx.recs, ctx.two = ckpts, dts, recs, two
        ctx.store_stages = store_stages
        ctx.last = (last, n_last, seg_states, seg_stages)
        return (U, V, W) if two else (U, V)

    @staticmethod
    def backward(ctx, *grads):
        s, two, every = ctx.solver, ctx.two, ctx.every
        nf = 3 if two else 2
        lam = [g.contiguous().clone() if g is not None else torch.zeros(s.prob.shape, dtype=s.prob.dtype,
                                                                        device=s.device)
               for g in grads[:nf]]
        out = [s.new_state() for _ in range(nf)]
        plane = s.prob.ncomp * s.prob.nx * s.prob.ny
        last, n_last, starts, stage_buf = ctx.last
        ctx.last = None

        def fields(k):
            return [starts[k, f * plane:(f + 1) * plane].view(s.prob.shape) for f in range(nf)]

        for seg, start in reversed(list(enumerate(range(0, ctx.steps, every)))):
            end = min(start + every, ctx.steps)
            if start != last:
                # recompute the segment from its checkpoint (the last one is
                # still held from the forward); each step writes the next
                # step-start state out of place
                for dst, src in zip(fields(0), ctx.ckpts[seg]):
                    dst.copy_(src)
                for k in range(start, end):
                    j = k - start
                    X = fields(j)
                    st = stage_buf[j] if stage_buf is not None else None
                    s.step_frozen(X[0], X[1], X[2] if two else None, ctx.dts[k:k + 1], ctx.recs[k],
                                  stages=st, out=fields(j + 1))
            for k in reversed(range(start, end)):
                j = k - start
                X = fields(j)
                st = stage_buf[j] if stage_buf is not None else None
                s.adjoint_step(X[0], X[1], X[2] if two else None, ctx.dts[k:k + 1], ctx.recs[k], lam,
                               out, stages=st)
                lam, out = out, lam
        gU, gV = lam[0], lam[1]
        gW = lam[2] if two else None
        return gU, gV, gW, None, None, None, None, None, None, None


def rollout(solver, U0, V0, W0=None, steps=1, rule='production', cfl=0.6, dt_fixed=0.0,
            checkpoint_every=20, store_stages=True):
    """Functional form of HwenoRollout.apply."""
    return HwenoRollout.apply(U0, V0, W0, solver, steps, rule, cfl, dt_fixed, checkpoint_every,
                              store_stages)
