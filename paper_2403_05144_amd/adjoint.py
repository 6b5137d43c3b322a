"""Differentiated form: a time trajectory of the partitioned P-ERK step as a
torch.autograd.Function, with the discrete adjoint of libperk (pe_step_adjoint) and
checkpointed recomputation.

forward: n steps of size dt from u0 (slot layout), keeping the state every `every` steps.
backward: for each segment, last first, recompute the segment from its checkpoint, keeping
each step's state and record (K_1 and the stage values, pe_step_record), then apply the step
adjoint backwards through the segment from those records (pe_step_adjoint_recorded): every
step of the segment is computed once in the backward pass.  Memory: the checkpoints plus the
states and records of one segment (S + 1 state arrays per step).
"""
from __future__ import annotations

import torch


class PerkTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, solver, dt, n_steps, every):
        if every < 1:
            raise ValueError("checkpoint interval must be >= 1")
        ckpts = []
        solver.u.copy_(u0)
        for k in range(n_steps):
            if k % every == 0:
                ckpts.append(solver.u.clone())
            solver.step(dt, 1)
        ctx.solver, ctx.dt, ctx.n_steps, ctx.every, ctx.ckpts = solver, float(dt), int(n_steps), int(every), ckpts
        return solver.u.clone()

    @staticmethod
    def backward(ctx, lam):
        s, dt, n, every = ctx.solver, ctx.dt, ctx.n_steps, ctx.every
        lam = lam.contiguous().clone()
        for seg in reversed(range(len(ctx.ckpts))):
            k0, k1 = seg * every, min(n, seg * every + every)
            u = ctx.ckpts[seg]
            states, records = [], []
            for _ in range(k0, k1):
                u_next, rec = s.step_record(u, dt)
                states.append(u)
                records.append(rec)
                u = u_next
            for k in reversed(range(k1 - k0)):
                lam = s.step_adjoint_recorded(states[k], records[k], lam, dt)
            del states, records
        return lam, None, None, None, None


def trajectory(u0, solver, dt, n_steps, every=10):
    """u_N = Phi^n(u0) (slot layout), differentiable with respect to u0."""
    return PerkTrajectory.apply(u0, solver, dt, n_steps, every)


def slot_node_weights(solver):
    """Quadrature weights of every node in slot layout, [n_elements, nodes] (element volume
    included), for objectives written on the slot-layout state."""
    import numpy as np
    W = solver.node_weights()
    full = np.ascontiguousarray(np.broadcast_to(W[:, None, :], solver.leaf_shape))
    return solver.to_slot(full).view(solver.nv, -1, solver.Nd)[0, : solver.n_elements].clone()


def kinetic_energy(solver, u_slot, weights):
    """Discrete total kinetic energy sum_nodes w 1/2 |rho v|^2 / rho of a slot-layout state."""
    U = u_slot.view(solver.nv, -1, solver.Nd)[:, : solver.n_elements]
    mom2 = (U[1: 1 + solver.dim] ** 2).sum(0)
    return (weights * 0.5 * mom2 / U[0]).sum()
