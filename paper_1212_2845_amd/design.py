"""Gradient-driven design through the adjoint (the use the paper's
conclusion points to: evolving or optimising soft actuated structures).

``optimize_phases`` tunes the per-voxel actuation phases of an object
standing on the floor so that its centre of mass travels furthest along an
axis in a fixed number of steps.  Each iteration starts a fresh simulation
from rest at t = 0, runs the differentiable rollout (``rollout``: one
recorded forward run and one reverse run in the library) and takes an Adam
step on the phases.
"""
import numpy as np


def com_travel(u, mass, axis=0):
    """Mass-weighted mean displacement along ``axis`` of the cells (u: ncell
    x 3 torch tensor, mass: ncell torch tensor, zero for empty cells)."""
    return (u[:, axis] * mass).sum() / mass.sum()


def optimize_phases(make_sim, E, rho, phase0, amp, steps, iters, lr=0.3, K=100, axis=0):
    """Maximise centre-of-mass travel along ``axis`` after ``steps`` steps
    over the per-voxel phases (radians, ncell values; empty cells ignored).
    make_sim() returns a fresh Sim at rest (parameter mode is set by the
    rollout); E and rho are the per-cell modulus and density (held fixed),
    amp the per-cell signal amplitude.  Returns the final phases and the
    travel of every iteration (evaluated before its update)."""
    import torch
    from . import rollout
    phase = torch.tensor(np.asarray(phase0, dtype=np.float64), requires_grad=True)
    Et = torch.tensor(np.asarray(E, dtype=np.float64))
    rt = torch.tensor(np.asarray(rho, dtype=np.float64))
    opt = torch.optim.Adam([phase], lr=lr)
    history = []
    for _ in range(int(iters)):
        sim = make_sim()
        sim.grad_bind(int(steps), int(K))
        l = float(sim._prm.voxel_size)
        mass = rt * l ** 3 * torch.tensor((sim.grid.reshape(-1) > 0).astype(np.float64))
        u, _ = rollout(sim, Et, rt, phase, amp, int(steps))
        travel = com_travel(u, mass, axis)
        opt.zero_grad()
        (-travel).backward()
        opt.step()
        history.append(float(travel.detach()))
    return phase.detach().numpy(), history
