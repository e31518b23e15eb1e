"""Static equilibrium by dynamic relaxation (the paper's static validation:
section Validation, Table 1), with convergence detected from the kinetic
energy reduction of the current state (``vx_energy``).

``relax`` steps the simulation in chunks and stops once the kinetic energy
has fallen below ``rel_tol`` times the elastic energy stored in the bonds at
``consecutive`` successive checks (one check can fall on a turning point of
an oscillation, where the kinetic energy passes through zero).  The damping that drives the relaxation is the
simulation's own (ground damping zeta_slow, bond damping zeta_bond): near
critical for the lowest mode the kinetic energy decays fastest.
"""


def relax(sim, rel_tol=1e-12, chunk=1000, max_steps=1_000_000, consecutive=2):
    """Relax ``sim`` towards static equilibrium.  Returns a dict with the
    number of steps taken, whether the criterion was met and the (steps,
    kinetic, elastic) history of the checks."""
    history = []
    steps = 0
    run = 0
    while steps < max_steps:
        n = min(int(chunk), int(max_steps) - steps)
        sim.step(n)
        steps += n
        e = sim.energy()
        history.append((steps, e["kinetic"], e["elastic"]))
        run = run + 1 if (e["elastic"] > 0.0 and e["kinetic"] <= rel_tol * e["elastic"]) else 0
        if run >= consecutive:
            return {"steps": steps, "converged": True, "history": history}
    return {"steps": steps, "converged": False, "history": history}
