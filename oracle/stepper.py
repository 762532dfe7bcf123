"""Adams-Bashforth rigid-body integration of spheres in a harmonic trap (test infrastructure only).

Kinematics of section II: dR/dt = V, dp/dt = Omega x p. The paper fixes no
integrator; this is the two-step Adams-Bashforth rule with a forward-Euler
first step, p renormalised after every step. Each step re-solves the many-body
problem with the trap force F^e = -k R, no torque, and slip modes rebuilt from
the current orientations.
"""
import numpy as np

from . import galerkin
from .basis import to5


class _State:
    def __init__(self, R, p, v1s, v2s, v3t, Fe, Te, eta, a):
        self.R, self.p, self.v1s, self.v2s, self.v3t, self.Fe, self.Te = R, p, v1s, v2s, v3t, Fe, Te
        self.eta, self.a = eta, a


def slip_from_orientation(p, coef):
    """V^(1s) = c1 p, V^(2s) = c2 3(pp - I/3) (5-basis), V^(3t) = c3 p."""
    pp = p[:, :, None] * p[:, None, :]
    return coef[0] * p, coef[1] * to5(3.0 * (pp - np.eye(3) / 3.0)), coef[2] * p


def run(R, p, k_trap, coef, dt, nsteps, prm: galerkin.Params, order=2, superposition=False, solve=None):
    """Integrate nsteps; returns (R, p, history of per-step dicts). With superposition the motion
    comes from the superposition approximation (section IV) instead of the many-body solve; `solve`
    (state, prm) -> dict with V, W replaces the unbounded-fluid solve (a bounded geometry)."""
    R = np.array(R, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    prev = None
    hist = []
    for _ in range(nsteps):
        v1s, v2s, v3t = slip_from_orientation(p, coef)
        st = _State(R, p, v1s, v2s, v3t, -k_trap * R, np.zeros_like(R), prm.eta, prm.a)
        if solve is not None:
            sol = solve(st, prm)
        else:
            sol = galerkin.superposition(st, prm) if superposition else galerkin.solve(st, prm)
        V, W = sol["V"], sol["W"]
        pdot = np.cross(W, p)
        if order == 1 or prev is None:
            R = R + dt * V
            p = p + dt * pdot
        else:
            R = R + dt * (1.5 * V - 0.5 * prev[0])
            p = p + dt * (1.5 * pdot - 0.5 * prev[1])
        p = p / np.linalg.norm(p, axis=1, keepdims=True)
        prev = (V, pdot)
        hist.append(dict(V=V, W=W))
    return R, p, hist
