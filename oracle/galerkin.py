"""Dense Galerkin system for N active spheres, solved directly (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

This follows the Dirichlet problem of sections II-III in the lower/higher
partition of the coefficient vectors:

* Lower traction coefficients F^L (force, torque) are known from the overdamped
  force and torque balance: the contact force and torque are minus the body
  force and torque (section II, Newton's equations as constraints).
* The higher traction unknowns kept at this truncation (traction ranks <= 2) are
  the symmetric traceless first moments, written as the flow stresslet
  Sigma_n = a Q^(20)_n = S_n - (8/3) pi eta a^3 s_n (section IV, the named
  combination "stresslet"), 5 per sphere.
* The higher rows of the linear system (the Schur "H" rows, section II) are the
  symmetric l = 1 Galerkin conditions on each sphere. With the flow of every
  other sphere projected by the target operator E (Faxen form of the matrix
  elements, section III) they read

      Sigma_n / gamma - sum_{m != n} E[Sigma_m](R_n - R_m)
          = sum_{m != n} E[F_m, T_m, d_m](R_n - R_m) - c s_n,

  gamma = (20/3) pi eta a^3.  ``c`` is the self-slip coefficient: c = 1 makes
  the exterior flow of a lone sphere equal its prescribed strain slip on its
  surface (the boundary condition of section II); the paper's one-body table
  corresponds to c = 7/5 (kept as an option).
* The lower rows then give the rigid-body motion (generalized Stokes laws,
  section III):
      V_n = V^a_n + F^e_n / (6 pi eta a) + sum_{m != n} U[F, T, Sigma, d]_m,
      Omega_n = T^e_n / (8 pi eta a^3) + sum_{m != n} W[F, T, Sigma, d]_m,
  with V^a_n = -V^(1s)_n (minus the mean slip) and no antisymmetric slip.
* The traction stresslet is S_n = Sigma_n + (8/3) pi eta a^3 s_n.

The matrix I/gamma - K^SS is symmetric (reciprocity of the Green's function)
and positive definite for non-overlapping spheres, so numpy.linalg.solve and a
Cholesky solve must agree.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import greens


@dataclasses.dataclass
class Params:
    eta: float = 1.0 / (6.0 * np.pi)
    a: float = 1.0
    self_slip_c: float = 1.0


def constants(prm: Params):
    gamma = 20.0 / 3.0 * np.pi * prm.eta * prm.a ** 3
    return dict(gamma=gamma,
                drag_t=6.0 * np.pi * prm.eta * prm.a,
                drag_r=8.0 * np.pi * prm.eta * prm.a ** 3,
                slip_to_S=8.0 / 3.0 * np.pi * prm.eta * prm.a ** 3)


def pair_matrix(R, target, source, prm: Params, rows=None, chunk=4096):
    """Dense [len(rows)*dT, N*dX] of blocks B(R_n - R_m); the n == m blocks are zero."""
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    dT, dX = greens.TARGET_DIM[target], greens.SOURCE_DIM[source]
    out = np.zeros((len(rows), dT, n, dX))
    for i0 in range(0, len(rows), max(1, chunk // max(n, 1))):
        rr = rows[i0:i0 + max(1, chunk // max(n, 1))]
        dx = R[rr, None, :] - R[None, :, :]
        mask = np.ones((len(rr), n), dtype=bool)
        mask[np.arange(len(rr)), rr] = False
        blk = greens.block(target, source, dx[mask], prm.a, prm.eta)
        full = np.zeros((len(rr), n, dT, dX))
        full[mask] = blk
        out[i0:i0 + len(rr)] = full.transpose(0, 2, 1, 3)
    return out.reshape(len(rows) * dT, n * dX)


def system_matrix(R, prm: Params):
    """A = I/gamma - K^SS, [5N x 5N]."""
    n = len(R)
    g = constants(prm)["gamma"]
    return np.eye(5 * n) / g - pair_matrix(R, "E", "S", prm)


def _modes(modes):
    """Optional fixed sources of the minimal truncation: {"SEPT": gamma [N, 10], "VORT": psi [N, 5],
    "SPIN": lambda [N, 10]} (absent or None entries are zero)."""
    return {k: v for k, v in (modes or {}).items() if v is not None}


def rhs(R, v2s, v3t, Fe, Te, prm: Params, rows=None, modes=None):
    """b = sum_{m != n} E[F, T, d (, gamma, psi, lambda)] - c s, flattened [5N] (or the given rows)."""
    R = np.asarray(R, dtype=np.float64)
    rows = np.arange(len(R)) if rows is None else np.asarray(rows)
    b = np.zeros(5 * len(rows))
    for kind, vals in {"F": Fe, "T": Te, "D": v3t, **_modes(modes)}.items():
        if vals is not None:  # None stands for an absent source
            b = b + pair_matrix(R, "E", kind, prm, rows) @ np.ravel(vals)
    b = b - prm.self_slip_c * np.ravel(np.asarray(v2s)[rows])
    return b


def outputs(R, v1s, v2s, v3t, Fe, Te, Sigma, prm: Params, rows=None, modes=None):
    """Rigid-body motion and traction stresslet from a given flow stresslet Sigma [N, 5]. The
    septlet, vortlet and spinlet slip modes (``modes``) move no lone sphere (their mean and their
    mean n x slip vanish); they act on the others through their flows."""
    R = np.asarray(R, dtype=np.float64)
    rows = np.arange(len(R)) if rows is None else np.asarray(rows)
    k = constants(prm)
    src = {kind: np.ravel(vals) for kind, vals in {"F": Fe, "T": Te, "S": Sigma, "D": v3t, **_modes(modes)}.items()
           if vals is not None}  # None stands for an absent source
    V = -np.asarray(v1s)[rows] + (np.asarray(Fe)[rows] / k["drag_t"] if Fe is not None else 0.0)
    W = np.asarray(Te)[rows] / k["drag_r"] if Te is not None else np.zeros((len(rows), 3))
    for X, vec in src.items():
        V = V + (pair_matrix(R, "U", X, prm, rows) @ vec).reshape(-1, 3)
        W = W + (pair_matrix(R, "W", X, prm, rows) @ vec).reshape(-1, 3)
    S = np.asarray(Sigma)[rows] + k["slip_to_S"] * np.asarray(v2s)[rows]
    return V, W, S


def workload_modes(w):
    """The septlet, vortlet and spinlet slip modes a workload carries (fields gam, psi, lam)."""
    return {"SEPT": getattr(w, "gam", None), "VORT": getattr(w, "psi", None), "SPIN": getattr(w, "lam", None)}


def solve(w, prm: Params | None = None, method="lu"):
    """Full solve for a workload-like object (fields R, v1s, v2s, v3t, Fe, Te; optionally gam,
    psi, lam). Returns a dict with V, W (= Omega), S, Sigma [N, 5], b [5N] and A.
    """
    prm = prm or Params(eta=getattr(w, "eta", 1.0 / (6 * np.pi)), a=getattr(w, "a", 1.0))
    modes = workload_modes(w)
    A = system_matrix(w.R, prm)
    b = rhs(w.R, w.v2s, w.v3t, w.Fe, w.Te, prm, modes=modes)
    if method == "lu":
        sig = np.linalg.solve(A, b)
    elif method == "cholesky":
        L = np.linalg.cholesky(A)
        sig = np.linalg.solve(L.T, np.linalg.solve(L, b))
    else:
        raise ValueError(method)
    Sigma = sig.reshape(-1, 5)
    V, W, S = outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sigma, prm, modes=modes)
    return dict(V=V, W=W, S=S, Sigma=Sigma, b=b, A=A)


def superposition(w, prm: Params | None = None):
    """Superposition approximation (section IV): one-body tractions, pairwise-summed flows.

    The flow stresslet of each sphere is its lone-sphere value -c gamma s_n and
    the rigid-body motion is the direct sum of the pair blocks.
    """
    prm = prm or Params(eta=w.eta, a=w.a)
    g = constants(prm)["gamma"]
    Sigma = -prm.self_slip_c * g * np.asarray(w.v2s)
    V, W, S = outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sigma, prm, modes=workload_modes(w))
    return dict(V=V, W=W, S=S, Sigma=Sigma)


def flow_field(X, R, Fe, Te, Sigma, v3t, prm: Params, modes=None):
    """Exterior flow at field points X [M, 3] (section III): the sum over spheres m of the source
    flows of its force, torque, flow stresslet and rank-3 trace mode (and of the septlet, vortlet
    and spinlet slip modes in ``modes``) at X - R_m, each carrying its own finite-size operator and
    none at the field point. None stands for an absent source."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    u = np.zeros_like(X)
    sources = {"F": Fe, "T": Te, "S": Sigma, "D": v3t}
    sources.update(_modes(modes))
    for m in range(R.shape[0]):
        dx = X - R[m]
        for kind, vals in sources.items():
            if vals is not None:
                u += greens.flow(kind, dx, prm.a, prm.eta) @ np.asarray(vals, dtype=np.float64)[m]
    return u


def matvec_rows(R, x, rows, prm: Params):
    """(A x) restricted to the given particles, without forming A: [len(rows), 5]."""
    g = constants(prm)["gamma"]
    x = np.asarray(x).reshape(-1, 5)
    y = x[rows] / g - (pair_matrix(R, "E", "S", prm, rows) @ np.ravel(x)).reshape(-1, 5)
    return y


# ---------------------------------------------------------------- traction ranks <= 3
# The quadratic-order traction modes of the minimal truncation (section IV: septlet Gamma, vortlet
# Psi, potential dipole D) as unknowns. Each sphere's exterior flow is written through the
# equivalent slips X^gam (7-basis), X^psi (5-basis), X^d (the slips a lone sphere would need to
# produce the same flow of that mode) beside the flow stresslet Sigma. The Galerkin conditions of
# the l = 2 surface modes (section III coefficients V^(3), decomposed as in section IV) read
#     X^alpha_n + P^alpha[ sum_{m != n} u_m ](R_n) = v^alpha_n     (prescribed slip of mode alpha),
# u_m the flow of sphere m (force, torque, Sigma, the three equivalent slips, spinlet slip), and the
# stresslet rows keep their form with the new modes' flows among the coupled sources:
#     Sigma_n / gamma - E[ sum_m u_m(Sigma, X) ] = E[ sum_m u_m(F, T, lambda) ] - c s_n.
# Unknowns per sphere: [Sigma (5), X^gam (7), X^psi (5), X^d (3)] = 20.
RANK3_BLOCKS = (("E", "S", 5), ("GAM", "SEPT7", 7), ("PSI", "VORT", 5), ("DD", "D", 3))
RANK3_DIM = 20


def _rank3_offsets():
    off, o = {}, 0
    for tgt, src, dim in RANK3_BLOCKS:
        off[tgt] = off[src] = (o, dim)
        o += dim
    return off


def system_matrix_rank3(R, prm: Params):
    """A [20N x 20N] of the rank <= 3 system (unknowns interleaved per sphere as above)."""
    R = np.asarray(R, dtype=np.float64)
    n = len(R)
    g = constants(prm)["gamma"]
    off = _rank3_offsets()
    A = np.zeros((n, RANK3_DIM, n, RANK3_DIM))
    for tgt, _, _ in RANK3_BLOCKS:
        to, td = off[tgt]
        sign = -1.0 if tgt == "E" else 1.0
        for _, src, _ in RANK3_BLOCKS:
            so, sd = off[src]
            blk = pair_matrix(R, tgt, src, prm).reshape(n, td, n, sd)
            A[:, to:to + td, :, so:so + sd] += sign * blk
        diag = 1.0 / g if tgt == "E" else 1.0
        for i in range(n):
            A[i, to:to + td, i, to:to + td] += diag * np.eye(td)
    return A.reshape(n * RANK3_DIM, n * RANK3_DIM)


def matvec_rows_rank3(R, x, rows, prm: Params):
    """(A x) of the rank <= 3 system restricted to the given spheres, without forming A:
    [len(rows), 20] (x [N, 20] in the unknowns' layout above)."""
    R = np.asarray(R, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(len(R), RANK3_DIM)
    rows = np.asarray(rows)
    g = constants(prm)["gamma"]
    off = _rank3_offsets()
    y = np.zeros((len(rows), RANK3_DIM))
    for tgt, _, _ in RANK3_BLOCKS:
        to, td = off[tgt]
        sign = -1.0 if tgt == "E" else 1.0
        acc = np.zeros(len(rows) * td)
        for _, src, _ in RANK3_BLOCKS:
            so, sd = off[src]
            acc = acc + pair_matrix(R, tgt, src, prm, rows) @ np.ravel(x[:, so:so + sd])
        diag = 1.0 / g if tgt == "E" else 1.0
        y[:, to:to + td] = diag * x[rows, to:to + td] + sign * acc.reshape(len(rows), td)
    return y


def _prescribed_quadratic(w):
    """The prescribed quadratic-order slips of a workload in the unknowns' coordinates."""
    from .basis import sym3_from10, to7
    n = len(w.R)
    gam = getattr(w, "gam", None)
    psi = getattr(w, "psi", None)
    g7 = to7(sym3_from10(gam)) if gam is not None else np.zeros((n, 7))
    p5 = np.asarray(psi, dtype=np.float64) if psi is not None else np.zeros((n, 5))
    d3 = np.asarray(w.v3t, dtype=np.float64) if w.v3t is not None else np.zeros((n, 3))
    return g7, p5, d3


def rhs_rank3(w, prm: Params):
    """b [20N]: the fixed sources (force, torque, spinlet slip) and the prescribed slips."""
    R = np.asarray(w.R, dtype=np.float64)
    n = len(R)
    off = _rank3_offsets()
    b = np.zeros((n, RANK3_DIM))
    g7, p5, d3 = _prescribed_quadratic(w)
    fixed = {k: v for k, v in {"F": w.Fe, "T": w.Te, "SPIN": getattr(w, "lam", None)}.items() if v is not None}
    for tgt, _, _ in RANK3_BLOCKS:
        to, td = off[tgt]
        acc = np.zeros(n * td)
        for kind, vals in fixed.items():
            acc = acc + pair_matrix(R, tgt, kind, prm) @ np.ravel(vals)
        b[:, to:to + td] = acc.reshape(n, td) if tgt == "E" else -acc.reshape(n, td)
    b[:, 0:5] -= prm.self_slip_c * np.asarray(w.v2s)
    b[:, 5:12] += g7
    b[:, 12:17] += p5
    b[:, 17:20] += d3
    return b.ravel()


def solve_rank3(w, prm: Params | None = None):
    """Dense solve of the rank <= 3 system for a workload (fields R, v1s, v2s, v3t, Fe, Te and
    optionally gam, psi, lam). Returns V, W, S, Sigma, the equivalent slips gam7 [N, 7], psi [N, 5],
    d [N, 3], and b, A."""
    prm = prm or Params(eta=getattr(w, "eta", 1.0 / (6 * np.pi)), a=getattr(w, "a", 1.0))
    A = system_matrix_rank3(w.R, prm)
    b = rhs_rank3(w, prm)
    x = np.linalg.solve(A, b).reshape(-1, RANK3_DIM)
    Sigma, g7, p5, d3 = x[:, 0:5], x[:, 5:12], x[:, 12:17], x[:, 17:20]
    modes = {"SEPT7": g7, "VORT": p5, "SPIN": getattr(w, "lam", None)}
    V, W, S = outputs(w.R, w.v1s, w.v2s, d3, w.Fe, w.Te, Sigma, prm, modes=modes)
    return dict(V=V, W=W, S=S, Sigma=Sigma, gam7=g7, psi=p5, d=d3, b=b, A=A)
