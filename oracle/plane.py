"""Spheres in the half space z > z_w bounded by a flat stress-free (free-slip) plane (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper notes (Discussion) that other geometries follow from the Green's function of that
geometry, naming plane walls. For a plane on which the fluid slips freely (zero normal velocity and
zero tangential stress: u_z = 0, d_z u_x = d_z u_y = 0 at z = z_w) the Green's function is the
free-space one plus its mirror image: with M = diag(1, 1, -1) and the mirror image y* of a point y,
the flow of a point force F at y together with that of the force M F at y* has u_z = 0 and
d_z u_parallel = 0 on the plane, because the sum is symmetric under the reflection. Every source
flow of the free-space blocks reflects in the same way, each by its own transformation law:

    force F (polar vector)          F* = M F
    torque T (axial vector)         T* = -M T
    stresslet Sigma                 Sigma* = M Sigma M        (5-basis: diag(1, 1, 1, -1, -1))
    rank-3 trace mode d (polar)     d* = M d

So the half-space system is the free-space one with every block B(R_n - R_m) (m != n) joined by the
image blocks B(R_n - R*_m) S_X (every m, the sphere's own image included), S_X the transformation of
the source coefficients, and the same target projections (the image flows are Stokes flows in the
fluid, so the Faxen operators act on them as on any incident flow). Spheres must lie in the fluid,
z_n - z_w >= a (then every image is at least 2a away).
"""
from __future__ import annotations

import numpy as np

from . import galerkin, greens

M3 = np.diag([1.0, 1.0, -1.0])
IMAGE_MAP = {
    "F": M3,
    "T": -M3,
    "S": np.diag([1.0, 1.0, 1.0, -1.0, -1.0]),  # Sigma -> M Sigma M in the 5-basis (xz, yz flip)
    "D": M3,
}


def mirror(R, z_w):
    """Mirror images of the centres in the plane z = z_w."""
    R = np.array(R, dtype=np.float64).reshape(-1, 3)
    Rs = R.copy()
    Rs[:, 2] = 2.0 * z_w - R[:, 2]
    return Rs


def image_matrix(R, target, source, prm: galerkin.Params, z_w, rows=None):
    """Dense [len(rows)*dT, N*dX] of the image blocks B(R_n - R*_m) S_X over every m (own image
    included)."""
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    n = R.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    Rs = mirror(R, z_w)
    dT, dX = greens.TARGET_DIM[target], greens.SOURCE_DIM[source]
    dx = (R[rows, None, :] - Rs[None, :, :]).reshape(-1, 3)
    blk = greens.block(target, source, dx, prm.a, prm.eta).reshape(len(rows), n, dT, dX)
    blk = blk @ IMAGE_MAP[source]
    return blk.transpose(0, 2, 1, 3).reshape(len(rows) * dT, n * dX)


def _check(R, prm, z_w):
    h = np.asarray(R, dtype=np.float64).reshape(-1, 3)[:, 2] - z_w
    if np.any(h < prm.a):
        raise ValueError("every sphere must lie in the fluid: z - z_w >= a")


def system_matrix(R, prm: galerkin.Params, z_w):
    """A = I/gamma - K^SS - K^SS_image (the half-space system)."""
    _check(R, prm, z_w)
    return galerkin.system_matrix(R, prm) - image_matrix(R, "E", "S", prm, z_w)


def rhs(R, v2s, v3t, Fe, Te, prm: galerkin.Params, z_w):
    """b = E[F, T, d] over the other spheres and every image - c s."""
    b = galerkin.rhs(R, v2s, v3t, Fe, Te, prm)
    for kind, vals in (("F", Fe), ("T", Te), ("D", v3t)):
        if vals is not None:
            b = b + image_matrix(R, "E", kind, prm, z_w) @ np.ravel(vals)
    return b


def outputs(R, v1s, v2s, v3t, Fe, Te, Sigma, prm: galerkin.Params, z_w):
    """V, Omega, S of the half-space system from a flow stresslet Sigma."""
    V, W, S = galerkin.outputs(R, v1s, v2s, v3t, Fe, Te, Sigma, prm)
    n = len(np.asarray(R).reshape(-1, 3))
    for kind, vals in (("F", Fe), ("T", Te), ("S", Sigma), ("D", v3t)):
        if vals is not None:
            V = V + (image_matrix(R, "U", kind, prm, z_w) @ np.ravel(vals)).reshape(n, 3)
            W = W + (image_matrix(R, "W", kind, prm, z_w) @ np.ravel(vals)).reshape(n, 3)
    return V, W, S


def solve(w, z_w, prm: galerkin.Params | None = None):
    """Dense solve of the half-space system for a workload (fields R, v1s, v2s, v3t, Fe, Te)."""
    prm = prm or galerkin.Params(eta=getattr(w, "eta", 1.0 / (6 * np.pi)), a=getattr(w, "a", 1.0))
    A = system_matrix(w.R, prm, z_w)
    b = rhs(w.R, w.v2s, w.v3t, w.Fe, w.Te, prm, z_w)
    Sigma = np.linalg.solve(A, b).reshape(-1, 5)
    V, W, S = outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sigma, prm, z_w)
    return dict(V=V, W=W, S=S, Sigma=Sigma, b=b, A=A)


def flow_field(X, R, Fe, Te, Sigma, v3t, prm: galerkin.Params, z_w):
    """Flow at field points X in the fluid: the free-space flow of every sphere and of its image."""
    u = galerkin.flow_field(X, R, Fe, Te, Sigma, v3t, prm)
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    Rs = mirror(R, z_w)
    for kind, vals in (("F", Fe), ("T", Te), ("S", Sigma), ("D", v3t)):
        if vals is None:
            continue
        vals = np.asarray(vals, dtype=np.float64)
        for m in range(Rs.shape[0]):
            u += greens.flow(kind, X - Rs[m], prm.a, prm.eta) @ (IMAGE_MAP[kind] @ vals[m])
    return u


def matvec_rows(R, x, rows, prm: galerkin.Params, z_w):
    """(A x) of the half-space system restricted to the given spheres, without forming A."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 5)
    img = image_matrix(R, "E", "S", prm, z_w, rows) @ np.ravel(x)
    return galerkin.matvec_rows(R, x, rows, prm) - img.reshape(-1, 5)
