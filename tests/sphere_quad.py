"""Product quadrature on a sphere: Gauss-Legendre in cos(theta) x trapezoid in phi.

Exact for spherical harmonics of degree < min(2 * n_theta, n_phi); used by the
tests to evaluate the Galerkin coefficients of a flow by their surface-integral
definitions (section III) instead of by the Faxen operators.
"""
import numpy as np


def sphere_rule(n_theta=40, n_phi=80):
    mu, wmu = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1 - mu ** 2)
    nhat = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)),
                     np.outer(mu, np.ones_like(phi))], axis=-1).reshape(-1, 3)
    w = np.outer(wmu, np.full(n_phi, 2 * np.pi / n_phi)).reshape(-1)
    return nhat, w  # sum(w) = 4 pi


def coefficients(u, nhat, w, a):
    """Galerkin coefficients of a surface field u [npts, 3] on a sphere of radius a.

    Returns (mean, V2) with mean = <u> (the l = 0 coefficient) and
    V2_ij = 3/(4 pi a^2) int u_i n_j dS (the rank-2 coefficient, l = 1).
    """
    mean = (w[:, None] * u).sum(0) / (4 * np.pi)
    V2 = 3.0 / (4 * np.pi) * np.einsum("p,pi,pj->ij", w, u, nhat)
    return mean, V2


def axial(V2, a):
    """Rotation carried by the antisymmetric part: -1/(2a) eps_mij V2_ij."""
    A = V2 / a
    return -0.5 * np.array([A[1, 2] - A[2, 1], A[2, 0] - A[0, 2], A[0, 1] - A[1, 0]])


def quadratic_coefficient(u, nhat, w):
    """V3_ijk = 5/(4 pi a^2) int u_i Y^(2)_jk dS with Y^(2) = 3 n n - I (the l = 2 coefficient)."""
    Y2 = 3.0 * nhat[:, :, None] * nhat[:, None, :] - np.eye(3)
    return 5.0 / (4 * np.pi) * np.einsum("p,pi,pjk->ijk", w, u, Y2)


def quadratic_parts(V3, a):
    """Irreducible parts of V^(3) = a^2 [gamma - (2/3) Delta.(eps.psi) + (3/5) Delta.delta d]:
    gamma (the fully symmetric traceless part / a^2), psi (minus the symmetric contraction of eps
    with the velocity index and the first harmonic index / a^2) and d (the trace over those two
    indices / a^2), computed here from their definitions."""
    import itertools
    S = sum(np.transpose(V3, p) for p in itertools.permutations(range(3))) / 6.0
    t = np.einsum("iik->k", S)
    d = np.eye(3)
    gam = S - (np.einsum("ij,k->ijk", d, t) + np.einsum("ik,j->ijk", d, t) + np.einsum("jk,i->ijk", d, t)) / 5.0
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    C = -np.einsum("lij,ijk->lk", eps, V3)
    psi = 0.5 * (C + C.T) - np.trace(C) / 3.0 * np.eye(3)
    dv = np.einsum("iik->k", V3)
    return gam / a ** 2, psi / a ** 2, dv / a ** 2
