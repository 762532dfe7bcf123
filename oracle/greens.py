"""Pair blocks of the sphere Galerkin operator, by exact symbolic differentiation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything here is generated from the unbounded-fluid Green's function of
section III,  G_ij(x) = delta_ij / r + x_i x_j / r^3  (x = field point minus
source point), and the finite-size operators  F^l = 1 + a^2/(4l+6) nabla^2  of
the boundary-integral evaluation (section III, "boundary integrals as
derivatives of G"; appendix B). No closed form is typed in by hand: every block
is a derivative of G computed by sympy, with the exact identity
r^2 = x^2 + y^2 + z^2 used to put expressions in a canonical form (so that the
biharmonic identity nabla^4 G = 0 holds exactly rather than up to rounding).

Source flows at field point x relative to a sphere centre (per unit source
component; P = 1/(8 pi eta)):

* ``F`` force (l = 0, sigma = 0 row of the irreducible-flow table):
  u = P F^0 G . F^e,  F^0 = 1 + a^2/6 nabla^2.
* ``T`` torque (l = 1, sigma = 1 row): u = P (1/2) curl(G . T^e).
* ``S`` flow stresslet Sigma = a Q^(20) (l = 1, sigma = 0 row):
  u_i = P F^1 d_k G_ij Sigma_jk,  F^1 = 1 + a^2/10 nabla^2.
* ``D`` the rank-3 trace slip mode d = V^(32)/a^2 (l = 2, sigma = 2 row, a
  Laplacian of G): u = -(a^5/20) nabla^2 G . d, the exterior flow whose
  surface value is the slip mode itself (a fixed source: its traction is the
  one-body one).

The other irreducible slip modes of the minimal truncation (section IV: the
quadratic coefficient V^(3) = a^2 [gamma - (2/3) Delta.(eps.psi) + (3/5) Delta.delta d]
and the rank-3 part lambda of the cubic one, V^(4) contains -(3/4) a^3 Delta.(eps.lambda)),
contracted with the surface harmonics Y^(2) = 3nn - I and Y^(3) = 15nnn - 3(n delta)_sym
and the weights 1/6 and 1/90 of the surface expansion, give the slip fields on r = a

  septlet mode gamma (symmetric traceless rank 3):  v = (a^2/2) gamma : n n
  vortlet mode psi   (symmetric traceless rank 2):  v = -(a^2/3) n x (psi . n)
  spinlet mode lambda (symmetric traceless rank 3): v = -(a^3/8) n x (lambda : n n)

Each is a fixed source (its traction is the one-body one, as for d). The flows
below are the decaying Stokes flows that take these values on the sphere:

* ``SEPT``: u_i = (7 a^5/48) F^2 [d_j d_k G_il] gamma_ljk, F^2 = 1 + a^2/14 nabla^2
  (the sigma = 0, l = 2 row of the irreducible-flow table with its finite-size
  operator; the amplitude makes the surface value equal the slip);
* ``VORT``: u = -(a^5/3) x x (psi . x) / r^5 (a degree-2 rotational flow);
* ``SPIN``: u = -(a^7/8) x x (lambda : x x) / r^7 (a degree-3 rotational flow).

Rank-3 coefficients enter through 10 symmetric components (order of
``basis.SYM3``), projected on their traceless part; psi uses the 5-basis.

Target projections at the centre of the receiving sphere (the Galerkin
coefficients of an incident flow, section III; Faxen form):

* ``U`` = F^0 u                      (l = 0 coefficient, a velocity)
* ``W`` = (1/2) curl u              (antisymmetric l = 1 coefficient)
* ``E`` = sym grad (F^1 u), 5-basis  (symmetric l = 1 coefficient / a)

A block B_TX(x) is the [dim T x dim X] matrix mapping the source coefficients
of sphere m to the projection at sphere n, x = R_n - R_m.
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as sp

from . import basis

x_, y_, z_, r_, a_, P_ = sp.symbols("x y z r a P", positive=True)
_X = (x_, y_, z_)

SOURCE_DIM = {"F": 3, "T": 3, "S": 5, "D": 3, "SEPT": 10, "VORT": 5, "SPIN": 10, "SEPT7": 7}
TARGET_DIM = {"U": 3, "W": 3, "E": 5, "GAM": 7, "PSI": 5, "DD": 3}


def _canon(f):
    """Expand and eliminate x^2 = r^2 - y^2 - z^2 (canonical representative)."""
    f = sp.expand(f)
    f = f.replace(lambda e: e.is_Pow and e.base == x_ and e.exp.is_Integer and e.exp >= 2,
                  lambda e: x_ ** (int(e.exp) % 2) * (r_ ** 2 - y_ ** 2 - z_ ** 2) ** (int(e.exp) // 2))
    return sp.expand(f)


def d(f, i):
    """Partial derivative along x_i, with r treated through dr/dx_i = x_i / r."""
    return _canon(sp.diff(f, _X[i]) + _X[i] / r_ * sp.diff(f, r_))


def lap(f):
    return _canon(sum(d(d(f, i), i) for i in range(3)))


def faxen(f, l):
    """Finite-size operator F^l = 1 + a^2/(4l+6) nabla^2 (section III)."""
    return _canon(f + a_ ** 2 / (4 * l + 6) * lap(f))


def curl(u):
    return [_canon(d(u[2], 1) - d(u[1], 2)), _canon(d(u[0], 2) - d(u[2], 0)),
            _canon(d(u[1], 0) - d(u[0], 1))]


_IDX3 = [(i, j, k) for i in range(3) for j in range(3) for k in range(3)]


def _cross(p, q):
    return [p[1] * q[2] - p[2] * q[1], p[2] * q[0] - p[0] * q[2], p[0] * q[1] - p[1] * q[0]]


def _stf3_unit(q):
    """Symmetric traceless part of the unit symmetric rank-3 tensor of component q (exact)."""
    T = [[[sp.Integer(0)] * 3 for _ in range(3)] for _ in range(3)]
    for i, j, k in _IDX3:
        if tuple(sorted((i, j, k))) == basis.SYM3[q]:
            T[i][j][k] = sp.Integer(1)
    t = [sum(T[i][i][k] for i in range(3)) for k in range(3)]
    return [[[T[i][j][k] - sp.Rational(1, 5) * (int(i == j) * t[k] + int(i == k) * t[j] + int(j == k) * t[i])
              for k in range(3)] for j in range(3)] for i in range(3)]


@functools.lru_cache(maxsize=None)
def oseen():
    """G_ij = delta_ij/r + x_i x_j/r^3 (section III, unbounded fluid)."""
    return tuple(tuple(sp.Integer(int(i == j)) / r_ + _X[i] * _X[j] / r_ ** 3 for j in range(3))
                 for i in range(3))


@functools.lru_cache(maxsize=None)
def source_flow(kind):
    """Columns of the source flow: tuple over source components of (u_x, u_y, u_z)."""
    G = oseen()
    cols = []
    if kind == "F":
        for j in range(3):
            cols.append([P_ * faxen(G[i][j], 0) for i in range(3)])
    elif kind == "T":
        for j in range(3):
            cols.append([P_ * sp.Rational(1, 2) * c for c in curl([G[i][j] for i in range(3)])])
    elif kind == "S":
        for c in range(5):
            B = basis.BASIS[c]
            u = []
            for i in range(3):
                acc = 0
                for j in range(3):
                    for k in range(3):
                        if B[j, k] != 0.0:
                            acc += d(G[i][j], k) * sp.nsimplify(B[j, k], [sp.sqrt(2), sp.sqrt(6)])
                u.append(P_ * faxen(acc, 1))
            cols.append(u)
    elif kind == "D":
        for j in range(3):
            cols.append([-a_ ** 5 / 20 * lap(G[i][j]) for i in range(3)])
    elif kind == "SEPT":
        for q in range(10):
            T = _stf3_unit(q)
            u = []
            for i in range(3):
                acc = 0
                for l, j, k in _IDX3:
                    if T[l][j][k] != 0:
                        acc += T[l][j][k] * d(d(G[i][l], j), k)
                u.append(sp.Rational(7, 48) * a_ ** 5 * faxen(acc, 2))
            cols.append(u)
    elif kind == "SEPT7":  # the septlet flow per unit coordinate of the 7-basis (basis.BASIS3)
        for T in basis.BASIS3_EXACT:
            u = []
            for i in range(3):
                acc = 0
                for l, j, k in _IDX3:
                    if T[l][j][k] != 0:
                        acc += T[l][j][k] * d(d(G[i][l], j), k)
                u.append(sp.Rational(7, 48) * a_ ** 5 * faxen(acc, 2))
            cols.append(u)
    elif kind == "VORT":
        for c in range(5):
            B = [[sp.nsimplify(basis.BASIS[c][i, j], [sp.sqrt(2), sp.sqrt(6)]) for j in range(3)] for i in range(3)]
            w = [sum(B[i][j] * _X[j] for j in range(3)) for i in range(3)]
            cols.append([-a_ ** 5 / 3 * e / r_ ** 5 for e in _cross(_X, w)])
    elif kind == "SPIN":
        for q in range(10):
            T = _stf3_unit(q)
            v = [sum(T[i][j][k] * _X[j] * _X[k] for j in range(3) for k in range(3)) for i in range(3)]
            cols.append([-a_ ** 7 / 8 * e / r_ ** 7 for e in _cross(_X, v)])
    else:
        raise ValueError(kind)
    return tuple(tuple(_canon(e) for e in col) for col in cols)


def _quadratic_coefficient(u):
    """V^(3) / a^2 of an incident flow: the l = 2 surface coefficient (5/(4 pi a^2)) int u_i Y^(2)_jk dS
    (section III), which for a biharmonic flow is a^2 times the part of F^2 d_j d_k u_i at the
    centre that is symmetric and traceless in (j, k)."""
    v = [faxen(ui, 2) for ui in u]
    H = [[[d(d(v[i], j), k) for k in range(3)] for j in range(3)] for i in range(3)]
    S = [[[None] * 3 for _ in range(3)] for _ in range(3)]
    for i in range(3):
        tr = H[i][0][0] + H[i][1][1] + H[i][2][2]
        for j in range(3):
            for k in range(3):
                S[i][j][k] = _canon(sp.Rational(1, 2) * (H[i][j][k] + H[i][k][j]) - int(j == k) * tr / 3)
    return S


def _target(kind, u):
    if kind in ("GAM", "PSI", "DD"):
        # irreducible parts of V^(3) = a^2 [gamma - (2/3) Delta.(eps.psi) + (3/5) Delta.delta d]
        # (section IV, minimal truncation): gamma its symmetric traceless part, d its contraction of
        # the velocity index with the first harmonic index, psi minus its symmetric contraction with
        # eps over those two indices; gamma in the 7-basis, psi in the 5-basis
        S = _quadratic_coefficient(u)
        if kind == "GAM":
            return [_canon(sum(B[i][j][k] * S[i][j][k] for i, j, k in _IDX3 if B[i][j][k] != 0))
                    for B in basis.BASIS3_EXACT]
        if kind == "DD":
            return [_canon(S[0][0][k] + S[1][1][k] + S[2][2][k]) for k in range(3)]
        eps = lambda p, q, s: sp.LeviCivita(p, q, s)  # noqa: E731
        C = [[-sum(eps(l, i, j) * S[i][j][k] for i in range(3) for j in range(3)) for k in range(3)]
             for l in range(3)]
        out = []
        for c in range(5):
            B = basis.BASIS[c]
            out.append(_canon(sum(sp.nsimplify(B[l, k], [sp.sqrt(2), sp.sqrt(6)]) * C[l][k]
                                  for l in range(3) for k in range(3) if B[l, k] != 0.0)))
        return out
    if kind == "U":
        return [faxen(ui, 0) for ui in u]
    if kind == "W":
        return [sp.Rational(1, 2) * c for c in curl(u)]
    if kind == "E":
        v = [faxen(ui, 1) for ui in u]
        M = [[sp.Rational(1, 2) * (d(v[i], j) + d(v[j], i)) for j in range(3)] for i in range(3)]
        out = []
        for c in range(5):
            B = basis.BASIS[c]
            acc = 0
            for i in range(3):
                for j in range(3):
                    if B[i, j] != 0.0:
                        acc += M[i][j] * sp.nsimplify(B[i, j], [sp.sqrt(2), sp.sqrt(6)])
            out.append(_canon(acc))
        return out
    raise ValueError(kind)


@functools.lru_cache(maxsize=None)
def block_expr(target, source):
    """sympy Matrix [dim target x dim source] of the block B_{target,source}(x)."""
    cols = source_flow(source)
    mat = [[None] * len(cols) for _ in range(TARGET_DIM[target])]
    for q, u in enumerate(cols):
        t = _target(target, list(u))
        for p_ in range(TARGET_DIM[target]):
            mat[p_][q] = _canon(t[p_])
    return sp.Matrix(mat)


@functools.lru_cache(maxsize=None)
def _block_fn(target, source):
    return sp.lambdify((x_, y_, z_, r_, a_, P_), block_expr(target, source).tolist(), "numpy", cse=True)


def block(target, source, dx, a, eta):
    """Numerical blocks for separations dx [npairs, 3] -> [npairs, dim T, dim X].

    dx = R_n - R_m (receiver minus source); every row must be non-zero.
    """
    dx = np.asarray(dx, dtype=np.float64).reshape(-1, 3)
    r = np.sqrt(np.einsum("pi,pi->p", dx, dx))
    P = 1.0 / (8.0 * np.pi * eta)
    raw = _block_fn(target, source)(dx[:, 0], dx[:, 1], dx[:, 2], r, float(a), P)
    dt, ds = TARGET_DIM[target], SOURCE_DIM[source]
    out = np.empty((dx.shape[0], dt, ds))
    for i in range(dt):
        for j in range(ds):
            out[:, i, j] = np.broadcast_to(np.asarray(raw[i][j], dtype=np.float64), (dx.shape[0],))
    return out


@functools.lru_cache(maxsize=None)
def _flow_fn(source):
    cols = source_flow(source)
    mat = [[cols[q][i] for q in range(len(cols))] for i in range(3)]
    return sp.lambdify((x_, y_, z_, r_, a_, P_), mat, "numpy", cse=True)


def flow(source, dx, a, eta):
    """Source flow per unit component at field points dx [npts, 3] -> [npts, 3, dim X]."""
    dx = np.asarray(dx, dtype=np.float64).reshape(-1, 3)
    r = np.sqrt(np.einsum("pi,pi->p", dx, dx))
    P = 1.0 / (8.0 * np.pi * eta)
    raw = _flow_fn(source)(dx[:, 0], dx[:, 1], dx[:, 2], r, float(a), P)
    ds = SOURCE_DIM[source]
    out = np.empty((dx.shape[0], 3, ds))
    for i in range(3):
        for j in range(ds):
            out[:, i, j] = np.broadcast_to(np.asarray(raw[i][j], dtype=np.float64), (dx.shape[0],))
    return out
