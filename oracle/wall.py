"""Spheres in the half space z > z_w bounded by a plane no-slip wall (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper notes (Discussion) that the method carries over to any geometry whose Green's function
is known, plane walls among them. At a no-slip wall the Green's function is Blake's: the free-space
Oseen tensor G(x - y) plus an image part H(x, y) that depends on the field point x and the source
point y separately, not on x - y alone. With the wall at z = 0, h = y_3 the source's height, its
mirror point y* = (y_1, y_2, -h), R = x - y* and M = diag(1, 1, -1),

    H_ij(x, y) = -G_ij(R) + 2 h M_jk d/dR_k [ h R_i / |R|^3 - (delta_i3 / |R| + R_i R_3 / |R|^3) ]

(a Stokeslet, a Stokes doublet and a source doublet at the mirror point; Blake, Proc. Camb. Phil.
Soc. 70, 303 (1971)), so that G + H vanishes for x on the wall.

The Galerkin blocks of the free-space operator are derivatives of G(x - R_m) in the field point
(module ``greens``). With a kernel K(x, y) that is not a function of x - y alone, the source side
of each block is written as the same surface moment of the traction taken against K in its source
argument: a Taylor expansion of K(x, y) about the centre y = R_m of the source sphere, integrated
against the traction's surface harmonics, gives the finite-size operators F^l in y (K is
biharmonic and divergence free in y by reciprocity, K_ij(x, y) = K_ji(y, x)), and the free-space
forms follow from d/dy = -d/dx for K = G(x - y):

    F  (force):        u_i = P F^0_y K_ij F_j
    T  (torque):       u_i = P (1/2) eps_klj T_k F^1_y dK_ij/dy_l
    S  (stresslet):    u_i = -P F^1_y dK_ij/dy_k Sigma_jk
    D  (rank-3 trace): u_i = -(a^5/20) lap_y K_ij d_j

and the receiver's projections are those of the free-space blocks (F^0 u, (1/2) curl u,
sym grad F^1 u, at the receiver's centre). Applied to K = G(x - y) this reproduces the free-space
blocks (a pin); applied to K = H it gives the image blocks, functions of R = R_n - R*_m and
h = z_m - z_w, for every pair (n, m) including n = m (the sphere's own image).

Symbols: R = (R1, R2, R3) is the field point minus the source's mirror point (for K = G(x - y): the
field point minus the source point), rr = |R|, h the source's height above the wall.
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as sp

from . import basis, galerkin

R1, R2, R3 = sp.symbols("R1 R2 R3", real=True)
h_, rr_, a_, P_ = sp.symbols("h rr a P", positive=True)
_R = (R1, R2, R3)
_M = (1, 1, -1)

SOURCE_DIM = {"F": 3, "T": 3, "S": 5, "D": 3}
TARGET_DIM = {"U": 3, "W": 3, "E": 5}


def _canon(f):
    """Expand and eliminate R1^2 = rr^2 - R2^2 - R3^2 (canonical representative)."""
    f = sp.expand(f)
    f = f.replace(lambda e: e.is_Pow and e.base == R1 and e.exp.is_Integer and e.exp >= 2,
                  lambda e: R1 ** (int(e.exp) % 2) * (rr_ ** 2 - R2 ** 2 - R3 ** 2) ** (int(e.exp) // 2))
    return sp.expand(f)


def _dR(f, i):
    """d/dR_i with rr treated through d rr/dR_i = R_i / rr."""
    return _canon(sp.diff(f, _R[i]) + _R[i] / rr_ * sp.diff(f, rr_))


# derivative rules of the two kernels: in the field point x, R moves with x in both; in the source
# point y, R = x - y moves against y for the free kernel, while R = x - y* moves against y along
# the wall and with it across the wall, and the image part also depends on y through h = y_3
def _dx(kernel, f, i):
    return _dR(f, i)


def _dy(kernel, f, i):
    if kernel == "free" or i < 2:
        return _canon(-_dR(f, i))
    return _canon(_dR(f, 2) + sp.diff(f, h_))


def _lap(kernel, f, side):
    dd = _dx if side == "x" else _dy
    return _canon(sum(dd(kernel, dd(kernel, f, i), i) for i in range(3)))


def _faxen(kernel, f, l, side):
    return _canon(f + a_ ** 2 / (4 * l + 6) * _lap(kernel, f, side))


@functools.lru_cache(maxsize=None)
def kernel_expr(kernel):
    """3 x 3 nested tuple K_ij: 'free' the Oseen tensor of R = x - y, 'wall' Blake's image part of
    R = x - y* and the source height h (wall at z = 0)."""
    d = lambda i, j: sp.Integer(int(i == j))  # noqa: E731
    G = [[d(i, j) / rr_ + _R[i] * _R[j] / rr_ ** 3 for j in range(3)] for i in range(3)]
    if kernel == "free":
        return tuple(tuple(_canon(G[i][j]) for j in range(3)) for i in range(3))
    if kernel != "wall":
        raise ValueError(kernel)
    phi = [h_ * _R[i] / rr_ ** 3 - d(i, 2) / rr_ - _R[i] * _R[2] / rr_ ** 3 for i in range(3)]
    return tuple(tuple(_canon(-G[i][j] + 2 * h_ * _M[j] * _dR(phi[i], j)) for j in range(3)) for i in range(3))


def _sym5(c):
    return [[sp.nsimplify(basis.BASIS[c][j, k], [sp.sqrt(2), sp.sqrt(6)]) for k in range(3)] for j in range(3)]


@functools.lru_cache(maxsize=None)
def source_flow(kernel, kind):
    """Columns of the source flow of one sphere through kernel K: tuple over source components of
    (u_x, u_y, u_z), functions of R, rr, h, a, P."""
    K = kernel_expr(kernel)
    cols = []
    if kind == "F":
        for j in range(3):
            cols.append([P_ * _faxen(kernel, K[i][j], 0, "y") for i in range(3)])
    elif kind == "T":
        for k in range(3):
            u = []
            for i in range(3):
                acc = 0
                for l in range(3):
                    for j in range(3):
                        e = sp.LeviCivita(k, l, j)
                        if e != 0:
                            acc += e * _dy(kernel, K[i][j], l)
                u.append(P_ * sp.Rational(1, 2) * _faxen(kernel, acc, 1, "y"))
            cols.append(u)
    elif kind == "S":
        for c in range(5):
            B = _sym5(c)
            u = []
            for i in range(3):
                acc = 0
                for j in range(3):
                    for k in range(3):
                        if B[j][k] != 0:
                            acc += _dy(kernel, K[i][j], k) * B[j][k]
                u.append(-P_ * _faxen(kernel, acc, 1, "y"))
            cols.append(u)
    elif kind == "D":
        for j in range(3):
            cols.append([-a_ ** 5 / 20 * _lap(kernel, K[i][j], "y") for i in range(3)])
    else:
        raise ValueError(kind)
    return tuple(tuple(_canon(e) for e in col) for col in cols)


def _target(kernel, kind, u):
    if kind == "U":
        return [_faxen(kernel, ui, 0, "x") for ui in u]
    if kind == "W":
        dx = lambda f, i: _dx(kernel, f, i)  # noqa: E731
        return [sp.Rational(1, 2) * _canon(dx(u[(i + 2) % 3], (i + 1) % 3) - dx(u[(i + 1) % 3], (i + 2) % 3))
                for i in range(3)]
    if kind == "E":
        v = [_faxen(kernel, ui, 1, "x") for ui in u]
        out = []
        for c in range(5):
            B = _sym5(c)
            acc = 0
            for i in range(3):
                for j in range(3):
                    if B[i][j] != 0:
                        acc += sp.Rational(1, 2) * (_dx(kernel, v[i], j) + _dx(kernel, v[j], i)) * B[i][j]
            out.append(_canon(acc))
        return out
    raise ValueError(kind)


@functools.lru_cache(maxsize=None)
def block_expr(kernel, target, source):
    """sympy Matrix [dim target x dim source] of the block through kernel K."""
    cols = source_flow(kernel, source)
    mat = [[None] * len(cols) for _ in range(TARGET_DIM[target])]
    for q, u in enumerate(cols):
        t = _target(kernel, target, list(u))
        for p in range(TARGET_DIM[target]):
            mat[p][q] = _canon(t[p])
    return sp.Matrix(mat)


@functools.lru_cache(maxsize=None)
def _block_fn(kernel, target, source):
    return sp.lambdify((R1, R2, R3, rr_, h_, a_, P_), block_expr(kernel, target, source).tolist(), "numpy",
                       cse=True)


@functools.lru_cache(maxsize=None)
def _flow_fn(kernel, source):
    cols = source_flow(kernel, source)
    mat = [[cols[q][i] for q in range(len(cols))] for i in range(3)]
    return sp.lambdify((R1, R2, R3, rr_, h_, a_, P_), mat, "numpy", cse=True)


def _eval(fn, R, h, a, eta, dt, ds):
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), (R.shape[0],))
    rr = np.sqrt(np.einsum("pi,pi->p", R, R))
    raw = fn(R[:, 0], R[:, 1], R[:, 2], rr, h, float(a), 1.0 / (8.0 * np.pi * eta))
    out = np.empty((R.shape[0], dt, ds))
    for i in range(dt):
        for j in range(ds):
            out[:, i, j] = np.broadcast_to(np.asarray(raw[i][j], dtype=np.float64), (R.shape[0],))
    return out


def block(kernel, target, source, R, h, a, eta):
    """Numerical blocks [npairs, dim T, dim X]: kernel 'free' at separations R = x - y (h unused),
    'wall' (image part) at R = x - y* and source heights h above the wall."""
    return _eval(_block_fn(kernel, target, source), R, h, a, eta, TARGET_DIM[target], SOURCE_DIM[source])


def flow(kernel, source, R, h, a, eta):
    """Source flow per unit component at field points, [npts, 3, dim X] (arguments as in block)."""
    return _eval(_flow_fn(kernel, source), R, h, a, eta, 3, SOURCE_DIM[source])


# ------------------------------------------------------------------ the half-space system
def mirror(R, z_w):
    """Mirror points of the centres in the wall z = z_w."""
    R = np.array(R, dtype=np.float64).reshape(-1, 3)
    Rs = R.copy()
    Rs[:, 2] = 2.0 * z_w - R[:, 2]
    return Rs


def image_matrix(R, target, source, prm: galerkin.Params, z_w, rows=None):
    """Dense [len(rows)*dT, N*dX] of the image blocks of every source m (own image included) at the
    receivers `rows`."""
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    n = R.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    Rs = mirror(R, z_w)
    dT, dX = TARGET_DIM[target], SOURCE_DIM[source]
    sep = (R[rows, None, :] - Rs[None, :, :]).reshape(-1, 3)
    hh = np.broadcast_to(R[None, :, 2] - z_w, (len(rows), n)).reshape(-1)
    blk = block("wall", target, source, sep, hh, prm.a, prm.eta).reshape(len(rows), n, dT, dX)
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
    """Flow at field points X in the fluid: the free-space flow of every sphere plus its image part."""
    u = galerkin.flow_field(X, R, Fe, Te, Sigma, v3t, prm)
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    Rs = mirror(R, z_w)
    for kind, vals in (("F", Fe), ("T", Te), ("S", Sigma), ("D", v3t)):
        if vals is None:
            continue
        vals = np.asarray(vals, dtype=np.float64)
        for m in range(R.shape[0]):
            u += flow("wall", kind, X - Rs[m], R[m, 2] - z_w, prm.a, prm.eta) @ vals[m]
    return u


def matvec_rows(R, x, rows, prm: galerkin.Params, z_w):
    """(A x) of the half-space system restricted to the given spheres, without forming A."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 5)
    img = image_matrix(R, "E", "S", prm, z_w, rows) @ np.ravel(x)
    return galerkin.matvec_rows(R, x, rows, prm) - img.reshape(-1, 5)
