"""Spheres in a periodic cubic box of side L (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper notes (Discussion) that periodic domains follow from the periodic Green's function, and
that the periodic sum of the flows converges only conditionally, so a limiting procedure is
needed. The procedure taken here is Hasimoto's: the fluid's mean velocity over the box is zero (the
k = 0 Fourier mode is left out; a net force on the spheres is balanced by a mean pressure gradient),
and the periodic Oseen tensor is split with a parameter xi into a screened real-space part, summed
over the periodic images within a cutoff, and a smooth Fourier part, summed over the reciprocal
lattice k = 2 pi n / L, n != 0:

    G_per(x) = sum_n G^R(x + n L) + (1/L^3) sum_{k != 0} G^(k) e^{i k.x},
    G^R_ij(r) = (erfc(xi r)/r - (2 xi/sqrt(pi)) e^{-xi^2 r^2}) delta_ij
              + (erfc(xi r)/r + (2 xi/sqrt(pi)) e^{-xi^2 r^2}) x_i x_j / r^2,
    G^(k) = (8 pi / k^2) (I - k k / k^2) phi(k),   phi(k) = (1 + k^2/(4 xi^2)) e^{-k^2/(4 xi^2)}.

The periodic tensor is biharmonic away from the lattice points, so each Galerkin block is the
free-space operator chain (module ``greens``: finite-size operators F^l, derivatives, curl) applied
to G_per, i.e. to each part: in real space by symbolic differentiation of G^R, in Fourier space as
the multiplier of the chain (d/dx -> i k, lap -> -k^2) times G^(k). The block of a sphere with its
own periodic images is the limit x -> 0 of the block of G_per - G, i.e. the images' real-space part,
plus the Fourier sum at x = 0, minus the smooth part of the sphere's own flow at its centre,
(1/(2 pi)^3) integral of the multiplier over all k (that last integral by exact quadrature: Gauss
rules in the polar angle and the radius, the trapezoid rule in the azimuth).
"""
from __future__ import annotations

import functools
import math

import numpy as np
import sympy as sp

from . import basis, galerkin, greens

x_, y_, z_, r_, a_, P_ = greens.x_, greens.y_, greens.z_, greens.r_, greens.a_, greens.P_
xi_ = sp.symbols("xi", positive=True)
# erfc(xi r) and exp(-xi^2 r^2) as symbols of their own, differentiated through r by the chain rule
ec_, ex_ = sp.symbols("ec ex", positive=True)
kx_, ky_, kz_ = sp.symbols("kx ky kz", real=True)
_X, _K = (x_, y_, z_), (kx_, ky_, kz_)

SOURCE_DIM = {"F": 3, "T": 3, "S": 5, "D": 3}
TARGET_DIM = {"U": 3, "W": 3, "E": 5}


# ------------------------------------------------------------------ the operator chain, generic
class _Rules:
    """Derivative rules of one representation: real space (functions of x, y, z, r) or Fourier
    space (functions of kx, ky, kz: d/dx_i -> i k_i, lap -> -k^2)."""

    def __init__(self, fourier):
        self.fourier = fourier

    def d(self, f, i):
        if self.fourier:
            return sp.I * _K[i] * f
        # d/dx_i through x_i itself and through r (dr/dx_i = x_i / r), with
        # d erfc(xi r)/dr = -(2 xi/sqrt(pi)) exp(-xi^2 r^2) and d exp(-xi^2 r^2)/dr = -2 xi^2 r exp(-xi^2 r^2)
        dr = sp.diff(f, r_) - 2 * xi_ / sp.sqrt(sp.pi) * ex_ * sp.diff(f, ec_) - 2 * xi_ ** 2 * r_ * ex_ * sp.diff(f, ex_)
        return greens._canon(sp.diff(f, _X[i]) + _X[i] / r_ * dr)

    def lap(self, f):
        if self.fourier:
            return -(kx_ ** 2 + ky_ ** 2 + kz_ ** 2) * f
        return greens._canon(sum(self.d(self.d(f, i), i) for i in range(3)))

    def faxen(self, f, l):
        return f + a_ ** 2 / (4 * l + 6) * self.lap(f)

    def canon(self, f):
        return sp.expand(f) if self.fourier else greens._canon(f)


def _sym5(c):
    return [[sp.nsimplify(basis.BASIS[c][j, k], [sp.sqrt(2), sp.sqrt(6)]) for k in range(3)] for j in range(3)]


def _flows(K, kind, ru):
    """Columns of the source flow of kernel K (3 x 3 nested) under rules ru (the free-space
    definitions of module greens, written for any representation)."""
    cols = []
    if kind == "F":
        for j in range(3):
            cols.append([P_ * ru.faxen(K[i][j], 0) for i in range(3)])
    elif kind == "T":
        for j in range(3):
            col = [K[i][j] for i in range(3)]
            curl = [ru.d(col[2], 1) - ru.d(col[1], 2), ru.d(col[0], 2) - ru.d(col[2], 0),
                    ru.d(col[1], 0) - ru.d(col[0], 1)]
            cols.append([P_ * sp.Rational(1, 2) * c for c in curl])
    elif kind == "S":
        for c in range(5):
            B = _sym5(c)
            u = []
            for i in range(3):
                acc = 0
                for j in range(3):
                    for k in range(3):
                        if B[j][k] != 0:
                            acc += ru.d(K[i][j], k) * B[j][k]
                u.append(P_ * ru.faxen(acc, 1))
            cols.append(u)
    elif kind == "D":
        for j in range(3):
            cols.append([-a_ ** 5 / 20 * ru.lap(K[i][j]) for i in range(3)])
    else:
        raise ValueError(kind)
    return [[ru.canon(e) for e in col] for col in cols]


def _target(kind, u, ru):
    if kind == "U":
        return [ru.faxen(ui, 0) for ui in u]
    if kind == "W":
        return [sp.Rational(1, 2) * (ru.d(u[(i + 2) % 3], (i + 1) % 3) - ru.d(u[(i + 1) % 3], (i + 2) % 3))
                for i in range(3)]
    if kind == "E":
        v = [ru.faxen(ui, 1) for ui in u]
        out = []
        for c in range(5):
            B = _sym5(c)
            acc = 0
            for i in range(3):
                for j in range(3):
                    if B[i][j] != 0:
                        acc += sp.Rational(1, 2) * (ru.d(v[i], j) + ru.d(v[j], i)) * B[i][j]
            out.append(acc)
        return out
    raise ValueError(kind)


def _block(K, target, source, ru):
    cols = _flows(K, source, ru)
    mat = [[None] * len(cols) for _ in range(TARGET_DIM[target])]
    for q, u in enumerate(cols):
        t = _target(target, u, ru)
        for p in range(TARGET_DIM[target]):
            mat[p][q] = ru.canon(t[p])
    return sp.Matrix(mat)


# ------------------------------------------------------------------ the three kernels
@functools.lru_cache(maxsize=None)
def kernel(which):
    """'free': G; 'real': the screened G^R (functions of x, y, z, r, xi); 'fourier': G^(k)
    (functions of kx, ky, kz, xi)."""
    kd = lambda i, j: sp.Integer(int(i == j))  # noqa: E731
    if which == "free":
        return greens.oseen()
    if which == "real":  # in the symbols ec = erfc(xi r), ex = exp(-xi^2 r^2)
        A = ec_ / r_ - 2 * xi_ / sp.sqrt(sp.pi) * ex_
        B = ec_ / r_ + 2 * xi_ / sp.sqrt(sp.pi) * ex_
        return tuple(tuple(A * kd(i, j) + B * _X[i] * _X[j] / r_ ** 2 for j in range(3)) for i in range(3))
    if which == "fourier":  # without the splitting factor phi(k), a scalar applied on evaluation
        k2 = kx_ ** 2 + ky_ ** 2 + kz_ ** 2
        return tuple(tuple(8 * sp.pi / k2 * (kd(i, j) - _K[i] * _K[j] / k2) for j in range(3)) for i in range(3))
    raise ValueError(which)


@functools.lru_cache(maxsize=None)
def block_expr(which, target, source):
    return _block(kernel(which), target, source, _Rules(which == "fourier"))


@functools.lru_cache(maxsize=None)
def _fn(which, target, source):
    args = (kx_, ky_, kz_, xi_, a_, P_) if which == "fourier" else (x_, y_, z_, r_, ec_, ex_, xi_, a_, P_)
    return sp.lambdify(args, block_expr(which, target, source).tolist(), "numpy", cse=True)


def _eval(fn, cols, dt, ds, npts):
    out = np.empty((npts, dt, ds), dtype=complex)
    for i in range(dt):
        for j in range(ds):
            out[:, i, j] = np.broadcast_to(np.asarray(cols[i][j], dtype=complex), (npts,))
    return out


def real_block(target, source, dx, xi, a, eta):
    """Screened real-space blocks at separations dx [npts, 3] (non-zero)."""
    dx = np.asarray(dx, dtype=np.float64).reshape(-1, 3)
    from scipy.special import erfc
    r = np.sqrt(np.einsum("pi,pi->p", dx, dx))
    raw = _fn("real", target, source)(dx[:, 0], dx[:, 1], dx[:, 2], r, erfc(xi * r), np.exp(-(xi * r) ** 2),
                                      xi, a, 1.0 / (8 * np.pi * eta))
    return _eval(None, raw, TARGET_DIM[target], SOURCE_DIM[source], dx.shape[0]).real


def fourier_block(target, source, k, xi, a, eta):
    """Fourier multipliers of the blocks at wave vectors k [nk, 3] (non-zero), complex: the
    operator chain's multiplier times G^(k) (the splitting factor phi(k) applied here)."""
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    raw = _fn("fourier", target, source)(k[:, 0], k[:, 1], k[:, 2], xi, a, 1.0 / (8 * np.pi * eta))
    q = np.einsum("pi,pi->p", k, k) / (4.0 * xi * xi)
    return _eval(None, raw, TARGET_DIM[target], SOURCE_DIM[source], k.shape[0]) * ((1.0 + q) * np.exp(-q))[:, None, None]


# ------------------------------------------------------------------ Ewald parameters and lattices
class Ewald:
    """Splitting xi, real-space cutoff rc and Fourier cutoff kmax for a box of side L: xi rc = 7 and
    kmax = 14 xi (the real-space tails fall as exp(-49) times powers of xi r, the Fourier tails as
    exp(-49) times powers of k / xi)."""

    def __init__(self, L, xi=None, rc=None, kmax=None):
        self.L = float(L)
        self.xi = float(xi) if xi is not None else 10.0 / self.L
        self.rc = float(rc) if rc is not None else 7.0 / self.xi
        self.kmax = float(kmax) if kmax is not None else 14.0 * self.xi

    def images(self):
        """Lattice vectors n L that can bring a wrapped separation (each component within L/2)
        within rc."""
        m = int(math.ceil(self.rc / self.L + math.sqrt(3) / 2))
        g = np.arange(-m, m + 1)
        n = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
        return n * self.L

    def kvecs(self):
        """Reciprocal lattice vectors 0 < |k| <= kmax."""
        m = int(math.floor(self.kmax * self.L / (2 * np.pi)))
        g = np.arange(-m, m + 1)
        n = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
        k = n * (2 * np.pi / self.L)
        k2 = np.einsum("pi,pi->p", k, k)
        return k[(k2 > 0) & (k2 <= self.kmax ** 2)]


def _wrap(dx, L):
    return dx - L * np.round(dx / L)


@functools.lru_cache(maxsize=None)
def _smooth_self(target, source, xi, a, eta):
    """(1/(2 pi)^3) integral over all k of the Fourier multiplier: the smooth part of a sphere's own
    flow, projected at its own centre. The integrand is a polynomial of degree at most 6 in the
    direction of k (times k^2 G^(k), a polynomial in k times a Gaussian), so Gauss-Legendre in
    cos(theta) with 8 nodes and the trapezoid rule in phi with 16 are exact in the angles;
    Gauss-Legendre with 96 nodes on [0, 14 xi] in the radius."""
    kr, wr = np.polynomial.legendre.leggauss(96)
    kr = 7.0 * xi * (kr + 1.0)
    wr = 7.0 * xi * wr
    ct, wt = np.polynomial.legendre.leggauss(8)
    ph = np.arange(16) * (2 * np.pi / 16)
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)), np.outer(ct, np.ones(16))], -1).reshape(-1, 3)
    wd = np.outer(wt, np.full(16, 2 * np.pi / 16)).reshape(-1)
    k = (kr[:, None, None] * dirs[None, :, :]).reshape(-1, 3)
    w = (wr[:, None] * kr[:, None] ** 2 * wd[None, :]).reshape(-1)
    M = fourier_block(target, source, k, xi, a, eta)
    return (np.einsum("p,pij->ij", w, M) / (2 * np.pi) ** 3).real


def periodic_blocks(target, source, R, ew: Ewald, a, eta, rows=None):
    """Dense [len(rows) * dT, N * dX] of the periodic blocks: every pair (m != n) with all its
    periodic images, and each sphere with its own images."""
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    n = R.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    dT, dX = TARGET_DIM[target], SOURCE_DIM[source]
    out = np.zeros((len(rows), n, dT, dX))
    nvec = ew.images()
    kv = ew.kvecs()
    Mk = fourier_block(target, source, kv, ew.xi, a, eta)  # [nk, dT, dX]
    V = ew.L ** 3
    Mf = Mk.reshape(len(kv), dT * dX)
    Ep = np.exp(1j * (R @ kv.T))   # [n, nk]
    Em = np.conj(Ep)
    chunk = max(1, 200000 // max(1, n * len(nvec)))
    for c0 in range(0, len(rows), chunk):
        rr = rows[c0:c0 + chunk]
        dx = _wrap(R[rr, None, :] - R[None, :, :], ew.L)  # [nr, n, 3]
        # real space: all images within rc (the receiver's own image n = 0 excluded)
        s = dx[:, :, None, :] + nvec[None, None, :, :]
        r = np.sqrt(np.einsum("abci,abci->abc", s, s))
        sel = (r <= ew.rc) & (r > 0)
        ia, ib, _ = np.nonzero(sel)
        if ia.size:
            blk = real_block(target, source, s[sel], ew.xi, a, eta)
            np.add.at(out, (c0 + ia, ib), blk)
        # Fourier space: every sphere, the receiver itself included; exp(i k.(R_i - R_m)) =
        # exp(i k.R_i) exp(-i k.R_m) on the reciprocal lattice (a wrap by L changes no phase)
        for d in range(dT * dX):
            out[c0:c0 + len(rr), :, d // dX, d % dX] += (((Ep[rr] * Mf[None, :, d]) @ Em.T) / V).real
        for q, i in enumerate(rr):
            out[c0 + q, i] -= _smooth_self(target, source, ew.xi, a, eta)
    return out.transpose(0, 2, 1, 3).reshape(len(rows) * dT, n * dX)


# ------------------------------------------------------------------ the periodic system
def system_matrix(R, prm: galerkin.Params, ew: Ewald):
    """A = I/gamma - K^SS_per (every pair and each sphere with its own images)."""
    n = len(np.asarray(R).reshape(-1, 3))
    gamma = galerkin.constants(prm)["gamma"]
    return np.eye(5 * n) / gamma - periodic_blocks("E", "S", R, ew, prm.a, prm.eta)


def rhs(R, v2s, v3t, Fe, Te, prm: galerkin.Params, ew: Ewald):
    """b = E_per[F, T, d] - c s."""
    b = -prm.self_slip_c * np.ravel(v2s)
    for kind, vals in (("F", Fe), ("T", Te), ("D", v3t)):
        if vals is not None:
            b = b + periodic_blocks("E", kind, R, ew, prm.a, prm.eta) @ np.ravel(vals)
    return b


def outputs(R, v1s, v2s, v3t, Fe, Te, Sigma, prm: galerkin.Params, ew: Ewald):
    """V, Omega, S of the periodic system from a flow stresslet Sigma (the one-body terms as in the
    unbounded fluid, the pair and own-image terms through the periodic blocks)."""
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    n = R.shape[0]
    c = galerkin.constants(prm)
    z3 = np.zeros((n, 3))
    V = (-np.asarray(v1s) if v1s is not None else z3) + (np.asarray(Fe) / c["drag_t"] if Fe is not None else z3)
    W = np.asarray(Te) / c["drag_r"] if Te is not None else z3.copy()
    for kind, vals in (("F", Fe), ("T", Te), ("S", Sigma), ("D", v3t)):
        if vals is not None:
            V = V + (periodic_blocks("U", kind, R, ew, prm.a, prm.eta) @ np.ravel(vals)).reshape(n, 3)
            W = W + (periodic_blocks("W", kind, R, ew, prm.a, prm.eta) @ np.ravel(vals)).reshape(n, 3)
    S = np.asarray(Sigma) + c["slip_to_S"] * np.asarray(v2s)
    return V, W, S


def solve(w, ew: Ewald, prm: galerkin.Params | None = None):
    prm = prm or galerkin.Params(eta=getattr(w, "eta", 1.0 / (6 * np.pi)), a=getattr(w, "a", 1.0))
    A = system_matrix(w.R, prm, ew)
    b = rhs(w.R, w.v2s, w.v3t, w.Fe, w.Te, prm, ew)
    Sigma = np.linalg.solve(A, b).reshape(-1, 5)
    V, W, S = outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sigma, prm, ew)
    return dict(V=V, W=W, S=S, Sigma=Sigma, b=b, A=A)


@functools.lru_cache(maxsize=None)
def _flow_fn(which, source):
    cols = _flows(kernel(which), source, _Rules(which == "fourier"))
    mat = [[cols[q][i] for q in range(len(cols))] for i in range(3)]
    args = (kx_, ky_, kz_, xi_, a_, P_) if which == "fourier" else (x_, y_, z_, r_, ec_, ex_, xi_, a_, P_)
    return sp.lambdify(args, mat, "numpy", cse=True)


def flow_field(X, R, Fe, Te, Sigma, v3t, prm: galerkin.Params, ew: Ewald):
    """Flow of the periodic suspension at field points X [m, 3] (no finite-size operator at the field
    point): every sphere with all its images, real-space part within rc plus the Fourier sum."""
    from scipy.special import erfc
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    P = 1.0 / (8 * np.pi * prm.eta)
    nvec = ew.images()
    kv = ew.kvecs()
    q = np.einsum("pi,pi->p", kv, kv) / (4.0 * ew.xi * ew.xi)
    phi = (1.0 + q) * np.exp(-q)
    Ex = np.exp(1j * (X @ kv.T))        # [m, nk]
    Er = np.exp(-1j * (R @ kv.T))       # [n, nk]
    u = np.zeros((X.shape[0], 3))
    for kind, vals in (("F", Fe), ("T", Te), ("S", Sigma), ("D", v3t)):
        if vals is None:
            continue
        vals = np.asarray(vals, dtype=np.float64)
        fr = _flow_fn("real", kind)
        for m in range(R.shape[0]):
            s = _wrap(X - R[m], ew.L)[:, None, :] + nvec[None, :, :]
            r = np.sqrt(np.einsum("abi,abi->ab", s, s))
            sel = (r <= ew.rc) & (r > 0)
            if np.any(sel):
                pts, rr = s[sel], r[sel]
                raw = fr(pts[:, 0], pts[:, 1], pts[:, 2], rr, erfc(ew.xi * rr), np.exp(-(ew.xi * rr) ** 2), ew.xi,
                         prm.a, P)
                blk = np.stack([np.stack([np.broadcast_to(np.asarray(raw[i][j], dtype=float), (len(rr),))
                                          for j in range(len(raw[0]))], -1) for i in range(3)], 1)
                ia = np.nonzero(sel)[0]
                np.add.at(u, ia, np.einsum("pij,j->pi", blk, vals[m]))
        raw = _flow_fn("fourier", kind)(kv[:, 0], kv[:, 1], kv[:, 2], ew.xi, prm.a, P)
        Mk = np.stack([np.stack([np.broadcast_to(np.asarray(raw[i][j], dtype=complex), (len(kv),))
                                 for j in range(len(raw[0]))], -1) for i in range(3)], 1) * phi[:, None, None]
        Sk = Er.T @ vals                   # [nk, dX]: sum_m exp(-i k.R_m) c_m
        Tk = np.einsum("kij,kj->ki", Mk, Sk)  # [nk, 3]
        u += ((Ex @ Tk) / ew.L ** 3).real
    return u


def matvec_rows(R, x, rows, prm: galerkin.Params, ew: Ewald):
    """(A x) restricted to the given spheres, without forming A."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 5)
    gamma = galerkin.constants(prm)["gamma"]
    K = periodic_blocks("E", "S", R, ew, prm.a, prm.eta, rows) @ np.ravel(x)
    return x[np.asarray(rows)] / gamma - K.reshape(-1, 5)
