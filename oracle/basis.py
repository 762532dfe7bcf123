"""Orthonormal basis of symmetric traceless 3x3 tensors (test infrastructure only).

Rank-2 symmetric traceless coefficients (the stresslet, the strain, the
symmetric linear slip mode) have 5 independent components; the paper's
irreducible decomposition (section III, irreducible parts of the coefficients)
keeps exactly this part. With the basis below the Frobenius inner product of
two such tensors equals the Euclidean product of their 5-vectors.
"""
import numpy as np

_s2 = np.sqrt(2.0)
_s6 = np.sqrt(6.0)

BASIS = np.zeros((5, 3, 3))
BASIS[0, 0, 0], BASIS[0, 1, 1] = 1 / _s2, -1 / _s2
BASIS[1, 0, 0], BASIS[1, 1, 1], BASIS[1, 2, 2] = -1 / _s6, -1 / _s6, 2 / _s6
BASIS[2, 0, 1] = BASIS[2, 1, 0] = 1 / _s2
BASIS[3, 0, 2] = BASIS[3, 2, 0] = 1 / _s2
BASIS[4, 1, 2] = BASIS[4, 2, 1] = 1 / _s2


def to5(m):
    """[..., 3, 3] -> [..., 5] by projection on the basis (drops trace and antisymmetric part)."""
    return np.einsum("...ij,cij->...c", np.asarray(m, dtype=np.float64), BASIS)


def from5(c):
    """[..., 5] -> [..., 3, 3]."""
    return np.einsum("...c,cij->...ij", np.asarray(c, dtype=np.float64), BASIS)


# Rank-3 symmetric tensors are exchanged as their 10 independent components in the order below;
# only the symmetric traceless part (7 independent components) enters the flows.
SYM3 = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2), (1, 2, 2),
        (2, 2, 2)]


# Symmetric traceless rank-3 tensors (the septlet mode) as 7 coordinates: c_k = T :. B3_k (full
# contraction), with B3_k = T^(k) / |T^(k)| and T^(k)_ijk = (1/6) d_i d_j d_k p_k for the seven real
# harmonic cubic polynomials below (orthogonal on the sphere, so the tensors are orthogonal under
# the full contraction); the Frobenius norm of T equals the Euclidean norm of its 7 coordinates.
CUBICS = ("2*z**3 - 3*x**2*z - 3*y**2*z", "4*x*z**2 - x**3 - x*y**2", "4*y*z**2 - x**2*y - y**3",
          "x**2*z - y**2*z", "x*y*z", "x**3 - 3*x*y**2", "3*x**2*y - y**3")


def _basis3_exact():
    import itertools

    import sympy as sp
    X = sp.symbols("x y z")
    out = []
    for expr in CUBICS:
        p = sp.sympify(expr, locals=dict(zip("xyz", X)))
        T = [[[sp.diff(p, X[i], X[j], X[k]) / 6 for k in range(3)] for j in range(3)] for i in range(3)]
        norm = sp.sqrt(sum(T[i][j][k] ** 2 for i, j, k in itertools.product(range(3), repeat=3)))
        out.append([[[sp.nsimplify(T[i][j][k] / norm) for k in range(3)] for j in range(3)] for i in range(3)])
    return out


BASIS3_EXACT = _basis3_exact()
BASIS3 = np.array([[[[float(B[i][j][k]) for k in range(3)] for j in range(3)] for i in range(3)]
                   for B in BASIS3_EXACT])


def to7(T):
    """[..., 3, 3, 3] symmetric traceless -> [..., 7] coordinates in the basis above."""
    return np.einsum("...ijk,cijk->...c", np.asarray(T, dtype=np.float64), BASIS3)


def from7(c):
    """[..., 7] -> [..., 3, 3, 3]."""
    return np.einsum("...c,cijk->...ijk", np.asarray(c, dtype=np.float64), BASIS3)


def sym3_from10(c):
    """[..., 10] symmetric rank-3 components in the SYM3 order -> [..., 3, 3, 3] symmetric tensor."""
    import itertools
    c = np.asarray(c, dtype=np.float64)
    T = np.zeros(c.shape[:-1] + (3, 3, 3))
    for q, idx in enumerate(SYM3):
        for perm in set(itertools.permutations(idx)):
            T[(...,) + perm] = c[..., q]
    return T
