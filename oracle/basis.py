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
