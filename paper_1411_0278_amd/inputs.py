"""Seeded synthetic workloads for the many-body active-sphere solver.

This module only draws particle placements and orientations and writes out the
slip-mode and body-force values a workload prescribes. It holds none of the
method's arithmetic (no Green's functions, no pair blocks, no solve) and it is
shared, unchanged, by the GPU path's tests and benchmark and by the CPU oracle.

Workload recipe (one reading of the paper's trap set-up, section V, and of the
benchmark configurations):

* spheres of radius a = 1 in an unbounded fluid of viscosity 1/(6 pi);
* centres uniform in the cube [-L/2, L/2]^3, sequential rejection: a candidate
  is kept when it is at least ``min_dist`` (2.2 a) from every centre kept so
  far; candidates come from ``numpy.random.default_rng(seed)`` in blocks and are
  consumed strictly in order;
* orientations p are Gaussian 3-vectors, normalised, drawn from a second
  stream ``default_rng((seed, 1))`` so that they do not depend on how many
  position candidates were rejected;
* slip modes: mean slip mode V^(1s) = p, symmetric-traceless linear slip
  V^(2s) = 3 (p p - I/3), optionally the rank-3 trace mode V^(3t) = p;
* harmonic trap force F^e = -k R with k = 0.5, no external torque.

Symmetric traceless 3x3 tensors are exchanged in the orthonormal 5-component
basis  B0 = (xx - yy)/sqrt2, B1 = (2zz - xx - yy)/sqrt6, B2 = (xy + yx)/sqrt2,
B3 = (xz + zx)/sqrt2, B4 = (yz + zy)/sqrt2  (coefficient c_i = M : B_i).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ETA = 1.0 / (6.0 * math.pi)
RADIUS = 1.0
MIN_DIST = 2.2
TRAP_K = 0.5

_S2 = math.sqrt(2.0)
_S6 = math.sqrt(6.0)


def sym_to_basis5(m: np.ndarray) -> np.ndarray:
    """[..., 3, 3] symmetric traceless -> [..., 5] coefficients in the basis above."""
    m = np.asarray(m, dtype=np.float64)
    out = np.empty(m.shape[:-2] + (5,), dtype=np.float64)
    out[..., 0] = (m[..., 0, 0] - m[..., 1, 1]) / _S2
    out[..., 1] = (2.0 * m[..., 2, 2] - m[..., 0, 0] - m[..., 1, 1]) / _S6
    out[..., 2] = _S2 * m[..., 0, 1]
    out[..., 3] = _S2 * m[..., 0, 2]
    out[..., 4] = _S2 * m[..., 1, 2]
    return out


def place_spheres(n: int, side: float, seed: int, min_dist: float = MIN_DIST) -> np.ndarray:
    """Sequential random sequential adsorption in a cube; returns [n, 3] float64."""
    if n <= 0:
        return np.zeros((0, 3))
    rng = np.random.default_rng(seed)
    half = 0.5 * side
    cell = float(min_dist)
    md2 = float(min_dist) ** 2
    grid: dict[tuple[int, int, int], list[int]] = {}
    pts = np.empty((n, 3), dtype=np.float64)
    k = 0
    drawn = 0
    max_draws = 2000 * n + 10000
    while k < n:
        block = rng.uniform(-half, half, size=(4096, 3))
        for c in block:
            drawn += 1
            ix = int(math.floor((c[0] + half) / cell))
            iy = int(math.floor((c[1] + half) / cell))
            iz = int(math.floor((c[2] + half) / cell))
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        for j in grid.get((ix + dx, iy + dy, iz + dz), ()):
                            d = c - pts[j]
                            if d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < md2:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                pts[k] = c
                grid.setdefault((ix, iy, iz), []).append(k)
                k += 1
                if k == n:
                    break
        if drawn > max_draws:
            raise RuntimeError(f"could not place {n} spheres in a cube of side {side}")
    return pts


def orientations(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng((seed, 1))
    p = rng.standard_normal((n, 3))
    return p / np.linalg.norm(p, axis=1, keepdims=True)


@dataclasses.dataclass
class Workload:
    """One configuration: every array is float64, row-major, particle-major."""
    R: np.ndarray      # [n, 3] centres
    p: np.ndarray      # [n, 3] unit orientations
    v1s: np.ndarray    # [n, 3] mean slip mode V^(1s)
    v2s: np.ndarray    # [n, 5] symmetric-traceless linear slip mode V^(2s) (5-basis)
    v3t: np.ndarray    # [n, 3] rank-3 trace slip mode V^(3t)
    Fe: np.ndarray     # [n, 3] external body force
    Te: np.ndarray     # [n, 3] external body torque
    eta: float = ETA
    a: float = RADIUS
    name: str = ""
    # optional slip modes of the minimal truncation (None = absent): septlet gamma [n, 10] and
    # spinlet lambda [n, 10] as symmetric rank-3 components (order SYM3), vortlet psi [n, 5]
    gam: np.ndarray | None = None
    psi: np.ndarray | None = None
    lam: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.R.shape[0])

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx)
        cut = lambda v: None if v is None else v[idx].copy()
        return Workload(self.R[idx].copy(), self.p[idx].copy(), self.v1s[idx].copy(),
                        self.v2s[idx].copy(), self.v3t[idx].copy(), self.Fe[idx].copy(),
                        self.Te[idx].copy(), self.eta, self.a, self.name + "[subset]",
                        cut(self.gam), cut(self.psi), cut(self.lam))


def slip_modes(p: np.ndarray, c1: float = 1.0, c2: float = 1.0, c3: float = 0.0):
    """Slip-mode values of the workloads: V^(1s) = c1 p, V^(2s) = c2 * 3(pp - I/3), V^(3t) = c3 p."""
    p = np.asarray(p, dtype=np.float64)
    pp = p[:, :, None] * p[:, None, :]
    m = 3.0 * (pp - np.eye(3)[None] / 3.0)
    return c1 * p, c2 * sym_to_basis5(m), c3 * p


# Rank-3 symmetric tensors as 10 components, in this order of index triples.
SYM3 = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2), (1, 2, 2),
        (2, 2, 2)]


def uniaxial_rank3(p: np.ndarray) -> np.ndarray:
    """[n, 3] unit vectors -> [n, 10]: the symmetric traceless part of p p p,
    p_i p_j p_k - (delta_ij p_k + delta_ik p_j + delta_jk p_i) / 5, in the SYM3 order."""
    p = np.asarray(p, dtype=np.float64)
    out = np.empty((p.shape[0], 10))
    for q, (i, j, k) in enumerate(SYM3):
        out[:, q] = (p[:, i] * p[:, j] * p[:, k]
                     - ((i == j) * p[:, k] + (i == k) * p[:, j] + (j == k) * p[:, i]) / 5.0)
    return out


def higher_slip_modes(p: np.ndarray, c_gam: float = 1.0, c_psi: float = 1.0, c_lam: float = 1.0):
    """Uniaxial septlet, vortlet and spinlet slip modes along p: gamma = c_gam STF(ppp),
    psi = c_psi (pp - I/3) (5-basis), lambda = c_lam STF(ppp)."""
    p = np.asarray(p, dtype=np.float64)
    pp = p[:, :, None] * p[:, None, :]
    u3 = uniaxial_rank3(p)
    return c_gam * u3, c_psi * sym_to_basis5(pp - np.eye(3)[None] / 3.0), c_lam * u3


def trap_workload(n: int, side: float, seed: int, k: float = TRAP_K, v3t: float = 0.0,
                  name: str = "") -> Workload:
    R = place_spheres(n, side, seed)
    p = orientations(n, seed)
    v1s, v2s, v3 = slip_modes(p, 1.0, 1.0, v3t)
    return Workload(R, p, v1s, v2s, v3, -k * R, np.zeros_like(R), name=name or f"trap_n{n}_L{side:g}_s{seed}")


def sphere_points(n: int, radius: float) -> np.ndarray:
    """n quasi-uniform points on a sphere (golden-angle spiral), deterministic."""
    k = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * k / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.pi * (3.0 - np.sqrt(5.0)) * k
    return radius * np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def paper_trap_workload(n: int = 10_000, radius_in_a: float = 1256.6, vs: float = 1.0) -> Workload:
    """The trap set-up of section V: active spheres spread uniformly over the sphere of radius
    R* = 6 pi eta a v_s / k (their stable state without interactions), each pointing outward, so the
    self-propulsion V^a = v_s p balances the trap force -k R. Only the mean slip is set (V^(1s) = -v_s p); the stresslet and rank-3 strengths are not given."""
    R = sphere_points(n, radius_in_a * RADIUS)
    p = R / np.linalg.norm(R, axis=1, keepdims=True)
    k = 6.0 * math.pi * ETA * RADIUS * vs / (radius_in_a * RADIUS)
    v1s, v2s, v3 = slip_modes(p, -vs, 0.0, 0.0)
    return Workload(R, p, v1s, v2s, v3, -k * R, np.zeros_like(R), name=f"paper_trap_n{n}_R{radius_in_a:g}")


# The benchmark configurations (sizes, boxes, seeds).
def config0(seed: int = 0) -> Workload:
    """N = 256 in a cube of side 40 (number density 0.004); mean + strain slip; trap k = 0.5."""
    return trap_workload(256, 40.0, seed, name="cfg0_n256_L40")


def config1(seed: int = 1, n: int = 10_000, side: float = 200.0) -> Workload:
    """N = 1e4 in a cube of side 200, plus the rank-3 trace slip mode V^(3t) = p (time-stepped)."""
    return trap_workload(n, side, seed, v3t=1.0, name=f"cfg1_n{n}_L{side:g}")


def config2(seed: int = 1000, n: int = 100_000, side: float = 430.0) -> Workload:
    """N = 1e5 in a cube of side 430 (number density 1.26e-3)."""
    return trap_workload(n, side, seed, name=f"cfg2_n{n}_L{side:g}_s{seed}")


def batched_sizes(count: int = 512, lo: int = 64, hi: int = 4096, seed: int = 4242) -> np.ndarray:
    """Particle counts log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return np.clip(np.rint(np.exp(u)).astype(np.int64), lo, hi)


def config3(count: int = 512, lo: int = 64, hi: int = 4096, density: float = 0.004,
            seed: int = 4242) -> list[Workload]:
    """Many independent configurations of uneven N at a fixed number density; config b uses seed 10000 + b."""
    sizes = batched_sizes(count, lo, hi, seed)
    out = []
    for b, nb in enumerate(sizes):
        side = (float(nb) / density) ** (1.0 / 3.0)
        out.append(trap_workload(int(nb), side, 10_000 + b, name=f"cfg3_b{b}_n{nb}"))
    return out


def nearest_to_origin(w: Workload, m: int) -> Workload:
    """The m particles closest to the trap centre, as a standalone configuration."""
    d = np.linalg.norm(w.R, axis=1)
    idx = np.sort(np.argsort(d, kind="stable")[:m])
    return w.subset(idx)
