"""Smooth particle-mesh Ewald in the periodic box on the GPU (params.ewald_mesh): every pass, the
solve and the flow at field points against the oracle's exact Ewald sums (the definition the mesh
approximates) at the mesh's error level, the error falling as the mesh is refined at a fixed
splitting, sampled rows at a thousand spheres, and the parameter checks."""
import functools
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import galerkin, periodic  # noqa: E402
from paper_1411_0278_amd import inputs, mbstokes  # noqa: E402

DEV = "cuda:0"
ETA, A = 1.0 / (6.0 * np.pi), 1.0
PRM = galerkin.Params(eta=ETA, a=A)

# The mesh's error, relative to the largest entry of a pass's result: B-splines of order 8 with the
# default splitting (xi = pi M / (14 L), at most 0.5/a) leave about 1e-6 of the Fourier part, itself
# a fraction of the whole result (measured: 2e-8 for the operator, 1e-7 for the outputs, boxes of
# 20a and more); the bar leaves room for other configurations of the same kind.
BAR = 1e-6


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _maxrel(got, want):
    got = _np(got) if hasattr(got, "detach") else np.asarray(got)
    return np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)


@pytest.fixture(scope="module")
def ctx():
    c = mbstokes.Context(0)
    yield c
    c.close()


def _place(n, L, seed, dmin=2.2):
    """Random sequential placement in [0, L)^3 with minimum-image distances >= dmin."""
    rng = np.random.default_rng(seed)
    R = np.empty((0, 3))
    while len(R) < n:
        x = rng.uniform(0, L, 3)
        d = R - x
        d -= L * np.round(d / L)
        if len(R) == 0 or np.min(np.einsum("pi,pi->p", d, d)) >= dmin * dmin:
            R = np.vstack([R, x])
    return R


def _workload(n, seed, L=None):
    L = L or max(20.0, (n / 0.004) ** (1 / 3))
    rng = np.random.default_rng(seed + 7)
    R = _place(n, L, seed)
    p = rng.standard_normal((n, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    v1s, v2s, v3t = inputs.slip_modes(p, 1.0, 1.0, 1.0)
    w = inputs.Workload(R, p, v1s, v2s, v3t, rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), ETA, A)
    return w, L


def _ew(L):
    return periodic.Ewald(L, xi=7.0 / L)  # the oracle's own splitting (its result does not depend on it)


@functools.lru_cache(maxsize=None)
def _system(n, seed):
    w, L = _workload(n, seed)
    return periodic.system_matrix(w.R, PRM, _ew(L))


class _Mesh:
    def __init__(self, ctx, L, M, **kw):
        self.ctx, self.L, self.M, self.kw = ctx, L, M, kw

    def __enter__(self):
        self.ctx.set_params(box=self.L, ewald_mesh=self.M, **self.kw)
        return self.ctx

    def __exit__(self, *exc):
        self.ctx.set_params(box=0.0, ewald_mesh=0, ewald_xi=0.0, tol=1e-10, precision=mbstokes.MBS_FP64,
                            near_cutoff=0.0, near_order=2, spatial_order=0)


@pytest.mark.parametrize("n,M", [(1, 64), (2, 64), (97, 64), (97, 128)])
def test_pme_operator_matches_oracle(ctx, n, M):
    print(f"pme matvec n={n} M={M}", flush=True)
    w, L = _workload(n, 4000 + n)
    x = np.random.default_rng(n).standard_normal((n, 5))
    want = (_system(n, 4000 + n) @ x.ravel()).reshape(n, 5)
    with _Mesh(ctx, L, M):
        got = ctx.mbs_matvec(_t(w.R), _t(x))
        again = ctx.mbs_matvec(_t(w.R), _t(x))
    err = _maxrel(got, want)
    print(f"  max rel error {err:.3e}", flush=True)
    assert err < BAR
    assert torch.equal(got, again)  # every sum in a fixed order: bitwise reproducible


@pytest.mark.parametrize("n,M", [(97, 64), (300, 128), (97, 512)])
def test_pme_rhs_and_outputs_match_oracle(ctx, n, M):
    # 300 spheres: the real space over the box grid's cells; M = 512: the multiplier in its own pass
    # (the x transforms fused with it need 2 NI M <= 4096 points of LDS)
    print(f"pme rhs/outputs n={n} M={M}", flush=True)
    w, L = _workload(n, 4100 + n)
    Sig = np.random.default_rng(5).standard_normal((n, 5))
    b = periodic.rhs(w.R, w.v2s, w.v3t, w.Fe, w.Te, PRM, _ew(L)).reshape(n, 5)
    V, W, S = periodic.outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sig, PRM, _ew(L))
    with _Mesh(ctx, L, M):
        gb = ctx.mbs_rhs(_t(w.R), _t(w.v2s), _t(w.v3t), _t(w.Fe), _t(w.Te))
        gV, gW, gS = ctx.mbs_outputs(_t(w.R), _t(Sig), _t(w.v1s), _t(w.v2s), _t(w.v3t), _t(w.Fe), _t(w.Te))
    errs = [_maxrel(gb, b), _maxrel(gV, V), _maxrel(gW, W), _maxrel(gS, S)]
    print("  rhs, V, W, S errors " + " ".join(f"{e:.3e}" for e in errs), flush=True)
    assert max(errs[:3]) < BAR and errs[3] < 1e-14


def test_pme_error_falls_as_the_mesh_is_refined(ctx):
    """At a fixed splitting the interpolation error falls steeply with the mesh spacing."""
    n = 97
    w, L = _workload(n, 4000 + n)
    x = np.random.default_rng(n).standard_normal((n, 5))
    want = (_system(n, 4000 + n) @ x.ravel()).reshape(n, 5)
    errs = []
    for M in (32, 64, 128):
        with _Mesh(ctx, L, M, ewald_xi=10.5 / L):
            errs.append(_maxrel(ctx.mbs_matvec(_t(w.R), _t(x)), want))
    print("  errors at M = 32, 64, 128: " + " ".join(f"{e:.3e}" for e in errs), flush=True)
    assert errs[0] > 100 * errs[1] > 0 and errs[2] < errs[1] < 1e-8


def test_pme_solve_matches_oracle(ctx):
    n, M = 97, 64
    w, L = _workload(n, 4200)
    sol = periodic.solve(w, _ew(L), PRM)
    d = mbstokes.to_device(w, DEV)
    Sig = torch.empty((n, 5), dtype=torch.float64, device=DEV)
    for prec, near, spatial in ((mbstokes.MBS_FP64, 0.0, 0), (mbstokes.MBS_MIXED, 8.0, 0), (mbstokes.MBS_FP64, 8.0, 1)):
        with _Mesh(ctx, L, M, tol=1e-12, precision=prec, near_cutoff=near, spatial_order=spatial):
            V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], Sigma=Sig)
            V2, W2, S2, st2 = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
        errs = [_maxrel(V, sol["V"]), _maxrel(W, sol["W"]), _maxrel(S, sol["S"]), _maxrel(Sig, sol["Sigma"])]
        print(f"  solve precision={prec} near={near} spatial={spatial}: " + " ".join(f"{e:.3e}" for e in errs),
              flush=True)
        assert max(errs) < 10 * BAR
        assert torch.equal(V, V2) and torch.equal(W, W2)  # the second solve replays the captured steps


@pytest.mark.parametrize("n,M", [(97, 64), (300, 128)])
def test_pme_flow_field_matches_oracle(ctx, n, M):
    # 300 spheres: the field points binned in a box grid like the spheres, real space over cells
    print(f"pme flow n={n} M={M}", flush=True)
    m = 240
    w, L = _workload(n, 4300 + n)
    Sig = np.random.default_rng(21).standard_normal((n, 5))
    X = np.random.default_rng(22).uniform(-0.5 * L, 1.5 * L, (m, 3))  # anywhere: taken modulo the box
    want = periodic.flow_field(X, w.R, w.Fe, w.Te, Sig, w.v3t, PRM, _ew(L))
    with _Mesh(ctx, L, M):
        got = ctx.mbs_flow(_t(X), _t(w.R), _t(Sig), _t(w.Fe), _t(w.Te), _t(w.v3t))
    err = _maxrel(got, want)
    print(f"  flow error {err:.3e}", flush=True)
    assert err < BAR


@pytest.mark.parametrize("n,M,nrows", [(300, 128, 40), (1000, 128, 5)])
def test_pme_operator_sampled_rows(ctx, n, M, nrows):
    print(f"pme sampled rows n={n} M={M}", flush=True)  # the real space over the box grid's cells
    w, L = _workload(n, 4400 + n)
    x = np.random.default_rng(11).standard_normal((n, 5))
    with _Mesh(ctx, L, M):
        got = _np(ctx.mbs_matvec(_t(w.R), _t(x)))
    rows = np.random.default_rng(12).choice(n, nrows, replace=False)
    want = periodic.matvec_rows(w.R, x, rows, PRM, _ew(L))
    err = _maxrel(got[rows], want)
    print(f"  sampled rows error {err:.3e}", flush=True)
    assert err < BAR


def test_pme_parameter_checks(ctx):
    L = 30.0
    for bad in ({"ewald_mesh": 48}, {"ewald_mesh": 8}, {"ewald_mesh": 1024}, {"ewald_mesh": -64}, {"ewald_mesh": -2},
                {"ewald_mesh": 64, "ewald_xi": 9.0 / L}):  # real-space cutoff beyond L/2
        with pytest.raises(mbstokes.MbsError) as e:
            ctx.set_params(box=L, **bad)
        assert e.value.code == mbstokes.MBS_EINVAL
        ctx.set_params(box=0.0, ewald_mesh=0, ewald_xi=0.0)
    with pytest.raises(mbstokes.MbsError) as e:
        ctx.set_params(box=0.0, ewald_mesh=64)  # a mesh needs a box
    assert e.value.code == mbstokes.MBS_EINVAL
    ctx.set_params(box=0.0, ewald_mesh=0, ewald_xi=0.0)


def test_pme_stepper_matches_oracle(ctx):
    """Force-free swimmers (slip modes 1, 1, 1 along p, no trap) stepped three times in the box on the
    mesh against the oracle's stepper on the exact periodic solve."""
    from oracle import stepper
    n = 24
    w, L = _workload(n, 4500, L=20.0)
    Rw, pw, _ = stepper.run(w.R, w.p, 0.0, (1.0, 1.0, 1.0), 0.05, 3, PRM,
                            solve=lambda st, pr: periodic.solve(st, _ew(L), pr))
    R, p = _t(w.R), _t(w.p)
    with _Mesh(ctx, L, 64, tol=1e-13):
        stats, md = ctx.mbs_step(R, p, 0.0, (1.0, 1.0, 1.0), 0.05, 3, order=2, want_min_dist=True)
    errs = (_maxrel(R, Rw), _maxrel(p, pw))
    print(f"  stepper errors R {errs[0]:.3e} p {errs[1]:.3e}", flush=True)
    assert max(errs) < 1e-8


@pytest.mark.parametrize("layout", ["random", "sparse"])
def test_pme_stepper_min_dist_from_the_box_grid(ctx, layout):
    """With a mesh and at least 3 cells per axis the stepper's smallest minimum-image distance comes
    from the box grid's neighbouring cells (300 spheres placed at random), or from all pairs when no
    pair is closer than a cell edge (8 spheres near the sites of a 2 x 2 x 2 lattice): exact either way."""
    print(f"pme min_dist {layout}", flush=True)
    L = 42.0  # M = 128: xi = 0.5/a, rc = 10a, 4 cells of 10.5a per axis
    if layout == "random":
        w, _ = _workload(300, 4600, L=L)
    else:
        w, _ = _workload(8, 4601, L=L)
        g = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float) * (L / 2) + 5.0
        w.R = g + np.random.default_rng(3).uniform(-1.0, 1.0, g.shape)
    n = len(w.R)
    d = w.R[:, None, :] - w.R[None, :, :]
    d -= L * np.round(d / L)
    want = (np.sqrt((d ** 2).sum(-1)) + np.eye(n) * 1e9).min()
    with _Mesh(ctx, L, 128, tol=1e-8):
        stats, md = ctx.mbs_step(_t(w.R), _t(w.p), 0.0, (1.0, 1.0, 1.0), 0.01, 1, order=1, want_min_dist=True)
    assert (want < 10.5) == (layout == "random")
    assert abs(md[0] - want) < 1e-12 * L


def test_pme_automatic_mesh_equals_its_explicit_size(ctx):
    """ewald_mesh = -1 takes the smallest power of 2 with spacing at most 1.25a: the same result, bit
    for bit, as naming that mesh."""
    n = 300
    w, L = _workload(n, 4700)  # box 42.2a: 64 points would space them 0.66a, 32 points 1.32a
    x = np.random.default_rng(8).standard_normal((n, 5))
    with _Mesh(ctx, L, -1):
        auto = ctx.mbs_matvec(_t(w.R), _t(x))
    with _Mesh(ctx, L, 64):
        named = ctx.mbs_matvec(_t(w.R), _t(x))
    assert torch.equal(auto, named)
