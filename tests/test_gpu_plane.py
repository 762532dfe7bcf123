"""Spheres above a plane on the GPU (params.plane: 1 a stress-free plane, 2 a no-slip wall): every
pass with the spheres' images and the solve against the oracle's half-space system of that kind,
element by element, at sizes that span several workgroups and source chunks with ragged tails, and
on sampled rows at 10^4 spheres."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import galerkin, plane, wall  # noqa: E402
from paper_1411_0278_amd import inputs, mbstokes  # noqa: E402

DEV = "cuda:0"
ORACLE = {1: plane, 2: wall}
KINDS = pytest.mark.parametrize("kind", [1, 2], ids=["free_slip", "no_slip"])


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


def _workload(n, seed, side=None, lift=1.5):
    """Trap spheres at the benchmark density with torques and rank-3 trace modes; the plane lies
    `lift` radii below the lowest sphere."""
    side = side or max(8.0, (n / 0.004) ** (1 / 3))
    w = inputs.trap_workload(n, side, seed, v3t=1.0)
    w.Te = np.random.default_rng(seed + 5).standard_normal((n, 3))
    return w, float(w.R[:, 2].min() - lift * w.a)


def _prm(w):
    return galerkin.Params(eta=w.eta, a=w.a)


class _Plane:
    def __init__(self, ctx, z_w, kind=1, **kw):
        self.ctx, self.z_w, self.kind, self.kw = ctx, z_w, kind, kw

    def __enter__(self):
        self.ctx.set_params(plane=self.kind, plane_z=self.z_w, **self.kw)
        return self.ctx

    def __exit__(self, *exc):
        self.ctx.set_params(plane=0, plane_z=0.0, tol=1e-10, precision=mbstokes.MBS_FP64, near_cutoff=0.0,
                            near_order=2, superposition=0, spatial_order=0, guess=mbstokes.MBS_GUESS_ZERO)


@KINDS
@pytest.mark.parametrize("n", [1, 2, 97, 257])
def test_plane_operator_matches_oracle(ctx, kind, n):
    print(f"plane {kind} matvec n={n}", flush=True)
    w, z_w = _workload(n, 1400 + n)
    x = np.random.default_rng(n).standard_normal((n, 5))
    want = (ORACLE[kind].system_matrix(w.R, _prm(w), z_w) @ x.ravel()).reshape(n, 5)
    with _Plane(ctx, z_w, kind):
        got = ctx.mbs_matvec(_t(w.R), _t(x))
        got32 = ctx.mbs_matvec(_t(w.R), _t(x), precision=mbstokes.MBS_FP32)
    assert _maxrel(got, want) < 1e-13
    # binary32 free-space part; the image part binary32 (stress-free) or binary64 (no-slip)
    assert _maxrel(got32, want) < 2e-6


@KINDS
@pytest.mark.parametrize("n", [1, 2, 97, 257])
def test_plane_rhs_and_outputs_match_oracle(ctx, kind, n):
    print(f"plane {kind} rhs/outputs n={n}", flush=True)
    w, z_w = _workload(n, 1500 + n)
    prm = _prm(w)
    Sig = np.random.default_rng(n + 3).standard_normal((n, 5))
    b = ORACLE[kind].rhs(w.R, w.v2s, w.v3t, w.Fe, w.Te, prm, z_w).reshape(n, 5)
    V, W, S = ORACLE[kind].outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sig, prm, z_w)
    with _Plane(ctx, z_w, kind):
        gb = ctx.mbs_rhs(_t(w.R), _t(w.v2s), _t(w.v3t), _t(w.Fe), _t(w.Te))
        gV, gW, gS = ctx.mbs_outputs(_t(w.R), _t(Sig), _t(w.v1s), _t(w.v2s), _t(w.v3t), _t(w.Fe), _t(w.Te))
    assert _maxrel(gb, b) < 1e-13
    assert _maxrel(gV, V) < 1e-13 and _maxrel(gW, W) < 1e-13 and _maxrel(gS, S) < 1e-14


@KINDS
def test_plane_flow_field_matches_oracle_and_meets_the_plane_condition(ctx, kind):
    n, m = 97, 300
    w, z_w = _workload(n, 1600)
    Sig = np.random.default_rng(2).standard_normal((n, 5))
    rng = np.random.default_rng(3)
    side = float(np.ptp(w.R[:, 0])) / 2
    X = np.column_stack([rng.uniform(-side, side, m), rng.uniform(-side, side, m), rng.uniform(z_w, z_w + 2 * side, m)])
    X[:40, 2] = z_w  # points on the plane itself
    want = ORACLE[kind].flow_field(X, w.R, w.Fe, w.Te, Sig, w.v3t, _prm(w), z_w)
    with _Plane(ctx, z_w, kind):
        got = ctx.mbs_flow(_t(X), _t(w.R), _t(Sig), _t(w.Fe), _t(w.Te), _t(w.v3t))
    assert _maxrel(got, want) < 1e-13
    on = _np(got)[:40] if kind == 2 else _np(got)[:40, 2]  # no flow at a wall / through a plane
    assert np.abs(on).max() < 1e-12 * np.abs(want).max()


@KINDS
@pytest.mark.parametrize("precision,near,order,spatial", [
    (mbstokes.MBS_FP64, 0.0, 2, 0), (mbstokes.MBS_FP64, 8.0, 2, 1), (mbstokes.MBS_MIXED, 0.0, 2, -1),
    (mbstokes.MBS_MIXED, 12.0, 4, 1)])
def test_plane_solve_matches_oracle(ctx, kind, precision, near, order, spatial):
    print(f"plane {kind} solve precision={precision} near={near} order={order} spatial={spatial}", flush=True)
    n = 257
    w, z_w = _workload(n, 1700)
    sol = ORACLE[kind].solve(w, z_w, _prm(w))
    d = mbstokes.to_device(w, DEV)
    Sig = torch.empty((n, 5), dtype=torch.float64, device=DEV)
    with _Plane(ctx, z_w, kind, tol=1e-12, precision=precision, near_cutoff=near, near_order=order, spatial_order=spatial):
        V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], Sigma=Sig)
        V2, W2, S2, st2 = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    bar = 1e-10 if precision == mbstokes.MBS_FP64 else 1e-9
    for got, want in ((V, sol["V"]), (W, sol["W"]), (S, sol["S"]), (Sig, sol["Sigma"])):
        assert _maxrel(got, want) < bar
    r = sol["b"] - sol["A"] @ _np(Sig).ravel()
    assert np.linalg.norm(r) <= 1.01e-12 * np.linalg.norm(sol["b"])
    assert torch.equal(V, V2) and torch.equal(W, W2)  # the second solve replays the captured steps


@KINDS
def test_plane_superposition_matches_oracle(ctx, kind):
    n = 97
    w, z_w = _workload(n, 1800)
    prm = _prm(w)
    Sig = -galerkin.constants(prm)["gamma"] * w.v2s
    V, W, S = ORACLE[kind].outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sig, prm, z_w)
    d = mbstokes.to_device(w, DEV)
    with _Plane(ctx, z_w, kind, superposition=1):
        gV, gW, gS, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    assert _maxrel(gV, V) < 1e-13 and _maxrel(gW, W) < 1e-13


@KINDS
def test_plane_operator_at_ten_thousand_spheres_sampled_rows(ctx, kind):
    """10^4 spheres in the trap box of side 200, the plane 1.5a below the lowest one: sampled
    receivers against all spheres and all images."""
    n = 10_000
    w, z_w = _workload(n, 1, side=200.0)
    x = np.random.default_rng(5).standard_normal((n, 5))
    with _Plane(ctx, z_w, kind):
        got = _np(ctx.mbs_matvec(_t(w.R), _t(x)))
        got32 = _np(ctx.mbs_matvec(_t(w.R), _t(x), precision=mbstokes.MBS_FP32))
    rows = np.concatenate([np.argsort(w.R[:, 2])[:4], np.random.default_rng(6).choice(n, 12, replace=False)])
    want = ORACLE[kind].matvec_rows(w.R, x, rows, _prm(w), z_w)
    assert _maxrel(got[rows], want) < 1e-12
    assert _maxrel(got32[rows], want) < 2e-6


@pytest.mark.parametrize("n", [257, 1300])
def test_plane_operator_every_launch_shape(ctx, n):
    """The images' part runs in the operator kernel's LDS variant with the context's launch shape
    (64, 128 or 256 records per tile; the streamed shapes fall back to 128): every candidate shape
    agrees with the oracle in both precisions."""
    w, z_w = _workload(n, 2100 + n)
    x = np.random.default_rng(n + 1).standard_normal((n, 5))
    want = (plane.system_matrix(w.R, _prm(w), z_w) @ x.ravel()).reshape(n, 5)
    R, xt = _t(w.R), _t(x)
    count = 0
    with _Plane(ctx, z_w):
        k = 1
        while True:
            try:
                ctx.set_params(tile=k)
            except mbstokes.MbsError:
                break
            print(f"plane matvec n={n} tile={k}", flush=True)
            assert _maxrel(ctx.mbs_matvec(R, xt), want) < 1e-13, k
            assert _maxrel(ctx.mbs_matvec(R, xt, precision=mbstokes.MBS_FP32), want) < 2e-6, k
            count += 1
            k += 1
        ctx.set_params(tile=0)
    assert count >= 8


@KINDS
def test_plane_errors(ctx, kind):
    n = 8
    w, z_w = _workload(n, 1900)
    R, x = _t(w.R), _t(np.ones((n, 5)))
    with _Plane(ctx, w.R[:, 2].min() - 0.5, kind):  # the lowest sphere reaches through the plane
        for call in (lambda: ctx.mbs_matvec(R, x), lambda: ctx.mbs_solve(R, None, _t(w.v1s), _t(w.v2s)),
                     lambda: ctx.mbs_step(R.clone(), _t(w.p), 0.5, (1.0, 1.0, 1.0), 0.01, 1)):
            with pytest.raises(mbstokes.MbsError) as e:
                call()
            assert e.value.code == mbstokes.MBS_EINVAL
    with _Plane(ctx, z_w, kind):
        X = _t(np.array([[0.0, 0.0, z_w - 1.0]]))
        with pytest.raises(mbstokes.MbsError) as e:  # a field point below the plane
            ctx.mbs_flow(X, R, x)
        assert e.value.code == mbstokes.MBS_EINVAL
        refused = [lambda: ctx.mbs_matvec_r3(R, _t(np.ones((n, 20)))),
                   lambda: ctx.mbs_matvec_static(R, x, torch.empty_like(x)),
                   lambda: ctx.mbs_solve_ex(R, None, _t(w.v1s), _t(w.v2s), gam=_t(np.ones((n, 10))))]
        for call in refused:
            with pytest.raises(mbstokes.MbsError) as e:
                call()
            assert e.value.code == mbstokes.MBS_EUNSUPPORTED
    for bad in (3, -1):
        with pytest.raises(mbstokes.MbsError):
            ctx.set_params(plane=bad)
    ctx.set_params(plane=0)


@KINDS
def test_plane_stepper_matches_oracle(ctx, kind):
    """Three Adams-Bashforth steps of trapped swimmers above the plane against the oracle's stepper
    with the half-space solve; min_dist counts each sphere's own image at twice its height."""
    from oracle import stepper
    n = 64
    w, z_w = _workload(n, 2300, lift=1.2)
    prm = _prm(w)
    Rw, pw, _ = stepper.run(w.R, w.p, 0.5, (1.0, 1.0, 1.0), 0.01, 3, prm,
                            solve=lambda st, pr: ORACLE[kind].solve(st, z_w, pr))
    R, p = _t(w.R), _t(w.p)
    with _Plane(ctx, z_w, kind, tol=1e-13):
        stats, md = ctx.mbs_step(R, p, 0.5, (1.0, 1.0, 1.0), 0.01, 3, order=2, want_min_dist=True)
    assert _maxrel(R, Rw) < 1e-12 and _maxrel(p, pw) < 1e-12
    dmin = min(np.linalg.norm(w.R[i] - w.R[j]) for i in range(n) for j in range(i))
    assert abs(md[0] - min(dmin, 2 * (w.R[:, 2].min() - z_w))) < 1e-12


@KINDS
def test_plane_stepper_stops_when_a_sphere_reaches_the_plane(ctx, kind):
    """A lone swimmer heading into the plane with a step long enough to carry its centre through it:
    the first step runs, the second finds the centre below the plane and ends the run with
    MBS_EINVAL; R holds the state after the first step."""
    z_w = -3.0
    R = _t(np.array([[0.0, 0.0, z_w + 1.5]]))
    p = _t(np.array([[0.0, 0.0, -1.0]]))
    with _Plane(ctx, z_w, kind):
        for coef in ((1.0, 0.0, 0.0), (-1.0, 0.0, 0.0)):  # one of the two swims towards the plane
            R1, p1 = R.clone(), p.clone()
            try:
                ctx.mbs_step(R1, p1, 0.0, coef, 20.0, 3, order=1)
            except mbstokes.MbsError as e:
                assert e.code == mbstokes.MBS_EINVAL and "reached the plane" in str(e)
                assert float(R1[0, 2]) <= z_w  # the first step was taken and carried it through
                break
        else:
            raise AssertionError("neither direction reached the plane")

