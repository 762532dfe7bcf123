"""Spheres in a periodic cubic box on the GPU (params.box, Ewald summation): every pass and the solve
against the oracle's periodic system (summed with its own splitting parameter, which the pinned
result does not depend on), the flow at field points, the stepper, Hasimoto's simple cubic
mobility, invariance under shifts by box vectors, and the entry points that refuse the box."""
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
    L = L or max(8.0, (n / 0.004) ** (1 / 3))
    rng = np.random.default_rng(seed + 7)
    R = _place(n, L, seed)
    p = rng.standard_normal((n, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    v1s, v2s, v3t = inputs.slip_modes(p, 1.0, 1.0, 1.0)
    w = inputs.Workload(R, p, v1s, v2s, v3t, rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), ETA, A)
    return w, L


def _ew(L):
    return periodic.Ewald(L, xi=7.0 / L)  # the oracle's own splitting (fewer wave vectors)


@functools.lru_cache(maxsize=None)
def _oracle_solve(n, seed):
    w, L = _workload(n, seed)
    return periodic.solve(w, _ew(L), PRM)


PRM = galerkin.Params(eta=ETA, a=A)


class _Box:
    def __init__(self, ctx, L, **kw):
        self.ctx, self.L, self.kw = ctx, L, kw

    def __enter__(self):
        self.ctx.set_params(box=self.L, **self.kw)
        return self.ctx

    def __exit__(self, *exc):
        self.ctx.set_params(box=0.0, ewald_xi=0.0, tol=1e-10, precision=mbstokes.MBS_FP64, near_cutoff=0.0,
                            near_order=2, superposition=0, spatial_order=0, guess=mbstokes.MBS_GUESS_ZERO)


@pytest.mark.parametrize("n", [1, 2, 97])
def test_periodic_operator_matches_oracle(ctx, n):
    print(f"periodic matvec n={n}", flush=True)
    w, L = _workload(n, 3000 + n)
    x = np.random.default_rng(n).standard_normal((n, 5))
    want = (periodic.system_matrix(w.R, PRM, _ew(L)) @ x.ravel()).reshape(n, 5)
    with _Box(ctx, L):
        got = ctx.mbs_matvec(_t(w.R), _t(x))
        got32 = ctx.mbs_matvec(_t(w.R), _t(x), precision=mbstokes.MBS_FP32)  # binary64 Ewald sums too
    # a sphere's Fourier self sum and its smooth self constant cancel to about an eighth of their size
    # in the smallest box (8a, default splitting), which multiplies their rounding accordingly
    assert _maxrel(got, want) < 2e-12
    assert _maxrel(got32, want) < 2e-12


@pytest.mark.parametrize("n", [1, 2, 97])
def test_periodic_rhs_and_outputs_match_oracle(ctx, n):
    print(f"periodic rhs/outputs n={n}", flush=True)
    w, L = _workload(n, 3100 + n)
    Sig = np.random.default_rng(n + 3).standard_normal((n, 5))
    b = periodic.rhs(w.R, w.v2s, w.v3t, w.Fe, w.Te, PRM, _ew(L)).reshape(n, 5)
    V, W, S = periodic.outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sig, PRM, _ew(L))
    with _Box(ctx, L):
        gb = ctx.mbs_rhs(_t(w.R), _t(w.v2s), _t(w.v3t), _t(w.Fe), _t(w.Te))
        gV, gW, gS = ctx.mbs_outputs(_t(w.R), _t(Sig), _t(w.v1s), _t(w.v2s), _t(w.v3t), _t(w.Fe), _t(w.Te))
    assert _maxrel(gb, b) < 1e-12
    assert _maxrel(gV, V) < 1e-12 and _maxrel(gW, W) < 1e-12 and _maxrel(gS, S) < 1e-14


@pytest.mark.parametrize("precision,near,order,spatial,superposition", [
    (mbstokes.MBS_FP64, 0.0, 2, 0, 0), (mbstokes.MBS_FP64, 8.0, 2, 1, 0), (mbstokes.MBS_MIXED, 8.0, 4, -1, 0),
    (mbstokes.MBS_FP64, 0.0, 2, 0, 1)])
def test_periodic_solve_matches_oracle(ctx, precision, near, order, spatial, superposition):
    print(f"periodic solve precision={precision} near={near} order={order} spatial={spatial} "
          f"superposition={superposition}", flush=True)
    n = 97
    w, L = _workload(n, 3200)
    d = mbstokes.to_device(w, DEV)
    Sig = torch.empty((n, 5), dtype=torch.float64, device=DEV)
    with _Box(ctx, L, tol=1e-12, precision=precision, near_cutoff=near, near_order=order, spatial_order=spatial,
              superposition=superposition):
        V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], Sigma=Sig)
        V2, W2, S2, st2 = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    if superposition:
        Sw = -galerkin.constants(PRM)["gamma"] * w.v2s
        Vw, Ww, _ = periodic.outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sw, PRM, _ew(L))
        assert _maxrel(V, Vw) < 1e-12 and _maxrel(W, Ww) < 1e-12
        return
    sol = _oracle_solve(n, 3200)
    bar = 1e-10 if precision == mbstokes.MBS_FP64 else 1e-9
    for got, want in ((V, sol["V"]), (W, sol["W"]), (S, sol["S"]), (Sig, sol["Sigma"])):
        assert _maxrel(got, want) < bar
    assert torch.equal(V, V2) and torch.equal(W, W2)  # the second solve replays the captured steps


def test_lone_sphere_in_a_periodic_box_moves_as_hasimoto_found_on_the_gpu(ctx):
    """A simple cubic array (one sphere per box) under a force parallel to an edge and along a face
    diagonal: V = mu0 F (1 - 2.8372974795 a/L + (4 pi/3)(a/L)^3) (Hasimoto), for the library's own
    splitting and for a larger one."""
    mu0 = 1 / (6 * np.pi * ETA * A)
    for L in (8.0, 20.0):
        e = A / L
        want = 1 - 2.8372974795 * e + 4 * np.pi / 3 * e ** 3
        for xi in (0.0, 20.0 / L):
            with _Box(ctx, L, ewald_xi=xi):
                for F in ([1.0, 0.0, 0.0], [0.0, 0.6, 0.8]):
                    V, W, S, st = ctx.mbs_solve(_t([[0.3, -1.1, 2.0]]), None, None, None, None, _t([F]), None)
                    assert np.abs(_np(V)[0] / mu0 - want * np.array(F)).max() < 1e-10


def test_periodic_results_do_not_change_under_box_shifts(ctx):
    """Shifting every sphere by the same vector, or single spheres by box vectors, changes nothing."""
    n = 64
    w, L = _workload(n, 3300)
    x = np.random.default_rng(9).standard_normal((n, 5))
    R2 = w.R + np.array([0.37, -2.1, 5.3])
    R3 = w.R.copy()
    R3[::3] += L * np.array([1.0, -2.0, 3.0])
    with _Box(ctx, L):
        y1 = _np(ctx.mbs_matvec(_t(w.R), _t(x)))
        y2 = _np(ctx.mbs_matvec(_t(R2), _t(x)))
        y3 = _np(ctx.mbs_matvec(_t(R3), _t(x)))
    assert np.abs(y2 - y1).max() < 1e-12 * np.abs(y1).max()
    assert np.abs(y3 - y1).max() < 1e-12 * np.abs(y1).max()


def test_periodic_operator_sampled_rows_at_a_thousand_spheres(ctx):
    n = 1000
    w, L = _workload(n, 3400)
    x = np.random.default_rng(11).standard_normal((n, 5))
    with _Box(ctx, L):
        got = _np(ctx.mbs_matvec(_t(w.R), _t(x)))
    rows = np.random.default_rng(12).choice(n, 5, replace=False)
    want = periodic.matvec_rows(w.R, x, rows, PRM, _ew(L))
    assert _maxrel(got[rows], want) < 1e-12


def test_periodic_flow_field_matches_oracle(ctx):
    n, m = 97, 240
    w, L = _workload(n, 3600)
    Sig = np.random.default_rng(21).standard_normal((n, 5))
    X = np.random.default_rng(22).uniform(-0.5 * L, 1.5 * L, (m, 3))  # anywhere: taken modulo the box
    want = periodic.flow_field(X, w.R, w.Fe, w.Te, Sig, w.v3t, PRM, _ew(L))
    with _Box(ctx, L):
        got = ctx.mbs_flow(_t(X), _t(w.R), _t(Sig), _t(w.Fe), _t(w.Te), _t(w.v3t))
    assert _maxrel(got, want) < 1e-12


def test_periodic_stepper_matches_oracle(ctx):
    """Force-free swimmers (no trap, slip modes 1, 1, 1 along p) stepped three times in the box
    against the oracle's stepper on the periodic solve; min_dist is the smallest minimum-image
    distance."""
    from oracle import stepper
    n = 24
    w, L = _workload(n, 3700, L=14.0)
    Rw, pw, _ = stepper.run(w.R, w.p, 0.0, (1.0, 1.0, 1.0), 0.05, 3, PRM,
                            solve=lambda st, pr: periodic.solve(st, _ew(L), pr))
    R, p = _t(w.R), _t(w.p)
    with _Box(ctx, L, tol=1e-13):
        stats, md = ctx.mbs_step(R, p, 0.0, (1.0, 1.0, 1.0), 0.05, 3, order=2, want_min_dist=True)
    assert _maxrel(R, Rw) < 1e-11 and _maxrel(p, pw) < 1e-11
    d = w.R[:, None, :] - w.R[None, :, :]
    d -= L * np.round(d / L)
    dist = np.sqrt((d ** 2).sum(-1)) + np.eye(n) * 1e9
    assert abs(md[0] - dist.min()) < 1e-12


def test_periodic_errors(ctx):
    n = 8
    w, L = _workload(n, 3500)
    R, x = _t(w.R), _t(np.ones((n, 5)))
    with pytest.raises(mbstokes.MbsError) as e:
        ctx.set_params(box=L, ewald_xi=10.0 / L)  # real-space cutoff beyond L/2
    assert e.value.code == mbstokes.MBS_EINVAL
    with pytest.raises(mbstokes.MbsError) as e:
        ctx.set_params(box=L, ewald_xi=0.0, plane=1)
    assert e.value.code == mbstokes.MBS_EINVAL
    ctx.set_params(box=0.0, plane=0, ewald_xi=0.0)
    with _Box(ctx, L):
        refused = [lambda: ctx.mbs_matvec_r3(R, _t(np.ones((n, 20)))),
                   lambda: ctx.mbs_matvec_static(R, x, torch.empty_like(x)),
                   lambda: ctx.mbs_solve_ex(R, None, _t(w.v1s), _t(w.v2s), gam=_t(np.ones((n, 10))))]
        for call in refused:
            with pytest.raises(mbstokes.MbsError) as e:
                call()
            assert e.value.code == mbstokes.MBS_EUNSUPPORTED
