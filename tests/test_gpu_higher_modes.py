"""GPU parity of the higher slip modes of the minimal truncation (septlet gamma, vortlet psi,
spinlet lambda; fixed sources) against the oracle, through the C ABI (mbs_*_ex).

Inputs: the benchmark-style trap workloads plus seeded Gaussian gamma [n, 10], psi [n, 5],
lambda [n, 10] (rank-3 tensors given by their 10 symmetric components, not traceless: both sides
use the traceless part), or the uniaxial modes along the orientations.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import galerkin  # noqa: E402
from paper_1411_0278_amd import inputs, mbstokes  # noqa: E402

DEV = "cuda:0"
MASKS = [1, 2, 4, 3, 5, 6, 7]  # bit 0 gamma, bit 1 psi, bit 2 lambda


def _t(a):
    return None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def _maxrel(got, want):
    got = got.detach().cpu().numpy() if hasattr(got, "detach") else np.asarray(got)
    return np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)


def _rel(got, want):
    got = got.detach().cpu().numpy() if hasattr(got, "detach") else np.asarray(got)
    return np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)


@pytest.fixture(scope="module")
def ctx():
    c = mbstokes.Context(0)
    yield c
    c.close()


def _workload(n, seed, mask, torque=True):
    side = max(8.0, (n / 0.004) ** (1 / 3))
    w = inputs.trap_workload(n, side, seed, v3t=1.0)
    rng = np.random.default_rng(seed + 7)
    if torque:
        w.Te = rng.standard_normal((n, 3))
    w.gam = rng.standard_normal((n, 10)) if mask & 1 else None
    w.psi = rng.standard_normal((n, 5)) if mask & 2 else None
    w.lam = rng.standard_normal((n, 10)) if mask & 4 else None
    return w


def _modes(w):
    return dict(gam=_t(w.gam), psi=_t(w.psi), lam=_t(w.lam))


@pytest.mark.parametrize("mask", MASKS)
@pytest.mark.parametrize("n", [1, 2, 67, 300])
def test_rhs_ex_matches_oracle(ctx, n, mask):
    print(f"rhs_ex n={n} mask={mask}", flush=True)
    w = _workload(n, 1300 + n, mask)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    want = galerkin.rhs(w.R, w.v2s, w.v3t, w.Fe, w.Te, prm, modes=galerkin.workload_modes(w)).reshape(n, 5)
    got = ctx.mbs_rhs_ex(_t(w.R), _t(w.v2s), _t(w.v3t), Fe=_t(w.Fe), Te=_t(w.Te), **_modes(w))
    assert _maxrel(got, want) < 1e-13


@pytest.mark.parametrize("mask", MASKS)
@pytest.mark.parametrize("n", [1, 2, 67, 300])
def test_outputs_ex_match_oracle(ctx, n, mask):
    print(f"outputs_ex n={n} mask={mask}", flush=True)
    w = _workload(n, 1400 + n, mask)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    Sig = np.random.default_rng(n + mask).standard_normal((n, 5))
    V, W, S = galerkin.outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sig, prm, modes=galerkin.workload_modes(w))
    gV, gW, gS = ctx.mbs_outputs_ex(_t(w.R), _t(Sig), _t(w.v1s), _t(w.v2s), _t(w.v3t), Fe=_t(w.Fe), Te=_t(w.Te),
                                    **_modes(w))
    assert _maxrel(gV, V) < 1e-13
    assert _maxrel(gW, W) < 1e-13
    assert _maxrel(gS, S) < 1e-14


def _field_points(R, m, seed, a=1.0):
    rng = np.random.default_rng(seed)
    lo, hi = R.min(0) - 3.0, R.max(0) + 3.0
    pts = []
    while len(pts) < m:
        X = rng.uniform(lo, hi, (2 * m, 3))
        D = np.linalg.norm(X[:, None] - R[None], axis=2).min(1)
        pts.extend(X[D > 1.05 * a])
    return np.array(pts[:m])


@pytest.mark.parametrize("mask", [1, 2, 4, 7])
@pytest.mark.parametrize("n,m", [(1, 5), (67, 300), (300, 129)])
def test_flow_ex_matches_oracle(ctx, n, m, mask):
    print(f"flow_ex n={n} m={m} mask={mask}", flush=True)
    w = _workload(n, 1500 + n, mask)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    Sig = np.random.default_rng(n + m).standard_normal((n, 5))
    X = _field_points(w.R, m, seed=m + mask)
    want = galerkin.flow_field(X, w.R, w.Fe, w.Te, Sig, w.v3t, prm, modes=galerkin.workload_modes(w))
    got = ctx.mbs_flow_ex(_t(X), _t(w.R), _t(Sig), Fe=_t(w.Fe), Te=_t(w.Te), v3t=_t(w.v3t), **_modes(w))
    assert _maxrel(got, want) < 1e-13


def test_flow_ex_on_a_lone_sphere_is_its_slip(ctx):
    """On the surface of a lone sphere with only the higher modes, the GPU flow equals the slip
    fields (a^2/2) gamma:nn - (a^2/3) n x (psi.n) - (a^3/8) n x (lambda:nn)."""
    from tests import sphere_quad
    rng = np.random.default_rng(17)
    a = 1.0
    R = np.array([[0.3, -1.2, 2.0]])
    gam, psi, lam = rng.standard_normal((1, 10)), rng.standard_normal((1, 5)), rng.standard_normal((1, 10))
    nh, _ = sphere_quad.sphere_rule(8, 16)
    X = R[0] + a * nh
    got = ctx.mbs_flow_ex(_t(X), _t(R), _t(np.zeros((1, 5))), gam=_t(gam), psi=_t(psi), lam=_t(lam)).cpu().numpy()

    def stf(c):
        import itertools
        idx = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2), (1, 2, 2),
               (2, 2, 2)]
        T = np.zeros((3, 3, 3))
        for q, ix in enumerate(idx):
            for p in itertools.permutations(ix):
                T[p] = c[q]
        t = np.einsum("iik->k", T)
        d = np.eye(3)
        return T - (np.einsum("ij,k->ijk", d, t) + np.einsum("ik,j->ijk", d, t) + np.einsum("jk,i->ijk", d, t)) / 5

    from oracle import basis
    G, L, Ps = stf(gam[0]), stf(lam[0]), basis.from5(psi[0])
    want = (a ** 2 / 2 * np.einsum("ijk,pj,pk->pi", G, nh, nh) - a ** 2 / 3 * np.cross(nh, nh @ Ps.T)
            - a ** 3 / 8 * np.cross(nh, np.einsum("ijk,pj,pk->pi", L, nh, nh)))
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("method", ["fp64", "mixed_pc", "superposition"])
def test_solve_ex_matches_oracle(ctx, method):
    """Config-0-sized trap workload with the uniaxial higher modes along the orientations."""
    print(f"solve_ex {method}", flush=True)
    w = inputs.config0()
    w.gam, w.psi, w.lam = inputs.higher_slip_modes(w.p, 0.8, -0.6, 0.5)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    ref = galerkin.superposition(w, prm) if method == "superposition" else galerkin.solve(w, prm)
    d = mbstokes.to_device(w, DEV)
    if method == "fp64":
        ctx.set_params(precision=mbstokes.MBS_FP64, tol=1e-12)
        bar = 1e-10
    elif method == "mixed_pc":
        ctx.set_params(precision=mbstokes.MBS_MIXED, tol=1e-11, near_cutoff=8.0)
        bar = 1e-9
    else:
        ctx.set_params(superposition=1)
        bar = 1e-13
    try:
        Sig = torch.empty((w.n, 5), dtype=torch.float64, device=DEV)
        V, W, S, st = ctx.mbs_solve_ex(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], gam=d["gam"], psi=d["psi"],
                                       lam=d["lam"], Fe=d["Fe"], Te=d["Te"], Sigma=Sig)
    finally:
        ctx.set_params(precision=mbstokes.MBS_FP64, tol=1e-10, near_cutoff=0.0, superposition=0)
    errs = {k: _rel(g, ref[k]) for k, g in (("V", V), ("W", W), ("S", S), ("Sigma", Sig))}
    print(f"  errors {errs}", flush=True)
    assert all(e < bar for e in errs.values()), errs
    # the modes change the answer: without them the motion differs at a visible level
    V0, W0, _, _ = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    assert _rel(W0, ref["W"]) > 1e-6


def test_solve_ex_without_modes_is_mbs_solve(ctx):
    w = inputs.config0()
    d = mbstokes.to_device(w, DEV)
    a = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    b = ctx.mbs_solve_ex(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], Fe=d["Fe"], Te=d["Te"])
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)


def test_ex_rejects_non_finite_modes(ctx):
    w = inputs.config0()
    d = mbstokes.to_device(w, DEV)
    gam = torch.zeros((w.n, 10), dtype=torch.float64, device=DEV)
    gam[5, 3] = float("nan")
    with pytest.raises(mbstokes.MbsError):
        ctx.mbs_solve_ex(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], gam=gam, Fe=d["Fe"])
