"""Solves in the Morton order of the centres (params.spatial_order = 1, forced here at sizes the
oracle solves densely; by default it applies from n = 65536 on) against the oracle, against the
same solve in the caller's order (spatial_order = -1), and under graph replays and time stepping.
Outputs always come back in the caller's order.

Inputs: the trap workloads of the parity tests (seeded, density 0.004, torque and the rank-3 mode
included), 700 spheres = three workgroups of 256 receivers with a ragged last one.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import galerkin, stepper  # noqa: E402
from paper_1411_0278_amd import inputs, mbstokes  # noqa: E402

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def _rel(got, want):
    got = got.detach().cpu().numpy() if hasattr(got, "detach") else np.asarray(got)
    want = want.detach().cpu().numpy() if hasattr(want, "detach") else np.asarray(want)
    return np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)


def _workload(n, seed):
    w = inputs.trap_workload(n, max(8.0, (n / 0.004) ** (1 / 3)), seed, v3t=1.0)
    w.Te = np.random.default_rng(seed + 99).standard_normal((n, 3))
    return w


@pytest.fixture(scope="module")
def ctx():
    c = mbstokes.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def case():
    w = _workload(700, seed=71)
    return w, galerkin.solve(w)


METHODS = {  # params, bar against the oracle, bar between the two orders
    "fp64": (dict(precision=mbstokes.MBS_FP64, tol=1e-12), 1e-10, 1e-11),
    "mixed_pc": (dict(precision=mbstokes.MBS_MIXED, tol=1e-11, near_cutoff=8.0, near_order=4), 1e-9, 1e-9),
    "user_guess": (dict(precision=mbstokes.MBS_FP64, tol=1e-12, guess=mbstokes.MBS_GUESS_USER, restart=5), 1e-10,
                   1e-11),
}
RESET = dict(precision=mbstokes.MBS_FP64, tol=1e-10, near_cutoff=0.0, near_order=2, guess=mbstokes.MBS_GUESS_ZERO,
             restart=30, spatial_order=0, superposition=0)


@pytest.mark.parametrize("method", list(METHODS))
def test_ordered_solve_matches_oracle_and_caller_order(ctx, case, method):
    w, ref = case
    prm, bar, bar_orders = METHODS[method]
    print(f"spatial order solve {method}", flush=True)
    d = mbstokes.to_device(w, DEV)
    s0 = None
    if method == "user_guess":
        s0 = _t(ref["Sigma"] * (1 + 1e-3 * np.random.default_rng(0).standard_normal(ref["Sigma"].shape)))
    out, stats = {}, {}
    args = (d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    try:
        for order in (1, -1):
            ctx.set_params(spatial_order=order, **prm)
            Sig = torch.empty((w.n, 5), dtype=torch.float64, device=DEV)
            V, W, S, st = ctx.mbs_solve(*args, sigma0=s0, Sigma=Sig)
            out[order], stats[order] = (V, W, S, Sig), st
            assert st["rel_resid"] <= prm["tol"], (order, st)
        if method == "user_guess":  # read in the caller's order, the close guess saves iterations
            ctx.set_params(spatial_order=1, **dict(prm, guess=mbstokes.MBS_GUESS_ZERO))
            _, _, _, st0 = ctx.mbs_solve(*args)
            assert stats[1]["iters"] < st0["iters"], (stats[1]["iters"], st0["iters"])
    finally:
        ctx.set_params(**RESET)
    for k, key in enumerate(("V", "W", "S", "Sigma")):
        assert _rel(out[1][k], ref[key]) < bar, key
        assert _rel(out[1][k], out[-1][k]) < bar_orders, key


def test_ordered_superposition_matches_oracle(ctx, case):
    w, _ = case
    ref = galerkin.superposition(w, galerkin.Params(eta=w.eta, a=w.a))
    d = mbstokes.to_device(w, DEV)
    ctx.set_params(spatial_order=1, superposition=1)
    try:
        V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    finally:
        ctx.set_params(**RESET)
    for got, key in ((V, "V"), (W, "W"), (S, "S")):
        assert _rel(got, ref[key]) < 1e-13, key


@pytest.mark.parametrize("precision", [mbstokes.MBS_FP64, mbstokes.MBS_MIXED])
def test_ordered_graph_replays_equal_eager_solves(ctx, case, precision):
    """Captured Arnoldi steps read the reordered copies at replay time: every replay equals the
    eager ordered solve bit for bit, also after a solve of other positions of the same size."""
    w, _ = case
    print(f"spatial order graph replays precision={precision}", flush=True)
    d = mbstokes.to_device(w, DEV)
    other = mbstokes.to_device(_workload(700, seed=72), DEV)
    args = (d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    oargs = (other["R"], other["p"], other["v1s"], other["v2s"], other["v3t"], other["Fe"], other["Te"])
    ctx.set_params(spatial_order=1, graph=0, precision=precision, near_cutoff=6.0, tol=1e-12,
                   guess=mbstokes.MBS_GUESS_DIAG, restart=6)
    try:
        V0, W0, S0, st0 = ctx.mbs_solve(*args)
        Vo0, _, _, _ = ctx.mbs_solve(*oargs)
        ctx.set_params(graph=1)
        for rep in range(4):  # new key (eager), then capture, then replays; the other set in between
            V, W, S, st = ctx.mbs_solve(*args)
            torch.cuda.synchronize()
            assert torch.equal(V, V0) and torch.equal(W, W0) and torch.equal(S, S0), rep
            assert st["iters"] == st0["iters"] and st["rel_resid"] == st0["rel_resid"], rep
            Vo, _, _, _ = ctx.mbs_solve(*oargs)
            assert torch.equal(Vo, Vo0), rep
    finally:
        ctx.set_params(graph=1, **RESET)


def test_ordered_stepper_matches_oracle(ctx):
    w = _workload(300, seed=14)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    Rw, pw, _ = stepper.run(w.R, w.p, 0.5, (1.0, 1.0, 1.0), 0.01, 3, prm)
    R, p = _t(w.R), _t(w.p)
    ctx.set_params(spatial_order=1, tol=1e-13)
    try:
        ctx.mbs_step(R, p, 0.5, (1.0, 1.0, 1.0), 0.01, 3, order=2)
    finally:
        ctx.set_params(**RESET)
    assert _rel(R, Rw) < 1e-12 and _rel(p, pw) < 1e-12


def test_ordered_solve_with_higher_modes_matches_oracle(ctx):
    w = inputs.config0()
    w.gam, w.psi, w.lam = inputs.higher_slip_modes(w.p, 0.8, -0.6, 0.5)
    ref = galerkin.solve(w, galerkin.Params(eta=w.eta, a=w.a))
    d = mbstokes.to_device(w, DEV)
    ctx.set_params(spatial_order=1, precision=mbstokes.MBS_MIXED, tol=1e-11, near_cutoff=8.0)
    try:
        V, W, S, st = ctx.mbs_solve_ex(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], gam=d["gam"], psi=d["psi"],
                                       lam=d["lam"], Fe=d["Fe"], Te=d["Te"])
    finally:
        ctx.set_params(**RESET)
    for got, key in ((V, "V"), (W, "W"), (S, "S")):
        assert _rel(got, ref[key]) < 1e-9, key


@pytest.mark.parametrize("shape", ["line", "plane"])
def test_ordered_solve_on_degenerate_geometries(ctx, shape):
    """Centres on a line or in a plane (the cell grid is flat in two or one axes), in a shuffled
    order: the ordered solve equals the oracle and the caller-order solve."""
    rng = np.random.default_rng(5)
    if shape == "line":
        R = np.stack([2.5 * np.arange(300.0), np.zeros(300), np.zeros(300)], axis=1)
    else:
        gx, gy = np.meshgrid(np.arange(18.0) * 2.5, np.arange(18.0) * 2.5, indexing="ij")
        R = np.stack([gx, gy, np.zeros_like(gx)], axis=-1).reshape(-1, 3)
    R = R[rng.permutation(len(R))]
    n = len(R)
    p = rng.standard_normal((n, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    v1s, v2s, v3 = inputs.slip_modes(p, 1.0, 1.0, 0.0)
    w = inputs.Workload(R, p, v1s, v2s, v3, -0.5 * R, np.zeros((n, 3)))
    ref = galerkin.solve(w)
    d = mbstokes.to_device(w, DEV)
    out = {}
    try:
        for order in (1, -1):
            ctx.set_params(spatial_order=order, tol=1e-12)
            out[order] = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)[:3]
    finally:
        ctx.set_params(**RESET)
    for k, key in enumerate(("V", "W", "S")):
        assert _rel(out[1][k], ref[key]) < 1e-10, key
        assert _rel(out[1][k], out[-1][k]) < 1e-11, key


@pytest.mark.slow
def test_stepper_at_benchmark_size_orders_by_default(ctx):
    """N = 10^5 (the benchmark workload): the stepper's solves reorder automatically (n >= 65536);
    two mixed preconditioned steps give the positions and orientations of the same steps in the
    caller's order to the solve tolerance, and every step converges."""
    w = inputs.config2()
    out = {}
    try:
        for order in (0, -1):
            ctx.set_params(spatial_order=order, precision=mbstokes.MBS_MIXED, near_cutoff=8.0, tol=1e-10)
            R, p = _t(w.R), _t(w.p)
            stats, _ = ctx.mbs_step(R, p, 0.5, (1.0, 1.0, 0.0), 0.01, 2, order=2)
            assert all(st["rel_resid"] <= 1e-10 for st in stats), (order, stats)
            out[order] = (R.cpu().numpy(), p.cpu().numpy())
    finally:
        ctx.set_params(**RESET)
    disp = np.linalg.norm(out[-1][0] - w.R)
    assert disp > 0
    assert np.linalg.norm(out[0][0] - out[-1][0]) <= 1e-8 * disp
    assert _rel(out[0][1], out[-1][1]) < 1e-10


def test_spatial_order_is_validated(ctx):
    for bad in (2, -2):
        with pytest.raises(mbstokes.MbsError):
            ctx.set_params(spatial_order=bad)
    ctx.params.spatial_order = 0
