"""Parity of the HIP path (through the C ABI) with the CPU oracle, on seeded synthetic inputs.

Tolerances:
* binary64 pair passes (matvec, right-hand side, outputs): the two sides sum the same O(N)
  terms in different orders and with fused multiply-adds; the error is a few ulps of the sum
  of |terms|, so 1e-13 relative (max-norm) is used.
* binary64 solve: ||X_gpu - X_oracle||_F / ||X_oracle||_F <= 1e-10 per output X in
  {V, Omega, S, Sigma} with the GMRES tolerance 1e-12 (condition number ~1.8).
* binary32 pair blocks: unit roundoff 6e-8; each block is a product of ~10 rounded factors
  and the receiver sum cancels partially (measured 1-4e-7 at these sizes), so 2e-6 normwise
  relative is used.
* mixed-precision solve: 1e-9 per output (binary64 residual 1e-11).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import galerkin, krylov, stepper  # noqa: E402
from paper_1411_0278_amd import inputs, mbstokes  # noqa: E402

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def _rel(got, want):
    got = got.detach().cpu().numpy() if hasattr(got, "detach") else np.asarray(got)
    return np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)


def _maxrel(got, want):
    got = got.detach().cpu().numpy() if hasattr(got, "detach") else np.asarray(got)
    return np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)


@pytest.fixture(scope="module")
def ctx():
    c = mbstokes.Context(0)
    yield c
    c.close()


def _workload(n, seed, v3t=1.0, torque=True):
    side = max(8.0, (n / 0.004) ** (1 / 3))
    w = inputs.trap_workload(n, side, seed, v3t=v3t)
    if torque:
        w.Te = np.random.default_rng(seed + 99).standard_normal((n, 3))
    return w


SIZES = [1, 2, 3, 63, 255, 256, 257, 700]


@pytest.mark.parametrize("n", SIZES)
def test_matvec_f64_matches_oracle(ctx, n):
    print(f"matvec_f64 n={n}", flush=True)
    w = _workload(n, seed=100 + n)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    x = np.random.default_rng(n).standard_normal((n, 5))
    A = galerkin.system_matrix(w.R, prm)
    want = (A @ x.ravel()).reshape(n, 5)
    got = ctx.mbs_matvec(_t(w.R), _t(x))
    assert _maxrel(got, want) < 1e-13


@pytest.mark.parametrize("n", [2, 257, 700])
def test_matvec_f32_matches_oracle(ctx, n):
    print(f"matvec_f32 n={n}", flush=True)
    w = _workload(n, seed=200 + n)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    x = np.random.default_rng(n).standard_normal((n, 5))
    want = (galerkin.system_matrix(w.R, prm) @ x.ravel()).reshape(n, 5)
    got = ctx.mbs_matvec(_t(w.R), _t(x), precision=mbstokes.MBS_FP32)
    assert _rel(got, want) < 2e-6


def _tiles(ctx):
    k = 1
    while True:
        try:
            ctx.set_params(tile=k)
        except mbstokes.MbsError:
            break
        yield k
        k += 1
    ctx.set_params(tile=0)


@pytest.mark.parametrize("n", [257, 1300])
def test_matvec_every_launch_shape(ctx, n):
    """Every candidate shape of the autotuner (LDS tiles, scalar streaming, splits) agrees."""
    w = _workload(n, seed=600 + n)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    x = np.random.default_rng(n).standard_normal((n, 5))
    want = (galerkin.system_matrix(w.R, prm) @ x.ravel()).reshape(n, 5)
    R, xt = _t(w.R), _t(x)
    count = 0
    for k in _tiles(ctx):
        print(f"matvec n={n} tile={k}", flush=True)
        assert _maxrel(ctx.mbs_matvec(R, xt), want) < 1e-13, k
        e32 = _rel(ctx.mbs_matvec(R, xt, precision=mbstokes.MBS_FP32), want)
        print(f"  binary32 error {e32:.2e}", flush=True)
        assert e32 < 2e-6, k
        count += 1
    assert count >= 8


def test_autotune_and_cache(ctx, tmp_path):
    w = _workload(2000, seed=17)
    R = _t(w.R)
    cache = str(tmp_path / "tiles.json")
    a = ctx.mbs_autotune(R, cache)
    b = ctx.mbs_autotune(R, cache)  # served from the cache
    assert a == b
    x = _t(np.random.default_rng(2).standard_normal((w.n, 5)))
    want = (galerkin.system_matrix(w.R, galerkin.Params()) @ x.cpu().numpy().ravel()).reshape(w.n, 5)
    assert _maxrel(ctx.mbs_matvec(R, x), want) < 1e-13


def test_matvec_is_bitwise_deterministic(ctx):
    w = _workload(1500, seed=5)
    x = _t(np.random.default_rng(1).standard_normal((w.n, 5)))
    R = _t(w.R)
    y1 = ctx.mbs_matvec(R, x).clone()
    y2 = ctx.mbs_matvec(R, x).clone()
    assert torch.equal(y1, y2)


@pytest.mark.parametrize("n", [1, 2, 255, 257, 700])
def test_rhs_matches_oracle(ctx, n):
    print(f"rhs n={n}", flush=True)
    w = _workload(n, seed=300 + n)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    want = galerkin.rhs(w.R, w.v2s, w.v3t, w.Fe, w.Te, prm).reshape(n, 5)
    got = ctx.mbs_rhs(_t(w.R), _t(w.v2s), _t(w.v3t), _t(w.Fe), _t(w.Te))
    assert _maxrel(got, want) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 255, 257, 700])
def test_outputs_match_oracle(ctx, n):
    print(f"outputs n={n}", flush=True)
    w = _workload(n, seed=400 + n)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    Sig = np.random.default_rng(n).standard_normal((n, 5))
    V, W, S = galerkin.outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, Sig, prm)
    gV, gW, gS = ctx.mbs_outputs(_t(w.R), _t(Sig), _t(w.v1s), _t(w.v2s), _t(w.v3t), _t(w.Fe), _t(w.Te))
    assert _maxrel(gV, V) < 1e-13
    assert _maxrel(gW, W) < 1e-13
    assert _maxrel(gS, S) < 1e-14


def _field_points(R, m, seed, a=1.0):
    """m points spread over the spheres' box, none inside a sphere."""
    rng = np.random.default_rng(seed)
    lo, hi = R.min(0) - 3.0, R.max(0) + 3.0
    pts = []
    while len(pts) < m:
        X = rng.uniform(lo, hi, (2 * m, 3))
        D = np.linalg.norm(X[:, None] - R[None], axis=2).min(1)
        pts.extend(X[D > 1.05 * a])
    return np.array(pts[:m])


@pytest.mark.parametrize("n,m", [(1, 1), (2, 257), (300, 1000), (700, 64)])
@pytest.mark.parametrize("full", [False, True])
def test_flow_field_matches_oracle(ctx, n, m, full):
    print(f"flow field n={n} m={m} full={full}", flush=True)
    w = _workload(n, seed=950 + n, v3t=1.0 if full else 0.0, torque=full)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    Sig = np.random.default_rng(n + m).standard_normal((n, 5))
    X = _field_points(w.R, m, seed=m)
    Te, v3t = (w.Te, w.v3t) if full else (None, None)
    want = galerkin.flow_field(X, w.R, w.Fe, Te, Sig, v3t, prm)
    got = ctx.mbs_flow(_t(X), _t(w.R), _t(Sig), Fe=_t(w.Fe), Te=_t(Te) if full else None,
                       v3t=_t(v3t) if full else None)
    assert _maxrel(got, want) < 1e-13


def test_flow_field_of_a_solution_meets_the_sphere_velocity(ctx):
    """On a sphere's surface the flow of the solved suspension averages to the sphere's V - V^a
    (the weak Dirichlet condition of the l = 0 mode), here with the GPU solve and the GPU flow."""
    w = _workload(40, seed=961, v3t=1.0, torque=True)
    d = mbstokes.to_device(w, DEV)
    ctx.set_params(tol=1e-13)
    try:
        Sig = torch.empty((w.n, 5), dtype=torch.float64, device=DEV)
        V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], Sigma=Sig)
    finally:
        ctx.set_params(tol=1e-10)
    from tests import sphere_quad
    nh, wq = sphere_quad.sphere_rule(48, 96)
    i = 7
    pts = w.R[i] + w.a * nh
    u = ctx.mbs_flow(_t(pts), d["R"], Sig, Fe=d["Fe"], Te=d["Te"], v3t=d["v3t"]).cpu().numpy()
    mean, _ = sphere_quad.coefficients(u, nh, wq, w.a)
    want = V.cpu().numpy()[i] + w.v1s[i]
    assert np.abs(mean - want).max() < 1e-9 * np.abs(u).max()


def test_null_optional_inputs_mean_zero(ctx):
    w = _workload(40, seed=7, v3t=0.0, torque=False)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    want = galerkin.rhs(w.R, w.v2s, w.v3t, np.zeros_like(w.Fe), w.Te, prm).reshape(w.n, 5)
    got = ctx.mbs_rhs(_t(w.R), _t(w.v2s), None, None, None)
    assert _maxrel(got, want) < 1e-13


@pytest.mark.parametrize("guess", [mbstokes.MBS_GUESS_ZERO, mbstokes.MBS_GUESS_DIAG])
def test_solve_config0_fp64(ctx, guess):
    print(f"solve cfg0 fp64 guess={guess}", flush=True)
    w = inputs.config0()
    ref = galerkin.solve(w)
    ctx.set_params(tol=1e-12, precision=mbstokes.MBS_FP64, guess=guess)
    d = mbstokes.to_device(w, DEV)
    Sig = torch.empty((w.n, 5), dtype=torch.float64, device=DEV)
    V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], Sigma=Sig)
    for got, want in ((V, ref["V"]), (W, ref["W"]), (S, ref["S"]), (Sig, ref["Sigma"])):
        assert _rel(got, want) < 1e-10
    assert st["rel_resid"] <= 1e-12 and st["iters"] < 30
    assert st["out_fused"] == 1  # the verified final residual also produced the outputs
    ctx.set_params(tol=1e-10, guess=mbstokes.MBS_GUESS_ZERO)


def test_solve_mixed_precision(ctx):
    w = _workload(300, seed=11)
    ref = galerkin.solve(w)
    ctx.set_params(tol=1e-11, precision=mbstokes.MBS_MIXED, inner_tol=1e-5)
    d = mbstokes.to_device(w, DEV)
    Sig = torch.empty((w.n, 5), dtype=torch.float64, device=DEV)
    V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], Sigma=Sig)
    ctx.set_params(tol=1e-10, precision=mbstokes.MBS_FP64)
    for got, want in ((V, ref["V"]), (W, ref["W"]), (S, ref["S"]), (Sig, ref["Sigma"])):
        assert _rel(got, want) < 1e-9
    assert st["rel_resid"] <= 1e-11 and st["refinements"] >= 1 and st["fp32_matvecs"] > 0


@pytest.mark.parametrize("precision", [mbstokes.MBS_FP64, mbstokes.MBS_MIXED])
@pytest.mark.parametrize("torque", [False, True])
def test_fused_final_pass_matches_separate_passes(ctx, precision, torque):
    """The final residual fused with the output pass: its outputs equal the separate output pass on
    the returned stresslet, and the reported residual equals b - A Sigma formed from the separate
    right-hand side and operator passes."""
    print(f"fused final pass precision={precision} torque={torque}", flush=True)
    w = _workload(500, seed=31, torque=torque)
    d = mbstokes.to_device(w, DEV)
    ctx.set_params(tol=1e-10, precision=precision, guess=mbstokes.MBS_GUESS_DIAG)
    try:
        Sig = torch.empty((w.n, 5), dtype=torch.float64, device=DEV)
        V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], Sigma=Sig)
    finally:
        ctx.set_params(precision=mbstokes.MBS_FP64, guess=mbstokes.MBS_GUESS_ZERO)
    assert st["out_fused"] == 1
    gV, gW, gS = ctx.mbs_outputs(d["R"], Sig, d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    assert _maxrel(V, gV.cpu().numpy()) < 1e-13
    assert _maxrel(W, gW.cpu().numpy()) < 1e-13
    assert _maxrel(S, gS.cpu().numpy()) < 1e-14
    b = ctx.mbs_rhs(d["R"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    r = b - ctx.mbs_matvec(d["R"], Sig)
    rel = float(r.norm() / b.norm())
    assert abs(rel - st["rel_resid"]) <= 1e-3 * rel + 1e-15


@pytest.mark.parametrize("precision", [mbstokes.MBS_FP64, mbstokes.MBS_MIXED])
@pytest.mark.parametrize("near_cutoff,near_order", [(0.0, 2), (6.0, 2), (10.0, 4)])
def test_solve_graph_replays_equal_eager_solves(ctx, precision, near_cutoff, near_order):
    """Small systems replay captured Arnoldi steps from the second solve of one configuration on:
    every replay (with other work and synchronisations in between) equals the eager solve bit for
    bit."""
    print(f"graph replays precision={precision} near_cutoff={near_cutoff}", flush=True)
    w = _workload(700, seed=41)
    d = mbstokes.to_device(w, DEV)
    args = (d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    ctx.set_params(graph=0, precision=precision, near_cutoff=near_cutoff, tol=1e-12,
                   guess=mbstokes.MBS_GUESS_DIAG, restart=6, near_order=near_order)
    try:
        V0, W0, S0, st0 = ctx.mbs_solve(*args)
        ctx.set_params(graph=1)
        for rep in range(4):   # new key (eager), then capture, then replays
            V, W, S, st = ctx.mbs_solve(*args)
            torch.cuda.synchronize()
            _ = ctx.mbs_matvec(d["R"][:50].contiguous(), torch.ones((50, 5), dtype=torch.float64, device=DEV))
            assert torch.equal(V, V0) and torch.equal(W, W0) and torch.equal(S, S0), rep
            assert st["iters"] == st0["iters"] and st["rel_resid"] == st0["rel_resid"], rep
    finally:
        ctx.set_params(graph=1, precision=mbstokes.MBS_FP64, near_cutoff=0.0, tol=1e-10,
                       guess=mbstokes.MBS_GUESS_ZERO, restart=30, near_order=2)


def test_solve_user_guess_and_restarts(ctx):
    w = _workload(200, seed=12)
    ref = galerkin.solve(w)
    ctx.set_params(tol=1e-12, restart=5, guess=mbstokes.MBS_GUESS_USER)
    d = mbstokes.to_device(w, DEV)
    s0 = _t(ref["Sigma"] * (1 + 1e-3 * np.random.default_rng(0).standard_normal(ref["Sigma"].shape)))
    V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], sigma0=s0)
    ctx.set_params(tol=1e-10, restart=30, guess=mbstokes.MBS_GUESS_ZERO)
    assert _rel(V, ref["V"]) < 1e-10 and _rel(S, ref["S"]) < 1e-10


def test_lone_sphere(ctx):
    w = inputs.Workload(np.zeros((1, 3)), np.array([[0, 0, 1.0]]), np.array([[0.3, -0.2, 1.0]]),
                        np.array([[0.1, 0.2, 0.3, 0.4, 0.5]]), np.zeros((1, 3)), np.array([[1.0, 2, 3]]),
                        np.array([[0.5, 0, 0]]))
    ref = galerkin.solve(w)
    d = mbstokes.to_device(w, DEV)
    V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    assert _maxrel(V, ref["V"]) < 1e-15 and _maxrel(W, ref["W"]) < 1e-15 and _maxrel(S, ref["S"]) < 1e-15


# ---------------------------------------------------------------- error contract
def test_errors(ctx):
    w = _workload(20, seed=13)
    d = mbstokes.to_device(w, DEV)
    with pytest.raises(mbstokes.MbsError) as e:
        bad = d["R"].clone()
        bad[3, 1] = float("nan")
        ctx.mbs_solve(bad, d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
    assert e.value.code == mbstokes.MBS_EINVAL
    ctx.set_params(check_overlap=1)
    with pytest.raises(mbstokes.MbsError) as e:
        R = d["R"].clone()
        R[1] = R[0] + torch.tensor([1.0, 0.5, 0.0], dtype=torch.float64, device=DEV)
        ctx.mbs_solve(R, d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
    assert e.value.code == mbstokes.MBS_EOVERLAP
    ctx.set_params(check_overlap=0, max_iter=1, tol=1e-14)
    V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None, allow_noconv=True)
    assert st["iters"] == 1 and st["rel_resid"] > 1e-14
    with pytest.raises(mbstokes.MbsError) as e:
        ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
    assert e.value.code == mbstokes.MBS_ENOCONV
    ctx.set_params(max_iter=300, tol=1e-10)
    with pytest.raises(mbstokes.MbsError) as e:
        ctx.set_params(lmax=3)
    assert e.value.code == mbstokes.MBS_EUNSUPPORTED
    ctx.params.lmax = 2
    for bad in (1, 3, 10, -2):
        with pytest.raises(mbstokes.MbsError) as e:
            ctx.set_params(near_order=bad)
        assert e.value.code == mbstokes.MBS_EINVAL
    ctx.params.near_order = 2
    lib = mbstokes.load()
    rc = lib.mbs_matvec(ctx.h, 0, None, None, None, 0, None)
    assert rc == mbstokes.MBS_EINVAL


def test_coincident_centres_are_rejected_or_reported(ctx):
    """Two distinct spheres at one centre: check_overlap rejects them (distance 0 < 2a); without
    the check their pair blocks are infinite and the solve reports it (MBS_ENOCONV, non-finite
    residual) instead of returning a finite answer."""
    w = _workload(600, seed=15)
    d = mbstokes.to_device(w, DEV)
    R = d["R"].clone()
    R[500] = R[3]  # in different receiver blocks of every launch shape
    ctx.set_params(check_overlap=1)
    try:
        with pytest.raises(mbstokes.MbsError) as e:
            ctx.mbs_solve(R, d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
        assert e.value.code == mbstokes.MBS_EOVERLAP
        ctx.set_params(check_overlap=0)
        V, W, S, st = ctx.mbs_solve(R, d["p"], d["v1s"], d["v2s"], None, d["Fe"], None, allow_noconv=True)
        assert not np.isfinite(st["rel_resid"])
        with pytest.raises(mbstokes.MbsError) as e:
            ctx.mbs_solve(R, d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
        assert e.value.code == mbstokes.MBS_ENOCONV
    finally:
        ctx.set_params(check_overlap=0)


def test_size_limits_are_rejected_before_any_work(ctx):
    """Every entry point refuses a size whose element count would overflow the 32-bit indexing of
    its kernels, with MBS_EINVAL and a message, before it touches memory or launches anything (the
    pointers passed are those of a 4-sphere buffer, valid but far too small)."""
    import ctypes
    lib = mbstokes.load()
    buf = torch.zeros(4 * 80, dtype=torch.float64, device=DEV)
    b = ctypes.c_void_p(buf.data_ptr())
    big6, big10, big12, big80 = 2**31 // 6 + 1, 2**31 // 10 + 1, 2**31 // 12 + 1, 2**31 // 80 + 1
    big20 = 2**31 // 20 + 1
    off = (ctypes.c_int64 * 2)(0, 2**31 // 20 + 1)
    chosen = (ctypes.c_int32 * 2)()
    coef = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    calls = {
        "solve": lambda: lib.mbs_solve(ctx.h, big6, *[b] * 12, None, None),
        "matvec": lambda: lib.mbs_matvec(ctx.h, big6, b, b, ctypes.c_void_p(buf.data_ptr() + 8), 0, None),
        "rhs": lambda: lib.mbs_rhs(ctx.h, big10, *[b] * 6, None),
        "outputs": lambda: lib.mbs_outputs(ctx.h, big10, *[b] * 10, None),
        "flow m": lambda: lib.mbs_flow(ctx.h, big12, b, 4, *[b] * 6, None),
        "flow n": lambda: lib.mbs_flow(ctx.h, 4, b, big10, *[b] * 6, None),
        "step": lambda: lib.mbs_step(ctx.h, big6, b, b, 0.5, coef, 0.01, 1, 2, None, 0, None, None, None),
        "autotune": lambda: lib.mbs_autotune(ctx.h, big6, b, None, chosen, None),
        "precond": lambda: lib.mbs_precond_apply(ctx.h, big6, b, b, ctypes.c_void_p(buf.data_ptr() + 8), None),
        "features": lambda: lib.mbs_features(ctx.h, big80, b, b, b, b, None),
        "warmstart forward": lambda: lib.mbs_warmstart_forward(ctx.h, big80, b, b, None),
        "initial guess": lambda: lib.mbs_initial_guess(ctx.h, big80, *[b] * 6, mbstokes.MBS_GUESS_DIAG, b, None),
        "warmstart target": lambda: lib.mbs_warmstart_target(ctx.h, big80, *[b] * 7, None),
        "batched": lambda: lib.mbs_solve_batched(ctx.h, 1, off, *[b] * 10, None, None, None),
        "autotune batched": lambda: lib.mbs_autotune_batched(ctx.h, 1, off, b, chosen, None, None),
        "matvec r3": lambda: lib.mbs_matvec_r3(ctx.h, big20, b, b, b, None),
        "rhs r3": lambda: lib.mbs_rhs_r3(ctx.h, big20, b, b, b, None, b, b, b, None),
        "outputs r3": lambda: lib.mbs_outputs_r3(ctx.h, big20, b, b, b, None, b, b, b, b, b, b, None),
        "solve r3": lambda: lib.mbs_solve_r3(ctx.h, big20, b, b, b, b, None, b, b, None, b, b, b, b, None, None),
        "precond r3": lambda: lib.mbs_precond_apply_r3(ctx.h, big20, b, b, b, None),
    }
    for name, call in calls.items():
        print(f"size limit: {name}", flush=True)
        assert call() == mbstokes.MBS_EINVAL, name
        msg = lib.mbs_last_error(ctx.h).decode()
        assert "too large" in msg or "too many" in msg, (name, msg)
    torch.cuda.synchronize()
    assert not buf.any()  # nothing was written


# ---------------------------------------------------------------- time stepping
def test_stepper_matches_oracle(ctx):
    w = _workload(64, seed=14, torque=False)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    Rw, pw, _ = stepper.run(w.R, w.p, 0.5, (1.0, 1.0, 1.0), 0.01, 3, prm)
    R, p = _t(w.R), _t(w.p)
    ctx.set_params(tol=1e-13)
    stats, md = ctx.mbs_step(R, p, 0.5, (1.0, 1.0, 1.0), 0.01, 3, order=2, want_min_dist=True)
    ctx.set_params(tol=1e-10)
    assert _maxrel(R, Rw) < 1e-12 and _maxrel(p, pw) < 1e-12
    dmin = min(np.linalg.norm(w.R[i] - w.R[j]) for i in range(w.n) for j in range(i))
    assert abs(md[0] - dmin) < 1e-12


@pytest.mark.parametrize("prec,order", [(mbstokes.MBS_MIXED, 0), (mbstokes.MBS_FP64, 0), (mbstokes.MBS_MIXED, 1)])
def test_stepper_as_benchmarked_matches_oracle(ctx, prec, order):
    """The time-stepping workload exactly as the benchmark runs it, at a size the oracle solves
    densely: the N = 10^4 workload's density (cube side 200, here 300 spheres), slip coefficients
    (1, 1, 1) with the rank-3 mode d = p, trap k = 0.5, Adams-Bashforth dt = 0.01, near-field
    preconditioner at 8a of order 2, the previous step's stresslet as the guess (the first step
    from the one-body guess), mixed precision or binary64, caller's order or Morton order. Four
    steps against the oracle's stepper (dense solves). The displacements, not the positions,
    are compared, so the bar measures the motion: 1e-9 (mixed) and 1e-10 (binary64)."""
    n = 300
    side = 200.0 * (n / 10_000) ** (1 / 3)
    w = inputs.trap_workload(n, side, seed=91, v3t=1.0)
    print(f"stepper as benchmarked n={n} prec={prec} spatial_order={order}", flush=True)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    Rw, pw, _ = stepper.run(w.R, w.p, 0.5, (1.0, 1.0, 1.0), 0.01, 4, prm)
    R, p = _t(w.R), _t(w.p)
    ctx.set_params(precision=prec, guess=mbstokes.MBS_GUESS_USER, tol=1e-11, near_cutoff=8.0, near_order=2,
                   max_iter=60, spatial_order=order)
    try:
        stats, md = ctx.mbs_step(R, p, 0.5, (1.0, 1.0, 1.0), 0.01, 4, order=2, want_min_dist=True)
    finally:
        ctx.set_params(precision=mbstokes.MBS_FP64, guess=mbstokes.MBS_GUESS_ZERO, tol=1e-10, near_cutoff=0.0,
                       max_iter=300, spatial_order=0)
    bar = 1e-9 if prec == mbstokes.MBS_MIXED else 1e-10
    dR = _rel(R.cpu().numpy() - w.R, Rw - w.R)
    dp = _rel(p.cpu().numpy() - w.p, pw - w.p)
    print(f"  displacement error R {dR:.2e} p {dp:.2e}; iterations {[s['iters'] for s in stats]}", flush=True)
    assert dR < bar and dp < bar
    assert all(s["rel_resid"] <= 1e-11 for s in stats)
    if prec == mbstokes.MBS_MIXED:
        assert all(s["fp32_matvecs"] > 0 for s in stats)
    assert md[0] >= 2.2 - 1e-12


def test_mixed_resolve_of_a_converged_guess_reports_a_binary64_residual():
    """MBS_MIXED started from a stresslet that already meets a loose tolerance: the call returns at
    once, and the residual it reports (and certifies against tol) is the binary64 one, equal to the
    oracle's residual of that stresslet, not the binary32 operator's (~1e-7)."""
    w = _workload(120, seed=61)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    ref = galerkin.solve(w, prm)
    c = mbstokes.Context(0, tol=1e-13)
    try:
        d = mbstokes.to_device(w, DEV)
        Sigma = torch.empty((w.n, 5), dtype=torch.float64, device=DEV)
        c.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], Sigma=Sigma)
        Sig_np = Sigma.cpu().numpy()
        res_oracle = np.linalg.norm(ref["b"] - ref["A"] @ Sig_np.ravel()) / np.linalg.norm(ref["b"])
        c.set_params(precision=mbstokes.MBS_MIXED, guess=mbstokes.MBS_GUESS_USER, tol=1e-6)
        V, W, S, st = c.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], sigma0=Sigma)
    finally:
        c.close()
    print(f"re-solve: residual {st['rel_resid']:.3e} (oracle {res_oracle:.3e}), iterations {st['iters']}", flush=True)
    assert st["iters"] == 0 and st["refinements"] == 0
    assert st["out_fused"] == 1 and st["fp32_matvecs"] == 1
    assert st["rel_resid"] < 1e-12
    assert abs(st["rel_resid"] - res_oracle) < 2e-15
    for name, got in (("V", V), ("W", W), ("S", S)):
        assert _rel(got, ref[name]) < 1e-11, name


def test_boundary_contract_rejects_non_unit_orientations_and_aliased_outputs(ctx):
    """|p| must be 1 to 1e-12 wherever p is read; an output may not overlap an input or another
    output. Each case returns MBS_EINVAL with a message and writes nothing."""
    w = _workload(40, seed=17)
    d = mbstokes.to_device(w, DEV)
    pbad = d["p"].clone()
    pbad[7] *= 1.0 + 1e-9
    for name, call in (
            ("solve", lambda: ctx.mbs_solve(d["R"], pbad, d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])),
            ("step", lambda: ctx.mbs_step(d["R"].clone(), pbad.clone(), 0.5, (1.0, 1.0, 1.0), 0.01, 1)),
            ("features", lambda: ctx.mbs_features(d["R"], pbad))):
        with pytest.raises(mbstokes.MbsError) as e:
            call()
        assert e.value.code == mbstokes.MBS_EINVAL and "unit" in str(e.value), name
    # a unit vector rounded to binary64 passes
    ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    import ctypes
    lib = mbstokes.load()
    n = w.n
    buf = torch.zeros(40 * n, dtype=torch.float64, device=DEV)
    base = buf.data_ptr()
    P = lambda k: ctypes.c_void_p(base + 8 * k)  # noqa: E731
    R = P(0)
    buf[:3 * n] = d["R"].reshape(-1)
    x = P(3 * n)
    cases = {
        "matvec y overlaps x": lambda: lib.mbs_matvec(ctx.h, n, R, x, P(3 * n + 7), 0, None),
        "matvec y overlaps R": lambda: lib.mbs_matvec(ctx.h, n, R, x, P(3 * n - 2), 0, None),
        "rhs b overlaps Fe": lambda: lib.mbs_rhs(ctx.h, n, R, None, None, P(20 * n), None, P(20 * n + 3 * n - 1), None),
        "outputs V overlaps W": lambda: lib.mbs_outputs(ctx.h, n, R, None, None, None, None, None, x,
                                                        P(10 * n), P(10 * n + 2), None, None),
        "flow U overlaps X": lambda: lib.mbs_flow(ctx.h, 4, P(30 * n), n, R, None, None, x, None, P(30 * n + 5), None),
    }
    snapshot = buf.clone()
    for name, call in cases.items():
        print(f"aliasing: {name}", flush=True)
        assert call() == mbstokes.MBS_EINVAL, name
        assert "overlap" in lib.mbs_last_error(ctx.h).decode(), name
    torch.cuda.synchronize()
    assert torch.equal(buf, snapshot)


def test_learned_guess_checks_apply_to_the_stepper():
    """mbs_step with the learned guess: without a network MBS_EUNSUPPORTED, with one but fewer than
    17 spheres MBS_EINVAL; both before any launch, so R and p are untouched."""
    c = mbstokes.Context(0, guess=mbstokes.MBS_GUESS_LEARNED)
    try:
        w = _workload(10, seed=19)
        R, p = _t(w.R), _t(w.p)
        with pytest.raises(mbstokes.MbsError) as e:
            c.mbs_step(R, p, 0.5, (1.0, 1.0, 1.0), 0.01, 1)
        assert e.value.code == mbstokes.MBS_EUNSUPPORTED
        c.mbs_warmstart_init(seed=1)
        with pytest.raises(mbstokes.MbsError) as e:
            c.mbs_step(R, p, 0.5, (1.0, 1.0, 1.0), 0.01, 1)
        assert e.value.code == mbstokes.MBS_EINVAL and "n >= 17" in str(e.value)
        assert torch.equal(R, _t(w.R)) and torch.equal(p, _t(w.p))
    finally:
        c.close()


@pytest.mark.parametrize("guess", [mbstokes.MBS_GUESS_USER, mbstokes.MBS_GUESS_DIAG])
def test_stepper_resume_from_checkpoint_is_bitwise(ctx, tmp_path, guess):
    """10 steps in one run equal 4 steps + checkpoint file + resume for 6 steps, bit for bit (the
    Adams-Bashforth history and the previous Sigma travel with the checkpoint)."""
    from paper_1411_0278_amd import trap
    w = _workload(200, seed=44)
    ctx.set_params(guess=guess, tol=1e-12)
    try:
        R1, p1 = _t(w.R), _t(w.p)
        trap.run(ctx, R1, p1, 0.5, (1.0, 1.0, 1.0), 0.01, 10)
        R2, p2 = _t(w.R), _t(w.p)
        path = str(tmp_path / "ck.npz")
        trap.run(ctx, R2, p2, 0.5, (1.0, 1.0, 1.0), 0.01, 4, checkpoint_every=2, path=path)
        R3, p3, _, _, step = trap.resume(ctx, path, 6)
    finally:
        ctx.set_params(guess=mbstokes.MBS_GUESS_ZERO, tol=1e-10)
    assert step == 10
    assert torch.equal(R1, R3) and torch.equal(p1, p3)
    assert not torch.equal(R1, _t(w.R))


@pytest.mark.parametrize("case", ["random", "dilute_lattice", "pair", "clustered"])
def test_minimum_distance_monitor(ctx, case):
    """The per-step minimum centre distance: cell-grid search when some pair is closer than a cell
    edge, all-pairs scan otherwise (a dilute lattice), exact either way."""
    print(f"min distance case={case}", flush=True)
    rng = np.random.default_rng(21)
    if case == "random":
        Rn = _workload(900, seed=22).R
    elif case == "dilute_lattice":
        Rn = np.array([[x, y, z] for x in range(4) for y in range(4) for z in range(4)], float) * 20.0
        Rn[5] += [0.0, 0.0, 3.5]  # one pair at 16.5: the closest, still farther than any cell edge
    elif case == "pair":
        Rn = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    else:
        Rn = np.r_[rng.normal(0, 3, (200, 3)), rng.normal(500, 3, (200, 3))]
    pn = rng.standard_normal(Rn.shape)
    pn /= np.linalg.norm(pn, axis=1, keepdims=True)
    R, p = _t(Rn), _t(pn)
    _, md = ctx.mbs_step(R, p, 0.0, (0.0, 0.0, 0.0), 0.0, 1, order=1, want_min_dist=True)
    D = np.linalg.norm(Rn[:, None] - Rn[None], axis=2)
    D[np.arange(len(Rn)), np.arange(len(Rn))] = np.inf
    assert abs(md[0] - D.min()) <= 1e-12 * D.min()


# ---------------------------------------------------------------- superposition approximation
def test_superposition_matches_oracle(ctx):
    w = _workload(300, seed=71, v3t=1.0, torque=True)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    ref = galerkin.superposition(w, prm)
    d = mbstokes.to_device(w, DEV)
    ctx.set_params(superposition=1)
    try:
        Sig = torch.empty((w.n, 5), dtype=torch.float64, device=DEV)
        V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"], Sigma=Sig)
    finally:
        ctx.set_params(superposition=0)
    for got, want in ((V, ref["V"]), (W, ref["W"]), (S, ref["S"]), (Sig, ref["Sigma"])):
        assert _maxrel(got, want) < 1e-13
    assert st["iters"] == 0


def test_superposition_stepper_matches_oracle(ctx):
    w = _workload(64, seed=72, torque=False)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    Rw, pw, _ = stepper.run(w.R, w.p, 0.5, (1.0, 1.0, 1.0), 0.01, 3, prm, superposition=True)
    R, p = _t(w.R), _t(w.p)
    ctx.set_params(superposition=1)
    try:
        ctx.mbs_step(R, p, 0.5, (1.0, 1.0, 1.0), 0.01, 3, order=2)
    finally:
        ctx.set_params(superposition=0)
    assert _maxrel(R, Rw) < 1e-12 and _maxrel(p, pw) < 1e-12


@pytest.mark.parametrize("superposition", [0, 1])
def test_antipodal_active_pair_keeps_its_orientation(ctx, superposition):
    """Two active spheres at opposite points of the trap sphere R* = 12.56a, pointing outward
    (section V): the interactions are along the axis, so nothing rotates and both stay on it."""
    rs = 12.56
    Rn = np.array([[0.0, 0.0, rs], [0.0, 0.0, -rs]])
    pn = Rn / rs
    R, p = _t(Rn), _t(pn)
    ctx.set_params(superposition=superposition, tol=1e-12)
    try:
        ctx.mbs_step(R, p, 1.0 / rs, (-1.0, 0.0, 0.0), 0.5, 40, order=2)
    finally:
        ctx.set_params(superposition=0, tol=1e-10)
    assert np.abs(p.cpu().numpy() - pn).max() < 1e-14
    assert np.abs(R.cpu().numpy()[:, :2]).max() < 1e-12


@pytest.mark.parametrize("theta0", [115, 260])
@pytest.mark.parametrize("superposition", [1, 0])
def test_two_particle_trap_orbit_matches_oracle(ctx, theta0, superposition):
    """The two-particle trap of section V (R* = 12.56a, sphere 2 at theta0 from sphere 1 in the x-z
    plane, both pointing outward, mean slip only): 200 AB2 steps of dt = 0.5 (six rotation times)
    against the oracle's stepper; the motion stays in the plane of the initial condition."""
    print(f"two-particle orbit theta0={theta0} superposition={superposition}", flush=True)
    rs = 12.56
    th = np.radians(theta0)
    Rn = rs * np.array([[0.0, 0.0, 1.0], [-np.sin(th), 0.0, np.cos(th)]])
    pn = Rn / rs
    k = 1.0 / rs  # 6 pi eta a v_s / R* with eta = 1/(6 pi), a = 1, v_s = 1
    prm = galerkin.Params(eta=1.0 / (6.0 * np.pi), a=1.0)
    Rw, pw, _ = stepper.run(Rn, pn, k, (-1.0, 0.0, 0.0), 0.5, 200, prm, order=2, superposition=bool(superposition))
    R, p = _t(Rn), _t(pn)
    ctx.set_params(superposition=superposition, tol=1e-13)
    try:
        ctx.mbs_step(R, p, k, (-1.0, 0.0, 0.0), 0.5, 200, order=2)
    finally:
        ctx.set_params(superposition=0, tol=1e-10)
    assert _maxrel(R, Rw) < 1e-9 and _maxrel(p, pw) < 1e-9
    assert np.abs(R.cpu().numpy()[:, 1]).max() < 1e-12 and np.abs(p.cpu().numpy()[:, 1]).max() < 1e-12
    assert np.linalg.norm(Rw[0] - Rn[0]) > 0.1  # the pair has started to move round the trap


# ---------------------------------------------------------------- batched
def _batch(ws):
    off = np.cumsum([0] + [w.n for w in ws])
    cat = lambda f: _t(np.concatenate([getattr(w, f) for w in ws]))
    return off, cat


@pytest.mark.parametrize("item", [64, 128, 256])
def test_batched_matches_individual_oracle_solves(ctx, item):
    print(f"batched item={item}", flush=True)
    ws = [_workload(n, seed=500 + n, v3t=0.0, torque=False) for n in (64, 90, 130, 33, 1, 2, 300)]
    off, cat = _batch(ws)
    ctx.set_params(tol=1e-12, batch_item=item)
    try:
        V, W, S, stats, lat = ctx.mbs_solve_batched(off, cat("R"), cat("v1s"), cat("v2s"), None, cat("Fe"), None)
    finally:
        ctx.set_params(tol=1e-10, batch_item=0)
    for b, w in enumerate(ws):
        ref = galerkin.solve(w)
        sl = slice(off[b], off[b + 1])
        assert _rel(V[sl], ref["V"]) < 1e-10 and _rel(W[sl], ref["W"]) < 1e-10 and _rel(S[sl], ref["S"]) < 1e-10
        assert stats[b]["rel_resid"] <= 1e-12
    assert all(l >= 0 for l in lat)


def test_batched_torque_trace_mode_and_restarts(ctx):
    ws = [_workload(n, seed=800 + n, v3t=1.0, torque=True) for n in (70, 200, 129)]
    off, cat = _batch(ws)
    ctx.set_params(tol=1e-12, restart=4)
    Sig = torch.empty((int(off[-1]), 5), dtype=torch.float64, device=DEV)
    V, W, S, stats, lat = ctx.mbs_solve_batched(off, cat("R"), cat("v1s"), cat("v2s"), cat("v3t"), cat("Fe"),
                                                cat("Te"), Sigma=Sig)
    ctx.set_params(tol=1e-10, restart=30)
    for b, w in enumerate(ws):
        ref = galerkin.solve(w)
        sl = slice(off[b], off[b + 1])
        for got, want in ((V[sl], ref["V"]), (W[sl], ref["W"]), (S[sl], ref["S"]), (Sig[sl], ref["Sigma"])):
            assert _rel(got, want) < 1e-10
        assert stats[b]["iters"] > 4          # went through restarts


@pytest.mark.parametrize("graph,near_order", [(0, 2), (1, 2), (1, 4)])
def test_batched_preconditioned_matches_oracle_in_fewer_iterations(ctx, graph, near_order):
    """Near-field right preconditioning inside the batch (lists within each configuration, restarts
    included): same solutions as the oracle, fewer iterations than without it."""
    print(f"batched preconditioned graph={graph}", flush=True)
    ws = [_workload(n, seed=900 + n, v3t=1.0, torque=True) for n in (300, 120, 64, 1, 2, 450)]
    off, cat = _batch(ws)
    args = (off, cat("R"), cat("v1s"), cat("v2s"), cat("v3t"), cat("Fe"), cat("Te"))
    ctx.set_params(tol=1e-12, graph=graph, restart=5)
    try:
        _, _, _, plain, _ = ctx.mbs_solve_batched(*args)
        ctx.set_params(near_cutoff=7.0, near_order=near_order)
        Sig = torch.empty((int(off[-1]), 5), dtype=torch.float64, device=DEV)
        V, W, S, stats, lat = ctx.mbs_solve_batched(*args, Sigma=Sig)
    finally:
        ctx.set_params(tol=1e-10, graph=1, restart=30, near_cutoff=0.0, near_order=2)
    for b, w in enumerate(ws):
        ref = galerkin.solve(w)
        sl = slice(off[b], off[b + 1])
        for got, want in ((V[sl], ref["V"]), (W[sl], ref["W"]), (S[sl], ref["S"]), (Sig[sl], ref["Sigma"])):
            assert _rel(got, want) < 1e-10
        assert stats[b]["rel_resid"] <= 1e-12
    assert sum(st["iters"] for st in stats) < sum(st["iters"] for st in plain)


def test_batched_autotune_picks_an_item_size(ctx):
    sizes = inputs.batched_sizes(20, 64, 900, seed=4242)
    ws = [_workload(int(n), seed=12_000 + b, v3t=0.0, torque=False) for b, n in enumerate(sizes)]
    off, cat = _batch(ws)
    item, ms = ctx.mbs_autotune_batched(off, cat("R"))
    assert item in (64, 128, 256) and all(t > 0 for t in ms.values()) and ms[item] == min(ms.values())
    V, W, S, stats, lat = ctx.mbs_solve_batched(off, cat("R"), cat("v1s"), cat("v2s"), None, cat("Fe"), None)
    for b in (0, 7, 19):
        ref = galerkin.solve(ws[b])
        assert _rel(V[off[b]:off[b + 1]], ref["V"]) < 1e-9


def test_batched_graph_replays_equal_direct_launches(ctx):
    sizes = inputs.batched_sizes(12, 64, 700, seed=4242)
    ws = [_workload(int(n), seed=10_000 + b, v3t=0.0, torque=False) for b, n in enumerate(sizes)]
    off, cat = _batch(ws)
    args = (off, cat("R"), cat("v1s"), cat("v2s"), None, cat("Fe"), None)
    ctx.set_params(graph=0)
    V0, W0, S0, _, _ = ctx.mbs_solve_batched(*args)
    V0, S0 = V0.clone(), S0.clone()
    ctx.set_params(graph=1)
    for rep in range(3):   # capture, then replays with eager work and syncs in between
        V, W, S, stats, lat = ctx.mbs_solve_batched(*args)
        torch.cuda.synchronize()
        _ = ctx.mbs_matvec(cat("R")[:50].contiguous(), torch.ones((50, 5), dtype=torch.float64, device=DEV))
        assert torch.equal(V, V0) and torch.equal(S, S0), rep
    for b in (0, 5, 11):
        ref = galerkin.solve(ws[b])
        assert _rel(V0[off[b]:off[b + 1]], ref["V"]) < 1e-9


def test_batched_single_graph_restarts_latencies_and_more_rounds(ctx):
    """From the second call of a batch shape on, the whole batched solve is one graph launch sized
    by the rounds the previous call took. Every call equals the direct launches bit for bit: with
    restarts (restart length 4, so the true-residual check sends configurations back through the
    restart gate), and after the data are overwritten in place by a denser placement that needs more
    rounds than the graph holds (the remaining rounds then run one by one). Configurations are
    certified in the round their iterations end: the lone sphere finishes before the largest one."""
    print("batched single graph", flush=True)
    sizes = (1, 2, 40, 150, 300)

    def make(density, seed):
        ws = [inputs.trap_workload(n, max(8.0, (n / density) ** (1 / 3)), seed + n) for n in sizes]
        return ws, _batch(ws)

    ws_a, (off, cat_a) = make(0.0005, 9100)
    ws_b, (_, cat_b) = make(0.01, 9200)
    R = cat_a("R").clone()
    v1, v2, Fe = cat_a("v1s").clone(), cat_a("v2s").clone(), cat_a("Fe").clone()
    ctx.set_params(tol=1e-12, restart=4, graph=0)
    try:
        ref_a = [t.clone() for t in ctx.mbs_solve_batched(off, R, v1, v2, None, Fe, None)[:3]]
        ctx.set_params(graph=1)
        lat = None
        for rep in range(3):  # loop (observes the rounds), then the single graph twice
            V, W, S, stats, lat = ctx.mbs_solve_batched(off, R, v1, v2, None, Fe, None)
            assert all(torch.equal(a, b) for a, b in zip((V, W, S), ref_a)), rep
            assert all(st["rel_resid"] <= 1e-12 for st in stats)
        assert max(st["iters"] for st in stats) > 4          # restarts happened
        assert lat[0] < lat[-1], lat
        for b in (0, 2, 4):
            assert _rel(ref_a[0][off[b]:off[b + 1]], galerkin.solve(ws_a[b])["V"]) < 1e-10
        # same buffers, denser data: more iterations than the graph's rounds
        for dst, name in ((R, "R"), (v1, "v1s"), (v2, "v2s"), (Fe, "Fe")):
            dst.copy_(cat_b(name))
        ctx.set_params(graph=0)
        ref_b = [t.clone() for t in ctx.mbs_solve_batched(off, R, v1, v2, None, Fe, None)[:3]]
        ctx.set_params(graph=1)
        V, W, S, stats, _ = ctx.mbs_solve_batched(off, R, v1, v2, None, Fe, None)
        assert all(torch.equal(a, b) for a, b in zip((V, W, S), ref_b))
        assert all(st["rel_resid"] <= 1e-12 for st in stats)
        for b in (1, 3, 4):
            assert _rel(ref_b[0][off[b]:off[b + 1]], galerkin.solve(ws_b[b])["V"]) < 1e-10
    finally:
        ctx.set_params(tol=1e-10, restart=30, graph=1)


def test_batched_graphs_follow_new_offsets(ctx):
    """Two batches with the same number of configurations and spheres but other sizes (so other
    work items), alternated: with graphs and cached descriptors every call equals the direct
    launches of the same batch, bit for bit."""
    print("batched alternating offsets", flush=True)
    ctx.set_params(batch_item=64)
    try:
        batches = []
        for sizes, seed in (((64, 300), 7100), ((100, 264), 7200)):
            ws = [_workload(n, seed=seed + n, v3t=0.0, torque=False) for n in sizes]
            off, cat = _batch(ws)
            batches.append((ws, (off, cat("R"), cat("v1s"), cat("v2s"), None, cat("Fe"), None)))
        ref = []
        ctx.set_params(graph=0)
        for _, args in batches:
            V, W, S, _, _ = ctx.mbs_solve_batched(*args)
            ref.append((V.clone(), W.clone(), S.clone()))
        ctx.set_params(graph=1)
        for k in (0, 1, 0, 1, 1, 0):
            V, W, S, _, _ = ctx.mbs_solve_batched(*batches[k][1])
            assert torch.equal(V, ref[k][0]) and torch.equal(W, ref[k][1]) and torch.equal(S, ref[k][2]), k
        for k, (ws, args) in enumerate(batches):
            off = args[0]
            for b, w in enumerate(ws):
                assert _rel(ref[k][0][off[b]:off[b + 1]], galerkin.solve(w)["V"]) < 1e-9
    finally:
        ctx.set_params(graph=1, batch_item=0)


# ---------------------------------------------------------------- full size, sampled
@pytest.mark.slow
def test_matvec_full_size_sampled_rows(ctx):
    w = inputs.config2()
    prm = galerkin.Params(eta=w.eta, a=w.a)
    x = np.random.default_rng(3).standard_normal((w.n, 5))
    print(f"matvec n={w.n} fp64+fp32, 24 sampled rows vs oracle", flush=True)
    y = ctx.mbs_matvec(_t(w.R), _t(x)).cpu().numpy()
    y32 = ctx.mbs_matvec(_t(w.R), _t(x), precision=mbstokes.MBS_FP32).cpu().numpy()
    rows = np.random.default_rng(4).choice(w.n, 24, replace=False)
    want = galerkin.matvec_rows(w.R, x, rows, prm)
    assert _maxrel(y[rows], want) < 1e-12
    assert _rel(y32[rows], want) < 5e-5


@pytest.mark.slow
def test_operator_full_size_is_symmetric_positive_definite(ctx):
    """Properties that hold at any size (reciprocity of the Green's function, section III): at
    N = 10^5 the binary64 operator satisfies x.(A y) = y.(A x) to rounding and x.(A x) > 0 with
    x.(A x) / |x|^2 inside the interval the one-body term 1/gamma and the pair coupling allow; the
    binary32 operator is symmetric to its own accuracy."""
    w = inputs.config2()
    rng = np.random.default_rng(11)
    x, y = rng.standard_normal((w.n, 5)), rng.standard_normal((w.n, 5))
    R = _t(w.R)
    Ax = ctx.mbs_matvec(R, _t(x)).cpu().numpy()
    Ay = ctx.mbs_matvec(R, _t(y)).cpu().numpy()
    xay, yax = float(np.sum(x * Ay)), float(np.sum(y * Ax))
    scale = np.linalg.norm(x) * np.linalg.norm(Ay)
    print(f"symmetry {abs(xay - yax) / scale:.2e}", flush=True)
    assert abs(xay - yax) <= 1e-13 * scale
    gam = galerkin.constants(galerkin.Params(eta=w.eta, a=w.a))["gamma"]
    rayleigh = float(np.sum(x * Ax)) / float(np.sum(x * x))
    assert 0.3 / gam < rayleigh < 3.0 / gam, rayleigh * gam
    Ax32 = ctx.mbs_matvec(R, _t(x), precision=mbstokes.MBS_FP32).cpu().numpy()
    Ay32 = ctx.mbs_matvec(R, _t(y), precision=mbstokes.MBS_FP32).cpu().numpy()
    assert abs(float(np.sum(x * Ay32)) - float(np.sum(y * Ax32))) <= 1e-5 * scale


@pytest.mark.slow
def test_operator_and_preconditioner_at_ten_times_the_benchmark_size(ctx):
    """N = 10^6 at the benchmark's density (cube side 430 * 10^(1/3)), the largest size the tests
    drive: sampled rows of the binary64 and binary32 operator against the oracle (first row, the
    last row of a ragged last workgroup, and random rows), symmetry x.(A y) = y.(A x), and sampled
    rows of the near-field preconditioner (8a, order 2) against the oracle's blocks of exactly the
    listed pairs. Binary32 bound: coordinates of this box round by up to 2^-24 * 463 = 2.8e-5,
    1.3e-5 of the closest separation (2.2); the r^-7 factor makes that about 9e-5 of a row that its
    nearest pair dominates, so 2e-4 (binary64 keeps the 1e-12 of the full-size test)."""
    from scipy.spatial import cKDTree

    from oracle import greens
    n = 1_000_000
    w = inputs.trap_workload(n, 430.0 * 10 ** (1 / 3), 77)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    rng = np.random.default_rng(12)
    x, y = rng.standard_normal((n, 5)), rng.standard_normal((n, 5))
    R = _t(w.R)
    print(f"n={n}: binary64 and binary32 operator, symmetry", flush=True)
    Ax = ctx.mbs_matvec(R, _t(x)).cpu().numpy()
    Ay = ctx.mbs_matvec(R, _t(y)).cpu().numpy()
    Ax32 = ctx.mbs_matvec(R, _t(x), precision=mbstokes.MBS_FP32).cpu().numpy()
    scale = np.linalg.norm(x) * np.linalg.norm(Ay)
    assert abs(float(np.sum(x * Ay)) - float(np.sum(y * Ax))) <= 1e-13 * scale
    rows = np.array([0, n - 1, int(rng.integers(1, n - 1))])
    print("oracle rows", rows, flush=True)
    want = galerkin.matvec_rows(w.R, x, rows, prm)
    assert _maxrel(Ax[rows], want) < 1e-12
    assert _rel(Ax32[rows], want) < 2e-4

    rc = 8.0
    print(f"n={n}: near-field preconditioner rc={rc} order 2", flush=True)
    ctx.set_params(near_cutoff=rc, near_order=2)
    try:
        Mx = ctx.mbs_precond_apply(R, _t(x)).cpu().numpy()
    finally:
        ctx.set_params(near_cutoff=0.0, near_order=2)
    tree = cKDTree(w.R)

    def partners(i):  # 2a <= r < rc, the 32 smallest indices
        js = sorted(j for j in tree.query_ball_point(w.R[i], rc) if j != i)
        return [j for j in js if 2 * w.a <= np.linalg.norm(w.R[i] - w.R[j]) < rc][:32]

    def k_near(i, v):
        js = partners(i)
        if not js:
            return np.zeros(5)
        return np.einsum("kab,kb->a", greens.block("E", "S", w.R[i] - w.R[js], prm.a, prm.eta), v[js])

    g = galerkin.constants(prm)["gamma"]
    sample = rng.choice(n, 40, replace=False)
    with_partners = 0
    for i in sample:
        js = partners(i)
        kx = k_near(i, x)
        kkx = np.zeros(5)
        if js:
            with_partners += 1
            kxj = np.array([k_near(j, x) for j in js])
            kkx = np.einsum("kab,kb->a", greens.block("E", "S", w.R[i] - w.R[js], prm.a, prm.eta), kxj)
        ref = g * x[i] + g * g * kx + g ** 3 * kkx
        assert np.abs(Mx[i] - ref).max() <= 1e-13 * np.abs(ref).max(), i
    assert with_partners >= 20


# ---------------------------------------------------------------- near-field preconditioner
@pytest.mark.parametrize("order", [2, 4, 8])
def test_precond_apply_matches_oracle(ctx, order):
    w = _workload(400, seed=21)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    rc = 7.0
    x = np.random.default_rng(5).standard_normal((w.n, 5))
    K = galerkin.pair_matrix(w.R, "E", "S", prm)
    D = np.linalg.norm(w.R[:, None] - w.R[None], axis=2)
    near = (D < rc) & (D > 0)
    assert near.sum(1).max() <= 32
    Kn = K * np.kron(near, np.ones((5, 5)))
    g = galerkin.constants(prm)["gamma"]
    term, want = x.ravel().copy(), x.ravel().copy()
    for _ in range(order):   # gamma sum_{i <= order} (gamma K_near)^i x
        term = g * (Kn @ term)
        want = want + term
    want = (g * want).reshape(-1, 5)
    ctx.set_params(near_cutoff=rc, near_order=order)
    try:
        got = ctx.mbs_precond_apply(_t(w.R), _t(x))
    finally:
        ctx.set_params(near_cutoff=0.0, near_order=2)
    assert _maxrel(got, want) < 1e-13


def _near_reference(R, x, rc, a, prm, cap=32):
    """gamma x + gamma^2 K_near x + gamma^3 K_near^2 x with K_near over the pairs 2a <= r < rc, each
    sphere keeping the cap partners of smallest index; blocks from the oracle's pair block for
    exactly those pairs."""
    from oracle import greens
    g = galerkin.constants(prm)["gamma"]
    nbrs, blocks = [], []
    for i in range(len(R)):
        D = np.linalg.norm(R[i] - R, axis=1)
        js = [j for j in np.nonzero((D >= 2 * a) & (D < rc))[0] if j != i][:cap]
        nbrs.append(js)
        blocks.append(greens.block("E", "S", R[i] - R[js], prm.a, prm.eta) if js else None)

    def kn(v):
        out = np.zeros_like(v)
        for i, js in enumerate(nbrs):
            if js:
                out[i] = np.einsum("kab,kb->a", blocks[i], v[js])
        return out

    kx = kn(x)
    return g * x + g * g * kx + g ** 3 * kn(kx), np.array([len(js) for js in nbrs])


@pytest.mark.parametrize("case", ["lattice_rc_on_shell", "lattice_over_capacity", "overlapping_pair", "lone",
                                  "cells_over_capacity"])
def test_precond_apply_hard_geometries(ctx, case):
    """Pairs exactly at r_c are out (strict), lists over capacity keep the 32 smallest indices,
    overlapping pairs are out, a lone sphere gets gamma x. The small sets take the all-pairs build
    (few grid cells), the 14^3 lattice the cell walk."""
    print(f"precond geometry={case}", flush=True)
    a = 1.0
    prm = galerkin.Params(eta=1 / (6 * np.pi), a=a)
    lat = np.array([[x, y, z] for x in range(6) for y in range(6) for z in range(6)], float) * 2.5
    if case == "lattice_rc_on_shell":
        R, rc = lat, 5.0
    elif case == "lattice_over_capacity":
        R, rc = lat, 5.6
    elif case == "cells_over_capacity":
        R, rc = np.array([[x, y, z] for x in range(14) for y in range(14) for z in range(14)], float) * 2.5, 5.6
    elif case == "overlapping_pair":
        R = np.r_[lat[:60], [[0.0, 0.0, 1.5]]]
        rc = 6.0
    else:
        R, rc = np.zeros((1, 3)), 6.0
    x = np.random.default_rng(6).standard_normal((len(R), 5))
    want, counts = _near_reference(R, x, rc, a, prm)
    if case.endswith("over_capacity"):
        assert counts.max() == 32
    ctx.set_params(near_cutoff=rc)
    try:
        got = ctx.mbs_precond_apply(_t(R), _t(x))
    finally:
        ctx.set_params(near_cutoff=0.0)
    assert _maxrel(got, want) < 1e-13


@pytest.mark.parametrize("precision", [mbstokes.MBS_FP64, mbstokes.MBS_MIXED])
def test_preconditioned_solve_matches_oracle_in_fewer_iterations(ctx, precision):
    w = inputs.config0()
    ref = galerkin.solve(w)
    d = mbstokes.to_device(w, DEV)
    its = {}
    for rc, order in ((0.0, 2), (6.0, 2), (10.0, 4)):
        ctx.set_params(tol=1e-11, precision=precision, near_cutoff=rc, guess=mbstokes.MBS_GUESS_DIAG,
                       near_order=order)
        V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
        tol = 1e-10 if precision == mbstokes.MBS_FP64 else 1e-9
        assert _rel(V, ref["V"]) < tol and _rel(W, ref["W"]) < tol and _rel(S, ref["S"]) < tol
        its[rc] = st["iters"]
    ctx.set_params(tol=1e-10, precision=mbstokes.MBS_FP64, near_cutoff=0.0, guess=mbstokes.MBS_GUESS_ZERO,
                   near_order=2)
    assert its[6.0] < its[0.0] and its[10.0] <= its[6.0], its
