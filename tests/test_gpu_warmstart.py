"""Learned warm start on the GPU against the CPU oracle (oracle/mlp.py).

Tolerances:
* neighbour lists: identical (ties by index on both sides); features: float32 rounding of
  binary64 values, 1e-6 relative.
* forward: both sides round inputs, weights and hidden activations to bfloat16; the GPU sums
  float32, the oracle float64, so an activation that lies within a float32 rounding of a bfloat16
  rounding boundary can round to the neighbouring bfloat16 value (one bfloat16 ulp, 2^-8
  relative) on one side only. This is rare and bounded: 2e-3 normwise relative.
* gradient: every backward product also takes bfloat16 operands on the GPU (deltas rounded,
  2^-9 relative each, three layers deep), the oracle keeps float64 deltas: 2e-2 normwise
  relative per parameter block.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import galerkin, mlp  # noqa: E402
from paper_1411_0278_amd import inputs, mbstokes  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = mbstokes.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n", [17, 300, 1500])
def test_features_match_oracle(ctx, n):
    print(f"features n={n}", flush=True)
    w = inputs.trap_workload(n, (n / 0.004) ** (1 / 3) + 8, seed=700 + n)
    R = torch.as_tensor(w.R).to(DEV)
    p = torch.as_tensor(w.p).to(DEV)
    feat, nbr = ctx.mbs_features(R, p, want_nbr=True)
    f_or, nb_or = mlp.features(w.R, w.p)
    assert np.array_equal(nbr.cpu().numpy(), nb_or)
    assert np.abs(feat.cpu().numpy() - f_or).max() <= 1e-6 * np.abs(f_or).max()


def _geometry(name):
    """Centre sets that stress the cell-grid search: exact distance ties, a flat or a linear set
    (one cell across), far-apart clusters with an isolated outlier, the smallest n."""
    rng = np.random.default_rng(11)
    if name == "lattice":
        return np.array([[x, y, z] for x in range(7) for y in range(7) for z in range(7)], float) * 3.0
    if name == "flat":
        return np.c_[rng.uniform(-40, 40, (400, 2)), np.zeros(400)]
    if name == "line":
        return np.c_[np.arange(60) * 2.5, np.zeros(60), np.zeros(60)]
    if name == "clusters":
        return np.r_[rng.normal(0, 4, (250, 3)), rng.normal(300, 4, (250, 3)), [[1500.0, -700.0, 9.0]]]
    if name == "n17":
        return rng.uniform(-6, 6, (17, 3))
    raise KeyError(name)


@pytest.mark.parametrize("name", ["lattice", "flat", "line", "clusters", "n17"])
def test_neighbours_match_oracle_on_hard_geometries(ctx, name):
    print(f"features geometry={name}", flush=True)
    Rn = _geometry(name)
    pn = np.random.default_rng(12).standard_normal(Rn.shape)
    pn /= np.linalg.norm(pn, axis=1, keepdims=True)
    feat, nbr = ctx.mbs_features(torch.as_tensor(Rn).to(DEV), torch.as_tensor(pn).to(DEV), want_nbr=True)
    f_or, nb_or = mlp.features(Rn, pn)
    assert np.array_equal(nbr.cpu().numpy(), nb_or)
    assert np.abs(feat.cpu().numpy() - f_or).max() <= 1e-6 * np.abs(f_or).max()


def _random_params(seed, n_in=mlp.N_IN):
    rng = np.random.default_rng(seed)
    P = {}
    for name, shp in mlp.shapes(n_in):
        fan = shp[0] if len(shp) == 2 else 1
        P[name] = rng.uniform(-1, 1, size=shp) * (np.sqrt(6.0 / fan) if len(shp) == 2 else 0.1)
    return mlp.pack(P).astype(np.float32)


def test_forward_matches_oracle(ctx):
    flat = _random_params(1)
    ctx.mbs_warmstart_set(flat)
    assert np.array_equal(ctx.mbs_warmstart_get(), flat)
    X = np.random.default_rng(2).standard_normal((1000, 80)).astype(np.float32)
    out = ctx.mbs_warmstart_forward(torch.as_tensor(X).to(DEV)).cpu().numpy()
    want, _ = mlp.forward(flat.astype(np.float64), X)
    assert _rel(out, want) < 2e-3


def test_forward_large_batch_chunks(ctx):
    flat = _random_params(3)
    ctx.mbs_warmstart_set(flat)
    X = np.random.default_rng(4).standard_normal((70001, 80)).astype(np.float32)
    out = ctx.mbs_warmstart_forward(torch.as_tensor(X).to(DEV)).cpu().numpy()
    rows = np.r_[0:5, 65530:65545, 69990:70001]
    want, _ = mlp.forward(flat.astype(np.float64), X[rows])
    assert _rel(out[rows], want) < 2e-3


def test_gradient_matches_oracle(ctx):
    flat = _random_params(5)
    ctx.mbs_warmstart_set(flat)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((999, 80)).astype(np.float32)
    T = rng.standard_normal((999, 5)).astype(np.float32)
    loss, g = ctx.mbs_warmstart_grad(torch.as_tensor(X).to(DEV), torch.as_tensor(T).to(DEV))
    l_or, g_or = mlp.loss_grad(flat.astype(np.float64), X, T.astype(np.float64))
    assert abs(loss - l_or) <= 2e-3 * l_or
    off = 0
    for name, shp in mlp.SHAPES:
        sz = int(np.prod(shp))
        assert _rel(g[off:off + sz], g_or[off:off + sz]) < 2e-2, name
        off += sz


def test_training_reduces_loss_and_is_reproducible(ctx, tmp_path):
    rng = np.random.default_rng(7)
    teacher = _random_params(8)
    X = rng.standard_normal((20000, 80)).astype(np.float32)
    T, _ = mlp.forward(teacher.astype(np.float64), X, quantize=False)
    Xd, Td = torch.as_tensor(X).to(DEV), torch.as_tensor(T.astype(np.float32)).to(DEV)
    res = []
    for _ in range(2):
        ctx.mbs_warmstart_init(11)
        hist = ctx.mbs_warmstart_train(Xd, Td, epochs=8, batch=1000, lr=2e-3, seed=5)
        res.append((hist, ctx.mbs_warmstart_get()))
    assert res[0][0] == res[1][0] and np.array_equal(res[0][1], res[1][1])
    hist = res[0][0]
    assert hist[-1] < 0.5 * hist[0], hist
    path = tmp_path / "w.bin"
    ctx.mbs_warmstart_save(path)
    ctx.mbs_warmstart_init(0)
    ctx.mbs_warmstart_load(path)
    assert np.array_equal(ctx.mbs_warmstart_get(), res[0][1])


def test_learned_guess_solve_matches_oracle(ctx):
    w = inputs.trap_workload(200, 40.0 * (200 / 256) ** (1 / 3), seed=9)
    ref = galerkin.solve(w)
    ctx.mbs_warmstart_set(_random_params(10) * 0.05)
    ctx.set_params(tol=1e-12, guess=mbstokes.MBS_GUESS_LEARNED)
    d = mbstokes.to_device(w, DEV)
    V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    ctx.set_params(tol=1e-10, guess=mbstokes.MBS_GUESS_ZERO)
    assert _rel(V.cpu().numpy(), ref["V"]) < 1e-10 and _rel(S.cpu().numpy(), ref["S"]) < 1e-10


# ---------------------------------------------------------------- the wider feature set (160 inputs)
@pytest.fixture()
def ctx_rhs():
    c = mbstokes.Context(0)
    c.mbs_warmstart_features(mbstokes.MBS_FEATURES_GEOMETRY_RHS)
    yield c
    c.close()


def test_rhs_features_match_oracle(ctx_rhs):
    """Each neighbour's five geometric features followed by its one-body stresslet gamma b_j: the
    GPU's right-hand side and features against the oracle's (1e-6, float32 rounding)."""
    n = 300
    w = inputs.trap_workload(n, (n / 0.004) ** (1 / 3) + 8, seed=731, v3t=1.0)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    d = mbstokes.to_device(w, DEV)
    b = ctx_rhs.mbs_rhs(d["R"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    feat, nbr = ctx_rhs.mbs_features_ex(d["R"], d["p"], b, want_nbr=True)
    gb = galerkin.constants(prm)["gamma"] * galerkin.rhs(w.R, w.v2s, w.v3t, w.Fe, w.Te, prm).reshape(-1, 5)
    f_or, nb_or = mlp.features_rhs(w.R, w.p, gb)
    assert np.array_equal(nbr.cpu().numpy(), nb_or)
    assert np.abs(feat.cpu().numpy() - f_or).max() <= 1e-6 * np.abs(f_or).max()


def test_rhs_network_forward_and_gradient_match_oracle(ctx_rhs):
    flat = _random_params(21, mlp.N_IN_RHS)
    ctx_rhs.mbs_warmstart_set(flat)
    rng = np.random.default_rng(22)
    X = rng.standard_normal((999, mlp.N_IN_RHS)).astype(np.float32)
    T = rng.standard_normal((999, 5)).astype(np.float32)
    out = ctx_rhs.mbs_warmstart_forward(torch.as_tensor(X).to(DEV)).cpu().numpy()
    want, _ = mlp.forward(flat.astype(np.float64), X)
    assert _rel(out, want) < 2e-3
    loss, g = ctx_rhs.mbs_warmstart_grad(torch.as_tensor(X).to(DEV), torch.as_tensor(T).to(DEV))
    l_or, g_or = mlp.loss_grad(flat.astype(np.float64), X, T.astype(np.float64))
    assert abs(loss - l_or) <= 2e-3 * l_or
    off = 0
    for name, shp in mlp.shapes(mlp.N_IN_RHS):
        sz = int(np.prod(shp))
        assert _rel(g[off:off + sz], g_or[off:off + sz]) < 2e-2, name
        off += sz


def test_rhs_learned_guess_and_solve_match_oracle(ctx_rhs, tmp_path):
    """The learned guess of the wider network is gamma b + net(features of the solve's own b);
    a solve started from it ends on the oracle's solution; a saved network reloads with its feature
    set into a context that had the other one."""
    w = inputs.trap_workload(200, 40.0 * (200 / 256) ** (1 / 3), seed=29, v3t=1.0)
    prm = galerkin.Params(eta=w.eta, a=w.a)
    ref = galerkin.solve(w, prm)
    flat = _random_params(23, mlp.N_IN_RHS) * 0.05
    ctx_rhs.mbs_warmstart_set(flat)
    d = mbstokes.to_device(w, DEV)
    s0 = ctx_rhs.mbs_initial_guess(d["R"], mbstokes.MBS_GUESS_LEARNED, d["p"], d["v2s"], d["v3t"], d["Fe"],
                                   d["Te"]).cpu().numpy()
    g = galerkin.constants(prm)["gamma"]
    gb = g * ref["b"].reshape(-1, 5)
    f_or, _ = mlp.features_rhs(w.R, w.p, gb)
    net, _ = mlp.forward(flat.astype(np.float64), f_or)
    assert _rel(s0 - gb, net) < 2e-3
    ctx_rhs.set_params(tol=1e-12, guess=mbstokes.MBS_GUESS_LEARNED)
    V, W, S, st = ctx_rhs.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
    assert _rel(V.cpu().numpy(), ref["V"]) < 1e-10 and _rel(S.cpu().numpy(), ref["S"]) < 1e-10
    path = tmp_path / "rhs.bin"
    ctx_rhs.mbs_warmstart_save(path)
    c = mbstokes.Context(0)
    try:
        c.mbs_warmstart_load(path)
        assert np.array_equal(c.mbs_warmstart_get(), flat)
        s1 = c.mbs_initial_guess(d["R"], mbstokes.MBS_GUESS_LEARNED, d["p"], d["v2s"], d["v3t"], d["Fe"],
                                 d["Te"]).cpu().numpy()
        assert np.array_equal(s0, s1)
    finally:
        c.close()


def test_trained_network_gain_on_method_generated_solves(tmp_path):
    """What the trained network gains over the method without it (the one-body guess gamma b): both
    feature sets trained on the method's own converged solves (100 configurations of 10^4 spheres at
    the N = 10^5 workload's density, seeds 0-99, the last 5 held out for validation; 10^6 samples),
    judged on an unseen configuration (seed 4321) by the surrogate error ||Sigma^0 - Sigma*|| /
    ||Sigma*|| against its converged binary64 solve and by the binary64 GMRES iterations to 1e-10
    from each guess. The geometric features alone cannot know a neighbour's slip or trap strain: that
    network must not do worse than gamma b. The wider features carry the neighbours' gamma b_j, and
    to first order the correction is gamma^2 sum_j K(x_ij) b_j: that network must beat both. The
    gain is a few per cent of the surrogate error, too little to save an iteration (each binary64
    iteration divides the residual by about 7 here), and the test shows that too."""
    from paper_1411_0278_amd import warmstart
    c = mbstokes.Context(0)
    files = {0: str(tmp_path / "set0.bin"), 1: str(tmp_path / "set1.bin")}
    try:
        print("training both feature sets on 100 method-generated solves of 10^4 spheres", flush=True)
        rep = warmstart.train_pipeline(c, n_configs=100, n_val=5, epochs=20, batch=4096, lr=1e-3, seed=0,
                                       feature_sets=(0, 1), weights=files)
        w = inputs.trap_workload(warmstart.N_TRAIN, warmstart.SIDE_TRAIN, seed=4321)
        d = mbstokes.to_device(w, DEV)
        c.set_params(tol=1e-12, guess=mbstokes.MBS_GUESS_ZERO)
        sig = torch.empty((w.n, 5), dtype=torch.float64, device=DEV)
        c.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None, Sigma=sig)
        res = {}
        for name, guess, fs in (("diag", mbstokes.MBS_GUESS_DIAG, None), ("learned_set0", mbstokes.MBS_GUESS_LEARNED, 0),
                                ("learned_set1", mbstokes.MBS_GUESS_LEARNED, 1)):
            if fs is not None:
                c.mbs_warmstart_load(files[fs])
            err = warmstart.surrogate_error(c, d, sig, guess)
            c.set_params(tol=1e-10, guess=guess)
            _, _, _, st = c.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
            res[name] = (err, st["iters"])
    finally:
        c.close()
    for fs in (0, 1):
        print(f"  set {fs}: validation mse {rep[fs]['val_mse']:.4e} (target mean square "
              f"{rep[fs]['val_target_ms']:.4e})", flush=True)
    for k, (err, it) in res.items():
        print(f"  {k}: surrogate error {err:.5f}, GMRES iterations to 1e-10: {it}", flush=True)
    assert rep[1]["val_mse"] < rep[1]["val_target_ms"]
    assert res["learned_set0"][0] <= 1.02 * res["diag"][0]
    assert res["learned_set1"][0] < res["diag"][0] and res["learned_set1"][0] < res["learned_set0"][0]
    assert res["learned_set0"][1] <= res["diag"][1] + 1 and res["learned_set1"][1] <= res["diag"][1]
