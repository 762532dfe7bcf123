"""Reference network and neighbourhood features of the learned warm start (test infrastructure only).

The paper has no learned component; this follows the warm-start definition of the benchmark:
a 3-layer perceptron 80 -> 128 -> 128 -> 5 with ReLU, whose input is each sphere's 16 nearest
neighbours (by centre distance, ties by index, nearest first), each contributing
(R_j - R_i)/|R_j - R_i|, 1/|R_j - R_i| and p_j . p_i, and whose output is the correction
Sigma - gamma b to the one-body (diagonal) guess of the stresslet rows. An optional wider input
(160 features, ``features_rhs``) adds each neighbour's one-body stresslet gamma b_j (5 values in
the orthonormal 5-basis) after its five geometric features; the network then reads 160 inputs.
The input width of a parameter vector follows from its length.

The GPU network multiplies bfloat16 operands with float32 accumulation. ``forward`` mirrors the
precision steps (round inputs, weights and hidden activations to bfloat16, round-to-nearest-even
from float32) and otherwise computes in float64; ``quantize=False`` gives the plain float64
network, whose gradient is checked against central finite differences.
"""
import numpy as np

N_IN, N_HID, N_OUT, K_NEIGH = 80, 128, 5, 16
N_IN_RHS = 160  # the wider input: 16 neighbours x (5 geometric features + gamma b_j)


def shapes(n_in=N_IN):
    return [("W1", (n_in, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
            ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,))]


def n_param(n_in=N_IN):
    return sum(int(np.prod(s)) for _, s in shapes(n_in))


SHAPES = shapes(N_IN)
N_PARAM = n_param(N_IN)


def input_width(flat):
    """Input width of a parameter vector (its length fixes the first layer)."""
    rest = n_param(0)
    n_in, r = divmod(len(np.ravel(flat)) - rest, N_HID)
    assert r == 0 and n_in > 0, len(np.ravel(flat))
    return n_in


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, k = {}, 0
    for name, shp in shapes(input_width(flat)):
        sz = int(np.prod(shp))
        out[name] = flat[k:k + sz].reshape(shp)
        k += sz
    return out


def pack(d):
    return np.concatenate([np.ravel(d[name]) for name, _ in shapes(d["W1"].shape[0])])


def bf16(x):
    """Round to bfloat16 (round to nearest, ties to even) via float32; returned as float64."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = x32.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(flat, X, quantize=True):
    """Returns (out [m, 5], cache)."""
    P = unpack(flat)
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    f32 = (lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)) if quantize else (lambda a: a)
    Xq = q(X)
    W1, W2, W3 = q(P["W1"]), q(P["W2"]), q(P["W3"])
    b1, b2, b3 = f32(P["b1"]), f32(P["b2"]), f32(P["b3"])
    z1 = Xq @ W1 + b1
    h1 = q(f32(np.maximum(z1, 0.0)))
    z2 = h1 @ W2 + b2
    h2 = q(f32(np.maximum(z2, 0.0)))
    out = h2 @ W3 + b3
    return out, dict(Xq=Xq, W1=W1, W2=W2, W3=W3, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_grad(flat, X, T, quantize=True):
    """Mean squared error over all m x 5 outputs and its gradient (straight through the rounding)."""
    out, c = forward(flat, X, quantize)
    m = out.shape[0]
    diff = out - T
    loss = float(np.mean(diff ** 2))
    d_out = 2.0 * diff / diff.size
    g = {}
    g["W3"] = c["h2"].T @ d_out
    g["b3"] = d_out.sum(0)
    d_z2 = (d_out @ c["W3"].T) * (c["z2"] > 0)
    g["W2"] = c["h1"].T @ d_z2
    g["b2"] = d_z2.sum(0)
    d_z1 = (d_z2 @ c["W2"].T) * (c["z1"] > 0)
    g["W1"] = c["Xq"].T @ d_z1
    g["b1"] = d_z1.sum(0)
    return loss, pack(g)


def knn(R, k=K_NEIGH):
    """Indices [n, k] of the k nearest other centres, nearest first, ties by index (brute force)."""
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    out = np.empty((n, k), dtype=np.int64)
    for i0 in range(0, n, 256):
        blk = R[i0:i0 + 256]
        d = R[None, :, :] - blk[:, None, :]
        d2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]
        rows = np.arange(i0, i0 + len(blk))
        d2[np.arange(len(blk)), rows] = np.inf
        idx = np.argsort(d2, axis=1, kind="stable")[:, :k]   # stable: equal distances by index
        out[i0:i0 + len(blk)] = idx
    return out


def features(R, p, k=K_NEIGH):
    """[n, 5k] features in the order of knn(): unit separation (3), inverse distance, p_j . p_i."""
    R = np.asarray(R, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    nb = knn(R, k)
    rel = R[nb] - R[:, None, :]
    r = np.linalg.norm(rel, axis=2)
    f = np.concatenate([rel / r[..., None], (1.0 / r)[..., None],
                        np.einsum("nkc,nc->nk", p[nb], p)[..., None]], axis=2)
    return f.reshape(R.shape[0], 5 * k), nb


def features_rhs(R, p, gb, k=K_NEIGH):
    """[n, 10k] features: for each neighbour (order of knn()) its five geometric features followed
    by its one-body stresslet gamma b_j [n, 5] (the diagonal solve of the stresslet rows)."""
    f, nb = features(R, p, k)
    gb = np.asarray(gb, dtype=np.float64)
    f = np.concatenate([f.reshape(-1, k, 5), gb[nb]], axis=2)
    return f.reshape(len(R), 10 * k), nb
