"""Restarted GMRES with modified Gram-Schmidt, FP64 (test infrastructure only).

The paper leaves the iterative solver unspecified (section IV: matrix-free
iterative solvers are announced but not described). This is the textbook
GMRES(m) of Saad & Schultz: Arnoldi with modified Gram-Schmidt, Givens
rotations on the Hessenberg matrix, and a least-squares update at every
restart. The stopping rule is the relative 2-norm of the true residual.
"""
import numpy as np


def gmres(matvec, b, x0=None, tol=1e-12, restart=30, max_iter=500):
    """Solve A x = b. Returns (x, info) with info = dict(iters, rel_resid, history)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), dict(iters=0, rel_resid=0.0, history=[0.0])
    iters = 0
    hist = []
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    hist.append(beta / bnorm)
    while beta / bnorm > tol and iters < max_iter:
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        while k < restart and iters < max_iter:
            w = matvec(V[k])
            for i in range(k + 1):
                H[i, k] = V[i] @ w
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            k += 1
            iters += 1
            hist.append(abs(g[k]) / bnorm)
            if abs(g[k]) / bnorm <= tol:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + V[:k].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        hist[-1] = beta / bnorm
    return x, dict(iters=iters, rel_resid=beta / bnorm, history=hist)
