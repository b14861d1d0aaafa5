"""Flexible GMRES (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Right-preconditioned flexible GMRES(m) (Saad 1993, the Krylov method named in
sections 2.2 and 6): zero initial guess, modified Gram-Schmidt Arnoldi with the
Hermitian inner product, the small least-squares problem min |beta e1 - H y|
solved directly at every step (its residual is the Arnoldi estimate of the
residual norm), stop when the estimate reaches tol*|b|, then x += Z y and a
restart from the true residual.  The iteration count is the number of
preconditioner applications ("preconditioning cycles" in section 6).
"""
from __future__ import annotations

import numpy as np


def fgmres(matvec, precond, b, tol=1e-6, restart=5, maxit=500, x0=None):
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.complex128).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, dict(iters=0, rel_res_true=0.0, rel_res_est=0.0, history=[0.0], converged=True)
    it = 0
    history = []
    converged = False
    est = np.inf
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if not history:
            history.append(beta / bnorm)
        if beta <= tol * bnorm or it >= maxit:
            converged = beta <= tol * bnorm
            break
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        y = None
        for j in range(restart):
            Z.append(precond(V[j]))
            w = matvec(Z[j])
            it += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] != 0 else w)
            g = np.zeros(j + 2, dtype=np.complex128)
            g[0] = beta
            y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], g, rcond=None)
            est = np.linalg.norm(g - H[:j + 2, :j + 1] @ y)
            history.append(est / bnorm)
            if est <= tol * bnorm or it >= maxit or H[j + 1, j] == 0:
                break
        x = x + np.array(Z).T @ y
    return x, dict(iters=it, rel_res_true=float(np.linalg.norm(b - matvec(x)) / bnorm),
                   rel_res_est=float(est / bnorm), history=history, converged=converged)


def convergence_factor(history, warmup=5):
    """c_f = (|r_k| / |r_0|)^(1/k) with r_0 taken after a warm-up (section 5.4)."""
    h = [v for v in history if v > 0]
    if len(h) <= warmup + 1:
        return float("nan")
    k = len(h) - 1 - warmup
    return float((h[-1] / h[warmup]) ** (1.0 / k))
