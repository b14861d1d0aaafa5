"""Adjoint-state gradient of a real misfit with respect to the cell media (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Setting (section 1: the solver is meant for full-waveform inversion, where each
model update needs the gradient of a data misfit): A(m) x_r = b_r for sources r,
a real misfit L(x_1, ..., x_R), and the media m = (lambda, mu, rho) per cell.
With g_r = dL/dRe x_r + i dL/dIm x_r and the adjoint fields A^H y_r = g_r,

    dL/dm_c = -Re sum_r y_r^H (dA/dm_c) x_r .

A of eq. (14) is complex symmetric, so A^H = conj(A).  dA/dm_c is taken term by
term from the assembly in ``discretisation`` (eqs. (4), (5), (14)); the result
is per SI unit at fixed units mu_bar, rho_bar (the operator is assembled in the
nondimensional media lambda/mu_bar, mu/mu_bar, rho/rho_bar; omega and the
attenuation are held fixed).

Pinned in the tests by central finite differences of the misfit through sparse
direct solves (no use of the formulas here) and, for the terms linear in mu and
rho, by the exact matrix difference A(m + e_c) - A(m).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import discretisation as D


def adjoint_solve(A, g):
    """y with A^H y = g for every row of g (sparse LU of the conjugate transpose)."""
    lu = spla.splu(sp.csc_matrix(A.conj().T))
    g = np.atleast_2d(np.asarray(g, dtype=np.complex128))
    return np.stack([lu.solve(gr) for gr in g])


def _blocks(n, x):
    """Split a global vector into its component arrays (flattened, x fastest)."""
    off = D.offsets(n)
    return [x[off[k]:off[k + 1]] for k in range(len(n) + 1)]


def media_gradient(n, omega, lam, mu, rho, gamma_hat, y, x, mu_bar=1.0, rho_bar=1.0):
    """(dL/dlambda, dL/dmu, dL/drho) per cell, each shaped like the media, from the
    adjoint fields y and forward fields x (arrays of shape (R, N)).  lam, mu, rho
    are the nondimensional media the operator was assembled with."""
    n = tuple(int(v) for v in n)
    d = len(n)
    lam = D._flat(lam)
    mu = D._flat(mu)
    rho = D._flat(rho)
    gam = D._flat(gamma_hat)
    dinv = 1.0 / (lam + mu)
    y = np.atleast_2d(y)
    x = np.atleast_2d(x)
    # Laplacian of u_k: sum_a G_a^T diag(W_a mu) G_a (see laplacian_block);
    # mass of u_k: diag(Af (rho (1 - i gamma))) with Af the two-cell face mean
    lap_ops = []
    mass_ops = []
    for k in range(d):
        for a in range(d):
            if a == k:
                Gk = D.kron_axes([D._d_face_to_cell(n[b], 1.0) if b == k else D._eye(n[b]) for b in range(d)])
                Wk = sp.identity(lam.size)
            else:
                Gk = D.kron_axes([D._d_cell_to_node(n[b], 1.0) if b == a else
                                  (D._eye(n[b] - 1) if b == k else D._eye(n[b])) for b in range(d)])
                Wk = D.kron_axes([D._avg_cell_to_node(n[b]) if b == a else
                                  (D._avg_cell_to_face(n[b]) if b == k else D._eye(n[b])) for b in range(d)])
            lap_ops.append((k, Gk, Wk))
        mass_ops.append(D.kron_axes([D._avg_cell_to_face(n[b]) if b == k else D._eye(n[b]) for b in range(d)]))
    g_pd = np.zeros(lam.size)       # Re sum conj(y_p) x_p
    g_lap = np.zeros(lam.size)      # d/dmu of Re y^H (grad^T A_e(mu) grad) x
    s_mass = np.zeros(lam.size, dtype=np.complex128)   # sum over faces of conj(y) x, per cell
    for yr, xr in zip(y, x):
        yb, xb = _blocks(n, yr), _blocks(n, xr)
        g_pd += np.real(np.conj(yb[d]) * xb[d])
        for k, Gk, Wk in lap_ops:
            g_lap += Wk.T @ np.real(np.conj(Gk @ yb[k]) * (Gk @ xb[k]))
        for k in range(d):
            s_mass += mass_ops[k].T @ (np.conj(yb[k]) * xb[k])
    # dA/dlambda_c = dA/dmu_c (pressure row) = +dinv^2 at (p_c, p_c)
    d_lam = -(dinv * dinv * g_pd) / mu_bar
    d_mu = -(dinv * dinv * g_pd + g_lap) / mu_bar
    # dA/drho_c = -omega^2 (1 - i gamma_c) Af^T e_c on the u blocks
    d_rho = -np.real(-omega * omega * (1.0 - 1j * gam) * s_mass) / rho_bar
    shape = tuple(reversed(n))
    return d_lam.reshape(shape), d_mu.reshape(shape), d_rho.reshape(shape)


def receiver_misfit(x, rec_index, d_obs):
    """L = 1/2 sum_r |x_r[rec] - d_r|^2 and its gradient g_r (complex, global layout)."""
    x = np.atleast_2d(x)
    res = x[:, rec_index] - d_obs
    g = np.zeros_like(x)
    g[:, rec_index] = res
    return 0.5 * float(np.sum(np.abs(res) ** 2)), g
