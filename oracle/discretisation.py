"""Staggered second-order discretisation of the elastic Helmholtz system (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grid and unknowns (paper section 2.1, Fig. 2): a box of n_0 x n_1 [x n_2] cells of
size h; Lame parameters, density and attenuation live at cell centres; the
displacement component u_k lives on the faces normal to axis k; the pressure of
the mixed formulation (eq. (13)) lives at cell centres.  Boundary reading: the
normal displacement vanishes on the outer walls, so only the interior faces
1..n_k-1 carry unknowns; a derivative taken across a wall in a tangential
direction uses a zero value beyond the wall.

Vector layout: per component a numpy array of shape (.., n_1, n_0) (x fastest,
C order), flattened and stacked as [u_0, u_1, (u_2), p].
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------- layout
def face_dims(n: Sequence[int], k: int):
    """Sizes (x, y[, z]) of the interior-face array of component k."""
    return tuple(n[a] - 1 if a == k else n[a] for a in range(len(n)))


def counts(n: Sequence[int]):
    d = len(n)
    c = [int(np.prod(face_dims(n, k))) for k in range(d)]
    c.append(int(np.prod(n)))
    return c


def offsets(n):
    c = counts(n)
    return np.concatenate([[0], np.cumsum(c)]).astype(np.int64)


def n_unknowns(n):
    return int(sum(counts(n)))


def face_flat_index(n, k, pos):
    """Flat index inside block k of the face of component k at position pos
    (x, y[, z]) with pos[k] in 1..n_k-1."""
    dims = face_dims(n, k)
    idx = 0
    stride = 1
    for a in range(len(n)):
        c = pos[a] - 1 if a == k else pos[a]
        assert 0 <= c < dims[a]
        idx += c * stride
        stride *= dims[a]
    return idx


def unknown_index(n, comp, pos):
    """Global unknown index; comp in 0..d-1 for u, d for p (pos = cell)."""
    off = offsets(n)
    d = len(n)
    if comp == d:
        idx = 0
        stride = 1
        for a in range(d):
            idx += pos[a] * stride
            stride *= n[a]
        return int(off[d] + idx)
    return int(off[comp] + face_flat_index(n, comp, pos))


def split(n, x):
    """Split a stacked vector into per-component arrays shaped (.., n_1, n_0)."""
    off = offsets(n)
    d = len(n)
    out = []
    for k in range(d + 1):
        shape = tuple(reversed(face_dims(n, k))) if k < d else tuple(reversed(n))
        out.append(np.asarray(x[off[k]:off[k + 1]]).reshape(shape))
    return out


def point_source_vector(n, sources):
    """Right-hand side with unit point forces; sources = [(comp, pos, amp)]."""
    b = np.zeros(n_unknowns(n), dtype=np.complex128)
    for comp, pos, amp in sources:
        b[unknown_index(n, comp, pos)] += amp
    return b


# ------------------------------------------------------------------ 1-D building blocks
def _d_face_to_cell(n, h):
    """D_n (n x (n-1)): (Dv)_c = (v_{c+1} - v_c)/h, wall faces 0 and n are zero.
    Column f-1 holds interior face f."""
    rows, cols, vals = [], [], []
    for c in range(n):
        if c + 1 <= n - 1:
            rows.append(c); cols.append(c); vals.append(1.0 / h)
        if c >= 1:
            rows.append(c); cols.append(c - 1); vals.append(-1.0 / h)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n - 1))


def _d_cell_to_node(n, h):
    """T_n ((n+1) x n): (Tv)_m = (v_m - v_{m-1})/h for nodes m = 0..n, with zero
    values beyond both walls."""
    rows, cols, vals = [], [], []
    for m in range(n + 1):
        if m <= n - 1:
            rows.append(m); cols.append(m); vals.append(1.0 / h)
        if m >= 1:
            rows.append(m); cols.append(m - 1); vals.append(-1.0 / h)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, n))


def _avg_cell_to_face(n):
    """((n-1) x n): arithmetic mean of the two cells beside interior face f."""
    rows, cols, vals = [], [], []
    for f in range(1, n):
        rows += [f - 1, f - 1]; cols += [f - 1, f]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n - 1, n))


def _avg_cell_to_node(n):
    """((n+1) x n): arithmetic mean of the existing cells beside node m."""
    rows, cols, vals = [], [], []
    for m in range(n + 1):
        nb = [c for c in (m - 1, m) if 0 <= c < n]
        for c in nb:
            rows.append(m); cols.append(c); vals.append(1.0 / len(nb))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, n))


def _eye(n):
    return sp.identity(n, format="csr")


def kron_axes(ops):
    """Operator acting on a field flattened x-fastest: ops[a] acts on axis a."""
    M = ops[-1]
    for a in range(len(ops) - 2, -1, -1):
        M = sp.kron(M, ops[a], format="csr")
    return sp.csr_matrix(M)


def _flat(a):
    return np.asarray(a, dtype=np.float64).reshape(-1)


# ---------------------------------------------------------------- coefficient setup
def abl_gamma(n, abl_cells, abl_max):
    """Absorbing-layer attenuation gamma/omega at cell centres (section 2.1): per axis
    a quadratic ramp t^2 that goes from 0 to abl_max towards both walls over
    abl_cells[a] cells, summed over the axes."""
    shape = tuple(reversed(n))
    g = np.zeros(shape)
    d = len(n)
    for a in range(d):
        L = abl_cells[a]
        if L <= 0:
            continue
        x = np.arange(n[a]) + 0.5
        t = np.maximum(0.0, np.maximum((L - x) / L, (x - (n[a] - L)) / L))
        bshape = [1] * d
        bshape[d - 1 - a] = n[a]
        g = g + abl_max * (t * t).reshape(bshape)
    return g


def total_gamma(n, omega_si, abl_cells, abl_max, atten0, gamma_phys=None):
    """gamma/omega per cell: the layer, the constant attenuation gamma_0 (section 6:
    a small attenuation added to gamma in the mass matrix, eq. (5)) and an
    optional physical attenuation field [1/s]."""
    g = abl_gamma(n, abl_cells, abl_max) + atten0 / omega_si
    if gamma_phys is not None:
        g = g + np.asarray(gamma_phys) / omega_si
    return g


def nondimensionalise(h, omega, lam, mu, rho, mu_bar=None, rho_bar=None):
    """Scale to h = 1, mean(mu) = 1, mean(rho) = 1.  Returns a dict with the
    nondimensional media and omega*h*sqrt(rho_bar/mu_bar).  If mu vanishes
    everywhere, mean(lambda + 2 mu) is the stiffness scale.  Units given by the
    caller (mu_bar, rho_bar > 0) replace the means, so that vectors keep their
    units while the media change (gradients at fixed units)."""
    if mu_bar is None or mu_bar <= 0.0:
        mu_bar = float(np.mean(mu))
        if mu_bar <= 0.0:
            mu_bar = float(np.mean(lam + 2.0 * mu))
    if rho_bar is None or rho_bar <= 0.0:
        rho_bar = float(np.mean(rho))
    mu_bar, rho_bar = float(mu_bar), float(rho_bar)
    return dict(h=1.0, omega=omega * h * math.sqrt(rho_bar / mu_bar),
                lam=np.asarray(lam) / mu_bar, mu=np.asarray(mu) / mu_bar,
                rho=np.asarray(rho) / rho_bar, mu_bar=mu_bar, rho_bar=rho_bar)


# ------------------------------------------------------------------------ assembly
def divergence_blocks(n, h):
    """Div_k: cells x faces_k, so that Div = [Div_0, Div_1, (Div_2)]; the gradient
    of eq. (4) is grad_h = -Div^T."""
    d = len(n)
    out = []
    for k in range(d):
        ops = [_d_face_to_cell(n[a], h) if a == k else _eye(n[a]) for a in range(d)]
        out.append(kron_axes(ops))
    return out


def laplacian_block(n, h, k, mu):
    """The weighted vector Laplacian grad^T A_e(mu) grad of eq. (4) on component k:
    normal derivatives sit at cell centres (weight mu), tangential derivatives at
    edges (nodes in 2D) with mu averaged over the existing adjacent cells."""
    d = len(n)
    mu_c = _flat(mu)
    L = None
    for a in range(d):
        if a == k:
            G = kron_axes([_d_face_to_cell(n[b], h) if b == k else _eye(n[b]) for b in range(d)])
            w = mu_c
        else:
            G = kron_axes([_d_cell_to_node(n[b], h) if b == a else
                           (_eye(n[b] - 1) if b == k else _eye(n[b])) for b in range(d)])
            Av = kron_axes([_avg_cell_to_node(n[b]) if b == a else
                            (_avg_cell_to_face(n[b]) if b == k else _eye(n[b])) for b in range(d)])
            w = Av @ mu_c
        term = G.T @ sp.diags(w) @ G
        L = term if L is None else L + term
    return sp.csr_matrix(L)


def face_average(n, k, field):
    d = len(n)
    Av = kron_axes([_avg_cell_to_face(n[b]) if b == k else _eye(n[b]) for b in range(d)])
    return Av @ np.asarray(field).reshape(-1)


def mass_block(n, k, rho, gamma_hat, shift=0.0):
    """A_f(rho (1 - i (gamma_hat + shift))) on the faces of component k: the mass of
    eq. (5); shift > 0 adds the shifted-Laplacian term of eq. (10) with
    M_s = A_f(rho), with the same sign as the attenuation."""
    z = _flat(rho) * (1.0 - 1j * (_flat(gamma_hat) + shift))
    return sp.diags(face_average(n, k, z))


def assemble(n, h, omega, lam, mu, rho, gamma_hat, shift=0.0, form="mixed"):
    """Sparse complex matrix of the staggered system.

    form = "mixed": [[grad^T A_e grad - w^2 M, grad_h], [grad_h^T, -D_c(1/(lam+mu))]],
                    eq. (14) (with the shift of eq. (10) on the u block only, section 3);
    form = "u":     H^e of eq. (4).
    """
    d = len(n)
    divs = divergence_blocks(n, h)
    uu = []
    for k in range(d):
        Lk = laplacian_block(n, h, k, mu)
        uu.append(Lk - omega * omega * mass_block(n, k, rho, gamma_hat, shift))
    Auu = sp.block_diag(uu, format="csr")
    Div = sp.hstack(divs, format="csr")
    if form == "u":
        lm = _flat(lam) + _flat(mu)
        return sp.csr_matrix(Auu + Div.T @ sp.diags(lm) @ Div)
    grad = -Div.T
    dinv = 1.0 / (_flat(lam) + _flat(mu))
    A = sp.bmat([[Auu, grad], [grad.T, -sp.diags(dinv)]], format="csr")
    return sp.csr_matrix(A.astype(np.complex128))


class Problem:
    """A discretised problem in the nondimensional scaling used for every solve:
    h = 1, mean mu = 1, mean rho = 1 (the residual norm is taken in these units)."""

    def __init__(self, n, h, omega, lam, mu, rho, abl_cells, abl_max=1.0, atten0=0.0,
                 gamma_phys=None, shift=0.0, mu_bar=None, rho_bar=None):
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        self.h_si = float(h)
        self.omega_si = float(omega)
        self.shift = float(shift)
        self.gamma_hat = total_gamma(self.n, omega, abl_cells, abl_max, atten0, gamma_phys)
        nd = nondimensionalise(h, omega, lam, mu, rho, mu_bar, rho_bar)
        self.nd = nd
        self.omega = nd["omega"]
        self.lam, self.mu, self.rho = nd["lam"], nd["mu"], nd["rho"]

    def matrix(self, shifted=False, form="mixed"):
        return assemble(self.n, 1.0, self.omega, self.lam, self.mu, self.rho,
                        self.gamma_hat, self.shift if shifted else 0.0, form)

    @property
    def size(self):
        return n_unknowns(self.n)
