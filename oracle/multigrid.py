"""Shifted-Laplacian multigrid for the mixed system (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows section 3 ("Summary of the multigrid method"): the hierarchy is built for
the shifted mixed operator (eq. (14) with the u-block shift of eq. (10)), coarse
operators are Galerkin products P^T A P (eq. (9)), the restriction is P^T
(section 2.2), the smoother is damped red-black cell-wise Vanka relaxation
(full block, or the economic block with a diagonal u part, section 3 and the
matrix B of section 5.2), and the coarsest level is solved exactly.  The cycle is
Algorithm 1 applied recursively: one recursive call gives a V-cycle, two a
W-cycle (section 2.2).

Transfer reading ("standard bilinear transfer operators for face-based staggered
discretisation"): u_k is interpolated linearly along its normal axis (a fine
face on a coarse face takes it with weight 1, a fine face between two coarse
faces takes 1/2 of each) and linearly along each tangential axis (weights 3/4
for the nearer coarse row, 1/4 for the other, zero beyond the wall); the
pressure is interpolated piecewise constantly.

MG-DD (section 4): the coarsest level may instead be solved by one sweep of
domain decomposition over its own subdomains (CoarseDD); with top-level DD
around the cycle (oracle.dd) this is DD-MG-DD.

Red-black reading ("simultaneously sweep over all the red cells"): within one
colour every cell's correction is computed from the residual at the start of
that half-sweep; cells of one colour share no unknown, so the corrections are
simply added.  Red = (sum of cell indices) even; both pre- and post-smoothing
visit red then black.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import discretisation as disc


# ---------------------------------------------------------------- transfer operators
def _p_normal(n):
    """(n-1) x (n/2-1): linear interpolation along the normal axis of a face field."""
    nc = n // 2
    rows, cols, vals = [], [], []
    for f in range(1, n):
        if f % 2 == 0:
            F = f // 2
            if 1 <= F <= nc - 1:
                rows.append(f - 1); cols.append(F - 1); vals.append(1.0)
        else:
            for F in ((f - 1) // 2, (f + 1) // 2):
                if 1 <= F <= nc - 1:
                    rows.append(f - 1); cols.append(F - 1); vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n - 1, nc - 1))


def _p_tangential(n):
    """n x n/2: linear interpolation of a cell-centred row position (3/4, 1/4)."""
    nc = n // 2
    rows, cols, vals = [], [], []
    for c in range(n):
        C = c // 2
        other = C - 1 if c % 2 == 0 else C + 1
        rows.append(c); cols.append(C); vals.append(0.75)
        if 0 <= other < nc:
            rows.append(c); cols.append(other); vals.append(0.25)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def _p_constant(n):
    nc = n // 2
    rows = list(range(n))
    cols = [c // 2 for c in range(n)]
    return sp.csr_matrix((np.ones(n), (rows, cols)), shape=(n, nc))


def prolongation(n):
    """Block-diagonal P from the coarse grid n/2 to the fine grid n."""
    d = len(n)
    blocks = []
    for k in range(d):
        blocks.append(disc.kron_axes([_p_normal(n[a]) if a == k else _p_tangential(n[a])
                                      for a in range(d)]))
    blocks.append(disc.kron_axes([_p_constant(n[a]) for a in range(d)]))
    return sp.csr_matrix(sp.block_diag(blocks, format="csr"))


# ------------------------------------------------------------------------ Vanka blocks
def cell_dofs(n):
    """(n_cells, 2d+1) unknown indices of every cell's block, ordered
    [u_0 low, u_0 high, u_1 low, u_1 high, (u_2 low, u_2 high,) p]; -1 marks a
    face on the wall (no unknown).  Cells are listed x fastest."""
    d = len(n)
    off = disc.offsets(n)
    grids = np.meshgrid(*[np.arange(n[a]) for a in range(d)], indexing="ij")
    # flatten x fastest: iterate with the last axis slowest
    pos = [g.transpose(tuple(reversed(range(d)))).reshape(-1) for g in grids]
    ncell = int(np.prod(n))
    dofs = -np.ones((ncell, 2 * d + 1), dtype=np.int64)
    for k in range(d):
        dims = disc.face_dims(n, k)
        for side in (0, 1):
            fpos = [p.copy() for p in pos]
            fpos[k] = pos[k] + side            # face position of the low/high face
            ok = (fpos[k] >= 1) & (fpos[k] <= n[k] - 1)
            idx = np.zeros(ncell, dtype=np.int64)
            stride = 1
            for a in range(d):
                c = fpos[a] - 1 if a == k else fpos[a]
                idx += c * stride
                stride *= dims[a]
            dofs[ok, 2 * k + side] = off[k] + idx[ok]
    cidx = np.zeros(ncell, dtype=np.int64)
    stride = 1
    for a in range(d):
        cidx += pos[a] * stride
        stride *= n[a]
    dofs[:, 2 * d] = off[d] + cidx
    colour = (sum(pos) % 2).astype(np.int64)
    return dofs, colour


def vanka_blocks(A, n, economic=False):
    """Local matrices B_K = A restricted to the unknowns of cell K (section 3).
    Missing wall faces get an identity row/column.  economic=True keeps only the
    diagonal of the u-u part (the matrix B of section 5.2)."""
    d = len(n)
    dofs, colour = cell_dofs(n)
    nb = 2 * d + 1
    ncell = dofs.shape[0]
    B = np.zeros((ncell, nb, nb), dtype=np.complex128)
    A = sp.csr_matrix(A)
    for a in range(nb):
        for b in range(nb):
            ra, cb = dofs[:, a], dofs[:, b]
            ok = (ra >= 0) & (cb >= 0)
            if economic and a != b and a < 2 * d and b < 2 * d:
                continue
            if np.any(ok):
                B[ok, a, b] = np.asarray(A[ra[ok], cb[ok]]).reshape(-1)
    for a in range(nb):
        miss = dofs[:, a] < 0
        B[miss, a, :] = 0.0
        B[miss, :, a] = 0.0
        B[miss, a, a] = 1.0
    return B, dofs, colour


def vanka_half_sweep(A, B, dofs, colour, c, b, e, w, wp=None):
    """One damped red-black half-sweep on colour c (Jacobi within the colour):
    r = b - A e; for every cell K of colour c, e_K += W B_K^{-1} r_K with
    W = diag(w, .., w, wp): the component-dependent damping of section 5.2
    (w on the displacement rows, wp on the pressure row; wp = w by default)."""
    r = b - A @ e
    sel = np.nonzero(colour == c)[0]
    D = dofs[sel]
    rK = np.where(D >= 0, r[np.maximum(D, 0)], 0.0)
    cK = np.linalg.solve(B[sel], rK[..., None])[..., 0]
    W = np.full(D.shape[1], float(w))
    W[-1] = float(w if wp is None else wp)
    cK = cK * W
    e = e.copy()
    ok = D >= 0
    e[D[ok]] += cK[ok]
    return e


# ------------------------------------------------------------------------- hierarchy
class CoarseDD:
    """Domain decomposition as the coarsest-grid solver (MG-DD, section 4).

    Reading: the coarsest grid is split into overlapping subdomains as the fine
    grid is (core n/parts per axis, the overlap split around each cut, no
    padding); the local operator of a subdomain is the coarsest Galerkin
    operator restricted to the unknowns of its extent (the shift already makes
    the coarse system local, so no absorbing layer is added), solved exactly.
    One application from the guess z is one sweep of Algorithm 2 over the
    colours (each colour from the residual b - A_c z left by the previous ones),
    or with one colour the corrections of all subdomains from the same residual,
    averaged over the subdomains that own an unknown."""

    def __init__(self, A, n, parts, overlap, colours=0):
        from . import dd as ddm
        self.A = sp.csr_matrix(A)
        self.subs = ddm.make_subdomains(n, parts, overlap, 0)
        self.colours = colours
        self.idx, self.lu = [], []
        cnt = np.zeros(self.A.shape[0])
        for sub in self.subs:
            m = ddm.local_to_global(n, sub)
            g = m[m >= 0]
            self.idx.append(g)
            self.lu.append(spla.splu(sp.csc_matrix(self.A[g][:, g])))
            cnt[g] += 1
        if np.any(cnt == 0):
            raise ValueError("coarse subdomains do not cover every unknown")
        self.weight = 1.0 / cnt

    def solve(self, b, z=None):
        b = np.asarray(b, dtype=np.complex128)
        z = np.zeros_like(b) if z is None else np.asarray(z, dtype=np.complex128).copy()
        if self.colours == 1:
            r = b - self.A @ z
            for g, lu in zip(self.idx, self.lu):
                z[g] += self.weight[g] * lu.solve(r[g])
            return z
        for c in sorted(set(s.colour for s in self.subs)):
            r = b - self.A @ z
            for sub, g, lu in zip(self.subs, self.idx, self.lu):
                if sub.colour == c:
                    z[g] += lu.solve(r[g])
        return z


class Hierarchy:
    """Galerkin hierarchy of a shifted operator A0 on grid n.  coarse_dd =
    (parts, overlap, colours) solves the coarsest level by domain
    decomposition (CoarseDD) instead of exactly."""

    def __init__(self, A0, n, levels, damping: Sequence[float], economic=False,
                 cycle=1, nu1=1, nu2=1, cycle_level=0, coarse_dd=None, damping_p=None):
        self.n = [tuple(n)]
        self.A = [sp.csr_matrix(A0)]
        self.P = []
        for l in range(levels - 1):
            nl = self.n[-1]
            if any(v % 2 for v in nl):
                raise ValueError("grid not divisible for %d levels" % levels)
            P = prolongation(nl)
            self.P.append(P)
            self.A.append(sp.csr_matrix(P.T @ self.A[-1] @ P))
            self.n.append(tuple(v // 2 for v in nl))
        self.levels = levels
        self.damping = list(damping)
        self.damping_p = list(damping_p) if damping_p is not None else list(damping)
        self.economic = economic
        self.cycle_index = cycle
        self.cycle_level = cycle_level
        self.nu1, self.nu2 = nu1, nu2
        self.blocks = []
        for l in range(levels - 1):
            self.blocks.append(vanka_blocks(self.A[l], self.n[l], economic))
        self.coarse_dd = None
        if coarse_dd is not None and any(v > 1 for v in coarse_dd[0]):
            self.coarse_dd = CoarseDD(self.A[-1], self.n[-1], coarse_dd[0], coarse_dd[1], coarse_dd[2])
            self.coarse_lu = None
        else:
            self.coarse_lu = spla.splu(sp.csc_matrix(self.A[-1]))

    def relax(self, l, b, e, c):
        B, dofs, colour = self.blocks[l]
        return vanka_half_sweep(self.A[l], B, dofs, colour, c, b, e, self.damping[l], self.damping_p[l])

    def cycle(self, b, l=0, e=None):
        """Algorithm 1 applied recursively; e = initial guess (zero if None)."""
        if l == self.levels - 1:
            if self.coarse_dd is not None:   # continues from the guess e (a second W call)
                return self.coarse_dd.solve(b, e)
            return self.coarse_lu.solve(np.asarray(b, dtype=np.complex128))
        e = np.zeros_like(b, dtype=np.complex128) if e is None else e.astype(np.complex128)
        for _ in range(self.nu1):
            e = self.relax(l, b, e, 0)
            e = self.relax(l, b, e, 1)
        rc = self.P[l].T @ (b - self.A[l] @ e)
        ec = None
        for _ in range(self.cycle_index if l >= self.cycle_level else 1):
            ec = self.cycle(rc, l + 1, ec)
        e = e + self.P[l] @ ec
        for _ in range(self.nu2):
            e = self.relax(l, b, e, 0)
            e = self.relax(l, b, e, 1)
        return e


def build_hierarchy(problem: disc.Problem, levels, damping, economic=False, cycle=1,
                    nu1=1, nu2=1, cycle_level=0, coarse_dd=None, damping_p=None):
    return Hierarchy(problem.matrix(shifted=True), problem.n, levels, damping,
                     economic, cycle, nu1, nu2, cycle_level, coarse_dd, damping_p)
