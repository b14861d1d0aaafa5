"""Direct solution of the assembled system (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The plain definition of the result of a solve: x = A^{-1} b with A the sparse
matrix of eq. (14) (or any matrix of the staggered layout), factorised once by
sparse LU (SuperLU) and applied to many right-hand sides.  The unknowns are
ordered by geometric nested dissection (George, 1973): the staggered grid is
cut recursively across its longest axis by a separator band of unknowns, the
two halves first, the band last, which keeps the fill of a 2D factorisation
near N log N (256^2 cells: 3.9e7 nonzeros in L + U against 4.5e7 with SuperLU's
column minimum-degree order, and a 3.4 times faster factorisation; 512^2: 21 s
against 186 s on one core).  The column order given to SuperLU is then the
natural one, with threshold partial pivoting kept.

Coupling range used for the separator (section 2.1): every row of A couples a
unknown only to unknowns within one cell width along each axis (u_k to u_k at
distance 1, u_k to the two cells at distance 1/2 along its normal, p to the
faces of its cell), so the unknowns whose coordinate along the cut axis lies in
[c - 1/2, c] separate those below from those above.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import discretisation as disc


def unknown_coordinates(n):
    """(N, d) positions of the unknowns in cell widths: u_k at its face
    (integer along axis k, half-integer across), p at the cell centre."""
    d = len(n)
    out = []
    for k in range(d + 1):
        dims = disc.face_dims(n, k) if k < d else tuple(n)
        grids = np.meshgrid(*[np.arange(v, dtype=float) for v in dims], indexing="ij")
        pos = [g.transpose(tuple(reversed(range(d)))).reshape(-1) for g in grids]
        cols = []
        for a in range(d):
            cols.append(pos[a] + 1.0 if a == k else pos[a] + 0.5)
        out.append(np.stack(cols, axis=1))
    return np.concatenate(out)


def nested_dissection(n, leaf=64):
    """Permutation (new position -> unknown) of the staggered unknowns of grid n."""
    X = unknown_coordinates(n)
    order = []

    def cut(idx):
        if idx.size <= leaf:
            order.append(idx)
            return
        pts = X[idx]
        ext = pts.max(axis=0) - pts.min(axis=0)
        a = int(np.argmax(ext))
        c = np.round(np.median(pts[:, a]))
        lo = pts[:, a] < c - 0.5
        hi = pts[:, a] > c
        band = ~(lo | hi)
        if not lo.any() or not hi.any():
            order.append(idx)
            return
        cut(idx[lo])
        cut(idx[hi])
        order.append(idx[band])

    cut(np.arange(X.shape[0]))
    perm = np.concatenate(order)
    return perm


class DirectSolver:
    """x = A^{-1} b for the staggered system of grid n (A any sparse matrix of
    that layout), factorised once."""

    def __init__(self, A, n):
        A = sp.csc_matrix(A)
        self.perm = nested_dissection(tuple(n))
        Ap = sp.csc_matrix(A[self.perm][:, self.perm])
        self.lu = spla.splu(Ap, permc_spec="NATURAL", diag_pivot_thresh=0.1,
                            options=dict(SymmetricMode=True))
        self.nnz = int(self.lu.L.nnz + self.lu.U.nnz)

    def solve(self, b):
        b = np.asarray(b, dtype=np.complex128)
        xp = self.lu.solve(b[self.perm])
        x = np.empty_like(xp)
        x[self.perm] = xp
        return x


def factorize(problem: "disc.Problem") -> DirectSolver:
    """Direct solver of the unshifted system of eq. (14) of a problem."""
    return DirectSolver(problem.matrix(), problem.n)
