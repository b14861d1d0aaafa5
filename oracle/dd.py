"""Overlapping domain decomposition around the multigrid cycle (oracle, DD-MG;
DD-MG-DD when the subdomain hierarchies solve their coarsest level by DD too).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.3 and section 4: the domain is split into overlapping subdomains; each
is padded on its interior sides with an absorbing layer (the same quadratic
ramp as the outer layer of section 2.1), the medium in the padding is copied
from the global model, and the local shifted operator is approximately inverted
by one multigrid cycle.  Two schedules:

* one colour ("parallel version", section 2.3): every subdomain sees the
  restriction of the same residual and the local corrections are averaged on
  the overlaps;
* multicolour (Algorithm 2): subdomains of one colour are disjoint and handled
  together; colours are visited in turn, each starting from the residual of the
  global (unshifted) operator after the previous colours' corrections.  Reading
  of Algorithm 2: its inner loop runs over the subdomains of colour c and the
  local system is solved with the local residual as right-hand side.

Extent reading: subdomain i owns the cells [lo, hi) per axis; a face belongs to
it when both adjacent cells are inside; everything in the padding is zero on
restriction and discarded on extension.
"""
from __future__ import annotations

import itertools
from typing import List

import numpy as np
import scipy.sparse as sp

from . import discretisation as disc
from . import multigrid as mg


class Subdomain:
    def __init__(self, n, lo, hi, pad_lo, pad_hi, colour):
        self.lo, self.hi = tuple(lo), tuple(hi)
        self.pad_lo, self.pad_hi = tuple(pad_lo), tuple(pad_hi)
        self.origin = tuple(l - p for l, p in zip(lo, pad_lo))
        self.nloc = tuple(h - l + a + b for l, h, a, b in zip(lo, hi, pad_lo, pad_hi))
        self.colour = colour


def make_subdomains(n, parts, overlap, pad) -> List[Subdomain]:
    d = len(n)
    ranges = []
    for a in range(d):
        core = n[a] // parts[a]
        ax = []
        for p in range(parts[a]):
            lo = max(0, p * core - overlap // 2)
            hi = min(n[a], (p + 1) * core + (overlap - overlap // 2)) if p < parts[a] - 1 else n[a]
            if p == 0:
                lo = 0
            pl = pad if lo > 0 else 0
            ph = pad if hi < n[a] else 0
            ax.append((lo, hi, pl, ph, p))
        ranges.append(ax)
    subs = []
    # x fastest in the subdomain numbering
    for combo in itertools.product(*[range(parts[a]) for a in reversed(range(d))]):
        idx = tuple(reversed(combo))
        lo = [ranges[a][idx[a]][0] for a in range(d)]
        hi = [ranges[a][idx[a]][1] for a in range(d)]
        pl = [ranges[a][idx[a]][2] for a in range(d)]
        ph = [ranges[a][idx[a]][3] for a in range(d)]
        colour = sum((idx[a] % 2) << a for a in range(d))
        subs.append(Subdomain(n, lo, hi, pl, ph, colour))
    return subs


def _take_cells(field, sub: Subdomain, n):
    """Copy a global cell field onto the padded local grid (edge-replicated)."""
    d = len(n)
    idx = []
    for a in range(d):
        g = np.clip(np.arange(sub.nloc[a]) + sub.origin[a], 0, n[a] - 1)
        idx.append(g)
    # numpy axes are reversed
    return np.asarray(field)[np.ix_(*[idx[a] for a in reversed(range(d))])]


def padding_gamma(sub: Subdomain, abl_max):
    d = len(sub.nloc)
    g = np.zeros(tuple(reversed(sub.nloc)))
    for a in range(d):
        x = np.arange(sub.nloc[a]) + 0.5
        t = np.zeros(sub.nloc[a])
        if sub.pad_lo[a] > 0:
            L = sub.pad_lo[a]
            t = np.maximum(t, (L - x) / L)
        if sub.pad_hi[a] > 0:
            L = sub.pad_hi[a]
            t = np.maximum(t, (x - (sub.nloc[a] - L)) / L)
        bshape = [1] * d
        bshape[d - 1 - a] = sub.nloc[a]
        g = g + abl_max * (t * t).reshape(bshape)
    return g


def local_to_global(n, sub: Subdomain):
    """Global unknown index of every local unknown, -1 where outside the extent."""
    d = len(n)
    nl = sub.nloc
    out = []
    for k in range(d + 1):
        dims = disc.face_dims(nl, k) if k < d else nl
        grids = np.meshgrid(*[np.arange(dims[a]) for a in range(d)], indexing="ij")
        pos = [g.transpose(tuple(reversed(range(d)))).reshape(-1) for g in grids]
        ok = np.ones(pos[0].shape, dtype=bool)
        gpos = []
        for a in range(d):
            if a == k:
                f = pos[a] + 1 + sub.origin[a]          # global face position
                ok &= (f > sub.lo[a]) & (f < sub.hi[a])
                gpos.append(f)
            else:
                c = pos[a] + sub.origin[a]
                ok &= (c >= sub.lo[a]) & (c < sub.hi[a])
                gpos.append(c)
        gidx = -np.ones(pos[0].shape, dtype=np.int64)
        sel = np.nonzero(ok)[0]
        for s in sel:
            gidx[s] = disc.unknown_index(n, k, tuple(int(gp[s]) for gp in gpos))
        out.append(gidx)
    return np.concatenate(out)


def local_operator(problem: disc.Problem, sub: Subdomain, abl_max=1.0):
    """Shifted operator of a padded subdomain (section 4): the global medium
    copied onto the local grid (edge-replicated outside the domain), the
    subdomain's padding given the quadratic absorbing ramp of section 2.1, and
    the global shift."""
    n = problem.n
    lam = _take_cells(problem.lam, sub, n)
    mu = _take_cells(problem.mu, sub, n)
    rho = _take_cells(problem.rho, sub, n)
    gam = _take_cells(problem.gamma_hat, sub, n) + padding_gamma(sub, abl_max)
    return disc.assemble(sub.nloc, 1.0, problem.omega, lam, mu, rho, gam, problem.shift)


class DDPreconditioner:
    """DD-MG: one multigrid cycle of the local shifted operator per subdomain."""

    def __init__(self, problem: disc.Problem, parts, overlap, pad, levels, damping,
                 economic=False, cycle=1, colours=1, abl_max=1.0, coarse_dd=None, cycle_level=0, damping_p=None,
                 nu1=1, nu2=1):
        n = problem.n
        self.n = n
        self.problem = problem
        self.subs = make_subdomains(n, parts, overlap, pad)
        self.colours = colours
        self.A = problem.matrix(shifted=False)
        self.maps, self.hier = [], []
        cnt = np.zeros(problem.size)
        for sub in self.subs:
            A_loc = local_operator(problem, sub, abl_max)
            self.hier.append(mg.Hierarchy(A_loc, sub.nloc, levels, damping, economic, cycle, nu1=nu1, nu2=nu2,
                                          cycle_level=cycle_level, coarse_dd=coarse_dd, damping_p=damping_p))
            m = local_to_global(n, sub)
            self.maps.append(m)
            cnt[m[m >= 0]] += 1
        if np.any(cnt == 0):
            raise ValueError("subdomains do not cover every unknown")
        self.weight = 1.0 / cnt

    def restrict(self, i, v):
        m = self.maps[i]
        out = np.zeros(m.shape[0], dtype=np.complex128)
        ok = m >= 0
        out[ok] = v[m[ok]]
        return out

    def apply(self, v):
        v = np.asarray(v, dtype=np.complex128)
        z = np.zeros_like(v)
        if self.colours == 1:
            for i in range(len(self.subs)):
                e = self.hier[i].cycle(self.restrict(i, v))
                m = self.maps[i]
                ok = m >= 0
                np.add.at(z, m[ok], self.weight[m[ok]] * e[ok])
            return z
        for c in sorted(set(s.colour for s in self.subs)):
            r = v - self.A @ z
            for i, sub in enumerate(self.subs):
                if sub.colour != c:
                    continue
                e = self.hier[i].cycle(self.restrict(i, r))
                m = self.maps[i]
                ok = m >= 0
                np.add.at(z, m[ok], e[ok])
        return z
