"""Pins of the oracle's adjoint-state media gradient (no GPU).

The gradient formulas are checked against things that do not use them:
central finite differences of the misfit through sparse direct solves, the exact
matrix difference where A is linear in the perturbation, and the adjoint
identity y^H b = g^H x."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from _helpers import small_hetero
from oracle import discretisation as D
from oracle import gradient as G


def _setup(n, nsrc, seed):
    w = small_hetero(n, f"grad{len(n)}d")
    m = w.media()
    rng = np.random.default_rng(seed)
    pb = D.Problem(w.n, w.h, w.omega, m["lam"], m["mu"], m["rho"], w.abl_cells, w.abl_max, w.atten0)
    N = pb.size
    # sources: x-forces near the top; receivers: every u_0 unknown of row 1
    B = np.zeros((nsrc, N), dtype=np.complex128)
    for s in range(nsrc):
        pos = (1 + (s * (n[0] - 2)) // max(nsrc, 1),) + (n[1] // 2,) * (len(n) - 2) + (1,)
        B[s, D.unknown_index(w.n, 0, pos)] = np.exp(1j * rng.uniform(0, 2 * np.pi))
    rec = np.array([D.unknown_index(w.n, 0, (i,) + (n[1] // 2,) * (len(n) - 2) + (2,))
                    for i in range(1, n[0])])
    d_obs = rng.standard_normal((nsrc, rec.size)) * 1e-3 + 1j * rng.standard_normal((nsrc, rec.size)) * 1e-3
    return w, m, pb, B, rec, d_obs


def _misfit(w, m, B, rec, d_obs, mu_bar, rho_bar, lam=None, mu=None, rho=None):
    pb = D.Problem(w.n, w.h, w.omega, m["lam"] if lam is None else lam, m["mu"] if mu is None else mu,
                   m["rho"] if rho is None else rho, w.abl_cells, w.abl_max, w.atten0,
                   mu_bar=mu_bar, rho_bar=rho_bar)
    lu = spla.splu(pb.matrix().tocsc())
    X = np.stack([lu.solve(b) for b in B])
    return G.receiver_misfit(X, rec, d_obs)[0]


def _gradient(pb, B, rec, d_obs):
    A = pb.matrix()
    lu = spla.splu(A.tocsc())
    X = np.stack([lu.solve(b) for b in B])
    L, g = G.receiver_misfit(X, rec, d_obs)
    Y = G.adjoint_solve(A, g)
    return X, Y, g, G.media_gradient(pb.n, pb.omega, pb.lam, pb.mu, pb.rho, pb.gamma_hat, Y, X,
                                     pb.nd["mu_bar"], pb.nd["rho_bar"])


@pytest.mark.parametrize("n,nsrc,ncells", [((14, 12), 3, 20), ((6, 5, 6), 2, 12)])
def test_gradient_matches_central_differences(n, nsrc, ncells):
    """Central differences with a step of 1e-4 of the cell value (fixed units)
    on random cells and all three media."""
    w, m, pb, B, rec, d_obs = _setup(n, nsrc, 11)
    mu_bar, rho_bar = pb.nd["mu_bar"], pb.nd["rho_bar"]
    _, _, _, grads = _gradient(pb, B, rec, d_obs)
    rng = np.random.default_rng(12)
    flat_cells = rng.choice(int(np.prod(n)), size=ncells, replace=False)
    names = ["lam", "mu", "rho"]
    for j, c in enumerate(flat_cells):
        which = j % 3
        base = m[names[which]]
        step = 1e-4 * abs(base.reshape(-1)[c])
        vals = []
        for sgn in (1.0, -1.0):
            pert = base.copy().reshape(-1)
            pert[c] += sgn * step
            vals.append(_misfit(w, m, B, rec, d_obs, mu_bar, rho_bar, **{names[which]: pert.reshape(base.shape)}))
        fd = (vals[0] - vals[1]) / (2 * step)
        an = grads[which].reshape(-1)[c]
        scale = np.abs(grads[which]).max()
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-7 * scale, (names[which], c, fd, an)


def test_laplacian_and_mass_terms_are_exact_matrix_differences():
    """A is linear in rho (mass) and, at fixed lambda + mu, in mu (Laplacian), so
    Re y^H (A(m + delta e_c) - A(m)) x / delta equals -(dL/dm_c) * unit exactly,
    for every cell of a small grid."""
    n = (6, 5)
    w, m, pb, B, rec, d_obs = _setup(n, 2, 21)
    mu_bar, rho_bar = pb.nd["mu_bar"], pb.nd["rho_bar"]
    X, Y, _, (g_lam, g_mu, g_rho) = _gradient(pb, B, rec, d_obs)
    A0 = pb.matrix()

    def contraction(A1, delta):
        dA = A1 - A0
        return sum(np.real(np.vdot(y, dA @ x)) for y, x in zip(Y, X)) / delta

    for c in range(int(np.prod(n))):
        delta = 0.3 * m["rho"].reshape(-1)[c]
        rho = m["rho"].copy().reshape(-1)
        rho[c] += delta
        A1 = D.Problem(w.n, w.h, w.omega, m["lam"], m["mu"], rho.reshape(m["rho"].shape), w.abl_cells,
                       w.abl_max, w.atten0, mu_bar=mu_bar, rho_bar=rho_bar).matrix()
        assert abs(contraction(A1, delta) + g_rho.reshape(-1)[c]) <= 1e-10 * np.abs(g_rho).max()
        delta = 0.2 * m["mu"].reshape(-1)[c]
        mu = m["mu"].copy().reshape(-1)
        lam = m["lam"].copy().reshape(-1)
        mu[c] += delta
        lam[c] -= delta
        A1 = D.Problem(w.n, w.h, w.omega, lam.reshape(m["lam"].shape), mu.reshape(m["mu"].shape), m["rho"],
                       w.abl_cells, w.abl_max, w.atten0, mu_bar=mu_bar, rho_bar=rho_bar).matrix()
        want = g_mu.reshape(-1)[c] - g_lam.reshape(-1)[c]
        assert abs(contraction(A1, delta) + want) <= 1e-10 * np.abs(g_mu).max()


def test_adjoint_identity():
    """For A x = b and A^H y = g: y^H b = g^H x."""
    n = (10, 8)
    w, m, pb, B, rec, d_obs = _setup(n, 2, 31)
    A = pb.matrix()
    lu = spla.splu(A.tocsc())
    rng = np.random.default_rng(32)
    g = rng.standard_normal((2, pb.size)) + 1j * rng.standard_normal((2, pb.size))
    Y = G.adjoint_solve(A, g)
    for r in range(2):
        x = lu.solve(B[r])
        assert abs(np.vdot(Y[r], B[r]) - np.vdot(g[r], x)) <= 1e-10 * abs(np.vdot(g[r], x))
        assert np.linalg.norm(A.conj().T @ Y[r] - g[r]) <= 1e-10 * np.linalg.norm(g[r])


def test_fixed_units_leave_the_operator_of_the_mean_units_unchanged():
    """Passing the media means as the units reproduces the default scaling."""
    w = small_hetero((8, 6), "units")
    m = w.media()
    p0 = D.Problem(w.n, w.h, w.omega, m["lam"], m["mu"], m["rho"], w.abl_cells, w.abl_max, w.atten0)
    p1 = D.Problem(w.n, w.h, w.omega, m["lam"], m["mu"], m["rho"], w.abl_cells, w.abl_max, w.atten0,
                   mu_bar=float(np.mean(m["mu"])), rho_bar=float(np.mean(m["rho"])))
    assert abs(p0.matrix() - p1.matrix()).max() == 0.0
