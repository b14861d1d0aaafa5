"""Pins of the oracle's discretisation against facts fixed by the paper and by the
mathematics (not against the oracle itself)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import discretisation as disc
from workloads import get_config


def _face_points(n, h, k):
    """Coordinates (x, y[, z]) of every unknown of component k, flattened x fastest."""
    d = len(n)
    dims = disc.face_dims(n, k)
    axes = []
    for a in range(d):
        if a == k:
            axes.append((np.arange(dims[a]) + 1) * h)
        else:
            axes.append((np.arange(dims[a]) + 0.5) * h)
    grids = np.meshgrid(*axes, indexing="ij")
    return [g.transpose(tuple(reversed(range(d)))).reshape(-1) for g in grids]


def _cell_points(n, h):
    d = len(n)
    axes = [(np.arange(n[a]) + 0.5) * h for a in range(d)]
    grids = np.meshgrid(*axes, indexing="ij")
    return [g.transpose(tuple(reversed(range(d)))).reshape(-1) for g in grids]


def _interior_masks(n):
    """Masks of rows whose stencil stays away from every wall."""
    d = len(n)
    masks = []
    for k in range(d):
        dims = disc.face_dims(n, k)
        grids = np.meshgrid(*[np.arange(dims[a]) for a in range(d)], indexing="ij")
        pos = [g.transpose(tuple(reversed(range(d)))).reshape(-1) for g in grids]
        ok = np.ones(pos[0].shape, dtype=bool)
        for a in range(d):
            if a == k:   # face index f = pos+1 must satisfy 2 <= f <= n-2
                ok &= (pos[a] + 1 >= 2) & (pos[a] + 1 <= n[a] - 2)
            else:
                ok &= (pos[a] >= 1) & (pos[a] <= n[a] - 2)
        masks.append(ok)
    grids = np.meshgrid(*[np.arange(n[a]) for a in range(d)], indexing="ij")
    pos = [g.transpose(tuple(reversed(range(d)))).reshape(-1) for g in grids]
    ok = np.ones(pos[0].shape, dtype=bool)
    for a in range(d):
        ok &= (pos[a] >= 1) & (pos[a] <= n[a] - 2)
    masks.append(ok)
    return masks


def _plane_wave(n, h, kvec, amp, lam, mu):
    """u_k = a_k exp(i k.x) at the staggered face points; p = (lam+mu) grad_h^T u written
    in closed form, p = -(lam+mu) (2i/h) (s.a) exp(i k.x) at cell centres (eq. (13))."""
    d = len(n)
    parts = []
    for k in range(d):
        X = _face_points(n, h, k)
        ph = sum(kvec[a] * X[a] for a in range(d))
        parts.append(amp[k] * np.exp(1j * ph))
    s = np.array([math.sin(kvec[a] * h / 2) for a in range(d)])
    X = _cell_points(n, h)
    ph = sum(kvec[a] * X[a] for a in range(d))
    parts.append(-(lam + mu) * (2j / h) * np.dot(s, amp) * np.exp(1j * ph))
    return np.concatenate(parts), s


@pytest.mark.parametrize("n", [(14, 11), (9, 8, 7)])
def test_plane_wave_symbol(n):
    """Homogeneous, undamped: p-rows vanish and u-rows equal the discrete symbol
    (4/h^2)[(lam+mu) s s^T + mu |s|^2 I] a - w^2 rho a (sections 2.1 and 5)."""
    d = len(n)
    h, lam, mu, rho, omega = 0.7, 2.3, 1.1, 0.9, 1.7
    shape = tuple(reversed(n))
    A = disc.assemble(n, h, omega, np.full(shape, lam), np.full(shape, mu), np.full(shape, rho),
                      np.zeros(shape), 0.0, "mixed")
    He = disc.assemble(n, h, omega, np.full(shape, lam), np.full(shape, mu), np.full(shape, rho),
                       np.zeros(shape), 0.0, "u")
    kvec = np.array([0.9, -0.55, 0.4][:d])
    amp = np.array([0.8, -0.3 + 0.2j, 0.5j][:d])
    x, s = _plane_wave(n, h, kvec, amp, lam, mu)
    y = A @ x
    sym = (4 / h ** 2) * ((lam + mu) * s * np.dot(s, amp) + mu * np.dot(s, s) * amp) - omega ** 2 * rho * amp
    off = disc.offsets(n)
    masks = _interior_masks(n)
    yp = y[off[d]:][masks[d]]
    assert np.max(np.abs(yp)) < 1e-12
    nu_ = sum(disc.counts(n)[:d])
    yu = He @ x[:nu_]
    for k in range(d):
        X = _face_points(n, h, k)
        ph = np.exp(1j * sum(kvec[a] * X[a] for a in range(d)))
        expect = sym[k] * ph
        got = y[off[k]:off[k + 1]]
        m = masks[k]
        assert np.max(np.abs(got[m] - expect[m])) < 1e-11 * np.max(np.abs(expect))
        got_u = yu[off[k]:off[k + 1]]
        assert np.max(np.abs(got_u[m] - expect[m])) < 1e-11 * np.max(np.abs(expect))


@pytest.mark.parametrize("kind", ["P", "S"])
def test_dispersion_relation(kind):
    """A P wave (a || s) is annihilated iff w^2 rho = (4/h^2)(lam+2mu)|s|^2 and an S
    wave (a perp s) iff w^2 rho = (4/h^2) mu |s|^2 (interior rows, exact to roundoff)."""
    n = (16, 13)
    h, lam, mu, rho = 0.5, 3.0, 1.0, 1.3
    kvec = np.array([0.7, 1.1])
    s = np.sin(kvec * h / 2)
    if kind == "P":
        amp = s.astype(complex)
        omega = math.sqrt(4 / h ** 2 * (lam + 2 * mu) * np.dot(s, s) / rho)
    else:
        amp = np.array([-s[1], s[0]], dtype=complex)
        omega = math.sqrt(4 / h ** 2 * mu * np.dot(s, s) / rho)
    shape = tuple(reversed(n))
    A = disc.assemble(n, h, omega, np.full(shape, lam), np.full(shape, mu), np.full(shape, rho),
                      np.zeros(shape), 0.0, "mixed")
    x, _ = _plane_wave(n, h, kvec, amp, lam, mu)
    y = A @ x
    off = disc.offsets(n)
    for k, m in enumerate(_interior_masks(n)):
        seg = y[off[k]:off[k + 1]][m]
        assert np.max(np.abs(seg)) < 1e-10 * (4 / h ** 2) * (lam + 2 * mu)


def test_interior_rows_equal_section5_stencils():
    """Constant coefficients: interior u-rows carry s00 = 4mu/h^2 - rho w^2 (1 - i gamma)
    and -mu/h^2 at the four neighbours (eq. (19)-(20)), and +-1/h on the two pressures
    (eq. (21)-(22)); the p-row carries the negated first differences and -1/(lam+mu)."""
    n = (8, 7)
    h, lam, mu, rho, omega, gam = 0.25, 5.0, 1.5, 2.0, 3.0, 0.3
    shape = tuple(reversed(n))
    A = disc.assemble(n, h, omega, np.full(shape, lam), np.full(shape, mu), np.full(shape, rho),
                      np.full(shape, gam), 0.0).tolil()
    s00 = 4 * mu / h ** 2 - rho * omega ** 2 * (1 - 1j * gam)
    i, j = 4, 3                      # interior u_0 face (x-face 4 in row 3)
    r = disc.unknown_index(n, 0, (i, j))
    assert abs(A[r, r] - s00) < 1e-12
    for pos in [(i + 1, j), (i - 1, j), (i, j + 1), (i, j - 1)]:
        assert abs(A[r, disc.unknown_index(n, 0, pos)] + mu / h ** 2) < 1e-12
    assert abs(A[r, disc.unknown_index(n, 2, (i, j))] - 1 / h) < 1e-12
    assert abs(A[r, disc.unknown_index(n, 2, (i - 1, j))] + 1 / h) < 1e-12
    assert A[r].nnz == 7
    c = disc.unknown_index(n, 2, (i, j))
    assert abs(A[c, c] + 1 / (lam + mu)) < 1e-15
    assert abs(A[c, disc.unknown_index(n, 0, (i, j))] - 1 / h) < 1e-12
    assert abs(A[c, disc.unknown_index(n, 0, (i + 1, j))] + 1 / h) < 1e-12
    assert abs(A[c, disc.unknown_index(n, 1, (i, j))] - 1 / h) < 1e-12
    assert abs(A[c, disc.unknown_index(n, 1, (i, j + 1))] + 1 / h) < 1e-12


def test_edge_weights_are_arithmetic_means_of_a_linear_mu():
    """For mu linear in x and y the arithmetic cell mean at a face/node equals mu at
    that point, so every Laplacian off-diagonal must be -mu(point)/h^2 with the point
    midway between the two coupled unknowns; at a wall node the mean of the two
    existing cells is taken."""
    n = (7, 6)
    h = 0.5
    X = _cell_points(n, h)
    mu_fn = lambda x, y: 1.0 + 0.3 * x + 0.2 * y
    mu = mu_fn(X[0], X[1]).reshape(tuple(reversed(n)))
    shape = tuple(reversed(n))
    A = disc.assemble(n, h, 0.0, np.full(shape, 1.0), mu, np.ones(shape), np.zeros(shape)).tolil()
    for (f, j) in [(1, 0), (3, 2), (5, 4), (2, 5)]:
        r = disc.unknown_index(n, 0, (f, j))
        # normal neighbour f+1: coupling through the cell f
        if f + 1 <= n[0] - 1:
            got = A[r, disc.unknown_index(n, 0, (f + 1, j))]
            assert abs(got + mu_fn((f + 0.5) * h, (j + 0.5) * h) / h ** 2) < 1e-12
        # tangential neighbour j+1: node at (f h, (j+1) h)
        if j + 1 <= n[1] - 1:
            got = A[r, disc.unknown_index(n, 0, (f, j + 1))]
            assert abs(got + mu_fn(f * h, (j + 1) * h) / h ** 2) < 1e-12
    # wall row j = 0: the diagonal holds the two cell weights, the interior node weight
    # and the wall node weight = mean of the two existing cells = mu(f h, h/2).
    f, j = 3, 0
    r = disc.unknown_index(n, 0, (f, j))
    expect = (mu_fn((f - 0.5) * h, 0.5 * h) + mu_fn((f + 0.5) * h, 0.5 * h)
              + mu_fn(f * h, h) + mu_fn(f * h, 0.5 * h)) / h ** 2
    assert abs(A[r, r] - expect) < 1e-12


def _hetero(n, seed=0):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    mu = rng.uniform(0.5, 2.0, shape)
    lam = mu * rng.uniform(0.5, 8.0, shape)
    rho = rng.uniform(0.7, 1.5, shape)
    gam = disc.abl_gamma(n, [2] * len(n), 1.0) + 0.01
    return lam, mu, rho, gam


@pytest.mark.parametrize("n", [(8, 6), (4, 5, 3)])
@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_complex_symmetry(n, shift):
    """A^T = A (no conjugation): real grad blocks appear transposed and M is diagonal."""
    lam, mu, rho, gam = _hetero(n)
    A = disc.assemble(n, 1.0, 1.3, lam, mu, rho, gam, shift)
    assert abs(A - A.T).max() == 0.0
    H = disc.assemble(n, 1.0, 1.3, lam, mu, rho, gam, shift, "u")
    assert abs(H - H.T).max() < 1e-14 * abs(H).max()


def test_schur_complement_equals_u_system():
    """H^e of eq. (4) is the Schur complement of eq. (14): the u parts of the two solves agree."""
    n = (10, 9)
    lam, mu, rho, gam = _hetero(n, 1)
    A = disc.assemble(n, 1.0, 0.9, lam, mu, rho, gam)
    H = disc.assemble(n, 1.0, 0.9, lam, mu, rho, gam, 0.0, "u")
    rng = np.random.default_rng(3)
    nu_ = sum(disc.counts(n)[:2])
    q = rng.standard_normal(nu_) + 1j * rng.standard_normal(nu_)
    b = np.concatenate([q, np.zeros(disc.counts(n)[2])])
    x = spla.spsolve(A.tocsc(), b)
    u = spla.spsolve(H.tocsc(), q)
    assert np.linalg.norm(x[:nu_] - u) < 1e-11 * np.linalg.norm(u)


def test_acoustic_reduction():
    """mu = 0, gamma = 0: eliminating u leaves (1/w^2) times the textbook cell-centred
    five-point discretisation of -div(rho^-1 grad p) - w^2 p / lambda with no-flux
    walls and face densities averaged arithmetically (section 3, eq. (15))."""
    n = (6, 5)
    h, omega = 0.4, 1.9
    rng = np.random.default_rng(5)
    shape = tuple(reversed(n))
    lam = rng.uniform(1.0, 3.0, shape)
    rho = rng.uniform(0.5, 2.0, shape)
    A = disc.assemble(n, h, omega, lam, np.zeros(shape), rho, np.zeros(shape)).toarray()
    nu_ = sum(disc.counts(n)[:2])
    Auu, Aup, Apu, App = A[:nu_, :nu_], A[:nu_, nu_:], A[nu_:, :nu_], A[nu_:, nu_:]
    S = App - Apu @ np.linalg.solve(Auu, Aup)
    # textbook scheme, written cell by cell
    N = n[0] * n[1]
    T = np.zeros((N, N))
    cid = lambda i, j: j * n[0] + i
    for j in range(n[1]):
        for i in range(n[0]):
            r = cid(i, j)
            for (ii, jj) in [(i + 1, j), (i - 1, j), (i, j + 1), (i, j - 1)]:
                if 0 <= ii < n[0] and 0 <= jj < n[1]:
                    rf = 0.5 * (rho[j, i] + rho[jj, ii])
                    T[r, r] += 1.0 / (rf * h * h)
                    T[r, cid(ii, jj)] -= 1.0 / (rf * h * h)
            T[r, r] -= omega ** 2 / lam[j, i]
    assert np.max(np.abs(omega ** 2 * S - T)) < 1e-10 * np.max(np.abs(T))


@pytest.mark.parametrize("n", [(6, 6), (8, 8), (4, 4, 4)])
def test_dense_bruteforce_matches_sparse_lu(n):
    lam, mu, rho, gam = _hetero(n, 7)
    A = disc.assemble(n, 1.0, 1.1, lam, mu, rho, gam, 0.2)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    x_dense = np.linalg.solve(A.toarray(), b)
    x_lu = spla.splu(A.tocsc()).solve(b)
    assert np.linalg.norm(x_dense - x_lu) <= 1e-12 * np.linalg.norm(x_dense) * 10


@pytest.mark.parametrize("n", [(12, 10), (16, 16), (6, 4, 6)])
def test_nested_dissection_direct_solve_matches_dense_bruteforce(n):
    """The oracle's direct solver (SuperLU on the nested-dissection order of the
    staggered unknowns) gives the dense brute-force solution, and its order is
    a permutation of every unknown."""
    from oracle import direct
    lam, mu, rho, gam = _hetero(n, 17)
    A = disc.assemble(n, 1.0, 0.9, lam, mu, rho, gam, 0.0)
    perm = direct.nested_dissection(n, leaf=8)
    assert np.array_equal(np.sort(perm), np.arange(A.shape[0]))
    rng = np.random.default_rng(18)
    b = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    x_dense = np.linalg.solve(A.toarray(), b)
    x = direct.DirectSolver(A, n).solve(b)
    assert np.linalg.norm(x - x_dense) <= 1e-11 * np.linalg.norm(x_dense)


@pytest.mark.parametrize("n", [(16, 12), (8, 6, 10)])
def test_nested_dissection_band_separates(n):
    """The separator reading: no nonzero of A couples an unknown below the band
    [c - 1/2, c] of the first cut with one above it."""
    from oracle import direct
    lam, mu, rho, gam = _hetero(n, 19)
    A = sp.coo_matrix(disc.assemble(n, 1.0, 0.9, lam, mu, rho, gam, 0.3))
    X = direct.unknown_coordinates(n)
    a = int(np.argmax(n))
    c = np.round(np.median(X[:, a]))
    lo, hi = X[:, a] < c - 0.5, X[:, a] > c
    nz = np.abs(A.data) > 0
    assert lo.sum() > 0 and hi.sum() > 0
    assert not np.any(nz & lo[A.row] & hi[A.col])
    assert not np.any(nz & hi[A.row] & lo[A.col])


def test_discrete_manufactured_solution():
    n = (24, 20)
    lam, mu, rho, gam = _hetero(n, 9)
    A = disc.assemble(n, 1.0, 0.8, lam, mu, rho, gam)
    rng = np.random.default_rng(10)
    xs = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    x = spla.splu(A.tocsc()).solve(A @ xs)
    assert np.linalg.norm(x - xs) < 1e-9 * np.linalg.norm(xs)


def _mms_error(nc):
    import sympy as S
    x, y = S.symbols("x y")
    lam, mu, rho, omega, gam, sig = 2.0, 1.0, 1.0, 4.0, 0.1, 0.1
    phi = S.exp(-((x - 0.5) ** 2 + (y - 0.45) ** 2) / sig ** 2)
    psi = 0.7 * S.exp(-((x - 0.48) ** 2 + (y - 0.52) ** 2) / sig ** 2)
    div = S.diff(phi, x) + S.diff(psi, y)
    m = rho * (1 - S.I * gam)
    q0 = -(lam + mu) * S.diff(div, x) - mu * (S.diff(phi, x, 2) + S.diff(phi, y, 2)) - omega ** 2 * m * phi
    q1 = -(lam + mu) * S.diff(div, y) - mu * (S.diff(psi, x, 2) + S.diff(psi, y, 2)) - omega ** 2 * m * psi
    f = {k: S.lambdify((x, y), e, "numpy") for k, e in
         dict(q0=q0, q1=q1, u0=phi, u1=psi, p=-(lam + mu) * div).items()}
    n = (nc, nc)
    h = 1.0 / nc
    shape = tuple(reversed(n))
    A = disc.assemble(n, h, omega, np.full(shape, lam), np.full(shape, mu), np.full(shape, rho),
                      np.full(shape, gam))
    X0, X1, XC = _face_points(n, h, 0), _face_points(n, h, 1), _cell_points(n, h)
    b = np.concatenate([f["q0"](*X0) + 0j, f["q1"](*X1) + 0j, np.zeros(nc * nc, complex)])
    sol = spla.splu(A.tocsc()).solve(b)
    ex = np.concatenate([f["u0"](*X0) + 0 * X0[0], f["u1"](*X1) + 0 * X1[0]])
    nu_ = ex.size
    eu = np.max(np.abs(sol[:nu_] - ex))
    ep = np.max(np.abs(sol[nu_:] - f["p"](*XC)))
    return eu, ep


def test_manufactured_solution_second_order():
    """Central differences of section 2.1 are second order: halving h divides the
    max error of u and p by about 4 (smooth bump far from the walls)."""
    e1u, e1p = _mms_error(32)
    e2u, e2p = _mms_error(64)
    assert 3.3 < e1u / e2u < 4.7
    assert 3.3 < e1p / e2p < 4.7


def test_reciprocity():
    """G_ab = G_ba (A^T = A) for a heterogeneous medium with the absorbing layer."""
    n = (12, 10)
    lam, mu, rho, gam = _hetero(n, 11)
    A = disc.assemble(n, 1.0, 1.0, lam, mu, rho, gam)
    lu = spla.splu(A.tocsc())
    a = disc.unknown_index(n, 0, (3, 4))
    b = disc.unknown_index(n, 1, (8, 6))
    ea = np.zeros(A.shape[0], complex); ea[a] = 1
    eb = np.zeros(A.shape[0], complex); eb[b] = 1
    assert abs(lu.solve(ea)[b] - lu.solve(eb)[a]) < 1e-12 * abs(lu.solve(ea)[b])


def _c1():
    w = get_config("c1_homog64")
    m = w.media()
    pb = disc.Problem(w.n, w.h, w.omega, m["lam"], m["mu"], m["rho"], w.abl_cells, w.abl_max, w.atten0)
    b = disc.point_source_vector(w.n, w.sources())
    return w, pb, b


def test_c1_mirror_symmetry():
    """Homogeneous c1 with the x-force on the central x-face: u_1 even, u_2 and p odd in x."""
    w, pb, b = _c1()
    A = pb.matrix()
    x = spla.splu(A.tocsc()).solve(b)
    u0, u1, p = disc.split(w.n, x)
    assert np.max(np.abs(u0 - u0[:, ::-1])) < 1e-10 * np.max(np.abs(u0))
    assert np.max(np.abs(u1 + u1[:, ::-1])) < 1e-10 * np.max(np.abs(u0))
    assert np.max(np.abs(p + p[:, ::-1])) < 1e-10 * np.max(np.abs(p))


def test_c1_gmres_equals_direct():
    w, pb, b = _c1()
    A = pb.matrix().tocsc()
    x = spla.splu(A).solve(b)
    lu = spla.splu(pb.matrix(shifted=True).tocsc())
    Mop = spla.LinearOperator(A.shape, matvec=lu.solve, dtype=complex)
    xg, info = spla.gmres(A, b, M=Mop, rtol=1e-10, restart=50, maxiter=200)
    assert info == 0
    assert np.linalg.norm(xg - x) < 1e-7 * np.linalg.norm(x)


def test_nondimensional_scaling_identity():
    """The SI system equals diag(mu/h^2, 1/h) A_nd diag(1, h/mu) (section 2.1 units)."""
    n = (6, 5)
    rng = np.random.default_rng(2)
    shape = tuple(reversed(n))
    mu = rng.uniform(1e9, 3e9, shape)
    lam = mu * rng.uniform(1.0, 5.0, shape)
    rho = rng.uniform(1500.0, 2500.0, shape)
    gam = disc.abl_gamma(n, (2, 2), 1.0)
    h, omega = 10.0, 40.0
    A_si = disc.assemble(n, h, omega, lam, mu, rho, gam, 0.3).toarray()
    nd = disc.nondimensionalise(h, omega, lam, mu, rho)
    A_nd = disc.assemble(n, 1.0, nd["omega"], nd["lam"], nd["mu"], nd["rho"], gam, 0.3).toarray()
    nu_ = sum(disc.counts(n)[:2])
    N = A_si.shape[0]
    left = np.concatenate([np.full(nu_, nd["mu_bar"] / h ** 2), np.full(N - nu_, 1.0 / h)])
    right = np.concatenate([np.ones(nu_), np.full(N - nu_, h / nd["mu_bar"])])
    rebuilt = left[:, None] * A_nd * right[None, :]
    assert np.max(np.abs(rebuilt - A_si)) < 1e-12 * np.max(np.abs(A_si))


def test_absorbing_layer_profile():
    """Quadratic ramp: zero outside the layer, increasing towards each wall, at most
    abl_max per axis, summed in corners."""
    n = (30, 30)
    g = disc.abl_gamma(n, (10, 10), 1.0)
    assert np.all(g[10:-10, 10:-10] == 0.0)
    row = g[15, :]
    assert np.all(np.diff(row[:10]) < 0) and np.all(np.diff(row[-10:]) > 0)
    assert row[0] == pytest.approx(0.95 ** 2) and row[9] == pytest.approx(0.05 ** 2)
    assert np.max(g) <= 2.0 and g[0, 0] == pytest.approx(2 * 0.95 ** 2)
