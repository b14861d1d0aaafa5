"""Pins of the oracle's multigrid, DD and FGMRES parts."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import discretisation as disc
from oracle import multigrid as mg
from oracle import dd as ddm
from oracle import krylov


def _hetero(n, seed=0, abl=2):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    mu = rng.uniform(0.5, 2.0, shape)
    lam = mu * rng.uniform(0.5, 8.0, shape)
    rho = rng.uniform(0.7, 1.5, shape)
    gam = disc.abl_gamma(n, [abl] * len(n), 1.0) + 0.01
    return lam, mu, rho, gam


def _positions(dims):
    d = len(dims)
    grids = np.meshgrid(*[np.arange(v) for v in dims], indexing="ij")
    return [g.transpose(tuple(reversed(range(d)))).reshape(-1) for g in grids]


@pytest.mark.parametrize("n", [(16, 12), (8, 8, 12)])
def test_prolongation_reproduces_linear_fields(n):
    """Bilinear staggered interpolation reproduces any linear field at fine points
    whose interpolation stencil stays inside the coarse grid (section 3)."""
    d = len(n)
    nc = tuple(v // 2 for v in n)
    P = mg.prolongation(n)
    coef = np.array([0.3, -0.7, 0.45][:d])
    xs = []
    fine_pos, fine_ok = [], []
    for k in range(d + 1):
        cd = disc.face_dims(nc, k) if k < d else nc
        fd = disc.face_dims(n, k) if k < d else n
        cp, fp = _positions(cd), _positions(fd)
        # physical coordinates in fine-cell units (coarse cell = 2 fine cells)
        cx = [2.0 * (cp[a] + 1) if a == k else 2.0 * (cp[a] + 0.5) for a in range(d)]
        fx = [(fp[a] + 1.0) if a == k else (fp[a] + 0.5) for a in range(d)]
        xs.append(sum(coef[a] * cx[a] for a in range(d)) + 1.0)
        ok = np.ones(fp[0].shape, dtype=bool)
        for a in range(d):
            if k == d:
                continue          # piecewise-constant pressure: checked separately
            if a == k:
                ok &= (fx[a] >= 2.0) & (fx[a] <= n[a] - 2.0)
            else:
                ok &= (fx[a] >= 1.0) & (fx[a] <= n[a] - 1.0)
        fine_pos.append(sum(coef[a] * fx[a] for a in range(d)) + 1.0)
        fine_ok.append(ok)
    y = P @ np.concatenate(xs)
    off = disc.offsets(n)
    for k in range(d):
        seg = y[off[k]:off[k + 1]]
        assert np.max(np.abs(seg[fine_ok[k]] - fine_pos[k][fine_ok[k]])) < 1e-13
    # pressure: each fine cell takes the value of its coarse parent
    pc = np.arange(int(np.prod(nc)), dtype=float)
    Pp = P[off[d]:, disc.offsets(nc)[d]:]
    fp = _positions(n)
    parent = np.zeros(fp[0].shape, dtype=np.int64)
    stride = 1
    for a in range(d):
        parent += (fp[a] // 2) * stride
        stride *= nc[a]
    assert np.array_equal(Pp @ pc, parent.astype(float))


def test_prolongation_interior_rows_sum_to_one():
    n = (16, 16)
    P = mg.prolongation(n)
    rs = np.asarray(P.sum(axis=1)).reshape(-1)
    off = disc.offsets(n)
    u0 = rs[off[0]:off[1]].reshape(16, 15)
    assert np.allclose(u0[1:-1, 1:-1], 1.0)
    assert np.allclose(rs[off[2]:], 1.0)


@pytest.mark.parametrize("n", [(16, 16), (8, 8, 8)])
def test_galerkin_footprint_and_symmetry(n):
    """Coarse Galerkin operators (eq. (9)) stay complex symmetric; the u_k-u_k stencil
    spans 3 normal x 5 tangential points, u_k-p 2 x 3 cells, p-p is diagonal and
    distinct displacement components never couple directly."""
    d = len(n)
    lam, mu, rho, gam = _hetero(n, 1)
    A = disc.assemble(n, 1.0, 0.7, lam, mu, rho, gam, 0.5)
    H = mg.Hierarchy(A, n, 3, [0.75, 0.5])
    for l in (1, 2):
        Ac = H.A[l]
        nl = H.n[l]
        assert abs(Ac - Ac.T).max() < 1e-13 * abs(Ac).max()
        off = disc.offsets(nl)
        C = sp.coo_matrix(Ac)
        blk = np.searchsorted(off, C.row, side="right") - 1
        bcol = np.searchsorted(off, C.col, side="right") - 1
        nz = np.abs(C.data) > 1e-14 * abs(Ac).max()
        for k in range(d):
            sel = nz & (blk == k)
            assert not np.any((bcol[sel] != k) & (bcol[sel] != d))
        assert not np.any(nz & (blk == d) & (bcol == d) & (C.row != C.col))
        # footprint of one interior u_0 face
        mid = tuple(v // 2 for v in nl)
        r = disc.unknown_index(nl, 0, mid)
        row = Ac[r].tocoo()
        for c, v in zip(row.col, row.data):
            if abs(v) < 1e-14 * abs(Ac).max():
                continue
            kb = np.searchsorted(off, c, side="right") - 1
            local = c - off[kb]
            dims = disc.face_dims(nl, kb) if kb < d else nl
            pos = []
            for a in range(d):
                pos.append(local % dims[a])
                local //= dims[a]
            if kb == 0:
                dn = (pos[0] + 1) - mid[0]
                assert abs(dn) <= 1
                assert all(abs(pos[a] - mid[a]) <= 2 for a in range(1, d))
            else:
                assert kb == d
                assert pos[0] - mid[0] in (-1, 0)
                assert all(abs(pos[a] - mid[a]) <= 1 for a in range(1, d))


def test_economic_block_is_the_matrix_B_of_section5():
    """For an interior cell of a homogeneous grid the economic local matrix is B of
    section 5.2: s00 on the u diagonal, +-1/h couplings to p, -1/(lam+mu) on p."""
    n = (8, 8)
    h, lam, mu, rho, omega, gam = 1.0, 7.0, 1.2, 0.8, 0.9, 0.35
    shape = tuple(reversed(n))
    A = disc.assemble(n, h, omega, np.full(shape, lam), np.full(shape, mu), np.full(shape, rho),
                      np.full(shape, gam))
    B, dofs, colour = mg.vanka_blocks(A, n, economic=True)
    s00 = 4 * mu / h ** 2 - rho * omega ** 2 * (1 - 1j * gam)
    sp_, sm = 1 / h, -1 / h          # s_{1/2} and s_{-1/2}
    paper_B = np.array([
        [s00, 0, 0, 0, sp_],
        [0, s00, 0, 0, sm],
        [0, 0, s00, 0, sp_],
        [0, 0, 0, s00, sm],
        [-sm, -sp_, -sm, -sp_, -1 / (lam + mu)]], dtype=complex)
    cell = 3 * 8 + 4
    assert np.max(np.abs(B[cell] - paper_B)) < 1e-12
    Bf, _, _ = mg.vanka_blocks(A, n, economic=False)
    assert abs(Bf[cell][0, 1] + mu / h ** 2) < 1e-12 and abs(Bf[cell][2, 3] + mu / h ** 2) < 1e-12


def test_red_black_cells_share_no_unknown():
    for n in [(8, 6), (4, 6, 4)]:
        dofs, colour = mg.cell_dofs(n)
        for c in (0, 1):
            d = dofs[colour == c]
            d = d[d >= 0]
            assert len(np.unique(d)) == d.size


@pytest.mark.parametrize("economic", [False, True])
def test_vanka_fixed_point(economic):
    n = (12, 10)
    lam, mu, rho, gam = _hetero(n, 2)
    A = disc.assemble(n, 1.0, 0.8, lam, mu, rho, gam, 0.5)
    rng = np.random.default_rng(0)
    e = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    b = A @ e
    B, dofs, colour = mg.vanka_blocks(A, n, economic)
    for c in (0, 1):
        e2 = mg.vanka_half_sweep(A, B, dofs, colour, c, b, e, 0.75)
        assert np.max(np.abs(e2 - e)) < 1e-12 * np.max(np.abs(e))


def test_full_vanka_solves_isolated_blocks_exactly():
    """Undamped full Vanka on a red cell makes that cell's residual vanish."""
    n = (8, 8)
    lam, mu, rho, gam = _hetero(n, 3)
    A = disc.assemble(n, 1.0, 0.8, lam, mu, rho, gam, 0.5)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    B, dofs, colour = mg.vanka_blocks(A, n, False)
    e = mg.vanka_half_sweep(A, B, dofs, colour, 0, b, np.zeros(A.shape[0], complex), 1.0)
    r = b - A @ e
    cell = 2 * 8 + 2          # red interior cell; its block sees only its own update
    d = dofs[cell]
    # residual of the cell's unknowns w.r.t. the block only (neighbours' updates excluded)
    own = np.zeros(A.shape[0], complex)
    own[d[d >= 0]] = e[d[d >= 0]]
    rb = b[d] - (A @ own)[d]
    assert np.max(np.abs(rb)) < 1e-12 * np.max(np.abs(b))


def test_one_level_cycle_is_exact_solve():
    n = (8, 8)
    lam, mu, rho, gam = _hetero(n, 5)
    A = disc.assemble(n, 1.0, 0.8, lam, mu, rho, gam, 0.5)
    H = mg.Hierarchy(A, n, 1, [])
    rng = np.random.default_rng(6)
    b = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    x = H.cycle(b)
    assert np.linalg.norm(A @ x - b) < 1e-12 * np.linalg.norm(b)


def test_two_level_without_smoothing_is_coarse_correction():
    n = (16, 16)
    lam, mu, rho, gam = _hetero(n, 6)
    A = disc.assemble(n, 1.0, 0.8, lam, mu, rho, gam, 0.5)
    H = mg.Hierarchy(A, n, 2, [0.75], nu1=0, nu2=0)
    rng = np.random.default_rng(7)
    b = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    P = H.P[0]
    Ac = (P.T @ A @ P).toarray()
    expect = P @ np.linalg.solve(Ac, P.T @ b)
    assert np.linalg.norm(H.cycle(b) - expect) < 1e-11 * np.linalg.norm(expect)


@pytest.mark.parametrize("cycle", [1, 2])
def test_cycle_is_linear(cycle):
    n = (16, 16)
    lam, mu, rho, gam = _hetero(n, 8)
    A = disc.assemble(n, 1.0, 0.8, lam, mu, rho, gam, 0.5)
    H = mg.Hierarchy(A, n, 3, [0.75, 0.5], cycle=cycle)
    rng = np.random.default_rng(9)
    b1 = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    b2 = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    a = 0.3 - 1.7j
    lhs = H.cycle(b1 + a * b2)
    rhs = H.cycle(b1) + a * H.cycle(b2)
    assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(rhs)


def test_fgmres_minimal_residual_property():
    """With a fixed linear preconditioner M, the k-th FGMRES iterate minimises
    |b - A x| over x in M K_k(A M, b); checked against an explicit dense least squares."""
    rng = np.random.default_rng(11)
    N = 30
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) + 6 * np.eye(N)
    Mi = np.diag(1.0 / np.diag(A))
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    for k in (1, 3, 6):
        _, st = krylov.fgmres(lambda v: A @ v, lambda v: Mi @ v, b, tol=1e-300, restart=k, maxit=k)
        AM = A @ Mi
        K = np.stack([np.linalg.matrix_power(AM, i) @ b for i in range(k)], axis=1)
        c, *_ = np.linalg.lstsq(AM @ K, b, rcond=None)
        best = np.linalg.norm(b - AM @ K @ c) / np.linalg.norm(b)
        assert abs(st["rel_res_true"] - best) < 1e-10


def test_fgmres_finite_termination_and_exact_preconditioner():
    rng = np.random.default_rng(12)
    N = 12
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) + 3 * np.eye(N)
    b = rng.standard_normal(N) + 0j
    x, st = krylov.fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-13, restart=N, maxit=N)
    assert st["iters"] <= N and st["rel_res_true"] < 1e-11
    Ainv = np.linalg.inv(A)
    x, st = krylov.fgmres(lambda v: A @ v, lambda v: Ainv @ v, b, tol=1e-12, restart=5, maxit=5)
    assert st["iters"] == 1 and st["rel_res_true"] < 1e-12


def test_mg_preconditioned_fgmres_reaches_true_residual():
    n = (32, 32)
    lam, mu, rho, gam = _hetero(n, 13, abl=6)
    pbA = disc.assemble(n, 1.0, 0.5, lam, mu, rho, gam, 0.0)
    As = disc.assemble(n, 1.0, 0.5, lam, mu, rho, gam, 0.5)
    H = mg.Hierarchy(As, n, 3, [0.75, 0.5])
    b = disc.point_source_vector(n, [(0, (16, 4), 1.0)])
    x, st = krylov.fgmres(lambda v: pbA @ v, H.cycle, b, tol=1e-8, restart=5, maxit=200)
    assert st["converged"] and st["rel_res_true"] <= 1e-8
    xd = spla.spsolve(pbA.tocsc(), b)
    assert np.linalg.norm(x - xd) < 1e-5 * np.linalg.norm(xd)


# ------------------------------------------------------------------------------ DD
def _dd_problem(n, seed=14):
    lam, mu, rho, gam = _hetero(n, seed, abl=4)
    pb = disc.Problem.__new__(disc.Problem)
    pb.n = tuple(n); pb.dim = len(n); pb.shift = 0.5; pb.omega = 0.6
    pb.lam, pb.mu, pb.rho, pb.gamma_hat = lam, mu, rho, gam
    return pb


@pytest.mark.parametrize("nu", [1, 2])
def test_single_subdomain_dd_equals_multigrid(nu):
    """One subdomain without padding: the DD preconditioner is the multigrid cycle
    itself, with the same number of smoothing steps (Algorithm 1 inside the
    subdomain solve); two steps give a different cycle than one."""
    n = (16, 16)
    pb = _dd_problem(n)
    P = ddm.DDPreconditioner(pb, (1, 1), 0, 0, 3, [0.75, 0.5], nu1=nu, nu2=nu)
    H = mg.Hierarchy(pb.matrix(shifted=True), n, 3, [0.75, 0.5], nu1=nu, nu2=nu)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(pb.size) + 1j * rng.standard_normal(pb.size)
    ref = H.cycle(v)
    assert np.linalg.norm(P.apply(v) - ref) < 1e-13 * np.linalg.norm(ref)
    if nu > 1:
        H1 = mg.Hierarchy(pb.matrix(shifted=True), n, 3, [0.75, 0.5])
        assert np.linalg.norm(H1.cycle(v) - ref) > 1e-3 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,parts", [((32, 16), (2, 2)), ((16, 16, 16), (2, 2, 2))])
def test_dd_overlap_weights_partition_unity(n, parts):
    subs = ddm.make_subdomains(n, parts, 4, 2)
    cnt = np.zeros(disc.n_unknowns(n))
    for s in subs:
        m = ddm.local_to_global(n, s)
        cnt[m[m >= 0]] += 1
        assert len(np.unique(m[m >= 0])) == np.count_nonzero(m >= 0)
    assert cnt.min() >= 1
    assert cnt.max() == 2 ** len(n)


def test_dd_local_operator_restricts_global_operator():
    """Away from the padding, the local shifted matrix equals the global one on the
    unknowns of the extent (the medium is copied, the layer only lives in the padding)."""
    n = (24, 16)
    pb = _dd_problem(n, 15)
    P = ddm.DDPreconditioner(pb, (2, 1), 4, 2, 2, [0.75])
    Ag = pb.matrix(shifted=True)
    sub, m = P.subs[0], P.maps[0]
    Al = P.hier[0].A[0]
    inside = np.nonzero(m >= 0)[0]
    # rows of local unknowns at least 2 cells away from the subdomain's interior side
    X = _positions(disc.face_dims(sub.nloc, 0))
    keep = []
    off = disc.offsets(sub.nloc)
    for li in inside:
        k = np.searchsorted(off, li, side="right") - 1
        dims = disc.face_dims(sub.nloc, k) if k < 2 else sub.nloc
        local = li - off[k]
        x = local % dims[0]
        if x + sub.origin[0] <= sub.hi[0] - 3:
            keep.append(li)
    keep = np.array(keep)
    sub_l = Al[keep][:, inside].toarray()
    sub_g = Ag[m[keep]][:, m[inside]].toarray()
    assert np.max(np.abs(sub_l - sub_g)) < 1e-14 * np.max(np.abs(sub_g))


@pytest.mark.parametrize("colours", [1, 4])
def test_dd_mg_fgmres_converges(colours):
    n = (32, 32)
    pb = _dd_problem(n, 16)
    P = ddm.DDPreconditioner(pb, (2, 2), 4, 4, 2, [0.75], colours=colours)
    A = pb.matrix()
    b = disc.point_source_vector(n, [(0, (10, 5), 1.0), (1, (20, 20), 0.5j)])
    x, st = krylov.fgmres(lambda v: A @ v, P.apply, b, tol=1e-8, restart=5, maxit=300)
    assert st["converged"] and st["rel_res_true"] <= 1e-8


# ------------------------------------------------- W-cycle and Algorithm 2 schedule pins
def _dense(M):
    return M.toarray() if sp.issparse(M) else np.asarray(M)


def _smoother_propagation(H, l):
    """Error propagation of one red-black Vanka step on level l (red, then
    black): S_c = I - w sum_K E_K B_K^{-1} E_K^T A over the cells K of colour c,
    B_K the cell's local matrix (section 3)."""
    B, dofs, colour = H.blocks[l]
    A = _dense(H.A[l])
    n = A.shape[0]
    S = np.eye(n, dtype=complex)
    for c in (0, 1):
        Wc = np.zeros((n, n), complex)
        for K in np.nonzero(colour == c)[0]:
            d = dofs[K]
            ok = d >= 0
            Bi = np.linalg.inv(B[K])[np.ix_(ok, ok)]
            Wc[np.ix_(d[ok], d[ok])] += H.damping[l] * Bi
        S = (np.eye(n) - Wc @ A) @ S
    return S


@pytest.mark.parametrize("levels,cycle_level", [(3, 0), (4, 1)])
def test_w_cycle_second_call_continues_from_the_first(levels, cycle_level):
    """Algorithm 1 with gamma recursive calls (section 2.2), written as the
    textbook error propagation: E_l = S^nu2 (I - P_l X_{l+1} P_l^T A_l) S^nu1 with
    X_{l+1} = (I - E_{l+1}^gamma) A_{l+1}^{-1} (gamma calls, each continuing from
    the previous one's result) and X_L = A_L^{-1}; one cycle from zero is
    (I - E_0) A_0^{-1}.  A second call that restarts from zero gives
    X = (I - E) A^{-1} instead and fails.  (Without smoothing both readings
    agree: the Galerkin coarse correction is a projection.)"""
    n = (32, 16) if levels == 4 else (16, 16)
    lam, mu, rho, gam = _hetero(n, 30)
    A = disc.assemble(n, 1.0, 0.8, lam, mu, rho, gam, 0.5)
    H = mg.Hierarchy(A, n, levels, [0.75, 0.5, 0.5], cycle=2, nu1=1, nu2=1, cycle_level=cycle_level)
    Ad = [_dense(a) for a in H.A]
    Pd = [_dense(p) for p in H.P]
    L = levels - 1

    def propagation(restart_second_call):
        X = np.linalg.inv(Ad[L])
        E = None
        for l in range(L - 1, -1, -1):
            I = np.eye(Ad[l].shape[0])
            S = _smoother_propagation(H, l)
            E = S @ (I - Pd[l] @ X @ Pd[l].T @ Ad[l]) @ S
            if l > 0:
                g = 2 if (l - 1 >= cycle_level and l < L) else 1
                Eg = E if (g == 1 or restart_second_call) else E @ E
                X = (I - Eg) @ np.linalg.inv(Ad[l])
        return E

    rng = np.random.default_rng(31)
    r = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    x = np.linalg.solve(Ad[0], r)
    want = x - propagation(False) @ x
    got = H.cycle(r)
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)
    wrong = x - propagation(True) @ x
    assert np.linalg.norm(got - wrong) > 1e-4 * np.linalg.norm(want)


def _alg2_rows_solved(P, pb, v):
    """Largest |v - A z| / |v| over the rows where Algorithm 2 with exact local
    solves must leave no residual: after the last colour c, for every subdomain
    of colour c, the rows of its extent whose global row couples only to unknowns
    of the extent and equals the local operator's row.  Returns (max residual,
    rows checked, rows of the subdomains)."""
    A = pb.matrix()
    z = P.apply(v)
    res = v - A @ z
    last = max(s.colour for s in P.subs)
    worst, count, total = 0.0, 0, 0
    for i, sub in enumerate(P.subs):
        if sub.colour != last:
            continue
        m = P.maps[i]
        inside = np.nonzero(m >= 0)[0]
        total += inside.size
        gset = np.zeros(A.shape[0], bool)
        gset[m[inside]] = True
        Al = sp.csr_matrix(P.hier[i].A[0])
        for li in inside:
            row = A.getrow(m[li]).tocoo()
            if np.any(~gset[row.col] & (np.abs(row.data) > 0)):
                continue
            # the local row, mapped to global columns
            lrow = Al.getrow(li).tocoo()
            if np.any(m[lrow.col] < 0) and np.any(np.abs(lrow.data[m[lrow.col] < 0]) > 0):
                continue
            a = np.zeros(A.shape[0], complex)
            a[row.col] = row.data
            b = np.zeros(A.shape[0], complex)
            ok = m[lrow.col] >= 0
            b[m[lrow.col[ok]]] = lrow.data[ok]
            if np.max(np.abs(a - b)) > 0:
                continue
            worst = max(worst, abs(res[m[li]]))
            count += 1
    return worst / np.linalg.norm(v), count, total


class _AdditiveColours(ddm.DDPreconditioner):
    """Planted mistake: every colour starts from v itself (no residual update
    between colours)."""

    def apply(self, v):
        v = np.asarray(v, dtype=np.complex128)
        z = np.zeros_like(v)
        for i in range(len(self.subs)):
            e = self.hier[i].cycle(self.restrict(i, v))
            m = self.maps[i]
            ok = m >= 0
            np.add.at(z, m[ok], e[ok])
        return z


@pytest.mark.parametrize("n,parts", [((24, 12), (2, 1)), ((24, 24), (2, 2))])
def test_algorithm2_colours_start_from_the_updated_residual(n, parts):
    """Algorithm 2 (section 2.3) with exact local solves (one level), no padding
    and no shift: each colour's local solve makes the global residual vanish on
    the rows of its subdomains that only couple inside the extent, so after the
    last colour those rows carry no residual.  The additive variant (all colours
    from the same residual) leaves residual on the overlap rows and fails."""
    pb = _dd_problem(n, 32)
    pb.shift = 0.0
    P = ddm.DDPreconditioner(pb, parts, 4, 0, 1, [], colours=2 ** len(n))
    rng = np.random.default_rng(33)
    v = rng.standard_normal(pb.size) + 1j * rng.standard_normal(pb.size)
    worst, count, total = _alg2_rows_solved(P, pb, v)
    assert count >= total // 2, (count, total)
    assert worst <= 1e-12
    bad = _AdditiveColours(pb, parts, 4, 0, 1, [], colours=2 ** len(n))
    worst_bad, _, _ = _alg2_rows_solved(bad, pb, v)
    assert worst_bad > 1e-3


def test_convergence_factor_of_a_geometric_history():
    """c_f = (r_k / r_w)^(1/(k - w)) (section 5.4): exactly rho for a residual
    history that decays by rho per iteration after an arbitrary warm-up."""
    rho = 0.83
    hist = [1.0, 3.0, 0.5, 2.0, 0.9] + [0.7 * rho ** k for k in range(40)]
    assert abs(krylov.convergence_factor(hist, warmup=5) - rho) < 1e-13
    assert np.isnan(krylov.convergence_factor([1.0, 0.5], warmup=5))


# ------------------------------------------------------ DD as the coarsest solver (MG-DD)
def _coarse_problem(n, seed):
    lam, mu, rho, gam = _hetero(n, seed)
    A = disc.assemble(n, 1.0, 0.8, lam, mu, rho, gam, 0.5)
    H = mg.Hierarchy(A, n, 3, [0.75, 0.5])
    return H.A[-1], H.n[-1]


def test_coarse_dd_with_one_subdomain_is_the_exact_solve():
    Ac, nc = _coarse_problem((32, 32), 40)
    cdd = mg.CoarseDD(Ac, nc, (1, 1), 2, 0)
    rng = np.random.default_rng(41)
    b = rng.standard_normal(Ac.shape[0]) + 1j * rng.standard_normal(Ac.shape[0])
    x = spla.spsolve(sp.csc_matrix(Ac), b)
    assert np.linalg.norm(cdd.solve(b) - x) <= 1e-12 * np.linalg.norm(x)


class _AdditiveCoarse(mg.CoarseDD):
    """Planted mistake: every colour from the same residual."""

    def solve(self, b, z=None):
        z = np.zeros_like(b, dtype=complex)
        r = b - self.A @ z
        for g, lu in zip(self.idx, self.lu):
            z[g] += lu.solve(r[g])
        return z


@pytest.mark.parametrize("n,parts", [((32, 32), (2, 2)), ((48, 16), (3, 1)), ((16, 16, 16), (2, 2, 1))])
def test_coarse_dd_colour_leaves_no_residual_on_its_rows(n, parts):
    """Algorithm 2 on the coarsest operator with restricted local operators and
    exact local solves: after the last colour, b - A_c z vanishes on every row of
    that colour's subdomains that couples only inside the extent (there the
    restricted local row is the global row); the additive variant leaves
    residual there."""
    Ac, nc = _coarse_problem(n, 42)
    cdd = mg.CoarseDD(Ac, nc, parts, 2, 0)
    rng = np.random.default_rng(43)
    b = rng.standard_normal(Ac.shape[0]) + 1j * rng.standard_normal(Ac.shape[0])

    def worst(solver):
        z = solver.solve(b)
        res = b - Ac @ z
        A = sp.csr_matrix(Ac)
        last = max(s_.colour for s_ in solver.subs)
        out, count = 0.0, 0
        for sub, g in zip(solver.subs, solver.idx):
            if sub.colour != last:
                continue
            inside = np.zeros(A.shape[0], bool)
            inside[g] = True
            for r in g:
                row = A.getrow(r)
                if np.all(inside[row.indices[np.abs(row.data) > 0]]):
                    out = max(out, abs(res[r]))
                    count += 1
        return out / np.linalg.norm(b), count

    w, count = worst(cdd)
    assert count > 0 and w <= 1e-12
    wb, _ = worst(_AdditiveCoarse(Ac, nc, parts, 2, 0))
    assert wb > 1e-4


def test_coarse_dd_one_colour_averages_the_corrections():
    """One colour: z = sum_i W E_i A_i^{-1} E_i^T b with W the inverse owner
    count, written out densely; its weights sum to one on every unknown."""
    Ac, nc = _coarse_problem((32, 32), 44)
    cdd = mg.CoarseDD(Ac, nc, (2, 2), 2, 1)
    rng = np.random.default_rng(45)
    b = rng.standard_normal(Ac.shape[0]) + 1j * rng.standard_normal(Ac.shape[0])
    Ad = Ac.toarray()
    want = np.zeros_like(b)
    cnt = np.zeros(Ac.shape[0])
    for g in cdd.idx:
        cnt[g] += 1
    for g in cdd.idx:
        want[g] += np.linalg.solve(Ad[np.ix_(g, g)], b[g]) / cnt[g]
    assert np.linalg.norm(cdd.solve(b) - want) <= 1e-12 * np.linalg.norm(want)
    assert cnt.max() == 4 and cnt.min() == 1


def test_mg_dd_w_cycle_continues_the_coarse_solve():
    """With an inexact coarsest solve the W-cycle's second call into the
    coarsest level continues from the first call's result: z + DD(b - A_c z)."""
    Ac, nc = _coarse_problem((32, 32), 46)
    cdd = mg.CoarseDD(Ac, nc, (2, 2), 2, 0)
    rng = np.random.default_rng(47)
    b = rng.standard_normal(Ac.shape[0]) + 1j * rng.standard_normal(Ac.shape[0])
    z1 = cdd.solve(b)
    z2 = cdd.solve(b, z1)
    assert np.linalg.norm(z2 - (z1 + cdd.solve(b - Ac @ z1))) <= 1e-12 * np.linalg.norm(z2)
    x = spla.spsolve(sp.csc_matrix(Ac), b)
    assert np.linalg.norm(z2 - x) < np.linalg.norm(z1 - x)


def test_mg_dd_preconditioned_fgmres_converges_like_mg_exact():
    """MG-DD (section 4, Table 5): FGMRES with 3-level cycles whose coarsest
    level is solved by 2 x 2 overlapping subdomains converges to 1e-8, within a
    few iterations of the exact coarsest solve."""
    n = (64, 64)
    lam, mu, rho, gam = _hetero(n, 48, abl=8)
    A = disc.assemble(n, 1.0, 0.6, lam, mu, rho, gam, 0.0)
    As = disc.assemble(n, 1.0, 0.6, lam, mu, rho, gam, 0.5)
    b = disc.point_source_vector(n, [(0, (32, 6), 1.0)])
    its = {}
    for key, cdd in (("exact", None), ("dd", ((2, 2), 2, 0))):
        H = mg.Hierarchy(As, n, 3, [0.75, 0.5], cycle=2, coarse_dd=cdd)
        x, st = krylov.fgmres(lambda v: A @ v, H.cycle, b, tol=1e-8, restart=5, maxit=300)
        assert st["converged"] and st["rel_res_true"] <= 1e-8
        its[key] = st["iters"]
    assert its["dd"] <= 1.5 * its["exact"] + 5, its


@pytest.mark.parametrize("economic", [False, True])
def test_component_damping_leaves_the_undamped_fraction_of_each_block_row(economic):
    """Damped block update with W = diag(w_u, .., w_u, w_p) (section 5.2): for a
    cell K of the colour whose unknowns couple to no other cell of that colour,
    solving its block again after the half-sweep gives (I - W) times the block
    solution before it, i.e. the fraction 1 - w_u of the displacement rows and
    1 - w_p of the pressure row remains."""
    n = (10, 8)
    lam, mu, rho, gam = _hetero(n, 50)
    A = disc.assemble(n, 1.0, 0.8, lam, mu, rho, gam, 0.5)
    B, dofs, colour = mg.vanka_blocks(A, n, economic)
    rng = np.random.default_rng(51)
    b = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    e0 = np.zeros(A.shape[0], complex)
    wu, wp = 0.85, 0.65
    e1 = mg.vanka_half_sweep(A, B, dofs, colour, 0, b, e0, wu, wp)
    r0, r1 = b - A @ e0, b - A @ e1
    cell = 3 * n[0] + 5          # interior red cell
    assert colour[cell] == 0
    d = dofs[cell]
    before = np.linalg.solve(B[cell], r0[d])
    after = np.linalg.solve(B[cell], r1[d])
    # the residual on K's rows also changed through the neighbours' updates: take
    # the block's own part only (the neighbours of a red cell are black)
    own = np.zeros(A.shape[0], complex)
    own[d] = e1[d]
    after_own = np.linalg.solve(B[cell], (b - A @ own)[d])
    W = np.array([wu] * 4 + [wp])
    if not economic:
        assert np.max(np.abs(after_own - (1 - W) * before)) <= 1e-12 * np.max(np.abs(before))
    else:   # the economic block is not the cell's full matrix: only the diagonal scaling is exact
        assert np.max(np.abs(e1[d] - W * before)) <= 1e-12 * np.max(np.abs(before))
    assert np.linalg.norm(after) > 0
