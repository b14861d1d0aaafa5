"""Kernel-by-kernel parity of the HIP path (through the C ABI) with the oracle."""
import numpy as np
import pytest

from _helpers import (say, workload, small_hetero, oracle_problem, oracle_hierarchy, rand_cvec,
                      to_dev, from_dev, rel_err)

pytestmark = pytest.mark.gpu

CASES = {
    "c1": lambda **o: workload("c1_homog64", **o),
    "het2d": lambda **o: small_hetero((48, 40), "het2d", **{"levels": 3, "damping": (0.75, 0.5), **o}),
    "het3d": lambda **o: small_hetero((12, 8, 16), "het3d", **{"levels": 3, "damping": (0.5, 0.5), **o}),
}


def _solver(w):
    import torch
    from paper_1806_11277_amd import ehh
    torch.cuda.synchronize()
    return ehh.solver_for_workload(w)


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    w = CASES[request.param](precond_bits=64)
    say(f"[case {request.param}] n={w.n} levels={w.levels}")
    pb = oracle_problem(w)
    H = oracle_hierarchy(w, pb)
    S = _solver(w)
    yield request.param, w, pb, H, S
    S.close()


def test_library_is_the_in_tree_build():
    from paper_1806_11277_amd import ehh
    L = ehh.lib()
    assert L._name.endswith("paper_1806_11277_amd/libehh.so")


@pytest.mark.parametrize("shifted", [False, True])
def test_apply(case, shifted):
    import torch
    name, w, pb, H, S = case
    say(f"[apply {name} shifted={shifted}]")
    A = pb.matrix(shifted=shifted)
    x = rand_cvec(A.shape[0], 2, 1)
    y = torch.zeros_like(to_dev(x))
    S.apply(to_dev(x), y, shifted=shifted)
    torch.cuda.synchronize()
    got = from_dev(y)
    for r in range(2):
        assert rel_err(got[r], A @ x[r]) < 1e-13


def test_level_operators_are_galerkin(case):
    import torch
    name, w, pb, H, S = case
    for l in range(w.levels):
        say(f"[level_apply {name} level={l}]")
        info = S.level_info(0, l)
        assert info["N"] == H.A[l].shape[0]
        x = rand_cvec(info["N"], 2, 10 + l)
        y = torch.zeros_like(to_dev(x))
        S.level_apply(0, l, to_dev(x), y)
        torch.cuda.synchronize()
        got = from_dev(y)
        for r in range(2):
            assert rel_err(got[r], H.A[l] @ x[r]) < 1e-12


@pytest.mark.parametrize("with_e", [False, True])
@pytest.mark.parametrize("colour", [0, 1])
def test_relax(case, colour, with_e):
    import torch
    name, w, pb, H, S = case
    for l in range(w.levels - 1):
        say(f"[relax {name} level={l} colour={colour} e_in={with_e}]")
        N = H.A[l].shape[0]
        b = rand_cvec(N, 2, 20 + l)
        e = rand_cvec(N, 2, 30 + l) if with_e else np.zeros((2, N), complex)
        out = torch.zeros_like(to_dev(b))
        S.level_relax(0, l, colour, to_dev(b), to_dev(e) if with_e else None, out)
        torch.cuda.synchronize()
        got = from_dev(out)
        for r in range(2):
            ref = H.relax(l, b[r], e[r], colour)
            assert rel_err(got[r], ref) < 1e-11


def test_restrict_prolong_coarse(case):
    import torch
    name, w, pb, H, S = case
    for l in range(w.levels - 1):
        say(f"[transfer {name} level={l}]")
        N, Nc = H.A[l].shape[0], H.A[l + 1].shape[0]
        b, e = rand_cvec(N, 2, 40), rand_cvec(N, 2, 41)
        rc = torch.zeros((2, 2 * Nc), dtype=torch.float64, device="cuda")
        S.level_restrict(0, l, to_dev(b), to_dev(e), rc)
        ec = rand_cvec(Nc, 2, 42)
        ef = to_dev(e)
        S.level_prolong(0, l, to_dev(ec), ef)
        torch.cuda.synchronize()
        for r in range(2):
            assert rel_err(from_dev(rc)[r], H.P[l].T @ (b[r] - H.A[l] @ e[r])) < 1e-12
            assert rel_err(from_dev(ef)[r], e[r] + H.P[l] @ ec[r]) < 1e-13
    say(f"[coarse {name}]")
    Nc = H.A[-1].shape[0]
    r_ = rand_cvec(Nc, 3, 43)
    out = torch.zeros((3, 2 * Nc), dtype=torch.float64, device="cuda")
    S.coarse_solve(0, to_dev(r_), out)
    torch.cuda.synchronize()
    for r in range(3):
        assert rel_err(from_dev(out)[r], H.coarse_lu.solve(r_[r])) < 1e-10


@pytest.mark.parametrize("bits,cycle,vanka,cycle_level", [(64, 1, 1, 0), (64, 2, 1, 0), (64, 1, 0, 0),
                                                          (32, 1, 1, 0), (64, 2, 1, 1)])
@pytest.mark.parametrize("name", sorted(CASES))
def test_vcycle(name, bits, cycle, vanka, cycle_level):
    import torch
    w = CASES[name](precond_bits=bits, cycle=cycle, vanka=vanka, cycle_level=cycle_level)
    if cycle_level and name != "het3d":     # four levels, so that level 1 makes two calls
        w = CASES[name](precond_bits=bits, cycle=cycle, vanka=vanka, cycle_level=cycle_level, levels=4,
                        damping=(0.75, 0.5, 0.5))
    say(f"[vcycle {name} bits={bits} cycle={cycle} vanka={vanka} cycle_level={cycle_level} levels={w.levels}]")
    H = oracle_hierarchy(w)
    S = _solver(w)
    N = H.A[0].shape[0]
    r = rand_cvec(N, 3, 50)
    dt = torch.float32 if bits == 32 else torch.float64
    e = torch.zeros((3, 2 * N), dtype=dt, device="cuda")
    S.vcycle(to_dev(r, dt), e)
    torch.cuda.synchronize()
    got = from_dev(e)
    tol = 1e-11 if bits == 64 else 2e-5
    for q in range(3):
        ref = H.cycle(r[q])
        assert np.linalg.norm(got[q] - ref) <= tol * np.linalg.norm(ref)
    S.close()


@pytest.mark.parametrize("nrhs", [1, 6, 12, 32])
@pytest.mark.parametrize("bits", [64, 32])
def test_coarse_solve_widths(bits, nrhs):
    """Coarsest solve of the 2D case (338 unknowns: five full 64-column panels of
    the blocked inverse and a ragged one) for every right-hand-side width of the
    coarse apply; FP64 inverse, vectors in the cycle precision."""
    import torch
    w = CASES["het2d"](precond_bits=bits)
    say(f"[coarse widths bits={bits} nrhs={nrhs}]")
    H = oracle_hierarchy(w)
    S = _solver(w)
    Nc = H.A[-1].shape[0]
    r_ = rand_cvec(Nc, nrhs, 44)
    dt = torch.float32 if bits == 32 else torch.float64
    out = torch.full((nrhs, 2 * Nc), float("nan"), dtype=dt, device="cuda")
    S.coarse_solve(0, to_dev(r_, dt), out)
    torch.cuda.synchronize()
    got = from_dev(out)
    tol = 1e-10 if bits == 64 else 1e-5
    rin = from_dev(to_dev(r_, dt))       # the inputs as rounded to the cycle precision
    for r in range(nrhs):
        ref = H.coarse_lu.solve(rin[r])
        assert np.linalg.norm(got[r] - ref) <= tol * np.linalg.norm(ref)
    S.close()


@pytest.mark.parametrize("nrhs", [1, 32])
def test_dense_inverse_of_the_whole_grid(nrhs):
    """One level: the cycle is the exact solve of the shifted operator, so the
    blocked inverse of the 12,160-unknown 64^2 system (190 panels) applied to
    random vectors must match the sparse LU of the oracle."""
    import torch
    import scipy.sparse.linalg as spla
    w = workload("c1_homog64", levels=1, precond_bits=64)
    say(f"[dense inverse 64^2 nrhs={nrhs}]")
    pb = oracle_problem(w)
    lu = spla.splu(pb.matrix(shifted=True).tocsc())
    S = _solver(w)
    r_ = rand_cvec(pb.size, nrhs, 45)
    e = torch.zeros((nrhs, 2 * pb.size), dtype=torch.float64, device="cuda")
    S.vcycle(to_dev(r_), e)
    torch.cuda.synchronize()
    got = from_dev(e)
    for r in range(nrhs):
        ref = lu.solve(r_[r])
        assert np.linalg.norm(got[r] - ref) <= 1e-10 * np.linalg.norm(ref)
    S.close()


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("name", ["het2d", "het3d"])
def test_relax_component_damping(name, bits):
    """Half-sweeps with the component damping (w_u, w_p) = (0.85, 0.65) on the
    finest level and (0.6, 0.4) below (section 5.2, Table 2), every level and
    colour from a nonzero e_in, against the oracle's damped block update."""
    import torch
    w = CASES[name](precond_bits=bits, damping=(0.85, 0.6), damping_p=(0.65, 0.4))
    say(f"[component damping {name} bits={bits}]")
    H = oracle_hierarchy(w)
    S = _solver(w)
    dt = torch.float32 if bits == 32 else torch.float64
    tol = 1e-11 if bits == 64 else 2e-5
    for l in range(w.levels - 1):
        N = H.A[l].shape[0]
        b = rand_cvec(N, 2, 150 + l)
        e = rand_cvec(N, 2, 160 + l)
        for colour in (0, 1):
            out = torch.zeros((2, 2 * N), dtype=dt, device="cuda")
            S.level_relax(0, l, colour, to_dev(b, dt), to_dev(e, dt), out)
            torch.cuda.synchronize()
            got = from_dev(out)
            for r in range(2):
                ref = H.relax(l, b[r], e[r], colour)
                assert rel_err(got[r], ref) < tol, (l, colour, r)
    S.close()
