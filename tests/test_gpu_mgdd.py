"""DD as the coarsest-grid solver (MG-DD, section 4) and with top-level DD around
it (DD-MG-DD), through the C ABI, against the oracle: the coarsest solve by
itself, whole cycles (V and W, whose second call into the coarsest level
continues from the first), the DD-MG-DD preconditioner and solves against the
direct solution."""
import numpy as np
import pytest

from _helpers import (say, workload, small_hetero, oracle_problem, oracle_hierarchy, oracle_dd, rand_cvec, to_dev,
                      from_dev, component_errors, rhs_matrix)

pytestmark = pytest.mark.gpu


def _solver(w, **over):
    import torch
    from paper_1806_11277_amd import ehh
    torch.cuda.synchronize()
    return ehh.solver_for_workload(w, **over)


CASES = {
    "2d_2x2": dict(n=(64, 48), levels=3, coarse_dd_parts=(2, 2, 1)),
    "2d_3x1": dict(n=(96, 32), levels=3, coarse_dd_parts=(3, 1, 1)),
    "3d_2x2x1": dict(n=(32, 32, 16), levels=3, coarse_dd_parts=(2, 2, 1)),
}


def _case(name, bits, colors, cycle=2, cycle_level=0):
    c = CASES[name]
    damping = (0.75, 0.5) if len(c["n"]) == 2 else (0.5, 0.5)
    return small_hetero(c["n"], f"mgdd_{name}", levels=c["levels"], damping=damping, precond_bits=bits,
                        cycle=cycle, cycle_level=cycle_level, coarse_dd_parts=c["coarse_dd_parts"],
                        coarse_dd_overlap=2, coarse_dd_colors=colors)


@pytest.mark.parametrize("colors", [0, 1])
@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("name", sorted(CASES))
def test_coarse_dd_solve_matches_oracle(name, bits, colors):
    import torch
    w = _case(name, bits, colors)
    say(f"[coarse DD solve {name} bits={bits} colors={colors}]")
    H = oracle_hierarchy(w)
    S = _solver(w)
    L = w.levels - 1
    N = H.A[L].shape[0]
    assert S.level_info(0, L)["N"] == N
    dt = torch.float32 if bits == 32 else torch.float64
    r = rand_cvec(N, 3, 140)
    e = torch.zeros((3, 2 * N), dtype=dt, device="cuda")
    S.coarse_solve(0, to_dev(r, dt), e)
    torch.cuda.synchronize()
    got = from_dev(e)
    tol = 1e-11 if bits == 64 else 2e-6
    for q in range(3):
        ref = H.coarse_dd.solve(r[q])
        assert np.linalg.norm(got[q] - ref) <= tol * np.linalg.norm(ref), q
    S.close()


@pytest.mark.parametrize("cycle,cycle_level", [(1, 0), (2, 0), (2, 1)])
@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("name", ["2d_2x2", "3d_2x2x1"])
def test_mg_dd_cycle_matches_oracle(name, bits, cycle, cycle_level):
    import torch
    w = _case(name, bits, 0, cycle, cycle_level)
    say(f"[MG-DD cycle {name} bits={bits} cycle={cycle} level={cycle_level}]")
    H = oracle_hierarchy(w)
    S = _solver(w)
    N = H.A[0].shape[0]
    dt = torch.float32 if bits == 32 else torch.float64
    r = rand_cvec(N, 2, 141)
    e = torch.zeros((2, 2 * N), dtype=dt, device="cuda")
    S.vcycle(to_dev(r, dt), e)
    torch.cuda.synchronize()
    got = from_dev(e)
    tol = 1e-11 if bits == 64 else 2e-5
    for q in range(2):
        ref = H.cycle(r[q])
        assert np.linalg.norm(got[q] - ref) <= tol * np.linalg.norm(ref), q
        assert max(component_errors(w.n, got[q], ref)) <= (1e-10 if bits == 64 else 1e-4)
    S.close()


@pytest.mark.parametrize("bits,colors", [(64, 0), (32, 0), (64, 1)])
def test_dd_mg_dd_precondition_matches_oracle(bits, colors):
    """Top-level 2 x 2 x 2 DD (padding 4, Algorithm 2 or one colour) around
    3-level W-cycles on the 20^3 padded subdomains, whose 5^3 coarsest levels are
    solved by 2 x 2 x 1 DD (overlap 1)."""
    import torch
    w = small_hetero((32, 32, 32), "ddmgdd", levels=3, damping=(0.5, 0.5), precond_bits=bits, cycle=2,
                     dd_parts=(2, 2, 2), dd_overlap=4, dd_pad=2, dd_colors=colors, coarse_dd_parts=(2, 2, 1),
                     coarse_dd_overlap=1, coarse_dd_colors=0)
    say(f"[DD-MG-DD precondition bits={bits} colors={colors}]")
    pb = oracle_problem(w)
    P = oracle_dd(w, pb)
    assert P.hier[0].coarse_dd is not None
    S = _solver(w)
    v = rand_cvec(pb.size, 2, 142)
    z = torch.zeros_like(to_dev(v))
    S.precondition(to_dev(v), z)
    torch.cuda.synchronize()
    got = from_dev(z)
    tol = 1e-11 if bits == 64 else 2e-5
    for r in range(2):
        ref = P.apply(v[r])
        assert np.linalg.norm(got[r] - ref) <= tol * np.linalg.norm(ref), r
        assert max(component_errors(w.n, got[r], ref)) <= (1e-10 if bits == 64 else 1e-4)
    S.close()


@pytest.mark.parametrize("bits", [64, 32])
def test_mg_dd_solve_matches_direct_solution(bits):
    """MG-DD FGMRES at tol 1e-10 on 128^2 (4 levels, 16^2 coarsest split 2 x 2):
    within 1e-6 of the direct solution, iterations within 2 of the oracle's
    FGMRES with the same preconditioner (FP64 cycle)."""
    import torch
    from oracle import direct, krylov
    w = workload("c2s_hetero128_fp64", precond_bits=bits, cycle=2, coarse_dd_parts=(2, 2, 1), coarse_dd_overlap=2)
    say(f"[MG-DD solve 128^2 bits={bits}]")
    pb = oracle_problem(w)
    B = rhs_matrix(w)
    xd = direct.factorize(pb).solve(B[0])
    S = _solver(w)
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-10, maxit=800)
    torch.cuda.synchronize()
    S.close()
    assert st == 0, stats
    err = np.linalg.norm(from_dev(x)[0] - xd) / np.linalg.norm(xd)
    assert stats[0]["rel_res_true"] <= 1e-10 and err <= 1e-6
    if bits == 64:
        H = oracle_hierarchy(w, pb)
        A = pb.matrix()
        _, ost = krylov.fgmres(lambda v: A @ v, H.cycle, B[0], tol=1e-10, restart=w.restart, maxit=800)
        say(f"  gpu iters {stats[0]['iters']} oracle iters {ost['iters']} error {err:.2e}")
        assert abs(stats[0]["iters"] - ost["iters"]) <= 2


def test_noalloc_coarse_solve_rejects_a_dd_coarsest_level():
    import torch
    from paper_1806_11277_amd import ehh
    w = _case("2d_2x2", 64, 0)
    S = _solver(w)
    N = S.level_info(0, w.levels - 1)["N"]
    r = to_dev(rand_cvec(N, 1, 143))
    with pytest.raises(ehh.EHHError) as ei:
        S.coarse_solve_noalloc(0, r, torch.zeros_like(r))
    assert ei.value.status == ehh.EHH_ERR_UNSUPPORTED
    S.close()
