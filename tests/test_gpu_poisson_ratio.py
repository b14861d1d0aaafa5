"""The mixed formulation with cell-wise Vanka is robust in the Poisson ratio
(section 6, first experiment, Fig. 5): with constant mu = rho = 1 the number of
preconditioning cycles stays nearly constant as lambda grows from 0.5 to 16
(Poisson ratio 0.17 to 0.47).  On 256x128 the GPU's iteration counts equal the
oracle's FGMRES with the same preconditioner within 2, for both Vanka
variants and for Table 2's component damping.  Against the paper's counts the
comparison is a loose band only (parity unpinned: the paper's discretisation
details are not stated); flatness is the property asserted on the larger
grids, including 1024x512 at 12 pi, whose coarsest level is solved by DD."""
import pytest

from _helpers import say, oracle_problem, oracle_hierarchy, rhs_matrix

pytestmark = pytest.mark.gpu

# Fig. 5 mixed-formulation counts (full / economic Vanka), per grid
PAPER = {256: {1: (41, 42), 0: (50, 57)}, 512: {1: (75, 80), 0: (104, 113)},
         1024: {1: (181, 202), 0: (266, 284)}}


def _iters(w):
    import torch
    import bench
    from paper_1806_11277_amd import ehh
    S = ehh.solver_for_workload(w)
    b = bench.rhs_tensor(S, w)
    x = torch.zeros_like(b)
    st, stats = S.solve(b, x, tol=1e-6, maxit=600)
    torch.cuda.synchronize()
    S.close()
    assert st == 0 and stats[0]["rel_res_true"] <= 1e-6
    return stats[0]["iters"]


def _oracle_iters(w):
    from oracle import krylov
    pb = oracle_problem(w)
    H = oracle_hierarchy(w, pb)
    A = pb.matrix()
    _, st = krylov.fgmres(lambda v: A @ v, H.cycle, rhs_matrix(w)[0], tol=1e-6, restart=w.restart, maxit=600)
    assert st["converged"]
    return st["iters"]


@pytest.mark.parametrize("vanka,damping,lam", [(1, "constant", 0.5), (1, "constant", 2.0), (1, "constant", 16.0),
                                               (0, "constant", 0.5), (0, "constant", 16.0),
                                               (1, "component", 16.0)])
def test_iterations_match_the_oracle_on_256x128(vanka, damping, lam):
    from workloads.configs import poisson_sweep
    w = poisson_sweep(256, lam, vanka, damping)
    g, o = _iters(w), _oracle_iters(w)
    say(f"[256x128 lambda={lam} {'full' if vanka else 'economic'} {damping}] gpu {g} oracle {o}")
    assert abs(g - o) <= 2


@pytest.mark.parametrize("nx,vanka,lams", [(256, 1, (0.5, 2.0, 16.0)), (256, 0, (0.5, 2.0, 16.0)),
                                          (512, 1, (0.5, 16.0)), (1024, 1, (0.5, 16.0))])
def test_iterations_do_not_grow_with_lambda(nx, vanka, lams):
    from workloads.configs import poisson_sweep
    its = [_iters(poisson_sweep(nx, lam, vanka)) for lam in lams]
    say(f"[poisson ratio {nx} {'full' if vanka else 'economic'} Vanka] lambda {lams}: iterations {its}")
    assert max(its) <= 1.25 * min(its)
    lo, hi = PAPER[nx][vanka]
    assert 0.5 * lo <= min(its) and max(its) <= 1.5 * hi


# Table 2, red-black Vanka, lambda = 16: constant / component damping
TABLE2 = {256: (42, 38), 512: (84, 75), 1024: (186, 169)}


@pytest.mark.parametrize("nx", [512, 1024])
def test_table2_rows_converge_in_the_papers_band(nx):
    """Table 2 (lambda = 16, red-black Vanka) with constant damping (0.75, 0.5)
    and with the component damping (0.85, 0.65) / (0.6, 0.4): both converge
    within the loose band of the paper's counts (the component damping's
    arithmetic is pinned against the oracle on 256x128; on this discretisation
    it does not reproduce the paper's saving)."""
    from workloads.configs import poisson_sweep
    c = _iters(poisson_sweep(nx, 16.0, 1, "constant"))
    k = _iters(poisson_sweep(nx, 16.0, 1, "component"))
    pc, pk = TABLE2[nx]
    say(f"[Table 2, {nx}x{nx // 2}, lambda 16] constant {c} (paper {pc}), component {k} (paper {pk})")
    assert 0.5 * pc <= c <= 1.5 * pc and 0.5 * pk <= k <= 1.5 * pk
