"""Launch-shape autotuner (ehh_autotune / ehh_set_tuning): the number of source
groups per launch only moves sources between grid rows, so the preconditioner
gives the same bits for the heuristic shapes, extreme tables (every source in
its own group, all sources in one) and the tuned table, on the 2D levels of
both precisions, on the 3D cell kernels of the DD workload and with the
FP16-stored 3D Galerkin rows; a tuned solve takes the same iterations."""
import numpy as np
import pytest

from _helpers import say, workload, small_hetero, rand_cvec, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "c3s_fp32": lambda: workload("c3s_hetero128_batch8_fp32"),
    "c2s_fp64": lambda: workload("c2s_hetero128_fp64"),
    "2d_fp32_w": lambda: small_hetero((96, 64), "tw", levels=4, cycle=2, cycle_level=1,
                                      damping=(0.75, 0.5, 0.5), precond_bits=32),
    "c4m_alg2": lambda: workload("c4m_layered32_dd8_batch16_fp32"),
    "3d_fp16rows": lambda: small_hetero((32, 32, 32), "t16", levels=3, damping=(0.5, 0.5),
                                        precond_bits=32, coarse_bits=16),
}


def _z(S, v):
    import torch
    z = torch.zeros_like(v)
    S.precondition(v, z)
    torch.cuda.synchronize()
    return z.cpu().numpy()


@pytest.mark.parametrize("name", sorted(CASES))
def test_tuning_tables_do_not_change_the_bits(name):
    from paper_1806_11277_amd import ehh
    w = CASES[name]()
    nrhs = 16 if w.dim == 3 and name.startswith("c4m") else 8
    say(f"[tuning {name}] nrhs {nrhs}")
    S = ehh.solver_for_workload(w)
    v = to_dev(rand_cvec(S.stride // 2, nrhs, 77))
    z0 = _z(S, v)
    L = S.levels
    for table in ([1] * (2 * L), [nrhs] * (2 * L), [2, 4] * L, [3, 1] * L):
        S.set_tuning(table)
        z = _z(S, v)
        assert np.array_equal(z, z0), f"table {table}"
    t = S.autotune(nrhs)
    say(f"  tuned table {t}")
    assert len(t) == 2 * L and all(x in (0, 1, 2, 4, 8, 16, 32, 64) for x in t)
    assert t[2 * (L - 1)] == 0      # the coarsest level is not relaxed
    assert np.array_equal(_z(S, v), z0)
    S.set_tuning([0] * (2 * L))
    assert np.array_equal(_z(S, v), z0)
    S.close()


def test_tuned_solve_takes_the_same_iterations(tmp_path):
    import torch
    from paper_1806_11277_amd import ehh, tuning
    w = workload("c3s_hetero128_batch8_fp32")
    S = ehh.solver_for_workload(w)
    b = to_dev(rand_cvec(S.stride // 2, 8, 5))
    x0 = torch.zeros_like(b)
    _, st0 = S.solve(b, x0, tol=1e-8, maxit=200)
    path = str(tmp_path / "tune.json")
    t1, how1 = tuning.tune(S, 8, path=path)
    t2, how2 = tuning.tune(S, 8, path=path)
    say(f"  {how1} {t1}; {how2} {t2}")
    assert (how1, how2) == ("tuned", "cache") and t1 == t2
    x1 = torch.zeros_like(b)
    _, st1 = S.solve(b, x1, tol=1e-8, maxit=200)
    assert [s["iters"] for s in st1] == [s["iters"] for s in st0]
    assert torch.equal(x0, x1)
    S.close()
