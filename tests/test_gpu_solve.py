"""End-to-end parity of precondition / solve (single and batched right-hand sides,
FP64 and complex64 cycles, domain decomposition) with the oracle, plus the
error paths of the C ABI."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from _helpers import (say, workload, small_hetero, oracle_problem, oracle_hierarchy, oracle_dd,
                      rand_cvec, to_dev, from_dev, rel_err, rhs_matrix)
from oracle import krylov

pytestmark = pytest.mark.gpu


def _solver(w, **over):
    import torch
    from paper_1806_11277_amd import ehh
    torch.cuda.synchronize()
    return ehh.solver_for_workload(w, **over)


@pytest.mark.parametrize("name,bits", [("c1_homog64", 64), ("c1_homog64", 32),
                                       ("c2s_hetero128_fp64", 64)])
def test_solve_matches_direct_solution(name, bits):
    """At tol 1e-10 the FGMRES solution equals the sparse direct solution to 1e-6
    and the iteration count equals the oracle's FGMRES count within 2."""
    import torch
    w = workload(name, precond_bits=bits)
    say(f"[solve {name} bits={bits}]")
    pb = oracle_problem(w)
    A = pb.matrix()
    B = rhs_matrix(w)
    xd = spla.splu(A.tocsc()).solve(B[0])
    S = _solver(w)
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-10, maxit=600)
    torch.cuda.synchronize()
    got = from_dev(x)[0]
    assert st == 0, stats
    assert stats[0]["rel_res_true"] <= 1e-10
    assert np.linalg.norm(got - xd) <= 1e-6 * np.linalg.norm(xd)
    H = oracle_hierarchy(w, pb)
    _, ost = krylov.fgmres(lambda v: A @ v, H.cycle, B[0], tol=1e-10, restart=w.restart, maxit=600)
    say(f"  gpu iters {stats[0]['iters']} oracle iters {ost['iters']}")
    assert abs(stats[0]["iters"] - ost["iters"]) <= 2
    S.close()


def test_batched_fp32_solve_per_source():
    """c3 layout at parity size: 8 sources, complex64 cycle, FP64 Krylov; each
    source reaches its tolerance and matches the direct solution."""
    import torch
    w = workload("c3s_hetero128_batch8_fp32")
    say("[batched fp32 solve]")
    pb = oracle_problem(w)
    lu = spla.splu(pb.matrix().tocsc())
    B = rhs_matrix(w)
    S = _solver(w)
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-10, maxit=800)
    torch.cuda.synchronize()
    assert st == 0, stats
    got = from_dev(x)
    for r in range(B.shape[0]):
        xd = lu.solve(B[r])
        assert stats[r]["rel_res_true"] <= 1e-10
        assert np.linalg.norm(got[r] - xd) <= 1e-6 * np.linalg.norm(xd)
    S.close()


@pytest.mark.parametrize("bits,colors", [(64, 1), (32, 1), (64, 0)])
def test_dd_precondition_matches_oracle(bits, colors):
    import torch
    w = workload("c4s_layered32_dd8_batch4_fp32", precond_bits=bits, dd_colors=colors)
    say(f"[dd precondition bits={bits} colors={colors}]")
    pb = oracle_problem(w)
    P = oracle_dd(w, pb)
    S = _solver(w)
    assert S.num_subdomains() == len(P.subs)
    for i, sub in enumerate(P.subs):
        info = S.subdomain_info(i)
        assert tuple(info["n"][:3]) == tuple(sub.nloc)
        assert tuple(info["lo"][:3]) == tuple(sub.lo) and tuple(info["hi"][:3]) == tuple(sub.hi)
    v = rand_cvec(pb.size, 2, 60)
    z = torch.zeros_like(to_dev(v))
    S.precondition(to_dev(v), z)
    torch.cuda.synchronize()
    got = from_dev(z)
    tol = 1e-11 if bits == 64 else 2e-5
    for r in range(2):
        ref = P.apply(v[r])
        assert np.linalg.norm(got[r] - ref) <= tol * np.linalg.norm(ref)
    S.close()


def test_dd_solve_3d():
    import torch
    w = workload("c4s_layered32_dd8_batch4_fp32")
    say("[dd solve 3d]")
    pb = oracle_problem(w)
    A = pb.matrix()
    B = rhs_matrix(w)
    S = _solver(w)
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-8, maxit=600)
    torch.cuda.synchronize()
    assert st == 0, stats
    got = from_dev(x)
    for r in range(B.shape[0]):
        res = np.linalg.norm(B[r] - A @ got[r]) / np.linalg.norm(B[r])
        assert res <= 1.01e-8
    S.close()


def test_invalid_arguments_are_rejected():
    import torch
    from paper_1806_11277_amd import ehh
    w = workload("c1_homog64")
    say("[invalid arguments]")
    with pytest.raises(ehh.EHHError) as ei:
        ehh.solver_for_workload(w, levels=9)
    assert ei.value.status == ehh.EHH_ERR_INVALID
    with pytest.raises(ehh.EHHError) as ei:
        ehh.solver_for_workload(w, levels=7)          # 64 not divisible into 7 levels
    assert ei.value.status == ehh.EHH_ERR_INVALID
    m = w.media()
    bad = np.array(m["rho"], copy=True)
    bad[3, 4] = np.nan
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    with pytest.raises(ehh.EHHError) as ei:
        ehh.Solver(2, w.n, w.h, w.omega, w.shift, w.abl_cells, t(m["lam"]), t(m["mu"]), t(bad))
    assert ei.value.status == ehh.EHH_ERR_BREAKDOWN
    S = _solver(w)
    B = rhs_matrix(w)
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-10, maxit=3)
    assert st == ehh.EHH_NOT_CONVERGED and stats[0]["iters"] == 3
    assert stats[0]["rel_res_true"] > 1e-10
    S.close()


def test_graph_replay_matches_eager_launches():
    """The captured Arnoldi-step graphs, replayed many times with host work in
    between, give bit-identical iterates to eager launches."""
    import os
    import torch
    w = workload("c3s_hetero128_batch8_fp32")
    say("[graph vs eager]")
    B = rhs_matrix(w)
    S = _solver(w)
    xs = []
    for mode in ("0", "1", "1"):
        os.environ["EHH_GRAPHS"] = mode
        x = torch.zeros_like(to_dev(B))
        st, stats = S.solve(to_dev(B), x, tol=1e-8, maxit=400)
        torch.cuda.synchronize()
        assert st == 0
        xs.append(x.cpu().numpy())
    os.environ.pop("EHH_GRAPHS", None)
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[1], xs[2])
    S.close()


@pytest.mark.parametrize("colors", [0, 1])
def test_dd_2d_several_subdomains_per_colour(colors):
    """4 x 2 subdomains: with the multicolour schedule two subdomains share each
    colour and must both start from the residual before that colour's corrections."""
    import torch
    w = small_hetero((64, 32), "dd2d", levels=2, damping=(0.75,), dd_parts=(4, 2, 1),
                     dd_overlap=4, dd_pad=4, dd_colors=colors, precond_bits=64)
    say(f"[dd 2d 4x2 colors={colors}]")
    pb = oracle_problem(w)
    P = oracle_dd(w, pb)
    S = _solver(w)
    v = rand_cvec(pb.size, 2, 61)
    z = torch.zeros_like(to_dev(v))
    S.precondition(to_dev(v), z)
    torch.cuda.synchronize()
    got = from_dev(z)
    for r in range(2):
        ref = P.apply(v[r])
        assert np.linalg.norm(got[r] - ref) <= 1e-11 * np.linalg.norm(ref)
    S.close()


def test_cached_device_buffers_give_identical_solves():
    """Buffers released by a closed solver are reused by the next one (the
    library's device memory cache): solving again with a new solver on reused
    buffers, and after the cache was handed back to the driver, gives the same
    bits and the direct solution."""
    import torch
    from paper_1806_11277_amd import ehh
    w = workload("c2s_hetero128_fp64")
    say("[cached buffers]")
    pb = oracle_problem(w)
    B = rhs_matrix(w)
    xd = spla.splu(pb.matrix().tocsc()).solve(B[0])
    got = []
    for k in range(3):
        if k == 2:
            ehh.release_cached_memory()
        S = _solver(w)
        x = torch.zeros_like(to_dev(B))
        st, stats = S.solve(to_dev(B), x, tol=1e-8, maxit=600)
        torch.cuda.synchronize()
        assert st == 0, stats
        got.append(from_dev(x)[0])
        S.close()
    assert np.array_equal(got[0], got[1]) and np.array_equal(got[0], got[2])
    assert np.linalg.norm(got[0] - xd) <= 1e-6 * np.linalg.norm(xd)


def test_fp16_coarse_rows_3d():
    """coarse_bits = 16 (section 3: half-precision storage of coarse data): the
    3D Galerkin level's stored rows in FP16 change the DD preconditioner by no
    more than twice the FP16 unit roundoff of its coefficients (2 * 2^-11
    relative; measured on MI355X: 8.8e-5 against 1.1e-7 with FP32 rows), the
    FGMRES solve still reaches the true residual tolerance, and in no more than
    10 % more iterations than with FP32 rows.  Asking for it with the FP64 cycle
    is an invalid argument."""
    import torch
    from paper_1806_11277_amd import ehh
    w = workload("c4s_layered32_dd8_batch4_fp32")
    say("[fp16 coarse rows 3d]")
    pb = oracle_problem(w)
    P = oracle_dd(w, pb)
    A = pb.matrix()
    B = rhs_matrix(w)
    v = rand_cvec(pb.size, 2, 61)
    out, iters = {}, {}
    for cb in (32, 16):
        S = _solver(w, coarse_bits=cb)
        z = torch.zeros_like(to_dev(v))
        S.precondition(to_dev(v), z)
        torch.cuda.synchronize()
        out[cb] = from_dev(z)
        x = torch.zeros_like(to_dev(B))
        st, stats = S.solve(to_dev(B), x, tol=1e-8, maxit=600)
        torch.cuda.synchronize()
        assert st == 0, stats
        got = from_dev(x)
        for r in range(B.shape[0]):
            assert np.linalg.norm(B[r] - A @ got[r]) / np.linalg.norm(B[r]) <= 1.01e-8
        iters[cb] = max(s_["iters"] for s_ in stats)
        S.close()
    for r in range(2):
        ref = P.apply(v[r])
        e16 = np.linalg.norm(out[16][r] - ref) / np.linalg.norm(ref)
        e32 = np.linalg.norm(out[32][r] - ref) / np.linalg.norm(ref)
        say(f"  source {r}: preconditioner error vs oracle fp32 rows {e32:.2e}, fp16 rows {e16:.2e}")
        assert e32 <= 2e-5
        assert 0 < e16 <= 2 * 2.0 ** -11
    say(f"  iterations fp32 rows {iters[32]}, fp16 rows {iters[16]}")
    assert iters[16] <= int(1.1 * iters[32]) + 1
    with pytest.raises(ehh.EHHError) as ei:
        _solver(w, precond_bits=64, coarse_bits=16)
    assert ei.value.status == ehh.EHH_ERR_INVALID
