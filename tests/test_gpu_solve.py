"""End-to-end parity of precondition / solve (single and batched right-hand sides,
FP64 and complex64 cycles, domain decomposition) with the oracle, plus the
error paths of the C ABI."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from _helpers import (say, workload, small_hetero, oracle_problem, oracle_hierarchy, oracle_dd,
                      rand_cvec, to_dev, from_dev, rel_err, rhs_matrix, component_errors)
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


def test_exact_preconditioner_takes_the_second_gram_schmidt_pass():
    """With one level and no shift the preconditioner is the exact inverse of A,
    so A M^-1 v_0 = v_0 lies in the Krylov basis: the first Gram-Schmidt pass
    removes all of w and the step must reorthogonalise.  FGMRES then stops after
    one step per source with the direct solution (three sources at once)."""
    import torch
    w = workload("c1_homog64", levels=1, precond_bits=64, shift=0.0)
    say("[exact preconditioner, shift 0]")
    pb = oracle_problem(w)
    lu = spla.splu(pb.matrix().tocsc())
    B = rand_cvec(pb.size, 3, 47)
    S = _solver(w)
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-10, maxit=20)
    torch.cuda.synchronize()
    assert st == 0, stats
    got = from_dev(x)
    for r in range(B.shape[0]):
        xd = lu.solve(B[r])
        say(f"  source {r}: iters {stats[r]['iters']} rel_res {stats[r]['rel_res_true']:.2e}")
        assert stats[r]["iters"] <= 2
        assert stats[r]["rel_res_true"] <= 1e-10
        assert np.linalg.norm(got[r] - xd) <= 1e-9 * np.linalg.norm(xd)
    S.close()


@pytest.mark.parametrize("name", ["c2s_hetero128_fp64", "c3s_hetero128_batch8_fp32"])
def test_two_gram_schmidt_passes_give_the_same_solve(name):
    """With reorth = 1 every Arnoldi step takes the second Gram-Schmidt pass
    (its fused projection, the second update and the normalisation from the
    partial sums); with the default the steps of these workloads take one.  Both
    reach 1e-10 with the direct solution for every source, in the same number of
    iterations within 1, and (FP64 cycle) within 2 of the oracle's FGMRES."""
    import torch
    w = workload(name)
    say(f"[two Gram-Schmidt passes {name}]")
    pb = oracle_problem(w)
    A = pb.matrix()
    lu = spla.splu(A.tocsc())
    B = rhs_matrix(w)
    its = {}
    for reorth in (0, 1):
        S = _solver(w, reorth=reorth)
        x = torch.zeros_like(to_dev(B))
        st, stats = S.solve(to_dev(B), x, tol=1e-10, maxit=800)
        torch.cuda.synchronize()
        assert st == 0, stats
        got = from_dev(x)
        for r in range(B.shape[0]):
            xd = lu.solve(B[r])
            assert stats[r]["rel_res_true"] <= 1e-10
            assert np.linalg.norm(got[r] - xd) <= 1e-6 * np.linalg.norm(xd)
        its[reorth] = [st_["iters"] for st_ in stats]
        S.close()
    say(f"  iterations one pass {its[0]}, two passes {its[1]}")
    assert all(abs(a - b) <= 1 for a, b in zip(its[0], its[1]))
    if w.precond_bits == 64:
        H = oracle_hierarchy(w, pb)
        _, ost = krylov.fgmres(lambda v: A @ v, H.cycle, B[0], tol=1e-10, restart=w.restart, maxit=800)
        assert abs(its[1][0] - ost["iters"]) <= 2


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


@pytest.mark.parametrize("bits,colors,nu", [(64, 1, 1), (32, 1, 1), (64, 0, 1), (64, 0, 2), (32, 1, 2)])
def test_dd_precondition_matches_oracle(bits, colors, nu):
    """DD around the cycles (3D 2 x 2 x 2 subdomains, both schedules) against the
    oracle, including two pre- and post-smoothing steps per level inside every
    subdomain's cycle."""
    import torch
    w = workload("c4s_layered32_dd8_batch4_fp32", precond_bits=bits, dd_colors=colors, nu1=nu, nu2=nu)
    say(f"[dd precondition bits={bits} colors={colors} nu={nu}]")
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
        assert max(component_errors(w.n, got[r], ref)) <= (1e-10 if bits == 64 else 2e-4)
    S.close()


@pytest.fixture(scope="module")
def c4m_oracle():
    w = workload("c4m_layered32_dd8_batch16_fp32")
    say("[c4 configuration at 32^3: oracle DD preconditioner]")
    pb = oracle_problem(w)
    return w, pb, oracle_dd(w, pb)


def test_c4_configuration_precondition_matches_oracle(c4m_oracle):
    """The bench's c4 solver configuration at 32^3: complex64 cycle on 24^3 padded
    subdomains (padding 6, 4 levels: the 12^3 and 6^3 Galerkin levels run the
    stored-row half-sweep in two full groups of 8 sources), Algorithm 2 with its
    local residual gather, V(2,1), shift 0.6, all 16 sources compared with the FP64
    oracle, norm-wise and per component."""
    import torch
    w, pb, P = c4m_oracle
    say("[c4 configuration precondition, 16 sources]")
    S = _solver(w)
    assert S.num_subdomains() == 8 and S.subdomain_info(0)["n"] == [24, 24, 24]
    assert S.level_info(0, 1)["n"] == [12, 12, 12]
    v = rand_cvec(pb.size, 16, 62)
    z = torch.zeros_like(to_dev(v))
    S.precondition(to_dev(v), z)
    torch.cuda.synchronize()
    got = from_dev(z)
    worst = [0.0, 0.0]
    for r in range(16):
        ref = P.apply(v[r])
        e2 = np.linalg.norm(got[r] - ref) / np.linalg.norm(ref)
        ec = max(component_errors(w.n, got[r], ref))
        worst = [max(worst[0], e2), max(worst[1], ec)]
        assert e2 <= 2e-5 and ec <= 2e-4, (r, e2, ec)
    say(f"  worst norm-wise {worst[0]:.2e}, worst per component {worst[1]:.2e}")
    S.close()


def test_c4_configuration_solve_matches_direct_solution():
    """c4's solver settings (2 x 2 x 2 subdomains, padding 6, 4 levels, Algorithm 2,
    V(2,1), shift 0.6, complex64 cycle) on a 16^3 grid, whose direct factorisation takes
    seconds: 16 random right-hand sides solved to 1e-10, every solution within
    1e-6 of the oracle's direct solution."""
    import torch
    from oracle import direct
    c4 = workload("c4m_layered32_dd8_batch16_fp32")
    w = small_hetero((16, 16, 16), "c4cfg16", levels=4, damping=c4.damping, shift=c4.shift, nu1=c4.nu1,
                     nu2=c4.nu2, precond_bits=32, dd_parts=(2, 2, 2), dd_overlap=4, dd_pad=6, dd_colors=0,
                     abl_cells=(4, 4, 4))
    say("[c4 configuration at 16^3: solve vs direct, 16 sources]")
    pb = oracle_problem(w)
    lu = direct.factorize(pb)
    B = rand_cvec(pb.size, 16, 63)
    S = _solver(w)
    assert S.subdomain_info(0)["n"] == [16, 16, 16]
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-10, maxit=1500)
    torch.cuda.synchronize()
    assert st == 0, stats
    got = from_dev(x)
    worst = 0.0
    for r in range(16):
        xd = lu.solve(B[r])
        err = np.linalg.norm(got[r] - xd) / np.linalg.norm(xd)
        worst = max(worst, err)
        assert stats[r]["rel_res_true"] <= 1e-10
        assert err <= 1e-6, (r, err)
    say(f"  iterations {min(s_['iters'] for s_ in stats)}-{max(s_['iters'] for s_ in stats)}, "
        f"worst error vs direct {worst:.2e}")
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
    with pytest.raises(ehh.EHHError) as ei:
        ehh.solver_for_workload(w, reorth=2)
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


_OOM_SCRIPT = r'''
import os, sys
import numpy as np
import torch
sys.path[:0] = [sys.argv[1], os.path.join(sys.argv[1], "tests")]
from paper_1806_11277_amd import ehh
from _helpers import workload, rhs_matrix, to_dev, from_dev
w = workload("c2s_hetero128_fp64", levels=3, damping=(0.75, 0.5))
B1 = rhs_matrix(w)
B2 = np.concatenate([B1, 1j * B1])
def solve(S, B):
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-8, maxit=300)
    torch.cuda.synchronize()
    return st, from_dev(x)
S = ehh.solver_for_workload(w)
st, ref1 = solve(S, B1)
assert st == 0
S.close()
counts = {"setup": 0, "solve": 0}
for k in range(0, 400):
    os.environ["EHH_FAIL_ALLOC_AFTER"] = str(k)
    try:
        S = ehh.solver_for_workload(w)
    except ehh.EHHError as e:
        assert e.status == ehh.EHH_ERR_OOM, e
        counts["setup"] += 1
        continue
    try:
        st, _ = solve(S, B2)
        injected = False
    except ehh.EHHError as e:
        assert e.status == ehh.EHH_ERR_OOM, e
        injected = True
        counts["solve"] += 1
    # a smaller follow-up solve on the same handle allocates again and matches
    st, got = solve(S, B1)
    assert st == 0 and np.array_equal(got, ref1), (k, st)
    S.close()
    if not injected:
        break
os.environ.pop("EHH_FAIL_ALLOC_AFTER")
print("injected failures", counts, "last point", k, flush=True)
assert counts["setup"] > 5 and counts["solve"] > 5 and k < 399
'''


def test_injected_allocation_failures_leave_a_usable_library():
    """EHH_FAIL_ALLOC_AFTER=k fails the device allocation that follows k
    successful ones.  Swept over every allocation point of a setup and of a
    two-source solve (fresh process): each failure reports EHH_ERR_OOM, a failed
    setup returns no handle, and after a failed solve a one-source solve on the
    same handle allocates its workspaces again and gives the same bits as a
    solve that never failed."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    say("[injected allocation failures, fresh process]")
    env = dict(os.environ)
    env.pop("EHH_FAIL_ALLOC_AFTER", None)
    r = subprocess.run([sys.executable, "-c", _OOM_SCRIPT, root], env=env, capture_output=True, text=True,
                       timeout=110)
    say(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0


def test_host_and_device_media_build_the_same_operator():
    """Media handed over as host arrays (copied at setup) and as device arrays
    (read in place) give bit-identical solves."""
    import torch
    from paper_1806_11277_amd import ehh
    w = workload("c2s_hetero128_fp64")
    say("[host vs device media]")
    m = w.media()
    B = rhs_matrix(w)
    out = []
    for dev in (False, True):
        conv = (lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")) if dev else (lambda a: a)
        S = ehh.Solver(w.dim, w.n, w.h, w.omega, w.shift, w.abl_cells, conv(m["lam"]), conv(m["mu"]),
                       conv(m["rho"]), levels=w.levels, damping=w.damping, atten0=w.atten0)
        x = torch.zeros_like(to_dev(B))
        st, _ = S.solve(to_dev(B), x, tol=1e-8, maxit=400)
        torch.cuda.synchronize()
        assert st == 0
        out.append(x.cpu().numpy())
        S.close()
    assert np.array_equal(out[0], out[1])
