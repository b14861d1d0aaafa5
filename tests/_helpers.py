"""Shared helpers of the GPU parity tests: building matching oracle/HIP problems
from one workload and moving complex vectors between the two layouts."""
import dataclasses
import sys

import numpy as np

from oracle import discretisation as disc
from oracle import multigrid as mg
from oracle import dd as ddm
from workloads import get_config, media as M


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def workload(name, **over):
    w = dataclasses.replace(get_config(name), **over) if over else get_config(name)
    if over:
        w._media_cache = None
    return w


def small_hetero(n, name, **over):
    """A c2-like heterogeneous workload on an arbitrary grid."""
    base = get_config("c2s_hetero128_fp64" if len(n) == 2 else "c4s_layered32_dd8_batch4_fp32")
    fn = (lambda: M.heterogeneous_2d_media(n, corr_vp=max(2.0, n[0] / 8), corr_nu=max(4.0, n[0] / 4))) \
        if len(n) == 2 else (lambda: M.layered_3d_media(n, n_layers=4, corr_pert=3.0, corr_nu=6.0))
    kw = dict(name=name, n=tuple(n), media_fn=fn, abl_cells=tuple(max(2, v // 6) for v in n),
              dd_parts=(1, 1, 1), dd_overlap=0, dd_pad=0)
    kw.update(over)
    w = dataclasses.replace(base, **kw)
    w._media_cache = None
    return w


def oracle_problem(w):
    m = w.media()
    return disc.Problem(w.n, w.h, w.omega, m["lam"], m["mu"], m["rho"], w.abl_cells, w.abl_max,
                        w.atten0, shift=w.shift)


def coarse_dd_of(w):
    """(parts, overlap, colours) of the workload's coarsest-level DD, or None."""
    parts = tuple(w.coarse_dd_parts[:w.dim])
    if all(v == 1 for v in parts):
        return None
    return parts, w.coarse_dd_overlap, w.coarse_dd_colors


def oracle_hierarchy(w, pb=None):
    pb = pb or oracle_problem(w)
    return mg.build_hierarchy(pb, w.levels, list(w.damping), economic=(w.vanka == 0), cycle=w.cycle,
                              nu1=w.nu1, nu2=w.nu2, cycle_level=w.cycle_level, coarse_dd=coarse_dd_of(w),
                              damping_p=(list(w.damping_p) if w.damping_p is not None else None))


def oracle_dd(w, pb=None):
    pb = pb or oracle_problem(w)
    return ddm.DDPreconditioner(pb, w.dd_parts[:w.dim], w.dd_overlap, w.dd_pad, w.levels,
                                list(w.damping), economic=(w.vanka == 0), cycle=w.cycle,
                                colours=(1 if w.dd_colors == 1 else 2 ** w.dim), abl_max=w.abl_max,
                                coarse_dd=coarse_dd_of(w), cycle_level=w.cycle_level,
                                damping_p=(list(w.damping_p) if w.damping_p is not None else None),
                                nu1=w.nu1, nu2=w.nu2)


def rand_cvec(N, nrhs, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, N)) + 1j * rng.standard_normal((nrhs, N))


def to_dev(x, dtype=None):
    import torch
    x = np.atleast_2d(x)
    out = np.concatenate([x.real, x.imag], axis=1)
    return torch.as_tensor(out, dtype=dtype or torch.float64, device="cuda").contiguous()


def from_dev(t):
    a = t.detach().double().cpu().numpy()
    N = a.shape[1] // 2
    return a[:, :N] + 1j * a[:, N:]


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rhs_matrix(w):
    n = w.n
    return np.stack([disc.point_source_vector(n, [s]) for s in w.sources()])


def component_errors(n, got, ref):
    """max |got - ref| / max |ref| within each component block u_0, u_1, (u_2), p
    of a vector of grid n (an error confined to one block, or to the small
    entries of the absorbing layer, is not hidden by the others)."""
    off = disc.offsets(n)
    out = []
    for k in range(len(off) - 1):
        a, b = got[off[k]:off[k + 1]], ref[off[k]:off[k + 1]]
        out.append(float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)))
    return out
