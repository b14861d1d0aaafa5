"""ctypes binding of libehh.so (include/ehh.h), with the same names.

Argument marshalling only: torch tensors provide device memory and the current
HIP stream; every arithmetic step runs in the library's kernels.  The library
must be built (``python -m paper_1806_11277_amd.build``); nothing falls back to
another implementation when it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libehh.so")

EHH_OK, EHH_NOT_CONVERGED = 0, 1
EHH_ERR_INVALID, EHH_ERR_HIP, EHH_ERR_OOM, EHH_ERR_BREAKDOWN, EHH_ERR_UNSUPPORTED = -1, -2, -3, -4, -5
EHH_MAX_LEVELS = 8
EHH_MAX_RESTART = 16

STATUS_NAMES = {0: "EHH_OK", 1: "EHH_NOT_CONVERGED", -1: "EHH_ERR_INVALID", -2: "EHH_ERR_HIP",
                -3: "EHH_ERR_OOM", -4: "EHH_ERR_BREAKDOWN", -5: "EHH_ERR_UNSUPPORTED"}


class ehh_problem_t(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("h", ctypes.c_double),
                ("omega", ctypes.c_double), ("shift", ctypes.c_double),
                ("abl_cells", ctypes.c_int32 * 3), ("abl_max", ctypes.c_double),
                ("atten0", ctypes.c_double), ("mu_bar", ctypes.c_double), ("rho_bar", ctypes.c_double)]


class ehh_options_t(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("cycle", ctypes.c_int32), ("cycle_level", ctypes.c_int32),
                ("nu1", ctypes.c_int32),
                ("nu2", ctypes.c_int32), ("vanka", ctypes.c_int32), ("precond_bits", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("dd_parts", ctypes.c_int32 * 3),
                ("dd_overlap", ctypes.c_int32), ("dd_pad", ctypes.c_int32),
                ("dd_colors", ctypes.c_int32), ("damping", ctypes.c_double * EHH_MAX_LEVELS),
                ("coarse_bits", ctypes.c_int32), ("coarse_dd_parts", ctypes.c_int32 * 3),
                ("coarse_dd_overlap", ctypes.c_int32), ("coarse_dd_colors", ctypes.c_int32),
                ("dd_batch", ctypes.c_int32), ("damping_p", ctypes.c_double * EHH_MAX_LEVELS),
                ("reorth", ctypes.c_int32)]


class ehh_stats_t(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("rel_res_est", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("conv_factor", ctypes.c_double)]


class ehh_kernel_time_t(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 128), ("launches", ctypes.c_int32), ("avg_us", ctypes.c_double),
                ("avg_us_warm", ctypes.c_double), ("bytes", ctypes.c_double), ("bytes_model", ctypes.c_double),
                ("avg_us_seq", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_SIGS = {
    "ehh_default_options": (None, [ctypes.POINTER(ehh_options_t)]),
    "ehh_setup_operator": (_I, [ctypes.POINTER(ehh_problem_t), _P, _P, _P, _P,
                                ctypes.POINTER(ehh_options_t), _P, ctypes.POINTER(_P)]),
    "ehh_destroy": (None, [_P]),
    "ehh_release_cached_memory": (None, []),
    "ehh_vector_layout": (_I, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "ehh_scaling": (_I, [_P, ctypes.POINTER(ctypes.c_double)]),
    "ehh_apply": (_I, [_P, _I, _P, _P, _I, _P]),
    "ehh_vcycle": (_I, [_P, _I, _P, _P, _I, _P]),
    "ehh_precondition": (_I, [_P, _P, _P, _I, _P]),
    "ehh_solve": (_I, [_P, _P, _P, _I, ctypes.c_double, _I, ctypes.POINTER(ehh_stats_t), _P]),
    "ehh_solve_adjoint": (_I, [_P, _P, _P, _I, ctypes.c_double, _I, ctypes.POINTER(ehh_stats_t), _P]),
    "ehh_media_gradient": (_I, [_P, _P, _P, _I, _P, _P, _P, _I, _P]),
    "ehh_num_subdomains": (_I, [_P]),
    "ehh_subdomain_info": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                                ctypes.POINTER(_I)]),
    "ehh_level_info": (_I, [_P, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(ctypes.c_int64)]),
    "ehh_level_apply": (_I, [_P, _I, _I, _P, _P, _I, _P]),
    "ehh_level_relax": (_I, [_P, _I, _I, _I, _P, _P, _P, _I, _P]),
    "ehh_level_restrict": (_I, [_P, _I, _I, _P, _P, _P, _I, _P]),
    "ehh_level_prolong": (_I, [_P, _I, _I, _P, _P, _I, _P]),
    "ehh_coarse_solve": (_I, [_P, _I, _P, _P, _I, _P]),
    "ehh_coarse_solve_noalloc": (_I, [_P, _I, _P, _P, _I, _P]),
    "ehh_autotune": (_I, [_P, _I, ctypes.POINTER(_I), _I, _P]),
    "ehh_set_tuning": (_I, [_P, ctypes.POINTER(_I), _I]),
    "ehh_profile_precondition": (_I, [_P, _P, _P, _I, _I, _P, ctypes.c_int64, ctypes.POINTER(ehh_kernel_time_t),
                                      _I, ctypes.POINTER(_I), _P]),
    "ehh_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libehh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1806_11277_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class EHHError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status, allow=(EHH_OK,)):
    if status not in allow:
        raise EHHError(status, lib().ehh_last_error().decode(errors="replace"))
    return status


def default_options() -> ehh_options_t:
    o = ehh_options_t()
    lib().ehh_default_options(ctypes.byref(o))
    return o


def release_cached_memory():
    """Return the library's cached device buffers (kept after Solver.close for
    reuse by later solvers) to the driver."""
    lib().ehh_release_cached_memory()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("vectors must be contiguous device tensors")
    return ctypes.c_void_p(t.data_ptr())


def _media(a, ncell, name):
    """(keep-alive object, address) of a media array with exactly ncell float64
    entries: a float64 device tensor is passed in place (read on the device at
    setup), anything else (numpy, a CPU tensor) as a contiguous host copy that
    the library uploads."""
    import numpy as np
    try:
        import torch
        if isinstance(a, torch.Tensor):
            if a.is_cuda and a.dtype == torch.float64:
                t = a.detach().contiguous()
                if t.numel() != ncell:
                    raise ValueError(f"{name} has {t.numel()} entries, the grid has {ncell} cells")
                return t, t.data_ptr()
            a = a.detach().to("cpu", torch.float64).numpy()
    except ImportError:  # pragma: no cover
        pass
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if out.size != ncell:
        raise ValueError(f"{name} has {out.size} entries, the grid has {ncell} cells")
    return out, out.ctypes.data


def _overlap(a, b):
    a0, b0 = a.data_ptr(), b.data_ptr()
    return a0 < b0 + b.numel() * b.element_size() and b0 < a0 + a.numel() * a.element_size()


def _check_vectors(named, dtype, rows, cols, outputs=()):
    """Every (name, tensor) in named must be a contiguous device tensor of the
    given dtype and shape (rows, cols); a tensor named in `outputs` must not
    share memory with any other listed tensor.  Raises ValueError before
    anything reaches the library."""
    for name, t in named:
        if t is None:
            continue
        if not getattr(t, "is_cuda", False) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous device tensor")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != (rows, cols):
            raise ValueError(f"{name} must have shape ({rows}, {cols}), got {tuple(t.shape)}")
    for on, o in named:
        if on not in outputs or o is None:
            continue
        for n_, t in named:
            if n_ != on and t is not None and _overlap(o, t):
                raise ValueError(f"{on} must not overlap {n_}")


class Solver:
    """Owns one ehh handle.  Media: float64 arrays shaped like the cell grid (x
    fastest): numpy or CPU tensors (host arrays, uploaded at setup) or float64
    device tensors (read in place).  Vectors: (nrhs, 2N) tensors on the device,
    float64 for the global vectors, the cycle precision for level vectors."""

    def __init__(self, dim: int, n: Sequence[int], h: float, omega: float, shift: float,
                 abl_cells: Sequence[int], lam, mu, rho, gamma=None, abl_max: float = 1.0,
                 atten0: float = 0.0, levels: int = 3, cycle: int = 1, cycle_level: int = 0,
                 nu1: int = 1, nu2: int = 1,
                 vanka: int = 1, precond_bits: int = 64, restart: int = 5,
                 dd_parts: Sequence[int] = (1, 1, 1), dd_overlap: int = 0, dd_pad: int = 0,
                 dd_colors: int = 1, damping: Optional[Sequence[float]] = None,
                 mu_bar: float = 0.0, rho_bar: float = 0.0, coarse_bits: int = 32,
                 coarse_dd_parts: Sequence[int] = (1, 1, 1), coarse_dd_overlap: int = 2, coarse_dd_colors: int = 0,
                 damping_p: Optional[Sequence[float]] = None, dd_batch: int = 1, reorth: int = 0, stream=None):
        import torch
        p = ehh_problem_t()
        p.dim = dim
        nn = list(n) + [1] * (3 - len(n))
        ab = list(abl_cells) + [0] * (3 - len(abl_cells))
        for a in range(3):
            p.n[a] = int(nn[a])
            p.abl_cells[a] = int(ab[a])
        p.h, p.omega, p.shift, p.abl_max, p.atten0 = float(h), float(omega), float(shift), float(abl_max), float(atten0)
        p.mu_bar, p.rho_bar = float(mu_bar), float(rho_bar)
        o = default_options()
        o.levels, o.cycle, o.cycle_level, o.nu1, o.nu2, o.vanka = levels, cycle, cycle_level, nu1, nu2, vanka
        o.precond_bits, o.restart, o.coarse_bits = precond_bits, restart, coarse_bits
        cp = list(coarse_dd_parts) + [1] * (3 - len(coarse_dd_parts))
        for a in range(3):
            o.coarse_dd_parts[a] = int(cp[a])
        o.coarse_dd_overlap, o.coarse_dd_colors = int(coarse_dd_overlap), int(coarse_dd_colors)
        o.dd_batch = int(dd_batch)
        o.reorth = int(reorth)
        dp = list(dd_parts) + [1] * (3 - len(dd_parts))
        for a in range(3):
            o.dd_parts[a] = int(dp[a])
        o.dd_overlap, o.dd_pad, o.dd_colors = dd_overlap, dd_pad, dd_colors
        if damping is not None:
            for l, w in enumerate(damping[:EHH_MAX_LEVELS]):
                o.damping[l] = float(w)
        if damping_p is not None:
            for l, w in enumerate(damping_p[:EHH_MAX_LEVELS]):
                o.damping_p[l] = float(w)
        self.problem, self.options = p, o
        self.levels = int(levels)
        self.dim = dim
        self.precond_bits = precond_bits
        ncell = 1
        for a in range(dim):
            ncell *= int(nn[a])
        names = ("lambda", "mu", "rho", "gamma")
        media = [_media(t, ncell, nm) for t, nm in zip((lam, mu, rho, gamma), names) if t is not None]
        hp = [ctypes.c_void_p(addr) for _, addr in media] + [None] * (4 - len(media))
        h_ = ctypes.c_void_p()
        _check(lib().ehh_setup_operator(ctypes.byref(p), hp[0], hp[1], hp[2], hp[3],
                                        ctypes.byref(o), _stream(stream), ctypes.byref(h_)))
        del media
        self.handle = h_
        counts = (ctypes.c_int64 * 4)()
        stride = ctypes.c_int64()
        _check(lib().ehh_vector_layout(self.handle, counts, ctypes.byref(stride)))
        self.counts = list(counts)
        self.N = sum(self.counts)
        self.stride = stride.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().ehh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- queries
    def scaling(self):
        out = (ctypes.c_double * 3)()
        _check(lib().ehh_scaling(self.handle, out))
        return dict(mu_bar=out[0], rho_bar=out[1], omega_nd=out[2])

    def num_subdomains(self):
        return lib().ehh_num_subdomains(self.handle)

    def subdomain_info(self, sub):
        n, o, lo, hi = ((_I * 3)() for _ in range(4))
        _check(lib().ehh_subdomain_info(self.handle, sub, n, o, lo, hi))
        return dict(n=list(n), origin=list(o), lo=list(lo), hi=list(hi))

    def level_info(self, sub, level):
        n = (_I * 3)()
        counts = (ctypes.c_int64 * 4)()
        stride = ctypes.c_int64()
        _check(lib().ehh_level_info(self.handle, sub, level, n, counts, ctypes.byref(stride)))
        return dict(n=list(n), counts=list(counts), N=sum(counts), stride=stride.value)

    # ------------------------------------------------------------- argument checks
    def _cycle_dtype(self):
        import torch
        return torch.float32 if self.precond_bits == 32 else torch.float64

    def _global(self, outputs=(), **vecs):
        """Validate global FP64 vectors (nrhs, 2N) with a common nrhs."""
        import torch
        first = next(t for t in vecs.values() if t is not None)
        if first.dim() != 2 or first.shape[0] < 1:
            raise ValueError("vectors must be 2-D tensors (nrhs, 2N) with nrhs >= 1")
        _check_vectors(list(vecs.items()), torch.float64, first.shape[0], self.stride, outputs)
        return first.shape[0]

    def _level(self, sub, level, outputs=(), **vecs):
        """Validate level vectors (nrhs, 2 N_level) in the cycle precision."""
        stride = self.level_info(sub, level)["stride"]
        first = next(t for t in vecs.values() if t is not None)
        if first.dim() != 2 or first.shape[0] < 1:
            raise ValueError("vectors must be 2-D tensors (nrhs, 2N) with nrhs >= 1")
        _check_vectors(list(vecs.items()), self._cycle_dtype(), first.shape[0], stride, outputs)
        return first.shape[0]

    # ------------------------------------------------------------- calls
    def apply(self, x, y, shifted=False, stream=None):
        nrhs = self._global(outputs=("y",), x=x, y=y)
        _check(lib().ehh_apply(self.handle, int(shifted), _ptr(x), _ptr(y), nrhs, _stream(stream)))

    def vcycle(self, r, e, sub=0, stream=None):
        nrhs = self._level(sub, 0, outputs=("e",), r=r, e=e)
        _check(lib().ehh_vcycle(self.handle, sub, _ptr(r), _ptr(e), nrhs, _stream(stream)))

    def precondition(self, v, z, stream=None):
        nrhs = self._global(outputs=("z",), v=v, z=z)
        _check(lib().ehh_precondition(self.handle, _ptr(v), _ptr(z), nrhs, _stream(stream)))

    def solve(self, b, x, tol=1e-6, maxit=500, stream=None, raise_on_fail=False):
        nrhs = self._global(outputs=("x",), b=b, x=x)
        stats = (ehh_stats_t * nrhs)()
        st = lib().ehh_solve(self.handle, _ptr(b), _ptr(x), nrhs, float(tol), int(maxit), stats,
                             _stream(stream))
        _check(st, allow=(EHH_OK,) if raise_on_fail else (EHH_OK, EHH_NOT_CONVERGED))
        return st, [dict(status=s.status, iters=s.iters, rel_res_est=s.rel_res_est,
                         rel_res_true=s.rel_res_true, conv_factor=s.conv_factor) for s in stats]

    def solve_adjoint(self, g, y, tol=1e-6, maxit=500, stream=None, raise_on_fail=False):
        nrhs = self._global(outputs=("y",), g=g, y=y)
        stats = (ehh_stats_t * nrhs)()
        st = lib().ehh_solve_adjoint(self.handle, _ptr(g), _ptr(y), nrhs, float(tol), int(maxit), stats,
                                     _stream(stream))
        _check(st, allow=(EHH_OK,) if raise_on_fail else (EHH_OK, EHH_NOT_CONVERGED))
        return st, [dict(status=s.status, iters=s.iters, rel_res_est=s.rel_res_est,
                         rel_res_true=s.rel_res_true, conv_factor=s.conv_factor) for s in stats]

    def autotune(self, nrhs, stream=None):
        """Launch shapes for nrhs sources chosen by timing (ehh_autotune): the
        table, 2 entries per level."""
        t = (_I * (2 * self.levels))()
        _check(lib().ehh_autotune(self.handle, int(nrhs), t, len(t), _stream(stream)))
        return list(t)

    def set_tuning(self, table):
        t = (_I * len(table))(*[int(v) for v in table])
        _check(lib().ehh_set_tuning(self.handle, t, len(t)))

    def profile_precondition(self, v, z, reps=5, evict=None, stream=None, cap=256):
        """Per-kernel timing of one preconditioner application (ehh_profile_precondition):
        a list of dicts (kernel, launches, avg_us, avg_us_warm, avg_us_seq, bytes, bytes_model) in order of
        first launch.  evict: a device tensor written before every replayed launch."""
        nrhs = self._global(outputs=("z",), v=v, z=z)
        if evict is not None and (not evict.is_cuda or not evict.is_contiguous()):
            raise ValueError("evict must be a contiguous device tensor")
        nbytes = 0 if evict is None else (evict.numel() * evict.element_size()) // 4 * 4
        out = (ehh_kernel_time_t * cap)()
        cnt = _I()
        _check(lib().ehh_profile_precondition(self.handle, _ptr(v), _ptr(z), nrhs, int(reps),
                                              _ptr(evict) if evict is not None else None, nbytes, out, cap,
                                              ctypes.byref(cnt), _stream(stream)))
        return [dict(kernel=o.kernel.decode(), launches=o.launches, avg_us=o.avg_us, avg_us_warm=o.avg_us_warm,
                     avg_us_seq=o.avg_us_seq,
                     bytes=o.bytes, bytes_model=o.bytes_model) for o in out[:cnt.value]]

    def media_gradient(self, y, x, grad_lambda, grad_mu, grad_rho, accumulate=False, stream=None):
        import torch
        nrhs = self._global(y=y, x=x)
        ncell = self.counts[3]
        for nm, t in (("grad_lambda", grad_lambda), ("grad_mu", grad_mu), ("grad_rho", grad_rho)):
            if not getattr(t, "is_cuda", False) or not t.is_contiguous() or t.dtype != torch.float64 \
                    or t.numel() != ncell:
                raise ValueError(f"{nm} must be a contiguous float64 device tensor of {ncell} cells")
        _check_vectors([("gl", grad_lambda.view(1, -1)), ("gm", grad_mu.view(1, -1)),
                        ("gr", grad_rho.view(1, -1))], torch.float64, 1, ncell, ("gl", "gm", "gr"))
        for g in (grad_lambda, grad_mu, grad_rho):
            for v in (y, x):
                if _overlap(g, v):
                    raise ValueError("gradient outputs must not overlap the fields")
        _check(lib().ehh_media_gradient(self.handle, _ptr(y), _ptr(x), nrhs, _ptr(grad_lambda),
                                        _ptr(grad_mu), _ptr(grad_rho), int(bool(accumulate)), _stream(stream)))

    def level_apply(self, sub, level, x, y, stream=None):
        nrhs = self._level(sub, level, outputs=("y",), x=x, y=y)
        _check(lib().ehh_level_apply(self.handle, sub, level, _ptr(x), _ptr(y), nrhs, _stream(stream)))

    def level_relax(self, sub, level, colour, b, e_in, e_out, stream=None):
        nrhs = self._level(sub, level, outputs=("e_out",), b=b, e_in=e_in, e_out=e_out)
        _check(lib().ehh_level_relax(self.handle, sub, level, colour, _ptr(b), _ptr(e_in), _ptr(e_out),
                                     nrhs, _stream(stream)))

    def level_restrict(self, sub, level, b, e, rc, stream=None):
        nrhs = self._level(sub, level, b=b, e=e)
        self._level(sub, level + 1, rc=rc) if level + 1 < self.levels else None
        if rc.shape[0] != nrhs:
            raise ValueError("rc must have as many right-hand sides as b")
        _check(lib().ehh_level_restrict(self.handle, sub, level, _ptr(b), _ptr(e), _ptr(rc), nrhs,
                                        _stream(stream)))

    def level_prolong(self, sub, level, ec, e, stream=None):
        nrhs = self._level(sub, level, e=e)
        self._level(sub, level + 1, ec=ec) if level + 1 < self.levels else None
        if ec.shape[0] != nrhs:
            raise ValueError("ec must have as many right-hand sides as e")
        _check(lib().ehh_level_prolong(self.handle, sub, level, _ptr(ec), _ptr(e), nrhs, _stream(stream)))

    def coarse_solve(self, sub, r, e, stream=None):
        nrhs = self._level(sub, self.levels - 1, outputs=("e",), r=r, e=e)
        _check(lib().ehh_coarse_solve(self.handle, sub, _ptr(r), _ptr(e), nrhs, _stream(stream)))

    def coarse_solve_noalloc(self, sub, r, e, stream=None):
        nrhs = self._level(sub, self.levels - 1, outputs=("e",), r=r, e=e)
        _check(lib().ehh_coarse_solve_noalloc(self.handle, sub, _ptr(r), _ptr(e), nrhs, _stream(stream)))


def solver_for_workload(w, **overrides):
    """Solver for a workloads.Workload (its host media are copied at setup)."""
    m = w.media()
    kw = dict(levels=w.levels, cycle=w.cycle, cycle_level=w.cycle_level, nu1=w.nu1, nu2=w.nu2, vanka=w.vanka,
              precond_bits=w.precond_bits, restart=w.restart, dd_parts=w.dd_parts,
              dd_overlap=w.dd_overlap, dd_pad=w.dd_pad, dd_colors=w.dd_colors, damping=w.damping,
              abl_max=w.abl_max, atten0=w.atten0, coarse_bits=getattr(w, "coarse_bits", 32),
              coarse_dd_parts=getattr(w, "coarse_dd_parts", (1, 1, 1)),
              coarse_dd_overlap=getattr(w, "coarse_dd_overlap", 2), coarse_dd_colors=getattr(w, "coarse_dd_colors", 0),
              damping_p=getattr(w, "damping_p", None))
    kw.update(overrides)
    return Solver(w.dim, w.n, w.h, w.omega, kw.pop("shift", w.shift), w.abl_cells,
                  m["lam"], m["mu"], m["rho"], **kw)
