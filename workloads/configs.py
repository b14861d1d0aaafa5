"""Named workload configurations.

Each configuration fixes a grid, a seeded medium, a frequency rule, the
absorbing layer, the point sources and the solver settings.  Sources are listed
as (component, position, amplitude): component k in 0..dim-1 is the displacement
u_{k+1} on faces normal to axis k, and position is given in face/cell
coordinates (x, y[, z]) where the normal coordinate is the face index
1..n_k-1 (face i sits between cells i-1 and i).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Tuple

import numpy as np

from . import media as M

Source = Tuple[int, Tuple[int, ...], complex]


@dataclasses.dataclass
class Workload:
    name: str
    description: str
    dim: int
    n: Tuple[int, ...]
    h: float
    media_fn: Callable[[], dict]
    ppw: float                      # cells per minimum shear wavelength
    abl_cells: Tuple[int, ...]
    abl_max: float = 1.0
    atten0: float = 0.01 * math.pi  # constant attenuation gamma_0 [1/s]
    shift: float = 0.5
    levels: int = 3
    cycle: int = 1                  # 1 = V, 2 = W
    cycle_level: int = 0            # levels >= this use `cycle` calls, finer ones one call
    nu1: int = 1
    nu2: int = 1
    vanka: int = 1                  # 1 = full, 0 = economic
    damping: Tuple[float, ...] = (0.75, 0.5, 0.25)
    precond_bits: int = 64
    restart: int = 5
    tol: float = 1e-6
    maxit: int = 400
    dd_parts: Tuple[int, ...] = (1, 1, 1)
    dd_overlap: int = 0
    dd_pad: int = 0
    dd_colors: int = 1
    coarse_bits: int = 32           # 16: FP16 stored rows on 3D Galerkin levels (complex64 cycle)
    coarse_dd_parts: Tuple[int, ...] = (1, 1, 1)   # subdomains of the coarsest level (MG-DD); 1s: exact
    coarse_dd_overlap: int = 2
    coarse_dd_colors: int = 0       # 0: Algorithm 2 over the coarsest level's subdomains, 1: one colour
    damping_p: Tuple[float, ...] = None   # pressure-row damping per level (component damping); None: = damping
    sources_fn: Callable[["Workload"], List[Source]] = None
    receivers_fn: Callable[["Workload"], List[Tuple[int, Tuple[int, ...]]]] = None
    true_media_fn: Callable[[], dict] = None

    _media_cache: dict = dataclasses.field(default=None, repr=False)

    def media(self) -> dict:
        if self._media_cache is None:
            self._media_cache = self.media_fn()
        return self._media_cache

    @property
    def omega(self) -> float:
        vs_min = float(self.media()["vs"].min())
        return M.shear_frequency(vs_min, self.h, self.ppw)

    def sources(self) -> List[Source]:
        return self.sources_fn(self)

    @property
    def nrhs(self) -> int:
        return len(self.sources())


def _src_centre(w: Workload) -> List[Source]:
    return [(0, tuple(v // 2 for v in w.n), 1.0 + 0j)]


def _src_top_single(w: Workload) -> List[Source]:
    # x-force on the u1 face in the middle of the top, 5 cells deep
    if w.dim == 2:
        return [(0, (w.n[0] // 2, 5), 1.0 + 0j)]
    return [(0, (w.n[0] // 2, w.n[1] // 2, 5), 1.0 + 0j)]


def _src_line(count: int, spacing: int, first: int, depth: int, seed: int):
    def fn(w: Workload) -> List[Source]:
        rng = np.random.default_rng(seed)
        phases = rng.uniform(0.0, 2.0 * np.pi, size=count)
        out = []
        for s in range(count):
            i = first + spacing * s
            out.append((0, (i, depth), complex(np.exp(1j * phases[s]))))
        return out
    return fn


def _src_lattice(per_axis: int, spacing: int, first: int, depth: int, seed: int):
    def fn(w: Workload) -> List[Source]:
        rng = np.random.default_rng(seed)
        phases = rng.uniform(0.0, 2.0 * np.pi, size=per_axis * per_axis)
        out = []
        for b in range(per_axis):
            for a in range(per_axis):
                s = b * per_axis + a
                out.append((0, (first + spacing * a, first + spacing * b, depth),
                            complex(np.exp(1j * phases[s]))))
        return out
    return fn


def _scaled_line(count: int, depth: int, seed: int):
    """count x-forces equally spaced along x at the given depth."""
    def fn(w: Workload) -> List[Source]:
        spacing = w.n[0] // count
        return _src_line(count, spacing, spacing // 2, depth, seed)(w)
    return fn


CONFIGS = {}


def _add(w: Workload):
    CONFIGS[w.name] = w


_add(Workload(
    name="c1_homog64",
    description="2D 64x64 homogeneous (Vp 2000, Vs 2000/sqrt3, rho 1000), h=10 m, "
                "10 cells per shear wavelength, 10-cell absorbing layer, unit x-force at the centre",
    dim=2, n=(64, 64), h=10.0, media_fn=lambda: M.homogeneous_media((64, 64)), ppw=10.0,
    abl_cells=(10, 10), shift=0.5, levels=3, damping=(0.75, 0.5), tol=1e-8,
    sources_fn=_src_centre))

_add(Workload(
    name="c2_hetero512_fp64",
    description="2D 512x512 heterogeneous (Vp GRF 1500-4500, Poisson 0.25-0.45, Gardner rho), "
                "h=10 m, 10 cells per minimum shear wavelength, shift 0.5, 20-cell layer, one source, "
                "FP64 FGMRES(5) + FP64 (1,1) cycle on 5 levels: V on the finest level, W below, exact "
                "solve of the 32^2 level",
    dim=2, n=(512, 512), h=10.0, media_fn=lambda: M.heterogeneous_2d_media((512, 512)), ppw=10.0,
    abl_cells=(20, 20), shift=0.5, levels=5, cycle=2, cycle_level=1, damping=(0.75, 0.5, 0.5, 0.5),
    precond_bits=64, sources_fn=_src_top_single))

_add(Workload(
    name="c3_hetero512_batch32_fp32",
    description="as c2, 32 x-forces at depth 5 (x = 8 + 16 s, seeded phases), complex64 cycle "
                "inside FP64 FGMRES with FP64 coarsest solve",
    dim=2, n=(512, 512), h=10.0, media_fn=lambda: M.heterogeneous_2d_media((512, 512)), ppw=10.0,
    abl_cells=(20, 20), shift=0.5, levels=5, cycle=2, cycle_level=1, damping=(0.75, 0.5, 0.5, 0.5),
    precond_bits=32, sources_fn=_src_line(32, 16, 8, 5, seed=3)))

_add(Workload(
    name="c4_layered128_dd8_batch16_fp32",
    description="3D 128^3 layered (8 layers, Vp 1500-4500, 5% perturbation, Poisson 0.30-0.45), "
                "h=10 m, 8 cells per minimum shear wavelength, 12-cell layer, 2x2x2 overlapping "
                "subdomains (overlap 4, padding 6, multicolour schedule), 16 sources, shift 0.6, "
                "complex64 DD-MG V(2,1) preconditioner (two pre-, one post-smoothing step)",
    dim=3, n=(128, 128, 128), h=10.0, media_fn=lambda: M.layered_3d_media((128, 128, 128)),
    ppw=8.0, abl_cells=(12, 12, 12), shift=0.6, levels=4, nu1=2, nu2=1, damping=(0.5, 0.5, 0.2),
    precond_bits=32, dd_parts=(2, 2, 2), dd_overlap=4, dd_pad=6, dd_colors=0, maxit=500,
    sources_fn=_src_lattice(4, 32, 16, 5, seed=7)))

# Reduced-size relatives used where the oracle has to factorise the full operator.
_add(Workload(
    name="c2s_hetero128_fp64",
    description="c2 media generator at 128x128 (parity size)",
    dim=2, n=(128, 128), h=10.0, media_fn=lambda: M.heterogeneous_2d_media((128, 128)), ppw=10.0,
    abl_cells=(20, 20), shift=0.5, levels=4, damping=(0.75, 0.5, 0.5), precond_bits=64,
    sources_fn=_src_top_single))

_add(Workload(
    name="c3s_hetero128_batch8_fp32",
    description="c3 at 128x128 with 8 sources (parity size)",
    dim=2, n=(128, 128), h=10.0, media_fn=lambda: M.heterogeneous_2d_media((128, 128)), ppw=10.0,
    abl_cells=(20, 20), shift=0.5, levels=4, damping=(0.75, 0.5, 0.5), precond_bits=32,
    sources_fn=_scaled_line(8, 5, seed=3)))

_add(Workload(
    name="c4s_layered32_dd8_batch4_fp32",
    description="c4 generator at 32^3 with 2x2x2 subdomains and 4 sources (parity size)",
    dim=3, n=(32, 32, 32), h=10.0, media_fn=lambda: M.layered_3d_media((32, 32, 32)),
    ppw=8.0, abl_cells=(6, 6, 6), shift=0.4, levels=3, damping=(0.5, 0.5),
    precond_bits=32, dd_parts=(2, 2, 2), dd_overlap=4, dd_pad=2, dd_colors=1,
    sources_fn=_src_lattice(2, 16, 8, 5, seed=7)))

_add(Workload(
    name="c4m_layered32_dd8_batch16_fp32",
    description="c4 at 32^3 in c4's solver configuration: 2x2x2 subdomains (overlap 4, padding 6, "
                "multicolour schedule), 4 levels per 24^3 subdomain, V(2,1), shift 0.6, 16 sources, complex64 "
                "cycle (parity size of the bench configuration)",
    dim=3, n=(32, 32, 32), h=10.0, media_fn=lambda: M.layered_3d_media((32, 32, 32)),
    ppw=8.0, abl_cells=(6, 6, 6), shift=0.6, levels=4, nu1=2, nu2=1, damping=(0.5, 0.5, 0.2),
    precond_bits=32, dd_parts=(2, 2, 2), dd_overlap=4, dd_pad=6, dd_colors=0,
    sources_fn=_src_lattice(4, 8, 4, 5, seed=7)))


def _rec_line(count: int, spacing: int, first: int, depth: int):
    def fn(w: Workload):
        return [(0, (first + spacing * r, depth)) for r in range(count)]
    return fn


def unknown_offset(w: Workload, comp: int, pos) -> int:
    """Position of an unknown in one right-hand side's vector: component blocks
    [u_0, u_1, (u_2), p] in turn, each x fastest; u_k has n_k - 1 interior faces
    along its axis (pos[k] = 1..n_k - 1)."""
    dims = []
    for k in range(w.dim + 1):
        dims.append([w.n[a] - 1 if a == k else w.n[a] for a in range(w.dim)])
    off = sum(int(np.prod(dims[k])) for k in range(comp))
    d = dims[comp]
    q = [pos[a] - 1 if a == comp else pos[a] for a in range(w.dim)]
    idx = 0
    for a in reversed(range(w.dim)):
        idx = idx * d[a] + q[a]
    return off + idx


def receiver_offsets(w: Workload) -> np.ndarray:
    return np.array([unknown_offset(w, c, p) for c, p in w.receivers_fn(w)], dtype=np.int64)


_add(Workload(
    name="c5_fwi256_batch16",
    description="differentiable 2D solve: the c2 media generator at 256x256 (background model) "
                "and the same with a +10% Gaussian anomaly in mu (true model), 16 x-forces at depth "
                "5 (x = 8 + 16 s, seeded phases), 128 receivers of u_1 at depth 3 (x = 1 + 2 r), "
                "least-squares data misfit",
    dim=2, n=(256, 256), h=10.0, media_fn=lambda: M.heterogeneous_2d_media((256, 256)), ppw=10.0,
    abl_cells=(20, 20), shift=0.5, levels=5, cycle=2, damping=(0.75, 0.5, 0.5, 0.5),
    precond_bits=32, tol=1e-10, maxit=600, sources_fn=_src_line(16, 16, 8, 5, seed=8),
    receivers_fn=_rec_line(128, 2, 1, 3), true_media_fn=lambda: M.fwi_true_media((256, 256))))

_add(Workload(
    name="c5s_fwi64_batch4",
    description="c5 at 64x64 with 4 sources and 32 receivers (parity size)",
    dim=2, n=(64, 64), h=10.0, media_fn=lambda: M.heterogeneous_2d_media((64, 64), corr_vp=5.0, corr_nu=16.0),
    ppw=10.0, abl_cells=(8, 8), shift=0.5, levels=3, cycle=2, damping=(0.75, 0.5), precond_bits=64,
    tol=1e-12, maxit=600, sources_fn=_src_line(4, 16, 8, 5, seed=8), receivers_fn=_rec_line(32, 2, 1, 3),
    true_media_fn=lambda: M.fwi_true_media((64, 64), corr_vp=5.0, corr_nu=16.0)))


def _constant_media(n, lam: float):
    shape = tuple(reversed(n))
    one = np.ones(shape)
    return dict(lam=lam * one, mu=one.copy(), rho=one.copy(), vp=np.sqrt(lam + 2.0) * one, vs=one.copy())


# Poisson-ratio sweep (section 6, first experiment, Fig. 5): constant mu = rho = 1,
# lambda from 0.5 to 16 (Poisson ratio 0.17 to 0.47) on 256x128, 512x256 and
# 1024x512 cells of a 16 x 8 box (h = 1/16, 1/32, 1/64) at w = 3 pi, 6 pi, 12 pi
# (10.7 cells per shear wavelength), 20-cell layer, three-level W(1,1) cycles
# with red-black Vanka damped 0.75 / 0.5 and the shift of section 6 for three
# levels (0.3), one x-force in the middle of the top, 5 cells deep.  The
# 1024x512 grid's 256x128 coarsest level is solved by 8 x 4 overlapping
# subdomains (MG-DD, section 4): its dense inverse would need 154 GB.  Measured
# on MI355X (full Vanka, lambda 0.5 / 16): overlap 2 gives 113 / 264 cycles,
# overlap 6 gives 109 / 124, 4 x 2 subdomains with overlap 8 give 109 / 125.
# Table 2: lambda = 16 with constant damping (0.75, 0.5) against the
# component damping (w_u, w_p) = (0.85, 0.65) on the finest grid, (0.6, 0.4) on
# the second.
SWEEP_LAMBDAS = (0.5, 1.0, 2.0, 4.0, 8.0, 16.0)
SWEEP_GRIDS = {256: (3, 0.3), 512: (3, 0.3), 1024: (3, 0.3)}   # n_x: (levels, shift)
SWEEP_COARSE_DD = {1024: ((8, 4, 1), 6)}                         # coarsest-level subdomains, overlap
TABLE2_DAMPING = {"constant": ((0.75, 0.5), None), "component": ((0.85, 0.6), (0.65, 0.4))}


def poisson_sweep(nx: int, lam: float, vanka: int = 1, damping: str = "constant") -> Workload:
    levels, shift = SWEEP_GRIDS[nx]
    n = (nx, nx // 2)
    dmp, dmp_p = TABLE2_DAMPING[damping]
    return Workload(
        name=f"e3_const{nx}_lam{lam:g}_{'full' if vanka else 'econ'}_{damping}",
        description=f"constant mu = rho = 1, lambda = {lam:g}, {nx}x{nx // 2} cells, h = {16 / nx:g}",
        dim=2, n=n, h=16.0 / nx, media_fn=lambda: _constant_media(n, lam), ppw=32.0 / 3.0,
        abl_cells=(20, 20), shift=shift, levels=levels, cycle=2, damping=dmp, damping_p=dmp_p, vanka=vanka,
        precond_bits=64, tol=1e-6, maxit=600, sources_fn=_src_top_single,
        coarse_dd_parts=SWEEP_COARSE_DD.get(nx, ((1, 1, 1), 2))[0],
        coarse_dd_overlap=SWEEP_COARSE_DD.get(nx, ((1, 1, 1), 2))[1])


def get_config(name: str) -> Workload:
    return CONFIGS[name]
