"""Seeded synthetic elastic media.

Arrays are numpy float64 with shape (ny, nx) in 2D and (nz, ny, nx) in 3D, i.e.
x is the fastest axis and the last grid axis (y in 2D, z in 3D) is depth.  The
media stand in for the paper's geophysical models (Marmousi2, SEG/EAGE
Overthrust, the "linear" model of section 6), which are not available here: they
have the same kind of structure (smooth heterogeneity, layering, Poisson ratios
up to nearly incompressible) but none of their values.
"""
from __future__ import annotations

import numpy as np


def gaussian_random_field(shape, corr_len: float, seed: int, lo: float, hi: float) -> np.ndarray:
    """White noise convolved (periodically, via FFT) with exp(-r^2 / (2 l^2)),
    standardised, then min-max mapped onto [lo, hi]."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    kernel = np.ones(shape)
    for ax, n in enumerate(shape):
        r = np.arange(n, dtype=np.float64)
        r = np.minimum(r, n - r)                      # periodic distance to index 0
        g = np.exp(-r * r / (2.0 * corr_len * corr_len))
        bshape = [1] * len(shape)
        bshape[ax] = n
        kernel = kernel * g.reshape(bshape)
    field = np.real(np.fft.ifftn(np.fft.fftn(noise) * np.fft.fftn(kernel)))
    field = (field - field.mean()) / field.std()
    fmin, fmax = field.min(), field.max()
    return lo + (hi - lo) * (field - fmin) / (fmax - fmin)


def gardner_density(vp: np.ndarray) -> np.ndarray:
    """Gardner-like density [kg/m^3] from P velocity [m/s]."""
    return 310.0 * vp ** 0.25


def vs_from_poisson(vp: np.ndarray, nu: np.ndarray) -> np.ndarray:
    return vp * np.sqrt((1.0 - 2.0 * nu) / (2.0 * (1.0 - nu)))


def lame_from_velocities(vp, vs, rho):
    """Return (lambda, mu) [Pa] from Vp, Vs [m/s] and rho [kg/m^3]."""
    mu = rho * vs * vs
    lam = rho * vp * vp - 2.0 * mu
    return lam, mu


def shear_frequency(vs_min: float, h: float, points_per_wavelength: float) -> float:
    """Angular frequency with the given number of cells per minimum shear wavelength."""
    f = vs_min / (points_per_wavelength * h)
    return 2.0 * np.pi * f


def homogeneous_media(n, vp=2000.0, vs=2000.0 / np.sqrt(3.0), rho=1000.0):
    shape = tuple(reversed(n))
    vp_a = np.full(shape, vp)
    vs_a = np.full(shape, vs)
    rho_a = np.full(shape, rho)
    lam, mu = lame_from_velocities(vp_a, vs_a, rho_a)
    return dict(lam=lam, mu=mu, rho=rho_a, vp=vp_a, vs=vs_a)


def heterogeneous_2d_media(n, seed_vp=1, seed_nu=2, vp_range=(1500.0, 4500.0),
                           nu_range=(0.25, 0.45), corr_vp=20.0, corr_nu=64.0):
    shape = tuple(reversed(n))
    vp = gaussian_random_field(shape, corr_vp, seed_vp, *vp_range)
    nu = gaussian_random_field(shape, corr_nu, seed_nu, *nu_range)
    vs = vs_from_poisson(vp, nu)
    rho = gardner_density(vp)
    lam, mu = lame_from_velocities(vp, vs, rho)
    return dict(lam=lam, mu=mu, rho=rho, vp=vp, vs=vs)


def layered_3d_media(n, n_layers=8, seed_layers=4, seed_pert=5, seed_nu=6,
                     vp_range=(1500.0, 4500.0), nu_range=(0.30, 0.45),
                     corr_pert=10.0, corr_nu=32.0, pert=0.05):
    nx, ny, nz = n
    shape = (nz, ny, nx)
    rng = np.random.default_rng(seed_layers)
    layer_vp = np.sort(rng.uniform(vp_range[0], vp_range[1], size=n_layers))
    thick = nz // n_layers
    idx = np.minimum(np.arange(nz) // max(thick, 1), n_layers - 1)
    vp = np.broadcast_to(layer_vp[idx][:, None, None], shape).copy()
    g = gaussian_random_field(shape, corr_pert, seed_pert, -1.0, 1.0)
    g = g / np.abs(g).max()
    vp = vp * (1.0 + pert * g)
    nu = gaussian_random_field(shape, corr_nu, seed_nu, *nu_range)
    vs = vs_from_poisson(vp, nu)
    rho = gardner_density(vp)
    lam, mu = lame_from_velocities(vp, vs, rho)
    return dict(lam=lam, mu=mu, rho=rho, vp=vp, vs=vs)


def gaussian_anomaly(shape, centre, width: float, amplitude: float) -> np.ndarray:
    """1 + amplitude * exp(-|x - centre|^2 / (2 width^2)) on the cell grid; centre
    is given in cell coordinates (x, y[, z]), shape as the media arrays."""
    grids = np.meshgrid(*[np.arange(v) + 0.5 for v in shape], indexing="ij")
    r2 = np.zeros(shape)
    for ax, g in enumerate(grids):
        r2 = r2 + (g - centre[len(shape) - 1 - ax]) ** 2
    return 1.0 + amplitude * np.exp(-r2 / (2.0 * width * width))


def fwi_true_media(n, amplitude=0.10, **kw):
    """The 2D heterogeneous medium with a smooth Gaussian anomaly in mu (the
    'true' model of an inversion test); lambda and rho are unchanged."""
    m = heterogeneous_2d_media(n, **kw)
    shape = tuple(reversed(n))
    bump = gaussian_anomaly(shape, (n[0] / 2.0, 0.4 * n[1]), n[0] / 16.0, amplitude)
    out = dict(m)
    out["mu"] = m["mu"] * bump
    out["vs"] = np.sqrt(out["mu"] / m["rho"])
    return out
