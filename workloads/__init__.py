"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds input generation only (velocity models, acquisition
geometry, source wavelet samples, request streams).  It contains none of the
solver's arithmetic: no stencil, CFL limit, damping, interpolation or codec.

The paper's workload is the 3-D Overthrust model (287x881x881 incl. a 40-cell
absorbing layer, 25 m, 2526 steps, Ricker source at the surface; Sec.
"Problem and test case").  That model is not available, so every config below
is a synthetic stand-in of the same kind: layered / smooth velocity, a Ricker
point source near the surface, a surface receiver line or grid.

Conventions: grids are given by their interior point counts (axis 0 = x
fastest, last axis = depth z); ``nbl`` absorbing cells are added on every
side; velocities are m/s; positions are metres measured from the first
interior grid point and ordered like the axes (x[, y], z).  Arrays are C-order
with depth slowest: [z][x] in 2-D, [z][y][x] in 3-D.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


@dataclass
class Shot:
    name: str
    ndim: int
    n: tuple                 # interior points (x[, y], z)
    h: tuple                 # spacing (m) per axis
    nbl: int
    order: int               # space order 2K
    nt: int                  # time steps N
    f0: float                # Ricker peak frequency (Hz)
    vel: np.ndarray          # interior velocity of the simulated model, float32, [z]([y])[x]
    vel_true: np.ndarray     # interior velocity of the model that makes d_obs
    src: np.ndarray          # (nsrc, ndim) metres
    rec: np.ndarray          # (nrec, ndim) metres
    cfl_frac: float = 0.4
    extra: dict = field(default_factory=dict)

    @property
    def vmax(self) -> float:
        """Largest velocity over both models (one dt and one damping profile serve both)."""
        return float(max(self.vel.max(), self.vel_true.max()))

    def padded_shape(self) -> tuple:
        return tuple(reversed([self.n[d] + 2 * self.nbl for d in range(self.ndim)]))

    def padded(self, which: str = "vel") -> np.ndarray:
        v = self.vel if which == "vel" else self.vel_true
        return pad_edge(v, self.nbl)

    @property
    def npoints(self) -> int:
        return int(np.prod(self.padded_shape()))


def pad_edge(v: np.ndarray, nbl: int) -> np.ndarray:
    """Velocity in the absorbing layer: the nearest interior value."""
    return np.ascontiguousarray(np.pad(v, nbl, mode="edge"), dtype=np.float32)


def ricker(f0: float, dt: float, nt: int) -> np.ndarray:
    """Ricker wavelet samples r(n dt), n = 0..nt-1, peak at t0 = 1/f0, amplitude 1."""
    t = np.arange(nt, dtype=np.float64) * dt - 1.0 / f0
    a = (math.pi * f0 * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float64)


def _axes(n, h):
    """Physical coordinate arrays (metres) per axis, x first."""
    return [np.arange(n[d]) * h[d] for d in range(len(n))]


def _grid(n, h):
    ax = _axes(n, h)
    # array order is reversed (depth slowest)
    return np.meshgrid(*reversed(ax), indexing="ij")   # returns [z, (y,) x]


def gaussian_anomaly(n, h, amp: float, sigma_m: float, centre_m) -> np.ndarray:
    g = _grid(n, h)
    coords = list(reversed(g))        # x, (y,) z
    r2 = sum((coords[d] - centre_m[d]) ** 2 for d in range(len(n)))
    return amp * np.exp(-r2 / (2.0 * sigma_m ** 2))


def surface_geometry(n, h, depth_cells: int = 2, rec_every: int = 1):
    """Source at the lateral centre, depth_cells below the top; receivers on every
    rec_every-th grid point of the same depth."""
    nd = len(n)
    zdepth = depth_cells * h[nd - 1]
    lat = [(n[d] - 1) * h[d] / 2.0 for d in range(nd - 1)]
    src = np.array([lat + [zdepth]], dtype=np.float64)
    lines = [np.arange(0, n[d], rec_every) * h[d] for d in range(nd - 1)]
    if nd == 2:
        rec = np.stack([lines[0], np.full(len(lines[0]), zdepth)], axis=1)
    else:
        yy, xx = np.meshgrid(lines[1], lines[0], indexing="ij")
        rec = np.stack([xx.ravel(), yy.ravel(), np.full(xx.size, zdepth)], axis=1)
    return src, np.ascontiguousarray(rec, dtype=np.float64)


# ------------------------------------------------------------------ configs

def two_layer_2d(n=(101, 101), h=(10.0, 10.0), nbl=20, nt=500, order=4, interface_z=500.0,
                 anomaly_centre=(500.0, 500.0), src_x=500.0, f0=10.0) -> Shot:
    """2-D, two layers 1.5 / 2.5 km/s split at z = 500 m (z >= 500 m below), Ricker 10 Hz
    at (500 m, 20 m), 101 receivers at z = 20 m; d_obs from the same model plus a
    Gaussian +0.2 km/s anomaly (sigma 100 m) at (500 m, 500 m).  The keyword arguments
    move the interface, anomaly and source for smaller test variants."""
    g = _grid(n, h)
    z = g[0]
    vel = np.where(z < interface_z - 1e-9, 1500.0, 2500.0)
    anom = gaussian_anomaly(n, h, 200.0, 100.0, anomaly_centre)
    src = np.array([[src_x, 20.0]])
    rec = np.stack([np.arange(n[0]) * h[0], np.full(n[0], 20.0)], axis=1)
    return Shot("two_layer_2d", 2, tuple(n), tuple(h), nbl, order, nt, f0,
                vel.astype(np.float32), (vel + anom).astype(np.float32), src, rec)


def near_anomaly_2d(n=(61, 61), nt=400, order=4, nbl=20) -> Shot:
    """Small two-layer variant whose anomaly the wave reaches early (well-conditioned residual)."""
    return two_layer_2d(n=n, nbl=nbl, nt=nt, order=order, interface_z=200.0, anomaly_centre=(300.0, 250.0),
                        src_x=300.0, f0=10.0)


def layered_noise_3d(n=(128, 128, 128), h=(10.0, 10.0, 10.0), nbl=20, nt=1000, order=8, seed=2,
                     f0=15.0) -> Shot:
    """3-D, five flat layers 1.5/2.0/2.5/3.0/3.5 km/s times (1 + U(-0.02, 0.02)) (seeded),
    Ricker 15 Hz near the top centre, a receiver on every surface grid point at the
    source depth; d_obs model adds +0.2 km/s, sigma 10 cells, at the interior centre."""
    rng = np.random.default_rng(seed)
    nz = n[2]
    layer = np.minimum((np.arange(nz) * 5) // nz, 4)
    base = (1500.0 + 500.0 * layer)[:, None, None] * np.ones((nz, n[1], n[0]))
    vel = base * (1.0 + rng.uniform(-0.02, 0.02, size=base.shape))
    centre = [(n[d] - 1) * h[d] / 2.0 for d in range(3)]
    anom = gaussian_anomaly(n, h, 200.0, 10 * h[0], centre)
    src, rec = surface_geometry(n, h)
    return Shot("layered_noise_3d", 3, tuple(n), tuple(h), nbl, order, nt, f0,
                vel.astype(np.float32), (vel + anom).astype(np.float32), src, rec)


def smooth_random_2d(n=(400, 400), h=(5.0, 5.0), nbl=20, nt=2000, order=8, seed=3, f0=20.0) -> Shot:
    """2-D smooth random medium: N(0,1) noise (seeded) filtered by a Gaussian of sigma
    50 m, mapped affinely onto [1.5, 3.0] km/s; Ricker 20 Hz, one receiver per surface
    grid point; d_obs model adds +0.2 km/s, sigma 10 cells, centred laterally at a
    quarter of the depth (its reflection returns well within the 2000 steps)."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n[1], n[0]))
    s = gaussian_filter(noise, sigma=50.0 / h[0], mode="reflect")
    s = (s - s.min()) / (s.max() - s.min())
    vel = 1500.0 + 1500.0 * s
    centre = [(n[0] - 1) * h[0] / 2.0, (n[1] - 1) * h[1] / 4.0]
    anom = gaussian_anomaly(n, h, 200.0, 10 * h[0], centre)
    src, rec = surface_geometry(n, h)
    return Shot("smooth_random_2d", 2, tuple(n), tuple(h), nbl, order, nt, f0,
                vel.astype(np.float32), (vel + anom).astype(np.float32), src, rec)


def fault_body_3d(n=(320, 320, 320), h=(12.5, 12.5, 12.5), nbl=40, nt=3000, order=16, f0=8.0) -> Shot:
    """3-D large shot: seven layers 1.5..4.5 km/s (0.5 km/s steps, equal thickness); a
    planar fault through the centre dipping 60 degrees and striking along y, hanging
    wall shifted down 100 m; a 4.5 km/s ellipsoid centred at (0.5, 0.5, 0.7) of the
    extent with semi-axes 600/600/250 m; Ricker 8 Hz, a receiver on every surface grid
    point; d_obs model adds +0.2 km/s, sigma 10 cells, at the interior centre."""
    ext = [(n[d] - 1) * h[d] for d in range(3)]
    z = (np.arange(n[2]) * h[2])[:, None, None]
    y = (np.arange(n[1]) * h[1])[None, :, None]
    x = (np.arange(n[0]) * h[0])[None, None, :]
    xc, zc = ext[0] / 2.0, ext[2] / 2.0
    hanging = z < zc + math.tan(math.radians(60.0)) * (x - xc)
    zeff = np.where(hanging, z - 100.0, z) + 0.0 * y
    thick = (n[2] * h[2]) / 7.0
    layer = np.clip(np.floor(zeff / thick), 0, 6)
    vel = 1500.0 + 500.0 * layer
    c = (0.5 * ext[0], 0.5 * ext[1], 0.7 * ext[2])
    ell = ((x - c[0]) / 600.0) ** 2 + ((y - c[1]) / 600.0) ** 2 + ((z - c[2]) / 250.0) ** 2 <= 1.0
    vel = np.where(ell, 4500.0, vel).astype(np.float32)
    centre = [e / 2.0 for e in ext]
    anom = gaussian_anomaly(n, h, 200.0, 10 * h[0], centre).astype(np.float32)
    src, rec = surface_geometry(n, h)
    return Shot("fault_body_3d", 3, tuple(n), tuple(h), nbl, order, nt, f0,
                vel, (vel + anom).astype(np.float32), src, rec)


def random_layers(n, h, nbl, order, nt, rng, f0) -> Shot:
    """Layered random velocity: 3..7 layers, velocities sorted U(1.5, 3.5) km/s."""
    nd = len(n)
    L = int(rng.integers(3, 8))
    vs = np.sort(rng.uniform(1500.0, 3500.0, size=L))
    nz = n[nd - 1]
    layer = np.minimum((np.arange(nz) * L) // nz, L - 1)
    shape = tuple(reversed(n))
    vel = vs[layer].reshape((nz,) + (1,) * (nd - 1)) * np.ones(shape)
    centre = [(n[d] - 1) * h[d] / 2.0 for d in range(nd)]
    anom = gaussian_anomaly(n, h, 200.0, 10 * h[0], centre)
    src, rec = surface_geometry(n, h)
    return Shot(f"layers{nd}d_{n[0]}", nd, tuple(n), tuple(h), nbl, order, nt, f0,
                vel.astype(np.float32), (vel + anom).astype(np.float32), src, rec)


@dataclass
class Request:
    rid: int
    arrival: float           # seconds from the start of the stream
    shot: Shot


SERVING_CLASSES = [
    # (probability, ndim, n, order, nt)
    (0.6, 2, (512, 512), 8, 1500),
    (0.3, 3, (160, 160, 160), 8, 1200),
    (0.1, 3, (256, 256, 256), 12, 2000),
]


def serving_stream(nreq: int = 200, rate: float = 2.0, seed: int = 5, h: float = 10.0, nbl: int = 20,
                   classes=None, scale: float = 1.0, nt_scale: float = 1.0) -> list:
    """Poisson arrivals of shot-gradient requests with seeded random sizes.
    scale / nt_scale shrink the grids and step counts for small test streams."""
    rng = np.random.default_rng(seed)
    classes = classes or SERVING_CLASSES
    probs = np.array([c[0] for c in classes])
    t = 0.0
    out = []
    for i in range(nreq):
        t += float(rng.exponential(1.0 / rate))
        ci = int(rng.choice(len(classes), p=probs / probs.sum()))
        _, nd, n, order, nt = classes[ci]
        n = tuple(max(8, int(round(x * scale))) for x in n)
        nt = max(4, int(round(nt * nt_scale)))
        f0 = float(rng.uniform(10.0, 20.0))
        shot = random_layers(n, (h,) * nd, nbl, order, nt, rng, f0)
        shot.extra["class"] = ci
        out.append(Request(i, t, shot))
    return out


CONFIGS = {
    "two_layer_2d": two_layer_2d,
    "layered_noise_3d": layered_noise_3d,
    "smooth_random_2d": smooth_random_2d,
    "fault_body_3d": fault_body_3d,
}


def small(shot_fn, **kw) -> Shot:
    return shot_fn(**kw)


__all__ = ["Shot", "pad_edge", "ricker", "surface_geometry", "two_layer_2d", "layered_noise_3d",
           "smooth_random_2d", "fault_body_3d", "near_anomaly_2d", "random_layers", "serving_stream", "CONFIGS", "replace",
           "Request", "gaussian_anomaly"]
