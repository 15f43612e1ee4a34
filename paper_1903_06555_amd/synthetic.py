"""Seeded synthetic inputs: baseline coordinates, weights and sky images.

This module holds no arithmetic of the imaging method (no kernels, no
tapers, no stacking).  It only lays out arrays of the shapes and value
distributions used by the paper's MWA observation (Sec. 4: 2048^2 image,
45 arcsec pixels, 25 deg field, w up to ~600 wavelengths after folding),
so that the GPU library and the FP64 oracle can be fed identical inputs.

The MWA Fornax A visibilities of Sec. 4 are not available; Earth-rotation
synthesis of a seeded random 128-antenna layout stands in for them.  The
geometry follows the standard ENU -> equatorial -> (u, v, w) rotation
(Thompson, Moran & Swenson, "Interferometry and Synthesis in Radio
Astronomy", ch. 4).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_LIGHT = 299_792_458.0          # m/s
EARTH_OMEGA = 7.2921e-5          # rad/s, sidereal rotation rate
MWA_LATITUDE_DEG = -26.703       # MWA site latitude
PHASE_CENTRE_DEC_DEG = -36.3     # ~9.6 deg from zenith at transit -> |w| up to ~500


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic imaging problem (image side, field, visibilities, stacks)."""
    name: str
    n: int                  # image side in pixels
    fov_deg: float          # full field of view (direction-cosine width, degrees)
    m_vis: int              # number of visibilities
    n_stacks: int           # number of w-stacks K
    fold: bool              # conjugate-symmetry folding of w < 0
    precision: str          # "fp32_fp64phase" or "fp64"
    uvw_recipe: str         # "uniform_box" or "mwa_rotation"
    duration_s: float = 0.0  # Earth-rotation span for "mwa_rotation"
    sky: str = "gaussian20"  # "gaussian20" or "exp500"
    seed: int = 1
    oversample: float = 2.0
    kb_support: int = 4


WORKLOADS = {
    # 64x64 image on a 128^2 grid, 2000 visibilities in a box, one stack, FP64.
    "tiny_box_64": Workload("tiny_box_64", 64, 10.0, 2000, 1, False, "fp64",
                            "uniform_box", sky="gaussian20", seed=1),
    # MWA-like single stack: 1024^2 image, 25 deg, 1e6 visibilities over 2 min.
    "mwa_1024_single_stack": Workload("mwa_1024_single_stack", 1024, 25.0,
                                      1_000_000, 1, False, "fp32_fp64phase",
                                      "mwa_rotation", duration_s=120.0,
                                      sky="exp500", seed=2),
    # Hybrid w-stacking, one GPU's share: 4096^2, 2.5e7 visibilities, 16 stacks.
    "mwa_4096_16_stacks": Workload("mwa_4096_16_stacks", 4096, 25.0,
                                   25_000_000, 16, True, "fp32_fp64phase",
                                   "mwa_rotation", duration_s=1800.0,
                                   sky="exp500", seed=3),
    # Kernel construction at the paper's own set-up (Sec. 4): 2048^2, 25 deg,
    # w folded onto w >= 0 and split into 50 k-means stacks; 1e7 visibilities
    # (the paper's run had 126.6e6 on 50 nodes).
    "mwa_2048_50_stacks": Workload("mwa_2048_50_stacks", 2048, 25.0, 10_000_000, 50, True,
                                   "fp32_fp64phase", "mwa_rotation", duration_s=1800.0,
                                   sky="exp500", seed=6),
    # Differentiable operator: 2048^2, 5e6 visibilities, 8 stacks.
    "mwa_2048_8_stacks": Workload("mwa_2048_8_stacks", 2048, 25.0, 5_000_000,
                                  8, True, "fp32_fp64phase", "mwa_rotation",
                                  duration_s=1800.0, sky="exp500", seed=4),
}


def wavelength_m(freq_hz: float = 150e6) -> float:
    return C_LIGHT / freq_hz


def antenna_layout(n_ant: int = 128, radius_m: float = 3000.0, seed: int = 0) -> np.ndarray:
    """East/North/Up positions (metres) uniform in a flat disc."""
    rng = np.random.default_rng(seed)
    rad = radius_m * np.sqrt(rng.uniform(0.0, 1.0, n_ant))
    ang = rng.uniform(0.0, 2.0 * math.pi, n_ant)
    enu = np.zeros((n_ant, 3))
    enu[:, 0] = rad * np.cos(ang)
    enu[:, 1] = rad * np.sin(ang)
    return enu


def baselines_enu(enu: np.ndarray) -> np.ndarray:
    i, j = np.triu_indices(enu.shape[0], k=1)
    return enu[j] - enu[i]


def mwa_rotation_uvw(m_vis: int, duration_s: float, freq_hz: float = 150e6,
                     n_ant: int = 128, radius_m: float = 3000.0,
                     latitude_deg: float = MWA_LATITUDE_DEG,
                     dec_deg: float = PHASE_CENTRE_DEC_DEG,
                     layout_seed: int = 0) -> np.ndarray:
    """(u, v, w) in wavelengths, [m_vis, 3] float64, time-major.

    n_ant*(n_ant-1)/2 baselines are sampled at T = ceil(M / n_bl) hour
    angles spread symmetrically about transit over ``duration_s``; the first
    ``m_vis`` rows are kept.
    """
    bl = baselines_enu(antenna_layout(n_ant, radius_m, layout_seed))
    n_bl = bl.shape[0]
    n_t = max(1, -(-m_vis // n_bl))
    lat = math.radians(latitude_deg)
    dec = math.radians(dec_deg)
    # ENU -> equatorial XYZ
    e, n, u_up = bl[:, 0], bl[:, 1], bl[:, 2]
    X = -math.sin(lat) * n + math.cos(lat) * u_up
    Y = e
    Z = math.cos(lat) * n + math.sin(lat) * u_up
    if n_t == 1:
        hours = np.zeros(1)
    else:
        hours = (np.arange(n_t) - 0.5 * (n_t - 1)) * (duration_s / (n_t - 1)) * EARTH_OMEGA
    lam = wavelength_m(freq_hz)
    out = np.empty((n_t, n_bl, 3))
    sd, cd = math.sin(dec), math.cos(dec)
    for t, h in enumerate(hours):
        sh, ch = math.sin(h), math.cos(h)
        out[t, :, 0] = sh * X + ch * Y
        out[t, :, 1] = -sd * ch * X + sd * sh * Y + cd * Z
        out[t, :, 2] = cd * ch * X - cd * sh * Y + sd * Z
    return (out.reshape(-1, 3)[:m_vis] / lam).copy()


def uniform_box_uvw(m_vis: int, u_max: float = 40.0, w_max: float = 20.0,
                    seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    uvw = np.empty((m_vis, 3))
    uvw[:, 0] = rng.uniform(-u_max, u_max, m_vis)
    uvw[:, 1] = rng.uniform(-u_max, u_max, m_vis)
    uvw[:, 2] = rng.uniform(-w_max, w_max, m_vis)
    return uvw


def point_source_sky(n: int, n_src: int, amplitudes: str, seed: int,
                     margin: int = 0) -> np.ndarray:
    """Real [n, n] float64 image (row = m index, column = l index).

    Sources sit on integer pixels drawn uniformly (optionally ``margin``
    pixels away from the border); amplitudes are N(0, 1) ("gaussian") or
    exponential with 1 Jy scale ("exp").
    """
    rng = np.random.default_rng(seed)
    x = np.zeros((n, n))
    rows = rng.integers(margin, n - margin, n_src)
    cols = rng.integers(margin, n - margin, n_src)
    if amplitudes == "gaussian":
        amp = rng.normal(0.0, 1.0, n_src)
    elif amplitudes == "exp":
        amp = rng.exponential(1.0, n_src)
    else:
        raise ValueError(amplitudes)
    np.add.at(x, (rows, cols), amp)
    return x


def workload_uvw(wl: Workload, m_vis: int | None = None) -> np.ndarray:
    m = wl.m_vis if m_vis is None else m_vis
    if wl.uvw_recipe == "uniform_box":
        return uniform_box_uvw(m, seed=wl.seed)
    if wl.uvw_recipe == "mwa_rotation":
        return mwa_rotation_uvw(m, wl.duration_s)
    raise ValueError(wl.uvw_recipe)


def workload_sky(wl: Workload) -> np.ndarray:
    if wl.sky == "gaussian20":
        return point_source_sky(wl.n, 20, "gaussian", wl.seed)
    if wl.sky == "exp500":
        return point_source_sky(wl.n, 500, "exp", wl.seed)
    raise ValueError(wl.sky)


def random_vis(m_vis: int, seed: int) -> np.ndarray:
    """Complex128 [m_vis] standard-normal visibilities (adjoint inputs)."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=m_vis) + 1j * rng.normal(size=m_vis)


def random_image(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, n))


def random_weights(m_vis: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 1.5, m_vis)
