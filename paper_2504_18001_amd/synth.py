"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only draws numbers and builds scene descriptions (cameras,
transfer functions, parameter arrays).  It contains none of the rendering
method's arithmetic: no hash-grid encoding, no MLP, no brick or page-table
logic.  Everything is deterministic for a given seed (NumPy PCG64).

The paper's datasets (Table 1) and trained networks are not available; the
random-init INRs, Gaussian-blob grid and Fourier field below stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# INR architecture (hash grid of Section 3 / Figure 2, then a small MLP)
# ----------------------------------------------------------------------------


@dataclass(frozen=True)
class InrArch:
    """Architecture of a hash-grid INR (Section 3).

    dims       LoD-0 volume size (Vx, Vy, Vz) in voxels.
    n_levels   number of grid levels m; n_features entries per table slot n.
    log2_table log2 of the per-level hash-table capacity T.
    n_min, growth  per-level resolution N_l = floor(n_min * growth**l).
    widths     MLP widths, widths[0] = n_levels * n_features, widths[-1] = 1.
    """

    dims: tuple
    n_levels: int
    n_features: int
    log2_table: int
    n_min: int
    growth: float
    widths: tuple

    @property
    def level_res(self) -> list:
        # floor in FP64; the tiny epsilon keeps exact powers (e.g. 4*2560 at the
        # last level of the tera-shaped domain) from rounding down.
        return [int(math.floor(self.n_min * self.growth ** l + 1e-7)) for l in range(self.n_levels)]

    @property
    def level_sizes(self) -> list:
        T = 1 << self.log2_table
        return [min(T, (n + 1) ** 3) for n in self.level_res]

    @property
    def table_entries(self) -> int:
        return int(sum(self.level_sizes))

    @property
    def n_weights(self) -> int:
        w = self.widths
        return int(sum(w[i] * w[i + 1] for i in range(len(w) - 1)))


def random_inr_params(arch: InrArch, seed: int):
    """Random-init parameters: table entries ~ U(-1, 1); each weight matrix
    [out][in] ~ He-uniform U(-sqrt(6/fan_in), +sqrt(6/fan_in)).  Returned as
    float32 arrays (table [entries][F], weights concatenated per layer)."""
    rng = np.random.default_rng(seed)
    table = rng.uniform(-1.0, 1.0, size=(arch.table_entries, arch.n_features)).astype(np.float32)
    ws = []
    w = arch.widths
    for i in range(len(w) - 1):
        lim = math.sqrt(6.0 / w[i])
        ws.append(rng.uniform(-lim, lim, size=(w[i + 1], w[i])).astype(np.float32).ravel())
    return table, np.concatenate(ws).astype(np.float32)


def halton_points(n: int) -> np.ndarray:
    """First n points (index 1..n) of the Halton sequence in bases 2, 3, 5;
    used as a fixed probe set inside (0,1)^3."""
    out = np.zeros((n, 3), dtype=np.float64)
    idx = np.arange(1, n + 1, dtype=np.int64)
    for a, base in enumerate((2, 3, 5)):
        k = idx.copy()
        f = 1.0
        while np.any(k > 0):
            f /= base
            out[:, a] += f * (k % base)
            k //= base
    return out


# ----------------------------------------------------------------------------
# Transfer functions: 256 RGBA rows, float32
# ----------------------------------------------------------------------------


def tf_ramp() -> np.ndarray:
    r = (np.arange(256, dtype=np.float64) / 255.0).astype(np.float32)
    return np.repeat(r[:, None], 4, axis=1).copy()


def tf_random(seed: int, n_ctrl: int = 9) -> np.ndarray:
    """Random RGBA table, piecewise linear through `n_ctrl` random control
    rows (U(0,1) per channel).  Its slope is bounded (<= (n_ctrl-1) per unit
    value), so a value error maps to a colour error of the same order."""
    rng = np.random.default_rng(seed)
    ctrl = rng.uniform(0.0, 1.0, size=(n_ctrl, 4))
    xs = np.linspace(0.0, 255.0, n_ctrl)
    rows = np.arange(256, dtype=np.float64)
    out = np.stack([np.interp(rows, xs, ctrl[:, c]) for c in range(4)], axis=1)
    return out.astype(np.float32)


def tf_iid(seed: int) -> np.ndarray:
    """Random RGBA table with every row and channel drawn independently from
    U(0,1): neighbouring rows are unrelated, so the linear interpolation
    between rows has slopes of up to 255 per unit value and a value error can
    reach the colour about 255 times larger."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(256, 4)).astype(np.float32)


def tf_window(lo: int, hi: int, edge: int = 32) -> np.ndarray:
    """Ramp colours with opacity zero outside rows [lo, hi] and rising over
    `edge` rows from lo (opacity is exactly zero at and below row lo)."""
    t = tf_ramp()
    r = np.arange(256, dtype=np.float64)
    a = np.clip((r - lo) / edge, 0.0, 1.0) * r / 255.0
    a[r > hi] = 0.0
    t[:, 3] = a.astype(np.float32)
    return t


# ----------------------------------------------------------------------------
# Cameras: basis computed in FP64 and rounded to float32
# ----------------------------------------------------------------------------

PERSPECTIVE = 0
ORTHOGRAPHIC = 1


@dataclass
class Camera:
    projection: int
    eye: np.ndarray
    forward: np.ndarray
    right: np.ndarray
    up: np.ndarray
    width: int
    height: int
    tan_half_x: float = 0.0
    tan_half_y: float = 0.0
    ortho_w: float = 0.0
    ortho_h: float = 0.0


def _basis(eye, target, world_up=(0.0, 1.0, 0.0)):
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(world_up, np.float64))
    nr = np.linalg.norm(r)
    if nr < 1e-12:
        r = np.cross(f, np.array([0.0, 0.0, 1.0]))
        nr = np.linalg.norm(r)
    r /= nr
    u = np.cross(r, f)
    return f, r, u


def look_at(projection, eye, target, width, height, fov_y_deg=45.0, ortho_w=0.0, ortho_h=0.0,
            world_up=(0.0, 1.0, 0.0)) -> Camera:
    f, r, u = _basis(eye, target, world_up)
    cam = Camera(projection=projection, eye=np.asarray(eye, np.float64).astype(np.float32),
                 forward=f.astype(np.float32), right=r.astype(np.float32), up=u.astype(np.float32),
                 width=int(width), height=int(height))
    if projection == PERSPECTIVE:
        ty = math.tan(math.radians(fov_y_deg) / 2.0)
        cam.tan_half_y = float(np.float32(ty))
        cam.tan_half_x = float(np.float32(ty * width / height))
    else:
        cam.ortho_w = float(np.float32(ortho_w))
        cam.ortho_h = float(np.float32(ortho_h))
    return cam


def orbit_camera(projection, dims, radius, angle_deg, elevation_deg, width, height, fov_y_deg=45.0,
                 ortho_w=0.0, ortho_h=0.0, center=None) -> Camera:
    """Eye on a circle about the volume centre (rotation about the y axis),
    lifted by `elevation_deg`."""
    c = np.array([(d - 1) / 2.0 for d in dims], np.float64) if center is None else np.asarray(center, np.float64)
    th, el = math.radians(angle_deg), math.radians(elevation_deg)
    eye = c + radius * np.array([math.sin(th) * math.cos(el), math.sin(el), math.cos(th) * math.cos(el)])
    return look_at(projection, eye, c, width, height, fov_y_deg, ortho_w, ortho_h)


# ----------------------------------------------------------------------------
# Explicit volumes
# ----------------------------------------------------------------------------


def blob_volume(dims, n_blobs=32, seed=0) -> np.ndarray:
    """Sum of isotropic Gaussian blobs clamped to [0,1], float32 [Vz][Vy][Vx]."""
    rng = np.random.default_rng(seed)
    V = np.asarray(dims)
    c = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * V
    s = rng.uniform(3.0, 10.0, size=n_blobs)
    a = rng.uniform(0.2, 1.0, size=n_blobs)
    z, y, x = np.meshgrid(np.arange(dims[2]), np.arange(dims[1]), np.arange(dims[0]), indexing="ij")
    out = np.zeros((dims[2], dims[1], dims[0]), np.float64)
    for i in range(n_blobs):
        r2 = (x - c[i, 0]) ** 2 + (y - c[i, 1]) ** 2 + (z - c[i, 2]) ** 2
        out += a[i] * np.exp(-r2 / (2.0 * s[i] ** 2))
    return np.clip(out, 0.0, 1.0).astype(np.float32)


def fourier_modes(n_modes=512, kmax=128, seed=0):
    """Integer wave-vectors with uniformly random direction and |k| ~ U[1,kmax]
    (rounded), amplitudes |k|^(-5/3) and phases U[0, 2pi)."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_modes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    mag = rng.uniform(1.0, kmax, size=n_modes)
    k = np.rint(d * mag[:, None]).astype(np.int64)
    k[np.all(k == 0, axis=1)] = (1, 0, 0)
    amp = np.linalg.norm(k, axis=1) ** (-5.0 / 3.0)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    return k, amp, ph


def fourier_field(V: int, modes, device="cpu", z_block=32):
    """The periodic field sum_j A_j cos(2 pi k_j . x / V + phi_j) on the V^3
    lattice x in [0, V)^3, normalised to [0, 1] by its minimum and maximum;
    float32 [V][V][V] (z, y, x).  Evaluated as a separable complex product
    (per z slice a [V x J] by [J x V] product) with torch on `device`."""
    import torch
    k, amp, ph = modes
    dev = torch.device(device)
    kk = torch.as_tensor(k, dtype=torch.float64, device=dev)
    c = torch.as_tensor(amp, dtype=torch.float64, device=dev) * torch.exp(
        1j * torch.as_tensor(ph, dtype=torch.float64, device=dev))
    xs = torch.arange(V, dtype=torch.float64, device=dev)
    # E_a[j][x] = exp(i 2 pi k_ja x / V)
    E = [torch.exp(2j * math.pi * kk[:, a:a + 1] * xs[None, :] / V) for a in range(3)]
    ex = E[0].to(torch.complex64)  # [J][V]
    out = torch.empty((V, V, V), dtype=torch.float32, device=dev)
    for z0 in range(0, V, z_block):
        z1 = min(V, z0 + z_block)
        # P[z][y][j] = c_j Ez[j][z] Ey[j][y]
        pz = (c[:, None] * E[2][:, z0:z1]).T  # [Z][J]
        P = (pz[:, None, :] * E[1].T[None, :, :]).to(torch.complex64)  # [Z][V(y)][J]
        out[z0:z1] = torch.matmul(P.real, ex.real) - torch.matmul(P.imag, ex.imag)
    lo, hi = out.min(), out.max()
    out.sub_(lo).div_(hi - lo)
    return out


# ----------------------------------------------------------------------------
# Random brick requests / residency
# ----------------------------------------------------------------------------


def random_requests(nb_per_lod, n, seed=0) -> np.ndarray:
    """n random (lod, bx, by, bz) int32 rows, LoD uniform over the given levels."""
    rng = np.random.default_rng(seed)
    out = np.empty((n, 4), np.int32)
    lods = rng.integers(0, len(nb_per_lod), size=n)
    for i, L in enumerate(lods):
        nb = nb_per_lod[L]
        out[i] = (L, rng.integers(0, nb[0]), rng.integers(0, nb[1]), rng.integers(0, nb[2]))
    return out


def random_subset(n_total, fraction, seed=0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    k = int(round(n_total * fraction))
    return np.sort(rng.choice(n_total, size=k, replace=False)).astype(np.int32)
