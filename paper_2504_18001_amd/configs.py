"""Named workloads.

Each workload fixes the INR architecture, the camera path, the transfer
functions, the marching parameters and the cache shape.  The synthetic INRs
and fields stand in for the paper's datasets (Table 1), which are not
available.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

from . import synth
from .synth import InrArch

# -- INR architectures --------------------------------------------------------

# 64^3 blob-scale volume: 8 levels x 2 features, T = 2^14, N_min 4, growth 1.5,
# MLP 16 -> 32 -> 32 -> 1.
ARCH_SMALL = InrArch(dims=(64, 64, 64), n_levels=8, n_features=2, log2_table=14, n_min=4,
                     growth=1.5, widths=(16, 32, 32, 1))

# 512^3 virtual volume: 16 levels x 2 features, T = 2^19, growth 1.38,
# MLP 32 -> 64 -> 64 -> 1.
ARCH_512 = InrArch(dims=(512, 512, 512), n_levels=16, n_features=2, log2_table=19, n_min=4,
                   growth=1.38, widths=(32, 64, 64, 1))

# Tera-shaped virtual domain with the channel-flow dimensions of Table 1:
# 16 levels x 4 features, T = 2^22, finest level 10240, MLP 64 -> 64 -> 64 -> 1.
ARCH_TERA = InrArch(dims=(10240, 7680, 1536), n_levels=16, n_features=4, log2_table=22, n_min=4,
                    growth=2560.0 ** (1.0 / 15.0), widths=(64, 64, 64, 1))

# Learned part: 1024^3 field, 16 levels x 2 features, T = 2^20, finest level 1024.
ARCH_LEARN = InrArch(dims=(1024, 1024, 1024), n_levels=16, n_features=2, log2_table=20, n_min=4,
                     growth=256.0 ** (1.0 / 15.0), widths=(32, 64, 64, 1))


@dataclass
class CacheShape:
    brick: int            # stored brick side B (samples per axis)
    n_lods: int
    pool_bricks: int
    max_requests: int
    rank_window: int = 1000
    ranking: int = 1      # 0 = timestamp/key order, 1 = priority ranking
    preload_period: int = 0
    miss_log_capacity: int = 0
    evict_log_capacity: int = 4096


@dataclass
class Workload:
    name: str
    arch: InrArch
    inr_seed: int
    width: int
    height: int
    projection: int
    n_frames: int
    step: float
    lod_scale: float
    cache: CacheShape
    macro_cell: int = 16
    ert_threshold: float = 0.999
    samples_per_iter: int = 32
    seed: int = 1234
    orbit_radius: float = 0.0
    orbit_elev_deg: float = 0.0
    orbit_step_deg: float = 0.0
    fov_y_deg: float = 45.0
    ortho_extent: float = 0.0
    tf_switch_frame: int = -1     # from this frame (mod n_frames) on, a random TF is used
    tf_seed: int = 77
    tf_kind: str = "iid"          # the random TF: "iid" rows, or "smooth" (piecewise linear)

    def camera(self, frame: int, dims=None) -> synth.Camera:
        ang = self.orbit_step_deg * (frame % self.n_frames)
        return synth.orbit_camera(self.projection, dims or self.arch.dims, self.orbit_radius, ang,
                                  self.orbit_elev_deg, self.width, self.height, self.fov_y_deg,
                                  self.ortho_extent, self.ortho_extent)

    def tf(self, frame: int):
        if self.tf_switch_frame >= 0 and (frame % self.n_frames) >= self.tf_switch_frame:
            return synth.tf_iid(self.tf_seed) if self.tf_kind == "iid" else synth.tf_random(self.tf_seed)
        return synth.tf_ramp()


# 64^3, orthographic 128x128, 4 frames at 5 degree steps, B = 8, 2 LoDs, 96-slot pool.
SMALL = Workload(
    name="blob64_ortho128", arch=ARCH_SMALL, inr_seed=0, width=128, height=128,
    projection=synth.ORTHOGRAPHIC, n_frames=4, step=0.5, lod_scale=1.0 / 96.0,
    cache=CacheShape(brick=8, n_lods=2, pool_bricks=96, max_requests=16),
    orbit_radius=96.0, orbit_elev_deg=0.0, orbit_step_deg=5.0, ortho_extent=64.0 * math.sqrt(3.0),
    samples_per_iter=8,
)

# 512^3 random INR at 1920x1080 perspective, 60-frame orbit (6 degrees per frame,
# 20 degree elevation), TF switched at frame 30 from the ramp to a random table
# drawn i.i.d. per row and channel, B = 16, 4 LoDs, 2 GiB pool, up to 256
# bricks decoded per frame (1.05 M voxels, within the 40 bricks of 40^3 =
# 2.56 M voxels per frame of Sec. 6.1).
HD512 = Workload(
    name="inr512_persp1080p", arch=ARCH_512, inr_seed=0, width=1920, height=1080,
    projection=synth.PERSPECTIVE, n_frames=60, step=0.5, lod_scale=1.0 / 800.0,
    cache=CacheShape(brick=16, n_lods=4, pool_bricks=(2 << 30) // (16 ** 3 * 4), max_requests=256,
                     preload_period=4),
    orbit_radius=1159.0, orbit_elev_deg=20.0, orbit_step_deg=6.0, tf_switch_frame=30,
    samples_per_iter=32,
)


@dataclass
class PathShape:
    """Path-tracing parameters (the renderer's `path` argument)."""
    density: float            # majorant extinction per LoD-0 voxel
    light_dir: tuple          # unit vector toward the light (binary32 values)
    light: tuple
    ambient: tuple
    max_bounces: int
    spp: int
    seed: int

    def as_dict(self):
        return dict(density=self.density, light_dir=self.light_dir, light=self.light, ambient=self.ambient,
                    max_bounces=self.max_bounces, spp=self.spp, seed=self.seed)


# Path tracing of the 1080p workload: mean free path 50 voxels at TF opacity 1,
# a light along (1, 3, 2) / sqrt(14), a dim blue environment, up to 4
# scattering events and one path per pixel per frame.
PATH_HD512 = PathShape(density=0.02, light_dir=(0.26726124, 0.8017837, 0.5345225), light=(3.0, 3.0, 3.0),
                       ambient=(0.25, 0.3, 0.35), max_bounces=4, spp=1, seed=99)


def scaled(w: Workload, width: int, height: int, **kw) -> Workload:
    """Same workload at another resolution (and optional overrides)."""
    return replace(w, width=width, height=height, **kw)


# 16 views of 4 random-init INRs of the 512^3 architecture (seeds 0-3):
# view v shows INR v mod 4 at (256 * 2^(v // 4))^2 pixels, perspective 45
# degrees, orbiting the volume centre at the radius where the bounding sphere
# fills the view; each view has its own orbit (start angle, elevation and
# speed from a generator seeded with 100 + v).  One cache of 16^3 bricks, 4
# LoDs and a shared 32 GiB pool serves all views.
@dataclass
class MultiView:
    name: str = "multiview16_inr512x4"
    arch: InrArch = ARCH_512
    n_views: int = 16
    n_inrs: int = 4
    step: float = 0.5
    lod_scale: float = 1.0 / 800.0
    ert_threshold: float = 0.999
    samples_per_iter: int = 32
    seed: int = 1234
    radius: float = 1159.0
    cache: CacheShape = field(default_factory=lambda: CacheShape(
        brick=16, n_lods=4, pool_bricks=(32 << 30) // (16 ** 3 * 4), max_requests=256, preload_period=4))

    def view_inr(self, v: int) -> int:
        return v % self.n_inrs

    def view_size(self, v: int) -> int:
        return 256 << (v // 4)

    def camera(self, v: int, frame: int) -> synth.Camera:
        import numpy as np
        rng = np.random.default_rng(100 + v)
        start = rng.uniform(0.0, 360.0)
        elev = rng.uniform(-45.0, 45.0)
        speed = rng.uniform(2.0, 8.0)
        n = self.view_size(v)
        return synth.orbit_camera(synth.PERSPECTIVE, self.arch.dims, self.radius, start + speed * frame, elev, n, n,
                                  45.0)

    def tf(self, frame: int):
        return synth.tf_ramp() if (frame % 60) < 30 else synth.tf_iid(77)


MULTIVIEW = MultiView()
