"""Named workloads: synthetic input recipe plus solver parameters.

Images are seeded Voronoi mosaics (see ``synth``) standing in for the
paper's test pictures.  Where the paper gives a value (dt, E, eps0, Armijo
constants, rho, gamma) the library defaults carry it; the sizes, window
radii, step counts and iteration schedules below are this project's choices.
"""
from __future__ import annotations

from dataclasses import dataclass

from .binding import Params
from .synth import voronoi_image


@dataclass(frozen=True)
class Workload:
    name: str
    H: int
    W: int
    C: int
    regions: int
    sigma: float
    seed: int
    gradient_amp: float = 0.0
    spectra: bool = False
    R: int = 2
    K: int = 20
    max_outer: int = 5
    max_inner: int = 50
    tol_alm: float = 0.0
    alpha: float = 3000.0

    def image(self):
        return voronoi_image(self.H, self.W, self.C, self.regions, self.sigma, self.seed,
                             gradient_amp=self.gradient_amp, spectra=self.spectra)

    def params(self, **kw) -> Params:
        p = Params(K=self.K, R=self.R, max_outer=self.max_outer, max_inner=self.max_inner,
                   tol_alm=self.tol_alm, alpha=self.alpha)
        return p.replace(**kw) if kw else p


# 32x32 RGB, 4 regions, sigma 0.05; R=2, 20 steps, 5 multiplier x 50 DAL iterations.
VORONOI32 = Workload("voronoi32_rgb_r2_k20", 32, 32, 3, 4, 0.05, 1001, R=2, K=20, max_outer=5, max_inner=50)

# 512x512 RGB, 12 regions with linear colour gradients (amplitude 0.1), sigma 0.08;
# R=5, 50 steps, run to ALM residual 1e-5 (capped).
VORONOI512 = Workload("voronoi512_rgb_r5_k50", 512, 512, 3, 12, 0.08, 1002, gradient_amp=0.1, R=5, K=50,
                      max_outer=200, max_inner=50, tol_alm=1e-5)

# 2048x2048 with 31 smooth-spectrum channels, 24 regions, sigma 0.05; R=2, 100 steps.
HYPER2048 = Workload("hyperspectral2048_c31_r2_k100", 2048, 2048, 31, 24, 0.05, 1003, spectra=True, R=2, K=100)

ALL = {w.name: w for w in (VORONOI32, VORONOI512, HYPER2048)}


@dataclass(frozen=True)
class BatchWorkload:
    """64 RGB Voronoi images with uneven, non-square sides uniform in [128, 1024],
    4-16 regions, noise sigma uniform in [0.02, 0.1]; the 512 x 512 dynamics
    (R = 5, K = 50) and a fixed 5 x 10 multiplier / DAL schedule."""
    name: str = "batch64_rgb_128to1024_r5_k50"
    n: int = 64
    seed: int = 1004
    C: int = 3
    R: int = 5
    K: int = 50
    max_outer: int = 5
    max_inner: int = 10
    alpha: float = 3000.0

    def specs(self):
        from .synth import batch_shapes
        return batch_shapes(self.n, self.seed)

    def images(self):
        return [voronoi_image(H, W, self.C, reg, sig, s) for (H, W, reg, sig, s) in self.specs()]

    def params(self, **kw) -> Params:
        p = Params(K=self.K, R=self.R, max_outer=self.max_outer, max_inner=self.max_inner, alpha=self.alpha)
        return p.replace(**kw) if kw else p


BATCH64 = BatchWorkload()
