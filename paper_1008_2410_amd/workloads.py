"""Seeded synthetic vortex-particle workloads.

This module only draws inputs: particle positions, circulations, the blob core
sigma and the tree parameters.  It holds none of the FMM's arithmetic, imports
nothing else from this package, and is the one module that both the CPU oracle
tests and the GPU path are fed from.

The vorticity fields follow the paper's test problem (section "Test problem"):
vortex particles carry circulations Gamma_i that discretise a vorticity field
with Gaussian blobs of core sigma (eqs. omega and zeta).

Workloads (sizes fixed by the benchmark configuration list):

  uniform_lamb_oseen   N uniform-random points in [0,1]^2, sigma = 2/sqrt(N),
                       Lamb-Oseen circulations (4096 particles, depth 4, p=10).
  lattice_lamb_oseen   jittered n x n lattice, sigma = 1.5 h (1024^2, depth 8, p=12).
  gaussian_patches     N points from K signed Gaussian vortex patches,
                       sigma = 0.01/64 (2^24 points, 8 patches, depth 10, p=16).
  uniform_target_field N uniform points with a smooth random target velocity
                       field u* (2^20 points, depth 8, p=12), for the loss
                       L = 0.5 * sum |u - u*|^2.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Lamb-Oseen vorticity omega(r) = exp(-r^2/RC2) / (RC2*pi), centred at (0.5, 0.5);
# its total circulation is 1.
LAMB_OSEEN_RC2 = 0.01
LAMB_OSEEN_CENTRE = (0.5, 0.5)


@dataclasses.dataclass
class Workload:
    """One synthetic evaluation problem.

    xy:       (N, 2) float64 particle positions (user order).
    gamma:    (N,) float64 circulations Gamma_i.
    sigma:    Gaussian blob core.
    depth:    uniform quadtree depth L (4^L leaves).
    p:        number of expansion terms (m = 0..p-1).
    root_box: (x0, y0, side) of the root cell, or None for the bounding square.
    precision: "fp64" or "mixed".
    extra:    workload-specific arrays (target field, sample indices, ...).
    """

    name: str
    xy: np.ndarray
    gamma: np.ndarray
    sigma: float
    depth: int
    p: int
    root_box: tuple | None
    precision: str
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])


def lamb_oseen_vorticity(xy: np.ndarray) -> np.ndarray:
    dx = xy[:, 0] - LAMB_OSEEN_CENTRE[0]
    dy = xy[:, 1] - LAMB_OSEEN_CENTRE[1]
    return np.exp(-(dx * dx + dy * dy) / LAMB_OSEEN_RC2) / (LAMB_OSEEN_RC2 * math.pi)


def uniform_lamb_oseen(n: int = 4096, seed: int = 1, depth: int = 4, p: int = 10,
                       precision: str = "fp64") -> Workload:
    """Uniform-random particles in [0,1]^2 with Lamb-Oseen circulations Gamma_i = omega(x_i)/N."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xy = rng.random((n, 2))
    gamma = lamb_oseen_vorticity(xy) / n
    return Workload("uniform_lamb_oseen", xy, gamma, 2.0 / math.sqrt(n), depth, p,
                    (0.0, 0.0, 1.0), precision)


def lattice_lamb_oseen(side: int = 1024, seed: int = 2, depth: int = 8, p: int = 12,
                       jitter: float = 0.25, precision: str = "fp64") -> Workload:
    """side x side lattice with spacing h = 1/side, each point jittered by U(-jitter*h, jitter*h)
    per coordinate; sigma = 1.5 h; Gamma_i = omega(x_i) h^2.  With jitter < 0.5 every
    leaf of a depth-L tree with 4^L <= side^2 holds the same number of particles."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / side
    i, j = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    xy = np.stack([(i.ravel() + 0.5) * h, (j.ravel() + 0.5) * h], axis=1)
    if jitter:
        xy = xy + rng.uniform(-jitter * h, jitter * h, size=xy.shape)
    gamma = lamb_oseen_vorticity(xy) * h * h
    return Workload("lattice_lamb_oseen", xy, gamma, 1.5 * h, depth, p, (0.0, 0.0, 1.0),
                    precision, {"h": h})


def gaussian_patches(n: int = 1 << 24, n_patches: int = 8, seed: int = 3, depth: int = 10,
                     p: int = 16, sigma: float = 0.01 / 64, precision: str = "mixed",
                     n_sample: int = 4096, sample_seed: int = 33) -> Workload:
    """Particles drawn from a mixture of signed Gaussian vortex patches.

    Patch k: centre c_k ~ U[0.1, 0.9]^2, radius R_k ~ U(0.02, 0.1) (the Gaussian's
    standard deviation), sign s_k = +-1, peak vorticity w_k ~ U(1, 5).  Equal
    particle counts per patch, x ~ N(c_k, R_k^2 I).  The vorticity is
    omega(x) = sum_k s_k w_k exp(-|x - c_k|^2 / (2 R_k^2)) and each particle carries
    the Monte-Carlo quadrature weight Gamma_i = omega(x_i) / (N rho(x_i)), where rho
    is the sampling density.  The root cell is the bounding square (root_box None).
    extra["sample"] is a seeded random subsample of target indices for accuracy checks.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.1, 0.9, size=(n_patches, 2))
    radii = rng.uniform(0.02, 0.1, size=n_patches)
    signs = np.where(rng.random(n_patches) < 0.5, -1.0, 1.0)
    peaks = rng.uniform(1.0, 5.0, size=n_patches)
    counts = np.full(n_patches, n // n_patches, dtype=np.int64)
    counts[: n - counts.sum()] += 1
    xy = np.empty((n, 2), dtype=np.float64)
    start = 0
    for k in range(n_patches):
        c = counts[k]
        xy[start:start + c] = centres[k] + radii[k] * rng.standard_normal((c, 2))
        start += c
    # Shuffle so that the user order carries no spatial structure.
    xy = xy[rng.permutation(n)]
    omega = np.zeros(n)
    rho = np.zeros(n)
    for k in range(n_patches):
        r2 = ((xy - centres[k]) ** 2).sum(axis=1)
        gk = np.exp(-r2 / (2.0 * radii[k] ** 2))
        omega += signs[k] * peaks[k] * gk
        rho += (counts[k] / n) * gk / (2.0 * math.pi * radii[k] ** 2)
    gamma = omega / (n * rho)
    srng = np.random.Generator(np.random.PCG64(sample_seed))
    sample = np.sort(srng.choice(n, size=min(n_sample, n), replace=False))
    return Workload("gaussian_patches", xy, gamma, sigma, depth, p, None, precision,
                    {"sample": sample, "centres": centres, "radii": radii, "signs": signs,
                     "peaks": peaks})


def clustered_background(n: int = 1 << 24, n_clusters: int = 8, background: float = 0.5, seed: int = 7,
                         p: int = 16, sigma: float = 3.5e-6, radius=(0.002, 0.005), precision: str = "mixed",
                         n_sample: int = 256, sample_seed: int = 34) -> Workload:
    """An uneven distribution for the adaptive tree: a fraction `background` of the
    particles uniform on [0, 1]^2, the rest in n_clusters equal Gaussian clusters with
    centres ~ U[0.2, 0.8]^2 and standard deviations ~ U(radius).  Circulations
    Gamma_i ~ N(0, 1)/N.  The particle density spans five orders of magnitude, so no
    single uniform depth suits both the background and the cluster cores; sigma is small
    enough that leaves down to depth 15 stay wider than 8 sigma.  Root cell: the bounding
    square.  extra["sample"]: seeded target indices for accuracy checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = int(round(background * n))
    centres = rng.uniform(0.2, 0.8, size=(n_clusters, 2))
    radii = rng.uniform(radius[0], radius[1], size=n_clusters)
    counts = np.full(n_clusters, (n - nb) // n_clusters, dtype=np.int64)
    counts[: n - nb - counts.sum()] += 1
    parts = [rng.random((nb, 2))]
    for k in range(n_clusters):
        parts.append(centres[k] + radii[k] * rng.standard_normal((counts[k], 2)))
    xy = np.concatenate(parts)[rng.permutation(n)]
    gamma = rng.standard_normal(n) / n
    srng = np.random.Generator(np.random.PCG64(sample_seed))
    sample = np.sort(srng.choice(n, size=min(n_sample, n), replace=False))
    return Workload("clustered_background", xy, gamma, sigma, 15, p, None, precision,
                    {"sample": sample, "centres": centres, "radii": radii})


def transport_patches(n: int = 1 << 25, n_patches: int = 16, seed: int = 5, depth: int = 11, p: int = 16,
                      sigma: float = 0.01 / 64, dt: float = 1e-3, steps: int = 5,
                      precision: str = "mixed") -> Workload:
    """The time-stepped workload: Gaussian patches (as gaussian_patches) advected by
    `steps` midpoint-RK2 steps of size dt, every velocity an FMM evaluation over a tree
    rebuilt for the current positions (bounding square).  extra["dt"], extra["steps"];
    extra["target"] is a seeded target field for a loss L = 0.5 |x_N - target|^2."""
    w = gaussian_patches(n=n, n_patches=n_patches, seed=seed, depth=depth, p=p, sigma=sigma, precision=precision)
    w.name = "transport_patches"
    w.extra.update(dt=dt, steps=steps)
    return w


def smooth_target_field(xy: np.ndarray, seed: int = 44, n_modes: int = 16) -> np.ndarray:
    """u* = (d psi/dy, -d psi/dx) of the random stream function
    psi = sum_m A_m cos(2 pi k_m . x + phi_m), k_m in Z^2 with 1 <= |k_m|_inf <= 3,
    A_m ~ N(0,1)/(8 pi |k_m|), phi_m ~ U(0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(-3, 4, size=2)
        if np.abs(k).max() >= 1:
            ks.append(k)
    ks = np.array(ks, dtype=np.float64)
    amp = rng.standard_normal(n_modes) / (8.0 * math.pi * np.linalg.norm(ks, axis=1))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    u = np.zeros(xy.shape[0])
    v = np.zeros(xy.shape[0])
    for m in range(n_modes):
        arg = 2.0 * math.pi * (xy @ ks[m]) + phase[m]
        s = -amp[m] * np.sin(arg) * 2.0 * math.pi
        u += s * ks[m, 1]   # d psi / dy
        v -= s * ks[m, 0]   # -d psi / dx
    return np.stack([u, v], axis=1)


def uniform_target_field(n: int = 1 << 20, seed: int = 4, depth: int = 8, p: int = 12,
                         precision: str = "mixed", target_seed: int = 44,
                         fd_seed: int = 45, n_fd: int = 64) -> Workload:
    """Uniform particles in [0,1]^2, sigma = 2/sqrt(N), Lamb-Oseen circulations, a smooth
    target field u*, and a seeded choice of coordinates for finite-difference checks
    (half circulations, half evaluation positions)."""
    w = uniform_lamb_oseen(n=n, seed=seed, depth=depth, p=p, precision=precision)
    w.name = "uniform_target_field"
    w.extra["u_target"] = smooth_target_field(w.xy, seed=target_seed)
    frng = np.random.Generator(np.random.PCG64(fd_seed))
    w.extra["fd_gamma_idx"] = frng.choice(n, size=n_fd // 2, replace=False)
    w.extra["fd_x_idx"] = frng.choice(n, size=n_fd // 2, replace=False)
    w.extra["fd_x_comp"] = frng.integers(0, 2, size=n_fd // 2)
    return w


def by_name(name: str, **kw) -> Workload:
    return {
        "uniform_lamb_oseen": uniform_lamb_oseen,
        "lattice_lamb_oseen": lattice_lamb_oseen,
        "gaussian_patches": gaussian_patches,
        "uniform_target_field": uniform_target_field,
    }[name](**kw)
