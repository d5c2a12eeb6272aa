"""The complexity model of section "Complexity Estimates" and section "Concurrency",
and its fit to measured stage times on one GPU.

Paper model (eq. complexity, Table tab:coeff), for N particles, B per finest-level box,
P processes, flop rate r and expansion order t:

    T = a N/P + b log_4 P + c N/(B P) + d N B/P,
    a = (16 t - 15)/r,  b = (84 - 48 t + 571 t^2)/(3 r),
    c = (128 - 48 t + 844 t^2)/(3 r),  d = 198/r.

Minimising T over B gives B_opt = sqrt(c/d); the coarse-level work b L_root is hidden
behind the direct work d N B/P when B >= (b/d) P L_root / N (the cover condition).

On one GPU the same terms are the measured stages of an evaluation, each timed alone
(serial schedule), with the counts a GPU launch actually pays for:
    per particle (pack, finalize):                    T_part = a_g N
    far field: per fine-level cell (M2M, M2L, L2L
    above L_c), per cell of the single-workgroup
    coarse sweep (levels <= L_c; the paper's b term),
    per fine level (launches):                        T_far = c_g C_fine + b_g C_coarse + h_g (L - L_c)
    near field: per pair, per leaf visit (a 64-lane
    wavefront visiting a neighbour leaf, staging it):  T_near = d_g pairs + g_g 9 N_leaves
For a uniform distribution, pairs ~= 9 N B and C_fine ~= (4/3) N/B, so the per-particle
cost (4/3) c_g/B + 9 d_g B is smallest at B_opt = sqrt(4 c_g/(27 d_g)); the coarse
sweep is covered by the near field when T_near >= b_g C_coarse.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# --- the paper's model --------------------------------------------------------------------

def paper_coefficients(t: int, r: float = 1.0) -> dict:
    """Table tab:coeff: a, b, c, d for expansion order t and flop rate r."""
    return {
        "a": (16 * t - 15) / r,
        "b": (84 - 48 * t + 571 * t * t) / (3 * r),
        "c": (128 - 48 * t + 844 * t * t) / (3 * r),
        "d": 198 / r,
    }


def paper_time(N: float, B: float, P: float, t: int, r: float = 1.0) -> float:
    """Eq. complexity without the lower-order term e(N, P)."""
    k = paper_coefficients(t, r)
    return k["a"] * N / P + k["b"] * math.log(P, 4) + k["c"] * N / (B * P) + k["d"] * N * B / P


def paper_b_opt(t: int) -> float:
    """B_opt = sqrt(c/d) of section "Concurrency"."""
    k = paper_coefficients(t)
    return math.sqrt(k["c"] / k["d"])


def paper_cover_coefficient(t: int) -> float:
    """b/d: the cover condition reads B >= (b/d) P L_root / N."""
    k = paper_coefficients(t)
    return k["b"] / k["d"]


def paper_min_b(N: float, P: float, t: int, L_root: float | None = None) -> float:
    """Smallest B that hides the coarse work, with L_root = log_4 P unless given."""
    L_root = math.log(P, 4) if L_root is None else L_root
    return paper_cover_coefficient(t) * P * L_root / N


def paper_min_particles_per_process(P: float, t: int, B: float) -> float:
    """N/P = M >= (b/d) log_4 P / B: the memory-scalable form at fixed B."""
    return paper_cover_coefficient(t) * math.log(P, 4) / B


# --- the one-GPU fit -----------------------------------------------------------------------

@dataclass
class Sample:
    """One measured evaluation: sizes and stage times (ms) with the stages run serially."""
    n: int
    depth: int
    lc: int
    pairs: int
    fine_cells: int
    t_part: float
    t_far: float
    t_near: float
    t_overlap: float | None = None   # the whole call with the two-stream schedule
    coarse_cells: int = 0
    leaves: int = 0                  # non-empty leaves


@dataclass
class Fit:
    a: float   # ms per particle
    b: float   # ms per coarse-level cell (single-workgroup sweep)
    c: float   # ms per non-empty fine-level cell
    d: float   # ms per near-field pair
    far0: float
    part0: float
    near0: float
    g: float = 0.0   # ms per near-field leaf visit
    h: float = 0.0   # ms per fine level

    def near(self, pairs: float, leaves: float) -> float:
        return self.near0 + self.d * pairs + self.g * 9.0 * leaves

    def far(self, fine_cells: float, coarse_cells: float, fine_levels: float) -> float:
        return self.far0 + self.c * fine_cells + self.b * coarse_cells + self.h * fine_levels

    def predict(self, s: Sample) -> dict:
        part = self.part0 + self.a * s.n
        far = self.far(s.fine_cells, s.coarse_cells, s.depth - s.lc)
        near = self.near(s.pairs, s.leaves)
        return {"part": part, "far": far, "near": near, "serial": part + far + near}

    def b_opt_uniform(self) -> float:
        """B minimising (4/3) c_g N/B + 9 d_g N B (uniform distribution)."""
        return math.sqrt(4.0 * self.c / (27.0 * self.d))

    def coarse_ms(self, s: Sample) -> float:
        """The single-workgroup coarse sweep (the b term) of a sample."""
        return self.b * s.coarse_cells

    def covered(self, s: Sample) -> bool:
        """Cover condition on one GPU: the near field lasts at least as long as the coarse sweep."""
        return self.near(s.pairs, s.leaves) >= self.coarse_ms(s)

    def uniform_sample(self, n: int, L: int, lc: int) -> Sample:
        """Counts of a uniform distribution filling every cell (interior approximation)."""
        B = n / 4.0 ** L
        return Sample(n=n, depth=L, lc=lc, pairs=int(9 * n * B), fine_cells=int((4.0 ** (L + 1) - 4.0 ** (lc + 1)) / 3.0),
                      t_part=0, t_far=0, t_near=0, coarse_cells=int((4.0 ** (lc + 1) - 16) / 3.0),
                      leaves=int(min(n, 4 ** L)))

    def best_depth(self, n: int, lc: int, depths) -> int:
        """Depth minimising the predicted serial time of a uniform distribution."""
        return min(depths, key=lambda L: self.predict(self.uniform_sample(n, L, lc))["serial"])


def fit(samples: list[Sample]) -> Fit:
    """Least-squares fit of the three stage models (each with an intercept)."""
    n = np.array([s.n for s in samples], dtype=float)
    part = np.array([s.t_part for s in samples])
    A = np.stack([np.ones_like(n), n], axis=1)
    (part0, a), *_ = np.linalg.lstsq(A, part, rcond=None)
    cells = np.array([s.fine_cells for s in samples], dtype=float)
    coarse = np.array([s.coarse_cells for s in samples], dtype=float)
    lev = np.array([s.depth - s.lc for s in samples], dtype=float)
    far = np.array([s.t_far for s in samples])
    A = np.stack([np.ones_like(cells), cells, coarse, lev], axis=1)
    (far0, c, b, h), *_ = np.linalg.lstsq(A, far, rcond=None)
    pairs = np.array([s.pairs for s in samples], dtype=float)
    leaves = np.array([s.leaves for s in samples], dtype=float)
    near = np.array([s.t_near for s in samples])
    A = np.stack([np.ones_like(pairs), pairs, 9.0 * leaves], axis=1)
    (near0, d, g), *_ = np.linalg.lstsq(A, near, rcond=None)
    return Fit(a=float(a), b=float(b), c=float(c), d=float(d), far0=float(far0), part0=float(part0),
               near0=float(near0), g=float(g), h=float(h))


def fine_cells(counts_per_level: list[int], lc: int) -> int:
    """Non-empty cells of the levels handled per cell (lc + 1 .. L)."""
    return int(sum(counts_per_level[l] for l in range(lc + 1, len(counts_per_level))))


def coarse_cells(counts_per_level: list[int], lc: int) -> int:
    """Non-empty cells of the levels of the single-workgroup sweep (2 .. lc)."""
    return int(sum(counts_per_level[l] for l in range(2, min(lc, len(counts_per_level) - 1) + 1)))
