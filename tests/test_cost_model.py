"""The complexity model against the numbers the paper prints, and the one-GPU fit on
synthetic stage times."""
import json
import math
import os

import numpy as np

from paper_1008_2410_amd import costmodel as cm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cost_model_paper.json")


def test_paper_numbers():
    """Section "Concurrency": B_opt ~= 18 for t = 15, the cover coefficient 215.22, B >= 14.30
    for N = 1e6, P = 1e4 (L_root = log_4 P), and M >= 12 log_4 P at B = 18."""
    g = json.load(open(GOLDEN))
    t = g["t"]
    assert round(cm.paper_b_opt(t)) == g["B_opt_approx"]
    assert round(cm.paper_cover_coefficient(t), 2) == g["cover_coefficient"]
    ex = g["example"]
    assert round(cm.paper_min_b(ex["N"], ex["P"], t), 2) == ex["B_min"]
    ms = g["memory_scalable"]
    coef = cm.paper_min_particles_per_process(4.0, t, ms["B"])  # log_4 4 = 1
    assert round(coef) == ms["M_coefficient_approx"]


def test_paper_b_opt_minimises_the_model():
    t, N, P = 15, 1e6, 1e4
    b = cm.paper_b_opt(t)
    T0 = cm.paper_time(N, b, P, t)
    for f in (0.8, 0.95, 1.05, 1.25):
        assert cm.paper_time(N, b * f, P, t) > T0


def test_fit_recovers_synthetic_constants():
    truth = dict(a=2e-8, b=4e-4, c=3e-6, d=2.5e-10, far0=0.02, part0=0.01, near0=0.03, g=2e-7, h=0.01)
    rng = np.random.Generator(np.random.PCG64(0))
    samples = []
    for n in (1 << 20, 1 << 22):
        for L in range(5, 11):
            for lc in (2, 3, 4):
                B = n / 4 ** L
                pairs = int(9 * n * B * rng.uniform(0.8, 1.0))
                cells = int((4 ** (L + 1) - 4 ** (lc + 1)) / 3 * rng.uniform(0.9, 1.0))
                coarse = int((4 ** (lc + 1) - 16) / 3 * rng.uniform(0.9, 1.0))
                leaves = int(min(n, 4 ** L) * rng.uniform(0.9, 1.0))
                samples.append(cm.Sample(n, L, lc, pairs, cells,
                                         truth["part0"] + truth["a"] * n,
                                         truth["far0"] + truth["c"] * cells + truth["b"] * coarse + truth["h"] * (L - lc),
                                         truth["near0"] + truth["d"] * pairs + truth["g"] * 9 * leaves,
                                         coarse_cells=coarse, leaves=leaves))
    f = cm.fit(samples)
    for k, v in truth.items():
        assert math.isclose(getattr(f, k), v, rel_tol=1e-6, abs_tol=1e-12), (k, getattr(f, k), v)
    assert math.isclose(f.b_opt_uniform(), math.sqrt(4 * truth["c"] / (27 * truth["d"])), rel_tol=1e-6)
