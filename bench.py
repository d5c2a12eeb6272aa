"""Benchmark: FMM velocity evaluation throughput on one MI355X.

Workload: 2^24 particles drawn from 8 signed Gaussian vortex patches, blob core
sigma = 0.01/64, uniform quadtree depth 10 over the bounding square, p = 16 terms,
mixed precision (FP32 near field and fine-level far field, FP64 coarse levels and
final sum), coarse levels overlapped with the near field on a second HIP stream.
A step is one fmm_velocity call (stages 4-10) with the particles, circulations and
tree already resident in HBM; the tree build (stages 1-3) is outside the timed
region.

Prints one JSON line (see the README of the repository root for the fields).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

# Published MI355X peaks used for the roofline fractions.
PEAK_FP32_VECTOR_TFLOPS = 157.3   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
PEAK_FP64_VECTOR_TFLOPS = 78.6    # the same without the packed dual issue
# The FP32 rate the kernels can issue: the build switches packed FP32 off, so one FMA per lane
# per cycle, 256 x 4 x 16 x 2 x 2.4 GHz.
ISSUABLE_FP32_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic flops per ordered (target, source) pair of the near-field sum, section
# "Complexity Estimates" (a complex division and an exponential).
P2P_FLOPS_PER_PAIR = 22
# HBM traffic of the near-field kernel comes from the rocprofv3 --pmc summary under
# profiles/, which records the hash of the kernel sources it was taken with; the line
# reports it only while the sources still hash the same.
PROFILE_WITH_TRAFFIC = os.path.join(HERE, "profiles", "p2p_near_gaussian_patches_16M.md")
KERNEL_SOURCES = ("paper_1008_2410_amd/csrc/kernels.hip", "paper_1008_2410_amd/csrc/device_common.h")


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str):
    """(bytes per launch, note) of `kernel` from the profile summary's machine-readable
    traffic lines, or (None, reason) when absent or taken with other kernel sources."""
    try:
        with open(PROFILE_WITH_TRAFFIC) as f:
            lines = [ln for ln in f if ln.startswith("<!-- traffic ")]
    except OSError:
        return None, "no profile summary"
    cur = kernel_sources_hash()
    for ln in lines:
        rec = json.loads(ln[len("<!-- traffic "):].rsplit("-->", 1)[0])
        if rec.get("kernel") != kernel:
            continue
        if rec.get("sources") != cur:
            return None, f"kernel sources changed since the counters were taken ({rec.get('sources')} -> {cur})"
        return rec["bytes"], f"rocprofv3 --pmc FETCH_SIZE/WRITE_SIZE, sources {cur}"
    return None, "no counter record for this kernel"


def p2p_roofline(kernel: str, pairs: int, plan: dict, ms: float, peak: float, issuable: float):
    """Roofline of the near-field kernel: the paper's 22 flops per ordered pair against the
    published vector peak (the algorithmic fraction), and the evaluations the kernel really
    performs (each unordered pair of the mutual form once, each ordered pair of the
    target-centric form once) at 22 flops against the rate the build can issue."""
    evals = plan["mutual_pairs"] // 2 + (pairs - plan["mutual_pairs"])
    achieved = P2P_FLOPS_PER_PAIR * pairs / (ms * 1e-3) / 1e12
    executed = P2P_FLOPS_PER_PAIR * evals / (ms * 1e-3) / 1e12
    traffic, note = profiled_traffic(kernel)
    return {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic, "traffic_source": note,
            "flops_per_pair": P2P_FLOPS_PER_PAIR, "pairs_per_launch": pairs, "avg_launch_ms": round(ms, 4),
            "executed": {"evaluations_per_launch": evals, "evaluations_per_s": round(evals / (ms * 1e-3), 1),
                         "achieved": round(executed, 3), "peak": issuable, "frac": round(executed / issuable, 4),
                         "note": "mutual form counted once per unordered pair; peak = non-packed issue rate"}}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def adjoint_only_leg(torch, dev, tree, w, gamma, info, args):
    """The adjoint of the headline configuration alone (mixed, dL/dGamma and dL/dx_eval for a
    seeded cotangent): warm-up calls, then `steps` timed calls with the stage events, and the
    rate of the adjoint near field (target-centric: every ordered near pair evaluated once,
    about 19 VALU operations and two transcendentals each)."""
    from paper_1008_2410_amd import _lib
    dl = torch.empty((w.n, 2), dtype=torch.float64, device=dev).normal_(generator=torch.Generator(dev).manual_seed(0))
    for _ in range(args.warmup):
        tree.velocity_backward(gamma, w.sigma, w.p, "mixed", dl)
    tree.set_option(_lib.FMM_OPT_TIMING, 1)
    tree.timings()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        tree.velocity_backward(gamma, w.sigma, w.p, "mixed", dl)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    st = tree.timings()
    tree.set_option(_lib.FMM_OPT_TIMING, 0)
    stages = {k: round(v / st["calls"], 4) for k, v in st.items() if k != "calls"}
    pairs = info["p2p_pairs"]
    print(json.dumps({"adjoint": "mixed", "ms_per_step": round(ms, 4), "stages_ms": stages,
                      "near_kernel": "p2p_backward_kernel<float, false>", "pairs_per_launch": pairs,
                      "pair_evaluations_per_s": round(pairs / (stages["p2p"] * 1e-3), 1),
                      "kernel_sources": kernel_sources_hash(), "steps": args.steps, "warmup": args.warmup}),
          flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cpu_baseline_leg(w, sample_frac_log4=0):
    """The CPU oracle on the machine's host cores: (1) accuracy gate of the GPU result on the
    4096-particle subsample, (2) throughput of the oracle's full FMM (stages 1-10) on the
    benchmark workload itself (k = 0: all N particles at depth L, about a minute on 16
    threads), or with k > 0 on the first N/4^k particles of the (shuffled) draw with the tree
    depth lowered by k, which keeps the particles per leaf of the full problem."""
    import oracle
    oracle.build()
    idx = w.extra["sample"]
    t0 = time.perf_counter()
    ref = oracle.fmm_velocity(w.xy, w.gamma, w.sigma, w.depth, w.p, None, targets=w.xy[idx])
    t_gate = time.perf_counter() - t0
    k = sample_frac_log4
    ns = w.n >> (2 * k)
    xs, gs = w.xy[:ns], w.gamma[:ns]
    t0 = time.perf_counter()
    oracle.fmm_velocity(xs, gs, w.sigma, w.depth - k, w.p, None)
    t_run = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return ref, t_gate, {
        "value": ns / t_run / 1e6,
        "unit": "Mparticles/s",
        "cores": threads,
        "host_cpus": os.cpu_count(),
        "cpu_model": model,
        "kind": "oracle",
        "sample": (f"oracle FMM stages 1-10 (FP64 C, OpenMP) on the whole workload: N = {ns}, depth {w.depth}, "
                   f"p={w.p}; {t_run:.2f} s" if k == 0 else
                   f"oracle FMM stages 1-10 (FP64 C, OpenMP) on the first {ns} particles of the same draw, "
                   f"depth {w.depth - k}, p={w.p} (same particles per leaf); {t_run:.2f} s"),
    }


def lattice_overlap_leg(torch, dev, workloads, steps):
    """The jittered 1024^2 lattice as configured (FP64, depth 8, p = 12, coarse levels <= 5
    in the one-workgroup kernel on the second stream): the evaluation overlapped and
    serialised, and the overlap fraction (T_P2P + T_far - T_both) / min(T_P2P, T_far) from
    the serialised stage times and the overlapped span between the pack and final stages."""
    from paper_1008_2410_amd import _lib, fmm
    w = workloads.lattice_lamb_oseen()
    xy = torch.from_numpy(w.xy).to(dev)
    g = torch.from_numpy(w.gamma).to(dev)
    tree = fmm.Tree(xy, w.depth, w.root_box)
    tree.set_option(_lib.FMM_OPT_COARSE_LEVEL, 5)
    out = torch.empty((w.n, 2), dtype=torch.float64, device=dev)
    res = {}
    for sched in (0, 1):  # concurrent, then serialised
        tree.set_option(_lib.FMM_OPT_SCHEDULE, sched)
        for _ in range(3):
            tree.velocity(g, w.sigma, w.p, "fp64", out=out)
        # the calls timed as a whole, without the stage events (eight per call), then the
        # same number of calls with them for the stage times
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            tree.velocity(g, w.sigma, w.p, "fp64", out=out)
        e1.record()
        torch.cuda.synchronize()
        tree.set_option(_lib.FMM_OPT_TIMING, 1)
        tree.timings()
        for _ in range(steps):
            tree.velocity(g, w.sigma, w.p, "fp64", out=out)
        torch.cuda.synchronize()
        st = tree.timings()
        tree.set_option(_lib.FMM_OPT_TIMING, 0)
        res[sched] = (e0.elapsed_time(e1) / steps, {k: v / st["calls"] for k, v in st.items() if k != "calls"})
    tree.close()
    (ms_o, st_o), (ms_s, st_s) = res[0], res[1]
    both = st_o["total"] - st_o["pack"] - st_o["final"]
    frac = (st_s["p2p"] + st_s["far"] - both) / min(st_s["p2p"], st_s["far"])
    log(f"[bench] lattice fp64 L_c=5: overlap {ms_o:.3f} ms, serial {ms_s:.3f} ms, near {st_s['p2p']:.3f} ms, "
        f"far {st_s['far']:.3f} ms, overlap fraction {frac:.3f}")
    return {"workload": "lattice_lamb_oseen", "n": w.n, "depth": w.depth, "p": w.p, "precision": "fp64",
            "coarse_level": 5, "ms_per_step": round(ms_o, 4), "serial_ms_per_step": round(ms_s, 4),
            "mparticles_per_s": round(w.n / (ms_o * 1e-3) / 1e6, 1), "near_ms_serial": round(st_s["p2p"], 4),
            "far_ms_serial": round(st_s["far"], 4), "overlap_fraction": round(frac, 4)}


def cost_model_leg(torch, dev, workloads):
    """Sweep of depth L and coarse cutoff L_c over uniform particles (p = 16, mixed):
    each point timed with the stages serialised (per-stage times) and with the two-stream
    schedule; the paper's four terms are fitted to the stage times and used to choose the
    depth and check the cover condition against the measured overlap."""
    from paper_1008_2410_amd import _lib, costmodel, fmm
    samples, points = [], []
    for n, depths in ((1 << 20, range(5, 10)), (1 << 22, range(6, 11))):
        w = workloads.uniform_lamb_oseen(n=n, seed=4, depth=8, p=16)
        xy = torch.from_numpy(w.xy).to(dev)
        g = torch.from_numpy(w.gamma).to(dev)
        for L in depths:
            tree = fmm.Tree(xy, L, w.root_box)
            info, levels = tree.info(), tree.levels()
            out = torch.empty((n, 2), dtype=torch.float64, device=dev)
            for lc in (2, 3, 4, 5):
                if lc > L:
                    continue
                tree.set_option(_lib.FMM_OPT_COARSE_LEVEL, lc)
                res = {}
                for sched in (1, 0):  # serialised, then concurrent
                    tree.set_option(_lib.FMM_OPT_SCHEDULE, sched)
                    for _ in range(2):
                        tree.velocity(g, w.sigma, w.p, "mixed", out=out)
                    tree.set_option(_lib.FMM_OPT_TIMING, 1)
                    tree.timings()
                    k = 5
                    for _ in range(k):
                        tree.velocity(g, w.sigma, w.p, "mixed", out=out)
                    torch.cuda.synchronize()
                    st = tree.timings()
                    tree.set_option(_lib.FMM_OPT_TIMING, 0)
                    res[sched] = {a: v / st["calls"] for a, v in st.items() if a != "calls"}
                ser, ovl = res[1], res[0]
                s = costmodel.Sample(n=n, depth=L, lc=lc, pairs=info["p2p_pairs"],
                                     fine_cells=costmodel.fine_cells(levels, lc),
                                     t_part=ser["pack"] + ser["final"], t_far=ser["far"], t_near=ser["p2p"],
                                     t_overlap=ovl["total"], coarse_cells=costmodel.coarse_cells(levels, lc),
                                     leaves=info["nonempty_leaves"])
                samples.append(s)
                both = ovl["total"] - ovl["pack"] - ovl["final"]
                overlap = (ser["p2p"] + ser["far"] - both) / min(ser["p2p"], ser["far"])
                points.append({"n": n, "depth": L, "lc": lc, "B": round(n / 4 ** L, 2), "serial_ms": round(ser["total"], 4),
                               "overlap_ms": round(ovl["total"], 4), "near_ms": round(ser["p2p"], 4),
                               "far_ms": round(ser["far"], 4), "part_ms": round(ser["pack"] + ser["final"], 4),
                               "overlap_fraction": round(overlap, 3)})
                log(f"[bench] cost model n={n} L={L} lc={lc}: {points[-1]}")
            tree.close()
    f = costmodel.fit(samples)
    errs = []
    for s, pt in zip(samples, points):
        pr = f.predict(s)
        pt["predicted_serial_ms"] = round(pr["serial"], 4)
        pt["coarse_ms_model"] = round(f.coarse_ms(s), 4)
        pt["covered"] = f.covered(s)
        errs.append(abs(pr["serial"] - pt["serial_ms"]) / pt["serial_ms"])
    best = {}
    for n in (1 << 20, 1 << 22):
        pts = [p for p in points if p["n"] == n]
        meas = min(pts, key=lambda p: p["serial_ms"])
        sel = min(zip(samples, points), key=lambda sp: f.predict(sp[0])["serial"] if sp[1]["n"] == n else 1e30)[1]
        best[str(n)] = {"measured_serial": {"depth": meas["depth"], "lc": meas["lc"], "ms": meas["serial_ms"]},
                        "predicted_serial": {"depth": sel["depth"], "lc": sel["lc"], "ms_measured": sel["serial_ms"]},
                        "uniform_model_depth": f.best_depth(n, meas["lc"], sorted({p["depth"] for p in pts})),
                        "measured_overlap_best": min(pts, key=lambda p: p["overlap_ms"])["overlap_ms"]}
    print(json.dumps({
        "cost_model": {"a_ns_per_particle": f.a * 1e6, "b_ns_per_coarse_cell": f.b * 1e6,
                       "c_ns_per_fine_cell": f.c * 1e6, "d_ps_per_pair": f.d * 1e9,
                       "g_ns_per_leaf_visit": f.g * 1e6, "h_us_per_fine_level": f.h * 1e3,
                       "intercepts_ms": {"part": f.part0, "far": f.far0, "near": f.near0},
                       "B_opt_uniform": round(f.b_opt_uniform(), 2),
                       "paper_B_opt_t15": round(costmodel.paper_b_opt(15), 2),
                       "max_rel_err_serial": round(max(errs), 4)},
        "best": best, "points": points}), flush=True)


def rk2_leg(torch, dev, workloads, adaptive=False):
    """Time-stepped workload: forward transport and its discrete adjoint (per-step
    checkpoints), with tree builds, velocity evaluations and adjoint calls timed
    separately, and the peak of device memory in use (hipMemGetInfo, all allocations).
    adaptive: the clustered workload (2^24 particles) with an adaptive tree (leaves of at
    most 64 particles, depth <= 15) built for every evaluation, instead of the 2^25-particle
    patches with the uniform depth-11 tree."""
    from paper_1008_2410_amd import fmm, rk2
    t0 = time.perf_counter()
    if adaptive:
        w = workloads.clustered_background()
        dt, steps, atree = 1e-3, 5, (64, 15)
    else:
        w = workloads.transport_patches()
        dt, steps, atree = w.extra["dt"], w.extra["steps"], None
    target = workloads.smooth_target_field(w.xy, seed=55)
    log(f"[bench] transport workload {w.name}: N={w.n} depth={w.depth} adaptive={atree} p={w.p} dt={dt} "
        f"steps={steps} ({time.perf_counter() - t0:.1f} s)")
    xy = torch.from_numpy(w.xy).to(dev)
    gamma = torch.from_numpy(w.gamma).to(dev)
    tgt = torch.from_numpy(target).to(dev)
    # warm-up: one evaluation (library load, tables, first-use allocations)
    tree = fmm.ATree(xy, *atree) if adaptive else fmm.Tree(xy, w.depth, None)
    tree.velocity(gamma, w.sigma, w.p, "mixed")
    tree.close()
    del tree
    torch.cuda.synchronize()
    sf = rk2.RK2Stats()
    t0 = time.perf_counter()
    xN, ck = rk2.rk2_forward(xy, gamma, w.sigma, w.depth, w.p, dt, steps, "mixed", None, sf, adaptive=atree)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    log(f"[bench] rk2 forward {t_fwd:.2f} s: tree builds {sf.tree_build:.2f} s, velocities {sf.velocity:.3f} s "
        f"({sf.evals} evaluations)")
    sb = rk2.RK2Stats()
    t0 = time.perf_counter()
    dx0, dg = rk2.rk2_backward(ck, gamma, w.sigma, w.depth, w.p, dt, xN - tgt, "mixed", None, sb, adaptive=atree)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    log(f"[bench] rk2 adjoint {t_bwd:.2f} s: tree builds {sb.tree_build:.2f} s, velocities {sb.velocity:.3f} s, "
        f"adjoint calls {sb.backward:.3f} s ({sb.vjps})")
    peak = max(sf.peak_bytes, sb.peak_bytes)
    torch_at_peak = sf.torch_reserved_bytes if sf.peak_bytes >= sb.peak_bytes else sb.torch_reserved_bytes
    evals = sf.evals
    print(json.dumps({
        "workload": w.name, "n": w.n, "tree": ({"adaptive": {"max_leaf": atree[0], "max_depth": atree[1]}}
                                              if adaptive else {"uniform_depth": w.depth}),
        "p": w.p, "dt": dt, "steps": steps,
        "precision": "mixed", "fwd_s": round(t_fwd, 3), "bwd_s": round(t_bwd, 3),
        "fwd_tree_build_s": round(sf.tree_build, 3), "fwd_velocity_s": round(sf.velocity, 4),
        "velocity_ms_per_eval": round(sf.velocity / evals * 1e3, 3),
        "velocity_mparticles_per_s": round(w.n * evals / sf.velocity / 1e6, 1),
        "tree_build_ms_per_eval": round(sf.tree_build / evals * 1e3, 2),
        "bwd_tree_build_s": round(sb.tree_build, 3), "bwd_recompute_velocity_s": round(sb.velocity, 4),
        "bwd_adjoint_s": round(sb.backward, 4),
        "adjoint_ms_per_vjp": round(sb.backward / sb.vjps * 1e3, 3),
        "bwd_fwd_device": round(sb.backward / sf.velocity, 3),
        "peak_hbm_gb": round(peak / 1e9, 2),
        "peak_torch_reserved_gb": round(torch_at_peak / 1e9, 2),
        "grad_norms": {"x0": float(torch.linalg.norm(dx0)), "gamma": float(torch.linalg.norm(dg))},
    }), flush=True)


def adaptive_leg(torch, dev, workloads):
    """Uneven distributions: the adaptive tree (leaves capped at max_leaf particles) against
    the uniform tree at several depths, on the 2^24-particle patch workload (depth <= 10,
    every leaf wider than 8 sigma) and on a clustered workload with a uniform background
    (density range 1e5).  Per tree: build time (both trees built on the device; host clock
    around the synchronised build), the mixed evaluation's device time, near-field pairs,
    and the error against the direct sum on sampled particles; for the adaptive tree also
    the adjoint's device time (all three outputs, the source positions included).  One JSON
    line of its own."""
    import oracle
    from paper_1008_2410_amd import fmm
    oracle.build()

    def dev_ms(fn, k):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    result = {"metric": "ms per mixed velocity evaluation, adaptive vs uniform tree", "unit": "ms",
              "higher_is_better": False, "workloads": []}
    cases = ((workloads.gaussian_patches(), (9, 10), ((32, 10), (64, 10), (128, 10), (256, 10))),
             (workloads.clustered_background(), (11, 12), ((32, 15), (64, 15), (128, 15), (256, 15))))
    for w, depths, cfgs in cases:
        xy = torch.from_numpy(w.xy).to(dev)
        g = torch.from_numpy(w.gamma).to(dev)
        out = torch.empty((w.n, 2), dtype=torch.float64, device=dev)
        idx = w.extra["sample"][:256]
        t0 = time.perf_counter()
        ref = oracle.direct(w.xy, w.gamma, w.sigma, targets=w.xy[idx])
        log(f"[adaptive] {w.name}: direct sum on {len(idx)} particles in {time.perf_counter() - t0:.1f} s")
        rows = []
        for kind, a, b in [("uniform", d, None) for d in depths] + [("adaptive", s, l) for s, l in cfgs]:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tree = fmm.Tree(xy, a, None) if kind == "uniform" else fmm.ATree(xy, a, b)
            torch.cuda.synchronize()
            t_build = time.perf_counter() - t0
            info = tree.info()
            ms = dev_ms(lambda: tree.velocity(g, w.sigma, w.p, "mixed", out=out), 5)
            bwd_ms = None
            if kind == "adaptive":
                dl = torch.ones((w.n, 2), dtype=torch.float64, device=dev)
                bwd_ms = dev_ms(lambda: tree.velocity_backward(g, w.sigma, w.p, "mixed", dl, need_src=True), 3)
            err = rel_l2(out.cpu().numpy()[idx], ref)
            row = {"tree": kind, "build_ms": round(1e3 * t_build, 2), "ms": round(ms, 3), "rel_l2_vs_direct": float(f"{err:.3e}"),
                   "p2p_pairs": info["p2p_pairs"]}
            if kind == "uniform":
                row["depth"] = a
            else:
                row.update(max_leaf=a, max_depth=b, cells=info["cells"], leaves=info["leaves"], deepest=info["deepest"],
                           v=info["v"], w=info["w"], bwd_ms=round(bwd_ms, 3), bwd_fwd=round(bwd_ms / ms, 2))
            log(f"[adaptive] {w.name}: {row}")
            rows.append(row)
            tree.close()
        ok = [r for r in rows if r["rel_l2_vs_direct"] <= 1e-5]
        best_u = min((r for r in ok if r["tree"] == "uniform"), key=lambda r: r["ms"], default=None)
        best_a = min((r for r in ok if r["tree"] == "adaptive"), key=lambda r: r["ms"], default=None)
        result["workloads"].append({
            "workload": w.name, "n": w.n, "sigma": w.sigma, "p": w.p, "trees": rows,
            "best_uniform_ms": best_u and best_u["ms"], "best_adaptive_ms": best_a and best_a["ms"],
            "speedup_at_1e-5": round(best_u["ms"] / best_a["ms"], 3) if best_u and best_a else None})
        del xy, g, out
        torch.cuda.empty_cache()
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--depth", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-sample-log4", type=int, default=0,
                    help="CPU oracle leg on the first N/4^k particles at depth L-k (default 0: the whole workload)")
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--bwd-steps", type=int, default=3)
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the timed adjoint of the headline configuration (mixed; dL/dGamma and dL/dx_eval), "
                         "for kernel profiling of exactly that work")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed headline region (for kernel profiling of exactly that work)")
    ap.add_argument("--headline-precision", choices=["mixed", "fp64"], default="mixed",
                    help="with --headline-only: the precision of the timed evaluations (fp64: the FP64 leg's "
                         "near-field kernel, for its counters)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run only a device-to-device copy of MIB MiB ten times (HBM counter calibration)")
    ap.add_argument("--cost-model", action="store_true",
                    help="only the cost-model sweep (uniform particles, depth and coarse-level sweep, fit of the "
                         "paper's complexity terms to the measured stages): one JSON line of its own")
    ap.add_argument("--rk2", action="store_true",
                    help="only the time-stepped workload (2^25 particles, 16 patches, 5 midpoint-RK2 steps, trees "
                         "rebuilt per evaluation): forward and adjoint, one JSON line of its own")
    ap.add_argument("--rk2-adaptive", action="store_true",
                    help="only the time-stepped workload on the clustered distribution (2^24 particles) with an "
                         "adaptive tree built per evaluation: forward and adjoint, one JSON line of its own")
    ap.add_argument("--lattice", action="store_true",
                    help="only the 1024^2 lattice in FP64 with coarse levels <= 5 overlapped and serialised "
                         "(overlap fraction): one JSON line of its own")
    ap.add_argument("--adaptive", action="store_true",
                    help="only the uneven-distribution comparison (adaptive tree against uniform depths on the "
                         "patch workload and on a clustered workload): one JSON line of its own")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1008_2410_amd import _lib, fmm, workloads

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "copies": 10}), flush=True)
        return
    if args.rk2 or args.rk2_adaptive:
        rk2_leg(torch, dev, workloads, adaptive=args.rk2_adaptive)
        return
    if args.cost_model:
        cost_model_leg(torch, dev, workloads)
        return
    if args.adaptive:
        adaptive_leg(torch, dev, workloads)
        return
    if args.lattice:
        print(json.dumps(lattice_overlap_leg(torch, dev, workloads, args.steps)), flush=True)
        return
    t0 = time.perf_counter()
    w = workloads.gaussian_patches(n=args.n, depth=args.depth)
    log(f"[bench] workload generated: N={w.n} depth={w.depth} p={w.p} ({time.perf_counter() - t0:.1f} s)")
    xy = torch.from_numpy(w.xy).to(dev)
    gamma = torch.from_numpy(w.gamma).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree = fmm.Tree(xy, w.depth, None)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = tree.info()
    plan = tree.near_plan()
    log(f"[bench] tree built on the device in {t_build:.3f} s: {info}; near-field plan {plan}")
    out = torch.empty((w.n, 2), dtype=torch.float64, device=dev)
    if args.adjoint_only:
        adjoint_only_leg(torch, dev, tree, w, gamma, info, args)
        return

    def run(k, precision="mixed"):
        for _ in range(k):
            tree.velocity(gamma, w.sigma, w.p, precision, out=out)

    def timed(k, precision="mixed", timing=True):
        tree.set_option(_lib.FMM_OPT_TIMING, 1 if timing else 0)
        tree.timings()  # reset
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        run(k, precision)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / k
        st = tree.timings()
        tree.set_option(_lib.FMM_OPT_TIMING, 0)
        per = {kk: (v / st["calls"] if st["calls"] else None) for kk, v in st.items() if kk != "calls"}
        return ms, per

    hp = args.headline_precision if args.headline_only else "mixed"
    # warmup
    run(args.warmup, hp)
    torch.cuda.synchronize()
    log("[bench] warmup done")
    # timed region: overlapped schedule
    ms, stages = timed(args.steps, hp)
    log(f"[bench] {hp} overlap: {ms:.3f} ms/step, stages {stages}")
    if args.headline_only:
        if hp == "fp64":
            rl = p2p_roofline("p2p_near_kernel<double>", info["p2p_pairs"], plan, stages["p2p"],
                              PEAK_FP64_VECTOR_TFLOPS, PEAK_FP64_VECTOR_TFLOPS)
        else:
            rl = p2p_roofline("p2p_near_kernel<float>", info["p2p_pairs"], plan, stages["p2p"],
                              PEAK_FP32_VECTOR_TFLOPS, ISSUABLE_FP32_VECTOR_TFLOPS)
        print(json.dumps({"precision": hp, "ms_per_step": round(ms, 4), "value": round(w.n / (ms * 1e-3) / 1e6, 3),
                          "p2p_avg_ms": round(stages["p2p"], 4), "p2p_tflops": rl["achieved"],
                          "p2p_executed_tflops": rl["executed"]["achieved"], "kernel_sources": kernel_sources_hash(),
                          "steps": args.steps, "warmup": args.warmup}), flush=True)
        return
    # serial schedule of the same work, for the overlap fraction
    tree.set_option(_lib.FMM_OPT_SCHEDULE, 1)
    run(1)
    ms_serial, stages_serial = timed(args.steps)
    tree.set_option(_lib.FMM_OPT_SCHEDULE, 2)  # back to the default (automatic)
    log(f"[bench] mixed serial: {ms_serial:.3f} ms/step, stages {stages_serial}")
    # overlap fraction: how much of the shorter of P2P / far field is hidden, from the
    # serial stage times and the overlapped span between the pack and final stages
    t_p2p, t_far = stages_serial["p2p"], stages_serial["far"]
    t_both = stages["total"] - stages["pack"] - stages["final"]
    overlap = (t_p2p + t_far - t_both) / min(t_p2p, t_far) if min(t_p2p, t_far) > 0 else None
    # accuracy sample of the mixed result
    run(1)
    uv_mixed = out.cpu().numpy()
    # plain FP64 GPU FMM at the same configuration
    run(1, "fp64")
    ms_fp64, stages_fp64 = timed(args.fp64_steps, "fp64")
    uv_fp64 = out.cpu().numpy()
    log(f"[bench] fp64: {ms_fp64:.3f} ms/step, stages {stages_fp64}")

    # backward pass (adjoint) at the same configuration: bwd/fwd time ratio
    dl = torch.empty((w.n, 2), dtype=torch.float64, device=dev).normal_(generator=torch.Generator(dev).manual_seed(0))

    def run_bwd(k, t=tree, g=gamma, sig=w.sigma, p=w.p, d=dl):
        for _ in range(k):
            t.velocity_backward(g, sig, p, "mixed", d)

    run_bwd(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    run_bwd(args.bwd_steps)
    e1.record()
    torch.cuda.synchronize()
    ms_bwd = e0.elapsed_time(e1) / args.bwd_steps
    log(f"[bench] mixed backward: {ms_bwd:.3f} ms/step (bwd/fwd {ms_bwd / ms:.3f})")
    del dl
    # 2^20 uniform particles, depth 8, p = 12 (the differentiation configuration)
    wu = workloads.uniform_target_field()
    xu = torch.from_numpy(wu.xy).to(dev)
    gu = torch.from_numpy(wu.gamma).to(dev)
    tu = fmm.Tree(xu, wu.depth, wu.root_box)
    du = torch.from_numpy(wu.extra["u_target"]).to(dev)
    ou = torch.empty((wu.n, 2), dtype=torch.float64, device=dev)

    def time_it(fn, k):
        fn()
        torch.cuda.synchronize()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record()
        for _ in range(k):
            fn()
        a1.record()
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / k

    ms_fu = time_it(lambda: tu.velocity(gu, wu.sigma, wu.p, "mixed", out=ou), args.steps)
    ms_bu = time_it(lambda: tu.velocity_backward(gu, wu.sigma, wu.p, "mixed", du), args.steps)
    log(f"[bench] uniform 2^20 mixed: fwd {ms_fu:.3f} ms, bwd {ms_bu:.3f} ms (bwd/fwd {ms_bu / ms_fu:.3f})")
    tu.close()
    del xu, gu, du, ou
    lattice = lattice_overlap_leg(torch, dev, workloads, args.steps)

    idx = w.extra["sample"]
    cpu = None
    err_mixed = err_fp64 = None
    if not args.no_cpu:
        ref, t_gate, cpu = cpu_baseline_leg(w, args.cpu_sample_log4)
        err_mixed = rel_l2(uv_mixed[idx], ref)
        err_fp64 = rel_l2(uv_fp64[idx], ref)
        log(f"[bench] oracle gate: mixed rel-L2 {err_mixed:.3e}, fp64 {err_fp64:.3e} ({t_gate:.1f} s); cpu {cpu}")
    err_mixed_vs_fp64 = rel_l2(uv_mixed[idx], uv_fp64[idx])

    pairs = info["p2p_pairs"]
    value = w.n / (ms * 1e-3) / 1e6
    rec = {
        "metric": "Mparticles/s FMM velocity eval, N=16M, p=16, rel-L2<=1e-5 vs FP64; bwd/fwd",
        "value": round(value, 3),
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "gaussian_patches", "n": w.n, "patches": 8, "sigma": w.sigma, "depth": w.depth,
                   "p": w.p, "precision": "mixed", "schedule": "overlap", "root": "bounding square"},
        "roofline": p2p_roofline("p2p_near_kernel<float>", pairs, plan, stages["p2p"], PEAK_FP32_VECTOR_TFLOPS,
                                 ISSUABLE_FP32_VECTOR_TFLOPS),
        "cpu_baseline": cpu,
        "accuracy": {"mixed_vs_oracle_rel_l2": err_mixed, "fp64_vs_oracle_rel_l2": err_fp64,
                     "mixed_vs_gpu_fp64_rel_l2": err_mixed_vs_fp64,
                     "sample": len(idx), "gate": 1e-5},
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "near_field": {"mutual_items": plan["mutual_items"], "mutual_pairs": plan["mutual_pairs"],
                       "target_units": plan["target_units"], "all_pairs": info["p2p_pairs"]},
        "serial_ms_per_step": round(ms_serial, 4),
        "serial_stages_ms": {k: round(v, 4) for k, v in stages_serial.items()},
        "overlap_fraction": None if overlap is None else round(overlap, 4),
        "fp64": {"ms_per_step": round(ms_fp64, 4), "value": round(w.n / (ms_fp64 * 1e-3) / 1e6, 3),
                 "stages_ms": {k: round(v, 4) for k, v in stages_fp64.items()},
                 "roofline": p2p_roofline("p2p_near_kernel<double>", pairs, plan, stages_fp64["p2p"],
                                          PEAK_FP64_VECTOR_TFLOPS, PEAK_FP64_VECTOR_TFLOPS)},
        "lattice_fp64_overlap": lattice,
        "bwd_fwd": {"gaussian_patches_16M": round(ms_bwd / ms, 4), "bwd_ms": round(ms_bwd, 4),
                    "uniform_1M_p12": round(ms_bu / ms_fu, 4), "uniform_fwd_ms": round(ms_fu, 4),
                    "uniform_bwd_ms": round(ms_bu, 4)},
        "tree": info,
        "tree_build_s": round(t_build, 4),
    }
    if err_mixed is not None and err_mixed > 1e-5:
        rec["value_invalid_reason"] = f"mixed rel-L2 {err_mixed:.3e} exceeds 1e-5"
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
