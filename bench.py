"""Benchmark: particles/s of one polarizable FMM step (tree, charge field, dipole solve to the
stated tolerance, energy, forces, and the adjoint backward) on one MI355X, float64 path and mixed
path, with the error of each against the CPU oracle stated.

    python bench.py [--steps K] [--warmup W] [--workload scaling_1m] [--gpus 1]

Prints ONE JSON line.  Inputs are synthetic (seeded), resident on the GPU before timing starts.
The dominant kernel's roofline fraction is measured live with HIP events on the library's stream.
The CPU oracle (direct sums in C++/OpenMP on all host cores) runs on a bounded sample of the same
workload: the exact fields at S sampled targets from each path's own dipoles give the force error
of each path at fixed dipoles (the estimator the GPU tests check against the oracle's full solution
at 50k and 250k particles), and, timed, the CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Workload presets: geometry generator, expansion order, separation, leaf edge, dipole tolerance,
# M2L order slack (-1: fixed order p; s >= 0: per-offset truncation order at the nearest offsets'
# error bound, plus s), dipole-solve preconditioner cutoff (A, 0: plain scaled CG) and its inner
# iterations, and the residual below which the solve's field evaluations cap the M2L order (0: never;
# the stopping rule is still checked at the full orders).  The 1M-particle preset is the fastest
# setting measured whose float64 force error on the sampled oracle check stays below 1e-5.
WORKLOADS = {
    # mixed_target: the settings of the mixed path at its own stated error (relative force error
    # <= 1e-4 instead of the float64 path's 1e-5), timed beside the shared settings
    "scaling_1m": dict(gen="scaling_1m", p=10, ws=2, leaf=6.0, tol=1e-6, slack=2, pc=5.5, pc_iters=3,
                       relax=0.03, mixed_target=dict(p=8, leaf=5.5, slack=1, relax=0.01, pc=5.0)),
    "scaling_250k": dict(gen="scaling_250k", p=10, ws=2, leaf=6.0, tol=1e-6, slack=2, pc=5.5, pc_iters=3,
                         relax=0.03, mixed_target=dict(p=8, leaf=5.5, slack=1, relax=0.01, pc=5.0)),
    "scaling_4m": dict(gen="scaling_4m", p=10, ws=2, leaf=6.0, tol=1e-6, slack=3, pc=5.5, pc_iters=3,
                       relax=0.03, mixed_target=dict(p=8, leaf=5.5, slack=1, relax=0.01, pc=5.0)),
    "globular_50k": dict(gen="globular_50k", p=6, ws=2, leaf=4.0, tol=1e-6, slack=-1, pc=4.0, pc_iters=4,
                         relax=0.0),
    "uniform_cube_1k": dict(gen="uniform_cube_1k", p=4, ws=1, leaf=5.0, tol=1e-8, slack=-1, pc=0.0, pc_iters=4,
                            relax=0.0),
    "hexamer_shell_160k": dict(gen="hexamer_shell_160k", p=8, ws=2, leaf=5.0, tol=1e-6, slack=2, pc=5.0,
                               pc_iters=4, relax=0.0),
    # the paper's random sphere (4,096 points, 45 A, +/-1 e) at its order 5, polarisation off
    "sphere_4096": dict(gen="sphere_4096", p=5, ws=2, leaf=6.0, tol=1e-6, slack=-1, pc=0.0, pc_iters=4,
                        relax=0.0),
}

# HBM traffic of the dominant kernel from rocprofv3 counters (profiles/), valid only while the
# kernel sources hash to the value recorded with the counters
TRAFFIC_SOURCES = ["paper_1408_6527_amd/csrc/m2l.hip", "paper_1408_6527_amd/csrc/schedule.hpp",
                   "paper_1408_6527_amd/csrc/mac.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str, precision: str):
    """Calibrated HBM bytes per launch of M2L recorded in profiles/<workload>_m2l_traffic.txt
    ('key: value' lines), or None when absent or taken from other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{workload}_m2l_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash() or kv.get("precision") != precision:
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None

PEAK = {"fp64_vector": 78.6, "fp64_mfma": 78.6, "fp32_mfma": 157.3, "fp32_vector": 157.3, "hbm": 8000.0}
P2P_SCF_FLOPS_PER_PAIR = 44  # damped dipole field of one source at one target (p2p.hip)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="scaling_1m", choices=sorted(WORKLOADS))
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--ws", type=int, default=None)
    ap.add_argument("--leaf", type=float, default=None)
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--slack", type=int, default=None, help="M2L order slack (-1: fixed order p)")
    ap.add_argument("--pc", type=float, default=None, help="preconditioner cutoff in A (0: plain CG)")
    ap.add_argument("--pc-iters", type=int, default=None, help="inner preconditioner iterations")
    ap.add_argument("--relax", type=float, default=None,
                    help="residual below which the dipole solve caps the M2L order (0: never)")
    ap.add_argument("--pair-dl", type=float, default=0.0,
                    help="dipole multipoles from +/- q^mu charge pairs this far apart (A; 0: point dipoles)")
    ap.add_argument("--field-charges", action="store_true",
                    help="polarise the dipoles with separate field charges (a seeded reshuffle of q)")
    ap.add_argument("--exclusions", type=int, default=0,
                    help="exclude the pairs (i, i + d), d = 1 .. K, of the generator's particle order")
    ap.add_argument("--polarisable-fraction", type=float, default=1.0,
                    help="keep the polarisability of a seeded fraction of the particles, zero for the rest "
                         "(the paper's systems: about 1/3)")
    ap.add_argument("--dipole-tree", action="store_true",
                    help="run the dipole solve on a tree of the polarisable sites alone (T^mu)")
    ap.add_argument("--theta", type=float, default=0.0,
                    help="interaction lists of the acceptance criterion with this theta (0: the ws lists); every "
                         "M2L at order p (the order slack is dropped)")
    ap.add_argument("--ndirect", type=int, default=64,
                    help="with --theta: cell pairs holding fewer particles together are summed directly")
    ap.add_argument("--leaf-direct", type=int, default=1, choices=[0, 1],
                    help="with --theta: leaf pairs are always summed directly")
    ap.add_argument("--leaf-max", type=int, default=0,
                    help="the adaptive octree: cells above the finest level split only when they hold more than "
                         "this many particles (0: every leaf at the finest level)")
    ap.add_argument("--oracle-sample", type=int, default=0,
                    help="targets of the sampled oracle check (0: about 2e9 / n, between 64 and 4096)")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the extra float64 solve at tolerance 1e-10 that splits the force error into the "
                         "FMM evaluation error and the part the solver tolerance adds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed-target", action="store_true",
                    help="skip the mixed path at its own error target (the workload's mixed_target settings)")
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB before the benchmark, so that a "
                         "profiler's memory counters can be calibrated against a kernel of known traffic")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1408_6527_amd import api, inputs

    wl = dict(WORKLOADS[args.workload])
    mixed_target = wl.pop("mixed_target", None)
    for k in ("p", "ws", "leaf", "tol", "slack", "pc", "pc_iters", "relax"):
        if getattr(args, k) is not None:
            wl[k] = getattr(args, k)
            mixed_target = None  # settings given by hand: no second set
    if args.theta > 0.0:
        wl["slack"] = -1
    ps = inputs.make(wl["gen"])
    n = ps.n
    if args.polarisable_fraction < 1.0:
        keep = np.random.default_rng(13).permutation(n) < int(round(args.polarisable_fraction * n))
        ps.alpha = np.where(keep, ps.alpha, 0.0)
    dev = torch.device("cuda", 0)
    variant = args.field_charges or args.exclusions > 0
    qE = None
    if args.field_charges:
        qE = torch.as_tensor(np.random.default_rng(11).permutation(ps.q), dtype=torch.float64, device=dev)
    pairs = None
    if args.exclusions > 0:
        pairs = np.concatenate([np.stack([np.arange(n - d), np.arange(d, n)], axis=1)
                                for d in range(1, args.exclusions + 1)])
    pos = torch.as_tensor(ps.pos, dtype=torch.float64, device=dev)
    q = torch.as_tensor(ps.q, dtype=torch.float64, device=dev)
    al = torch.as_tensor(ps.alpha, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def make(prec, timing=False, tol=None, over=None):
        w = dict(wl, **(over or {}))
        s = api.Solver(order_p=w["p"], ws=w["ws"], leaf_width=w["leaf"], scf_tol=tol or w["tol"],
                       m2l_order_slack=w["slack"], precond_cutoff=w["pc"], precond_iters=w["pc_iters"],
                       scf_relax=w["relax"], dipole_pair_dl=args.pair_dl, precision=prec, timing=timing,
                       dipole_tree=int(args.dipole_tree), mac_theta=args.theta, mac_ndirect=args.ndirect,
                       mac_leaf_direct=args.leaf_direct, adaptive_leaf_max=args.leaf_max)
        if pairs is not None:
            s.set_exclusions(n, pairs)
        return s

    def step(s):
        r = s.solve(pos, q, al, qE=qE)
        s.backward(1.0)
        return r

    def timed(prec, over=None):
        s = make(prec, over=over)
        for _ in range(args.warmup):
            step(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = step(s)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        return s, r, dt

    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    results = {}
    for prec in precs:
        s, r, dt = timed(prec)
        results[prec] = dict(solver=s, res=r, dt=dt)
        del s
    if args.no_mixed_target or args.precision != "both" or variant:
        mixed_target = None
    if mixed_target:
        s, r, dt = timed("mixed", over=mixed_target)
        results["mixed_target"] = dict(solver=s, res=r, dt=dt)
        del s

    prim = precs[0]
    from oracle import native as NT

    # --- errors on S sampled targets: exact forces from all n sources with each path's own dipoles
    # (with field charges or exclusions the sampled check does not apply: errors are left out)
    rng = np.random.default_rng(7)
    S = args.oracle_sample if args.oracle_sample > 0 else max(64, min(4096, int(2e9 / n)))
    S = min(S, n)
    idx = np.sort(rng.choice(n, S, replace=False))
    errs = {}
    t_full = None
    for prec in precs + (["mixed_target"] if mixed_target else []):
        r = results[prec]["res"]
        e = dict(scf_residual=float(r.residual), iters=int(r.iters), scf_restarts=int(r.stats["scf_restarts"]),
                 m2l_order_cap_min=int(r.stats["m2l_order_cap_min"]))
        if not variant:
            mu = r.mu.cpu().numpy()
            t0 = time.perf_counter()
            F_ref, res_ref = NT.forces_at(ps.pos, ps.q, mu, ps.alpha, idx)
            if prec == prim:
                t_full = time.perf_counter() - t0
            Fg = r.forces.cpu().numpy()[idx]
            fe = np.linalg.norm(Fg - F_ref, axis=1) / np.linalg.norm(F_ref, axis=1)
            e.update(force_rel_l2_at_fixed_dipoles=float(np.linalg.norm(Fg - F_ref) / np.linalg.norm(F_ref)),
                     per_atom_force_error={"median": float(np.median(fe)), "p80": float(np.percentile(fe, 80)),
                                           "p99": float(np.percentile(fe, 99)), "max": float(fe.max())},
                     dipole_residual_exact=float(np.linalg.norm(res_ref) / np.linalg.norm(res_ref + mu[idx])),
                     oracle_sample=int(S))
        errs[prec] = e
    if "mixed" in results and "fp64" in results:
        a = results["mixed"]["res"]; b = results["fp64"]["res"]
        errs["mixed"]["vs_fp64_force"] = float(torch.linalg.norm(a.forces - b.forces) / torch.linalg.norm(b.forces))
        errs["mixed"]["vs_fp64_energy"] = float(abs(a.U - b.U) / abs(b.U))
        errs["mixed"]["vs_fp64_dipole"] = float(torch.linalg.norm(a.mu - b.mu) / torch.linalg.norm(b.mu))
    # the float64 error split: FMM evaluation error of a solve to 1e-10, and what the benchmark's
    # tolerance adds to the forces (same settings otherwise)
    if not variant and not args.no_split and "fp64" in results:
        st = make("fp64", tol=1e-10)
        rt = st.solve(pos, q, al, qE=qE)
        F_t = rt.forces.cpu().numpy()
        F_ref_t, _ = NT.forces_at(ps.pos, ps.q, rt.mu.cpu().numpy(), ps.alpha, idx)
        F_b = results["fp64"]["res"].forces.cpu().numpy()
        errs["fp64"]["split"] = {
            "fmm_error_at_tol_1e-10": float(np.linalg.norm(F_t[idx] - F_ref_t) / np.linalg.norm(F_ref_t)),
            "scf_tolerance_part": float(np.linalg.norm(F_b - F_t) / np.linalg.norm(F_t)),
            "iters_at_tol_1e-10": int(rt.iters)}
        del st, rt
    if not variant:
        errs["estimator"] = ("force error at fixed dipoles on the sampled targets; checked against the oracle's "
                             "full solution at 50k and 250k particles in the GPU tests")

    # --- per-kernel device time of one step of each path, HIP events on the library's stream
    kinfo = {}
    for prec in precs:
        stt = make(prec, timing=True)
        rt = stt.solve(pos, q, al, qE=qE)
        kinfo[prec] = rt.stats
        del stt, rt
    kst = kinfo[prim]
    kms = kst["t_kernel_ms"]; kl = kst["kernel_launches"]
    dominant = max(kms, key=lambda k: kms[k])
    avg_ms = {k: (kms[k] / kl[k] if kl[k] else 0.0) for k in kms}
    p = wl["p"]

    def m2l_roof(stats, peak):
        """Useful M2L flops (2 C(q+6, 6) per cell pair at the order q it used) per launch over the
        launch's average device time: all launches, and the full-order and order-capped ones apart."""
        k_ms = stats["t_kernel_ms"]["m2l"]; k_n = stats["kernel_launches"]["m2l"]
        out = {"achieved": round(stats["m2l_flops_total"] / (k_ms * 1e-3) / 1e12, 3), "peak": peak,
               "frac": round(stats["m2l_flops_total"] / (k_ms * 1e-3) / 1e12 / peak, 4),
               "avg_launch_ms": round(k_ms / k_n, 4), "work_per_launch": round(stats["m2l_flops_total"] / k_n)}
        sp = stats["m2l_split"]
        for c, name in ((0, "full_order"), (1, "capped")):
            if sp["launches"][c]:
                a = sp["flops"][c] / (sp["ms"][c] * 1e-3) / 1e12
                out[name] = {"launches": sp["launches"][c], "avg_launch_ms": round(sp["ms"][c] / sp["launches"][c], 4),
                             "work_per_launch": round(sp["flops"][c] / sp["launches"][c]),
                             "achieved": round(a, 3), "frac": round(a / peak, 4)}
        return out

    def p2p_roof(stats, peak):
        ms = stats["t_kernel_ms"]["p2p_scf"]; nl = stats["kernel_launches"]["p2p_scf"]
        if not nl:
            return None
        work = stats["n_p2p"] * P2P_SCF_FLOPS_PER_PAIR
        a = work / (ms / nl * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(a, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(a / peak, 4),
                "avg_launch_ms": round(ms / nl, 4), "work_per_launch": work, "pairs": stats["n_p2p"],
                "flops_per_pair": P2P_SCF_FLOPS_PER_PAIR}

    if dominant == "m2l" and (args.theta > 0.0 or args.leaf_max > 0):
        # the M2L of the dual-walk lists runs on the float64 matrix cores on both paths
        mr = m2l_roof(kst, PEAK["fp64_mfma"])
        roofline = {"bound": "mfma", "kernel": "m2l_mac", "achieved": mr["achieved"], "peak": PEAK["fp64_mfma"],
                    "unit": "TFLOP/s", "frac": mr["frac"], "traffic": None,
                    "avg_launch_ms": mr["avg_launch_ms"], "work_per_launch": mr["work_per_launch"]}
    elif dominant == "m2l":
        peak = PEAK["fp32_mfma"] if prim == "mixed" else PEAK["fp64_mfma"]
        mr = m2l_roof(kst, peak)
        roofline = {"bound": "mfma", "kernel": "m2l", "achieved": mr["achieved"], "peak": peak, "unit": "TFLOP/s",
                    "frac": mr["frac"], "traffic": recorded_traffic(args.workload, prim),
                    "avg_launch_ms": mr["avg_launch_ms"], "work_per_launch": mr["work_per_launch"]}
        for k in ("full_order", "capped"):
            if k in mr:
                roofline[k] = mr[k]
    else:
        pr = p2p_roof(kst, PEAK["fp64_vector"] if prim == "fp64" else PEAK["fp32_vector"])
        roofline = dict(pr, kernel=dominant, traffic=None)
    roofline["kernel_ms_per_step"] = {k: round(v, 3) for k, v in kms.items()}
    roofline["launches_per_step"] = dict(kl)
    roofline["p2p_dipole_solve"] = p2p_roof(kst, PEAK["fp64_vector"] if prim == "fp64" else PEAK["fp32_vector"])
    if "mixed" in kinfo and prim != "mixed":
        # the mixed path's M2L: float32 MFMA below level 4 (float64 at levels <= 3), priced against the
        # float32 matrix peak
        roofline["mixed_path"] = {"m2l": m2l_roof(kinfo["mixed"], PEAK["fp32_mfma"]),
                                  "p2p_dipole_solve": p2p_roof(kinfo["mixed"], PEAK["fp32_vector"]),
                                  "kernel_ms_per_step": {k: round(v, 3) for k, v in kinfo["mixed"]["t_kernel_ms"].items()}}

    # --- CPU baseline: the oracle on all host cores on a bounded sample of the same step.  Its field
    # evaluations: the charge field and the final pass with all outputs (timed above: full fields at S
    # targets), and one damped dipole product per dipole-solve evaluation of the GPU path (timed here at
    # the same S targets); scaled by n / S.
    cpu = None
    if not args.no_cpu_baseline and not variant:
        mu_p = results[prim]["res"].mu.cpu().numpy()
        t0 = time.perf_counter()
        NT.dipole_field(ps.pos, ps.alpha, 2.0, mu_p, targets=idx)
        t_mv = time.perf_counter() - t0
        evals = results[prim]["res"].stats["n_evals"]
        t_step = (n / S) * (2 * t_full + (evals - 2) * t_mv)
        model = "unknown"
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        cpu = {"value": round(n / t_step, 3), "unit": "particles/s", "cores": NT.threads(), "kind": "oracle",
               "cpu_model": model,
               "sample": f"direct sums (C++/OpenMP, {NT.threads()} threads, float64) at {S} of {n} targets from all "
                         f"{n} sources: full fields {t_full:.2f} s, damped dipole product {t_mv:.2f} s; step = n/S x "
                         f"(2 full passes + {evals - 2} products, the field evaluations of the GPU step)"}

    r0 = results[prim]
    value = n / r0["dt"]
    out = {
        "metric": "particles/s per polarizable FMM step (SCF+forces), mixed vs FP64 at stated err",
        "value": round(value, 2), "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r0["dt"] * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prim == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "order_p": p, "ws": wl["ws"],
                   "leaf_width": wl["leaf"], "scf_tol": wl["tol"], "m2l_order_slack": wl["slack"],
                   "precond_cutoff": wl["pc"], "precond_iters": wl["pc_iters"], "scf_relax": wl["relax"],
                   "dipole_pair_dl": args.pair_dl, "field_charges": bool(args.field_charges),
                   "excluded_pairs": 0 if pairs is None else int(len(pairs)),
                   "polarisable_fraction": args.polarisable_fraction, "dipole_tree": bool(args.dipole_tree),
                   "dipole_solve_sites": int(r0["res"].stats["n_sites"]),
                   "mac_theta": args.theta, "mac_ndirect": args.ndirect if args.theta > 0 else None,
                   "mac_leaf_direct": args.leaf_direct if args.theta > 0 else None,
                   "adaptive_leaf_max": args.leaf_max,
                   "m2l_pairs": int(r0["res"].stats["n_m2l"]), "near_pairs": int(r0["res"].stats["n_p2p"]),
                   "levels": r0["res"].stats["levels"],
                   "step": "solve (tree, charge field, dipole CG, energy, forces) + backward",
                   "parallelism": "single GPU"},
        "errors": errs,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "mixed" in results and "fp64" in results:
        out["mixed"] = {"value": round(n / results["mixed"]["dt"], 2),
                        "ms_per_step": round(results["mixed"]["dt"] * 1e3, 3),
                        "speedup_vs_fp64": round(results["fp64"]["dt"] / results["mixed"]["dt"], 3)}
    if mixed_target:
        # the mixed path at its own stated error: the same step (solve + backward, same tolerance,
        # preconditioner and relaxation) at the workload's mixed_target order and leaf edge
        rm = results["mixed_target"]
        w = dict(wl, **mixed_target)
        stt = make("mixed", timing=True, over=mixed_target)
        kt = stt.solve(pos, q, al, qE=qE).stats
        del stt
        out["mixed_at_target"] = {
            "target": "relative force error <= 1e-4 (the mixed path's; float64 path <= 1e-5)",
            "config": {"order_p": w["p"], "leaf_width": w["leaf"], "m2l_order_slack": w["slack"],
                       "scf_relax": w["relax"], "levels": rm["res"].stats["levels"], "m2l_pairs": int(rm["res"].stats["n_m2l"]),
                       "near_pairs": int(rm["res"].stats["n_p2p"])},
            "value": round(n / rm["dt"], 2), "ms_per_step": round(rm["dt"] * 1e3, 3),
            "speedup_vs_fp64": round(results["fp64"]["dt"] / rm["dt"], 3),
            "errors": errs.pop("mixed_target"),
            "kernel_ms_per_step": {k: round(v, 3) for k, v in kt["t_kernel_ms"].items()}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
