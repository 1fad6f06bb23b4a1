"""Benchmark: particles/s of one polarizable FMM step (tree, charge field, dipole solve to the
stated tolerance, energy, forces, and the adjoint backward) on one MI355X, float64 path and mixed
path, with the error of each against the CPU oracle stated.

    python bench.py [--steps K] [--warmup W] [--workload scaling_1m] [--gpus 1]

Prints ONE JSON line.  Inputs are synthetic (seeded), resident on the GPU before timing starts.
The dominant kernel's roofline fraction is measured live with HIP events on the library's stream;
the CPU oracle is timed on a bounded sample of the same workload on the host cores, and the same
oracle run gives the force error of both paths on that sample.
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
    "scaling_1m": dict(gen="scaling_1m", p=10, ws=2, leaf=6.0, tol=1e-6, slack=2, pc=5.0, pc_iters=4,
                       relax=0.01),
    "scaling_250k": dict(gen="scaling_250k", p=10, ws=2, leaf=6.0, tol=1e-6, slack=2, pc=5.0, pc_iters=4,
                         relax=0.01),
    "scaling_4m": dict(gen="scaling_4m", p=10, ws=2, leaf=6.0, tol=1e-6, slack=3, pc=5.0, pc_iters=4,
                       relax=0.01),
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
TRAFFIC_SOURCES = ["paper_1408_6527_amd/csrc/m2l.hip", "paper_1408_6527_amd/csrc/schedule.hpp"]


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
    ap.add_argument("--oracle-sample", type=int, default=0,
                    help="targets of the sampled oracle check (0: about 2e7 / n, between 8 and 192)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    for k in ("p", "ws", "leaf", "tol", "slack", "pc", "pc_iters", "relax"):
        if getattr(args, k) is not None:
            wl[k] = getattr(args, k)
    ps = inputs.make(wl["gen"])
    n = ps.n
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

    def make(prec, timing=False):
        s = api.Solver(order_p=wl["p"], ws=wl["ws"], leaf_width=wl["leaf"], scf_tol=wl["tol"],
                       m2l_order_slack=wl["slack"], precond_cutoff=wl["pc"], precond_iters=wl["pc_iters"],
                       scf_relax=wl["relax"], dipole_pair_dl=args.pair_dl, precision=prec, timing=timing)
        if pairs is not None:
            s.set_exclusions(n, pairs)
        return s

    def step(s):
        r = s.solve(pos, q, al, qE=qE)
        s.backward(1.0)
        return r

    def timed(prec):
        s = make(prec)
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

    # One oracle run on a sample of S targets: exact fields there from all n sources with the
    # dipoles of the primary path.  It gives the reference forces for the error of both paths
    # (a path's error thus includes its dipoles' distance from the primary path's) and, timed, the
    # CPU baseline.
    # (with field charges or exclusions the sampled oracle check does not apply: errors are left out)
    from oracle import direct as D
    rng = np.random.default_rng(7)
    S = args.oracle_sample if args.oracle_sample > 0 else max(8, min(192, int(2e7 / n)))
    S = min(S, n)
    idx = np.sort(rng.choice(n, S, replace=False))
    prim = precs[0]
    mu_ref = results[prim]["res"].mu.cpu().numpy()
    from threadpoolctl import threadpool_limits
    if not variant:
        with threadpool_limits(limits=1):  # one host thread: the figure is per core
            t0 = time.perf_counter()
            phi_o, Eu_o, Ed_o, G_o = D.fields_at(idx, ps.pos, ps.q, mu_ref, ps.alpha, 2.0)
            t_oracle = time.perf_counter() - t0
        F_ref = D.COULOMB_K * (ps.q[idx, None] * Eu_o + np.einsum("ia,iab->ib", mu_ref[idx], G_o))
    errs = {}
    for prec in precs:
        r = results[prec]["res"]
        errs[prec] = dict(scf_residual=float(r.residual), iters=int(r.iters),
                          scf_restarts=int(r.stats["scf_restarts"]),
                          m2l_order_cap_min=int(r.stats["m2l_order_cap_min"]))
        if not variant:
            Fg = r.forces.cpu().numpy()[idx]
            errs[prec].update(force_rel_l2_vs_oracle=float(np.linalg.norm(Fg - F_ref) / np.linalg.norm(F_ref)),
                              oracle_sample=int(S))
    if not variant:
        errs[prim]["dipole_residual_exact"] = float(
            np.linalg.norm(ps.alpha[idx, None] * Ed_o - mu_ref[idx]) / np.linalg.norm(ps.alpha[idx, None] * Ed_o))
    if "mixed" in results and "fp64" in results:
        a = results["mixed"]["res"]; b = results["fp64"]["res"]
        errs["mixed"]["vs_fp64_force"] = float(torch.linalg.norm(a.forces - b.forces) / torch.linalg.norm(b.forces))
        errs["mixed"]["vs_fp64_energy"] = float(abs(a.U - b.U) / abs(b.U))
        errs["mixed"]["vs_fp64_dipole"] = float(torch.linalg.norm(a.mu - b.mu) / torch.linalg.norm(b.mu))

    # per-kernel device time of one step of the primary path, HIP events on the library's stream
    st = make(prim, timing=True)
    rt = st.solve(pos, q, al, qE=qE)
    kms = rt.stats["t_kernel_ms"]; kl = rt.stats["kernel_launches"]
    dominant = max(kms, key=lambda k: kms[k])
    avg_ms = {k: (kms[k] / kl[k] if kl[k] else 0.0) for k in kms}
    p = wl["p"]
    if dominant == "m2l":
        # useful flops: 2 C(q+6, 6) per cell pair at the truncation order q it used (capped in the
        # relaxed iterations), counted on the device, summed over the step's launches
        work = rt.stats["m2l_flops_total"] / kl["m2l"]
        peak = PEAK["fp32_mfma"] if prim == "mixed" else PEAK["fp64_mfma"]
        bound = "mfma"
    else:
        # P2P of the dipole solve (the launch repeated every iteration) and any other kernel are
        # priced as plain vector arithmetic
        work = rt.stats["n_p2p"] * P2P_SCF_FLOPS_PER_PAIR
        peak = PEAK["fp64_vector"] if prim == "fp64" else PEAK["fp32_vector"]
        bound = "alu"
    achieved = work / (avg_ms[dominant] * 1e-3) / 1e12
    traffic = recorded_traffic(args.workload, prim) if dominant == "m2l" else None
    roofline = {"bound": bound, "kernel": dominant, "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                "avg_launch_ms": round(avg_ms[dominant], 4),
                "work_per_launch": round(work),
                "kernel_ms_per_step": {k: round(v, 3) for k, v in kms.items()},
                "launches_per_step": dict(kl)}

    # CPU oracle on the bounded sample above: exact fields of all n sources at S targets,
    # extrapolated to the field evaluations of one step (charge field, initial residual, one per
    # iteration, final pass)
    cpu = None
    if not args.no_cpu_baseline and not variant:
        evals = results[prim]["res"].stats["n_evals"]
        t_step = t_oracle * (n / S) * evals
        cpu = {"value": round(n / t_step, 3), "unit": "particles/s", "cores": 1, "kind": "oracle",
               "sample": f"direct-sum fields (phi, E, damped E, grad E) at {S} of {n} particles from all "
                         f"{n} sources in {t_oracle:.1f} s (numpy, one thread), scaled by n/{S} and by the "
                         f"{evals} field evaluations of one step"}

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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
