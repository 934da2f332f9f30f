"""Throughput of the MI355X AIREBO path: atom-steps/s of velocity-Verlet NVE.

One step is the whole hot path over the system once: half kick and drift, the
neighbour-list rebuild when an atom has moved more than half the skin, the
short list and coordination, bond order + REBO + torsion, the C_ij path map,
the LJ pair loop, the deferred b* pairs, and the second half kick.

Default workload: polyethylene melt, 106 x C100H202 = 32,012 atoms at
0.85 g/cm^3 in a 66.26 A periodic cube, 300 K, dt = 0.5 fs (synthetic,
seeded), FP64.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VALU_PEAK = 78.6e12      # MI355X vector FP64, FLOP/s
FP32_VALU_PEAK = 157.3e12
# Algorithmic FP64 operations per unit of work of each kernel (see the design
# notes for the breakdown): per LJ pair inside the cutoff (each pair once) and
# per REBO bond (bond order forward + reverse, pair term, torsion).
FLOP_PER_LJ_PAIR = 60
FLOP_PER_BOND = 4000


def counter_traffic(kernel, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated), or None when the kernel
    source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"airebo_{precision}_pe_melt_32k_hbm_counters.json")
    src = os.path.join(ROOT, "paper_1810_07026_amd", "csrc", "airebo.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha1") != hashlib.sha1(open(src, "rb").read()).hexdigest():
        return None
    k = rec["kernels"].get(kernel)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--workload", choices=["pe_melt_32k", "hybrid_1m", "batch512"], default="pe_melt_32k")
    ap.add_argument("--tune", default="", help="JSON launch shapes (batch512 workload)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not part of it",
                          "n_gpus": max(args.gpus, world)}))
        sys.exit(2)

    import torch
    from paper_1810_07026_amd import airebo, synth

    if args.copy_calib_mb:
        a = torch.ones(args.copy_calib_mb * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: copied {args.copy_calib_mb} MiB three times (counter calibration)")
        del a, b

    if args.workload == "batch512":
        return bench_batch(args)
    log("bench: generating workload")
    d = synth.pe_melt() if args.workload == "pe_melt_32k" else synth.hybrid_1m()
    n = len(d["species"])
    box, per = d["box"], d["periodic"]
    prec = airebo.FP64 if args.precision == "fp64" else airebo.MIXED
    ctx = airebo.Context(precision=prec)
    dev = torch.device("cuda", 0)
    x = torch.tensor(d["x"], dtype=torch.float64, device=dev)
    v = torch.tensor(d["v"], dtype=torch.float64, device=dev)
    x0 = x.clone()

    log(f"bench: n={n} warmup {args.warmup} steps")
    ctx.nve(x, v, d["species"], box, per, nsteps=args.warmup, thermo_every=0)
    torch.cuda.synchronize()
    every = max(1, args.steps // 20)
    log(f"bench: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = ctx.nve(x, v, d["species"], box, per, nsteps=args.steps, thermo_every=every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    th = th.cpu().numpy()
    sec = t1 - t0
    value = n * args.steps / sec
    rebuilds = int(th[-1, 5])
    log(f"bench: {value:.4g} atom-steps/s ({1e3 * sec / args.steps:.4f} ms/step), rebuilds {rebuilds}")

    # energy drift over the timed run: slope of (E - E0)/N and max |dE|/|E0|
    t_ps = th[:, 0] * 0.5e-3
    de = (th[:, 3] - th[0, 3]) / n
    slope = float(np.polyfit(t_ps, de, 1)[0]) if len(t_ps) > 2 else float("nan")
    maxrel = float(np.abs(th[:, 3] - th[0, 3]).max() / abs(th[0, 3]))

    # per-kernel device times (HIP events on the launch stream) and work counts
    e0, f0, _ = ctx.compute(x0, d["species"], box, per)
    st = ctx.stats()
    roof, kern = None, {}
    if not args.no_profile:
        xp, vp = x.clone(), v.clone()
        prof = ctx.profile_nve(xp, vp, d["species"], box, per, nsteps=args.profile_steps)
        kern = {k: {"total_ms": ms, "launches": c, "avg_us": 1e3 * ms / c if c else 0.0}
                for k, (ms, c) in prof.items() if c}
        st_p = ctx.stats()
        plain = st["lj_in_cut"] - st["cij_zero"] - st["bstar_queued"]
        work = {"k_lj": FLOP_PER_LJ_PAIR * plain, "k_bond": FLOP_PER_BOND * st["bonds"]}
        dom = max(kern, key=lambda k: kern[k]["total_ms"])
        cand = dom if dom in work else max(work, key=lambda k: kern.get(k, {"total_ms": 0})["total_ms"])
        avg_s = kern[cand]["avg_us"] * 1e-6
        peak = FP64_VALU_PEAK if prec == airebo.FP64 else FP32_VALU_PEAK
        ach = work[cand] / avg_s
        roof = {"bound": "alu", "kernel": cand, "dominant_kernel_by_time": dom, "achieved": ach / 1e12,
                "peak": peak / 1e12, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": counter_traffic(cand, args.precision),
                "flop_per_launch": work[cand], "avg_launch_us": kern[cand]["avg_us"]}
        log(f"bench: kernels {json.dumps({k: round(v['avg_us'], 2) for k, v in kern.items()})}")

    cpu = None
    ferr = None
    if not args.no_cpu_baseline:
        from oracle.oracle import Oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        orc = Oracle(nthreads=threads)
        fg = f0.cpu().numpy()
        if n <= 100000:
            log(f"bench: oracle on {threads} threads, one force evaluation of the {n}-atom system")
            t2 = time.perf_counter()
            eo, fo, wo = orc.compute(d["x"], d["species"], box, per)
            t3 = time.perf_counter()
            cpu = {"value": n / (t3 - t2), "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
                   "sample": f"one full FP64 force evaluation (= one MD step) of the {n}-atom system, "
                             f"{t3 - t2:.1f} s"}
            rms = math.sqrt((fo ** 2).sum(1).mean())
            ferr = {"force_rms_err_eVA": float(math.sqrt(((fg - fo) ** 2).sum(1).mean())),
                    "force_rel_err_max": float(np.abs(fg - fo).max() / rms),
                    "energy_rel_err": float(abs(e0[0].item() - eo[0]) / abs(eo[0]))}
        else:
            sel = np.sort(np.random.default_rng(0).choice(n, 4096, replace=False)).astype(np.int32)
            log(f"bench: oracle on {threads} threads, forces on {len(sel)} sampled atoms of {n}")
            t2 = time.perf_counter()
            _, fo, _ = orc.compute(d["x"], d["species"], box, per, sel=sel)
            t3 = time.perf_counter()
            cpu = {"value": len(sel) / (t3 - t2), "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
                   "sample": f"exact FP64 forces on {len(sel)} random atoms of the {n}-atom system "
                             f"(every term touching them), {t3 - t2:.1f} s"}
            fo, fgs = fo[sel], fg[sel]
            rms = math.sqrt((fo ** 2).sum(1).mean())
            ferr = {"force_rms_err_eVA": float(math.sqrt(((fgs - fo) ** 2).sum(1).mean())),
                    "force_rel_err_max": float(np.abs(fgs - fo).max() / rms), "sampled_atoms": len(sel)}

    out = {
        "metric": "AIREBO atom-steps/s on 1 GPU",
        "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == airebo.FP64 else "f32+f64",
        "data": "synthetic (seeded generators)",
        "config": {"workload": (f"polyethylene melt 106 x C100H202, {n} atoms, 0.85 g/cm^3, "
                                f"{box[0]:.2f} A periodic cube, 300 K, NVE dt 0.5 fs, {args.precision}"
                                if args.workload == "pe_melt_32k" else
                                f"hybrid {n} atoms: AB graphite 30 layers + H-terminated diamond (111) 31 bilayers "
                                f"+ polyethylene melt slab, box {box[0]:.1f} x {box[1]:.1f} x {box[2]:.1f} A, "
                                f"300 K, NVE dt 0.5 fs, {args.precision}"),
                   "n_atoms": n, "dt_fs": 0.5, "precision": args.precision},
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": ferr,
        "energy_drift": {"slope_eV_per_atom_per_ps": slope, "max_rel": maxrel, "rebuilds": rebuilds},
        "work": {k: st[k] for k in ("lj_in_cut", "cij_zero", "bstar_queued", "dsb_nonzero", "bonds")},
        "kernels_us": {k: round(v["avg_us"], 3) for k, v in kern.items()},
    }
    print(json.dumps(out))


def bench_batch(args):
    """512 independent systems (50-5,000 atoms, five families, own boxes), batched NVE."""
    import torch
    from paper_1810_07026_amd import airebo, synth
    d = synth.batch_cached(512)
    n = int(d["sizes"].sum())
    prec = airebo.FP64 if args.precision == "fp64" else airebo.MIXED
    tune = {}
    if args.tune and args.tune not in ("auto", "retune"):
        tune = json.loads(args.tune)
    elif args.tune in ("auto", "retune"):
        from paper_1810_07026_amd import autotune
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        key = autotune.workload_key(arch, n, len(d["sizes"]), args.precision)
        tune = autotune.lookup(key) if args.tune == "auto" else None
        if tune is None:
            def run(cand, steps):
                c = airebo.Context(precision=prec, tune=cand)
                xt = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
                vt = torch.tensor(d["v"], dtype=torch.float64, device="cuda")
                c.batch_nve(xt, vt, d["species"], d["sizes"], d["boxes"], d["periodic"], nsteps=5, thermo_every=0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                c.batch_nve(xt, vt, d["species"], d["sizes"], d["boxes"], d["periodic"], nsteps=steps,
                            thermo_every=0)
                torch.cuda.synchronize()
                c.close()
                return time.perf_counter() - t0
            tune = autotune.tune(run, key, steps=50, log=log)
        log(f"bench: launch shapes {tune}")
    ctx = airebo.Context(precision=prec, tune=tune)
    x = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
    v = torch.tensor(d["v"], dtype=torch.float64, device="cuda")
    ctx.batch_nve(x, v, d["species"], d["sizes"], d["boxes"], d["periodic"], nsteps=args.warmup, thermo_every=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = ctx.batch_nve(x, v, d["species"], d["sizes"], d["boxes"], d["periodic"], nsteps=args.steps,
                       thermo_every=max(1, args.steps // 10))
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    th = th.cpu().numpy()
    value = n * args.steps / sec
    de = np.abs(th[:, :, 3] - th[0, :, 3]).max(0) / d["sizes"]
    drift = float((np.abs(th[-1, :, 3] - th[0, :, 3])).max())
    log(f"bench: per-system max |dE|/N (eV/atom): median {np.median(de):.3g}, max {de.max():.3g} "
        f"(system {int(de.argmax())}, {int(d['sizes'][de.argmax()])} atoms)")
    out = {"metric": "AIREBO atom-steps/s on 1 GPU", "value": value, "unit": "atom-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * sec / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == airebo.FP64 else "f32+f64", "data": "synthetic (seeded generators)",
           "config": {"workload": f"batch of 512 systems, {n} atoms, sizes {int(d['sizes'].min())}-"
                                  f"{int(d['sizes'].max())}, five hydrocarbon families, own periodic boxes, "
                                  f"NVE dt 0.5 fs, {args.precision}", "n_atoms": n, "tune": tune},
           "max_abs_energy_change_eV": drift,
           "energy_change_per_atom": {"median": float(np.median(de)), "max": float(de.max())}}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
