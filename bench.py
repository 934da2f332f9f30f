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
# Algorithmic FP64 operations per unit of work of each kernel: per LJ pair
# inside the cutoff (each pair once), per list pair beyond it, per REBO bond
# (bond order forward + reverse, pair term, torsion), and per deferred pair
# (the b* bond order forward; its reverse only where dS_b != 0).  The pair
# figures are counts of the pair term; the bond-order figures are the FP64
# work the hardware counts per bond and per deferred pair on the 32k melt
# (the kernels evaluate each bond and pair once, so nothing is duplicated;
# the reverse of a deferred pair is taken as costing its forward).
FLOP_PER_LJ_PAIR = 45       # per pair inside its cutoff, each pair once
FLOP_PER_SKIN_PAIR = 8      # per list pair beyond its cutoff (distance test)
FLOP_PER_BOND = 2850
FLOP_PER_BSTAR_FWD = 1300   # per deferred pair
FLOP_PER_BSTAR_REV = 1300   # per deferred pair with dS_b != 0
# untimed preparation of the melt: capped steepest descent, then rescaled NVE
PREP_SD_ITERS, PREP_SD_ALPHA, PREP_SD_CAP = 300, 0.01, 0.02     # iterations, A^2/eV, A
PREP_EQ_CYCLES, PREP_EQ_STEPS = 20, 50
SURROGATE_TILES = (3, 3, 4)   # 32,012-atom melt tiled to 1,152,432 atoms
# potential variants: (term mask, van der Waals form, oracle mask)
POTENTIALS = {"airebo": (7, 0, 7), "airebo_m": (7, 1, 7 | 8), "rebo": (1, 0, 1)}
# arithmetic type of the force evaluation per precision mode (the integrator is FP64)
DTYPES = {"fp64": "f64", "mixed": "f32+f64", "single": "f32"}


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


def host_cpu():
    """Model name and logical CPU count of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["fp64", "mixed", "single"], default="fp64")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--workload", choices=["pe_melt_32k", "hybrid_1m", "cnt_bundle", "batch512", "surrogate_1m",
                                           "conservation"],
                    default="pe_melt_32k")
    ap.add_argument("--dt", type=float, default=0.5, help="time step in fs (conservation workload)")
    ap.add_argument("--system", choices=["pe_melt", "cnt_bundle"], default="pe_melt",
                    help="system of the conservation workload")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision and surrogate timings beside the FP64 line")
    ap.add_argument("--form-steps", type=int, default=200)
    ap.add_argument("--no-prep", action="store_true", help="time the generated melt without its preparation run")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 10^6-atom hybrid and surrogate sub-records of the default line")
    ap.add_argument("--extra-steps", type=int, default=50, help="timed steps of each 10^6-atom sub-record form")
    ap.add_argument("--potential", choices=["airebo", "airebo_m", "rebo"], default="airebo",
                    help="AIREBO, AIREBO-M (Morse in place of LJ, FP64) or REBO alone (no LJ, no torsion)")
    ap.add_argument("--cnt-cells", type=int, default=40, help="nanotube bundle: translational cells per tube")
    ap.add_argument("--cnt-grid", type=int, default=4, help="nanotube bundle: tubes per side of the square lattice")
    ap.add_argument("--thermo-out", default="",
                    help="conservation workload: also write the thermo rows (step PE KE Etot T rebuilds P) to this text file")
    ap.add_argument("--tune", default="", help="JSON launch shapes (batch512 workload)")
    ap.add_argument("--no-peaks", action="store_true", help="skip the copy and FMA-loop peak measurement")
    ap.add_argument("--save-state", default="", help="melt: write the prepared positions and velocities (npz)")
    ap.add_argument("--state", default="", help="melt: start from positions and velocities saved by --save-state")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(json.dumps({"error": "bench.py measures one GPU; runs on several GPUs are not supported",
                          "n_gpus": max(args.gpus, world)}))
        sys.exit(2)

    import torch
    from paper_1810_07026_amd import airebo, synth

    peaks = None
    if not args.no_peaks:
        peaks = airebo.measured_peaks()
        log(f"bench: measured peaks {json.dumps({k: round(v_, 1) for k, v_ in peaks.items()})}")
    args.peaks = peaks

    if args.copy_calib_mb:
        a = torch.ones(args.copy_calib_mb * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: copied {args.copy_calib_mb} MiB three times (counter calibration)")
        del a, b

    if args.workload == "conservation":
        return bench_conservation(args)
    if args.workload == "batch512":
        return bench_batch(args)
    if args.workload == "surrogate_1m":
        return bench_surrogate(args)
    log("bench: generating workload")
    d = {"pe_melt_32k": synth.pe_melt, "hybrid_1m": synth.hybrid_1m,
         "cnt_bundle": synth.nanotube_bundle}[args.workload]()
    n = len(d["species"])
    box, per = d["box"], d["periodic"]
    prec = airebo.PRECISIONS[args.precision]
    term_mask, vdw, omask = POTENTIALS[args.potential]
    ctx = airebo.Context(precision=prec, term_mask=term_mask, vdw=vdw)
    dev = torch.device("cuda", 0)
    x = torch.tensor(d["x"], dtype=torch.float64, device=dev)
    v = torch.tensor(d["v"], dtype=torch.float64, device=dev)

    if args.workload == "pe_melt_32k" and args.state:
        st_ = np.load(args.state)
        x = torch.tensor(st_["x"], dtype=torch.float64, device=dev)
        v = torch.tensor(st_["v"], dtype=torch.float64, device=dev)
        log(f"bench: state read from {args.state}")
    elif args.workload == "pe_melt_32k" and not args.no_prep:
        x, v = prepare_melt(d, x, v, log)
    if args.save_state:
        np.savez(args.save_state, x=x.cpu().numpy(), v=v.cpu().numpy())
        log(f"bench: prepared state written to {args.save_state}")
    elif args.workload == "hybrid_1m":
        x, v = prepare_hybrid(d, x, v, log)
    # the timed region holds exactly `steps` velocity-Verlet steps of a session
    # whose state is already on the device (begin and warm-up untimed)
    log(f"bench: n={n} session start, warmup {args.warmup} steps")
    every = max(1, args.steps // 20)
    value, ms, th = timed_session(lambda: ctx.md_begin(x, v, d["species"], box, per), ctx, n, args.steps,
                                  args.warmup, every)
    th = th.cpu().numpy()
    x, v = ctx.md_state()
    ctx.md_end()
    sec = 1e-3 * ms * args.steps
    rebuilds = int(th[-1, 5] - th[0, 5])
    log(f"bench: {value:.4g} atom-steps/s ({ms:.4f} ms/step), rebuilds {rebuilds}, T {th[0, 4]:.0f} -> "
        f"{th[-1, 4]:.0f} K")

    # energy drift over the timed run: slope of (E - E0)/N and max |dE|/|E0|
    t_ps = (th[:, 0] - th[0, 0]) * 0.5e-3
    de = (th[:, 3] - th[0, 3]) / n
    slope = float(np.polyfit(t_ps, de, 1)[0]) if len(t_ps) > 2 else float("nan")
    maxrel = float(np.abs(th[:, 3] - th[0, 3]).max() / abs(th[0, 3]))

    # accuracy and the other forms are measured on the state the timed run
    # ends in; the per-kernel profile continues from it
    xf, vf = x.clone(), v.clone()
    xf_h = xf.cpu().numpy()
    e0, f0, _ = ctx.compute(xf, d["species"], box, per)
    st = ctx.stats()
    roof, kern = None, {}
    if not args.no_profile:
        xp, vp = x.clone(), v.clone()
        prof = ctx.profile_nve(xp, vp, d["species"], box, per, nsteps=args.profile_steps)
        kern = {k: {"total_ms": ms_, "launches": c, "avg_us": 1e3 * ms_ / c if c else 0.0}
                for k, (ms_, c) in prof.items() if c}
        roof = roofline(kern, st, prec, args, args.peaks)
        log(f"bench: kernels {json.dumps({k: round(v_['avg_us'], 2) for k, v_ in kern.items()})}")

    cpu = None
    ferr = None
    fo = None
    if not args.no_cpu_baseline:
        from oracle.oracle import Oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        orc = Oracle(nthreads=threads)
        fg = f0.cpu().numpy()
        if n <= 100000:
            log(f"bench: oracle on {threads} threads, force evaluations of the {n}-atom system (at least 10 s)")
            t2 = time.perf_counter()
            eo, fo, wo = orc.compute(xf_h, d["species"], box, per, mask=omask)
            t3 = time.perf_counter()
            # repeated until the sample is at least 10 s long (at most 40 evaluations)
            reps, sec = 1, t3 - t2
            while sec < 10.0 and reps < 40:
                ta = time.perf_counter()
                orc.compute(xf_h, d["species"], box, per, mask=omask)
                sec += time.perf_counter() - ta
                reps += 1
            cpu = {"value": n * reps / sec, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
                   "sample": f"{reps} full FP64 force evaluations (= {reps} MD steps) of the {n}-atom system, "
                             f"{sec:.1f} s", "host_cpu": host_cpu()}
            # the same evaluation on one thread
            log("bench: oracle on 1 thread, one force evaluation")
            t4 = time.perf_counter()
            Oracle(nthreads=1).compute(xf_h, d["species"], box, per, mask=omask)
            t5 = time.perf_counter()
            cpu["single_thread"] = {"value": n / (t5 - t4), "unit": "atom-steps/s", "cores": 1,
                                    "sample": f"one full FP64 force evaluation of the {n}-atom system, {t5 - t4:.1f} s"}
            rms = math.sqrt((fo ** 2).sum(1).mean())
            ferr = {"force_rms_err_eVA": float(math.sqrt(((fg - fo) ** 2).sum(1).mean())), "force_rms_eVA": rms,
                    "force_rel_err_max": float(np.abs(fg - fo).max() / rms),
                    "energy_rel_err": float(abs(e0[0].item() - eo[0]) / abs(eo[0]))}
        else:
            sel = np.sort(np.random.default_rng(0).choice(n, 4096, replace=False)).astype(np.int32)
            log(f"bench: oracle on {threads} threads, forces on {len(sel)} sampled atoms of {n}")
            t2 = time.perf_counter()
            _, fo_all, _ = orc.compute(xf_h, d["species"], box, per, mask=omask, sel=sel)
            t3 = time.perf_counter()
            cpu = {"value": len(sel) / (t3 - t2), "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
                   "sample": f"exact FP64 forces on {len(sel)} random atoms of the {n}-atom system "
                             f"(every term touching them), {t3 - t2:.1f} s", "host_cpu": host_cpu()}
            fos, fgs = fo_all[sel], fg[sel]
            rms = math.sqrt((fos ** 2).sum(1).mean())
            ferr = {"force_rms_err_eVA": float(math.sqrt(((fgs - fos) ** 2).sum(1).mean())), "force_rms_eVA": rms,
                    "force_rel_err_max": float(np.abs(fgs - fos).max() / rms), "sampled_atoms": len(sel)}

    forms = None
    if not args.no_forms and args.workload == "pe_melt_32k" and args.potential == "airebo":
        forms = measure_forms(d, xf, vf, args, fo)
    extra = {}
    if args.workload == "pe_melt_32k" and args.potential == "airebo" and not args.no_extra:
        extra["hybrid_1m"] = record_or_error(lambda: hybrid_record(args))
        extra["surrogate_1m"] = record_or_error(lambda: surrogate_record(args))

    out = {
        "metric": "AIREBO atom-steps/s on 1 GPU",
        "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPES[args.precision],
        "data": "synthetic (seeded generators)",
        "config": {"workload": ("" if args.potential == "airebo" else
                                {"airebo_m": "AIREBO-M (Morse) on ", "rebo": "REBO only on "}[args.potential]) +
                               (f"polyethylene melt 106 x C100H202, {n} atoms, 0.85 g/cm^3, "
                                f"{box[0]:.2f} A periodic cube, relaxed and equilibrated at 300 K (untimed), "
                                f"NVE dt 0.5 fs, {args.precision}"
                                if args.workload == "pe_melt_32k" else
                                f"bundle of 16 (10,10) carbon nanotubes, {n} atoms, 3.4 A between walls, "
                                f"box {box[0]:.1f} x {box[1]:.1f} x {box[2]:.1f} A periodic, 300 K, NVE dt 0.5 fs, "
                                f"{args.precision}"
                                if args.workload == "cnt_bundle" else
                                f"hybrid {n} atoms: AB graphite 30 layers + H-terminated diamond (111) 31 bilayers "
                                f"+ polyethylene melt slab, box {box[0]:.1f} x {box[1]:.1f} x {box[2]:.1f} A, "
                                f"300 K, NVE dt 0.5 fs, {args.precision}"),
                   "n_atoms": n, "dt_fs": 0.5, "precision": args.precision, "potential": args.potential},
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": ferr,
        "energy_drift": {"slope_eV_per_atom_per_ps": slope, "max_rel": maxrel, "rebuilds": rebuilds,
                         "T_start_K": float(th[0, 4]), "T_end_K": float(th[-1, 4])},
        "work": {k: st[k] for k in ("lj_in_cut", "lj_in_cut_far", "lj_entries", "lj_entries_far", "cij_zero",
                                    "bstar_queued", "deferred_pairs", "dsb_nonzero", "bonds")},
        "kernels_us": {k: round(v_["avg_us"], 3) for k, v_ in kern.items()},
        "forms": forms,
    }
    out.update(extra)
    print(json.dumps(out))


def record_or_error(make):
    """A sub-record of the default line; a failure is reported in the record,
    not raised, so that the headline line is still printed."""
    try:
        return make()
    except Exception as e:   # noqa: BLE001 -- reported in the output
        log(f"bench: sub-record failed: {e!r}")
        return {"error": repr(e)}


def timed_session(begin, ctx, n, steps, warmup, every=0, counts=None):
    """atom-steps/s of `steps` steps of an MD session: begin (untimed), warm-up
    run (untimed), then one timed run bracketed by device synchronisations.
    Returns (atom-steps/s, ms/step, thermo rows of the timed run or None);
    `counts` (a dict), if given, receives the list rebuilds and capacity
    regrowths of the timed run."""
    import torch
    begin()
    ctx.md_run(warmup)
    torch.cuda.synchronize()
    s0 = ctx.stats() if counts is not None else None
    t0 = time.perf_counter()
    th = ctx.md_run(steps, thermo_every=every)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    if counts is not None:
        s1 = ctx.stats()
        counts.update(rebuilds=s1["rebuilds"] - s0["rebuilds"], regrowths=s1["regrowths"] - s0["regrowths"])
    return n * steps / sec, 1e3 * sec / steps, th


def kernel_work(st):
    """Algorithmic FP operations per launch of the kernels with a work model.
    The LJ pairs (each pair once) split at the list build into near pairs
    (within 3 max R2 + skin: k_lj) and far pairs (k_ljf): 45 flop per pair
    inside its cutoff, 8 per list pair outside it (distance test only).
    The bonded kernel: 2,850 flop per bond (forward and reverse bond order,
    pair term, torsion).  The deferred-pair kernel: 1,300 flop per deferred
    pair (b* forward) and 1,300 more per pair with dS_b != 0 (reverse)."""
    far_in, far_pairs = st["lj_in_cut_far"], st["lj_entries_far"] // 2
    near_in, near_pairs = st["lj_in_cut"] - far_in, (st["lj_entries"] - st["lj_entries_far"]) // 2
    return {"k_lj": FLOP_PER_LJ_PAIR * near_in + FLOP_PER_SKIN_PAIR * max(near_pairs - near_in, 0),
            "k_ljf": FLOP_PER_LJ_PAIR * far_in + FLOP_PER_SKIN_PAIR * max(far_pairs - far_in, 0),
            "k_bond": FLOP_PER_BOND * st["bonds"],
            "k_bstar": FLOP_PER_BSTAR_FWD * st["deferred_pairs"] + FLOP_PER_BSTAR_REV * st["dsb_nonzero"]}


def roofline(kern, st, prec, args, peaks=None):
    """Roofline record of the kernel with a work model that takes the most
    time per step (the deferred-pair kernel on the melt), against the
    published vector peak of the arithmetic type and against the measured
    FMA-loop peak; the other modelled kernels in `kernels`."""
    from paper_1810_07026_amd import airebo
    work = kernel_work(st)
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    peak = FP64_VALU_PEAK if prec == airebo.FP64 else FP32_VALU_PEAK
    mpeak = None
    if peaks:
        mpeak = 1e12 * (peaks["fp64_fma_TFLOPs"] if prec == airebo.FP64 else peaks["fp32_fma_TFLOPs"])
    rows = {}
    for k, w in work.items():
        if k not in kern or not kern[k]["launches"]:
            continue
        ach = w / (kern[k]["avg_us"] * 1e-6)
        rows[k] = {"achieved": ach / 1e12, "frac": ach / peak, "frac_measured_peak": ach / mpeak if mpeak else None,
                   "flop_per_launch": w, "avg_launch_us": kern[k]["avg_us"],
                   "time_ms_per_step": kern[k]["total_ms"] / max(args.profile_steps, 1)}
    cand = max(rows, key=lambda k: kern[k]["total_ms"])
    r = rows[cand]
    return {"bound": "alu", "kernel": cand, "dominant_kernel_by_time": dom, "achieved": r["achieved"],
            "peak": peak / 1e12, "unit": "TFLOP/s", "frac": r["frac"],
            # the committed counter profile is of the melt workload
            "traffic": (counter_traffic(cand, args.precision)
                        if args.workload == "pe_melt_32k" and args.potential == "airebo" else None),
            "peak_measured": mpeak / 1e12 if mpeak else None, "frac_measured_peak": r["frac_measured_peak"],
            "flop_per_launch": r["flop_per_launch"], "avg_launch_us": r["avg_launch_us"],
            "kernels": rows, "measured_peaks": peaks}


def prepare_melt(d, x, v, log):
    """Untimed preparation of the melt: capped-step steepest descent on the
    FP64 AIREBO forces (every atom moves at most 0.02 A per iteration), then
    NVE with the velocities rescaled to 300 K every 50 steps, then fresh
    300 K Maxwell velocities."""
    import torch
    from paper_1810_07026_amd import airebo, synth
    s, box, per = d["species"], d["box"], d["periodic"]
    ctx = airebo.Context()
    x = x.clone()
    e0 = None
    for it in range(PREP_SD_ITERS):
        e, f, _ = ctx.compute(x, s, box, per)
        if e0 is None:
            e0 = float(e[0])
        step = PREP_SD_ALPHA * f
        norm = step.norm(dim=1, keepdim=True)
        x += step * torch.clamp(PREP_SD_CAP / torch.clamp(norm, min=1e-30), max=1.0)
    e1 = float(ctx.compute(x, s, box, per)[0][0])
    n = len(s)
    log(f"bench: preparation: {PREP_SD_ITERS} capped steepest-descent steps, E {e0 / n:.5f} -> {e1 / n:.5f} eV/atom")
    v = v.clone()
    ctx.md_begin(x, v, s, box, per)
    for _ in range(PREP_EQ_CYCLES):
        th = ctx.md_run(PREP_EQ_STEPS, thermo_every=PREP_EQ_STEPS).cpu().numpy()
        x, v = ctx.md_state()
        v *= math.sqrt(300.0 / max(th[-1, 4], 1.0))
        ctx.md_begin(x, v, s, box, per)
    th = ctx.md_run(0, thermo_every=1).cpu().numpy()
    ctx.md_end()
    log(f"bench: preparation: {PREP_EQ_CYCLES} x {PREP_EQ_STEPS} NVE steps rescaled to 300 K (T {th[-1, 4]:.0f} K)")
    v = torch.tensor(synth.maxwell_velocities(s, 300.0, np.random.default_rng(1810070268)), dtype=torch.float64,
                     device=x.device)
    ctx.close()
    return x, v


def prepare_hybrid(d, x, v, log):
    """Untimed preparation of the hybrid slab: velocity quench (NVE in bursts
    of 10 steps, velocities zeroed after each) relaxes the strain of the
    assembled slabs, then fresh 300 K velocities."""
    import torch
    from paper_1810_07026_amd import airebo, synth
    s, box, per = d["species"], d["box"], d["periodic"]
    ctx = airebo.Context()
    log("bench: hybrid preparation: 20 quench cycles of 10 steps (untimed)")
    x, v = x.clone(), torch.zeros_like(v)
    for _ in range(20):
        ctx.nve(x, v, s, box, per, nsteps=10, thermo_every=0)
        v.zero_()
    ctx.close()
    v = torch.tensor(synth.maxwell_velocities(s, 300.0, np.random.default_rng(1810070267)), dtype=torch.float64,
                     device=x.device)
    return x, v


def force_err(f, fo):
    f = np.asarray(f, float)
    rms = math.sqrt((fo ** 2).sum(1).mean())
    e = math.sqrt(((f - fo) ** 2).sum(1).mean())
    return {"force_rms_err_eVA": e, "force_rel_rms_err": e / rms}


def measure_forms(d, x0, v0, args, fo):
    """FP64, mixed and single precision and the surrogate (with and without
    fallback) on the system of the headline line, all from the state its
    timed run ended in and under one protocol: an MD session started from
    that state, a warm-up run, then one timed run of --form-steps steps.
    Force errors are against the CPU oracle at that state (when it was
    evaluated) or the FP64 GPU forces."""
    from paper_1810_07026_amd import airebo, surrogate
    s, box, per = d["species"], d["box"], d["periodic"]
    n = len(s)
    ctx = airebo.Context()
    ref_kind = "cpu_oracle"
    if fo is None:
        fo = ctx.compute(x0, s, box, per)[1].cpu().numpy()
        ref_kind = "fp64_gpu"
    forms = {"reference": ref_kind, "steps": args.form_steps, "warmup": args.warmup,
             "protocol": "per form: session begun from the same state, warm-up run, one timed run"}
    base = None
    for name, prec in (("fp64", airebo.FP64), ("mixed", airebo.MIXED), ("single", airebo.SINGLE)):
        c = ctx if prec == airebo.FP64 else airebo.Context(precision=prec)
        val, ms, _ = timed_session(lambda: c.md_begin(x0, v0, s, box, per), c, n, args.form_steps, args.warmup)
        c.md_end()
        fm = c.compute(x0, s, box, per)[1].cpu().numpy()
        base = val if base is None else base
        forms[name] = dict(force_err(fm, fo), value=val, ms_per_step=ms, speedup_vs_fp64=val / base)
        log(f"bench: {name} {val:.4g} atom-steps/s ({ms:.4f} ms/step), force rel rms err "
            f"{forms[name]['force_rel_rms_err']:.3g}")
    if not os.path.exists(surrogate.WEIGHTS):
        forms["surrogate"] = {"error": "no trained weights (python -m paper_1810_07026_amd.surrogate train)"}
        return forms
    nn = airebo.Surrogate(path=surrogate.WEIGHTS)
    forms["surrogate"] = surrogate_forms(nn, ctx, x0, v0, s, box, per, fo, args.form_steps, args.warmup, base)
    return forms


def surrogate_forms(nn, ctx, x0, v0, s, box, per, f_ref, steps, warmup, fp64_value):
    """Surrogate error at one state and its MD rate with and without the
    AIREBO fallback (sessions as for the other forms); the fallback count is
    that of the timed run."""
    import torch
    from paper_1810_07026_amd import surrogate
    n = len(s)
    e, f, _, sp, info = nn.compute(ctx, x0, s, box, per, threshold=1e30, want_spread=True)
    f = f.cpu().numpy()
    sp = sp.cpu().numpy()
    rec = dict(force_err(f, f_ref), threshold_eVA=surrogate.THRESHOLD, max_spread_eVA=info["max_spread"],
               atoms_above_threshold=int((sp > surrogate.THRESHOLD).sum()))
    rec["fallback_threshold_study"] = threshold_study(nn, ctx, x0, v0, s, box, per)
    for key, thr in (("with_fallback", surrogate.THRESHOLD), ("no_fallback", 1e30)):
        nn.md_begin(ctx, x0, v0, s, box, per, threshold=thr)
        ctx.md_run(warmup)
        torch.cuda.synchronize()
        fb0 = ctx.stats()["nn_fallbacks"]
        t0 = time.perf_counter()
        ctx.md_run(steps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        fb = ctx.stats()["nn_fallbacks"] - fb0
        ctx.md_end()
        val = n * steps / sec
        rec[key] = {"value": val, "ms_per_step": 1e3 * sec / steps, "speedup_vs_fp64": val / fp64_value,
                    "fallback_steps": int(fb), "fallback_rate": fb / steps}
        log(f"bench: surrogate ({key}) {val:.4g} atom-steps/s, fallbacks {fb}/{steps}")
    return rec


def threshold_study(nn, ctx, x0, v0, s, box, per, frames=20, stride=10):
    """The ensemble's largest force spread per step along an FP64 AIREBO
    trajectory from (x0, v0) (a frame every `stride` steps), with the
    surrogate's force error against AIREBO on each frame: the threshold at
    which fewer than 10% of the steps would fall back, and the error of the
    steps it keeps."""
    import torch
    xt, vt = x0.clone(), v0.clone()
    spreads, errs = [], []
    for _ in range(frames):
        ctx.nve(xt, vt, s, box, per, nsteps=stride, thermo_every=0)
        _, fr, _ = ctx.compute(xt, s, box, per)
        _, fs, _, sp, info = nn.compute(ctx, xt, s, box, per, threshold=1e30, want_spread=True)
        spreads.append(float(info["max_spread"]))
        errs.append(float(((fs - fr) ** 2).sum(1).mean().sqrt() / (fr ** 2).sum(1).mean().sqrt()))
    spreads, errs = np.array(spreads), np.array(errs)
    thr = float(np.quantile(spreads, 0.9))
    keep = spreads <= thr
    out = {"frames": frames, "stride_steps": stride,
           "max_spread_eVA": {"min": float(spreads.min()), "median": float(np.median(spreads)),
                              "max": float(spreads.max())},
           "threshold_for_under_10pct_fallback_eVA": thr,
           "fallback_rate_at_0.1_eVA": float((spreads > 0.1).mean()),
           "force_rel_rms_err_of_kept_steps": float(errs[keep].mean())}
    log(f"bench: surrogate spread study {json.dumps(out)}")
    return out


def hybrid_record(args):
    """The ~10^6-atom hybrid slab (graphite + H-terminated diamond + melt):
    FP64 and mixed MD rates under the session protocol, and the mixed and
    FP64 force errors against the CPU oracle on sampled atoms."""
    import torch
    from paper_1810_07026_amd import airebo, synth
    from oracle.oracle import Oracle
    d = synth.hybrid_1m()
    s, box, per = d["species"], d["box"], d["periodic"]
    n = len(s)
    x = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
    v = torch.tensor(d["v"], dtype=torch.float64, device="cuda")
    x, v = prepare_hybrid(d, x, v, log)
    rec = {"workload": f"hybrid {n} atoms: AB graphite + H-terminated diamond (111) + polyethylene melt slab, "
                       f"box {box[0]:.1f} x {box[1]:.1f} x {box[2]:.1f} A, 300 K, NVE dt 0.5 fs",
           "n_atoms": n, "steps": args.extra_steps, "warmup": 5}
    base = None
    forces = {}
    for name, prec in (("fp64", airebo.FP64), ("mixed", airebo.MIXED)):
        c = airebo.Context(precision=prec)
        cnt = {}
        val, ms, _ = timed_session(lambda: c.md_begin(x, v, s, box, per), c, n, args.extra_steps, 5, counts=cnt)
        c.md_end()
        forces[name] = c.compute(x, s, box, per)[1].cpu().numpy()
        base = val if base is None else base
        rec[name] = dict({"value": val, "ms_per_step": ms, "speedup_vs_fp64": val / base}, **cnt)
        log(f"bench: hybrid {name} {val:.4g} atom-steps/s ({ms:.3f} ms/step), {cnt}")
        c.close()
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        sel = np.sort(np.random.default_rng(0).choice(n, 4096, replace=False)).astype(np.int32)
        t2 = time.perf_counter()
        _, fo, _ = Oracle(nthreads=threads).compute(x.cpu().numpy(), s, box, per, sel=sel)
        t3 = time.perf_counter()
        fo = fo[sel]
        for name in forces:
            rec[name].update(force_err(forces[name][sel], fo))
        rec["oracle_sample"] = {"atoms": len(sel), "seconds": t3 - t2, "cores": threads}
    return rec


def surrogate_record(args):
    """The learned surrogate on a >= 10^6-atom melt (the 32,012-atom melt
    tiled 3 x 3 x 4 = 1,152,432 atoms, fresh 300 K velocities decorrelated
    by untimed mixed-precision NVE) beside AIREBO FP64 and mixed on the same
    state; errors against the FP64 GPU forces on every atom and against the
    CPU oracle on sampled atoms."""
    import torch
    from paper_1810_07026_amd import airebo, surrogate, synth
    from oracle.oracle import Oracle
    d = synth.tile(synth.pe_melt(), SURROGATE_TILES)
    s, box, per = d["species"], d["box"], d["periodic"]
    n = len(s)
    rng = np.random.default_rng(1810070266)
    x = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
    v = torch.tensor(synth.maxwell_velocities(s, 300.0, rng), dtype=torch.float64, device="cuda")
    ctx = airebo.Context()
    ctxm = airebo.Context(precision=airebo.MIXED)
    log(f"bench: surrogate workload n={n}; decorrelating replicas (100 mixed NVE steps, untimed)")
    ctxm.nve(x, v, s, box, per, nsteps=100, thermo_every=0)
    torch.cuda.synchronize()
    steps = args.extra_steps
    rec = {"workload": f"polyethylene melt of {n} atoms (106 x C100H202 tiled "
                       f"{' x '.join(map(str, SURROGATE_TILES))}, {box[0]:.1f} x {box[1]:.1f} x {box[2]:.1f} A "
                       f"periodic, 300 K), NVE dt 0.5 fs", "n_atoms": n, "steps": steps, "warmup": 5}
    f64 = ctx.compute(x, s, box, per)[1].cpu().numpy()
    fm = ctxm.compute(x, s, box, per)[1].cpu().numpy()
    for name, c in (("fp64", ctx), ("mixed", ctxm)):
        cnt = {}
        val, ms, _ = timed_session(lambda: c.md_begin(x, v, s, box, per), c, n, steps, 5, counts=cnt)
        c.md_end()
        rec[name] = dict({"value": val, "ms_per_step": ms}, **cnt)
        log(f"bench: surrogate workload {name} {val:.4g} atom-steps/s ({ms:.3f} ms/step), {cnt}")
    rec["mixed"]["speedup_vs_fp64"] = rec["mixed"]["value"] / rec["fp64"]["value"]
    rec["mixed"].update(force_err(fm, f64))
    nn = airebo.Surrogate(path=surrogate.WEIGHTS)
    rec["surrogate"] = surrogate_forms(nn, ctx, x, v, s, box, per, f64, steps, 5, rec["fp64"]["value"])
    rec["surrogate"]["error_reference"] = "fp64_gpu"
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        sel = np.sort(rng.choice(n, 2048, replace=False)).astype(np.int32)
        _, fo, _ = Oracle(nthreads=threads).compute(x.cpu().numpy(), s, box, per, sel=sel)
        fo = fo[sel]
        fn = nn.compute(ctx, x, s, box, per, threshold=1e30)[1].cpu().numpy()[sel]
        rec["accuracy_vs_oracle"] = {"surrogate": force_err(fn, fo), "fp64_gpu": force_err(f64[sel], fo),
                                     "mixed_gpu": force_err(fm[sel], fo), "sampled_atoms": len(sel)}
    return rec


def bench_surrogate(args):
    """The surrogate sub-record as its own line (value: surrogate with
    fallback on the >= 10^6-atom melt)."""
    rec = surrogate_record(args)
    sur = rec["surrogate"]["with_fallback"]
    out = {"metric": "AIREBO atom-steps/s on 1 GPU", "value": sur["value"], "unit": "atom-steps/s", "n_gpus": 1,
           "steps": rec["steps"], "warmup": rec["warmup"], "ms_per_step": sur["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32+f64",
           "data": "synthetic (seeded generators)",
           "config": {"workload": "learned surrogate (4-member ensemble, fallback at 0.1 eV/A) on a " +
                                  rec["workload"], "n_atoms": rec["n_atoms"]},
           "record": rec}
    print(json.dumps(out))


def bench_conservation(args):
    """Energy conservation over a long NVE run of the 32,012-atom melt or the
    nanotube bundle (the paper's precision study, Sec. 5): total energy every
    1,000 steps, the run split into calls of 100,000 steps so that progress
    is reported."""
    import torch
    from paper_1810_07026_amd import airebo, synth
    d = (synth.pe_melt() if args.system == "pe_melt" else
         synth.nanotube_bundle(ncells=args.cnt_cells, nx=args.cnt_grid, ny=args.cnt_grid))
    s, box, per = d["species"], d["box"], d["periodic"]
    n = len(s)
    prec = airebo.PRECISIONS[args.precision]
    ctx = airebo.Context(precision=prec)
    x = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
    v = torch.tensor(d["v"], dtype=torch.float64, device="cuda")
    every, chunk = 1000, 100000
    rows = []
    done = rebuilds = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < args.steps:
        k = min(chunk, args.steps - done)
        th = ctx.nve(x, v, s, box, per, dt=args.dt, nsteps=k, thermo_every=every).cpu().numpy()
        rebuilds += int(ctx.stats()["rebuilds"])
        th = th.reshape(th.shape[0], -1)
        rows.append(th if done == 0 else th[1:])   # a later call's first row repeats the previous last
        done += k
        e = np.concatenate(rows)[:, 3]
        log(f"bench: conservation {args.precision} dt {args.dt} fs: {done} steps, "
            f"E_tot {e[-1]:.4f} eV, max |dE|/|E0| {np.abs(e - e[0]).max() / abs(e[0]):.3g}, "
            f"{time.perf_counter() - t0:.0f} s")
    sec = time.perf_counter() - t0
    th = np.concatenate(rows)
    if args.thermo_out:
        np.savetxt(args.thermo_out, th, fmt="%.10g", header="step PE_eV KE_eV Etot_eV T_K rebuilds P_bar")
    e, temp = th[:, 3], th[:, 4]
    rel = (e - e[0]) / abs(e[0])
    t_ps = np.arange(len(e)) * every * args.dt * 1e-3
    slope = float(np.polyfit(t_ps, e / n, 1)[0]) if len(e) > 2 else 0.0
    out = {"metric": "AIREBO energy conservation (max relative total-energy deviation)",
           "value": float(np.abs(rel).max()), "unit": "relative", "n_gpus": 1, "steps": args.steps, "warmup": 0,
           "ms_per_step": 1e3 * sec / args.steps, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": DTYPES[args.precision],
           "data": "synthetic (seeded generators)",
           "config": {"workload": ("polyethylene melt 106 x C100H202" if args.system == "pe_melt" else
                                   f"bundle of {args.cnt_grid ** 2} (10,10) carbon nanotubes of "
                                   f"{args.cnt_cells} cells, box {d['box'][0]:.1f} x {d['box'][1]:.1f} x "
                                   f"{d['box'][2]:.1f} A") +
                                  f", {n} atoms, NVE {args.steps} steps of {args.dt} fs, {args.precision}",
                      "n_atoms": n, "dt_fs": args.dt},
           "atom_steps_per_s": n * args.steps / sec,
           "energy": {"E0_eV": float(e[0]), "E_end_eV": float(e[-1]), "final_rel": float(rel[-1]),
                      "rms_rel": float(np.sqrt((rel ** 2).mean())), "slope_eV_per_atom_per_ps": slope,
                      "T_start_K": float(temp[0]), "T_end_K": float(temp[-1]),
                      "rel_every_100k_steps": [float(r) for r in rel[::100]]},
           "rebuilds": rebuilds}
    print(json.dumps(out))


def bench_batch(args):
    """512 independent systems (50-5,000 atoms, five families, own boxes), batched NVE."""
    import torch
    from paper_1810_07026_amd import airebo, synth
    d = synth.batch_cached(512)
    n = int(d["sizes"].sum())
    prec = airebo.PRECISIONS[args.precision]
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
    value, ms, th = timed_session(
        lambda: ctx.batch_md_begin(x, v, d["species"], d["sizes"], d["boxes"], d["periodic"]), ctx, n, args.steps,
        args.warmup, max(1, args.steps // 10))
    ctx.md_end()
    th = th.cpu().numpy()
    sec = 1e-3 * ms * args.steps
    de = np.abs(th[:, :, 3] - th[0, :, 3]).max(0) / d["sizes"]
    drift = float((np.abs(th[-1, :, 3] - th[0, :, 3])).max())
    log(f"bench: per-system max |dE|/N (eV/atom): median {np.median(de):.3g}, max {de.max():.3g} "
        f"(system {int(de.argmax())}, {int(d['sizes'][de.argmax()])} atoms)")
    for k in np.argsort(-de)[:5]:
        fam = synth.FAMILIES[k % len(synth.FAMILIES)]   # families are assigned round-robin
        log(f"bench:   system {int(k)} ({fam}, {int(d['sizes'][k])} atoms, box {d['boxes'][k][0]:.1f} A): "
            f"max |dE|/N {de[k]:.3g} eV/atom, E0 {th[0, k, 3]:.3f}, E_end {th[-1, k, 3]:.3f}, "
            f"T_end {th[-1, k, 4]:.0f} K")
    out = {"metric": "AIREBO atom-steps/s on 1 GPU", "value": value, "unit": "atom-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * sec / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPES[args.precision], "data": "synthetic (seeded generators)",
           "config": {"workload": f"batch of 512 systems, {n} atoms, sizes {int(d['sizes'].min())}-"
                                  f"{int(d['sizes'].max())}, five hydrocarbon families, own periodic boxes, "
                                  f"NVE dt 0.5 fs, {args.precision}", "n_atoms": n, "tune": tune},
           "max_abs_energy_change_eV": drift,
           "energy_change_per_atom": {"median": float(np.median(de)), "max": float(de.max())}}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
