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
    ap.add_argument("--potential", choices=["airebo", "airebo_m", "rebo"], default="airebo",
                    help="AIREBO, AIREBO-M (Morse in place of LJ, FP64) or REBO alone (no LJ, no torsion)")
    ap.add_argument("--cnt-cells", type=int, default=40, help="nanotube bundle: translational cells per tube")
    ap.add_argument("--cnt-grid", type=int, default=4, help="nanotube bundle: tubes per side of the square lattice")
    ap.add_argument("--thermo-out", default="",
                    help="conservation workload: also write the thermo rows (step PE KE Etot T rebuilds) to this text file")
    ap.add_argument("--tune", default="", help="JSON launch shapes (batch512 workload)")
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

    if args.workload == "hybrid_1m":
        # untimed preparation: velocity quench (NVE in short bursts, velocities
        # zeroed after each) relaxes the strain of the assembled slabs, then
        # fresh 300 K velocities
        log("bench: hybrid preparation: 20 quench cycles of 10 steps (untimed)")
        for _ in range(20):
            ctx.nve(x, v, d["species"], box, per, nsteps=10, thermo_every=0)
            v.zero_()
        v.copy_(torch.tensor(synth.maxwell_velocities(d["species"], 300.0, np.random.default_rng(1810070267)),
                             dtype=torch.float64, device=dev))
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

    # accuracy and the other forms are measured on the state the timed run
    # ends in (equilibrated); the per-kernel profile continues from it
    xf, vf = x.clone(), v.clone()
    xf_h = xf.cpu().numpy()
    # per-kernel device times (HIP events on the launch stream) and work counts
    e0, f0, _ = ctx.compute(xf, d["species"], box, per)
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
                # the committed counter profile is of the melt workload
                "traffic": (counter_traffic(cand, args.precision)
                            if args.workload == "pe_melt_32k" and args.potential == "airebo" else None),
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
            eo, fo, wo = orc.compute(xf_h, d["species"], box, per, mask=omask)
            t3 = time.perf_counter()
            cpu = {"value": n / (t3 - t2), "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
                   "sample": f"one full FP64 force evaluation (= one MD step) of the {n}-atom system, "
                             f"{t3 - t2:.1f} s", "host_cpu": host_cpu()}
            # the same evaluation on one thread
            log("bench: oracle on 1 thread, one force evaluation")
            t4 = time.perf_counter()
            Oracle(nthreads=1).compute(xf_h, d["species"], box, per)
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
            _, fo, _ = orc.compute(xf_h, d["species"], box, per, mask=omask, sel=sel)
            t3 = time.perf_counter()
            cpu = {"value": len(sel) / (t3 - t2), "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
                   "sample": f"exact FP64 forces on {len(sel)} random atoms of the {n}-atom system "
                             f"(every term touching them), {t3 - t2:.1f} s"}
            fo, fgs = fo[sel], fg[sel]
            rms = math.sqrt((fo ** 2).sum(1).mean())
            ferr = {"force_rms_err_eVA": float(math.sqrt(((fgs - fo) ** 2).sum(1).mean())), "force_rms_eVA": rms,
                    "force_rel_err_max": float(np.abs(fgs - fo).max() / rms), "sampled_atoms": len(sel)}

    forms = None
    if not args.no_forms and args.workload == "pe_melt_32k" and args.potential == "airebo":
        forms = measure_forms(d, xf, vf, args, value, fo if ferr is not None and n <= 100000 else None)

    out = {
        "metric": "AIREBO atom-steps/s on 1 GPU",
        "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPES[args.precision],
        "data": "synthetic (seeded generators)",
        "config": {"workload": ("" if args.potential == "airebo" else
                                {"airebo_m": "AIREBO-M (Morse) on ", "rebo": "REBO only on "}[args.potential]) +
                               (f"polyethylene melt 106 x C100H202, {n} atoms, 0.85 g/cm^3, "
                                f"{box[0]:.2f} A periodic cube, 300 K, NVE dt 0.5 fs, {args.precision}"
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
        "energy_drift": {"slope_eV_per_atom_per_ps": slope, "max_rel": maxrel, "rebuilds": rebuilds},
        "work": {k: st[k] for k in ("lj_in_cut", "cij_zero", "bstar_queued", "dsb_nonzero", "bonds")},
        "kernels_us": {k: round(v["avg_us"], 3) for k, v in kern.items()},
        "forms": forms,
    }
    print(json.dumps(out))


def force_err(f, fo):
    f = np.asarray(f, float)
    rms = math.sqrt((fo ** 2).sum(1).mean())
    e = math.sqrt(((f - fo) ** 2).sum(1).mean())
    return {"force_rms_err_eVA": e, "force_rel_rms_err": e / rms}


def timed_nve(run, n, steps, warmup):
    """atom-steps/s of run(nsteps) after a warm-up call (device-synchronised)."""
    import torch
    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    extra = run(steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    return n * steps / sec, 1e3 * sec / steps, extra


def measure_forms(d, x0, v0, args, fp64_value, fo):
    """Mixed and single precision and the surrogate on the same system as the FP64 line,
    from the state its timed run ended in: atom-steps/s of NVE and force RMS
    error against the CPU oracle (when it was evaluated) or the FP64 GPU
    forces at that state."""
    import torch
    from paper_1810_07026_amd import airebo, surrogate
    s, box, per = d["species"], d["box"], d["periodic"]
    n = len(s)
    ctx = airebo.Context()
    ref_kind = "cpu_oracle"
    if fo is None:
        fo = ctx.compute(x0, s, box, per)[1].cpu().numpy()
        ref_kind = "fp64_gpu"
    forms = {"reference": ref_kind, "steps": args.form_steps}
    # mixed and single precision
    for name, prec in (("mixed", airebo.MIXED), ("single", airebo.SINGLE)):
        ctxm = airebo.Context(precision=prec)
        xm, vm = x0.clone(), v0.clone()
        val, ms, _ = timed_nve(lambda k: ctxm.nve(xm, vm, s, box, per, nsteps=k, thermo_every=0), n,
                               args.form_steps, args.warmup)
        fm = ctxm.compute(x0, s, box, per)[1].cpu().numpy()
        forms[name] = dict(force_err(fm, fo), value=val, ms_per_step=ms, speedup_vs_fp64=val / fp64_value)
        log(f"bench: {name} {val:.4g} atom-steps/s, force rel rms err {forms[name]['force_rel_rms_err']:.3g}")
        del ctxm
    # learned surrogate
    if not os.path.exists(surrogate.WEIGHTS):
        forms["surrogate"] = {"error": "no trained weights (python -m paper_1810_07026_amd.surrogate train)"}
        return forms
    nn = airebo.Surrogate(path=surrogate.WEIGHTS)
    e, f, _, sp, info = nn.compute(ctx, x0, s, box, per, threshold=1e30, want_spread=True)
    sur = dict(force_err(f.cpu().numpy(), fo), threshold_eVA=surrogate.THRESHOLD,
               max_spread_eVA=info["max_spread"], atoms_above_threshold=int((sp > surrogate.THRESHOLD).sum()))
    for key, thr in (("with_fallback", surrogate.THRESHOLD), ("no_fallback", 1e30)):
        xs, vs = x0.clone(), v0.clone()
        val, ms, fb = timed_nve(lambda k: nn.nve(ctx, xs, vs, s, box, per, nsteps=k, thermo_every=0,
                                                 threshold=thr)[1], n, args.form_steps, args.warmup)
        # the call's initial force evaluation is counted with its steps
        sur[key] = {"value": val, "ms_per_step": ms, "speedup_vs_fp64": val / fp64_value,
                    "fallback_evaluations": fb, "fallback_rate": fb / (args.form_steps + 1)}
        log(f"bench: surrogate ({key}) {val:.4g} atom-steps/s, fallbacks {fb}/{args.form_steps}")
    forms["surrogate"] = sur
    return forms


def bench_surrogate(args):
    """Learned surrogate on a ~1e6-atom polyethylene melt (the 32,012-atom melt
    tiled 3 x 3 x 3 = 864,324 atoms, fresh 300 K velocities, decorrelated by
    untimed mixed-precision NVE), against AIREBO FP64 and mixed on the same
    state; force errors against the FP64 GPU forces on every atom and
    against the CPU oracle on sampled atoms."""
    import torch
    from paper_1810_07026_amd import airebo, surrogate, synth
    d = synth.tile(synth.pe_melt(), (3, 3, 3))
    s, box, per = d["species"], d["box"], d["periodic"]
    n = len(s)
    rng = np.random.default_rng(1810070266)
    x = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
    v = torch.tensor(synth.maxwell_velocities(s, 300.0, rng), dtype=torch.float64, device="cuda")
    ctx = airebo.Context()
    ctxm = airebo.Context(precision=airebo.MIXED)
    log(f"bench: surrogate workload n={n}; decorrelating replicas ({args.warmup} mixed NVE steps, untimed)")
    ctxm.nve(x, v, s, box, per, nsteps=max(args.warmup, 100), thermo_every=0)
    torch.cuda.synchronize()
    x0, v0 = x.clone(), v.clone()
    e64, f64, _ = ctx.compute(x0, s, box, per)
    f64 = f64.cpu().numpy()
    nn = airebo.Surrogate(path=surrogate.WEIGHTS)
    err = surrogate.force_error(nn, ctx, x0, s, box, per, f64)
    fm = ctxm.compute(x0, s, box, per)[1].cpu().numpy()
    steps = args.steps
    res = {}
    for key, run in (
            ("fp64", lambda k: ctx.nve(x, v, s, box, per, nsteps=k, thermo_every=0)),
            ("mixed", lambda k: ctxm.nve(x, v, s, box, per, nsteps=k, thermo_every=0)),
            ("surrogate_with_fallback", lambda k: nn.nve(ctx, x, v, s, box, per, nsteps=k, thermo_every=0,
                                                         threshold=surrogate.THRESHOLD)[1]),
            ("surrogate_no_fallback", lambda k: nn.nve(ctx, x, v, s, box, per, nsteps=k, thermo_every=0,
                                                       threshold=1e30)[1])):
        x.copy_(x0)
        v.copy_(v0)
        val, ms, extra = timed_nve(run, n, steps, 5)
        res[key] = {"value": val, "ms_per_step": ms}
        if key.startswith("surrogate"):
            res[key]["fallback_steps"] = extra
        log(f"bench: {key} {val:.4g} atom-steps/s ({ms:.3f} ms/step)")
    for k in res:
        res[k]["speedup_vs_fp64"] = res[k]["value"] / res["fp64"]["value"]
    # per-kernel device time of the surrogate step
    x.copy_(x0)
    v.copy_(v0)
    prof = nn.profile_nve(ctx, x, v, s, box, per, nsteps=5, threshold=1e30)
    kern = {k: round(1e3 * ms / c, 2) for k, (ms, c) in prof.items() if c and k.startswith("nn")}
    # CPU oracle on sampled atoms
    cpu = None
    acc_or = None
    if not args.no_cpu_baseline:
        from oracle.oracle import Oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        sel = np.sort(rng.choice(n, 2048, replace=False)).astype(np.int32)
        xh = x0.cpu().numpy()
        t2 = time.perf_counter()
        _, fo, _ = Oracle(nthreads=threads).compute(xh, s, box, per, sel=sel)
        t3 = time.perf_counter()
        fo = fo[sel]
        fn = nn.compute(ctx, x0, s, box, per, threshold=1e30)[1].cpu().numpy()[sel]
        acc_or = {"surrogate": force_err(fn, fo), "fp64_gpu": force_err(f64[sel], fo),
                  "mixed_gpu": force_err(fm[sel], fo), "sampled_atoms": len(sel)}
        cpu = {"value": len(sel) / (t3 - t2), "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
               "sample": f"exact FP64 AIREBO forces on {len(sel)} random atoms of the {n}-atom melt, "
                         f"{t3 - t2:.1f} s"}
    out = {"metric": "AIREBO atom-steps/s on 1 GPU", "value": res["surrogate_with_fallback"]["value"],
           "unit": "atom-steps/s", "n_gpus": 1, "steps": steps, "warmup": 5,
           "ms_per_step": res["surrogate_with_fallback"]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32+f64", "data": "synthetic (seeded generators)",
           "config": {"workload": f"learned surrogate (4-member ensemble, fallback at {surrogate.THRESHOLD} eV/A) on "
                                  f"a polyethylene melt of {n} atoms (106 x C100H202 tiled 3x3x3, "
                                  f"{box[0]:.1f} A periodic cube, 300 K), NVE dt 0.5 fs", "n_atoms": n},
           "forms": res, "surrogate_error_vs_fp64_gpu": err,
           "mixed_error_vs_fp64_gpu": force_err(fm, f64), "accuracy_vs_oracle": acc_or,
           "cpu_baseline": cpu, "kernels_us": kern}
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
        np.savetxt(args.thermo_out, th, fmt="%.10g", header="step PE_eV KE_eV Etot_eV T_K rebuilds")
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
