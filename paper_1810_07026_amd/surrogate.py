"""Training and evaluation driver of the learned surrogate.

Every numerical step runs in the library's kernels:
  - AIREBO FP64 labels (airebo_compute) and the NVE that generates frames;
  - descriptors and their column moments;
  - the ensemble's loss gradient and Adam;
  - surrogate evaluation and dynamics.
This module only sequences those calls and keeps the labelled frames in
device memory.

Training data reading: labelled atom-centred environments from snapshots of
an AIREBO trajectory of the polyethylene melt (106 x C100H202, 32,012 atoms).
Half of the frames are at 300 K and half after heating to 600 K.  Each frame
contributes every atom's force label plus one energy label.  32 frames give
~1.02e6 labelled environments.

Usage (on the GPU):
  python -m paper_1810_07026_amd.surrogate train [--frames 32] [--steps 4000] [--out PATH]
"""
import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "data", "surrogate_pe_melt.bin")
THRESHOLD = 0.1          # eV/A: ensemble force spread above which AIREBO evaluates the step
STD_FLOOR = 0.05         # descriptor standard deviations below this are raised to it


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def label_frames(ctx, d, n_frames=32, stride=40, equil=400, seed=1810070264, hot=True):
    """AIREBO-labelled snapshots of an NVE trajectory (device tensors).

    Returns a list of (x [n,3], forces [n,3], energy) with x and forces on
    the device.  The second half of the frames comes after the velocities
    are scaled to 600 K and equilibrated for `equil` steps."""
    import torch
    from paper_1810_07026_amd import synth
    s, box, per = d["species"], d["box"], d["periodic"]
    x = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
    v = torch.tensor(synth.maxwell_velocities(s, 300.0, np.random.default_rng(seed)), dtype=torch.float64,
                     device="cuda")
    ctx.nve(x, v, s, box, per, nsteps=equil, thermo_every=0)
    frames = []
    for k in range(n_frames):
        if hot and k == n_frames // 2:
            v.mul_(math.sqrt(2.0))
            ctx.nve(x, v, s, box, per, nsteps=equil, thermo_every=0)
        ctx.nve(x, v, s, box, per, nsteps=stride, thermo_every=0)
        e, f, _ = ctx.compute(x, s, box, per)
        frames.append((x.clone(), f.clone(), float(e[0])))
    return frames, (x, v)


def fit_normalisation(nn, ctx, frames, s, box, per, scale=1.0):
    """Descriptor mean and inverse deviation over the frames (library
    moments kernel); output shift = mean energy per atom."""
    n = len(s)
    s1 = np.zeros(nn.dim)
    s2 = np.zeros(nn.dim)
    rows = 0
    for x, _, _ in frames:
        G = nn.descriptors(ctx, x, s, box, per)
        a, b = nn.moments(G)
        s1 += a
        s2 += b
        rows += n
    mean = s1 / rows
    std = np.sqrt(np.maximum(s2 / rows - mean ** 2, 0.0))
    istd = 1.0 / np.maximum(std, STD_FLOOR)
    e_atom = float(np.mean([e for _, _, e in frames])) / n
    nn.set_norm(mean.astype(np.float32), istd.astype(np.float32), scale, [e_atom, e_atom])
    return mean, istd, e_atom


def train(nn, ctx, frames, s, box, per, steps=4000, lr0=2e-3, lr1=2e-5, w_energy_per_atom=1.0, seed=7,
          every=200):
    """Adam on the per-member loss, one frame per step.

    The loss of member m is (1/3n) sum_i |F_m,i - F_target,i|^2
    + w (E_m - E_target)^2 / n^2.  The learning rate follows a cosine from
    lr0 to lr1.  Returns the history [(step, mean loss)]."""
    n = len(s)
    wF = 1.0 / (3 * n)
    wE = w_energy_per_atom / n ** 2
    rng = np.random.default_rng(seed)
    order = np.concatenate([rng.permutation(len(frames)) for _ in range(steps // len(frames) + 1)])
    hist = []
    t0 = time.perf_counter()
    run = []
    for it in range(steps):
        x, f, e = frames[order[it]]
        lr = lr1 + 0.5 * (lr0 - lr1) * (1 + math.cos(math.pi * it / max(steps - 1, 1)))
        L = nn.gradient(ctx, x, s, box, f, e, wF, wE, per)
        nn.adam(lr)
        run.append(L.mean())
        if (it + 1) % every == 0 or it == 0:
            hist.append((it + 1, float(np.mean(run))))
            log(f"surrogate: step {it + 1}/{steps} loss {np.mean(run):.5g} (eV/A)^2 lr {lr:.3g} "
                f"{time.perf_counter() - t0:.1f} s")
            run = []
    return hist


def force_error(nn, ctx, x, s, box, per, f_ref):
    """Surrogate (no fallback) forces against reference forces on one frame."""
    import torch
    e, f, w, sp, info = nn.compute(ctx, x, s, box, per, threshold=1e30, want_spread=True)
    f_ref = torch.as_tensor(f_ref, dtype=torch.float64, device=f.device)
    d2 = ((f - f_ref) ** 2).sum(1)
    r2 = (f_ref ** 2).sum(1)
    sp = sp.double()
    return {"force_rms_err_eVA": float(d2.mean().sqrt()), "force_rms_ref_eVA": float(r2.mean().sqrt()),
            "force_rel_rms_err": float((d2.mean() / r2.mean()).sqrt()),
            "force_max_err_eVA": float(d2.max().sqrt()),
            "spread_max_eVA": float(sp.max()), "spread_p999_eVA": float(torch.quantile(sp[:1 << 24], 0.999)),
            "atoms_above_threshold": int((sp > THRESHOLD).sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train"])
    ap.add_argument("--frames", type=int, default=32)
    ap.add_argument("--stride", type=int, default=40)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--models", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1810070265)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    import torch
    from paper_1810_07026_amd import airebo, synth
    d = synth.pe_melt()
    s, box, per = d["species"], d["box"], d["periodic"]
    ctx = airebo.Context()
    t0 = time.perf_counter()
    frames, (x, v) = label_frames(ctx, d, args.frames, args.stride)
    torch.cuda.synchronize()
    log(f"surrogate: {len(frames)} labelled frames of {len(s)} atoms in {time.perf_counter() - t0:.1f} s")
    # held-out frame: 200 steps after the last training frame
    ctx.nve(x, v, s, box, per, nsteps=200, thermo_every=0)
    e_t, f_t, _ = ctx.compute(x, s, box, per)
    nn = airebo.Surrogate(nmodels=args.models)
    nn.set_params(synth.nn_init_weights(args.models, args.seed))
    fit_normalisation(nn, ctx, frames, s, box, per)
    before = force_error(nn, ctx, x, s, box, per, f_t)
    t1 = time.perf_counter()
    train(nn, ctx, frames, s, box, per, steps=args.steps, lr0=args.lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    after = force_error(nn, ctx, x, s, box, per, f_t)
    log(f"surrogate: trained in {t_train:.1f} s; held-out frame before {before} after {after}")
    nn.save(args.out)
    log(f"surrogate: weights written to {args.out}")


if __name__ == "__main__":
    main()
