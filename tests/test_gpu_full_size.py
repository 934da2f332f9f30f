"""Parity at the benchmarked sizes, in the launch configuration bench.py times.

* The 32,012-atom polyethylene melt (106 x C100H202, the headline workload):
  GPU energy, every force and the virial against one full oracle evaluation,
  FP64 at the FP64 bar, mixed and single precision at their own bars.
* The 25,600-atom nanotube bundle, each precision at its bar.
* The 512-system batch (565,367 atoms) with the launch shapes the autotuner
  cached for it: the smallest and the largest system of each family,
  taken whole from the batched result, against the oracle on that system
  alone, FP64, mixed and single.

Bars: the FP64 bar of the parity tests (energy 1e-12 relative, max force
error 1e-10 of the RMS force, virial 1e-10 relative; only summation order
and last-bit differences of the math libraries separate the two sides) and
the mixed bar derived there (force 1e-4 of the RMS force, energy 1e-6) and
the single bar derived there (the mixed force bar, FP32 force sums, and the
force change from rounding positions to FP32, evaluated by the oracle;
energy 1e-5).
"""
import math

import numpy as np
import pytest

from paper_1810_07026_amd import synth

pytestmark = pytest.mark.gpu

TOL_E, TOL_F, TOL_W = 1e-12, 1e-10, 1e-10
TOL_MIXED_F, TOL_MIXED_E = 1e-4, 1e-6
TOL_SINGLE_E = 1e-5
U32 = 2.0 ** -24
PRECS = {"fp64": 0, "mixed": 1, "single": 2}


def tol_single_f(oracle, x, species, box, per, fo, rms):
    """Largest per-atom force error (eV/A) of single precision: FP32 term
    arithmetic (the mixed bar), FP32 sums of ~200 terms of up to 30 eV/A, and
    4 times the force change the oracle finds when the positions are rounded
    to FP32 (derivation beside the single-precision parity tests)."""
    x32 = np.asarray(x, np.float64).astype(np.float32).astype(np.float64)
    fpos = oracle.compute(x32, species, box, per)[1]
    return TOL_MIXED_F * rms + 4.0 * float(np.abs(fpos - fo).max()) + 200.0 * 30.0 * U32


def check(e, f, w, eo, fo, wo, prec, label, tol_single=None):
    rms = math.sqrt((fo ** 2).sum(1).mean())
    ferr = np.abs(f - fo).max() / rms
    if prec == "single":
        assert ferr * rms <= tol_single, (label, ferr * rms, tol_single)
        assert abs(e[0] - eo[0]) <= TOL_SINGLE_E * max(abs(eo[0]), 1.0), (label, e[0], eo[0])
    elif prec == "fp64":
        assert ferr <= TOL_F, (label, ferr)
        for t in range(4):
            assert abs(e[t] - eo[t]) <= TOL_E * max(abs(eo[t]), 1e-3 * abs(eo[0]), 1.0), (label, t, e, eo)
        assert np.linalg.norm(w - wo) <= TOL_W * np.linalg.norm(wo) + 1e-12, (label, w, wo)
    else:
        assert ferr <= TOL_MIXED_F, (label, ferr)
        assert abs(e[0] - eo[0]) <= TOL_MIXED_E * max(abs(eo[0]), 1.0), (label, e[0], eo[0])
    return ferr


@pytest.fixture(scope="module")
def melt(oracle):
    d = synth.pe_melt()
    return d, oracle.compute(d["x"], d["species"], d["box"], d["periodic"])


@pytest.mark.parametrize("prec", ["fp64", "mixed", "single"])
def test_melt_32k_full(melt, oracle, prec):
    from paper_1810_07026_amd import airebo
    d, (eo, fo, wo) = melt
    assert len(d["species"]) == 32012
    ctx = airebo.Context(precision=PRECS[prec])
    try:
        e, f, w = ctx.compute(d["x"], d["species"], d["box"], d["periodic"])
        e, f, w = e.cpu().numpy(), f.cpu().numpy(), w.cpu().numpy()
    finally:
        ctx.close()
    tol = None
    if prec == "single":
        tol = tol_single_f(oracle, d["x"], d["species"], d["box"], d["periodic"], fo,
                           math.sqrt((fo ** 2).sum(1).mean()))
    ferr = check(e, f, w, eo, fo, wo, prec, f"melt {prec}", tol)
    print(f"melt 32k {prec}: max force error / RMS force {ferr:.3g}")
    # Newton's third law over the whole periodic system (FP32 sums: to their rounding)
    assert np.abs(f.sum(0)).max() <= (1e-6 if prec == "single" else 1e-9) * np.abs(f).sum()


@pytest.fixture(scope="module")
def cnt(oracle):
    """The nanotube bundle after 1,000 FP64 steps of 0.5 fs, the state the
    bench's timed run ends in (the perfect lattice has RMS forces of only
    0.19 eV/A, below the scale the relative force bars are derived for)."""
    import torch
    from paper_1810_07026_amd import airebo
    d = dict(synth.nanotube_bundle())
    c64 = airebo.Context()
    try:
        x = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
        v = torch.tensor(d["v"], dtype=torch.float64, device="cuda")
        c64.nve(x, v, d["species"], d["box"], d["periodic"], dt=0.5, nsteps=1000, thermo_every=0)
        d["x"] = x.cpu().numpy()
    finally:
        c64.close()
    return d, oracle.compute(d["x"], d["species"], d["box"], d["periodic"])


@pytest.mark.parametrize("prec", ["fp64", "mixed", "single"])
def test_cnt_bundle_full(cnt, oracle, prec):
    """The 25,600-atom bundle of 16 (10,10) nanotubes (the nanotube workload
    bench.py times) at the end state of 1,000 steps: every force, the energy
    terms and the virial against one oracle evaluation, each precision at its
    bar."""
    from paper_1810_07026_amd import airebo
    d, (eo, fo, wo) = cnt
    assert len(d["species"]) == 25600
    ctx = airebo.Context(precision=PRECS[prec])
    try:
        e, f, w = ctx.compute(d["x"], d["species"], d["box"], d["periodic"])
        e, f, w = e.cpu().numpy(), f.cpu().numpy(), w.cpu().numpy()
    finally:
        ctx.close()
    rms = math.sqrt((fo ** 2).sum(1).mean())
    tol = None
    if prec == "single":
        tol = tol_single_f(oracle, d["x"], d["species"], d["box"], d["periodic"], fo, rms)
    ferr = check(e, f, w, eo, fo, wo, prec, f"cnt {prec}", tol)
    print(f"cnt bundle {prec}: max force error / RMS force {ferr:.3g}")
    assert np.abs(f.sum(0)).max() <= (1e-6 if prec == "single" else 1e-9) * np.abs(f).sum()


def test_melt_32k_single_hot(melt, oracle):
    """Single precision at a hot state of the melt: after 1,000 FP64 steps of
    0.5 fs (the generated melt relaxes and heats towards 760 K, with harder
    contacts than the start state), against the oracle at that state."""
    import torch
    from paper_1810_07026_amd import airebo
    d, _ = melt
    c64 = airebo.Context()
    try:
        x = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
        v = torch.tensor(d["v"], dtype=torch.float64, device="cuda")
        c64.nve(x, v, d["species"], d["box"], d["periodic"], dt=0.5, nsteps=1000, thermo_every=0)
        xh = x.cpu().numpy()
    finally:
        c64.close()
    eo, fo, wo = oracle.compute(xh, d["species"], d["box"], d["periodic"])
    cs = airebo.Context(precision=airebo.SINGLE)
    try:
        e, f, w = cs.compute(xh, d["species"], d["box"], d["periodic"])
        e, f, w = e.cpu().numpy(), f.cpu().numpy(), w.cpu().numpy()
    finally:
        cs.close()
    rms = math.sqrt((fo ** 2).sum(1).mean())
    tol = tol_single_f(oracle, xh, d["species"], d["box"], d["periodic"], fo, rms)
    ferr = check(e, f, w, eo, fo, wo, "single", "hot melt single", tol)
    print(f"hot melt single: RMS force {rms:.3g} eV/A, max force error {ferr * rms:.3g} eV/A, bound {tol:.3g}")


@pytest.mark.parametrize("prec", ["fp64", "mixed", "single"])
def test_batch_512_full(oracle, prec):
    import torch
    from paper_1810_07026_amd import airebo, autotune
    d = synth.batch_cached(512)
    n = int(d["sizes"].sum())
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    tune = autotune.lookup(autotune.workload_key(arch, n, 512, "mixed")) or {}
    ctx = airebo.Context(precision=PRECS[prec], tune=tune)
    try:
        e, f, w = ctx.batch_compute(d["x"], d["species"], d["sizes"], d["boxes"], d["periodic"])
        e, f, w = e.cpu().numpy(), f.cpu().numpy(), w.cpu().numpy()
    finally:
        ctx.close()
    off = np.concatenate([[0], np.cumsum(d["sizes"])])
    for fam in range(len(synth.FAMILIES)):
        ks = [k for k in range(512) if k % len(synth.FAMILIES) == fam]
        # the smallest and the largest system of the family
        for k in (min(ks, key=lambda q: d["sizes"][q]), max(ks, key=lambda q: d["sizes"][q])):
            a, b = off[k], off[k + 1]
            eo, fo, wo = oracle.compute(d["x"][a:b], d["species"][a:b], d["boxes"][k], d["periodic"][k])
            tol = None
            if prec == "single":
                tol = tol_single_f(oracle, d["x"][a:b], d["species"][a:b], d["boxes"][k], d["periodic"][k], fo,
                                   math.sqrt((fo ** 2).sum(1).mean()))
            ferr = check(e[k], f[a:b], w[k], eo, fo, wo, prec, f"batch {prec} system {k}", tol)
            print(f"batch {prec} system {k} ({synth.FAMILIES[fam]}, {b - a} atoms): "
                  f"max force error / RMS {ferr:.3g}")
