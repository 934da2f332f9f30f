"""Deterministic sums (a proposed airebo_options.deterministic = 1).

Forces, energies, the virial and the pair counters are summed in 64-bit fixed
point with integer atomics, whose sums do not depend on the order in which the
wavefronts reach them:

* two evaluations, evaluations under either force-kernel schedule, and
  repeated MD runs agree bit for bit; an MD run split into a session of two
  runs repeats the unsplit run bit for bit;
* against the default FP64-atomic sums the results move only by the
  fixed-point rounding: each force contribution is rounded to 2^-46 eV/A
  (1.4e-14) and each energy or virial partial sum to 2^-36 eV (1.5e-11), so
  with a few hundred contributions per atom and about 10^5 partial sums per
  accumulator the bar is max |dF| <= 1e-12 of the RMS force and 1e-12
  relative for the energies and the virial (absolute 1e-9 eV);
* against the oracle at the FP64 parity bar (1e-10 of the RMS force).
"""
import math

import numpy as np
import pytest

from paper_1810_07026_amd import synth

# The option is not in the library.  Its first GPU run (the first test below)
# ended in an illegal memory access that reading the code did not explain, so
# the code was taken out and these tests are not run.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="deterministic sums taken out: their first GPU run faulted, cause not found")]


def _np(t):
    return [a.cpu().numpy() for a in t]


def _dev(a):
    import torch
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def close_to(got, ref, bar=1e-12):
    e, f, w = got
    e0, f0, w0 = ref
    rms = math.sqrt((f0 ** 2).sum(-1).mean())
    assert np.abs(f - f0).max() <= bar * rms, np.abs(f - f0).max() / rms
    assert np.all(np.abs(e - e0) <= bar * np.abs(e0) + 1e-9), (e, e0)
    assert np.abs(w - w0).max() <= bar * np.abs(w0).max() + 1e-9, (w, w0)


def bitwise(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.fixture(scope="module")
def melt():
    return synth.pe_melt()


def test_repeatable_across_calls_and_schedules(melt):
    """The 32,012-atom melt: two evaluations and both schedules bit for bit;
    the default sums within the fixed-point rounding; the same counters."""
    from paper_1810_07026_amd import airebo
    d = melt
    args = (d["x"], d["species"], d["box"], d["periodic"])
    det1 = airebo.Context(deterministic=True, tune={"schedule": 1})
    det2 = airebo.Context(deterministic=True, tune={"schedule": 2})
    ref = airebo.Context()
    a = _np(det1.compute(*args))
    b = _np(det1.compute(*args))
    c = _np(det2.compute(*args))
    r = _np(ref.compute(*args))
    bitwise(a, b)
    bitwise(a, c)
    close_to(a, r)
    s_det, s_ref = det1.stats(), ref.stats()
    for k in ("lj_in_cut", "cij_zero", "bstar_queued", "dsb_nonzero", "bonds"):
        assert s_det[k] == s_ref[k], (k, s_det[k], s_ref[k])


@pytest.mark.parametrize("vdw", [0, 1])
def test_matches_oracle(oracle, vdw):
    """LJ and Morse (AIREBO-M) forms at the FP64 bar against the oracle."""
    from paper_1810_07026_amd import airebo
    d = synth.pe_small(seed=synth.SEED0 + 5)
    args = (d["x"], d["species"], d["box"], d["periodic"])
    from oracle.oracle import MASK_MORSE
    e, f, w = _np(airebo.Context(deterministic=True, vdw=vdw).compute(*args))
    eo, fo, wo = oracle.compute(*args, mask=7 | (MASK_MORSE if vdw else 0))
    rms = math.sqrt((fo ** 2).sum(1).mean())
    assert np.abs(f - fo).max() <= 1e-10 * rms
    assert np.all(np.abs(e - eo) <= 1e-12 * max(abs(eo[0]), 1.0))
    assert np.abs(w - wo).max() <= 1e-10 * np.abs(wo).max()


def test_mixed_precision():
    """Mixed precision: repeatable, and the default mixed sums within the
    fixed-point rounding (the FP32 arithmetic itself is the same)."""
    from paper_1810_07026_amd import airebo
    d = synth.pe_small(seed=synth.SEED0 + 6)
    args = (d["x"], d["species"], d["box"], d["periodic"])
    det = airebo.Context(precision=airebo.MIXED, deterministic=True)
    a, b = _np(det.compute(*args)), _np(det.compute(*args))
    bitwise(a, b)
    close_to(a, _np(airebo.Context(precision=airebo.MIXED).compute(*args)))


def test_md_repeats_bit_for_bit():
    """Two 40-step runs from one state, and a session of 20 + 20 steps, end in
    the same positions, velocities and thermo rows bit for bit."""
    from paper_1810_07026_amd import airebo
    d = synth.pe_small(seed=synth.SEED0 + 3)
    ctx = airebo.Context(deterministic=True)
    runs = []
    for _ in range(2):
        x, v = _dev(d["x"]), _dev(d["v"])
        th = ctx.nve(x, v, d["species"], d["box"], dt=0.5, nsteps=40, thermo_every=20)
        runs.append((x.cpu().numpy(), v.cpu().numpy(), th.cpu().numpy()))
    bitwise(runs[0], runs[1])
    x, v = _dev(d["x"]), _dev(d["v"])
    ctx.md_begin(x, v, d["species"], d["box"])
    ta = ctx.md_run(20, thermo_every=20).cpu().numpy()
    tb = ctx.md_run(20, thermo_every=20).cpu().numpy()
    xs, vs = ctx.md_state()
    ctx.md_end()
    assert np.array_equal(xs.cpu().numpy(), runs[0][0])
    assert np.array_equal(vs.cpu().numpy(), runs[0][1])
    assert np.array_equal(ta[:, 1:5], runs[0][2][:2, 1:5])
    assert np.array_equal(tb[-1, 1:5], runs[0][2][-1, 1:5])
    # against the default sums over the same run: the trajectories stay within 1e-9 A
    x, v = _dev(d["x"]), _dev(d["v"])
    airebo.Context().nve(x, v, d["species"], d["box"], dt=0.5, nsteps=40, thermo_every=0)
    dx = x.cpu().numpy() - runs[0][0]
    dx -= d["box"] * np.round(dx / d["box"])
    assert np.abs(dx).max() < 1e-9


def test_batch():
    """A batch of 7 systems: repeatable per system, and the default batch
    within the fixed-point rounding."""
    from paper_1810_07026_amd import airebo
    d = synth.batch_systems(7, nmin=30, nmax=400, seed=77)
    args = (d["x"], d["species"], d["sizes"], d["boxes"], d["periodic"])
    det = airebo.Context(deterministic=True)
    a, b = _np(det.batch_compute(*args)), _np(det.batch_compute(*args))
    bitwise(a, b)
    close_to(a, _np(airebo.Context().batch_compute(*args)))


def test_allocation_free_entry_point():
    """airebo_compute_static with deterministic sums equals airebo_compute
    with them within the fixed-point rounding, and repeats bit for bit."""
    from paper_1810_07026_amd import airebo
    d = synth.pe_small(seed=synth.SEED0 + 7)
    args = (d["x"], d["species"], d["box"], d["periodic"])
    ctx = airebo.Context(deterministic=True)
    a, b = _np(ctx.compute_static(*args)), _np(ctx.compute_static(*args))
    bitwise(a, b)
    close_to(a, _np(ctx.compute(*args)))


def test_rejected_where_not_supported():
    """Single precision (FP32 force sums) and the surrogate refuse the option."""
    from paper_1810_07026_amd import airebo, surrogate
    with pytest.raises(airebo.AireboError) as ei:
        airebo.Context(precision=airebo.SINGLE, deterministic=True)
    assert ei.value.code == -1
    d = synth.pe_small(seed=synth.SEED0 + 8)
    nn = airebo.Surrogate(path=surrogate.WEIGHTS)
    with pytest.raises(airebo.AireboError) as ei:
        nn.compute(airebo.Context(deterministic=True), d["x"], d["species"], d["box"], d["periodic"])
    assert ei.value.code == -1
