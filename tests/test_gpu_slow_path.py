"""Per-atom overflow handled inside the library (the paper keeps a correct
slow path for whatever its fast kernels do not cover, Sec. 3.2 and 4.3):

* an atom with more than 8 REBO neighbours grows the short list (to 16, 32);
* an atom with more than 48 atoms within R2 + skin grows the intermediate list;
* an atom with more than 64 atoms reachable over three short bonds (the C_ij
  path map kept in LDS) has its pairs within 3 max R2 resolved by the
  sequential path search of the deferred-pair kernel.

Each case is compared with the FP64 oracle at the FP64 bar (energy 1e-12
relative, forces 1e-10 of the RMS force, virial 1e-10), and the statistics
show that the slow path was taken.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL_E, TOL_F, TOL_W = 1e-12, 1e-10, 1e-10


def compare(got, ref, tol_f=TOL_F, tol_e=TOL_E, tol_w=TOL_W):
    e, f, w = [t.cpu().numpy() for t in got]
    eo, fo, wo = ref
    for t in range(4):
        assert abs(e[t] - eo[t]) <= tol_e * max(abs(eo[0]), 1.0), (t, e, eo)
    rms = math.sqrt((fo ** 2).sum(1).mean())
    assert np.abs(f - fo).max() <= tol_f * rms, np.abs(f - fo).max() / rms
    assert np.linalg.norm(w - wo) <= tol_w * max(np.linalg.norm(wo), 1.0)


def fibonacci_sphere(k, radius):
    i = np.arange(k) + 0.5
    phi = np.arccos(1 - 2 * i / k)
    th = math.pi * (1 + 5 ** 0.5) * i
    return radius * np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


def crowded_carbon(nh=10, r=1.45):
    """One carbon with `nh` hydrogens on a sphere of radius r (< the C-H
    REBO cutoff), next to a methane: the carbon has nh REBO neighbours."""
    x = np.concatenate([[[0.0, 0.0, 0.0]], fibonacci_sphere(nh, r),
                        [[4.0, 0.0, 0.0]], [4.0, 0.0, 0.0] + fibonacci_sphere(4, 1.09)]) + 15.0
    s = np.array([0] + [1] * nh + [0] + [1] * 4, np.int32)
    return dict(x=x, species=s, box=np.array([30.0, 30.0, 30.0]), periodic=np.zeros(3, np.int32))


def dense_cluster(seed, n=110, radius=5.0, lo=1.25, h_frac=0.2):
    """Random C/H atoms packed in a sphere at about 0.2 atoms/A^3 (at least
    `lo` apart): carbons have 5-7 neighbours within 2 A, so well over 64
    atoms are reachable from one atom over three short bonds."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(-radius, radius, 3)
        if np.linalg.norm(p) <= radius and all(np.linalg.norm(p - q) > lo for q in pts):
            pts.append(p)
    x = np.array(pts) + 20.0
    s = (rng.random(n) < h_frac).astype(np.int32)
    return dict(x=x, species=s, box=np.array([40.0, 40.0, 40.0]), periodic=np.zeros(3, np.int32))


def test_short_list_grows(oracle):
    from paper_1810_07026_amd import airebo
    d = crowded_carbon()
    ctx = airebo.Context()
    got = ctx.compute(d["x"], d["species"], d["box"], d["periodic"])
    st = ctx.stats()
    assert st["max_short"] >= 10 and st["regrowths"] >= 1, st
    compare(got, oracle.compute(d["x"], d["species"], d["box"], d["periodic"]))


@pytest.mark.parametrize("seed", [1, 2])
def test_path_map_overflow_searched(oracle, seed):
    from paper_1810_07026_amd import airebo
    d = dense_cluster(seed)
    ctx = airebo.Context()
    got = ctx.compute(d["x"], d["species"], d["box"], d["periodic"])
    st = ctx.stats()
    assert st["slow_path_pairs"] > 0, st
    ref = oracle.compute(d["x"], d["species"], d["box"], d["periodic"], stats=True)
    compare(got, ref[:3])
    # the integer counters do not depend on which path resolved a pair
    so = ref[3]
    assert st["lj_in_cut"] == so["lj_in_cut"] and st["cij_zero"] == so["cij_zero"]
    assert st["bstar_queued"] == so["bstar_needed"] and st["bonds"] == so["bonds"]


def test_path_map_overflow_mixed(oracle):
    """The sequential search under mixed precision, at the mixed bar
    (forces 1e-4 of the RMS force, energy 1e-6)."""
    from paper_1810_07026_amd import airebo
    d = dense_cluster(3)
    ctx = airebo.Context(precision=airebo.MIXED)
    got = ctx.compute(d["x"], d["species"], d["box"], d["periodic"])
    assert ctx.stats()["slow_path_pairs"] > 0
    compare(got, oracle.compute(d["x"], d["species"], d["box"], d["periodic"]), tol_f=1e-4, tol_e=1e-6, tol_w=1e-4)


def test_intermediate_list_grows(oracle):
    """A 2.5 A skin puts more than 48 atoms of the dense cluster within
    R2 + skin of an atom."""
    from paper_1810_07026_amd import airebo
    d = dense_cluster(4)
    ctx = airebo.Context(skin=2.5)
    got = ctx.compute(d["x"], d["species"], d["box"], d["periodic"])
    assert ctx.stats()["regrowths"] >= 1
    compare(got, oracle.compute(d["x"], d["species"], d["box"], d["periodic"]))


def test_slow_paths_in_md(oracle):
    """Ten velocity-Verlet steps of 0.1 fs of the dense cluster (path-map
    search every step) follow the oracle's trajectory."""
    import torch
    from paper_1810_07026_amd import airebo, synth
    d = dense_cluster(5, n=90)
    v0 = synth.maxwell_velocities(d["species"], 300.0, np.random.default_rng(7))
    ctx = airebo.Context()
    x = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
    v = torch.tensor(v0, dtype=torch.float64, device="cuda")
    ctx.nve(x, v, d["species"], d["box"], d["periodic"], dt=0.1, nsteps=10, thermo_every=0)
    assert ctx.stats()["slow_path_pairs"] > 0
    xo, vo, _ = oracle.nve(d["x"], v0, d["species"], d["box"], dt=0.1, nsteps=10, thermo_every=10,
                           periodic=d["periodic"])
    assert np.abs(x.cpu().numpy() - xo).max() < 1e-9
    assert np.abs(v.cpu().numpy() - vo).max() < 1e-8
