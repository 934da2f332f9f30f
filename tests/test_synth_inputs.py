"""Checks of the seeded input generators (host only).

The 512-system batch must hold only saturated molecules: every H bonded to
exactly one atom and every C to three or four, under each system's own
periodic images.  A bare carbon (a radical) reacts within picoseconds of
NVE, heats its box and ends in a blow-up that no force kernel can be
blamed for; an earlier flake builder produced such chain ends.
"""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1810_07026_amd import synth

# bonded-distance windows of the clean check (A)
CC_MAX, CH_MAX = 1.6, 1.15


def bonded_degree(x, s, box):
    """Number of bonded neighbours of every atom (periodic cube)."""
    tree = cKDTree(np.mod(x, box), boxsize=box)
    pairs = tree.query_pairs(CC_MAX, output_type="ndarray")
    a, b = pairs[:, 0], pairs[:, 1]
    d = x[a] - x[b]
    d -= box * np.round(d / box)
    r = np.linalg.norm(d, axis=1)
    kind = s[a] + s[b]
    keep = ((kind == 0) & (r < CC_MAX)) | ((kind == 1) & (r < CH_MAX))
    deg = np.zeros(len(s), int)
    np.add.at(deg, a[keep], 1)
    np.add.at(deg, b[keep], 1)
    return deg


@pytest.mark.parametrize("nx,ny", [(nx, ny) for nx in range(2, 5) for ny in range(2, 4)])
def test_flake_is_fused_rings(nx, ny):
    """Every flake carbon has two or three carbon neighbours; two-fold carbons
    carry one H; the count matches a parallelogram of fused hexagons."""
    x, s = synth.graphene_flake(nx, ny)
    C = x[s == 0]
    d = np.linalg.norm(C[:, None] - C[None], axis=2)
    ncc = ((d > 0.1) & (d < 1.42 * 1.1)).sum(1)
    assert set(np.unique(ncc)) <= {2, 3}
    assert (s == 1).sum() == (ncc == 2).sum()
    assert len(C) == 2 * (nx + 1) * (ny + 1) - 2
    assert synth._clean(x, s)


def test_clean_rejects_bare_carbon():
    """A carbon left with two neighbours (two H of a methyl removed) is
    rejected even though every remaining distance is fine."""
    x, s = synth.alkane(3)
    d = np.linalg.norm(x - x[0], axis=1)
    h_on_c0 = np.where((s == 1) & (d < CH_MAX))[0]
    assert len(h_on_c0) == 3
    keep = np.ones(len(s), bool)
    keep[h_on_c0[:2]] = False
    assert synth._clean(x, s)
    assert not synth._clean(x[keep], s[keep])


def test_batch_molecules_are_saturated():
    d = synth.batch_cached(512)
    off = np.concatenate([[0], np.cumsum(d["sizes"])])
    assert len(d["sizes"]) == 512
    assert d["sizes"].min() >= 30 and d["sizes"].max() <= 5500
    for k in range(512):
        a, b = off[k], off[k + 1]
        s = d["species"][a:b]
        deg = bonded_degree(d["x"][a:b], s, d["boxes"][k][0])
        assert np.all(deg[s == 1] == 1), f"system {k}: H with {sorted(set(deg[s == 1]))} neighbours"
        assert np.all((deg[s == 0] >= 3) & (deg[s == 0] <= 4)), \
            f"system {k}: C with {sorted(set(deg[s == 0]))} neighbours"


@pytest.mark.parametrize("n,m", [(5, 5), (10, 10), (10, 0), (8, 4)])
def test_nanotube_geometry(n, m):
    """A rolled (n, m) tube: every carbon has exactly three neighbours at the
    graphene bond length (minimum image along the periodic axis; curvature
    shortens the chord by well under 1%), and the radius is |C| / 2 pi with
    |C| = a sqrt(n^2 + nm + m^2), a = sqrt(3) 1.42 A."""
    x, s, box, per = synth.nanotube(n, m, 3)
    assert (s == 0).all() and list(per) == [0, 0, 1]
    d = x[:, None, :] - x[None, :, :]
    d[..., 2] -= box[2] * np.round(d[..., 2] / box[2])
    r = np.linalg.norm(d, axis=2)
    np.fill_diagonal(r, np.inf)
    near = (r < 1.6).sum(1)
    assert (near == 3).all()
    assert np.abs(r[r < 1.6] - 1.42).max() < 0.02
    a = math.sqrt(3) * 1.42
    radius = a * math.sqrt(n * n + n * m + m * m) / (2 * math.pi)
    c = box[:2] / 2
    assert np.allclose(np.linalg.norm(x[:, :2] - c, axis=1), radius, atol=1e-9)


def test_nanotube_bundle_layout():
    """16 (10,10) tubes of 40 cells: 25,600 atoms; walls of neighbouring tubes
    (through the periodic boundary too) are 3.4 A apart."""
    d = synth.nanotube_bundle()
    x, box = d["x"], d["box"]
    assert len(x) == 25600 and list(d["periodic"]) == [1, 1, 1]
    per_tube = 1600
    c0 = x[:per_tube, :2].mean(0)
    rad = np.linalg.norm(x[0, :2] - c0)
    centres = np.array([x[k * per_tube:(k + 1) * per_tube, :2].mean(0) for k in range(16)])
    dc = centres[:, None, :] - centres[None, :, :]
    dc -= box[:2] * np.round(dc / box[:2])
    dist = np.linalg.norm(dc, axis=2)
    np.fill_diagonal(dist, np.inf)
    assert np.allclose(dist.min(1), 2 * rad + 3.4, atol=1e-6)
