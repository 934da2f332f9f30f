"""Seeded surrogate test cases shared by the CPU pins and the GPU parity tests."""
import math

import numpy as np

from paper_1810_07026_amd import synth


def cluster(seed=3, nmol=4, box=13.0, periodic=True):
    """A few ethane / propane / methane molecules at random positions and
    orientations with 0.05 A jitter, in a periodic cube or isolated."""
    rng = np.random.default_rng(seed)
    X, S = [], []
    kinds = [lambda: synth.ethane(rng.uniform(0, 2 * math.pi)), lambda: synth.alkane(3), lambda: synth.alkane(1)]
    centres = []
    while len(centres) < nmol:
        c = rng.uniform(0, box, 3)
        if all(np.linalg.norm((c - d + box / 2) % box - box / 2) > 4.2 for d in centres):
            centres.append(c)
    for k, c in enumerate(centres):
        x, s = kinds[k % 3]()
        q = synth._random_rotation(rng)
        X.append((x - x.mean(0)) @ q.T + c)
        S.append(s)
    x = np.vstack(X) + rng.normal(0, 0.05, (sum(len(s) for s in S), 3))
    s = np.concatenate(S).astype(np.int32)
    if periodic:
        return x % box, s, [box] * 3, [1, 1, 1]
    return x, s, [50.0] * 3, [0, 0, 0]


def model_arrays(nm=2, seed=5, wscale=1.0, dim=112):
    """Seeded weights and a normalisation: (params, mean, istd, scale, shift)."""
    w = synth.nn_init_weights(nm, seed) * np.float32(wscale)
    rng = np.random.default_rng(seed + 100)
    mean = rng.normal(0, 0.3, dim).astype(np.float32)
    istd = rng.uniform(0.5, 2.0, dim).astype(np.float32)
    return w, mean, istd, 0.7, [-1.3, -0.4]
