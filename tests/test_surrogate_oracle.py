"""Pins of the surrogate's FP64 CPU reference (oracle/surrogate_ref.py).

Each check compares the reference with something other than itself:
  - central finite differences of its energy;
  - invariance under translation, rotation and permutation;
  - closed forms of symmetric geometries (a regular tetrahedron);
  - a scalar brute-force enumeration written here;
  - the virial identity of an isolated cluster;
  - finite differences of the training loss in the weights.
"""
import math

import numpy as np
import pytest
import torch

from oracle import surrogate_ref as sr
from paper_1810_07026_amd import synth
from tests.surrogate_cases import cluster, model_arrays

LJ = sr.lj_params()


def model(nm=2, seed=5, wscale=1.0):
    w, mean, istd, scale, shift = model_arrays(nm, seed, wscale)
    return sr.Model(w, mean, istd, scale, shift)


# ---------------------------------------------------------------------------
# descriptors
# ---------------------------------------------------------------------------
def brute_descriptors(x, s, box, per):
    """Scalar enumeration over atoms, images and neighbour pairs (math module)."""
    n = len(s)
    G = np.zeros((n, sr.DIM))
    imgs = [(a, b, c) for a in ((-1, 0, 1) if per[0] else (0,)) for b in ((-1, 0, 1) if per[1] else (0,))
            for c in ((-1, 0, 1) if per[2] else (0,))]
    xw = np.array([[x[i][k] % box[k] if per[k] else x[i][k] for k in range(3)] for i in range(n)])
    h = 5.2 / 31
    eta = 1 / (2 * (2 * h) ** 2)
    for i in range(n):
        nb = []
        for j in range(n):
            for im in imgs:
                if j == i and im == (0, 0, 0):
                    continue
                d = [xw[j][k] + im[k] * box[k] - xw[i][k] for k in range(3)]
                r = math.sqrt(sum(t * t for t in d))
                if r < 6.0:
                    cut = 0.5 * (1 + math.cos(math.pi * r / 6.0))
                    for m in range(32):
                        G[i, 32 * s[j] + m] += math.exp(-eta * (r - (0.8 + m * h)) ** 2) * cut
                if r < 3.5:
                    nb.append((j, d, r))
        for a in range(len(nb)):
            for b in range(a + 1, len(nb)):
                ja, da, ra = nb[a]
                jb, db, rb = nb[b]
                cs = sum(p * q for p, q in zip(da, db)) / (ra * rb)
                f = 0.25 * (1 + math.cos(math.pi * ra / 3.5)) * (1 + math.cos(math.pi * rb / 3.5))
                t = s[ja] + s[jb]
                for zi, zeta in enumerate((1, 2, 4, 8)):
                    for li, lam in enumerate((1.0, -1.0)):
                        for ei, ea in enumerate((0.005, 0.05)):
                            c = 4 * zi + 2 * li + ei
                            G[i, 64 + 16 * t + c] += (2.0 ** (1 - zeta) * (1 + lam * cs) ** zeta *
                                                      math.exp(-ea * (ra * ra + rb * rb)) * f)
    return G


@pytest.mark.parametrize("periodic", [True, False])
def test_descriptors_match_brute_force(periodic):
    x, s, box, per = cluster(periodic=periodic)
    G = sr.descriptors(x, s, box, per).numpy()
    Gb = brute_descriptors(x, s, box, per)
    assert np.abs(G - Gb).max() <= 1e-12 * max(1.0, np.abs(Gb).max())
    assert np.abs(Gb[:, 64:]).max() > 0.1   # angular terms present


def test_descriptors_tetrahedron_closed_form():
    """Regular CH4: all H-C-H angles have cos = -1/3; C sees 4 H at r."""
    r = 1.09
    x, s = synth.alkane(1)
    G = sr.descriptors(x + 5.0, s, [50.0] * 3, [0, 0, 0]).numpy()
    h = 5.2 / 31
    eta = 1 / (2 * (2 * h) ** 2)
    fc6 = 0.5 * (1 + math.cos(math.pi * r / 6))
    fc35 = 0.5 * (1 + math.cos(math.pi * r / 3.5))
    for m in range(32):
        assert G[0, 32 + m] == pytest.approx(4 * math.exp(-eta * (r - 0.8 - m * h) ** 2) * fc6, rel=1e-12, abs=1e-300)
        assert G[0, m] == 0.0
    for zi, zeta in enumerate((1, 2, 4, 8)):
        for li, lam in enumerate((1.0, -1.0)):
            for ei, ea in enumerate((0.005, 0.05)):
                c = 4 * zi + 2 * li + ei
                want = 6 * 2.0 ** (1 - zeta) * (1 - lam / 3) ** zeta * math.exp(-ea * 2 * r * r) * fc35 ** 2
                assert G[0, 64 + 32 + c] == pytest.approx(want, rel=1e-12)
                assert G[0, 64 + c] == 0.0 and G[0, 64 + 16 + c] == 0.0


def test_descriptors_invariance():
    x, s, box, per = cluster(periodic=False)
    G0 = sr.descriptors(x, s, box, per).numpy()
    rng = np.random.default_rng(1)
    q = synth._random_rotation(rng)
    G1 = sr.descriptors((x - 25) @ q.T + 25 + rng.normal(0, 1, 3), s, box, per).numpy()
    assert np.abs(G1 - G0).max() < 1e-11
    perm = rng.permutation(len(s))
    G2 = sr.descriptors(x[perm], s[perm], box, per).numpy()
    assert np.abs(G2 - G0[perm]).max() < 1e-11
    xp, sp_, boxp, perp = cluster(periodic=True)
    Gp = sr.descriptors(xp, sp_, boxp, perp).numpy()
    Gq = sr.descriptors(xp + np.array([7.3, -12.1, 30.2]), sp_, boxp, perp).numpy()
    assert np.abs(Gq - Gp).max() < 1e-11


# ---------------------------------------------------------------------------
# energy, forces, virial
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("periodic", [True, False])
def test_forces_are_minus_gradient(periodic):
    x, s, box, per = cluster(periodic=periodic)
    M = model()
    out = sr.evaluate(M, x, s, box, per, LJ)
    h = 1e-5
    rng = np.random.default_rng(7)
    for a in rng.choice(len(s), 6, replace=False):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[a, c] += h
            xm[a, c] -= h
            fd = -(sr.total_energy(M, xp, s, box, per, LJ) - sr.total_energy(M, xm, s, box, per, LJ)) / (2 * h)
            assert out["F"][a, c] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    assert np.abs(out["F"].sum(0)).max() < 1e-10 * np.abs(out["F"]).sum()
    assert out["E"] == pytest.approx(sr.total_energy(M, x, s, box, per, LJ), rel=1e-13)


def test_virial_isolated_cluster():
    """Non-periodic: W_ab = sum_a x_a,alpha F_a,beta (translation invariance)."""
    x, s, box, per = cluster(periodic=False)
    out = sr.evaluate(model(), x, s, box, per, LJ, want_virial=True)
    W = np.einsum("ia,ib->ab", x, out["F"])
    want = [W[0, 0], W[1, 1], W[2, 2], W[0, 1], W[0, 2], W[1, 2]]
    assert np.allclose(out["virial"], want, rtol=1e-9, atol=1e-9)


def test_virial_periodic_strain_fd():
    """Periodic: W_aa = -dE/d eps_aa under the box strain x -> (1 + eps) x."""
    x, s, box, per = cluster(periodic=True)
    M = model()
    out = sr.evaluate(M, x, s, box, per, LJ, want_virial=True)
    h = 1e-6
    for a in range(3):
        sc = np.ones(3)
        sc[a] = 1 + h
        ep = sr.total_energy(M, x * sc, s, np.asarray(box) * sc, per, LJ)
        sc[a] = 1 - h
        em = sr.total_energy(M, x * sc, s, np.asarray(box) * sc, per, LJ)
        assert out["virial"][a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-5, abs=1e-6)


def test_network_without_input_weights_is_constant():
    """W1 = 0: every atom energy is a constant and the network forces vanish."""
    M = model()
    p = M.params.copy()
    p[:, :, 0:64 * 112] = 0.0
    M0 = sr.Model(p, M.mean, M.istd, M.scale, M.shift)
    x, s, box, per = cluster(periodic=True)
    out = sr.evaluate(M0, x, s, box, per, LJ)
    assert np.abs(out["F_nn"]).max() < 1e-12
    for sp in (0, 1):
        e = out["E_atom"][0][s == sp]
        assert np.ptp(e) < 1e-12


def test_far_field_pair():
    """Two H atoms alone: zero below 5 A, plain LJ between 6 A and the
    outer switch, zero beyond the cutoff, continuous and smooth in between."""
    M = sr.Model(np.zeros((1, 2, sr.NPAR)), np.zeros(sr.DIM), np.ones(sr.DIM), 1.0, [0.0, 0.0])
    sig, eps, rc, sw = LJ

    def E(r):
        x = np.array([[10.0, 10, 10], [10.0 + r, 10, 10]])
        return sr.total_energy(M, x, np.array([1, 1]), [40.0] * 3, [0, 0, 0], LJ)

    lj = lambda r: 4 * eps[2] * ((sig[2] / r) ** 12 - (sig[2] / r) ** 6)
    assert E(4.9) == 0.0
    assert E(6.5) == pytest.approx(lj(6.5), rel=1e-13)
    assert E(rc[2] + 0.01) == 0.0
    for r0 in (5.0, 6.0, rc[2] - sw, rc[2]):
        assert abs(E(r0 + 1e-7) - E(r0 - 1e-7)) < 1e-9
        d1 = (E(r0 + 2e-4) - E(r0)) / 2e-4
        d0 = (E(r0) - E(r0 - 2e-4)) / 2e-4
        assert abs(d1 - d0) < 1e-4 * max(1e-3, abs(d1))
    r = 5.5
    t = 0.5
    assert E(r) == pytest.approx(t * t * (3 - 2 * t) * lj(r), rel=1e-13)


# ---------------------------------------------------------------------------
# training loss gradient
# ---------------------------------------------------------------------------
def test_loss_gradient_fd():
    x, s, box, per = cluster(periodic=True, nmol=3)
    M = model(nm=2, wscale=1.0)
    rng = np.random.default_rng(11)
    f_ref = rng.normal(0, 1.0, (len(s), 3))
    e_ref = -30.0
    wF, wE = 0.3, 0.02
    L, g = sr.loss_and_grad(M, x, s, box, per, f_ref, e_ref, wF, wE, LJ)
    offs = {"W1": 0, "b1": 64 * 112, "W2": 64 * 113, "b2": 64 * 177, "W3": 64 * 178, "b3": 64 * 242,
            "w4": 64 * 243, "b4": 64 * 244}
    picks = [(m, sp, offs[k] + int(rng.integers(0, 64 if k != "b4" else 1)) + (int(rng.integers(0, 40)) * 64
              if k in ("W1",) else 0)) for m in range(2) for sp in range(2) for k in offs]
    for m, sp, k in picks:
        h = 1e-5
        Pp, Pm = M.params.copy(), M.params.copy()
        Pp[m, sp, k] += h
        Pm[m, sp, k] -= h
        Lp = sr.loss_and_grad(sr.Model(Pp, M.mean, M.istd, M.scale, M.shift), x, s, box, per, f_ref, e_ref, wF, wE,
                              LJ)[0][m]
        Lm = sr.loss_and_grad(sr.Model(Pm, M.mean, M.istd, M.scale, M.shift), x, s, box, per, f_ref, e_ref, wF, wE,
                              LJ)[0][m]
        fd = (Lp - Lm) / (2 * h)
        assert g[m, sp, k] == pytest.approx(fd, rel=2e-5, abs=1e-6 * max(1.0, abs(L[m])))


def test_bf16_chain_is_the_exact_derivative_without_rounding(monkeypatch):
    """atom_energies_bf16 writes the input gradient out by hand; with the BF16
    rounding switched off it must equal the plain network and autograd's
    dE/dG, and with it on it must stay within the BF16 rounding of them."""
    import torch
    x, s, box, per = cluster(periodic=True)
    w, mean, istd, scale, shift = model_arrays(2, 9, 1.0)
    M = sr.Model(w, mean, istd, scale, shift)
    G = sr.descriptors(x, s, box, per)
    for m in range(2):
        nets = sr.unpack(M.params[m])
        Gl = G.clone().requires_grad_(True)
        E = sr.atom_energies(nets, M.norm(), Gl, s)
        dEdG, = torch.autograd.grad(E.sum(), Gl)
        Eb, dEb = sr.atom_energies_bf16(nets, M.norm(), G, s)
        assert np.abs(Eb.numpy() - E.detach().numpy()).max() <= 2e-2 * np.abs(E.detach().numpy()).max()
        assert np.abs(dEb.numpy() - dEdG.numpy()).max() <= 2e-2 * np.abs(dEdG.numpy()).max()
        with monkeypatch.context() as mp:
            mp.setattr(sr, "bf16", lambda t: t)
            E0, dE0 = sr.atom_energies_bf16(nets, M.norm(), G, s)
        assert np.abs(E0.numpy() - E.detach().numpy()).max() <= 1e-12 * np.abs(E.detach().numpy()).max()
        assert np.abs(dE0.numpy() - dEdG.numpy()).max() <= 1e-12 * np.abs(dEdG.numpy()).max()


def test_bf16_training_chain_without_rounding_is_autograd(monkeypatch):
    """loss_and_grad_bf16 writes the double backward out by hand; with the
    BF16 rounding switched off it equals torch's double backward of the
    plain definition (loss_and_grad)."""
    x, s, box, per = cluster(periodic=True)
    w, mean, istd, scale, shift = model_arrays(2, 13, 1.0)
    M = sr.Model(w, mean, istd, scale, shift)
    rng = np.random.default_rng(17)
    f_ref = rng.normal(0, 1.0, (len(s), 3))
    L, g = sr.loss_and_grad(M, x, s, box, per, f_ref, -40.0, 0.25, 0.01)
    with monkeypatch.context() as mp:
        mp.setattr(sr, "bf16", lambda t: t)
        L0, g0 = sr.loss_and_grad_bf16(M, x, s, box, per, f_ref, -40.0, 0.25, 0.01)
    assert np.allclose(L0, L, rtol=1e-10)
    assert np.abs(g0 - g).max() <= 1e-9 * np.abs(g).max()
    Lb, gb = sr.loss_and_grad_bf16(M, x, s, box, per, f_ref, -40.0, 0.25, 0.01)
    assert np.linalg.norm(gb - g) <= 5e-2 * np.linalg.norm(g)
