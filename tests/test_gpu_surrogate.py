"""GPU parity of the learned surrogate against its FP64 CPU reference.

Tolerances:
  - Descriptors and their JVP/VJP are FP32 arithmetic on FP64-formed pair
    vectors.  They are checked element by element to 2e-5 (values) and 1e-4
    (derivatives) of the largest magnitude.  That allows ~300 FP32 roundings
    of 6e-8 each.
  - The networks run on BF16 matrix-core tiles.  Every weight and activation
    enters a product rounded to BF16 (relative 2^-9), and accumulation is in
    FP32.  The forward pass and input gradient chain 7 such products, so
    their worst-case relative error is 7 * 2 * 2^-9 = 2.7e-2 of the
    magnitude sums.  Energies and forces are checked as an RMS over atoms
    relative to the RMS of the reference, bound 2e-2.
  - The weight gradient chains up to 12 products (bound 4.7e-2).  It is
    checked as a relative L2 error per member, bound 5e-2.
  - Element by element, the networks are compared with a reference that
    rounds every matrix-product operand to BF16 at the same points as the
    matrix cores (surrogate_ref.atom_energies_bf16, loss_and_grad_bf16):
    per-atom forces and force spreads within 3e-3 of their largest value,
    every weight gradient within 2e-3 of its layer block's largest (the
    bounds of test_network_elementwise and test_training_gradient_elementwise).
  - The far field is FP32 arithmetic on FP64 pair vectors with FP64 sums
    (1e-6 of the largest force and of the energy).  The AIREBO fallback is
    FP64 (1e-12).
"""
import os
import tempfile

import numpy as np
import pytest
import torch

from oracle import surrogate_ref as sr
from paper_1810_07026_amd import synth
from tests.surrogate_cases import cluster, model_arrays

pytestmark = pytest.mark.gpu

LJ = sr.lj_params()


@pytest.fixture(scope="module")
def lib():
    from paper_1810_07026_amd import airebo
    return airebo


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context()


def systems():
    pe = synth.pe_small()
    return {
        "cluster_periodic": cluster(periodic=True),
        "cluster_isolated": cluster(periodic=False),
        "pe_small": (pe["x"], pe["species"], list(pe["box"]), [1, 1, 1]),
    }


SYS = systems()


def bf16(a):
    """Round float32 values to BF16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def make_nn(lib, nm=2, seed=5, wscale=1.0):
    w, mean, istd, scale, shift = model_arrays(nm, seed, wscale)
    nn = lib.Surrogate(nmodels=nm)
    nn.set_params(w)
    nn.set_norm(mean, istd, scale, shift)
    return nn, sr.Model(w, mean, istd, scale, shift)


def rel_rms(a, b):
    return float(np.sqrt(np.mean((np.asarray(a) - np.asarray(b)) ** 2)) / max(np.sqrt(np.mean(np.asarray(b) ** 2)),
                                                                               1e-300))


def test_mfma_lane_layout(lib):
    rng = np.random.default_rng(0)
    A = rng.normal(size=(16, 16)).astype(np.float32)
    B = rng.normal(size=(16, 16)).astype(np.float32)
    D = lib.mfma_check(torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")).cpu().numpy()
    want = bf16(A) @ bf16(B)
    assert np.abs(D - want).max() <= 1e-5 * np.abs(want).max()


def test_mfma32_lane_layout(lib):
    """The 16x16x32 BF16 tile (gfx950) the networks use for full 32-deep
    slices of K."""
    rng = np.random.default_rng(1)
    A = rng.normal(size=(16, 32)).astype(np.float32)
    B = rng.normal(size=(32, 16)).astype(np.float32)
    D = lib.mfma32_check(torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")).cpu().numpy()
    want = bf16(A) @ bf16(B)
    assert np.abs(D - want).max() <= 1e-5 * np.abs(want).max()


@pytest.mark.parametrize("name", list(SYS))
def test_descriptors(lib, ctx, name):
    x, s, box, per = SYS[name]
    nn = lib.Surrogate(nmodels=1)
    G = nn.descriptors(ctx, x, s, box, per).cpu().numpy()
    Gr = sr.descriptors(x, s, box, per).numpy()
    print(name, "max |G|", np.abs(Gr).max(), "max err", np.abs(G - Gr).max())
    assert np.abs(G - Gr).max() <= 2e-5 * max(1.0, np.abs(Gr).max())


@pytest.mark.parametrize("name", ["cluster_periodic", "pe_small"])
def test_descriptor_jvp(lib, ctx, name):
    x, s, box, per = SYS[name]
    rng = np.random.default_rng(2)
    w = rng.normal(size=(len(s), 3)).astype(np.float32)
    nn = lib.Surrogate(nmodels=1)
    J = nn.descriptor_jvp(ctx, x, s, box, w, per).cpu().numpy()
    xt = torch.as_tensor(np.asarray(x, np.float64))
    _, Jr = torch.autograd.functional.jvp(lambda y: sr.descriptors(y, s, box, per), xt,
                                          torch.as_tensor(w, dtype=torch.float64))
    Jr = Jr.numpy()
    print(name, "max |J|", np.abs(Jr).max(), "max err", np.abs(J - Jr).max())
    assert np.abs(J - Jr).max() <= 1e-4 * np.abs(Jr).max()


@pytest.mark.parametrize("name", ["cluster_periodic", "cluster_isolated", "pe_small"])
def test_descriptor_vjp(lib, ctx, name):
    x, s, box, per = SYS[name]
    n = len(s)
    rng = np.random.default_rng(4)
    g = rng.normal(size=(2, n, sr.DIM)).astype(np.float32)
    nn = lib.Surrogate(nmodels=1)
    F, W = nn.descriptor_vjp(ctx, x, s, box, g, per)
    F, W = F.cpu().numpy(), W.cpu().numpy()
    xt = torch.as_tensor(np.asarray(x, np.float64)).requires_grad_(True)
    eps = torch.zeros(3, 3, dtype=torch.float64, requires_grad=True)
    I, J, d0 = sr.pair_vectors(xt, box, per, sr.RAD_CUT)
    d = d0 @ (torch.eye(3, dtype=torch.float64) + eps).T
    G = sr.descriptors_from_pairs(n, s, I, J, d)
    gt = torch.as_tensor(g, dtype=torch.float64)
    Fr = np.stack([-torch.autograd.grad((G * gt[k]).sum(), xt, retain_graph=True)[0].numpy() for k in range(2)])
    Wr = -torch.autograd.grad((G * gt.mean(0)).sum(), eps)[0].numpy()
    Wr = np.array([Wr[0, 0], Wr[1, 1], Wr[2, 2], Wr[0, 1], Wr[0, 2], Wr[1, 2]])
    print(name, "max |F|", np.abs(Fr).max(), "max err", np.abs(F - Fr).max(), "vir err", np.abs(W - Wr).max())
    assert np.abs(F - Fr).max() <= 1e-4 * np.abs(Fr).max()
    assert np.abs(W - Wr).max() <= 1e-4 * np.abs(Wr).max()


def test_far_field(lib, ctx):
    """Zero network weights: the forces and energy are the far field alone."""
    x, s, box, per = SYS["pe_small"]
    nn = lib.Surrogate(nmodels=2)
    e, f, w, _, info = nn.compute(ctx, x, s, box, per, threshold=1e30)
    ref = sr.evaluate(sr.Model(np.zeros((2, 2, sr.NPAR)), np.zeros(sr.DIM), np.ones(sr.DIM), 1.0, [0.0, 0.0]),
                      x, s, box, per, LJ, want_virial=True)
    assert info["fallback"] == 0.0
    print("far field: E", info["E_far"], ref["E_far"], "max |dF|", np.abs(f.cpu().numpy() - ref["F_far"]).max(),
          "max |F|", np.abs(ref["F_far"]).max())
    assert info["E_far"] == pytest.approx(ref["E_far"], rel=1e-6)
    assert np.abs(f.cpu().numpy() - ref["F_far"]).max() <= 1e-6 * np.abs(ref["F_far"]).max()
    assert np.abs(w.cpu().numpy() - ref["virial"]).max() <= 1e-6 * np.abs(ref["virial"]).max()


@pytest.mark.parametrize("name", ["cluster_periodic", "pe_small"])
def test_network_energy_forces(lib, ctx, name):
    x, s, box, per = SYS[name]
    nn, M = make_nn(lib, nm=4, seed=9)
    e, f, w, sp, info = nn.compute(ctx, x, s, box, per, threshold=1e30, want_spread=True)
    ref = sr.evaluate(M, x, s, box, per, LJ, want_virial=True)
    e = e.cpu().numpy()
    F = f.cpu().numpy()
    Fnn_ref = ref["F_nn"].mean(0)
    err_f = rel_rms(F - ref["F_far"], Fnn_ref)
    err_e = abs(info["E_nn"] - ref["E_nn"].mean()) / np.abs(ref["E_atom"]).sum(1).mean()
    spread_ref = np.sqrt(((ref["F_nn"] - Fnn_ref) ** 2).sum(2).mean(0))
    err_sp = rel_rms(sp.cpu().numpy(), spread_ref)
    err_w = np.abs(w.cpu().numpy() - ref["virial"]).max() / np.abs(ref["virial"]).max()
    print(name, "force rel rms", err_f, "energy rel", err_e, "spread rel rms", err_sp, "virial", err_w)
    assert err_f <= 2e-2 and err_e <= 2e-2 and err_sp <= 2e-2 and err_w <= 2e-2
    assert info["max_spread"] == pytest.approx(spread_ref.max(), rel=3e-2)
    assert e[0] == pytest.approx(info["E_nn"] + info["E_far"], rel=1e-12)


@pytest.mark.parametrize("name", ["cluster_periodic", "cluster_isolated", "pe_small"])
def test_network_elementwise(lib, ctx, name):
    """Per-atom forces and force spread, element by element, against the
    reference evaluated with the matrix cores' BF16 operand rounding
    (surrogate_ref.atom_energies_bf16).  What remains is FP32 accumulation
    (~112 terms, 1e-5 relative) and the occasional operand whose FP32 value
    lies within that of a BF16 rounding midpoint and rounds the other way
    (one BF16 ulp, 2^-8, of one of ~400 operands of an atom's chain: ~1e-3
    of that atom's contribution).  Bar: every force component within 3e-3 of
    the largest network force, every spread within 3e-3 of the largest
    spread, E_nn within 1e-3 of the summed per-atom magnitudes."""
    x, s, box, per = SYS[name]
    nn, M = make_nn(lib, nm=4, seed=9)
    e, f, w, sp, info = nn.compute(ctx, x, s, box, per, threshold=1e30, want_spread=True)
    ref = sr.evaluate(M, x, s, box, per, LJ, bf16_operands=True)
    Fnn_ref = ref["F_nn"].mean(0)
    F = f.cpu().numpy() - ref["F_far"]
    spread_ref = np.sqrt(((ref["F_nn"] - Fnn_ref) ** 2).sum(2).mean(0))
    err_f = np.abs(F - Fnn_ref).max() / np.abs(Fnn_ref).max()
    err_sp = np.abs(sp.cpu().numpy() - spread_ref).max() / spread_ref.max()
    err_e = abs(info["E_nn"] - ref["E_nn"].mean()) / np.abs(ref["E_atom"]).sum(1).mean()
    print(name, "max force err", err_f, "max spread err", err_sp, "energy err", err_e)
    assert err_f <= 3e-3 and err_sp <= 3e-3 and err_e <= 1e-3


def test_training_gradient(lib, ctx):
    x, s, box, per = SYS["cluster_periodic"]
    nn, M = make_nn(lib, nm=2, seed=13)
    rng = np.random.default_rng(17)
    f_ref = rng.normal(0, 1.0, (len(s), 3))
    e_ref, wF, wE = -40.0, 0.25, 0.01
    loss = nn.gradient(ctx, x, s, box, f_ref, e_ref, wF, wE, per)
    g = nn.get_grad().astype(np.float64)
    L_ref, g_ref = sr.loss_and_grad(M, x, s, box, per, f_ref, e_ref, wF, wE, LJ)
    for m in range(2):
        err = np.linalg.norm(g[m] - g_ref[m]) / np.linalg.norm(g_ref[m])
        print("member", m, "loss", loss[m], L_ref[m], "grad rel L2", err)
        assert loss[m] == pytest.approx(L_ref[m], rel=2e-2)
        assert err <= 5e-2
        # every layer's block individually
        off = 0
        for name, shape in sr.LAYOUT:
            k = int(np.prod(shape))
            blk, blk_ref = g[m][:, off:off + k], g_ref[m][:, off:off + k]
            if np.linalg.norm(blk_ref) > 1e-8 * np.linalg.norm(g_ref[m]):
                assert np.linalg.norm(blk - blk_ref) / np.linalg.norm(blk_ref) <= 8e-2, name
            off += k


def test_training_gradient_elementwise(lib, ctx):
    """Every weight's gradient against the reference whose training chain
    rounds the matrix-product operands to BF16 as the matrix cores do
    (surrogate_ref.loss_and_grad_bf16).  Left over: FP32 accumulation and
    the FP32 descriptor JVP of the force adjoint (~1e-5 relative), and the
    rare operand that rounds to the other BF16 neighbour (one BF16 ulp of
    one of several hundred operands per atom).  Bar: each weight within
    2e-3 of the largest gradient of its layer block; the losses within 1e-4."""
    x, s, box, per = SYS["cluster_periodic"]
    nn, M = make_nn(lib, nm=2, seed=13)
    rng = np.random.default_rng(17)
    f_ref = rng.normal(0, 1.0, (len(s), 3))
    e_ref, wF, wE = -40.0, 0.25, 0.01
    loss = nn.gradient(ctx, x, s, box, f_ref, e_ref, wF, wE, per)
    g = nn.get_grad().astype(np.float64)
    L_ref, g_ref = sr.loss_and_grad_bf16(M, x, s, box, per, f_ref, e_ref, wF, wE, LJ)
    for m in range(2):
        assert loss[m] == pytest.approx(L_ref[m], rel=1e-4)
        off = 0
        for name, shape in sr.LAYOUT:
            k = int(np.prod(shape))
            blk, blk_ref = g[m][:, off:off + k], g_ref[m][:, off:off + k]
            scale = np.abs(blk_ref).max()
            err = np.abs(blk - blk_ref).max() / max(scale, 1e-300)
            print("member", m, name, "max |g|", scale, "max err / max |g|", err)
            assert err <= 2e-3, (m, name, err)
            off += k


def test_training_lowers_loss(lib, ctx):
    """A few Adam steps on AIREBO labels of one configuration lower the loss."""
    x, s, box, per = SYS["pe_small"]
    e_ref, f_ref, _ = ctx.compute(x, s, box, per)
    nn = lib.Surrogate(nmodels=2)
    nn.set_params(synth.nn_init_weights(2, 21))
    G = nn.descriptors(ctx, x, s, box, per)
    s1, s2 = nn.moments(G)
    mean = s1 / len(s)
    istd = 1.0 / np.sqrt(np.maximum(s2 / len(s) - mean ** 2, 1e-4))
    nn.set_norm(mean, istd, 1.0, [float(e_ref[0]) / len(s)] * 2)
    wF = 1.0 / (3 * len(s))
    losses = []
    for it in range(60):
        losses.append(nn.gradient(ctx, x, s, box, f_ref, float(e_ref[0]), wF, 1.0 / len(s) ** 2, per))
        nn.adam(3e-3)
    print("loss", losses[0], losses[-1])
    assert np.all(losses[-1] < 0.5 * losses[0])


def test_fallback_to_airebo(lib, ctx):
    x, s, box, per = SYS["pe_small"]
    nn, _ = make_nn(lib, nm=4, seed=9)
    e, f, w, _, info = nn.compute(ctx, x, s, box, per, threshold=1e-12)
    assert ctx.stats()["nn_fallbacks"] == 1
    ea, fa, wa = ctx.compute(x, s, box, per)
    assert info["fallback"] == 1.0
    assert float(e[0]) == pytest.approx(float(ea[0]), rel=1e-12)
    assert torch.allclose(f, fa, rtol=0, atol=1e-12 * float(fa.abs().max()))
    assert torch.allclose(w, wa, rtol=0, atol=1e-12 * float(wa.abs().max()))
    e2, f2, _, _, info2 = nn.compute(ctx, x, s, box, per, threshold=1e30)
    assert info2["fallback"] == 0.0 and ctx.stats()["nn_fallbacks"] == 0
    assert float((f2 - fa).abs().max()) > 1e-3


def test_nve_matches_stepwise(lib, ctx):
    """The captured surrogate NVE equals velocity Verlet driven by single evaluations."""
    x, s, box, per = SYS["pe_small"]
    nn, _ = make_nn(lib, nm=4, seed=9, wscale=0.3)
    rng = np.random.default_rng(3)
    v0 = synth.maxwell_velocities(s, 300.0, rng)
    xg = torch.tensor(x, dtype=torch.float64, device="cuda")
    vg = torch.tensor(v0, dtype=torch.float64, device="cuda")
    th, nfb = nn.nve(ctx, xg, vg, s, box, per, dt=0.5, nsteps=5, thermo_every=1, threshold=1e30)
    assert nfb == 0
    m = np.where(np.asarray(s) == 0, 12.011, 1.008)[:, None]
    ftm = 1.0 / 103.642691
    xh, vh = np.array(x, float), np.array(v0, float)
    f = nn.compute(ctx, xh, s, box, per, threshold=1e30)[1].cpu().numpy()
    dt = 0.5
    for _ in range(5):
        vh = vh + 0.5 * dt * f / m * ftm
        xh = xh + dt * vh
        f = nn.compute(ctx, xh, s, box, per, threshold=1e30)[1].cpu().numpy()
        vh = vh + 0.5 * dt * f / m * ftm
    xw = xg.cpu().numpy()
    dx = (xw - xh + np.asarray(box) / 2) % np.asarray(box) - np.asarray(box) / 2
    assert np.abs(dx).max() < 1e-8
    assert np.abs(vg.cpu().numpy() - vh).max() < 1e-8


def test_save_load(lib, ctx):
    x, s, box, per = SYS["cluster_periodic"]
    nn, _ = make_nn(lib, nm=3, seed=31)
    path = os.path.join(tempfile.mkdtemp(), "nn.bin")
    nn.save(path)
    nn2 = lib.Surrogate(path=path)
    assert nn2.nmodels == 3
    assert np.array_equal(nn.get_params(), nn2.get_params())
    a = nn.compute(ctx, x, s, box, per, threshold=1e30)
    b = nn2.compute(ctx, x, s, box, per, threshold=1e30)
    assert abs(a[4]["E_nn"] - b[4]["E_nn"]) <= 1e-6 * abs(a[4]["E_nn"])
