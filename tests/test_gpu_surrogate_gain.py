"""What the trained surrogate gains over the method without it.

The committed ensemble (paper_1810_07026_amd/data/surrogate_pe_melt.bin) was
trained on the GPU by the library's own gradient and Adam kernels
(python -m paper_1810_07026_amd.surrogate train).  On an equilibrated state
of the 32,012-atom polyethylene melt, which is not one of its training
frames, it is compared with:
  - the same ensemble untrained (seeded initial weights);
  - the far field alone (network weights zero);
  - AIREBO FP64 on the GPU, which is the reference forces and the
    throughput baseline.
Accuracy gains are asserted.  Throughput and the fallback decision are
measured and printed; they are not asserted (the GPU surrogate is not faster
than GPU AIREBO on this system, see the printed ratio).
"""
import os
import time

import numpy as np
import pytest
import torch

from paper_1810_07026_amd import synth

pytestmark = pytest.mark.gpu


def test_trained_surrogate_gain():
    from paper_1810_07026_amd import airebo, surrogate
    assert os.path.exists(surrogate.WEIGHTS), "trained weights missing"
    d = synth.pe_melt()
    s, box, per = d["species"], d["box"], d["periodic"]
    n = len(s)
    ctx = airebo.Context()
    x = torch.tensor(d["x"], dtype=torch.float64, device="cuda")
    v = torch.tensor(synth.maxwell_velocities(s, 300.0, np.random.default_rng(77)), dtype=torch.float64,
                     device="cuda")
    ctx.nve(x, v, s, box, per, nsteps=400, thermo_every=0)
    _, fref, _ = ctx.compute(x, s, box, per)
    nn = airebo.Surrogate(path=surrogate.WEIGHTS)
    trained = surrogate.force_error(nn, ctx, x, s, box, per, fref)
    norm = nn.get_norm()
    raw = airebo.Surrogate(nmodels=nn.nmodels)
    raw.set_params(synth.nn_init_weights(nn.nmodels, 1810070265))
    raw.set_norm(*norm)
    untrained = surrogate.force_error(raw, ctx, x, s, box, per, fref)
    zero = airebo.Surrogate(nmodels=nn.nmodels)
    zero.set_norm(*norm)
    far_only = surrogate.force_error(zero, ctx, x, s, box, per, fref)
    print("trained", trained)
    print("untrained", untrained)
    print("far field only", far_only)
    assert trained["force_rel_rms_err"] < 0.3
    assert trained["force_rel_rms_err"] < 0.3 * untrained["force_rel_rms_err"]
    assert trained["force_rel_rms_err"] < 0.3 * far_only["force_rel_rms_err"]

    def rate(run, steps=100):
        xs, vs = x.clone(), v.clone()
        run(xs, vs, 5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = run(xs, vs, steps)
        torch.cuda.synchronize()
        return n * steps / (time.perf_counter() - t0), out

    r_fp64, _ = rate(lambda a, b, k: ctx.nve(a, b, s, box, per, nsteps=k, thermo_every=0))
    r_nn, _ = rate(lambda a, b, k: nn.nve(ctx, a, b, s, box, per, nsteps=k, thermo_every=0, threshold=1e30))
    r_fb, fb = rate(lambda a, b, k: nn.nve(ctx, a, b, s, box, per, nsteps=k, thermo_every=0,
                                           threshold=surrogate.THRESHOLD)[1])
    print(f"atom-steps/s: AIREBO FP64 {r_fp64:.4g}, surrogate {r_nn:.4g} ({r_nn / r_fp64:.3f}x), "
          f"surrogate with fallback at {surrogate.THRESHOLD} eV/A {r_fb:.4g} ({r_fb / r_fp64:.3f}x, "
          f"{fb} of 101 evaluations by AIREBO)")
    assert r_fp64 > 0 and r_nn > 0 and r_fb > 0
