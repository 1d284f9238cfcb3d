"""What the trained closure gains over the coarse method without it (GPU).

The learned-closure pipeline at reduced size, every stage on the GPU through
the C ABI with fixed seeds: a fine 256^3 D3Q27 BGK+Smagorinsky Taylor-Green
run (Re = 1600, u0 = 0.05) to 20 convective times, 16 snapshots box-filtered
4^3 into closure samples, 10^6 samples drawn (seed 1234), 30 Adam epochs,
then three coarse 64^3 runs of the same flow: no model (plain BGK), the
Smagorinsky fallback (C_s = 0.1) and the trained network fused into the
collision.  Score: relative L2 error of the dissipation rate eps(t) = -dk/dt
against the fine run over [0, 20] t_c; cost: MLUPS of each coarse run.

Measured on MI355X: the plain BGK run blows up (tau - 1/2 = 9.5e-4 on 64^3),
so either closure is needed; the trained network's eps error is 0.24 against
0.21 for Smagorinsky -- it does not beat the fallback at this resolution
(a smaller C_s does better: 0.13 at C_s = 0.05, so the coarse lattice wants
less eddy viscosity than the filtered fine run implies).  The test asserts
these signs and records the numbers.
"""
import numpy as np
import pytest

from paper_2506_09242_amd import closure, lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.lib()
    yield


def test_closure_gain_over_fallbacks_64():
    res, P = closure.experiment(n_fine=256, factor=4, n_snap=16, n_samples=1_000_000, epochs=30,
                                log=lambda m: print(m, flush=True))
    c = res["coarse"]
    smag, mlp = c["smagorinsky"], c["mlp"]
    gain = 1.0 - mlp["eps_rel_l2"] / smag["eps_rel_l2"]
    print(f"eps rel L2: smagorinsky {smag['eps_rel_l2']:.4f}, learned {mlp['eps_rel_l2']:.4f} "
          f"(gain over smagorinsky {gain:+.3f}); no model unstable: {c['bgk']['unstable']}; "
          f"coarse MLUPS smagorinsky {smag['MLUPS']:.0f}, learned {mlp['MLUPS']:.0f}", flush=True)
    assert np.all(np.isfinite(P))
    assert res["training"]["loss_last"] < res["training"]["loss_first"]
    # without any closure the coarse lattice is unstable; both closures keep it stable
    assert c["bgk"]["unstable"]
    assert not smag["unstable"] and not mlp["unstable"]
    # the trained closure does not beat the Smagorinsky fallback here (measured gain -0.14)
    assert -0.35 <= gain <= 0.0
    assert 0.15 <= smag["eps_rel_l2"] <= 0.3
