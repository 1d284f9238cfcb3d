"""lbm_step_reduce_noalloc (the allocation-free step + reduce) against
lbm_step_reduce on the GPU, through the C ABI.

Both run the same kernels on the same lattice state, so the populations and
every sampled reduction must agree bitwise.  Two calls in a row, the second
on a smaller lattice with fewer samples (the scratch array keeps the first
call's contents), and the limits (tiles, samples) are rejected with EINVAL
before any launch.
"""
import numpy as np
import pytest

from paper_2506_09242_amd import inputs, lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.lib()
    yield


def _lattice(case):
    if case == "cavity":
        n = 48
        nu = 0.1 * (n - 2) / 1000.0
        tags = inputs.cavity_tags(n)
        return tags, dict(q=19, prec=lbm.LBM_F32, tau=3 * nu + 0.5, wall_velocity=[(0.1, 0.0, 0.0)]), None, None
    if case == "tgv":
        n = 24
        rho, u = inputs.tgv3d_fields(n, 0.05)
        tags = inputs.all_fluid(n, n, n, inputs.TAG_SMAG)
        return tags, dict(q=27, prec=lbm.LBM_F64, tau=0.52, smag_cs=0.1), rho, u
    raise KeyError(case)


def _pair(case):
    tags, kw, rho, u = _lattice(case)
    a = lbm.Lattice(tags, **kw)
    b = lbm.Lattice(tags, **kw)
    for L in (a, b):
        L.init_equilibrium(rho, u)
    return a, b


def _same_series(s_ref, s_new):
    assert len(s_ref) == len(s_new)
    for x, y in zip(s_ref, s_new):
        for k in ("step", "n_fluid", "n_nonfinite", "mass", "mass_delta", "kinetic_energy", "kinetic_energy_rho"):
            assert x[k] == y[k], (k, x[k], y[k])
        assert np.array_equal(x["momentum"], y["momentum"])
        assert np.array_equal(x["velocity_sum"], y["velocity_sum"])


def test_noalloc_matches_step_reduce_twice():
    """Two calls in a row (a 48^3 cavity with 8 samples, then a smaller 24^3
    D3Q27 lattice with 4 samples): series and populations bitwise equal to
    lbm_step_reduce's."""
    for case, n, every in (("cavity", 37, 5), ("tgv", 12, 4)):
        a, b = _pair(case)
        print(f"noalloc case {case}: {n} steps, every {every}", flush=True)
        s_ref = a.step_reduce(n, every)
        s_new = b.step_reduce(n, every, noalloc=True)
        _same_series(s_ref, s_new)
        assert a.time == b.time == n
        assert np.array_equal(a.read_state(), b.read_state())
        # continue both from where they are (odd parity now), once more
        s_ref = a.step_reduce(every * 2, every)
        s_new = b.step_reduce(every * 2, every, noalloc=True)
        _same_series(s_ref, s_new)
        assert np.array_equal(a.read_state(), b.read_state())
        a.close()
        b.close()


def test_noalloc_limits():
    """More samples than LBM_NOALLOC_MAX_SAMPLES, or more tiles than
    LBM_NOALLOC_MAX_TILES (a 33 x 1 x 300000 lattice: two 32-wide tiles per
    row), are rejected with EINVAL and leave the lattice unchanged."""
    tags = inputs.all_fluid(16, 16, 16)
    L = lbm.Lattice(tags, q=19, prec=lbm.LBM_F32, tau=0.8)
    L.init_equilibrium()
    with pytest.raises(lbm.LbmError) as e:
        L.step_reduce(4096, 1, noalloc=True)
    assert e.value.status == lbm.LBM_EINVAL and "4097 samples" in str(e.value)
    assert L.time == 0
    L.step_reduce(4095, 1, noalloc=True)  # 4096 samples: at the limit
    assert L.time == 4095
    L.close()
    nz = 300_000
    L = lbm.Lattice(inputs.all_fluid(33, 1, nz), q=19, prec=lbm.LBM_F32, tau=0.8)
    L.set_launch(32, 8)
    with pytest.raises(lbm.LbmError) as e:
        L.step_reduce(2, 1, noalloc=True)
    assert e.value.status == lbm.LBM_EINVAL and "600000 tiles" in str(e.value)
    assert L.time == 0
    L.close()
