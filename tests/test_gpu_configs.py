"""Parity of the workload configurations at 64^3 against the FP64 oracle (GPU).

The three benchmark workloads, shrunk to 64^3 and run through their laminar
phase with their own collision model, boundaries, forcing and kernel variant:
  - lid-driven cavity (Sec. 3.2 shape): D3Q19 BGK, one-node solid shell, lid
    at u = 0.1, Re = 1000 over the 62-node cavity, 1000 steps (64-wide rows:
    the wall waves take the row-form addresses);
  - porous medium (Sec. 3.3 shape, synthetic rock): D3Q19 TRT with the magic
    parameter 3/16, tau = 1, body force 1e-5 along x, a Gaussian-random-field
    solid (correlation length 8) at porosity 0.20, 2000 steps (solid-rich with
    sides a multiple of 16: the brick storage layout);
  - Taylor-Green vortex (Sec. 3.1, Eqs. (1)-(4)): D3Q27 BGK + Smagorinsky
    (C_s = 0.1), u0 = 0.05, Re = 1600 on the reference length N / 2 pi,
    500 steps.
FP64 populations of every fluid node are compared with the oracle at 1e-12
relative.  FP32 and FP16 storage run the same configurations (the precisions
the benchmarks use) and are compared with the same oracle run; their error is
printed and bounded as stated at each test.
"""
import numpy as np
import pytest

import oracle
from paper_2506_09242_amd import inputs, lbm

from _util import fluid_mask, kinetic_energy_bound, max_rel_pop_error, momentum_bound, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-12
N = 64


def _config(name):
    """(tags, lattice keyword arguments, rho, u, steps) of a 64^3 workload."""
    if name == "cavity":
        L = N - 2
        nu = 0.1 * L / 1000.0
        return inputs.cavity_tags(N), dict(q=19, tau=3 * nu + 0.5, wall_velocity=[(0.1, 0.0, 0.0)]), None, None, 1000
    if name == "porous":
        tags = inputs.porous_tags(N, porosity=0.20, ell=8.0, seed=42)
        return tags, dict(q=19, tau=1.0, trt_lambda=3.0 / 16.0, force=(1e-5, 0.0, 0.0)), None, None, 2000
    if name == "tgv":
        u0, Re = 0.05, 1600.0
        nu = u0 * (N / (2 * np.pi)) / Re
        rho, u = inputs.tgv3d_fields(N, u0)
        tags = inputs.all_fluid(N, N, N, inputs.TAG_SMAG)
        return tags, dict(q=27, tau=3 * nu + 0.5, smag_cs=0.1), rho, u, 500
    raise KeyError(name)


_ORACLE = {}


def _oracle_run(name):
    """The oracle's state after the configuration's steps (computed once per module)."""
    if name not in _ORACLE:
        tags, kw, rho, u, steps = _config(name)
        o = oracle.Oracle(N, N, N, tags=tags, **kw)
        o.init_equilibrium(rho, u)
        o.run(steps)
        _ORACLE[name] = (o.f.copy(), o.fields(), o.moments())
    return _ORACLE[name]


def _gpu_run(name, prec):
    tags, kw, rho, u, steps = _config(name)
    L = lbm.Lattice(tags, prec=prec, **kw)
    L.init_equilibrium(rho, u)
    L.step(steps)
    f = L.read_populations()
    fields = L.read_fields()
    m = L.reduce()
    variant = L.variant
    L.close()
    return f, fields, m, variant


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.lib()
    yield


EXPECT_VARIANT = {
    "cavity": {lbm.LBM_F64: "D3Q19/f64/bgk/tagged/rows", lbm.LBM_F32: "D3Q19/f32/bgk/tagged/rows",
               lbm.LBM_F16S: "D3Q19/f16s/bgk/tagged/rows"},
    "porous": {lbm.LBM_F64: "D3Q19/f64/trt/tagged/bricks", lbm.LBM_F32: "D3Q19/f32/trt/tagged/bricks",
               lbm.LBM_F16S: "D3Q19/f16s/trt/tagged/bricks"},
    "tgv": {lbm.LBM_F64: "D3Q27/f64/bgk+smag/uniform", lbm.LBM_F32: "D3Q27/f32/bgk+smag/uniform",
            lbm.LBM_F16S: "D3Q27/f16s/bgk+smag/uniform/rows"},
}


@pytest.mark.parametrize("name", ["cavity", "porous", "tgv"])
def test_config64_fp64_matches_oracle(name):
    """Every population of every fluid node within 1e-12 relative of the oracle;
    density and velocity fields and the reductions likewise."""
    tags = _config(name)[0]
    f_o, (r_o, u_o), m_o = _oracle_run(name)
    f, (r_g, u_g), m, variant = _gpu_run(name, lbm.LBM_F64)
    err = max_rel_pop_error(f, f_o, tags)
    print(name, variant, "max rel pop err", err, "u rel L2", rel_l2(u_g, u_o), flush=True)
    assert variant == EXPECT_VARIANT[name][lbm.LBM_F64]
    assert err <= TOL
    assert rel_l2(u_g, u_o) <= TOL and rel_l2(r_g, r_o) <= TOL
    nf = m["n_fluid"]
    assert nf == m_o["n_fluid"]
    assert abs(m["mass_delta"] - m_o["mass_delta"]) <= TOL * nf
    # kinetic energy: quadratic in u, so bounded by the velocities' own
    # differences rather than by 1e-12 (with slow flow through the porous medium
    # its relative difference is about twice that of u)
    dk = abs(m["kinetic_energy"] * nf - m_o["ke_sum"])
    k_bound = kinetic_energy_bound(u_g, u_o, tags)
    print(name, "kinetic energy diff", dk, "bound", k_bound, "relative", dk / m_o["ke_sum"], flush=True)
    assert dk <= k_bound and dk <= 4 * TOL * m_o["ke_sum"]
    # momentum: no larger than the populations' own differences allow (the sum
    # cancels heavily, so its relative error exceeds theirs)
    bound = momentum_bound(f, f_o, tags, _config(name)[1]["q"])
    print(name, "momentum diff", np.abs(m["momentum"] - m_o["momentum"]), "bound", bound, flush=True)
    assert np.all(np.abs(m["momentum"] - m_o["momentum"]) <= bound)


# Reduced-precision bounds.  Relative error of the velocity field (L2 over the
# lattice) against the FP64 oracle after the configuration's steps: FP32
# arithmetic and storage round at 2^-24 per operation, FP16 storage rounds the
# stored h = f - w rho0 at 2^-11 once per step; both errors accumulate over
# the steps of a laminar run.  Bounds are five to ten times the errors
# measured on MI355X (printed by the test; velocity rel. L2 / k rel. error):
#   cavity  FP32 1.9e-5 / 2.4e-5   FP16 4.5e-4 / 3.7e-5
#   porous  FP32 3.9e-6 / 9.1e-7   FP16 4.8e-3 / 2.3e-3
#   TGV     FP32 1.0e-5 / 1.9e-5   FP16 1.0e-3 / 8.7e-5
# and far below the velocity scale itself.
REDUCED_BOUNDS = {
    ("cavity", lbm.LBM_F32): 1e-4, ("cavity", lbm.LBM_F16S): 3e-3,
    ("porous", lbm.LBM_F32): 3e-5, ("porous", lbm.LBM_F16S): 3e-2,
    ("tgv", lbm.LBM_F32): 1e-4, ("tgv", lbm.LBM_F16S): 6e-3,
}


@pytest.mark.parametrize("prec", [lbm.LBM_F32, lbm.LBM_F16S])
@pytest.mark.parametrize("name", ["cavity", "porous", "tgv"])
def test_config64_reduced_precision_vs_oracle(name, prec):
    """FP32 and FP16-storage runs of the same configuration against the FP64
    oracle: velocity-field relative L2 error and kinetic-energy error printed and
    bounded (REDUCED_BOUNDS)."""
    tags = _config(name)[0]
    f_o, (r_o, u_o), m_o = _oracle_run(name)
    f, (r_g, u_g), m, variant = _gpu_run(name, prec)
    assert variant == EXPECT_VARIANT[name][prec]
    fl = fluid_mask(tags)
    e_u = rel_l2(u_g[:, fl], u_o[:, fl])
    e_k = abs(m["kinetic_energy"] * m["n_fluid"] / m_o["ke_sum"] - 1.0)
    e_pop = max_rel_pop_error(f, f_o, tags)
    print(f"{name} {variant}: velocity rel L2 {e_u:.3e}, k rel err {e_k:.3e}, max rel pop err {e_pop:.3e}",
          flush=True)
    assert np.all(np.isfinite(f[:, fl]))
    bound = REDUCED_BOUNDS[(name, prec)]
    assert e_u <= bound and e_k <= bound
