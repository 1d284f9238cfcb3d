"""Parity of the HIP collide-and-stream path with the FP64 oracle (GPU).

Bar: FP64 populations of every fluid node within 1e-12 relative of the
oracle after N steps (both AA parities), reductions within 1e-12; launch
geometry and checkpoint round trips bitwise-exact.  Reduced-precision paths
are compared with the FP64 GPU path and their errors are stated.
"""
import numpy as np
import pytest

import oracle
from paper_2506_09242_amd import inputs, lbm

from _util import fluid_mask, make_pair, max_abs_pop_error, max_rel_pop_error, momentum_bound, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.lib()
    yield


def _print(*a):
    print(*a, flush=True)


# ------------------------------------------------------- Taylor-Green 32^3
def test_tgv32_d3q19_bgk_fp64_full():
    """D3Q19 BGK Taylor-Green 32^3, u0 = 0.04, Re = 100 with nu = u0 L / Re,
    200 steps, FP64: every population of every node vs the oracle."""
    n, u0, Re = 32, 0.04, 100.0
    tau = 3.0 * u0 * n / Re + 0.5
    rho, u = inputs.tgv3d_fields(n, u0)
    tags = inputs.all_fluid(n, n, n)
    o, L = make_pair(tags, q=19, tau=tau, rho=rho, u=u)
    assert L.variant == "D3Q19/f64/bgk/uniform"
    ser = L.step_reduce(200, 50)
    o_ser = []
    for k in range(5):
        o_ser.append(o.moments())
        if k < 4:
            o.run(50)
    f = L.read_populations()
    err = max_rel_pop_error(f, o.f, tags)
    _print("tgv32 max rel pop err", err)
    assert err <= TOL
    r_g, u_g = L.read_fields()
    r_o, u_o = o.fields()
    assert rel_l2(u_g, u_o) <= TOL and rel_l2(r_g, r_o) <= TOL
    for s, m in zip(ser, o_ser):
        assert abs(s["kinetic_energy"] * s["n_fluid"] - m["ke_sum"]) <= TOL * m["ke_sum"]
        assert abs(s["kinetic_energy_rho"] - m["ke_rho_sum"]) <= TOL * m["ke_rho_sum"]
        assert abs(s["mass_delta"] - m["mass_delta"]) <= TOL * n ** 3
        assert np.allclose(s["momentum"], m["momentum"], rtol=0, atol=TOL * n ** 3 * u0)
        assert np.allclose(s["velocity_sum"], m["sum_u"], rtol=0, atol=TOL * n ** 3 * u0)
        assert s["n_nonfinite"] == 0


# ---------------------------------------------------------------- cavity
@pytest.mark.parametrize("steps", [150, 151])
def test_cavity_d3q19_fp64(steps):
    """Lid-driven cavity (solid shell, moving lid), ragged tile coverage."""
    n = 26
    tags = inputs.cavity_tags(n)
    o, L = make_pair(tags, q=19, tau=0.6, wall_velocity=[(0.1, 0, 0)])
    assert L.variant == "D3Q19/f64/bgk/tagged"
    L.step(steps)
    o.run(steps)
    f = L.read_populations()
    err = max_rel_pop_error(f, o.f, tags)
    _print("cavity", steps, err)
    assert err <= TOL
    m = L.reduce()
    mo = o.moments()
    assert abs(m["mass_delta"] - mo["mass_delta"]) <= 1e-12 * m["mass"]
    # momentum sums differ by no more than the populations' differences allow
    bound = momentum_bound(f, o.f, tags, 19)
    dp = np.abs(m["momentum"] - mo["momentum"])
    _print("cavity momentum diff", dp, "bound", bound)
    assert np.all(dp <= bound)


# ---------------------------------------------------------------- porous
@pytest.mark.parametrize("q", [19, 27])
def test_porous_trt_force_fp64(q):
    """TRT (Lambda = 3/16) with a body force through a random solid, odd step count,
    non-cubic ragged lattice."""
    nx, ny, nz = 40, 22, 18
    tags = inputs.random_tags(nx, ny, nz, seed=3, solid_frac=0.3, wall_frac=0.0, fluid_tags=(inputs.TAG_TRT,))
    rho, u = inputs.random_fields(nx, ny, nz, seed=5)
    o, L = make_pair(tags, q=q, tau=1.0, force=(1e-5, 2e-6, 0.0), rho=rho, u=u)
    L.step(101)
    o.run(101)
    err = max_rel_pop_error(L.read_populations(), o.f, tags)
    _print("porous", q, err)
    assert err <= TOL


@pytest.mark.parametrize("q", [19, 27])
def test_mixed_models_and_walls_fp64(q):
    """Every fluid model and two moving walls in one lattice (the all-model kernel)."""
    nx, ny, nz = 37, 19, 11
    tags = inputs.random_tags(nx, ny, nz, seed=11, solid_frac=0.15, wall_frac=0.1,
                              fluid_tags=(inputs.TAG_BGK, inputs.TAG_TRT, inputs.TAG_SMAG, inputs.TAG_REG,
                                          inputs.TAG_RR))
    rho, u = inputs.random_fields(nx, ny, nz, seed=12)
    kw = dict(tau=0.7, smag_cs=0.15, force=(0.0, 1e-5, -1e-5), wall_velocity=[(0.05, 0, 0), (0, -0.04, 0.02)])
    o, L = make_pair(tags, q=q, rho=rho, u=u, **kw)
    assert L.variant.endswith("/all/tagged")
    L.step(57)
    o.run(57)
    err = max_rel_pop_error(L.read_populations(), o.f, tags)
    _print("mixed", q, err)
    assert err <= TOL


@pytest.mark.parametrize("q,steps", [(19, 101), (27, 64)])
def test_recursive_regularized_cavity_and_force_fp64(q, steps):
    """Recursive regularized model in a lid-driven cavity with a body force, from
    a random moving state (the rr-only kernel), odd and even step counts."""
    n = 22
    tags = inputs.cavity_tags(n, fluid_tag=inputs.TAG_RR)
    rho, u = inputs.random_fields(n, n, n, seed=91, du=0.03)
    o, L = make_pair(tags, q=q, tau=0.53, force=(1e-5, -2e-5, 0.0), wall_velocity=[(0.08, 0, 0)], rho=rho, u=u)
    assert L.variant == f"D3Q{q}/f64/rr/tagged"
    L.step(steps)
    o.run(steps)
    err = max_rel_pop_error(L.read_populations(), o.f, tags)
    _print("rr cavity", q, steps, err)
    assert err <= TOL


@pytest.mark.parametrize("q,steps", [(19, 101), (27, 64)])
def test_regularized_cavity_and_force_fp64(q, steps):
    """Regularized BGK in a lid-driven cavity with a body force (the regularized-
    only kernel), odd and even step counts."""
    n = 22
    tags = inputs.cavity_tags(n, fluid_tag=inputs.TAG_REG)
    o, L = make_pair(tags, q=q, tau=0.56, force=(1e-5, 0.0, -2e-5), wall_velocity=[(0.08, 0, 0)])
    assert L.variant == f"D3Q{q}/f64/reg/tagged"
    L.step(steps)
    o.run(steps)
    err = max_rel_pop_error(L.read_populations(), o.f, tags)
    _print("reg cavity", q, steps, err)
    assert err <= TOL


def _open_channel(nx, ny, nz, bulk, low=inputs.TAG_VIN, high=inputs.TAG_POUT):
    t = inputs.channel_tags(nx, ny, nz, fluid_tag=bulk)
    t[:, :, 0] = np.where(t[:, :, 0] == bulk, low, t[:, :, 0])
    t[:, :, -1] = np.where(t[:, :, -1] == bulk, high, t[:, :, -1])
    return t


@pytest.mark.parametrize("q,steps,pair", [(19, 301, (inputs.TAG_VIN, inputs.TAG_POUT)),
                                          (27, 120, (inputs.TAG_VIN, inputs.TAG_POUT)),
                                          (19, 201, (inputs.TAG_PIN, inputs.TAG_VOUT)),
                                          (27, 77, (inputs.TAG_PIN, inputs.TAG_POUT))])
def test_open_boundaries_channel_fp64(q, steps, pair):
    """Regularized velocity / pressure boundaries on both x planes between resting
    walls (TRT bulk, the trt+open kernel), developing channel flow."""
    tags = _open_channel(40, 5, 12, inputs.TAG_TRT, *pair)
    rho, u = inputs.random_fields(40, 5, 12, seed=41, du=0.0)
    o, L = make_pair(tags, q=q, tau=0.8, bc_velocity=(0.04, 0.0, 0.005), bc_density=(1.004, 0.998),
                     rho=rho, u=u)
    assert L.variant == f"D3Q{q}/f64/trt+open/tagged"
    L.step(steps)
    o.run(steps)
    err = max_rel_pop_error(L.read_populations(), o.f, tags)
    _print("open channel", q, steps, err)
    assert err <= TOL


def test_open_boundaries_with_every_model_fp64():
    """Open boundaries in the all-model kernel: regularized bulk, a moving lid and a
    body force (not applied on the boundary nodes)."""
    tags = _open_channel(33, 4, 10, inputs.TAG_REG)
    tags[-1, :, 1:-1] = inputs.TAG_WALL0
    tags[3:6, 1:3, 15] = inputs.TAG_SMAG
    tags[3:6, 1:3, 20] = inputs.TAG_BGK
    o, L = make_pair(tags, q=19, tau=0.7, smag_cs=0.12, force=(2e-6, 0, 0), bc_velocity=(0.03, 0, 0),
                     bc_density=(1.0, 1.0), wall_velocity=[(0.02, 0, 0)])
    assert L.variant.endswith("/all/tagged")
    L.step(151)
    o.run(151)
    err = max_rel_pop_error(L.read_populations(), o.f, tags)
    _print("open all", err)
    assert err <= TOL


def test_tgv_d3q27_smagorinsky_fp64():
    n = 24
    rho, u = inputs.tgv3d_fields(n, 0.05)
    tags = inputs.all_fluid(n, n, n, inputs.TAG_SMAG)
    o, L = make_pair(tags, q=27, tau=0.505, smag_cs=0.1, rho=rho, u=u)
    assert L.variant == "D3Q27/f64/bgk+smag/uniform"
    L.step(120)
    o.run(120)
    err = max_rel_pop_error(L.read_populations(), o.f, tags)
    _print("tgv27 smag", err)
    assert err <= TOL


@pytest.mark.parametrize("shape", [(1, 1, 18), (3, 1, 5), (65, 2, 3), (300, 3, 2)])
def test_degenerate_and_wide_shapes_fp64(shape):
    """Single-node-wide axes (periodic self-neighbours), wide rows, few planes."""
    nx, ny, nz = shape
    tags = inputs.random_tags(nx, ny, nz, seed=nx * 7 + ny, solid_frac=0.2, wall_frac=0.1)
    if not fluid_mask(tags).any():
        tags[0, 0, 0] = inputs.TAG_BGK
    rho, u = inputs.random_fields(nx, ny, nz, seed=2)
    o, L = make_pair(tags, q=19, tau=0.9, rho=rho, u=u, wall_velocity=[(0.03, 0, 0), (0, 0, 0.02)])
    L.step(33)
    o.run(33)
    assert max_rel_pop_error(L.read_populations(), o.f, tags) <= TOL


def test_zero_steps_and_single_cell():
    tags = np.zeros((3, 3, 3), np.uint8)
    tags[1, 1, 1] = inputs.TAG_BGK
    rho, u = inputs.random_fields(3, 3, 3, seed=1, du=0.05)
    o, L = make_pair(tags, q=27, tau=0.75, rho=rho, u=u)
    f0 = L.read_populations()
    L.step(0)
    assert np.array_equal(L.read_populations(), f0)
    L.step(9)
    o.run(9)
    assert max_rel_pop_error(L.read_populations(), o.f, tags) <= TOL


# ------------------------------------------------------- determinism (T6)
@pytest.mark.parametrize("prec", [lbm.LBM_F64, lbm.LBM_F32, lbm.LBM_F16S])
def test_launch_shape_is_bitwise_irrelevant(prec):
    nx, ny, nz = 70, 21, 9
    tags = inputs.random_tags(nx, ny, nz, seed=21, solid_frac=0.2, wall_frac=0.05)
    rho, u = inputs.random_fields(nx, ny, nz, seed=22)
    outs = []
    for tx, ty in ((32, 8), (64, 4), (128, 2), (256, 1)):
        L = lbm.Lattice(tags, q=19, prec=prec, tau=0.8, wall_velocity=[(0.05, 0, 0), (0, 0.02, 0)])
        L.set_launch(tx, ty)
        L.init_equilibrium(rho, u)
        L.step(13)
        outs.append(L.read_populations())
        L.close()
    for f in outs[1:]:
        assert np.array_equal(f, outs[0])



# Row-form addressing (nx a power of two in [64, 4096], tiles at least 64 wide;
# every wave in FP16 storage, the wall waves of mostly-fluid tagged lattices in
# FP32/FP64) must give exactly the node-form result (tiles 32 wide): the
# arithmetic is the same, only the addresses are formed differently.
F16S, F32, F64 = lbm.LBM_F16S, lbm.LBM_F32, lbm.LBM_F64


def _within_f16_rounding(a, b, q, rho0, n_steps):
    """Two FP16-storage runs that differ only where the compiler fused one
    multiply-add differently: few populations differ, each by at most about
    one FP16 rounding of its shifted value h = f - w rho0 per step taken."""
    w = np.array([lbm.lbm_velocity(q, i)[1] for i in range(q)])
    # populations first (read_populations) or last (read_cells)
    w = w.reshape((1, q) if a.ndim == 2 else (q, 1, 1, 1))
    h = np.abs(b - w * rho0)
    d = np.abs(a - b)
    frac = np.count_nonzero(d) / d.size
    bound = n_steps * 2.0 ** -10 * h.max()
    _print("f16 two-node vs one-node: differing fraction", frac, "max diff", d.max(), "bound", bound)
    return frac < 1e-3 and d.max() <= bound


@pytest.mark.parametrize("prec,q,nx,ny,nz,kind", [
    (F16S, 19, 64, 21, 9, "walls"), (F16S, 27, 128, 10, 7, "walls"), (F16S, 19, 4096, 3, 2, "walls"),
    (F16S, 19, 64, 5, 11, "periodic"), (F16S, 27, 128, 9, 4, "periodic"), (F16S, 19, 256, 5, 3, "periodic"),
    (F16S, 19, 128, 5, 3, "periodic"), (F16S, 19, 256, 6, 5, "cavity"),
    (F32, 19, 64, 21, 9, "walls"), (F32, 27, 128, 10, 7, "walls"), (F32, 19, 256, 12, 10, "cavity"),
    (F64, 19, 64, 21, 9, "walls"), (F64, 27, 256, 12, 10, "cavity"), (F32, 19, 64, 21, 9, "sparse"),
    (F64, 19, 64, 6, 8, "open"), (F16S, 27, 64, 6, 8, "open"),
    (F64, 19, 128, 9, 7, "mixed"), (F16S, 27, 64, 9, 7, "mixed")])
def test_row_form_matches_node_form(prec, q, nx, ny, nz, kind):
    if kind in ("walls", "sparse"):
        # "sparse": mostly solid, where FP32/FP64 keep the node form
        tags = inputs.random_tags(nx, ny, nz, seed=nx + ny, solid_frac=0.1 if kind == "walls" else 0.6,
                                  wall_frac=0.03)
        kw = dict(tau=0.8, wall_velocity=[(0.05, 0, 0), (0, 0.02, 0)])
    elif kind == "periodic":
        # D3Q27: the Smagorinsky model with a body force; D3Q19: plain BGK
        tags = inputs.all_fluid(nx, ny, nz, tag=inputs.TAG_SMAG if q == 27 else inputs.TAG_BGK)
        kw = dict(tau=0.52, smag_cs=0.1, force=(1e-5, 0, 0)) if q == 27 else dict(tau=0.7)
    elif kind == "open":
        # velocity inlet / pressure outlet on the x planes of a walled channel
        tags = _open_channel(nx, ny, nz, inputs.TAG_TRT)
        kw = dict(tau=0.7, bc_velocity=(0.03, 0, 0), bc_density=(1.0, 1.0))
    elif kind == "mixed":
        # every model in one lattice (the all-model kernel), walls and a force
        tags = inputs.random_tags(nx, ny, nz, seed=31, solid_frac=0.08, wall_frac=0.03,
                                  fluid_tags=(inputs.TAG_BGK, inputs.TAG_TRT, inputs.TAG_SMAG,
                                              inputs.TAG_REG, inputs.TAG_RR))
        kw = dict(tau=0.7, smag_cs=0.1, force=(1e-5, 0, 0), wall_velocity=[(0.05, 0, 0), (0, 0.02, 0)])
    else:
        tags = _box_cavity(nx, ny, nz)
        kw = dict(tau=0.6, wall_velocity=[(0.1, 0, 0)])
    rho, u = inputs.random_fields(nx, ny, nz, seed=7)
    outs, sers, names = [], [], []
    # explicit tiles (one node per lane), then the default launch, which for
    # FP16 lattices of one model without walls and power-of-two rows of at
    # least 128 nodes runs two nodes per lane
    for tx in (32, 64, 128, 256, None):
        L = lbm.Lattice(tags, q=q, prec=prec, **kw)
        if tx is not None:
            L.set_launch(tx, 256 // tx)
        names.append(L.variant)
        L.init_equilibrium(rho, u)
        sers.append(L.step_reduce(9, 3))
        L.step(4)
        outs.append(L.read_populations())
        L.close()
    _print(prec, q, nx, ny, nz, kind, names)
    fluid = int(((tags >= 1) & (tags <= 10)).sum())
    rows = prec == F16S or 2 * fluid >= tags.size
    assert not names[0].endswith("/rows") and all(n.endswith("/rows") == rows for n in names[1:4])
    pairs = prec == F16S and kind == "periodic" and nx >= 128
    assert names[4].endswith("/pairs") == pairs, names[4]
    for k, (f, ser) in enumerate(zip(outs[1:], sers[1:])):
        if k == 3 and pairs:
            # the two-node even step: one FP16 rounding apart at most, rarely
            assert _within_f16_rounding(f, outs[0], q, 1.0, 13)
        else:
            assert np.array_equal(f, outs[0])
        # reductions: the per-tile partials follow the tile shape, so the FP64
        # sums differ in summation order only
        for a, b in zip(ser, sers[0]):
            assert a.keys() == b.keys()
            for k in a:
                assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-10), k



def test_row_form_full_size_tgv512_f16():
    """The 512^3 D3Q27 Taylor-Green lattice in FP16 storage (3.6e9 population
    elements, past 2^31): the row form (256-wide tiles) and the node form
    (32-wide tiles) give bitwise-equal populations after an even and an odd
    step, and the default launch (its even step with two nodes per lane) the
    same up to a rare FP16 rounding, on sampled nodes that include the periodic
    faces and the last block of the array."""
    tags, kw, rho, u, _ = _bench_workload("tgv512_d3q27_smag")
    nz, ny, nx = tags.shape
    rng = np.random.default_rng(11)
    faces = [((z * ny + y) * nx + x) for z in (0, nz - 1) for y in (0, 17, ny - 1) for x in range(nx)]
    tail = list(range(nx * ny * nz - 5000, nx * ny * nz))
    cells = np.unique(np.concatenate([faces, tail, rng.choice(nx * ny * nz, 20000, replace=False)]))
    outs, names = [], []
    for tx in (None, 256, 32):
        L = lbm.Lattice(tags, prec=lbm.LBM_F16S, **kw)
        if tx is not None:
            L.set_launch(tx, 256 // tx)
        names.append(L.variant)
        L.init_equilibrium(rho, u)
        L.step(2)
        outs.append(L.read_cells(cells))
        L.close()
    _print("tgv512 f16", names, cells.size)
    assert names[0].endswith("/pairs") and names[1].endswith("/rows") and not names[2].endswith("/rows")
    assert np.array_equal(outs[1], outs[2])
    assert _within_f16_rounding(outs[0], outs[2], 27, kw.get("rho0", 1.0), 2)

def _box_cavity(nx, ny, nz):
    """Walls on all six faces, a moving lid (tag 16) on the top plane."""
    t = np.ones((nz, ny, nx), np.uint8)
    t[:, :, 0] = t[:, :, -1] = 0
    t[:, 0, :] = t[:, -1, :] = 0
    t[0] = 0
    t[-1] = 16
    return t

def test_reductions_repeatable():
    n = 40
    rho, u = inputs.tgv3d_fields(n, 0.05)
    L = lbm.Lattice(inputs.all_fluid(n, n, n), q=19, prec=lbm.LBM_F32, tau=0.6)
    L.init_equilibrium(rho, u)
    a = L.step_reduce(20, 5)
    L.init_equilibrium(rho, u)
    b = L.step_reduce(20, 5)
    for x, y in zip(a, b):
        assert x["kinetic_energy"] == y["kinetic_energy"] and x["mass_delta"] == y["mass_delta"]


def test_fused_and_standalone_reductions_agree():
    """The reduction fused into a step and the standalone pass see the same state."""
    n = 20
    tags = inputs.cavity_tags(n)
    L = lbm.Lattice(tags, q=19, prec=lbm.LBM_F64, tau=0.6, wall_velocity=[(0.1, 0, 0)])
    L.init_equilibrium()
    L.step(7)
    m_standalone = L.reduce()
    ser = L.step_reduce(3, 3)  # sample at t=7 fused into the next step, t=10 standalone
    assert ser[0]["step"] == 7 and ser[1]["step"] == 10
    for k in ("mass_delta", "kinetic_energy", "kinetic_energy_rho"):
        assert abs(ser[0][k] - m_standalone[k]) <= 1e-14 * max(1e-300, abs(m_standalone[k])) + 1e-18


# --------------------------------------------------------- checkpoint (T11)
@pytest.mark.parametrize("prec", [lbm.LBM_F64, lbm.LBM_F32, lbm.LBM_F16S])
@pytest.mark.parametrize("steps", [10, 11])
def test_checkpoint_roundtrip_bitwise(prec, steps):
    """Shifted-state checkpoints restore bit for bit in every precision and
    parity; unshifted ones are exact for FP32/FP16 storage and within one FP64
    rounding of f for FP64 storage."""
    nx, ny, nz = 33, 17, 12
    tags = inputs.random_tags(nx, ny, nz, seed=31, solid_frac=0.2, wall_frac=0.05)
    rho, u = inputs.random_fields(nx, ny, nz, seed=32)
    kw = dict(q=19, prec=prec, tau=0.7, wall_velocity=[(0.04, 0, 0), (0, 0, 0.03)])
    A = lbm.Lattice(tags, **kw)
    A.init_equilibrium(rho, u)
    A.step(steps)
    ck = A.read_state()
    fk = A.read_populations()
    B = lbm.Lattice(tags, **kw)
    B.write_state(ck, t=A.time)
    assert B.time == steps
    C = lbm.Lattice(tags, **kw)
    C.write_populations(fk, t=A.time)
    A.step(8)
    B.step(8)
    C.step(8)
    fa = A.read_populations()
    assert np.array_equal(fa, B.read_populations())
    fc = C.read_populations()
    if prec == lbm.LBM_F64:
        assert max_rel_pop_error(fc, fa, tags) <= 1e-14
    else:
        assert np.array_equal(fa, fc)


def test_read_cells_matches_full_read():
    nx, ny, nz = 29, 13, 7
    tags = inputs.random_tags(nx, ny, nz, seed=41)
    L = lbm.Lattice(tags, q=27, prec=lbm.LBM_F64, tau=0.7, wall_velocity=[(0.02, 0, 0), (0, 0, 0)])
    rho, u = inputs.random_fields(nx, ny, nz, seed=42)
    L.init_equilibrium(rho, u)
    L.step(5)
    f = L.read_populations().reshape(27, -1)
    cells = np.array([0, 5, 100, nx * ny * nz - 1, 777])
    assert np.array_equal(L.read_cells(cells), f[:, cells].T)


def test_torch_owned_buffer():
    n = 16
    rho, u = inputs.tgv3d_fields(n, 0.04)
    A = lbm.Lattice(inputs.all_fluid(n, n, n), q=19, tau=0.6)
    B = lbm.Lattice(inputs.all_fluid(n, n, n), q=19, tau=0.6, torch_buffer=True)
    for L in (A, B):
        L.init_equilibrium(rho, u)
        L.step(10)
    assert np.array_equal(A.read_populations(), B.read_populations())


def test_nonfinite_detection():
    n = 8
    L = lbm.Lattice(inputs.all_fluid(n, n, n), q=19, prec=lbm.LBM_F32, tau=0.6)
    rho = np.ones((n, n, n))
    rho[3, 3, 3] = np.nan
    L.init_equilibrium(rho, None)
    with pytest.raises(lbm.LbmError) as e:
        L.reduce()
    assert e.value.status == lbm.LBM_EUNSTABLE


# ------------------------------------------------------ reduced precision
@pytest.mark.parametrize("prec,bound", [(lbm.LBM_F32, 1e-4), (lbm.LBM_F16S, 3e-2)])
def test_reduced_precision_error_is_stated(prec, bound):
    """FP32-shifted and FP16-storage vs the FP64 GPU path on the 32^3 Taylor-Green
    (200 steps): relative L2 velocity error printed; sanity bound only."""
    n, u0 = 32, 0.04
    tau = 3.0 * u0 * n / 100.0 + 0.5
    rho, u = inputs.tgv3d_fields(n, u0)
    res = {}
    for p in (lbm.LBM_F64, prec):
        L = lbm.Lattice(inputs.all_fluid(n, n, n), q=19, prec=p, tau=tau)
        L.init_equilibrium(rho, u)
        ser = L.step_reduce(200, 200)
        res[p] = (L.read_fields()[1], ser[-1]["kinetic_energy"])
    e_u = rel_l2(res[prec][0], res[lbm.LBM_F64][0])
    e_k = abs(res[prec][1] / res[lbm.LBM_F64][1] - 1.0)
    _print(f"precision {prec}: velocity rel L2 {e_u:.3e}, k rel err {e_k:.3e}")
    assert e_u < bound and e_k < bound


def test_enstrophy_vs_oracle():
    """Eighth-order finite-difference enstrophy (Eq. 5) of a running D3Q27
    Taylor-Green lattice: GPU vs oracle (on the oracle's own run), 1e-12."""
    n = 24
    rho, u = inputs.tgv3d_fields(n, 0.05)
    tags = inputs.all_fluid(n, n, n, inputs.TAG_SMAG)
    o, L = make_pair(tags, q=27, tau=0.51, smag_cs=0.1, rho=rho, u=u)
    L.step(31)
    o.run(31)
    _, uo = o.fields()
    e_o = oracle.enstrophy(uo)
    e_g = L.enstrophy()
    _print("enstrophy", e_g, e_o)
    assert abs(e_g / e_o - 1.0) <= 1e-12
    walled = lbm.Lattice(inputs.cavity_tags(12), q=19, tau=0.6)
    with pytest.raises(lbm.LbmError) as e:
        walled.enstrophy()
    assert e.value.status == lbm.LBM_EUNSUPPORTED


# ------------------------------------------- full-size cavity, sampled cells
def _bench_workload(name):
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    return bench.build_workload(name)


def test_full_size_tgv512_sampled_cells():
    """The headline workload at its full size and launch configuration (512^3
    D3Q27 BGK+Smagorinsky Taylor-Green: the uniform kernels; in FP16 the
    two-node even step) from the Taylor-Green state with random perturbations,
    3 steps (an odd count: even and odd launches), in every precision: sampled
    nodes (the periodic faces, the last storage block, random nodes) match the
    oracle's populations (FP64 to 1e-12 relative; FP32 storage within 1e-6;
    FP16 storage within 3 roundings of h)."""
    tags, kw, rho, u, _ = _bench_workload("tgv512_d3q27_smag")
    nz, ny, nx = tags.shape
    r2, u2 = inputs.random_fields(nx, ny, nz, seed=79, du=0.005, drho=0.002)
    rho, u = rho + (r2 - 1.0), u + u2
    o = oracle.Oracle(nx, ny, nz, tags=tags, **kw)
    o.init_equilibrium(rho, u)
    o.run(3)
    rng = np.random.default_rng(12)
    faces = [((z * ny + y) * nx + x) for z in (0, nz - 1) for y in (0, 255, ny - 1) for x in range(nx)]
    tail = list(range(nx * ny * nz - 4096, nx * ny * nz))
    cells = np.unique(np.concatenate([faces, tail, rng.choice(nx * ny * nz, 20000, replace=False)]))
    ref = o.f.reshape(kw["q"], -1)[:, cells].T
    del o
    for prec, bound in ((lbm.LBM_F64, TOL), (lbm.LBM_F32, 1e-6), (lbm.LBM_F16S, 3 * 2.0**-11)):
        L = lbm.Lattice(tags, prec=prec, **kw)
        L.init_equilibrium(rho, u)
        L.step(3)
        g = L.read_cells(cells)
        name = L.variant
        L.close()
        err = float(np.abs(g / ref - 1.0).max())
        _print("full tgv512", name, cells.size, err)
        assert err <= bound
    assert name.endswith("/pairs")


@pytest.mark.parametrize("workload", ["porous400_d3q19_trt", "porous480_open_d3q19_trt"])
def test_full_size_porous_sampled_cells(workload):
    """The porous-rock workloads at their full size and launch configuration
    (400^3 D3Q19 TRT with a body force, and the same rock between 40-plane
    buffers with pressure boundaries, 480 x 400 x 400: brick layout, waves
    only for the bricks that hold fluid) from a random near-rest state, 11
    steps, in every precision: sampled fluid nodes (random ones, nodes next to
    the rock and, with buffers, the boundary planes) match the oracle's
    populations (FP64 to 1e-12 relative; FP32 storage within 1e-5; FP16
    storage within 11 roundings of h, as for the cavity)."""
    tags, kw, _, _, _ = _bench_workload(workload)
    nz, ny, nx = tags.shape
    rho, u = inputs.random_fields(nx, ny, nz, seed=78, du=0.01, drho=0.005)
    o = oracle.Oracle(nx, ny, nz, tags=tags, **kw)
    o.init_equilibrium(rho, u)
    o.run(11)
    fl3 = fluid_mask(tags)
    fl = np.flatnonzero(fl3.reshape(-1))
    # fluid nodes with a non-fluid face neighbour (bounce-back links)
    near = fl3 & ~(np.roll(fl3, 1, 0) & np.roll(fl3, -1, 0) & np.roll(fl3, 1, 1) & np.roll(fl3, -1, 1)
                   & np.roll(fl3, 1, 2) & np.roll(fl3, -1, 2))
    rng = np.random.default_rng(6)
    picks = [rng.choice(fl, 20000, replace=False), rng.choice(np.flatnonzero(near.reshape(-1)), 5000, replace=False)]
    if workload == "porous480_open_d3q19_trt":
        # the inlet and outlet planes and their neighbours
        for x in (0, 1, nx - 2, nx - 1):
            picks.append(rng.choice(np.arange(ny * nz) * nx + x, 1000, replace=False))
    cells = np.unique(np.concatenate(picks))
    ref = o.f.reshape(kw["q"], -1)[:, cells].T
    del o
    for prec, bound in ((lbm.LBM_F64, TOL), (lbm.LBM_F32, 1e-5), (lbm.LBM_F16S, 11 * 2.0**-11)):
        L = lbm.Lattice(tags, prec=prec, **kw)
        assert L.variant.endswith("/bricks"), L.variant
        L.init_equilibrium(rho, u)
        L.step(11)
        g = L.read_cells(cells)
        L.close()
        err = float(np.abs(g / ref - 1.0).max())
        _print("full porous", prec, cells.size, err)
        assert err <= bound


# FP16 storage: each step rounds h = f - w rho0 once (unit roundoff 2^-11), and
# |h| <= f next to the moving lid, so 11 steps stay within 11 * 2^-11 of f.
@pytest.mark.parametrize("prec,bound", [(lbm.LBM_F64, TOL), (lbm.LBM_F32, 1e-5), (lbm.LBM_F16S, 11 * 2.0**-11)])
def test_full_size_cavity_sampled_cells(prec, bound):
    """The benchmark's workload at its full size and launch configuration (the
    256^3 lid-driven cavity, default tiling) from a random near-rest state, 11
    steps: sampled cells (all lid-adjacent nodes of four rows, the x-wall
    columns, and random nodes) match the oracle's populations (FP64 to 1e-12
    relative; FP32 storage within 1e-5; FP16 storage within its rounding bound)."""
    tags, kw, _, _, _ = _bench_workload("cavity256_d3q19_bgk")
    nz, ny, nx = tags.shape
    rho, u = inputs.random_fields(nx, ny, nz, seed=77, du=0.01, drho=0.005)
    o, L = make_pair(tags, prec=prec, rho=rho, u=u, **kw)
    L.step(11)
    o.run(11)
    rng = np.random.default_rng(5)
    fl = np.flatnonzero(fluid_mask(tags).reshape(-1))
    lid = [((nz - 2) * ny + y) * nx + x for y in (1, 2, 127, ny - 2) for x in range(1, nx - 1)]
    xwall = [(z * ny + y) * nx + x for z in (1, 128, nz - 2) for y in range(1, ny - 1) for x in (1, nx - 2)]
    cells = np.unique(np.concatenate([lid, xwall, rng.choice(fl, 20000, replace=False)]))
    g = L.read_cells(cells)
    ref = o.f.reshape(kw["q"], -1)[:, cells].T
    err = float(np.abs(g / ref - 1.0).max())
    _print("full cavity", prec, cells.size, err)
    assert err <= bound
