"""GPU checks of the learned closure: fused BF16-MFMA inference, the fused
collision, the box filter and the FP32 training kernels, against the FP64
oracle (oracle.mlp and the C oracle's BF16-emulated network)."""
import numpy as np
import pytest

import oracle
from oracle import mlp as om
from paper_2506_09242_amd import inputs, lbm

from _util import make_pair, max_rel_pop_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.lib()
    yield


def _print(*a):
    print(*a, flush=True)


def _features(n, seed):
    """Feature rows with the magnitudes a coarse Taylor-Green lattice shows:
    stress moments ~1e-4, density ~1."""
    rng = np.random.default_rng(seed)
    X = np.empty((n, 7))
    X[:, :6] = 1e-4 * rng.standard_normal((n, 6))
    X[:, 6] = 1.0 + 1e-3 * rng.standard_normal(n)
    return X


def _params(seed, X):
    P = inputs.mlp_he_init(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    P[om.OB1:om.OW2] = 0.1 * rng.standard_normal(32)
    P[om.OB2:om.OW3] = 0.1 * rng.standard_normal(32)
    P[om.OB3] = 0.2
    P[om.OMEAN:om.OSTD] = X.mean(0)
    P[om.OSTD:om.NP] = X.std(0)
    return P.astype(np.float32)


def _infer_gpu(P, X, nu0):
    import torch
    feat = torch.tensor(X, dtype=torch.float32, device="cuda")
    out = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
    lbm.lbm_mlp_infer(P, nu0, feat, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def test_mfma_inference_vs_bf16_oracle():
    """Fused-network inference (BF16 MFMA, FP32 accumulate) vs the oracle with
    BF16 inputs/weights/activations and FP64 sums: within 1e-2 relative (one
    BF16 ulp is 2^-8; accumulation order can flip a rounding)."""
    n, nu0 = 4096 + 37, 6.4e-4
    X = _features(n, 1)
    P = _params(1234, X)
    g = _infer_gpu(P, X.astype(np.float32), nu0)
    o = om.infer_deployed(P, X.astype(np.float32), nu0)
    rel = np.abs(g - o) / np.abs(o)
    _print("mlp infer: max rel", rel.max(), "median", np.median(rel))
    assert rel.max() <= 1e-2
    assert np.median(rel) <= 1e-5


def test_mfma_inference_special_cases():
    n, nu0 = 300, 1e-3
    X = _features(n, 2)
    P = np.zeros(om.NP, np.float32)
    P[om.OSTD:] = 1.0
    g = _infer_gpu(P, X.astype(np.float32), nu0)
    assert np.allclose(g, nu0 * np.log(2.0), rtol=1e-6)
    P = _params(5, X)
    P[om.OW3:om.OB3] = 0.0
    P[om.OB3] = -40.0
    g = _infer_gpu(P, X.astype(np.float32), nu0)
    assert np.all(g < 1e-17 * nu0)


def _tgv_mlp_pair(P, n=16, steps=0, tag=inputs.TAG_MLP, oracle_tag=None, prec=lbm.LBM_F64):
    u0 = 0.05
    tau = 3 * u0 * (n / (2 * np.pi)) / 1600.0 + 0.5
    rho, u = inputs.tgv3d_fields(n, u0)
    tags = inputs.all_fluid(n, n, n, tag)
    otags = inputs.all_fluid(n, n, n, oracle_tag or tag)
    o = oracle.Oracle(n, n, n, q=27, tau=tau, smag_cs=0.1, tags=otags, mlp=P)
    o.init_equilibrium(rho, u)
    L = lbm.Lattice(tags, q=27, prec=prec, tau=tau, smag_cs=0.1)
    L.set_mlp(P)
    L.init_equilibrium(rho, u)
    return o, L, tags


def test_fused_closure_switched_off_is_bgk():
    """W3 = 0, b3 = -40: nu_t ~ 4e-18 nu0, the MLP node is BGK at tau0 (1e-12)."""
    X = _features(100, 3)
    P = _params(7, X)
    P[om.OW3:om.OB3] = 0.0
    P[om.OB3] = -40.0
    o, L, tags = _tgv_mlp_pair(P, oracle_tag=inputs.TAG_BGK)
    assert L.variant == "D3Q27/f64/bgk+smag+mlp/uniform"
    L.step(25)
    o.run(25)
    assert max_rel_pop_error(L.read_populations(), o.f, tags) <= 1e-12


def test_fused_closure_fallback_is_smagorinsky():
    """nu_t > 10 nu0 falls back to the Smagorinsky relaxation time (1e-12)."""
    X = _features(100, 4)
    P = _params(8, X)
    P[om.OW3:om.OB3] = 0.0
    P[om.OB3] = 50.0
    o, L, tags = _tgv_mlp_pair(P, oracle_tag=inputs.TAG_SMAG)
    L.step(25)
    o.run(25)
    assert max_rel_pop_error(L.read_populations(), o.f, tags) <= 1e-12


def test_fused_closure_active_matches_oracle():
    """Active network inside the FP64 collision vs the oracle's BF16-emulated
    closure.  nu_t agrees to <= 1e-2 relative per node (BF16 flips), so tau_eff
    to 3e-2 nu_t ~ 2e-5 and, with |f - feq| / f ~ 1e-3, the populations to
    ~1e-7 per step: bound 1e-6 after 5 steps."""
    n = 16
    X = _features(1000, 5)
    P = _params(9, X)
    P[om.OB3] = -1.0
    o, L, tags = _tgv_mlp_pair(P, n=n)
    L.step(5)
    o.run(5)
    err = max_rel_pop_error(L.read_populations(), o.f, tags)
    _print("fused active closure max rel pop err", err)
    assert err <= 1e-6
    # and it is not the Smagorinsky or BGK result
    o2 = oracle.Oracle(n, n, n, q=27, tau=o.cfg.tau, smag_cs=0.1, tags=inputs.all_fluid(n, n, n, inputs.TAG_SMAG))
    rho, u = inputs.tgv3d_fields(n, 0.05)
    o2.init_equilibrium(rho, u)
    o2.run(5)
    assert max_rel_pop_error(L.read_populations(), o2.f, tags) > 1e-5


def test_filter_snapshot_vs_oracle():
    """Box filter + targets of a fine lattice, GPU (FP32 out) vs the oracle's
    numpy filter of its own fine run."""
    import torch
    n, f = 32, 4
    u0 = 0.05
    tau = 0.51
    rho, u = inputs.tgv3d_fields(n, u0)
    tags = inputs.all_fluid(n, n, n, inputs.TAG_SMAG)
    o, L = make_pair(tags, q=27, tau=tau, smag_cs=0.1, rho=rho, u=u)
    L.step(41)
    o.run(41)
    nc = (n // f) ** 3
    feat = torch.empty((nc, 7), dtype=torch.float32, device="cuda")
    tgt = torch.empty(nc, dtype=torch.float32, device="cuda")
    L.filter_snapshot(f, feat, tgt)
    r_o, u_o = o.fields()
    nu_c = (tau - 0.5) / 3.0 / f
    F_o, T_o, _ = om.box_filter_targets(r_o, u_o, f, nu_c)
    F_g = feat.cpu().numpy().astype(np.float64)
    T_g = tgt.cpu().numpy().astype(np.float64)
    scale = np.abs(F_o).max(0)
    assert np.all(np.abs(F_g - F_o) <= 1e-6 * scale + 1e-6 * np.abs(F_o))
    assert np.all(np.abs(T_g - T_o) <= 1e-5 * np.abs(T_o).max() + 1e-5 * np.abs(T_o))
    assert np.count_nonzero(T_o) > nc // 10


def test_training_gradient_vs_oracle():
    """FP32 forward/backward kernels vs FP64 backprop: <= 1e-4 relative (of the
    largest component), and the loss."""
    import torch
    n = 3000
    X = _features(n, 6)
    P = _params(10, X)
    Y = np.abs(np.random.default_rng(7).normal(1.0, 0.5, n))
    loss_o, g_o = om.loss_and_grad(P.astype(np.float64), X.astype(np.float32).astype(np.float64), Y.astype(np.float32))
    dev = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    gp, gl = torch.empty(om.NP, device="cuda"), torch.empty(1, device="cuda")
    lbm.lbm_mlp_grad(dev(P), dev(X), dev(Y), gp, gl)
    torch.cuda.synchronize()
    g = gp.cpu().numpy().astype(np.float64)
    err = np.abs(g - g_o).max() / np.abs(g_o).max()
    _print("grad max err / max |g|", err, "loss", gl.item(), loss_o)
    assert err <= 1e-4
    assert abs(gl.item() / loss_o - 1.0) <= 1e-4


def test_training_adam_vs_oracle():
    """Two epochs of mini-batch Adam (batch 256, seeded permutation): FP32 GPU
    training vs FP64 oracle training; per-epoch losses within 1e-3 relative,
    parameters within 1e-2 of one step's size (lr) everywhere."""
    import torch
    n, batch, epochs, lr = 1024, 256, 2, 1e-3
    X = _features(n, 8)
    P = _params(11, X)
    Y = np.abs(np.random.default_rng(9).normal(1.0, 0.5, n)).astype(np.float32)
    perm = np.concatenate([inputs.permutation(n, 1234 + e) for e in range(epochs)])
    P_o, log_o = om.adam_train(P.astype(np.float64), X.astype(np.float32).astype(np.float64), Y.astype(np.float64),
                               perm, batch, epochs, lr)
    dev = lambda a, dt=torch.float32: torch.tensor(np.asarray(a), dtype=dt, device="cuda")
    Pd = dev(P)
    log = torch.empty(epochs, device="cuda")
    lbm.lbm_mlp_train(Pd, dev(X.astype(np.float32)), dev(Y), dev(perm, torch.int64), batch, epochs, lr, log)
    torch.cuda.synchronize()
    Pg = Pd.cpu().numpy().astype(np.float64)
    d = np.abs(Pg - P_o)
    _print("adam: max |dP|/lr", d.max() / lr, "median", np.median(d) / lr, "log", log.cpu().numpy(), log_o)
    assert np.allclose(log.cpu().numpy(), log_o, rtol=1e-3)
    assert d.max() <= 1e-2 * lr * 8
    assert np.array_equal(Pg[om.OMEAN:], P[om.OMEAN:].astype(np.float64))


def test_closure_pipeline_small():
    """End-to-end learned-closure pipeline at reduced size (fine 64^3 -> coarse
    16^3, 4 snapshots, 2 epochs): every stage runs, training lowers the loss,
    the coarse runs produce finite dissipation errors (reported)."""
    from paper_2506_09242_amd import closure
    res, P = closure.experiment(n_fine=64, factor=4, n_snap=4, n_samples=8192, epochs=3, t_end_tc=4.0,
                                every_fine=20, log=_print)
    assert res["training"]["loss_last"] < res["training"]["loss_first"]
    for name in ("bgk", "smagorinsky", "mlp"):
        e = res["coarse"][name]
        assert not e["unstable"] and np.isfinite(e["eps_rel_l2"])
    assert np.all(np.isfinite(P))
