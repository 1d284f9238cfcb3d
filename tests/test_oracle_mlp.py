"""Pins of the learned-closure oracle (FP64 numpy + the C BF16 emulation)."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp as om
from paper_2506_09242_amd import inputs


def _params(seed=1234, mean=None, sd=None):
    P = inputs.mlp_he_init(seed).astype(np.float64)
    rng = np.random.default_rng(seed)
    P[om.OB1:om.OW2] = 0.1 * rng.standard_normal(32)
    P[om.OB2:om.OW3] = 0.1 * rng.standard_normal(32)
    P[om.OB3] = -0.5
    P[om.OMEAN:om.OSTD] = mean if mean is not None else 0.0
    P[om.OSTD:om.NP] = sd if sd is not None else 1.0
    return P


def test_backprop_matches_finite_differences():
    """Oracle gradient vs central differences (h = 1e-6) of the FP64 loss."""
    rng = np.random.default_rng(0)
    P = _params(7, mean=rng.normal(0, 0.1, 7), sd=rng.uniform(0.5, 2, 7))
    X = rng.standard_normal((64, 7))
    Y = rng.uniform(0, 2, 64)
    _, g = om.loss_and_grad(P, X, Y)
    h = 1e-6
    idx = list(range(0, om.OMEAN, 7)) + [om.OB3, om.OW3 + 3, om.OB2 + 5, om.OB1 + 1]
    for k in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (om.loss_and_grad(Pp, X, Y)[0] - om.loss_and_grad(Pm, X, Y)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])
    assert np.all(g[om.OMEAN:] == 0.0)


def test_bf16_rounding_matches_torch():
    """RNE to bfloat16 against torch's conversion (a library routine), incl. ties."""
    import torch
    rng = np.random.default_rng(1)
    vals = list(rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 8, 2000))
    # exact ties: 1 + 2^-8 (tie to even -> 1), 1 + 3*2^-8 (-> 1 + 2^-6), negatives
    vals += [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, -0.0, 3.0e38]
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    ours = np.array([oracle.bf16(v) for v in np.array(vals, np.float32)])
    assert np.array_equal(ours, ref)


def test_network_special_cases():
    nu0 = 0.01
    P = np.zeros(om.NP)
    P[om.OSTD:] = 1.0
    x = np.array([0.3, -0.2, 0.1, 0.05, 0.0, -0.1, 1.0])
    # zero weights and biases: softplus(0) = ln 2
    assert abs(oracle.mlp_eddy_viscosity(P, x, nu0) - nu0 * math.log(2.0)) < 1e-18
    # zero last layer, b3 = -40: closure switched off (nu_t ~ 4e-18 nu0)
    P2 = _params(3)
    P2[om.OW3:om.OB3] = 0.0
    P2[om.OB3] = -40.0
    assert oracle.mlp_eddy_viscosity(P2, x, nu0) < 1e-17 * nu0
    # one active path: W1[0][0] = W2[0][0] = W3[0] = 1 -> softplus(relu(x0))
    P3 = np.zeros(om.NP)
    P3[om.OSTD:] = 1.0
    P3[om.OW1] = 1.0
    P3[om.OW2] = 1.0
    P3[om.OW3] = 1.0
    for x0 in (0.75, -0.5, 2.5):
        xx = x.copy()
        xx[0] = x0
        expect = nu0 * math.log1p(math.exp(max(x0, 0.0)))
        assert abs(oracle.mlp_eddy_viscosity(P3, xx, nu0) - expect) < 1e-15
    # the deployed (BF16) network is the FP64 network up to BF16 rounding
    rng = np.random.default_rng(5)
    P4 = _params(9)
    X = rng.standard_normal((200, 7))
    y64, _ = om.forward(P4, X)
    yb = om.infer_deployed(P4, X, 1.0)
    assert np.max(np.abs(yb - y64) / np.abs(y64)) < 0.05


def test_adam_first_step_is_signed_lr():
    """From zero moments, Adam's first update is lr * g / (|g| + eps')."""
    rng = np.random.default_rng(2)
    P = _params(11)
    X = rng.standard_normal((32, 7))
    Y = rng.uniform(0, 1, 32)
    _, g = om.loss_and_grad(P, X, Y)
    P1, log = om.adam_train(P, X, Y, np.arange(32), 32, 1, 1e-3)
    d = (P - P1)[:om.OMEAN]
    gg = g[:om.OMEAN]
    # bias-corrected m = g, sqrt(v) = |g| after one step
    assert np.allclose(d, 1e-3 * gg / (np.abs(gg) + 1e-8), rtol=1e-9, atol=1e-18)
    assert np.array_equal(P1[om.OMEAN:], P[om.OMEAN:])


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((512, 7))
    Y = np.log1p(np.exp(X[:, 0] - 0.5 * X[:, 1]))
    P = _params(13)
    perm = np.concatenate([inputs.permutation(512, 100 + e) for e in range(20)])
    _, log = om.adam_train(P, X, Y, perm, 64, 20, 3e-3)
    assert log[-1] < 0.2 * log[0]


def test_filter_uniform_and_blockwise_constant_fields():
    """Blockwise-constant fine fields: no subgrid stress; targets 0."""
    f, n = 2, 8
    rng = np.random.default_rng(4)
    coarse = rng.uniform(-0.05, 0.05, (3, n // f, n // f, n // f))
    u = coarse.repeat(f, 1).repeat(f, 2).repeat(f, 3)
    rho = np.ones((n, n, n))
    feat, tgt, aux = om.box_filter_targets(rho, u, f, 0.01)
    assert np.abs(aux["T"]).max() < 1e-17
    assert np.all(tgt == 0.0)
    assert np.allclose(aux["U"], coarse, atol=1e-17)


def test_filter_subgrid_variance_and_strain():
    """u_x = U0 + a (-1)^x on the fine grid: T_xx = a^2 exactly; a coarse shear
    U_x = s sin(k Z) has the discrete central-difference strain
    S_xz = (s/2) cos(k Z) sin(k)."""
    f, n = 2, 16
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    a, U0 = 0.01, 0.02
    u = np.zeros((3, n, n, n))
    u[0] = U0 + a * (-1.0) ** x
    feat, tgt, aux = om.box_filter_targets(np.ones((n, n, n)), u, f, 0.01)
    assert np.allclose(aux["T"][0, 0], a * a, rtol=1e-12)
    assert np.abs(aux["T"][1, 1]).max() < 1e-18
    nc = n // f
    s, k = 0.03, 2 * np.pi / nc
    Z = np.arange(nc)
    uc = np.zeros((3, n, n, n))
    uc[0] = (s * np.sin(k * Z)).repeat(f)[z]
    _, _, aux2 = om.box_filter_targets(np.ones((n, n, n)), uc, f, 0.01)
    expect = 0.5 * s * np.cos(k * Z) * np.sin(k)
    assert np.allclose(aux2["S"][0, 2][:, 0, 0], expect, atol=1e-15)
    assert np.allclose(aux2["S"][2, 0], aux2["S"][0, 2])


def test_favre_filter_weights_by_density():
    """One 2^3 block pattern with rho = 1 + a s, u_x = U0 + b s, u_y = V0 + c s
    (s = +1 on the block's low-x half, -1 on the other): the density-weighted
    means are U_x = U0 + a b, U_y = V0 + a c and the covariances
    T_xx = b^2 (1 - a^2), T_xy = b c (1 - a^2), T_yy = c^2 (1 - a^2), worked by
    hand (a plain block mean would give U_x = U0 and T_xx = b^2)."""
    f, n = 2, 4
    a, b, c, U0, V0 = 0.5, 0.1, -0.04, 0.2, 0.03
    x = np.arange(n)[None, None, :] * np.ones((n, n, n))
    s = np.where(x % f == 0, 1.0, -1.0)
    rho = 1.0 + a * s
    u = np.zeros((3, n, n, n))
    u[0] = U0 + b * s
    u[1] = V0 + c * s
    rbar, U, T = om.favre_filter(rho, u, f)
    assert np.allclose(rbar, 1.0, rtol=0, atol=1e-15)
    assert np.allclose(U[0], 0.25, rtol=0, atol=1e-15)
    assert np.allclose(U[1], 0.01, rtol=0, atol=1e-15)
    assert np.allclose(U[2], 0.0, rtol=0, atol=1e-15)
    assert np.allclose(T[0, 0], 0.0075, rtol=0, atol=1e-15)
    assert np.allclose(T[0, 1], -0.003, rtol=0, atol=1e-15)
    assert np.allclose(T[1, 0], -0.003, rtol=0, atol=1e-15)
    assert np.allclose(T[1, 1], 0.0012, rtol=0, atol=1e-15)
    assert np.abs(T[2]).max() < 1e-15
    # the full pipeline passes the same filter through
    _, _, aux = om.box_filter_targets(rho, u, f, 0.01)
    assert np.allclose(aux["U"][0], 0.25, rtol=0, atol=1e-15)


def _fine_field_with_stress(Uc, Tc, f):
    """Fine velocity whose factor-f box filter (rho = 1) has coarse mean Uc[3][Z][Y][X]
    and subgrid stress Tc[3][3][Z][Y][X]: each fine node carries Uc + L s with
    L L^T = Tc (Cholesky) and s_a = +1 on the block's low half along axis a, -1 on
    the high half; the eight sign patterns are orthogonal with mean zero, so the
    block covariance is L I L^T = Tc."""
    cz, cy, cx = Uc.shape[1:]
    nz, ny, nx = cz * f, cy * f, cx * f
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sgn = np.stack([np.where(x % f < f // 2, 1.0, -1.0), np.where(y % f < f // 2, 1.0, -1.0),
                    np.where(z % f < f // 2, 1.0, -1.0)])
    Tm = np.moveaxis(Tc, (0, 1), (-2, -1))          # [Z][Y][X][3][3]
    Lc = np.linalg.cholesky(Tm)
    Lf = Lc[z // f, y // f, x // f]                  # [nz][ny][nx][3][3]
    v = np.einsum("...ab,b...->a...", Lf, sgn)
    return Uc[:, z // f, y // f, x // f] + v


@pytest.mark.parametrize("kind", ["shear", "axial"])
def test_eddy_viscosity_target_of_known_stress(kind):
    """Coarse flows with the closed-form discrete strain of a sine (pinned above)
    and a subgrid stress T = -2 nu S + alpha I built into the fine field.  The
    least-squares target of dev(T) on -2 nu_t S is nu for a traceless shear, and
    (2/3) nu for the axial strain S = diag(s, 0, 0) (dev(S):S = (2/3) s^2), in
    either case independent of alpha; a backscattering stress T = +2 nu S + alpha I
    gives 0 (clipped)."""
    f, nc, s, nu = 2, 8, 0.02, 3e-3
    k = 2 * np.pi / nc
    Z = np.arange(nc)
    Uc = np.zeros((3, nc, nc, nc))
    S = np.zeros((3, 3, nc, nc, nc))
    if kind == "shear":
        Uc[0] = (s * np.sin(k * Z))[:, None, None]
        S[0, 2] = S[2, 0] = (0.5 * s * np.cos(k * Z) * np.sin(k))[:, None, None]
        expect = nu
    else:
        Uc[0] = (s * np.sin(k * Z))[None, None, :]
        S[0, 0] = (s * np.cos(k * Z) * np.sin(k))[None, None, :]
        expect = 2.0 / 3.0 * nu
    live = np.einsum("ab...,ab...->...", S, S) > 1e-20
    smax = np.abs(S).max()
    for alpha_mult in (3.0, 40.0):
        alpha = alpha_mult * 2 * nu * smax
        for sign, want in ((-1.0, expect), (1.0, 0.0)):
            T = sign * 2 * nu * S + alpha * np.eye(3)[:, :, None, None, None]
            u = _fine_field_with_stress(Uc, T, f)
            feat, tgt, aux = om.box_filter_targets(np.ones((nc * f,) * 3), u, f, 1.0)
            assert np.allclose(aux["T"], T, rtol=0, atol=1e-14)
            assert np.allclose(aux["S"], S, rtol=0, atol=1e-15)
            nut = tgt.reshape(nc, nc, nc)
            assert np.allclose(nut[live], want, rtol=1e-9, atol=0)


@pytest.mark.parametrize("tau", [0.62, 1.3])
def test_features_equal_couette_nonequilibrium_flux(tau):
    """The feature formula Pi = -2 rho c_s^2 tau_e S against a lattice that carries
    it: the oracle's steady BGK Couette flow at tau = tau_e (linear profile, exact
    for this flow).  Pi^neq_xz measured from its populations, sum c_x c_z (f - f^eq),
    equals the xz feature computed from the flow's own density and central-difference
    strain, with nu_c + nu_t = (tau - 1/2)/3 split between the two."""
    nz, U = 14, 0.02
    tags = inputs.channel_tags(1, 1, nz, top=inputs.TAG_WALL0)
    o = oracle.Oracle(1, 1, nz, q=19, tau=tau, tags=tags, wall_velocity=[(U, 0, 0)])
    o.init_equilibrium()
    o.run(20000)
    rho, u = o.fields()
    c, _, _ = oracle.tables(19)
    nu_tot = (tau - 0.5) / 3.0
    for z in (3, 7, 10):
        fz = o.f[:, z, 0, 0]
        feq = oracle.equilibrium(19, rho[z, 0, 0], u[:, z, 0, 0])
        pi_xz = float(np.sum(c[:, 0] * c[:, 2] * (fz - feq)))
        S = np.zeros((3, 3, 1, 1, 1))
        S[0, 2] = S[2, 0] = 0.25 * (u[0, z + 1, 0, 0] - u[0, z - 1, 0, 0])
        feat = om.closure_features(S, np.full((1, 1, 1), rho[z, 0, 0]), np.full((1, 1, 1), 0.6 * nu_tot),
                                   0.4 * nu_tot)
        assert abs(feat[0, 4] / pi_xz - 1.0) < 1e-9
        assert feat[0, 6] == rho[z, 0, 0]
        assert np.all(feat[0, [0, 1, 2, 3, 5]] == 0.0)
