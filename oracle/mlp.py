"""FP64 oracle of the learned eddy-viscosity closure (test infrastructure only).

Plain numpy, written from the definitions:
  - network 7 -> 32 -> 32 -> 1, ReLU hidden layers, softplus output, inputs
    z-scored with the packed mean/std (packing documented in include/lbm.h);
  - loss = mean over samples of (softplus(net(x)) - y)^2, gradients by
    ordinary backpropagation in FP64;
  - Adam (Kingma & Ba 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
    bias-corrected moments, one step per mini-batch, samples visited in the
    caller's permutation order;
  - inference as deployed: inputs, weights and hidden activations rounded to
    bfloat16 (the C oracle's routine), FP64 sums;
  - training data: box filter over factor^3 fine nodes, Favre velocity
    U = <rho u>/<rho>, subgrid stress T_ij = <rho u_i u_j>/<rho> - U_i U_j,
    resolved strain S from second-order central differences of U on the
    periodic coarse grid, eddy-viscosity target
    nu_t = max(0, -dev(T):S / (2 S:S + 1e-30)) (least-squares projection of
    the deviatoric stress on the eddy-viscosity form -2 nu_t S), and features
    Pi = -2 rho c_s^2 tau_e S (first-order Chapman-Enskog non-equilibrium
    flux a coarse lattice would carry at tau_e = 3 (nu_c + nu_t) + 1/2),
    with c_s^2 = 1/3, plus <rho>.
This module does not import the HIP package.
"""
import numpy as np

from . import bf16, mlp_eddy_viscosity

OW1, OB1, OW2, OB2, OW3, OB3, OMEAN, OSTD, NP = 0, 224, 256, 1280, 1312, 1344, 1345, 1352, 1359


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    return (P[OW1:OB1].reshape(32, 7), P[OB1:OW2], P[OW2:OB2].reshape(32, 32), P[OB2:OW3],
            P[OW3:OB3], P[OB3], P[OMEAN:OSTD], P[OSTD:NP])


def softplus(z):
    return np.where(z > 30.0, z, np.log1p(np.exp(np.minimum(z, 30.0))))


def forward(P, X):
    """Returns softplus(net(x)) and the intermediates (FP64)."""
    W1, b1, W2, b2, W3, b3, mean, sd = unpack(P)
    x = (np.asarray(X, np.float64) - mean) / sd
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ W3 + b3
    return softplus(z3), (x, z1, h1, z2, h2, z3)


def loss_and_grad(P, X, Y):
    """Mean squared error and its gradient w.r.t. the packed vector (mean/std: 0)."""
    W1, b1, W2, b2, W3, b3, mean, sd = unpack(P)
    y, (x, z1, h1, z2, h2, z3) = forward(P, X)
    n = X.shape[0]
    r = y - np.asarray(Y, np.float64)
    loss = np.mean(r * r)
    dz3 = 2.0 * r / n / (1.0 + np.exp(-z3))
    dW3 = dz3 @ h2
    db3 = dz3.sum()
    dz2 = np.outer(dz3, W3) * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    dW1 = dz1.T @ x
    db1 = dz1.sum(0)
    g = np.zeros(NP)
    g[OW1:OB1] = dW1.ravel()
    g[OB1:OW2] = db1
    g[OW2:OB2] = dW2.ravel()
    g[OB2:OW3] = db2
    g[OW3:OB3] = dW3
    g[OB3] = db3
    return loss, g


def adam_train(P, X, Y, perm, batch, epochs, lr):
    """Mini-batch Adam; perm has epochs*n entries (sample order per epoch).
    Returns the final packed vector and the per-epoch mean batch loss."""
    P = np.array(P, dtype=np.float64)
    n = X.shape[0]
    m = np.zeros(NP)
    v = np.zeros(NP)
    b1, b2, eps = 0.9, 0.999, 1e-8
    nb = (n + batch - 1) // batch
    log = []
    t = 0
    for ep in range(epochs):
        acc = 0.0
        for bi in range(nb):
            idx = perm[ep * n + bi * batch: ep * n + min(n, (bi + 1) * batch)]
            loss, g = loss_and_grad(P, X[idx], Y[idx])
            acc += loss / nb
            t += 1
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            upd = lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
            P[:OMEAN] -= upd[:OMEAN]
        log.append(acc)
    return P, np.array(log)


def infer_deployed(P, X, nu0):
    """nu_t of each row as the fused closure computes it (BF16 emulation)."""
    return np.array([mlp_eddy_viscosity(P, row, nu0) for row in np.asarray(X, np.float64)])


def favre_filter(rho, u, factor):
    """Box filter over factor^3 fine blocks: coarse density <rho> (block mean),
    Favre velocity U = <rho u>/<rho> and subgrid stress
    T_ab = <rho u_a u_b>/<rho> - U_a U_b (density-weighted, so that T is the
    block's mass-weighted velocity covariance)."""
    nz, ny, nx = rho.shape
    f = factor
    cz, cy, cx = nz // f, ny // f, nx // f

    def blocks(a):
        return a.reshape(cz, f, cy, f, cx, f).sum(axis=(1, 3, 5))

    sr = blocks(rho)
    U = [blocks(rho * u[a]) / sr for a in range(3)]
    T = np.empty((3, 3) + sr.shape)
    for a in range(3):
        for b in range(3):
            T[a, b] = blocks(rho * u[a] * u[b]) / sr - U[a] * U[b]
    return sr / f ** 3, np.stack(U), T


def central_strain(U):
    """Resolved strain S_ab = (dU_a/dx_b + dU_b/dx_a)/2 of a coarse field
    U[3][Z][Y][X] by second-order central differences on the periodic grid."""
    # G[a][b] = dU_b/dx_a; axis of x_a in the (Z, Y, X) array is 2 - a
    G = np.empty((3, 3) + U.shape[1:])
    for a in range(3):
        ax = 2 - a
        for b in range(3):
            G[a, b] = 0.5 * (np.roll(U[b], -1, axis=ax) - np.roll(U[b], 1, axis=ax))
    return 0.5 * (G + G.transpose(1, 0, 2, 3, 4))


def eddy_viscosity_target(T, S):
    """Least-squares eddy viscosity of the deviatoric subgrid stress on the
    form -2 nu_t S, clipped at zero: nu_t = max(0, -dev(T):S / (2 S:S + 1e-30))."""
    trT = (T[0, 0] + T[1, 1] + T[2, 2]) / 3.0
    Td = T - np.eye(3)[:, :, None, None, None] * trT
    num = np.einsum("ab...,ab...->...", Td, S)
    ss = np.einsum("ab...,ab...->...", S, S)
    return np.maximum(0.0, -num / (2.0 * ss + 1e-30))


def closure_features(S, rbar, nut, nu_c):
    """Features of each coarse node (n x 7): the non-equilibrium momentum flux
    Pi = -2 rho c_s^2 tau_e S (first-order Chapman-Enskog, c_s^2 = 1/3) a
    coarse lattice relaxing with tau_e = 3 (nu_c + nu_t) + 1/2 carries, in the
    order xx, yy, zz, xy, xz, yz, then <rho>."""
    tau_e = 3.0 * (nu_c + nut) + 0.5
    c = -2.0 / 3.0 * rbar * tau_e
    return np.stack([c * S[0, 0], c * S[1, 1], c * S[2, 2], c * S[0, 1], c * S[0, 2], c * S[1, 2], rbar],
                    axis=-1).reshape(-1, 7)


def box_filter_targets(rho, u, factor, nu_c):
    """Training features (n_coarse x 7) and targets nu_t / nu_c from fine fields
    rho[nz,ny,nx], u[3,nz,ny,nx]; coarse order (Z, Y, X) with X fastest.
    The four steps above in order: filter, strain, target, features."""
    rbar, U, T = favre_filter(rho, u, factor)
    S = central_strain(U)
    nut = eddy_viscosity_target(T, S)
    feat = closure_features(S, rbar, nut, nu_c)
    return feat, (nut / nu_c).reshape(-1), {"T": T, "S": S, "U": U, "rho": rbar}


def bf16_array(a):
    return np.array([bf16(float(v)) for v in np.ravel(a)]).reshape(np.shape(a))
