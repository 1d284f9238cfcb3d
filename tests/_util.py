"""Shared helpers of the GPU tests: run the HIP path and the oracle on the same
seeded inputs and compare what is unique (fluid-node populations)."""
import numpy as np

import oracle
from paper_2506_09242_amd import lbm

FLUID = (1, 2, 3, 4, 5, 6, 7, 8, 9, 10)


def fluid_mask(tags):
    return np.isin(tags, FLUID)


def make_pair(tags, q=19, prec=lbm.LBM_F64, rho=None, u=None, mlp=None, layout=None, **kw):
    """Oracle and HIP lattices with the same configuration and initial state
    (layout: the HIP lattice's storage layout, None for its default)."""
    nz, ny, nx = tags.shape
    o = oracle.Oracle(nx, ny, nz, q=q, tags=tags, mlp=mlp, **kw)
    o.init_equilibrium(rho, u)
    L = lbm.Lattice(tags, q=q, prec=prec, layout=layout, **kw)
    if mlp is not None:
        L.set_mlp(mlp)
    L.init_equilibrium(rho, u)
    return o, L


def max_rel_pop_error(f_gpu, f_orc, tags):
    m = fluid_mask(tags)
    a = f_gpu[:, m]
    b = f_orc[:, m]
    return float(np.max(np.abs(a - b) / np.abs(b)))


def max_abs_pop_error(f_gpu, f_orc, tags):
    m = fluid_mask(tags)
    return float(np.max(np.abs(f_gpu[:, m] - f_orc[:, m])))


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def momentum_bound(f_gpu, f_orc, tags, q):
    """Largest difference two domain momentum sums can show when their node
    populations differ by f_gpu - f_orc: |dP_a| <= sum over fluid nodes and i of
    |c_ia| |df_i| (triangle inequality), plus the rounding of two sums of the
    same terms (64 unit roundoffs of sum |c_ia| f_i).  Per axis a."""
    m = fluid_mask(tags)
    c = np.array([lbm.lbm_velocity(q, i)[0] for i in range(q)], dtype=np.float64)  # [q][3]
    d = np.abs(f_gpu[:, m] - f_orc[:, m]).sum(axis=1)      # [q]
    s = np.abs(f_orc[:, m]).sum(axis=1)                    # [q]
    return np.abs(c).T @ d + 64 * 2.0 ** -53 * (np.abs(c).T @ s)


def kinetic_energy_bound(u_gpu, u_orc, tags):
    """Largest difference two sums K = sum 1/2 |u|^2 over fluid nodes can show when
    the node velocities differ by u_gpu - u_orc: per node
    |1/2 |a|^2 - 1/2 |b|^2| = 1/2 |(a - b) . (a + b)| <= 1/2 |a - b| |a + b|
    (Cauchy-Schwarz), summed, plus the rounding of two sums of the same terms
    (64 unit roundoffs of K).  K is quadratic in u, so its relative difference
    is about twice that of the velocity field."""
    m = fluid_mask(tags)
    a, b = u_gpu[:, m], u_orc[:, m]
    per_node = 0.5 * np.linalg.norm(a - b, axis=0) * np.linalg.norm(a + b, axis=0)
    return float(per_node.sum() + 64 * 2.0 ** -53 * 0.5 * (b * b).sum())
