"""Learned eddy-viscosity closure pipeline, driven through the C ABI.

1. Fine run: D3Q27 BGK+Smagorinsky (C_s = 0.1) Taylor-Green vortex at
   Re = 1600 (Sec. 3.1 workload shape) on n_f^3 nodes, FP32 storage, to
   20 convective times; k(t) sampled by the fused FP64 reductions.
2. Snapshots: `n_snap` states evenly spaced in time are box-filtered by
   `factor`^3 on the GPU (lbm_filter_snapshot) into closure features and
   eddy-viscosity targets.
3. Training: `n_samples` samples drawn without replacement from the pooled
   snapshots (seeded), z-score normalisation from the training set, He-normal
   initial weights (seeded), mini-batch Adam on the GPU (lbm_mlp_train).
4. Coarse runs on (n_f/factor)^3 nodes with the same Re (convective scaling)
   and three closures: none (BGK), Smagorinsky, learned MLP (BF16 MFMA inside
   the collision, Smagorinsky fallback).
5. Score: the dissipation rate eps(t) = -dk/dt (central differences of the
   FP64 k series) of each coarse run against the fine run at the same
   convective times, relative L2 over [0, 20 t_c]; cost as MLUPS.

Host code here only sequences calls, computes the normalisation constants and
differentiates the sampled k series (derived outputs); all lattice and network
arithmetic runs in the HIP library.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs, lbm


def tgv_setup(n, u0=0.05, Re=1600.0):
    nu = u0 * (n / (2 * math.pi)) / Re
    tc = n / (2 * math.pi * u0)
    return nu, 3 * nu + 0.5, tc


def dissipation(t, k):
    """eps = -dk/dt by central differences (one-sided at the ends)."""
    return -np.gradient(np.asarray(k), np.asarray(t))


def run_tgv(n, tag, steps, every, prec=lbm.LBM_F32, cs=0.1, mlp=None, snapshots=(), factor=4, stream=None,
            log=None):
    """Run a D3Q27 Taylor-Green lattice; returns (t_steps, k, snapshots, seconds)."""
    import torch
    nu, tau, tc = tgv_setup(n)
    rho, u = inputs.tgv3d_fields(n, 0.05)
    L = lbm.Lattice(inputs.all_fluid(n, n, n, tag), q=27, prec=prec, tau=tau, smag_cs=cs, stream=stream)
    if mlp is not None:
        L.set_mlp(mlp)
    L.init_equilibrium(rho, u)
    del rho, u
    snaps = []
    ts, ks = [], []
    marks = sorted(set(int(s) for s in snapshots))
    t = 0
    elapsed = 0.0
    stop_points = sorted(set(marks + [steps]))
    unstable = False
    for sp in stop_points:
        n_run = sp - t
        if n_run > 0:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                ser = L.step_reduce(n_run, every)
            except lbm.LbmError as e:
                if e.status != lbm.LBM_EUNSTABLE:
                    raise
                unstable = True
                break
            elapsed += time.perf_counter() - t0
            for m in ser:
                if not ts or m["step"] > ts[-1]:
                    ts.append(m["step"])
                    ks.append(m["kinetic_energy"])
            t = sp
            if log is not None:
                log(f"{n}^3 tag {tag}: step {t}/{steps}, {elapsed:.1f} s")
        if sp in marks:
            nc = (n // factor) ** 3
            feat = torch.empty((nc, 7), dtype=torch.float32, device="cuda")
            tgt = torch.empty(nc, dtype=torch.float32, device="cuda")
            L.filter_snapshot(factor, feat, tgt)
            snaps.append((feat, tgt))
    L.close()
    return np.array(ts), np.array(ks), snaps, elapsed, unstable


def train_closure(snaps, n_samples=1_000_000, epochs=30, batch=4096, lr=1e-3, seed=1234):
    import torch
    feat = torch.cat([s[0] for s in snaps])
    tgt = torch.cat([s[1] for s in snaps])
    pool = feat.shape[0]
    n = min(n_samples, pool)
    pick = torch.as_tensor(inputs.sample_without_replacement(pool, n, seed), device="cuda")
    X = feat[pick].contiguous()
    Y = tgt[pick].contiguous()
    Xh = X.cpu().numpy().astype(np.float64)
    P = inputs.mlp_he_init(seed)
    P[1345:1352] = Xh.mean(0)
    P[1352:1359] = np.maximum(Xh.std(0), 1e-12)
    perm = np.concatenate([inputs.permutation_by_keys(n, seed + 1 + e) for e in range(epochs)])
    Pd = torch.tensor(P, device="cuda")
    log = torch.empty(max(epochs, 1), device="cuda")
    t0 = time.perf_counter()
    lbm.lbm_mlp_train(Pd, X, Y, torch.as_tensor(perm, device="cuda"), batch, epochs, lr, log)
    torch.cuda.synchronize()
    return Pd.cpu().numpy(), log.cpu().numpy(), time.perf_counter() - t0, {"pool": pool, "samples": n}


def experiment(n_fine=512, factor=4, n_snap=16, n_samples=1_000_000, epochs=30, t_end_tc=20.0, every_fine=100,
               log=print):
    """Full pipeline; returns a result dictionary."""
    nu_f, tau_f, tc_f = tgv_setup(n_fine)
    steps_f = int(round(t_end_tc * tc_f))
    snap_at = [int(round(s)) for s in np.linspace(0, steps_f, n_snap)]
    log(f"fine run {n_fine}^3, {steps_f} steps, snapshots at {snap_at[:3]}...")
    t_f, k_f, snaps, sec_f, bad_f = run_tgv(n_fine, inputs.TAG_SMAG, steps_f, every_fine, snapshots=snap_at,
                                           factor=factor, log=log)
    P, loss_log, sec_train, info = train_closure(snaps, n_samples=n_samples, epochs=epochs)
    del snaps
    log(f"trained on {info['samples']} of {info['pool']} samples, loss {loss_log[0]:.4g} -> {loss_log[-1]:.4g}")
    n_c = n_fine // factor
    nu_c, tau_c, tc_c = tgv_setup(n_c)
    steps_c = int(round(t_end_tc * tc_c))
    every_c = max(1, every_fine // factor)
    eps_f = dissipation(t_f / tc_f, k_f)
    res = {"fine": {"n": n_fine, "steps": steps_f, "tau": tau_f, "seconds": sec_f, "unstable": bad_f,
                    "MLUPS": n_fine ** 3 * steps_f / max(sec_f, 1e-9) / 1e6},
           "training": {"loss_first": float(loss_log[0]), "loss_last": float(loss_log[-1]), "seconds": sec_train,
                        **info},
           "coarse": {}}
    for name, tag, mlp in (("bgk", inputs.TAG_BGK, None), ("smagorinsky", inputs.TAG_SMAG, None),
                           ("mlp", inputs.TAG_MLP, P)):
        t_c, k_c, _, sec, bad = run_tgv(n_c, tag, steps_c, every_c, mlp=mlp)
        entry = {"seconds": sec, "MLUPS": n_c ** 3 * steps_c / max(sec, 1e-9) / 1e6, "unstable": bad}
        if len(t_c) > 2:
            tt = t_c / tc_c
            eps_c = dissipation(tt, k_c)
            ef = np.interp(tt, t_f / tc_f, eps_f)
            entry["eps_rel_l2"] = float(np.linalg.norm(eps_c - ef) / np.linalg.norm(ef))
            entry["k_rel_l2"] = float(np.linalg.norm(k_c - np.interp(tt, t_f / tc_f, k_f)) / np.linalg.norm(k_f))
            entry["eps_peak_t"] = float(tt[int(np.argmax(eps_c))])
        res["coarse"][name] = entry
        log(f"coarse {name}: {entry}")
    res["fine"]["eps_peak_t"] = float((t_f / tc_f)[int(np.argmax(eps_f))])
    return res, P
