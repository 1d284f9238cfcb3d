"""Benchmark of the fused collide-and-stream hot path on one MI355X.

Default workload: the D3Q27 BGK + Smagorinsky (C_s = 0.1) Taylor-Green vortex
(Sec. 3.1, Eqs. (1)-(4)) on 512^3 nodes, u0 = 0.05, Re = 1600 on the
reference length N / 2 pi, stored as FP32 shifted populations (the reported
value), with FP16 storage and FP64 alongside.  One "step" is one fused
collide+stream update of the whole lattice (even and odd AA steps alternate)
with the FP64 domain reductions sampled every 100 steps (fused into the step).
Inputs are resident in HBM before timing starts.  Each timed run is repeated
three times back to back and the median is reported.  Kinetic-energy and
dissipation errors against the FP64 run are reported, and the 256^3 D3Q19
lid-driven cavity (Sec. 3.2 shape) is measured the same way as an extra block.

Other modes: --workload picks another workload as the headline; --ceiling
measures the HBM ceilings (plain copy / read / write probes and the step's
own access pattern with the collision switched off); --slab times one GPU's
share of a z-slab decomposition and its face pack / unpack kernels.

Prints ONE JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
METRIC = "MLUPS and % of HBM roofline per dtype at 1 GPU; energy error vs FP64"

WORKLOADS = {
    # name: (builder, q, description)
    "cavity256_d3q19_bgk": "D3Q19 BGK lid-driven cavity 256^3, lid u=0.1, Re=1000",
    "cavity256_d3q19_reg": "D3Q19 regularized-BGK lid-driven cavity 256^3, lid u=0.1, Re=1000",
    "cavity400_d3q19_rr": "D3Q19 recursive-regularized lid-driven cavity 400^3, lid u=0.1, Re=10000",
    "tgv512_d3q27_smag": "D3Q27 BGK+Smagorinsky(Cs=0.1) Taylor-Green 512^3, u0=0.05, Re=1600",
    "porous400_d3q19_trt": "D3Q19 TRT(3/16) body-force porous 400^3, phi=0.20, corr. length 8",
    "tgv32_d3q19_bgk": "D3Q19 BGK Taylor-Green 32^3, u0=0.04, Re=100 (cache-resident)",
    "porous480_open_d3q19_trt": "D3Q19 TRT(3/16) porous 400^3 rock between 40-plane buffers, regularized "
                                "pressure inlet / pressure outlet (480x400x400)",
    "closure_tgv128_d3q27": "learned closure: D3Q27 TGV Re=1600, fine 512^3 -> coarse 128^3, MLP vs Smagorinsky vs BGK",
}
DEFAULT_WORKLOAD = "tgv512_d3q27_smag"
EXTRA_WORKLOAD = "cavity256_d3q19_bgk"
FLUID_TAGS = (1, 2, 3, 4, 5, 6, 7, 8, 9, 10)


def source_hash():
    """Hash of the kernel sources (to tell whether stored counters still apply)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_09242_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def build_workload(name):
    from paper_2506_09242_amd import inputs
    if name == "cavity256_d3q19_bgk":
        n = 256
        L = n - 2
        nu = 0.1 * L / 1000.0
        tags = inputs.cavity_tags(n)
        kw = dict(q=19, tau=3 * nu + 0.5, wall_velocity=[(0.1, 0.0, 0.0)])
        return tags, kw, None, None, {"cells": n ** 3, "lid_u": 0.1, "Re": 1000, "cavity_length": L}
    if name == "cavity256_d3q19_reg":
        n = 256
        L = n - 2
        nu = 0.1 * L / 1000.0
        tags = inputs.cavity_tags(n, fluid_tag=inputs.TAG_REG)
        kw = dict(q=19, tau=3 * nu + 0.5, wall_velocity=[(0.1, 0.0, 0.0)])
        return tags, kw, None, None, {"cells": n ** 3, "lid_u": 0.1, "Re": 1000, "cavity_length": L}
    if name == "cavity400_d3q19_rr":
        # the paper's turbulent cavity (Sec. 3.2): Re = 10000 on L = 400 with the
        # recursive regularized model and bulk relaxation 1
        n = 400
        L = n - 2
        nu = 0.1 * L / 10000.0
        tags = inputs.cavity_tags(n, fluid_tag=inputs.TAG_RR)
        kw = dict(q=19, tau=3 * nu + 0.5, wall_velocity=[(0.1, 0.0, 0.0)])
        return tags, kw, None, None, {"cells": n ** 3, "lid_u": 0.1, "Re": 10000, "cavity_length": L}
    if name == "tgv512_d3q27_smag":
        n, u0, Re = 512, 0.05, 1600.0
        nu = u0 * (n / (2 * np.pi)) / Re
        rho, u = inputs.tgv3d_fields(n, u0)
        tags = inputs.all_fluid(n, n, n, inputs.TAG_SMAG)
        kw = dict(q=27, tau=3 * nu + 0.5, smag_cs=0.1)
        return tags, kw, rho, u, {"cells": n ** 3, "u0": u0, "Re": Re}
    if name == "porous400_d3q19_trt":
        n = 400
        tags = inputs.porous_tags(n, porosity=0.20, ell=8.0, seed=42)
        kw = dict(q=19, tau=1.0, trt_lambda=3.0 / 16.0, force=(1e-5, 0.0, 0.0))
        return tags, kw, None, None, {"cells": n ** 3, "porosity": 0.2, "seed": 42}
    if name == "porous480_open_d3q19_trt":
        # the paper's Berea layout (Sec. 3.3): 40 fluid planes upstream, the
        # 400^3 rock, 40 downstream; regularized pressure boundaries at x = 0
        # (rho 1.006) and x = nx-1 (rho 1); periodic in y and z
        n, buf = 400, 40
        tags = np.full((n, n, n + 2 * buf), inputs.TAG_TRT, dtype=np.uint8)
        tags[:, :, buf:buf + n] = inputs.porous_tags(n, porosity=0.20, ell=8.0, seed=42)
        tags[:, :, 0] = inputs.TAG_PIN
        tags[:, :, -1] = inputs.TAG_POUT
        kw = dict(q=19, tau=1.0, trt_lambda=3.0 / 16.0, bc_density=(1.006, 1.0))
        return tags, kw, None, None, {"cells": tags.size, "porosity": 0.2, "seed": 42, "buffer": buf,
                                      "rock": n, "rho_in": 1.006, "rho_out": 1.0}
    if name == "tgv32_d3q19_bgk":
        n, u0 = 32, 0.04
        rho, u = inputs.tgv3d_fields(n, u0)
        tags = inputs.all_fluid(n, n, n)
        kw = dict(q=19, tau=3 * u0 * n / 100.0 + 0.5)
        return tags, kw, rho, u, {"cells": n ** 3, "u0": u0, "Re": 100}
    raise SystemExit(f"unknown workload {name}")


def alg_bytes_per_launch(tags, q, prec_bytes, tagged=True):
    """Algorithmic HBM bytes of one collide-stream launch: every fluid node reads
    and writes its Q populations once; on a tagged lattice every node's tag byte
    is read once (a lattice of one fluid model without walls reads no tags)."""
    fluid = int(np.isin(tags, FLUID_TAGS).sum())
    return fluid * 2 * q * prec_bytes + (tags.size if tagged else 0), fluid


def run_dtype(tags, kw, rho, u, prec, steps, warmup, every, repeats=1, chunk=2000, label="", keep_rho=False,
              sample=None, parity_launches=0):
    """Time `steps` steps (reductions every `every`, fused) after `warmup`, `repeats`
    times back to back on the same lattice.  Long runs go in chunks of about
    `chunk` steps (a multiple of `every`) with one progress line each; the events
    bracket all chunks of one repeat.  The series and the final fields are those
    of the first repeat (state after warmup + steps); the series always ends with
    the final state (sampled by a standalone reduction after the timed region if
    the step count is not a multiple of `every`).  `sample(L)`, if given, is
    called on the first repeat after every chunk (and at the start); each chunk
    is then timed by its own events so that the sampling stays out of the time.
    `parity_launches` > 0: afterwards, time that many even and odd launches one
    by one (events around each) for the per-parity launch durations."""
    import torch
    from paper_2506_09242_amd import lbm
    stream = torch.cuda.current_stream()
    L = lbm.Lattice(tags, prec=prec, stream=stream, **kw)
    L.init_equilibrium(rho, u)
    if warmup:
        L.step(warmup)
    chunk = max(every, chunk // every * every)
    runs, first = [], None
    for rep in range(repeats):
        L.synchronize()
        torch.cuda.synchronize()
        sampling = sample is not None and rep == 0
        samples = [(L.time, sample(L))] if sampling else []
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        series, done, chunk_ms = [], 0, 0.0
        while done < steps:
            n = min(chunk, steps - done)
            if sampling:
                c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                c0.record(stream)
            part = L.step_reduce(n, every)  # synchronizes at its end
            if sampling:
                c1.record(stream)
                torch.cuda.synchronize()
                chunk_ms += c0.elapsed_time(c1)
                samples.append((L.time, sample(L)))
            series.extend(part if not series else part[1:])
            done += n
            if steps > chunk:
                print(f"# {label}: {done}/{steps} steps, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                      flush=True)
        e1.record(stream)
        torch.cuda.synchronize()
        runs.append(chunk_ms if sampling else e0.elapsed_time(e1))
        if rep == 0:
            if series[-1]["step"] != L.time:
                series.append(L.reduce())
            rf, uf = L.read_fields()
            first = {"wall_s": time.perf_counter() - t0, "series": series, "u": uf, "samples": samples}
            if keep_rho:
                first["rho"] = rf
    per_parity = None
    if parity_launches:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * parity_launches + 1)]
        L.synchronize()
        if L.time % 2:
            L.step(1)
        ev[0].record(stream)
        for k in range(2 * parity_launches):
            L.step(1)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        d = [ev[k].elapsed_time(ev[k + 1]) for k in range(2 * parity_launches)]
        per_parity = {"even_ms": float(np.mean(d[0::2])), "odd_ms": float(np.mean(d[1::2])),
                      "launches_each": parity_launches}
    variant = L.variant
    L.close()
    return dict(first, ms=float(np.median(runs)), runs_ms=runs, variant=variant, per_parity=per_parity)


def measure(tags, kw, rho, u, prec_names, args, label_prefix="", sample=None, keep_rho=False, steps=None):
    """Timed runs of every dtype in prec_names; returns per-dtype results."""
    from paper_2506_09242_amd import lbm
    steps = args.steps if steps is None else steps
    results = {}
    for pn in prec_names:
        prec = lbm.PREC_NAMES[pn]
        r = run_dtype(tags, kw, rho, u, prec, steps, args.warmup, args.every, args.repeats,
                      label=label_prefix + pn, keep_rho=keep_rho, sample=sample, parity_launches=10)
        nbytes, nfluid = alg_bytes_per_launch(tags, kw["q"], lbm.PREC_BYTES[prec], "/uniform" not in r["variant"])
        launch_s = r["ms"] * 1e-3 / steps
        achieved = nbytes / launch_s / 1e9
        res = {"MLUPS": tags.size * steps / (r["ms"] * 1e-3) / 1e6,
               "MFLUPS_fluid": nfluid * steps / (r["ms"] * 1e-3) / 1e6,
               "ms_per_step": r["ms"] / steps,
               "alg_GBps": achieved, "hbm_frac": achieved / HBM_PEAK_GBS,
               "bytes_per_launch": nbytes, "variant": r["variant"],
               "runs_ms_per_step": [round(v / steps, 5) for v in r["runs_ms"]],
               "k_final": r["series"][-1]["kinetic_energy"], "series": r["series"], "u": r["u"],
               "rho": r.get("rho"), "samples": r.get("samples"), "wall_s": r["wall_s"]}
        if r["per_parity"]:
            pp = r["per_parity"]
            res["even_ms"], res["odd_ms"] = round(pp["even_ms"], 5), round(pp["odd_ms"], 5)
            res["even_hbm_frac"] = round(nbytes / (pp["even_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            res["odd_hbm_frac"] = round(nbytes / (pp["odd_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        results[pn] = res
        print(f"# {label_prefix}{pn}: {res['MLUPS']:.1f} MLUPS, {achieved:.1f} GB/s algorithmic "
              f"({100 * achieved / HBM_PEAK_GBS:.1f}% of 8 TB/s; even {res.get('even_hbm_frac', 0) * 100:.1f}%, "
              f"odd {res.get('odd_hbm_frac', 0) * 100:.1f}%), {r['variant']}", file=sys.stderr, flush=True)
    return results


def errors_vs_fp64(results):
    """Errors of the reduced-precision runs against the FP64 run of the same
    workload, over the timed steps: final kinetic energy, the k series, the
    dissipation series eps = -dk/dt (central differences) and the final
    velocity field."""
    errors = {}
    if "f64" not in results:
        return errors
    ref = results["f64"]
    k_ref = np.array([m["kinetic_energy"] for m in ref["series"]])
    t_ref = np.array([m["step"] for m in ref["series"]], dtype=np.float64)
    eps_ref = -np.gradient(k_ref, t_ref) if len(t_ref) > 2 else None
    for pn, r in results.items():
        if pn == "f64":
            continue
        k = np.array([m["kinetic_energy"] for m in r["series"]])
        du = r["u"] - ref["u"]
        errors[pn] = {"steps_compared": int(t_ref[-1]),
                      "k_rel_err_final": float(abs(k[-1] / k_ref[-1] - 1.0)),
                      "k_rel_l2_series": float(np.linalg.norm(k - k_ref) / np.linalg.norm(k_ref)),
                      "u_rel_l2": float(np.linalg.norm(du) / np.linalg.norm(ref["u"])),
                      "u_max_abs": float(np.abs(du).max())}
        if eps_ref is not None:
            eps = -np.gradient(k, t_ref)
            errors[pn]["eps_rel_l2_series"] = float(np.linalg.norm(eps - eps_ref) / np.linalg.norm(eps_ref))
    return errors


def slim(results):
    keep = ("MLUPS", "MFLUPS_fluid", "ms_per_step", "alg_GBps", "hbm_frac", "variant", "runs_ms_per_step",
            "even_ms", "odd_ms", "even_hbm_frac", "odd_hbm_frac")
    return {pn: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items() if k in keep}
            for pn, r in results.items()}


def cpu_baseline(name, tags, kw, rho, u, steps):
    """The FP64 oracle (two-population push, all host threads) on `steps` steps
    of the workload; the 512^3 Taylor-Green lattice (58 GB in two-population
    FP64) is replaced by the same flow on 256^3 nodes, reported per node."""
    import oracle
    from paper_2506_09242_amd import inputs
    desc = f"the full {name} lattice"
    if name == "tgv512_d3q27_smag":
        n, u0, Re = 256, 0.05, 1600.0
        rho, u = inputs.tgv3d_fields(n, u0)
        tags = inputs.all_fluid(n, n, n, inputs.TAG_SMAG)
        kw = dict(kw, tau=3 * u0 * (n / (2 * np.pi)) / Re + 0.5)
        desc = "the same D3Q27 BGK+Smagorinsky Taylor-Green flow on 256^3 nodes (the 512^3 lattice needs 58 GB " \
               "as two FP64 population arrays), MLUPS per node"
    nz, ny, nx = tags.shape
    okw = {k: v for k, v in kw.items() if k in ("tau", "trt_lambda", "smag_cs", "force", "wall_velocity")}
    o = oracle.Oracle(nx, ny, nz, q=kw["q"], tags=tags, **okw)
    o.init_equilibrium(rho, u)
    o.run(1)  # warm-up (first touch of both arrays)
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    o.run(steps)
    dt = time.perf_counter() - t0
    # the same oracle on one thread, one step
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    o.run(1)
    dt1 = time.perf_counter() - t1
    oracle.set_num_threads(cores)
    return {"value": tags.size * steps / dt / 1e6, "unit": "MLUPS", "cores": cores,
            "kind": "oracle", "sample": f"{steps} FP64 two-population steps of {desc} ({tags.size} cells), "
                                        f"after 1 warm-up step",
            "value_single_thread": tags.size / dt1 / 1e6,
            "sample_single_thread": "1 step of the same lattice on one thread"}


def stored_traffic(workload, prec_name):
    """HBM bytes per collide-stream launch from committed rocprofv3 counter runs,
    valid only if the kernel sources are unchanged since they were taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec_name}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch")


def derived_outputs(name, tags, kw, wl_cfg, results, args):
    """Host-side derived quantities of the FP64 reductions (permeability,
    dissipation and enstrophy series)."""
    derived = {}
    if name == "porous400_d3q19_trt":
        # permeability of the porous case (mean over all nodes, solids counted as
        # zero velocity), lattice units and millidarcy at the Berea voxel 5.345 um
        nu = (kw["tau"] - 0.5) / 3.0
        F = kw["force"][0]
        for pn, r in results.items():
            ux_mean = r["series"][-1]["velocity_sum"][0] / tags.size
            k_lu = nu * ux_mean / F
            derived[pn] = {"permeability_lu": k_lu, "permeability_mD": k_lu * (5.345e-6) ** 2 / 9.869233e-16,
                           "porosity": float(np.isin(tags, FLUID_TAGS).mean()),
                           "steps_total": args.warmup + args.steps,
                           "k_series_lu": [nu * m["velocity_sum"][0] / tags.size / F for m in r["series"][::20]]}
        from paper_2506_09242_amd import inputs as _inp
        derived["percolates_x"] = bool(_inp.percolates_x(tags))
    if name == "porous480_open_d3q19_trt":
        # Darcy permeability from the pressure drop across the rock (Eq. 6):
        # k = u_mean nu L / dP, u_mean over every rock node (solids 0), dP = cs^2
        # (mean fluid density of the plane before the rock - of the plane after it)
        nu = (kw["tau"] - 0.5) / 3.0
        buf, n = wl_cfg["buffer"], wl_cfg["rock"]
        fl = np.isin(tags, FLUID_TAGS)
        for pn, r in results.items():
            ux = r["u"][0]
            u_mean = float(ux[:, :, buf:buf + n].mean())
            rho_f = r["rho"]
            r_up = float(rho_f[:, :, buf - 1][fl[:, :, buf - 1]].mean())
            r_dn = float(rho_f[:, :, buf + n][fl[:, :, buf + n]].mean())
            dP = (r_up - r_dn) / 3.0
            k_lu = u_mean * nu * n / dP
            derived[pn] = {"permeability_lu": k_lu, "permeability_mD": k_lu * (5.345e-6) ** 2 / 9.869233e-16,
                           "u_mean_rock": u_mean, "rho_upstream": r_up, "rho_downstream": r_dn,
                           "steps_total": args.warmup + args.steps}
            del r["rho"]
    if name.startswith("tgv"):
        # convective time t_c = N / (2 pi u0); dissipation eps = -dk/dt by central
        # differences of the FP64 k series; eps* = eps t_c / u0^2
        n, u0 = tags.shape[0], wl_cfg["u0"]
        tc = n / (2 * np.pi * u0)
        for pn, r in results.items():
            t = np.array([m_["step"] for m_ in r["series"]], dtype=np.float64)
            k = np.array([m_["kinetic_energy"] for m_ in r["series"]])
            if len(t) < 3:
                continue
            eps = -np.gradient(k, t) * tc / u0 ** 2
            j = int(np.argmax(eps))
            stride = max(1, int(round(0.5 * tc / max(t[1] - t[0], 1.0))))
            derived[pn] = {"t_c_steps": tc, "eps_peak_tc": float(t[j] / tc), "eps_peak_nondim": float(eps[j]),
                           "k_final_over_k0": float(k[-1] / k[0]),
                           "t_over_tc": [round(float(v / tc), 3) for v in t[::stride]],
                           "eps_nondim": [float(v) for v in eps[::stride]]}
            if r.get("samples"):
                # enstrophy (1/N) sum |curl u|^2 / 2 in units of u0^2 / L_ref^2, L_ref = N / (2 pi);
                # with the viscous dissipation 2 nu Omega beside eps (the rest is the subgrid model's)
                nu = (kw["tau"] - 0.5) / 3.0
                ts = np.array([a for a, _ in r["samples"]], dtype=np.float64)
                om = np.array([b for _, b in r["samples"]])
                lref = n / (2 * np.pi)
                jj = int(np.argmax(om))
                derived[pn]["enstrophy_t_over_tc"] = [round(float(v / tc), 3) for v in ts]
                derived[pn]["enstrophy_nondim"] = [float(v * lref ** 2 / u0 ** 2) for v in om]
                derived[pn]["enstrophy_peak_tc"] = float(ts[jj] / tc)
                derived[pn]["viscous_eps_nondim"] = [float(2 * nu * v * tc / u0 ** 2) for v in om]
    return derived


def time_stream(stream, fn, reps):
    """Average duration (ms) of fn() over reps calls, HIP events on `stream`."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def ceiling_mode(args):
    """HBM ceilings: the plain copy / read / write probes (4, 8 and 16 bytes per
    lane, 4 GiB buffers) and the step's own access pattern with the collision
    switched off (LBM_FLAG_FREE_STREAM) on the headline and cavity shapes, as
    fractions of 8 TB/s; the runtime's own device copy for comparison."""
    import torch
    from paper_2506_09242_amd import inputs, lbm
    stream = torch.cuda.current_stream()
    nbytes = 4 << 30
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    out = {"probe_bytes": nbytes, "probes": {}}
    for kind, kname, moved in ((0, "copy", 2), (1, "read", 1), (2, "write", 1)):
        for lane in (4, 8, 16):
            ms = time_stream(stream, lambda: lbm.lbm_probe_bandwidth(kind, b, a, nbytes, lane, stream), 10)
            gbs = moved * nbytes / (ms * 1e-3) / 1e9
            out["probes"][f"{kname}_{lane}B"] = {"GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
            print(f"# probe {kname} {lane} B/lane: {gbs:.0f} GB/s", file=sys.stderr, flush=True)
    ms = time_stream(stream, lambda: b.copy_(a), 10)
    out["torch_copy_GBps"] = round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    out["free_stream"] = {}
    for wname in (DEFAULT_WORKLOAD, EXTRA_WORKLOAD):
        tags, kw, _, _, _ = build_workload(wname)
        for pn in args.dtypes.split(","):
            prec = lbm.PREC_NAMES[pn]
            L = lbm.Lattice(tags, prec=prec, stream=stream, free_stream=True, **kw)
            L.init_equilibrium()
            L.step(4)
            nb, _ = alg_bytes_per_launch(tags, kw["q"], lbm.PREC_BYTES[prec], "/uniform" not in L.variant)
            even = time_stream(stream, lambda: L.step(2), 10)  # an even + odd pair
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(21)]
            ev[0].record(stream)
            for k in range(20):
                L.step(1)
                ev[k + 1].record(stream)
            torch.cuda.synchronize()
            d = [ev[k].elapsed_time(ev[k + 1]) for k in range(20)]
            e_ms, o_ms = float(np.mean(d[0::2])), float(np.mean(d[1::2]))
            out["free_stream"][f"{wname}_{pn}"] = {
                "variant": L.variant, "even_ms": round(e_ms, 5), "odd_ms": round(o_ms, 5),
                "even_frac": round(nb / (e_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "odd_frac": round(nb / (o_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "pair_frac": round(2 * nb / (even * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            print(f"# free stream {wname} {pn}: {out['free_stream'][f'{wname}_{pn}']}", file=sys.stderr, flush=True)
            L.close()
    print(json.dumps({"mode": "ceiling", **out}), flush=True)


def slab_mode(args):
    """One GPU's share of a z-slab decomposition of the headline lattice
    (512 x 512 x 64 of the 512^3 D3Q27 Taylor-Green, 8 slabs): launch durations
    of the even and odd steps and of the face pack / unpack kernels that carry
    the crossing populations (9 per node for D3Q27) before and after each odd
    step; the faces' bandwidth counts their bytes read plus written."""
    import torch
    from paper_2506_09242_amd import inputs, lbm
    stream = torch.cuda.current_stream()
    n, h, u0, Re = 512, 64, 0.05, 1600.0
    tags_full, kw, rho, u, _ = build_workload(DEFAULT_WORKLOAD)
    rho, u = rho[:h].copy(), u[:, :h].copy()
    tags = inputs.all_fluid(n, n, h, inputs.TAG_SMAG)
    out = {"slab": [n, n, h], "dtypes": {}}
    for pn in args.dtypes.split(","):
        prec = lbm.PREC_NAMES[pn]
        L = lbm.Lattice(tags, prec=prec, stream=stream, **kw)
        L.init_equilibrium(rho, u)
        L.step(4)
        m = lbm.lbm_face_populations(kw["q"])
        s = lbm.PREC_BYTES[prec]
        dt = {1: torch.float32, 0: torch.float64, 2: torch.float16}[prec]
        bufs = [torch.empty(m * n * n, dtype=dt, device="cuda") for _ in range(2)]
        nb, _ = alg_bytes_per_launch(tags, kw["q"], s, "/uniform" not in L.variant)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(21)]
        ev[0].record(stream)
        for k in range(20):
            L.step(1)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        d = [ev[k].elapsed_time(ev[k + 1]) for k in range(20)]
        e_ms, o_ms = float(np.mean(d[0::2])), float(np.mean(d[1::2]))
        pack = time_stream(stream, lambda: (L.face_pack(0, bufs[0]), L.face_pack(1, bufs[1])), 20) / 2
        unpack = time_stream(stream, lambda: (L.face_unpack(0, bufs[0]), L.face_unpack(1, bufs[1])), 20) / 2
        face_bytes = 2 * m * n * n * s
        out["dtypes"][pn] = {"variant": L.variant, "even_ms": round(e_ms, 5), "odd_ms": round(o_ms, 5),
                             "even_frac": round(nb / (e_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "odd_frac": round(nb / (o_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "face_bytes_each": face_bytes // 2,
                             "pack_ms": round(pack, 5), "unpack_ms": round(unpack, 5),
                             "pack_GBps": round(face_bytes / (pack * 1e-3) / 1e9, 1),
                             "unpack_GBps": round(face_bytes / (unpack * 1e-3) / 1e9, 1),
                             "exchange_share_of_odd_step": round(4 * (pack + unpack) / o_ms, 4)}
        print(f"# slab {pn}: {out['dtypes'][pn]}", file=sys.stderr, flush=True)
        L.close()
    print(json.dumps({"mode": "slab", **out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--every", type=int, default=100, help="reduction sampling period (steps)")
    ap.add_argument("--repeats", type=int, default=3, help="timed runs per dtype; the median is reported")
    ap.add_argument("--enstrophy", action="store_true",
                    help="sample the enstrophy (Eq. 5 vorticity) after every chunk of the first run")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--dtypes", default="f32,f16s,f64", help="first one is the reported value")
    ap.add_argument("--layout", choices=["rows", "bricks"], default=None,
                    help="force the storage layout of the headline workload (default: the library's choice)")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra cavity block")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--closure-fine", type=int, default=512)
    ap.add_argument("--closure-samples", type=int, default=1_000_000)
    ap.add_argument("--closure-epochs", type=int, default=30)
    ap.add_argument("--ceiling", action="store_true", help="measure the HBM ceilings instead")
    ap.add_argument("--slab", action="store_true", help="time one GPU's slab share and its face kernels instead")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the slab decomposition is measured on one GPU's share: --slab).", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_calibration:
        from paper_2506_09242_amd import lbm
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        stream = torch.cuda.current_stream()
        ms = time_stream(stream, lambda: lbm.lbm_probe_bandwidth(0, b, a, 1 << 30, 16, stream), 20)
        gbs = 2 * (1 << 30) / (ms * 1e-3) / 1e9
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "copy_GBps": gbs,
                          "kernel": "k_probe (16 B per lane)"}))
        return
    if args.ceiling:
        ceiling_mode(args)
        return
    if args.slab:
        slab_mode(args)
        return

    if args.workload == "closure_tgv128_d3q27":
        from paper_2506_09242_amd import closure
        log = lambda m: print("# " + m, file=sys.stderr, flush=True)
        res, _ = closure.experiment(n_fine=args.closure_fine, factor=4, n_snap=16,
                                    n_samples=args.closure_samples, epochs=args.closure_epochs, log=log)
        mlp = res["coarse"]["mlp"]
        print(json.dumps({"metric": METRIC, "value": round(mlp["MLUPS"], 2), "unit": "MLUPS", "n_gpus": 1,
                          "steps": None, "warmup": 0, "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": args.workload, "n_fine": args.closure_fine,
                                     "n_coarse": args.closure_fine // 4, "samples": args.closure_samples,
                                     "epochs": args.closure_epochs},
                          "closure": res}), flush=True)
        return

    t_start = time.perf_counter()
    tags, kw, rho, u, wl_cfg = build_workload(args.workload)
    if args.layout:
        kw = dict(kw, layout=args.layout)
    print(f"# {args.workload}: inputs built in {time.perf_counter() - t_start:.1f} s", file=sys.stderr, flush=True)
    prec_names = [p.strip() for p in args.dtypes.split(",") if p.strip()]
    sample = (lambda L: L.enstrophy()) if args.enstrophy else None
    results = measure(tags, kw, rho, u, prec_names, args, sample=sample,
                      keep_rho=args.workload == "porous480_open_d3q19_trt")
    errors = errors_vs_fp64(results)
    derived = derived_outputs(args.workload, tags, kw, wl_cfg, results, args)

    main_p = prec_names[0]
    m = results[main_p]
    traffic = stored_traffic(args.workload, main_p)
    roofline = {"bound": "hbm", "achieved": round(m["alg_GBps"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(m["alg_GBps"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_collide_stream (even/odd AA steps, averaged over the timed region)",
                "alg_bytes_per_launch": m["bytes_per_launch"],
                "even_frac": m.get("even_hbm_frac"), "odd_frac": m.get("odd_hbm_frac")}

    extra = {}
    if not args.no_extra and args.workload != EXTRA_WORKLOAD:
        del rho, u
        etags, ekw, erho, eu, ecfg = build_workload(EXTRA_WORKLOAD)
        eres = measure(etags, ekw, erho, eu, prec_names, args, label_prefix=EXTRA_WORKLOAD + " ")
        extra[EXTRA_WORKLOAD] = {"description": WORKLOADS[EXTRA_WORKLOAD], "steps": args.steps,
                                 "per_dtype": slim(eres), "error_vs_fp64": errors_vs_fp64(eres),
                                 "traffic_f32": stored_traffic(EXTRA_WORKLOAD, "f32"), **ecfg}
        rho = u = None

    cpu = None
    if not args.no_cpu_baseline:
        if args.workload == "tgv512_d3q27_smag":
            cpu = cpu_baseline(args.workload, None, kw, None, None, args.cpu_steps)
        else:
            cpu = cpu_baseline(args.workload, tags, kw, rho, u, args.cpu_steps)

    line = {
        "metric": METRIC, "value": round(m["MLUPS"], 2), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(m["ms_per_step"], 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"f32": "f32", "f64": "f64", "f16s": "f16-storage/f32"}[main_p],
        "data": "synthetic",
        "config": dict({"workload": args.workload, "description": WORKLOADS[args.workload], "q": kw["q"],
                        "tau": kw["tau"], "storage": main_p + "-shifted", "reduce_every": args.every}, **wl_cfg),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_dtype": slim(results),
        "error_vs_fp64": errors,
        "derived": derived,
        "extra": extra,
        "kernel_source_hash": source_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
