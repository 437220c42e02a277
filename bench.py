#!/usr/bin/env python
"""Benchmark of the density-kernel hot path on one MI355X.

A step is one pass of the whole path on the 32-atom aluminium-like cell
(48^3 grid, N_s = 512, kT = 2 Ha, filter degree 24, expansion degree 200):
spectral bounds of H_s, Chebyshev filter, CholQR2, projection, density kernel
with its Fermi level, density, band/entropy energies and forces.  Both the FP64
path and the mixed path (FP32 block and stencil, split-BF16 projection and
density products) are run; the JSON line leads with the mixed path and carries
the FP64 numbers and the mixed-vs-FP64 accuracy beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

`value` is the H.X throughput: algorithmic bytes of the filter's Hamiltonian
applications (3 block arrays per application, 2 for the first, plus V_eff)
divided by the GPU time of the filter calls.  `ms_per_step` is the wall time
of a whole step.  Inputs are resident in HBM before the timed region starts.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}

# HBM bytes per launch of each kernel kind of the al32 mixed step, from the
# rocprofv3 FETCH_SIZE / WRITE_SIZE runs summarised in profiles/al32_mixed_bytes.md
# (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000 by the plain-copy calibration there).
# An entry must be removed when its kernels change.
MEASURED_TRAFFIC = {
    ("al32", "mixed"): {
        "stencil": (490.1e6, 226.5e6),
        "nl_scatter": (455.9e6, 226.5e6),
        # the filter steps' two-piece integrals (24 of the 25 applications) plus
        # the reduction of their partials
        "nl_gather": (286.3e6 + 37.8e6, 32.5e6 + 0.4e6),
    },
}


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="al32")
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 256-atom cell (one SCF electronic step per precision)")
    ap.add_argument("--large-workload", default="al256")
    ap.add_argument("--large-passes", type=int, default=6,
                    help="filter passes of the large cell's first SCF iteration")
    ap.add_argument("--large-only", action="store_true",
                    help="only the large-cell electronic step (one JSON object)")
    ap.add_argument("--cpu-columns", type=int, default=32,
                    help="columns of the block in the oracle's timed filter sample")
    ap.add_argument("--scf", action="store_true",
                    help="time the self-consistent loop instead (default workload al108)")
    ap.add_argument("--qmd", action="store_true",
                    help="time molecular-dynamics steps instead (default workload al32_md)")
    ap.add_argument("--iters", type=int, default=40, help="SCF iterations (--scf) or cap (--qmd)")
    ap.add_argument("--md-steps", type=int, default=20)
    ap.add_argument("--ensemble", default="nve", choices=["nve", "nvk"],
                    help="--qmd: NVE, or isokinetic (Gaussian thermostat)")
    ap.add_argument("--stress", action="store_true",
                    help="--qmd: stress per step and the Green-Kubo D and eta of the run")
    ap.add_argument("--learned", type=int, default=0,
                    help="--qmd: train the learned start on this many 32-atom snapshots (at the "
                    "workload's kT) and start every mixed-precision SCF from its prediction")
    ap.add_argument("--learned-steps", type=int, default=2000, help="Adam steps of --learned")
    ap.add_argument("--poisson", action="store_true",
                    help="time the Poisson solve of the SCF by CG and by AAR (default workload al108)")
    ap.add_argument("--solver", default="cg", choices=["cg", "aar"],
                    help="--scf/--qmd: linear solver of the Poisson and Kerker solves")
    ap.add_argument("--restart", action="store_true",
                    help="--scf/--qmd with --mixing kerker: restarted periodic Pulay")
    ap.add_argument("--mixing", default="pulay", choices=["pulay", "kerker"],
                    help="--scf/--qmd: Pulay, or Kerker-preconditioned periodic Pulay")
    return ap.parse_args()


def algorithmic_work(problem, precision, steps, degree, n_pl, prof):
    """Algorithmic bytes / flops of each kernel kind over the timed steps."""
    ng, ns, npj = problem.n_grid, problem.n_s, problem.n_proj
    s = 8 if precision == "fp64" else 4
    nnz = len(problem.proj["values"])
    # H.X applications per step: m in the filter (first has no Y_{k-1}) + 1 in the projection
    arrays = (3 * degree - 1) + 2
    hx_launches = degree + 1
    work = {
        "stencil": ("hbm", steps * (arrays * ng * ns * s + hx_launches * ng * s)),
        # projector products: 2 nnz N_s flops against N_grid N_s block bytes, an
        # intensity (<= 14 flop/B) below the FP32 MFMA / HBM balance (19.7): HBM-bound.
        # gather reads X and the table's nonzeros, writes C; scatter reads and
        # writes Y and reads the nonzeros and C
        "nl_gather": ("hbm", steps * hx_launches * (ng * ns * s + nnz * s + npj * ns * s)),
        "nl_scatter": ("hbm", steps * hx_launches * (2 * ng * ns * s + nnz * s + npj * ns * s)),
        "gram": ("mfma", steps * 2 * 1.0 * ng * ns * ns),
        "orth_apply": ("mfma", steps * 2 * 1.0 * ng * ns * ns),
        "project": ("mfma", steps * 2.0 * ng * ns * ns),
        # the T_j are symmetric: a product's unique work is its upper half, N_s^3
        "foe_gemm": ("mfma", steps * (n_pl - 1) * 1.0 * ns ** 3),
        "density": ("mfma", steps * 2.0 * ng * ns * ns),
    }
    return work


def mfma_dtype(kind, precision):
    if precision == "fp64":
        return "f64"
    # split-BF16 products run on the BF16 MFMA; the Gram and the FOE stay FP64
    return {"nl_gather": "bf16", "nl_scatter": "f32", "project": "bf16", "density": "bf16",
            "orth_apply": "bf16"}.get(kind, "f64")


# MFMA products per algorithmic product of the split-BF16 forms (mixed path)
SPLIT_PRODUCTS = {"project": 3, "density": 6, "orth_apply": 6}


def run_gpu(problem, precision, steps, warmup):
    import torch
    from paper_2112_08639_amd import _lib as L
    from paper_2112_08639_amd.pipeline import (Context, filter_pass, kernel_and_density, start,
                                                tau_length)

    spec = problem.spec
    degree, n_pl = spec.filter_degree, spec.n_pl
    ctx = Context(problem, precision)
    ctx.ensure_workspace(problem.n_s, n_pl)
    dev = ctx.device
    X = ctx.block(problem.x0)
    ns = X.shape[0]
    Hs = torch.zeros((ns, ns), dtype=torch.float64, device=dev)
    Ds = torch.zeros_like(Hs)
    tau = torch.zeros(tau_length(n_pl), dtype=torch.float64, device=dev)
    rho = torch.zeros(problem.n_grid, dtype=torch.float64, device=dev)
    gradv = torch.as_tensor(problem.gradv, dtype=torch.float64, device=dev).contiguous()

    last = {}

    def step():
        # the density kernel of the previous step already bounded this H_s
        b = (last["lo"], last["hi"]) if last else None
        filter_pass(ctx, X, Hs, degree, bounds=b)
        out = kernel_and_density(ctx, X, Hs, Ds, tau, rho, problem.n_e, spec.kT, n_pl, gradv)
        last["lo"], last["hi"] = out[0].lam_min, out[0].lam_max
        return out

    start(ctx, X, Hs)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    L.dk_profile_enable(ctx.h, True)
    filter_ms = 0.0
    call_ms = np.zeros(8)
    t0 = time.perf_counter()
    for _ in range(steps):
        info, e_band, e_ent, forces = step()
        t = L.dk_get_timings(ctx.h)
        filter_ms += t[0]
        call_ms += np.array(t)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = L.dk_profile_read(ctx.h)
    L.dk_profile_enable(ctx.h, False)
    stress = stress_of(ctx, problem, X, Ds)
    out = {
        "ms_per_step": (t1 - t0) * 1e3 / steps,
        "filter_ms_per_step": filter_ms / steps,
        "call_ms_per_step": dict(zip(["filter", "orthonormalize", "project", "bounds",
                                      "density_kernel", "density", "energy", "forces"],
                                     (call_ms / steps).round(4).tolist())),
        "kernel_ms": {k: (v[0], v[1]) for k, v in prof.items()},
        "info": info.as_dict(),
        "e_band": e_band, "e_ent": e_ent, "free_energy": e_band + e_ent,
        "forces": forces, "rho": rho.cpu().numpy(),
        "stress": stress,
    }
    ctx.close()
    return out


def stress_of(ctx, problem, X, Ds, reps=3):
    """Kinetic and nonlocal stress of the last step's orbitals (outside the timed
    steps): device-built projector tables for the same atoms, one untimed call,
    then reps calls timed by libdk's own HIP events."""
    from paper_2112_08639_amd import _lib as L
    from paper_2112_08639_amd.pipeline import ProjectorModel
    from workloads.cells import PROJ_CHANNELS, PROJ_CUTOFF_REL

    ctx.move_atoms(problem.positions, ProjectorModel(PROJ_CHANNELS, PROJ_CUTOFF_REL))
    kin, nl = L.dk_stress(ctx.h, X, Ds)
    L.dk_profile_enable(ctx.h, True)
    for _ in range(reps):
        kin, nl = L.dk_stress(ctx.h, X, Ds)
    prof = L.dk_profile_read(ctx.h)
    L.dk_profile_enable(ctx.h, False)
    return {"ms_per_call": round(prof["stress"][0] / reps, 3), "kinetic": kin.tolist(),
            "nonlocal": nl.tolist(), "unit": "Ha/bohr^3"}


def roofline_of(problem, precision, res, steps):
    spec = problem.spec
    measured = MEASURED_TRAFFIC.get((spec.name, precision), {})
    work = algorithmic_work(problem, precision, steps, spec.filter_degree, spec.n_pl, None)
    kern = res["kernel_ms"]
    # dominant kernel: largest total time among those with an algorithmic model
    cands = [(kern[k][0], k) for k in work if k in kern]
    total_ms, kind = max(cands)
    bound, amount = work[kind]
    launches = kern[kind][1]
    avg_ms = total_ms / launches
    per_launch = amount / launches
    if bound == "hbm":
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        peak, unit = HBM_PEAK_GBS, "GB/s"
    else:
        achieved = per_launch / (avg_ms * 1e-3) / 1e12
        peak, unit = PEAK_TFLOPS[mfma_dtype(kind, precision)], "TFLOP/s"
    table = {}
    for k, (b, amt) in work.items():
        if k not in kern:
            continue
        ms, n = kern[k]
        rate = amt / (ms * 1e-3)
        if b == "hbm":
            table[k] = {"ms": round(ms / steps, 4), "launches": n // steps, "GB/s": round(rate / 1e9, 1),
                        "frac": round(rate / 1e9 / HBM_PEAK_GBS, 4)}
        else:
            pk = PEAK_TFLOPS[mfma_dtype(k, precision)]
            table[k] = {"ms": round(ms / steps, 4), "launches": n // steps,
                        "TFLOP/s": round(rate / 1e12, 2), "frac": round(rate / 1e12 / pk, 4)}
            if precision == "mixed" and k in SPLIT_PRODUCTS:
                # the BF16 MFMA work actually issued (3 or 6 products per product)
                hw = rate * SPLIT_PRODUCTS[k] / 1e12
                table[k].update({"mfma_TFLOP/s": round(hw, 2), "mfma_frac": round(hw / pk, 4)})
    for k, (ms, n) in kern.items():
        if k not in table:
            table[k] = {"ms": round(ms / steps, 4), "launches": n // steps}
    traffic = None
    detail = None
    if kind in measured:
        rd, wr = measured[kind]
        traffic = rd + wr
        detail = {"read_bytes": rd, "write_bytes": wr, "unit": "bytes per launch",
                  "source": "profiles/al32_mixed_bytes.md"}
    roof = {"kernel": kind, "bound": bound, "achieved": round(achieved, 2), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 4), "traffic": traffic,
            "traffic_detail": detail, "avg_launch_ms": round(avg_ms, 5), "per_launch": per_launch}
    return roof, table


def hx_bytes(problem, precision, degree):
    s = 8 if precision == "fp64" else 4
    ng, ns = problem.n_grid, problem.n_s
    return (3 * degree - 1) * ng * ns * s + degree * ng * s


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(problem, columns, runs=3):
    """The oracle, as it stands, on a bounded sample of the same workload: the
    median of `runs` timings of the filter on `columns` columns and of the FOE
    at the full subspace size."""
    from threadpoolctl import threadpool_info

    from oracle import foe as ofoe
    from oracle.filter import chebyshev_filter
    from oracle.hamiltonian import Hamiltonian
    from oracle.orth import cholqr2

    spec = problem.spec
    H = Hamiltonian(problem)
    cols = min(columns, problem.n_s)
    X = cholqr2(problem.x0[:cols].T.copy(), problem.h)
    b = H.upper_bound()
    # FOE at the full subspace size on a seeded symmetric matrix of the same order
    rng = np.random.Generator(np.random.PCG64(9))
    ns = problem.n_s
    Q, _ = np.linalg.qr(rng.standard_normal((ns, ns)))
    Hs = (Q * np.sort(rng.uniform(-4.0, 12.0, ns))) @ Q.T
    t_filter, t_foe = [], []
    for _ in range(runs):
        t0 = time.perf_counter()
        chebyshev_filter(H, X, spec.filter_degree, 4.0, b, -1.0)
        t_filter.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        ofoe.density_kernel(Hs, problem.n_e, spec.kT, spec.n_pl)
        t_foe.append(time.perf_counter() - t0)
    tf, tk = float(np.median(t_filter)), float(np.median(t_foe))
    s = 8
    ng = problem.n_grid
    sample_bytes = (3 * spec.filter_degree - 1) * ng * cols * s + spec.filter_degree * ng * s
    pools = threadpool_info()
    threads = max([t.get("num_threads", 1) for t in pools] + [1])
    blas = sorted({f"{t.get('internal_api')} {t.get('version')} ({os.path.basename(t.get('filepath', ''))})"
                   for t in pools if t.get("user_api") == "blas"})
    est_step_s = tf * ns / cols + tk
    return {
        "value": round(sample_bytes / tf / 1e9, 3), "unit": "GB/s", "cores": threads,
        "kind": "oracle",
        "sample": (f"median of {runs}: filter on {cols} of {ns} columns x {spec.filter_degree} "
                   f"applications ({tf:.2f} s); FOE on a full {ns}x{ns} matrix, n_pl={spec.n_pl} "
                   f"({tk:.2f} s)"),
        "runs_s": {"filter": [round(t, 3) for t in t_filter], "foe": [round(t, 3) for t in t_foe]},
        "est_s_per_step_filter_plus_foe": round(est_step_s, 2),
        "cpu_model": _cpu_model(), "blas": blas, "host_cpus": os.cpu_count(),
    }


def large_rates(spec, prec, kern, n_pl):
    """Rates of the kernel kinds with an algorithmic model in one SCF iteration of the
    large cell (one filter pass of degree m, one H.X for the projection, CholQR2, one
    projection, the expansion to degree n_pl, one density product), and the roofline
    object of the slowest of them."""
    ng, ns, m = spec.n_grid, spec.n_s, spec.filter_degree
    s = 8 if prec == "fp64" else 4
    work = {
        "stencil": ("hbm", ((3 * m - 1) + 2) * ng * ns * s + (m + 1) * ng * s),
        "gram": ("mfma", 2 * 1.0 * ng * ns * ns),
        "orth_apply": ("mfma", 2 * 1.0 * ng * ns * ns),
        "project": ("mfma", 2.0 * ng * ns * ns),
        "density": ("mfma", 2.0 * ng * ns * ns),
        "foe_gemm": ("mfma", (n_pl - 1) * 1.0 * ns ** 3),
    }
    rates = {}
    for k, (b, amt) in work.items():
        ms = kern.get(k, 0.0)
        if ms <= 0:
            continue
        if b == "hbm":
            a, pk, unit = amt / (ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            a, pk, unit = amt / (ms * 1e-3) / 1e12, PEAK_TFLOPS[mfma_dtype(k, prec)], "TFLOP/s"
        rates[k] = {"ms": ms, unit: round(a, 2), "frac": round(a / pk, 4)}
        if prec == "mixed" and k in SPLIT_PRODUCTS:
            rates[k]["mfma_frac"] = round(a * SPLIT_PRODUCTS[k] / pk, 4)
    if not rates:
        return rates, None
    kind = max(rates, key=lambda k: rates[k]["ms"])
    b = work[kind][0]
    unit = "GB/s" if b == "hbm" else "TFLOP/s"
    pk = HBM_PEAK_GBS if b == "hbm" else PEAK_TFLOPS[mfma_dtype(kind, prec)]
    roof = {"kernel": kind, "bound": b if b == "hbm" else "mfma", "achieved": rates[kind][unit],
            "peak": pk, "unit": unit, "frac": rates[kind]["frac"],
            "dtype": "f64" if b == "hbm" and s == 8 else
                     ("f32" if b == "hbm" else mfma_dtype(kind, prec)),
            "per_step": "one launch-set per SCF iteration (times from HIP events)"}
    return rates, roof


def large_cell_step(name, precs, first_passes=2):
    """One SCF electronic step of the large cell in each precision, on tables built
    on the device from the atom positions (no host tables, no host block): SAD start,
    a seeded random start block drawn on the GPU (the same for both precisions),
    `first_passes` filter passes in the first iteration, then one timed iteration:
    one filter pass, CholQR2, projection, density kernel with the tail-rule degree,
    density, mixing and the next effective potential (Poisson, LDA), then forces."""
    import torch
    from paper_2112_08639_amd import _lib as L
    from paper_2112_08639_amd.pipeline import Context, ProjectorModel
    from paper_2112_08639_amd.scf import scf
    from workloads import Problem, spec_for
    from workloads.cells import PROJ_CHANNELS, PROJ_CUTOFF_REL, atom_positions

    spec = spec_for(name)
    pos = atom_positions(spec)
    ng = spec.n_grid
    empty = {"offsets": np.zeros(1, np.int64), "indices": np.zeros(0, np.int32),
             "values": np.zeros(0), "gamma": np.zeros(0), "atom": np.zeros(0, np.int32)}
    p0 = Problem(spec, pos, np.zeros(ng), empty, np.zeros((0, ng)))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3000 + spec.index)
    # an FP32-representable start block: both precisions start from the same values
    X64 = torch.randn((spec.n_s, ng), dtype=torch.float64, device="cuda", generator=gen)
    X64 = X64.to(torch.float32).to(torch.float64)
    res = {}
    for prec in precs:
        print(f"{name} {prec}: setting up", file=sys.stderr, flush=True)
        ctx = Context(p0, prec)
        ctx.move_atoms(pos, ProjectorModel(PROJ_CHANNELS, PROJ_CUTOFF_REL))
        X = X64.clone() if prec == "fp64" else X64.to(torch.float32)
        prof = {}

        def cb(it, r, F, ms):
            print(f"{name} {prec} scf {it}: residual {r:.3e} ms {ms:.0f}", file=sys.stderr,
                  flush=True)
            if it == 1:  # profile the second iteration only
                L.dk_profile_enable(ctx.h, True)
            else:
                prof.update(L.dk_profile_read(ctx.h))
                prof["filter_ms"] = L.dk_get_timings(ctx.h)[0]
        r = scf(p0, local_model(), prec, tol=1e-12, max_iter=2, first_passes=first_passes,
                X_init=X, ctx=ctx, callback=cb)
        L.dk_profile_enable(ctx.h, False)
        res[prec] = {"r": r, "prof": prof}
        del X
        ctx.close()
        torch.cuda.empty_cache()
    del X64
    torch.cuda.empty_cache()
    out = {"workload": f"{spec.name}: {spec.n_atoms} atoms, a={spec.a} bohr, grid {spec.n}^3, "
                       f"N_s={spec.n_s}, kT={spec.kT} Ha, filter degree {spec.filter_degree}, "
                       f"n_pl by the tail rule, device-built projector tables",
           "step": f"SCF iteration 2 (iteration 1: {first_passes} filter passes from the random "
                   "block); one filter pass, CholQR2, projection, density kernel, density, "
                   "mixing, next potential"}
    for prec, v in res.items():
        r, prof = v["r"], v["prof"]
        s = 8 if prec == "fp64" else 4
        # filter: degree applications, 3 arrays each (2 for the first) + V_eff
        hx = (3 * spec.filter_degree - 1) * ng * spec.n_s * s + spec.filter_degree * ng * s
        fm = prof.get("filter_ms", 0.0)
        kern = {k: round(v[0], 2) for k, v in prof.items() if isinstance(v, tuple) and v[1] > 0}
        top = max(((v, k) for k, v in kern.items()), default=(0, None))
        rates, roof = large_rates(spec, prec, kern, r.n_pl)
        out[prec] = {"s_per_step": round(r.iteration_ms[1] / 1e3, 3),
                     "first_iteration_s": round(r.iteration_ms[0] / 1e3, 3),
                     "filter_ms": round(fm, 1),
                     "hx_GB/s": round(hx / (fm * 1e-3) / 1e9, 1) if fm > 0 else None,
                     "hx_frac_of_hbm": round(hx / (fm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if fm > 0 else None,
                     "n_pl": r.n_pl, "kernel_ms": kern, "top_kernel": top[1],
                     "roofline": roof, "rates": rates,
                     "free_energy": r.free_energy, "e_band": r.e_band, "e_ent": r.e_ent,
                     "mu": r.mu}
    if len(res) == 2:
        a, b = res["mixed"]["r"], res["fp64"]["r"]
        ra, rb = a.rho.cpu().numpy(), b.rho.cpu().numpy()
        h3 = spec.volume / ng
        out["accuracy_mixed_vs_fp64"] = {
            "drho_per_ne": float(h3 * np.abs(ra - rb).sum() / spec.n_e),
            "dF_per_atom": abs(a.free_energy - b.free_energy) / spec.n_atoms,
            "dforce_max": float(np.abs(a.forces - b.forces).max()),
            "de_band_per_atom": abs(a.e_band - b.e_band) / spec.n_atoms,
            "de_ent_per_atom": abs(a.e_ent - b.e_ent) / spec.n_atoms,
            "dmu": abs(a.mu - b.mu),
            "reference": "FP64 GPU path, same start block and schedule"}
        out["speedup_mixed_vs_fp64"] = round(res["fp64"]["r"].iteration_ms[1]
                                             / res["mixed"]["r"].iteration_ms[1], 3)
    return out


def local_model():
    from paper_2112_08639_amd.scf import LocalModel
    from workloads.cells import CORE_AMP, CORE_W2, RC_LOC, Z_VALENCE
    return LocalModel(Z_VALENCE, RC_LOC, CORE_AMP, CORE_W2)


def scf_bench(args):
    """Wall time per SCF iteration, mixed vs FP64, on the same iteration schedule."""
    import torch
    from paper_2112_08639_amd import _lib as L
    from paper_2112_08639_amd.pipeline import Context
    from paper_2112_08639_amd.scf import scf
    from workloads import make_problem, spec_for

    name = args.workload if args.workload != "al32" else "al108"
    spec = spec_for(name)
    problem = make_problem(spec)
    out = {}
    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    for prec in precs:
        ctx = Context(problem, prec)
        L.dk_profile_enable(ctx.h, True)
        cb = lambda it, r, F, ms: print(f"{prec} scf {it}: residual {r:.3e} ms {ms:.1f}",
                                        file=sys.stderr, flush=True)
        r = scf(problem, local_model(), prec, tol=1e-6, max_iter=args.iters, ctx=ctx, callback=cb,
                mixing=args.mixing, restart=args.restart, solver=args.solver)
        prof = L.dk_profile_read(ctx.h)
        out[prec] = {
            "iterations": r.iterations, "converged": r.converged,
            "first_iteration_ms": round(r.iteration_ms[0], 1),
            "ms_per_iteration": round(float(np.median(r.iteration_ms[1:])), 2),
            "final_residual": r.residuals[-1], "free_energy": r.free_energy, "n_pl": r.n_pl,
            "residuals": [float(x) for x in r.residuals],
            "poisson_iters_median": int(np.median(r.poisson_iters[1:])),
            "kernel_ms_per_iteration": {k: round(v[0] / r.iterations, 2) for k, v in prof.items()},
            "rho": r.rho.cpu().numpy(), "forces": r.forces,
        }
        ctx.close()
    acc = speedup = None
    if len(out) == 2:
        a, b = out["mixed"], out["fp64"]
        acc = {"drho_per_ne": float(problem.h ** 3 * np.abs(a["rho"] - b["rho"]).sum() / problem.n_e),
               "dF_per_atom": abs(a["free_energy"] - b["free_energy"]) / spec.n_atoms,
               "dforce_max": float(np.abs(a["forces"] - b["forces"]).max())}
        speedup = round(b["ms_per_iteration"] / a["ms_per_iteration"], 3)
    for v in out.values():
        v.pop("rho"), v.pop("forces")
    lead = out["mixed"] if "mixed" in out else out[precs[0]]
    mixing = "Pulay(7)" if args.mixing == "pulay" else "Kerker-preconditioned periodic Pulay(7, period 2)"
    print(json.dumps({
        "metric": "s per SCF iteration, mixed vs FP64", "workload": f"{spec.name}: {spec.n_atoms} atoms, "
        f"grid {spec.n}^3, N_s={spec.n_s}, kT={spec.kT} Ha, PW92, CG Poisson, {mixing}",
        "value": lead["ms_per_iteration"] / 1e3, "unit": "s", "higher_is_better": False,
        "speedup_mixed_vs_fp64": speedup, **out, "accuracy_mixed_vs_fp64": acc,
        "data": "synthetic"}, default=float))


def green_kubo_of(problem, tr):
    """Green-Kubo D and eta of a finished trajectory (libdk: dk_deviatoric_stress,
    dk_time_correlation), over lags up to half the run."""
    from paper_2112_08639_amd.pipeline import Context
    from paper_2112_08639_amd.qmd import EV, FS, M_AL
    from paper_2112_08639_amd.transport import green_kubo

    ctx = Context(problem, "fp64")
    try:
        n = len(tr.velocities)
        g = green_kubo(ctx.h, np.stack(tr.velocities), tr.total_stress(), 0.5 * FS, 10.0 * EV,
                       M_AL, problem.spec.volume, max(2, n // 2))
    finally:
        ctx.close()
    return {**g.summary(), "vacf_over_3": g.vacf_over_3.tolist(), "sacf": g.sacf.tolist(),
            "note": "one short run: a smoke test of the Green-Kubo path, not converged statistics"}


def poisson_bench(args, reps=5):
    """CG against AAR on the electrostatic solve of the SCF, -Lap_h V = 4 pi (rho + b),
    for a net charge rho + b = 1e-2 rho_SAD w1 (w1 seeded white noise: every wave
    vector of the grid), from zero ("cold"), and from the solution for that source
    when the source changes by 1e-4 rho_SAD w2 ("warm", as between SCF iterations)."""
    import torch
    from paper_2112_08639_amd import _lib as L
    from paper_2112_08639_amd.pipeline import Context
    from workloads import make_problem, spec_for

    name = args.workload if args.workload != "al32" else "al108"
    spec = spec_for(name)
    problem = make_problem(spec, with_block=False)
    m = local_model()
    ctx = Context(problem, "fp64")
    ctx.ensure_workspace(1, 16)
    f64 = dict(dtype=torch.float64, device=ctx.device)
    L.dk_set_atoms(ctx.h, problem.positions, m.z, m.rc, m.core_amp, m.core_w2)
    b = torch.zeros(problem.n_grid, **f64)
    L.dk_get_local_fields(ctx.h, b, None)
    rho = torch.zeros_like(b)
    L.dk_start_density(ctx.h, rho)
    rng = np.random.Generator(np.random.PCG64(11))
    w1 = torch.as_tensor(rng.standard_normal(problem.n_grid), **f64)
    w2 = torch.as_tensor(rng.standard_normal(problem.n_grid), **f64)
    src_warm = 1e-2 * rho * w1
    src = src_warm + 1e-4 * rho * w2
    out = {}
    for name_s, solver in (("cg", L.DK_SOLVER_CG), ("aar", L.DK_SOLVER_AAR)):
        L.dk_set_linear_solver(ctx.h, solver)
        v0 = torch.zeros_like(b)
        L.dk_poisson(ctx.h, src_warm, v0, 1e-10, 50000)
        res = {}
        for start in ("cold", "warm"):
            its, ms = [], []
            for _ in range(reps):
                v = torch.zeros_like(b) if start == "cold" else v0.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                it, rr = L.dk_poisson(ctx.h, src, v, 1e-10, 50000)
                torch.cuda.synchronize()
                ms.append((time.perf_counter() - t0) * 1e3)
                its.append(it)
            res[start] = {"iterations": its[0], "ms": round(float(np.median(ms)), 3)}
        out[name_s] = res
    ctx.close()
    print(json.dumps({"metric": "ms per electrostatic solve (tol 1e-10), CG vs AAR",
                      "workload": f"{spec.name}: grid {spec.n}^3, white-noise net charge",
                      "aar_parameters": {"omega": 0.6, "beta": 0.6, "history": 7, "period": 6},
                      **out, "data": "synthetic"}))


def train_learned_start(target, n_train, adam_steps, scf_iters=30):
    """Learned start trained on converged densities of the 32-atom cell (positions
    jittered N(0, 0.3 bohr), snapshot s seeded 4000 + s) at the electronic temperature
    of `target`, by the mixed SCF; returns a predictor on the target cell."""
    import dataclasses

    import torch
    from paper_2112_08639_amd import _lib as L
    from paper_2112_08639_amd.learned import LearnedStart, MlpConfig
    from paper_2112_08639_amd.pipeline import PRECISIONS, Context
    from paper_2112_08639_amd.scf import scf
    from workloads import make_problem, spec_for

    spec = dataclasses.replace(spec_for("al32_md"), kT=target.kT)
    base = make_problem(spec, snapshot=0)
    ctx = Context(base, "mixed")
    ls = LearnedStart(ctx.h, base.n_grid, spec.volume, base.n_e, MlpConfig(steps=adam_steps),
                      max_snapshots=n_train)
    t0 = time.perf_counter()
    res = []
    for s in range(n_train):
        p = make_problem(spec, snapshot=s, with_block=False)
        p.x0 = base.x0
        ctx.set_problem(p)
        r = scf(p, local_model(), "mixed", tol=1e-6, max_iter=scf_iters, forces=False, ctx=ctx)
        ls.add_snapshot(p.positions, r.rho)
        res.append(r.residuals[-1])
        print(f"learned start: snapshot {s} residual {r.residuals[-1]:.2e}", file=sys.stderr,
              flush=True)
    t_data = time.perf_counter() - t0
    log = ls.fit()
    nx, ny, nz = target.shape
    lx, ly, lz = target.cell
    stream = torch.cuda.current_stream()
    h = L.dk_create(nx, ny, nz, lx, ly, lz, PRECISIONS["mixed"], 0, stream)
    pred = ls.for_cell(h, target.n_grid, target.volume, target.n_e)
    ctx.close()
    info = {"train_cell": f"32 atoms, grid {spec.n}^3, N_s={spec.n_s}, kT={spec.kT} Ha, "
                          f"jitter N(0, {spec.jitter_amp} bohr)",
            "train_snapshots": n_train, "train_scf_iterations": scf_iters,
            "train_final_residual_median": float(np.median(res)),
            "train_data_s": round(t_data, 1), "adam_steps": adam_steps,
            "ms_per_adam_step": round(log.ms_per_step, 3),
            "loss_first": log.losses[0], "loss_last": log.losses[-1]}
    return pred, h, info


def qmd_bench(args):
    """Wall time per molecular-dynamics step and energy drift, mixed vs FP64."""
    import torch
    from paper_2112_08639_amd import _lib as L
    from paper_2112_08639_amd.qmd import qmd
    from workloads import make_problem, spec_for

    from paper_2112_08639_amd.pipeline import ProjectorModel
    from workloads.cells import PROJ_CHANNELS, PROJ_CUTOFF_REL

    name = args.workload if args.workload != "al32" else "al32_md"
    spec = spec_for(name)
    base = make_problem(spec)
    # every ionic step builds its projector tables on the device
    projectors = ProjectorModel(PROJ_CHANNELS, PROJ_CUTOFF_REL)

    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    out = {}
    learned = pred_h = None
    if args.learned > 0 and "mixed" in precs:
        learned, pred_h, learned_info = train_learned_start(spec, args.learned, args.learned_steps)
        out["learned_start"] = learned_info
    for prec in precs:
        start = None
        if learned is not None and prec == "mixed":
            start = lambda pos: learned.predict(pos)
        cb = lambda step, tr: print(f"{prec} md {step}: E {tr.energies[-1]:.8f} scf "
                                    f"{tr.scf_iterations[-1]} ms {tr.step_ms[-1]:.0f}",
                                    file=sys.stderr, flush=True)
        scb = lambda it, res, F, ms: print(f"{prec} scf {it}: residual {res:.2e} ms {ms:.0f}",
                                           file=sys.stderr, flush=True)
        tr = qmd(base, None, local_model(), prec, steps=args.md_steps, scf_max_iter=args.iters,
                 callback=cb, projectors=projectors,
                 scf_callback=scb if spec.n_atoms > 100 else None, ensemble=args.ensemble,
                 mixing=args.mixing, stress=args.stress, restart=args.restart,
                 solver=args.solver, start_density=start)
        e = np.array(tr.energies)
        gk = None
        if args.stress:
            gk = green_kubo_of(base, tr)
        out[prec] = {"ms_per_step": round(float(np.median(tr.step_ms[1:])), 1),
                     "first_step_ms": round(tr.step_ms[0], 1),
                     "start": "learned" if start is not None else
                              "SAD, then the previous step's density",
                     "scf_iterations": tr.scf_iterations,
                     "scf_final_residuals": [float(r) for r in tr.scf_residuals],
                     "drift_per_atom": float((e[-1] - e[0]) / spec.n_atoms),
                     "max_dev_per_atom": float(np.abs(e - e[0]).max() / spec.n_atoms),
                     "kinetic_range": float(np.ptp(tr.kinetic)),
                     "potential_range_per_atom": float(np.ptp(tr.free_energies) / spec.n_atoms),
                     "positions": tr.positions[-1]}
        if gk is not None:
            out[prec]["green_kubo"] = gk
    if pred_h is not None:
        L.dk_destroy(pred_h)
    dpos = (float(np.abs(out["mixed"]["positions"] - out["fp64"]["positions"]).max())
            if "mixed" in out and "fp64" in out else None)
    for k in precs:
        out[k].pop("positions")
    lead = "mixed" if "mixed" in out else precs[0]
    print(json.dumps({
        "metric": "s per QMD step, mixed vs FP64", "workload": f"{spec.name}: {spec.n_atoms} atoms, "
        f"grid {spec.n}^3, N_s={spec.n_s}, kT={spec.kT} Ha, {args.ensemble.upper()} dt=0.5 fs, "
        f"ions at 10 eV",
        "value": out[lead]["ms_per_step"] / 1e3, "unit": "s", "higher_is_better": False,
        "steps": args.md_steps, **out, "max_position_difference_bohr": dpos,
        "data": "synthetic"}, default=float))


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design, not a build.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from workloads import make_problem, spec_for

    if args.large_only:
        print(json.dumps(large_cell_step(args.large_workload, ["mixed", "fp64"],
                                         args.large_passes), default=float))
        return
    if args.poisson:
        return poisson_bench(args)
    if args.scf:
        return scf_bench(args)
    if args.qmd:
        return qmd_bench(args)
    spec = spec_for(args.workload)
    problem = make_problem(spec)
    _ = problem.gradv  # built before the timed region
    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    res = {p: run_gpu(problem, p, args.steps, args.warmup) for p in precs}
    lines = {}
    for p in precs:
        r = res[p]
        roof, table = roofline_of(problem, p, r, args.steps)
        gbs = hx_bytes(problem, p, spec.filter_degree) / (r["filter_ms_per_step"] * 1e-3) / 1e9
        lines[p] = {"value": round(gbs, 1), "ms_per_step": round(r["ms_per_step"], 3),
                    "filter_ms_per_step": round(r["filter_ms_per_step"], 3),
                    "roofline": roof, "kernels": table, "calls_ms": r["call_ms_per_step"],
                    "mu": r["info"]["mu"], "free_energy": r["free_energy"],
                    "stress": r["stress"]}
    lead = "mixed" if "mixed" in precs else precs[0]
    acc = None
    if len(precs) == 2:
        a, b = res["mixed"], res["fp64"]
        acc = {
            "drho_per_ne": float(problem.h ** 3 * np.abs(a["rho"] - b["rho"]).sum() / problem.n_e),
            "dF_per_atom": abs(a["free_energy"] - b["free_energy"]) / spec.n_atoms,
            "dforce_max": float(np.abs(a["forces"] - b["forces"]).max()),
            "dstress_max": float(max(
                np.abs(np.asarray(a["stress"][t]) - np.asarray(b["stress"][t])).max()
                for t in ("kinetic", "nonlocal"))),
            "reference": "FP64 GPU path (parity-tested against the FP64 oracle)",
        }
    out = {
        "metric": "H.X stencil GB/s + s per density-kernel step, mixed vs FP64, at drho/N_e<=1e-5",
        "value": lines[lead]["value"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": lines[lead]["ms_per_step"],
        "s_per_dk_step": round(lines[lead]["ms_per_step"] / 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if lead == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{spec.name}: {spec.n_atoms} atoms, a={spec.a} bohr, grid {spec.n}^3, "
                               f"N_s={spec.n_s}, kT={spec.kT} Ha, filter degree {spec.filter_degree}, "
                               f"n_pl={spec.n_pl}", "precision": lead},
        "roofline": lines[lead]["roofline"],
        "kernels": lines[lead]["kernels"],
        "calls_ms": lines[lead]["calls_ms"],
        "stress": lines[lead]["stress"],
    }
    if "fp64" in lines and lead != "fp64":
        out["fp64"] = {k: lines["fp64"][k] for k in ("value", "ms_per_step", "filter_ms_per_step",
                                                      "roofline", "kernels", "calls_ms", "stress")}
    if acc:
        out["accuracy_mixed_vs_fp64"] = acc
    if not args.no_large:
        out["large_cell"] = large_cell_step(args.large_workload, ["mixed", "fp64"],
                                            args.large_passes)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problem, args.cpu_columns)
    print(json.dumps(out, default=float))


if __name__ == "__main__":
    main()
