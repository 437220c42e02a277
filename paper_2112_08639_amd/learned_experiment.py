"""Train the learned start density on SCF densities and compare it with SAD.

    python -m paper_2112_08639_amd.learned_experiment [--train 200] [--test 50]

Workload: the 32-atom aluminium-like cell with positions jittered by
N(0, 0.3 bohr) per snapshot (snapshot s seeded 4000 + s).  Each training
snapshot is run by the mixed-precision SCF from the superposition-of-atomic-
densities (SAD) start; its final density is a training target.  The network
(32 descriptors -> 3 x 64 SiLU -> 1) is trained by Adam on the GPU.  Each
held-out snapshot is then run twice, from SAD and from the network's
prediction, with the same SCF settings; reported per start: the error of the
start density against the SCF result (h^3 sum |rho_0 - rho| / N_e), the
iterations until the residual first drops below each threshold, and the
final free energy.  One JSON line on stdout; progress lines on stderr.
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

THRESHOLDS = (1e-2, 3e-3, 1e-3)


def first_below(res, thr):
    for i, r in enumerate(res):
        if r <= thr:
            return i + 1
    return None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="al32_md")
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--test", type=int, default=50)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--scf-iters", type=int, default=30)
    ap.add_argument("--precision", default="mixed")
    args = ap.parse_args(argv)

    from workloads import make_problem, spec_for
    from workloads.cells import CORE_AMP, CORE_W2, RC_LOC, Z_VALENCE

    from .learned import LearnedStart, MlpConfig
    from .pipeline import Context
    from .scf import LocalModel, scf

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    spec = spec_for(args.workload)
    model = LocalModel(Z_VALENCE, RC_LOC, CORE_AMP, CORE_W2)
    base = make_problem(spec, snapshot=0)
    ctx = Context(base, args.precision)

    def problem(s):
        p = make_problem(spec, snapshot=s, with_block=False)
        p.x0 = base.x0
        ctx.set_problem(p)
        return p

    def run(p, rho0=None):
        return scf(p, model, args.precision, tol=1e-6, max_iter=args.scf_iters, rho0=rho0,
                   forces=False, ctx=ctx)

    cfg = MlpConfig(steps=args.steps, batch=args.batch)
    ls = LearnedStart(ctx.h, base.n_grid, spec.a ** 3, base.n_e, cfg, max_snapshots=args.train)
    t0 = time.perf_counter()
    train_res = []
    for s in range(args.train):
        p = problem(s)
        r = run(p)
        ls.add_snapshot(p.positions, r.rho)
        train_res.append(r.residuals[-1])
        if s % 10 == 0:
            log(f"train snapshot {s}: final residual {r.residuals[-1]:.2e}, "
                f"{(time.perf_counter() - t0):.0f} s")
    t_data = time.perf_counter() - t0
    tl = ls.fit(log_every=200)
    log(f"trained {cfg.steps} steps, {tl.ms_per_step:.2f} ms/step, loss {tl.losses[-1]:.3e}")

    rows = []
    for j in range(args.test):
        s = args.train + j
        p = problem(s)
        rho_sad = torch.zeros(p.n_grid, dtype=torch.float64, device=ctx.device)
        from . import _lib as L
        L.dk_set_atoms(ctx.h, p.positions, model.z, model.rc, model.core_amp, model.core_w2)
        L.dk_start_density(ctx.h, rho_sad)
        rho_mlp = ls.predict(p.positions).clone()
        ra = run(p)
        rb = run(p, rho0=rho_mlp)
        ref = ra.rho
        row = {"snapshot": s}
        for name, r0, rr in (("sad", rho_sad, ra), ("mlp", rho_mlp, rb)):
            err0 = float(p.h ** 3 * (r0 - ref).abs().sum().item() / p.n_e)
            row[name] = {"start_err": err0,
                         "iters_to": [first_below(rr.residuals, t) for t in THRESHOLDS],
                         "final_res": rr.residuals[-1], "free_energy": rr.free_energy}
        row["drho_final"] = float(p.h ** 3 * (ra.rho - rb.rho).abs().sum().item() / p.n_e)
        rows.append(row)
        log(f"test {s}: start err sad {row['sad']['start_err']:.3e} mlp {row['mlp']['start_err']:.3e}; "
            f"iters sad {row['sad']['iters_to']} mlp {row['mlp']['iters_to']}")

    def agg(name, key):
        return float(np.mean([r[name][key] for r in rows]))

    def iters(name, k):
        v = [r[name]["iters_to"][k] for r in rows]
        hit = [x for x in v if x is not None]
        return {"mean": float(np.mean(hit)) if hit else None, "reached": len(hit), "of": len(v)}

    out = {
        "experiment": "learned start density vs SAD",
        "workload": f"{spec.name}: {spec.n_atoms} atoms, grid {spec.n}^3, N_s={spec.n_s}, kT={spec.kT} Ha",
        "precision": args.precision, "train_snapshots": args.train, "test_snapshots": args.test,
        "scf_iterations_per_run": args.scf_iters, "train_data_s": round(t_data, 1),
        "train_final_residual_median": float(np.median(train_res)),
        "mlp": {"steps": cfg.steps, "batch": cfg.batch, "ms_per_step": round(tl.ms_per_step, 3),
                "loss_first": tl.losses[0], "loss_last": tl.losses[-1]},
        "start_err_mean": {"sad": agg("sad", "start_err"), "mlp": agg("mlp", "start_err")},
        "iters_to_threshold": {f"{t:g}": {"sad": iters("sad", i), "mlp": iters("mlp", i)}
                               for i, t in enumerate(THRESHOLDS)},
        "final_residual_mean": {"sad": agg("sad", "final_res"), "mlp": agg("mlp", "final_res")},
        "drho_final_mean": float(np.mean([r["drho_final"] for r in rows])),
        "dF_final_per_atom_mean": float(np.mean([abs(r["sad"]["free_energy"] - r["mlp"]["free_energy"])
                                                 for r in rows]) / spec.n_atoms),
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
