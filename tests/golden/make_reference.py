"""Write the oracle's results for a full workload to tests/golden/<name>_oracle.json.

    python tests/golden/make_reference.py al32

Calls only the oracle (and the seeded input generator).  Stored: Fermi level,
band and entropy energies, band free energy, forces, the spectral bounds used
by each filter pass, h^3 sum rho, and rho at 4096 seeded sample points, so the
library can be checked at the full size without rerunning the oracle.
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import sq3  # noqa: E402
from workloads import make_problem, spec_for  # noqa: E402


def sample_indices(n_grid: int, count: int = 4096) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(7777))
    return np.sort(rng.choice(n_grid, size=min(count, n_grid), replace=False))


def main(name: str) -> None:
    spec = spec_for(name)
    t0 = time.time()
    p = make_problem(spec)
    r = sq3.run(p)
    idx = sample_indices(p.n_grid)
    out = {
        "workload": name,
        "source": "oracle.sq3.run (FP64 NumPy), inputs from workloads.make_problem",
        "mu": r.dk.mu,
        "e_band": r.e_band,
        "e_ent": r.e_ent,
        "free_energy": r.free_energy,
        "lam_min": r.dk.lam_min,
        "lam_max": r.dk.lam_max,
        "n_pl": r.dk.n_pl,
        "integral_rho": float(p.h ** 3 * r.rho.sum()),
        "abs_rho_sum": float(np.abs(r.rho).sum()),
        "forces": r.forces.tolist(),
        "bounds": [list(b) for b in r.bounds],
        "rho_sample_index": idx.tolist(),
        "rho_sample": r.rho[idx].tolist(),
        "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path} in {out['seconds']:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "al32")
