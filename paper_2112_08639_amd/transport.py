"""Green-Kubo self-diffusion and viscosity of a QMD run (libdk calls only).

Sec. 5 (high-temperature QMD) computes the self-diffusion coefficient and the
shear viscosity as time integrals of the velocity and stress autocorrelation
functions.  The series are uploaded once; the deviatoric stress components
(with the ions' momentum flux removed from the Hellmann-Feynman stress), the
correlations over time origins and their trapezoid integrals are libdk calls
(dk_deviatoric_stress, dk_time_correlation).

Units: atomic (bohr, a.u. of time, Ha).  1 bohr^2 / a.u. of time =
1.15767 cm^2/s; 1 Ha a.u.-time / bohr^3 = 0.711664 mPa s.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

BOHR_CM = 0.529177210903e-8
AU_TIME_S = 2.4188843265857e-17
HA_PER_BOHR3_PA = 4.3597447222071e-18 / (0.529177210903e-10) ** 3
D_AU_TO_CM2_S = BOHR_CM ** 2 / AU_TIME_S
ETA_AU_TO_MPA_S = HA_PER_BOHR3_PA * AU_TIME_S * 1e3


@dataclass
class GreenKubo:
    dt: float                 # sample spacing (a.u. of time)
    vacf_over_3: np.ndarray   # (1/3N) sum_i <v_i(t) . v_i(0)>
    diffusion: np.ndarray     # D(t_k), bohr^2 / a.u. of time
    sacf: np.ndarray          # (1/5) sum_m <s_m(t) s_m(0)>, (Ha/bohr^3)^2
    viscosity: np.ndarray     # eta(t_k), Ha a.u.-time / bohr^3

    def summary(self) -> dict:
        return {"D_cm2_per_s": float(self.diffusion[-1] * D_AU_TO_CM2_S),
                "eta_mPa_s": float(self.viscosity[-1] * ETA_AU_TO_MPA_S),
                "lags": len(self.diffusion), "t_max_fs": float(self.dt * (len(self.diffusion) - 1)
                                                               / 41.341374575751)}


def green_kubo(h, velocities, stresses, dt: float, kT: float, mass: float, volume: float,
               max_lag: int) -> GreenKubo:
    """velocities (T, N, 3) and HF stresses (T, 3, 3) per ionic step (host or
    device); dt the step; kT the ion temperature (Ha); volume the cell."""
    dev = torch.device("cuda", torch.cuda.current_device())
    f64 = dict(dtype=torch.float64, device=dev)
    v = torch.as_tensor(np.asarray(velocities, dtype=np.float64), **f64).contiguous()
    sig = torch.as_tensor(np.asarray(stresses, dtype=np.float64), **f64).contiguous()
    T, n_atoms = v.shape[0], v.shape[1]
    c_v = torch.zeros(max_lag, **f64)
    d = torch.zeros(max_lag, **f64)
    L.dk_time_correlation(h, v.view(T, 3 * n_atoms), max_lag, dt, 1.0, corr=c_v, integral=d)
    s = L.dk_deviatoric_stress(h, sig, v, mass)
    c_s = torch.zeros(max_lag, **f64)
    eta = torch.zeros(max_lag, **f64)
    L.dk_time_correlation(h, s, max_lag, dt, volume / kT, corr=c_s, integral=eta)
    return GreenKubo(dt, c_v.cpu().numpy(), d.cpu().numpy(), c_s.cpu().numpy(),
                     eta.cpu().numpy())
