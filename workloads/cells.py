"""Synthetic aluminium-like cells: atoms, fixed potential, projectors, start block.

The workloads stand in for the paper's fcc aluminium systems (Sec. 5: fcc Al at
2.7 g/cc, atoms perturbed from their lattice sites, three valence electrons per
atom, twelfth-order finite differences, Gamma point).  The paper's ONCV
pseudopotential is not available, so the local potential and the
Kleinman-Bylander projectors (Eq. nonlocaloperator) are analytic model forms:

* local potential of atom J:  v(r) = -Z erf(r / 0.8) / r  -  1.5 exp(-r^2 / 0.5)
  with Z = 3.  The erf part is the periodic potential of Gaussian charges with
  a neutralising background (G = 0 term dropped), summed analytically in
  reciprocal space; the short-range core part is a periodic image sum.
* fixed effective potential V_eff = sum_J v + 0.05 N(0,1) noise convolved with
  a unit-integral Gaussian of width 1 bohr (only the noise is smoothed).
* two projector channels per atom: l = 0, chi = A0 exp(-r^2/1.2^2), gamma
  +0.5 Ha; l = 1, chi_alpha = A1 x_alpha exp(-r^2/1.4^2) (alpha = x, y, z),
  gamma -0.3 Ha.  A_l normalise each function to unit continuum L2 norm.  The
  periodic extension sums every image whose Gaussian factor exceeds 1e-8 of
  its peak, i.e. |x - R - L| <= rc sqrt(ln 1e8).

Grid convention: n points per axis, h = a / n, point (i, j, k) at (ih, jh, kh)
with flat index i + n (j + n k) (x fastest).  Blocks of N_s grid vectors are
float64 arrays of shape (N_s, N_grid): row c is column c of the paper's
N_grid x N_s block, i.e. the memory layout is column-major N_grid x N_s.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

Z_VALENCE = 3.0
RC_LOC = 0.8
CORE_AMP = 1.5
CORE_W2 = 0.5
NOISE_AMP = 0.05
NOISE_SIGMA = 1.0
# (l, rc, gamma) of the two projector channels
PROJ_CHANNELS = ((0, 1.2, 0.5), (1, 1.4, -0.3))
PROJ_CUTOFF_REL = 1e-8
FD_RADIUS = 6  # twelfth-order central differences


@dataclass(frozen=True)
class CellSpec:
    """One workload: cell, grid, subspace size and expansion degrees."""

    name: str
    index: int            # seeds: jitter 1000+index, noise 2000+index, block 3000+index
    a0: float             # edge of the conventional cube (bohr)
    reps: int             # cubes per axis
    n: int                # grid points per axis
    n_s: int              # auxiliary orbitals
    kT: float             # smearing sigma (Ha)
    filter_degree: int
    filter_passes: int
    n_pl: int             # Chebyshev degree of the Fermi-operator expansion
    jitter: str = "uniform"   # "uniform" | "normal" | "none"
    jitter_amp: float = 0.2
    basis: str = "fcc"        # "fcc" (4 atoms per cube) or "sc" (1 atom per cube)
    noise: bool = True
    # orthorhombic cells: points (nx, ny, nz) and edges (lx, ly, lz) per axis;
    # None = the cube of n points and edge a on every axis
    dims: Optional[Tuple[int, int, int]] = None
    lens: Optional[Tuple[float, float, float]] = None

    @property
    def a(self) -> float:
        return self.a0 * self.reps

    @property
    def cubic(self) -> bool:
        return self.dims is None and self.lens is None

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.n, self.n, self.n) if self.dims is None else tuple(self.dims)

    @property
    def cell(self) -> Tuple[float, float, float]:
        return (self.a, self.a, self.a) if self.lens is None else tuple(self.lens)

    @property
    def spacing(self) -> Tuple[float, float, float]:
        return tuple(l / m for l, m in zip(self.cell, self.shape))

    @property
    def h(self) -> float:
        """Grid spacing of a cubic grid; (hx hy hz)^(1/3) otherwise (the volume
        element is h^3)."""
        if self.cubic:
            return self.a / self.n
        hx, hy, hz = self.spacing
        return (hx * hy * hz) ** (1.0 / 3.0)

    @property
    def volume(self) -> float:
        if self.cubic:
            return self.a ** 3
        lx, ly, lz = self.cell
        return lx * ly * lz

    @property
    def n_grid(self) -> int:
        if self.cubic:
            return self.n ** 3
        nx, ny, nz = self.shape
        return nx * ny * nz

    @property
    def n_atoms(self) -> int:
        per = 4 if self.basis == "fcc" else 1
        return per * self.reps ** 3

    @property
    def n_e(self) -> float:
        return Z_VALENCE * self.n_atoms


# The five workloads (cell edge 7.6 bohr per cube gives h = 0.31667 bohr on every grid).
CONFIGS: Dict[str, CellSpec] = {
    "al4": CellSpec("al4", 0, 7.6, 1, 24, 64, 1.0, 20, 6, 120),
    "al32": CellSpec("al32", 1, 7.6, 2, 48, 512, 2.0, 24, 6, 200),
    "al108": CellSpec("al108", 2, 7.6, 3, 72, 2048, 5.0, 24, 6, 0),
    "al32_md": CellSpec("al32_md", 3, 7.6, 2, 48, 512, 2.0, 24, 6, 0,
                        jitter="normal", jitter_amp=0.3),
    "al256": CellSpec("al256", 4, 7.6, 4, 96, 4096, 10.0, 24, 6, 0),
}


def spec_for(name: str) -> CellSpec:
    return CONFIGS[name]


def custom_spec(name: str, index: int, a0: float, reps: int, n: int, n_s: int,
                kT: float, filter_degree: int = 10, filter_passes: int = 2,
                n_pl: int = 60, **kw) -> CellSpec:
    """A small cell for tests (e.g. grids the oracle can diagonalise densely)."""
    return CellSpec(name, index, a0, reps, n, n_s, kT, filter_degree,
                    filter_passes, n_pl, **kw)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def lattice_positions(spec: CellSpec) -> np.ndarray:
    if spec.basis == "fcc":
        basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    else:
        basis = np.zeros((1, 3))
    r = np.arange(spec.reps)
    cubes = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    pos = (cubes[:, None, :] + basis[None, :, :]).reshape(-1, 3) * spec.a0
    return pos.astype(np.float64)


def atom_positions(spec: CellSpec, snapshot: Optional[int] = None) -> np.ndarray:
    """Lattice sites plus seeded jitter, wrapped into [0, a)."""
    seed = 1000 + spec.index if snapshot is None else 4000 + snapshot
    rng = _rng(seed)
    pos = lattice_positions(spec)
    if spec.jitter == "uniform":
        pos = pos + rng.uniform(-spec.jitter_amp, spec.jitter_amp, pos.shape)
    elif spec.jitter == "normal":
        pos = pos + rng.normal(0.0, spec.jitter_amp, pos.shape)
    return np.mod(pos, spec.a) if spec.cubic else np.mod(pos, np.asarray(spec.cell))


# ----------------------------------------------------------------------------
# periodic one-dimensional factors
# ----------------------------------------------------------------------------

def _wrapped_disp(x: np.ndarray, r0: float, a: float) -> np.ndarray:
    d = x - r0
    return d - a * np.round(d / a)


def _periodic_gauss_1d(x: np.ndarray, r0: float, a: float, w2: float,
                       moment: int = 0) -> np.ndarray:
    """sum_n d^moment exp(-d^2 / w2), d = x - r0 - n a, over all relevant images."""
    d0 = _wrapped_disp(x, r0, a)
    reach = math.sqrt(w2 * 45.0)  # exp(-45) ~ 3e-20
    m = int(math.ceil(reach / a)) + 1
    out = np.zeros_like(x)
    for img in range(-m, m + 1):
        d = d0 - img * a
        out += (d ** moment) * np.exp(-d * d / w2)
    return out


def _gvectors(n: int, a: float):
    g = 2.0 * np.pi * np.fft.fftfreq(n, d=a / n)
    return g


# ----------------------------------------------------------------------------
# local potential
# ----------------------------------------------------------------------------

def _erf_part_fine(spec: CellSpec, pos: np.ndarray) -> np.ndarray:
    """Periodic erf potential sampled on a grid twice as fine, then sub-sampled.

    The reciprocal-space sum is truncated at the fine grid's Nyquist frequency
    (2 pi / h), where exp(-G^2 rc^2 / 4) < 1e-27: the sum is converged.
    """
    nfx, nfy, nfz = (2 * m for m in spec.shape)
    lx, ly, lz = spec.cell
    omega = spec.volume
    g1x, g1y, g1z = _gvectors(nfx, lx), _gvectors(nfy, ly), _gvectors(nfz, lz)
    gz, gy, gx = np.meshgrid(g1z, g1y, g1x, indexing="ij")
    g2 = gx * gx + gy * gy + gz * gz
    with np.errstate(divide="ignore", invalid="ignore"):
        base = -4.0 * np.pi * Z_VALENCE / omega * np.exp(-g2 * RC_LOC ** 2 / 4.0) / g2
    base[0, 0, 0] = 0.0
    # structure factor S(G) = sum_J exp(-i G.R_J), separable per axis
    ex = np.exp(-1j * np.outer(pos[:, 0], g1x))  # (J, nfx)
    ey = np.exp(-1j * np.outer(pos[:, 1], g1y))
    ez = np.exp(-1j * np.outer(pos[:, 2], g1z))
    pyx = (ey[:, :, None] * ex[:, None, :]).reshape(len(pos), -1)
    s = (ez.T @ pyx).reshape(nfz, nfy, nfx)
    vf = np.real(np.fft.ifftn(base * s)) * (nfx * nfy * nfz)
    return vf[::2, ::2, ::2]


def _axis_points(spec: CellSpec, k: int) -> np.ndarray:
    """Coordinates of the grid points along axis k."""
    if spec.cubic:
        return np.arange(spec.n) * spec.h
    return np.arange(spec.shape[k]) * spec.spacing[k]


def _core_part(spec: CellSpec, pos: np.ndarray) -> np.ndarray:
    nx, ny, nz = spec.shape
    cell = spec.cell
    gx = np.stack([_periodic_gauss_1d(_axis_points(spec, 0), p[0], cell[0], CORE_W2) for p in pos])
    gy = np.stack([_periodic_gauss_1d(_axis_points(spec, 1), p[1], cell[1], CORE_W2) for p in pos])
    gz = np.stack([_periodic_gauss_1d(_axis_points(spec, 2), p[2], cell[2], CORE_W2) for p in pos])
    pyx = (gy[:, :, None] * gx[:, None, :]).reshape(len(pos), -1)
    return -CORE_AMP * (gz.T @ pyx).reshape(nz, ny, nx)


def local_potential(spec: CellSpec, pos: np.ndarray) -> np.ndarray:
    return (_erf_part_fine(spec, pos) + _core_part(spec, pos)).reshape(-1)


def smoothed_noise(spec: CellSpec) -> np.ndarray:
    nx, ny, nz = spec.shape
    if not spec.noise:
        return np.zeros(spec.n_grid)
    rng = _rng(2000 + spec.index)
    w = NOISE_AMP * rng.standard_normal((nz, ny, nx))
    lx, ly, lz = spec.cell
    gz, gy, gx = np.meshgrid(_gvectors(nz, lz), _gvectors(ny, ly), _gvectors(nx, lx),
                             indexing="ij")
    filt = np.exp(-(gx * gx + gy * gy + gz * gz) * NOISE_SIGMA ** 2 / 2.0)
    return np.real(np.fft.ifftn(np.fft.fftn(w) * filt)).reshape(-1)


def local_potential_gradients(spec: CellSpec, pos: np.ndarray) -> np.ndarray:
    """(N_atoms, 3, N_grid): grad_x of atom J's local potential v(x - R_J).

    Used for the local Hellmann-Feynman force h^3 sum_x rho(x) grad v_J(x) of the
    fixed-potential workloads (the smoothed noise does not depend on R).
    """
    nfx, nfy, nfz = (2 * m for m in spec.shape)
    cell = spec.cell
    omega = spec.volume
    g1x, g1y, g1z = _gvectors(nfx, cell[0]), _gvectors(nfy, cell[1]), _gvectors(nfz, cell[2])
    gz, gy, gx = np.meshgrid(g1z, g1y, g1x, indexing="ij")
    g2 = gx * gx + gy * gy + gz * gz
    with np.errstate(divide="ignore", invalid="ignore"):
        base = -4.0 * np.pi * Z_VALENCE / omega * np.exp(-g2 * RC_LOC ** 2 / 4.0) / g2
    base[0, 0, 0] = 0.0
    out = np.empty((len(pos), 3, spec.n_grid))
    for j, p in enumerate(pos):
        ph = (np.exp(-1j * g1z * p[2])[:, None, None] * np.exp(-1j * g1y * p[1])[None, :, None]
              * np.exp(-1j * g1x * p[0])[None, None, :])
        vg = base * ph
        for ax, gcomp in enumerate((gx, gy, gz)):
            f = np.real(np.fft.ifftn(1j * gcomp * vg)) * (nfx * nfy * nfz)
            out[j, ax] = f[::2, ::2, ::2].reshape(-1)
        # core part: -1.5 prod_alpha G_alpha, derivative of one factor
        gax = [_periodic_gauss_1d(_axis_points(spec, k), p[k], cell[k], CORE_W2)
               for k in range(3)]
        dax = [-2.0 / CORE_W2 * _periodic_gauss_1d(_axis_points(spec, k), p[k], cell[k], CORE_W2,
                                                   moment=1)
               for k in range(3)]
        fx = [gax[0], gax[1], gax[2]]
        for ax in range(3):
            f = list(fx)
            f[ax] = dax[ax]
            core = -CORE_AMP * (f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :])
            out[j, ax] += core.reshape(-1)
    return out


# ----------------------------------------------------------------------------
# projectors
# ----------------------------------------------------------------------------

def _norm_l(l: int, rc: float) -> float:
    a0 = (2.0 / (np.pi * rc * rc)) ** 0.75
    return a0 if l == 0 else a0 * 2.0 / rc


def projector_cutoff(rc: float) -> float:
    return rc * math.sqrt(math.log(1.0 / PROJ_CUTOFF_REL))


def projector_tables(spec: CellSpec, pos: np.ndarray) -> Dict[str, np.ndarray]:
    """CSR tables of the periodically extended projectors.

    Projector p has grid indices indices[offsets[p]:offsets[p+1]] (sorted,
    unique) and values values[...] (chi~_p at those points, 1/bohr^{3/2}).
    Ordering: atom-major; per atom l=0, then l=1 x, y, z.  moments[b][...]
    holds the first moments sum over images of chi_p(x - R - L) (x - R - L)_b
    at the same points (b = x, y, z).
    """
    nx, ny, nz = spec.shape
    hv = np.array([spec.h] * 3) if spec.cubic else np.array(spec.spacing)
    offsets = [0]
    idx_list, val_list, mom_list = [], [], []
    gamma, atom, ell, mm = [], [], [], []
    for j, p in enumerate(pos):
        for (l, rc, gam) in PROJ_CHANNELS:
            rcut = projector_cutoff(rc)
            lo = np.ceil((p - rcut) / hv).astype(int)
            hi = np.floor((p + rcut) / hv).astype(int)
            ix = np.arange(lo[0], hi[0] + 1)
            iy = np.arange(lo[1], hi[1] + 1)
            iz = np.arange(lo[2], hi[2] + 1)
            dz, dy, dx = np.meshgrid(iz * hv[2] - p[2], iy * hv[1] - p[1], ix * hv[0] - p[0],
                                     indexing="ij")
            r2 = dx * dx + dy * dy + dz * dz
            inside = r2 <= rcut * rcut
            wz, wy, wx = np.meshgrid(np.mod(iz, nz), np.mod(iy, ny), np.mod(ix, nx), indexing="ij")
            flat = (wx + nx * (wy + ny * wz))[inside]
            gau = _norm_l(l, rc) * np.exp(-r2[inside] / (rc * rc))
            if l == 0:
                funcs = [(0, gau)]
            else:
                funcs = [(m, gau * d[inside]) for m, d in ((0, dx), (1, dy), (2, dz))]
            uniq, inv = np.unique(flat, return_inverse=True)
            disp = (dx[inside], dy[inside], dz[inside])
            for m, v in funcs:
                vals = np.bincount(inv, weights=v, minlength=len(uniq))
                idx_list.append(uniq.astype(np.int32))
                val_list.append(vals)
                mom_list.append(np.stack([np.bincount(inv, weights=v * d, minlength=len(uniq))
                                          for d in disp]))
                offsets.append(offsets[-1] + len(uniq))
                gamma.append(gam)
                atom.append(j)
                ell.append(l)
                mm.append(m)
    return {
        "offsets": np.asarray(offsets, dtype=np.int64),
        "indices": np.concatenate(idx_list).astype(np.int32),
        "values": np.concatenate(val_list).astype(np.float64),
        "moments": np.concatenate(mom_list, axis=1).astype(np.float64),
        "gamma": np.asarray(gamma, dtype=np.float64),
        "atom": np.asarray(atom, dtype=np.int32),
        "l": np.asarray(ell, dtype=np.int32),
        "m": np.asarray(mm, dtype=np.int32),
    }


# ----------------------------------------------------------------------------
# problem bundle
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    spec: CellSpec
    positions: np.ndarray
    veff: np.ndarray
    proj: Dict[str, np.ndarray]
    x0: np.ndarray                       # (N_s, N_grid) start block
    _gradv: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def n(self) -> int:
        return self.spec.n

    @property
    def h(self) -> float:
        return self.spec.h

    @property
    def fd_n(self):
        """Points per axis for the FD operators: n on a cubic grid, else (nx, ny, nz)."""
        return self.spec.n if self.spec.cubic else self.spec.shape

    @property
    def fd_h(self):
        """Spacing per axis for the FD operators: h on a cubic grid, else (hx, hy, hz)."""
        return self.spec.h if self.spec.cubic else self.spec.spacing

    @property
    def n_grid(self) -> int:
        return self.spec.n_grid

    @property
    def n_s(self) -> int:
        return self.x0.shape[0]

    @property
    def n_e(self) -> float:
        return self.spec.n_e

    @property
    def n_proj(self) -> int:
        return len(self.proj["gamma"])

    @property
    def gradv(self) -> np.ndarray:
        if self._gradv is None:
            self._gradv = local_potential_gradients(self.spec, self.positions)
        return self._gradv


def start_block(spec: CellSpec, n_s: Optional[int] = None) -> np.ndarray:
    rng = _rng(3000 + spec.index)
    ns = spec.n_s if n_s is None else n_s
    return rng.standard_normal((ns, spec.n_grid))


def make_problem(spec: CellSpec, positions: Optional[np.ndarray] = None,
                 snapshot: Optional[int] = None, with_block: bool = True) -> Problem:
    if positions is None:
        pos = atom_positions(spec, snapshot)
    else:
        pos = np.mod(positions, spec.a if spec.cubic else np.asarray(spec.cell))
    veff = local_potential(spec, pos) + smoothed_noise(spec)
    proj = projector_tables(spec, pos)
    x0 = start_block(spec) if with_block else np.zeros((0, spec.n_grid))
    return Problem(spec, pos, veff, proj, x0)
