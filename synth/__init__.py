"""Seeded synthetic inputs shaped like the paper's dust-emission workloads.

This module is shared by the CPU oracle's tests, the GPU path's tests and the
benchmark.  It only *describes inputs*: wavelength grids with their quadrature
weights, grain sets (absorption cross-sections, size-distribution weights,
sizes), per-cell radiation-field parameters and the radiation field itself.
It performs none of the method's steps (heating sum, temperature solve,
emission sum).

The paper's own inputs (a Sunrise Sbc snapshot, Laor & Draine graphite
cross-sections with 81 sizes, the Draine & Li Milky-Way size distribution and
a 968-point wavelength grid from the Lyman limit to 1000 um; Section 5) are not
available, so every array here is a synthetic stand-in of the same kind:

* wavelengths: log-spaced, inclusive endpoints, 0.09-1000 um by default;
* quadrature weights: trapezoid rule in ln(lambda), i.e.
  dlam_l = lam_l * dln(lambda), halved at both ends (the paper leaves the
  weights of its sums, Eqs. 6-8, to the caller);
* grains: C_abs = pi a^2 (1 - exp(-kappa (2 pi a / lambda)^beta)) per species,
  sizes log-spaced, MRN weights n(a) ~ a^-3.5 da normalised to unit total
  grain volume per species (the paper's n_s, Eq. 10, is "grains per unit dust
  mass"; the normalisation is a pure scale);
* radiation field (mean intensity, W m^-2 m^-1 sr^-1): a sum of 1-3 diluted
  blackbodies W B_lambda(T*) with T* ~ U(3000, 30000) K and
  log10 W ~ U(-16, -10), attenuated by exp(-tau_V (lambda / 0.55 um)^-1) with
  tau_V ~ U(0, 5);
* dust mass per cell (the paper's m_d;c): log-uniform over 0.1-10 (arbitrary
  mass unit).

Units are SI throughout (metres, m^2, W).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

UM = 1.0e-6  # one micrometre in metres

# Species of the synthetic grain model: (beta, kappa, a_min_um, a_max_um).
SPECIES = (
    (1.5, 1.0, 0.001, 1.0),     # "species 1"
    (2.0, 0.6, 0.001, 1.0),     # "species 2"
    (1.0, 2.0, 0.00035, 0.01),  # "species 3": very small grains
)

# Exact SI constants (2019 redefinition) used only to synthesise the input
# radiation field.
_H = 6.62607015e-34
_C = 299792458.0
_K = 1.380649e-23


@dataclasses.dataclass
class Grid:
    """Per-grid tables a caller hands to the dust library (host, float64)."""
    lam: np.ndarray      # [NL] wavelengths (m), strictly increasing
    dlam: np.ndarray     # [NL] quadrature weights (m)
    c_abs: np.ndarray    # [S, NL] absorption cross-sections (m^2)
    weight: np.ndarray   # [S] grains per unit dust amount (n_s)
    size: np.ndarray     # [S] grain radius (m)
    species: np.ndarray  # [S] species index of each grain (0-based)

    @property
    def n_lambda(self) -> int:
        return int(self.lam.shape[0])

    @property
    def n_grains(self) -> int:
        return int(self.c_abs.shape[0])


@dataclasses.dataclass
class CellParams:
    """Per-cell radiation-field and dust-mass parameters (host arrays)."""
    n_bb: np.ndarray    # [C] number of diluted blackbodies (1..3)
    tau_v: np.ndarray   # [C] V-band optical depth
    tstar: np.ndarray   # [C, 3] blackbody temperatures (K); unused beyond n_bb
    logw: np.ndarray    # [C, 3] log10 dilution factors
    m_dust: np.ndarray  # [C] dust mass (arbitrary unit)

    @property
    def n_cells(self) -> int:
        return int(self.n_bb.shape[0])

    def subset(self, idx) -> "CellParams":
        return CellParams(self.n_bb[idx], self.tau_v[idx], self.tstar[idx],
                          self.logw[idx], self.m_dust[idx])


def wavelength_grid(n: int, lo_um: float = 0.09, hi_um: float = 1000.0):
    """Log-spaced wavelengths (inclusive endpoints) and ln-trapezoid weights."""
    if n < 2:
        raise ValueError("need at least two wavelengths")
    lam = np.geomspace(lo_um * UM, hi_um * UM, n)
    dln = math.log(hi_um / lo_um) / (n - 1)
    dlam = lam * dln
    dlam[0] *= 0.5
    dlam[-1] *= 0.5
    return lam, dlam


def species_grains(lam: np.ndarray, beta: float, kappa: float,
                   a_min_um: float, a_max_um: float, n_sizes: int):
    """Cross-sections, MRN weights and sizes for one species."""
    a = np.geomspace(a_min_um * UM, a_max_um * UM, n_sizes)
    x = 2.0 * math.pi * a[:, None] / lam[None, :]
    c_abs = math.pi * a[:, None] ** 2 * (-np.expm1(-kappa * x ** beta))
    if n_sizes > 1:
        r = a[1] / a[0]
        da = a * (math.sqrt(r) - 1.0 / math.sqrt(r))
    else:
        da = a.copy()
    w = a ** -3.5 * da
    w = w / np.sum(w * (4.0 * math.pi / 3.0) * a ** 3)
    return c_abs, w, a


def make_grid(n_lambda: int, n_species: int, n_sizes, lo_um: float = 0.09,
              hi_um: float = 1000.0) -> Grid:
    """A grid with the first ``n_species`` species, ``n_sizes`` sizes each."""
    lam, dlam = wavelength_grid(n_lambda, lo_um, hi_um)
    if np.isscalar(n_sizes):
        n_sizes = [int(n_sizes)] * n_species
    cs, ws, as_, sp = [], [], [], []
    for i in range(n_species):
        beta, kappa, amin, amax = SPECIES[i]
        c, w, a = species_grains(lam, beta, kappa, amin, amax, n_sizes[i])
        cs.append(c)
        ws.append(w)
        as_.append(a)
        sp.append(np.full(n_sizes[i], i, dtype=np.int32))
    return Grid(lam, dlam, np.concatenate(cs), np.concatenate(ws),
                np.concatenate(as_), np.concatenate(sp))


def cell_params(n_cells: int, seed: int) -> CellParams:
    """Per-cell parameters, drawn in a fixed order from one seeded stream."""
    rng = np.random.default_rng(seed)
    n_bb = rng.integers(1, 4, size=n_cells)
    tau_v = rng.uniform(0.0, 5.0, size=n_cells)
    tstar = rng.uniform(3000.0, 30000.0, size=(n_cells, 3))
    logw = rng.uniform(-16.0, -10.0, size=(n_cells, 3))
    m_dust = 10.0 ** rng.uniform(-1.0, 1.0, size=n_cells)
    return CellParams(n_bb, tau_v, tstar, logw, m_dust)


def _blackbody_field(lam, tstar, w):
    """W * B_lambda(T*) for broadcastable torch tensors (float64)."""
    import torch
    c1 = 2.0 * _H * _C * _C
    c2 = _H * _C / _K
    return w * c1 / lam ** 5 / torch.expm1(c2 / (lam * tstar))


def radiation_field(params: CellParams, lam: np.ndarray, device="cpu",
                    chunk: int = 65536, out=None):
    """Mean intensity J[C, NL] as a float32 torch tensor on ``device``.

    Synthesised in float64 (chunk by chunk) and rounded once to float32.
    ``out`` may be a preallocated float32 tensor with row stride >= NL.
    """
    import torch
    C = params.n_cells
    NL = lam.shape[0]
    if out is None:
        out = torch.empty((C, NL), dtype=torch.float32, device=device)
    lam_t = torch.as_tensor(lam, dtype=torch.float64, device=device)[None, :]
    for c0 in range(0, C, chunk):
        c1 = min(C, c0 + chunk)
        sl = slice(c0, c1)
        n_bb = torch.as_tensor(params.n_bb[sl], device=device)
        tau = torch.as_tensor(params.tau_v[sl], dtype=torch.float64, device=device)
        ts = torch.as_tensor(params.tstar[sl], dtype=torch.float64, device=device)
        lw = torch.as_tensor(params.logw[sl], dtype=torch.float64, device=device)
        acc = torch.zeros((c1 - c0, NL), dtype=torch.float64, device=device)
        for i in range(3):
            on = (n_bb > i).to(torch.float64)[:, None]
            w = (10.0 ** lw[:, i])[:, None] * on
            acc += _blackbody_field(lam_t, ts[:, i:i + 1], w)
        acc *= torch.exp(-tau[:, None] * (0.55 * UM) / lam_t)
        out[c0:c1, :NL] = acc.to(torch.float32)
    return out


# ---------------------------------------------------------------------------
# Named workloads.  Each is identified by what it is and its sizes.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    n_cells: int
    n_lambda: int
    n_species: int
    n_sizes: int
    seed: int
    mode: str  # "plain" or "mixed" (the form the workload is quoted for)

    @property
    def n_grains(self) -> int:
        return self.n_species * self.n_sizes

    def grid(self) -> Grid:
        return make_grid(self.n_lambda, self.n_species, self.n_sizes)

    def cells(self) -> CellParams:
        return cell_params(self.n_cells, self.seed)


WORKLOADS = {
    # small full-compare case: 1024 cells x 120 wavelengths x 2 species x 10 sizes
    "small-1024x120x20": Workload("small-1024x120x20", 1024, 120, 2, 10, 0, "plain"),
    # 262144 cells x 250 wavelengths x 2 species x 40 sizes
    "plain-262144x250x80": Workload("plain-262144x250x80", 262144, 250, 2, 40, 1, "plain"),
    # 1048576 cells x 500 wavelengths x 2 species x 64 sizes
    "mixed-1048576x500x128": Workload("mixed-1048576x500x128", 1048576, 500, 2, 64, 2, "mixed"),
    # 4194304 cells x 1000 wavelengths x 3 species x 80 sizes (J is 16.8 GB)
    "full-4194304x1000x240": Workload("full-4194304x1000x240", 4194304, 1000, 3, 80, 4, "mixed"),
}


@dataclasses.dataclass
class BatchGridSpec:
    n_cells: int
    n_lambda: int
    n_species: int
    n_sizes: int
    seed: int

    def grid(self) -> Grid:
        return make_grid(self.n_lambda, self.n_species, self.n_sizes)

    def cells(self) -> CellParams:
        return cell_params(self.n_cells, self.seed)


def batch_specs(n_grids: int = 64, seed: int = 3, cells_lo: float = 1e3,
                cells_hi: float = 2e5, scale: float = 1.0) -> List[BatchGridSpec]:
    """Uneven independent grids: log-uniform cell counts, 100-600 wavelengths,
    1-3 species (species 1; 1+2; 1+2+3) with 10-80 sizes each.

    ``scale`` multiplies every cell count (for reduced test sizes)."""
    rng = np.random.default_rng(seed)
    specs = []
    for g in range(n_grids):
        c = int(round(10.0 ** rng.uniform(math.log10(cells_lo), math.log10(cells_hi))))
        nl = int(rng.integers(100, 601))
        ns = int(rng.integers(1, 4))
        nz = int(rng.integers(10, 81))
        specs.append(BatchGridSpec(max(1, int(round(c * scale))), nl, ns, nz,
                                   1000 * seed + g))
    return specs


def extra_heating(grid: Grid, n_cells: int, seed: int) -> np.ndarray:
    """Stand-in for heating that is not absorbed radiation (e.g. collisions
    with energetic electrons): Q[c, s] = eps_c * pi a_s^2 in the units of H
    (W sr^-1), log10 eps_c ~ U(-8, -3), so that Q/H spans several decades
    either side of 1 on the synthetic fields.  Float32, [C, S]."""
    rng = np.random.default_rng(seed)
    eps = 10.0 ** rng.uniform(-8.0, -3.0, size=n_cells)
    area = np.pi * grid.size ** 2
    return (eps[:, None] * area[None, :]).astype(np.float32)


def reheat_coupling(grid: Grid, m_dust: np.ndarray, seed: int) -> np.ndarray:
    """Coupling g[c] of the stand-in for re-propagating a cell's own emission
    between passes of the global iteration: J_next = J0 + g[c] L[c, :].

    With kappa_l = sum_s w_s C[s, l] (cross-section per unit dust mass), the
    power one pass re-absorbs from g L is at most f_c of what the cell emitted
    when g[c] = f_c / (m[c] max_l kappa_l); f_c ~ U(0.1, 0.5) from its own
    seeded stream, so the iteration contracts.  Float64, [C]."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.1, 0.5, size=m_dust.shape[0])
    kappa_max = float((grid.weight[:, None] * grid.c_abs).sum(axis=0).max())
    return f / (np.asarray(m_dust, dtype=np.float64) * kappa_max)


# ---------------------------------------------------------------------------
# Thermally fluctuating grains: enthalpy levels from a heat-capacity model.
#
# The paper's discussion of fluctuating grains needs each grain's heat
# capacity, which is not among its inputs.  Stand-in: a three-dimensional
# Debye solid of carbon atoms (graphite-like density 2240 kg m^-3, 12 u per
# atom) with Debye temperature 420 K; a grain of radius a holds
# N = (4 pi / 3) a^3 rho / m_atom atoms and its enthalpy above the ground
# state at temperature T is
#   E(T) = 9 N k T (T / theta)^3 int_0^{theta/T} x^3 / (e^x - 1) dx.
# Levels: E_0 = 0 at T_0 = 0, then temperatures log-spaced over
# [t_lo, t_hi] and their enthalpies.
# ---------------------------------------------------------------------------

DEBYE_THETA_K = 420.0
GRAIN_DENSITY = 2240.0                     # kg m^-3
ATOM_MASS = 12.0 * 1.66053906660e-27       # kg


def grain_atoms(a_m):
    """Atoms in a grain of radius a (m) of the Debye stand-in."""
    return 4.0 / 3.0 * math.pi * np.asarray(a_m, dtype=np.float64) ** 3 * GRAIN_DENSITY / ATOM_MASS


def debye_enthalpy(T, n_atoms, theta=DEBYE_THETA_K):
    """E(T) of the Debye stand-in (J) for temperatures T (K) >= 0."""
    from scipy.integrate import quad
    T = np.asarray(T, dtype=np.float64)
    out = np.zeros_like(T)
    for idx, t in np.ndenumerate(T):
        if t <= 0.0:
            continue
        y = theta / t
        val, _ = quad(lambda x: x ** 3 / math.expm1(x) if x > 0 else 0.0, 0.0, y,
                      epsabs=0.0, epsrel=1e-13, limit=200)
        out[idx] = 9.0 * n_atoms * _K * t * (t / theta) ** 3 * val
    return out


def fluct_levels(grid: Grid, n_levels: int = 64, t_lo: float = 2.0, t_hi: float = 2500.0):
    """Level temperatures and enthalpies [S, n_levels] of every grain of the
    grid: level 0 the ground state (T = 0, E = 0), levels 1 .. n - 1 at
    temperatures log-spaced over [t_lo, t_hi]."""
    S = grid.n_grains
    T1 = np.concatenate([[0.0], np.geomspace(t_lo, t_hi, n_levels - 1)])
    lev_T = np.repeat(T1[None, :], S, axis=0)
    lev_E = np.empty_like(lev_T)
    for s in range(S):
        lev_E[s] = debye_enthalpy(T1, float(grain_atoms(grid.size[s])))
    return lev_T, lev_E


def make_species_grid(n_lambda: int, species: Sequence[int], n_sizes: int,
                      lo_um: float = 0.09, hi_um: float = 1000.0) -> Grid:
    """A grid with the listed species (0-based indices), n_sizes sizes each."""
    lam, dlam = wavelength_grid(n_lambda, lo_um, hi_um)
    cs, ws, as_, sp = [], [], [], []
    for i in species:
        beta, kappa, amin, amax = SPECIES[i]
        c, w, a = species_grains(lam, beta, kappa, amin, amax, n_sizes)
        cs.append(c)
        ws.append(w)
        as_.append(a)
        sp.append(np.full(n_sizes, i, dtype=np.int32))
    return Grid(lam, dlam, np.concatenate(cs), np.concatenate(ws), np.concatenate(as_),
                np.concatenate(sp))


@dataclasses.dataclass
class FluctWorkload:
    """Fluctuating very small grains: species 3 (0.35-10 nm), n_sizes sizes,
    n_levels enthalpy levels from the Debye stand-in over 2-2500 K."""
    name: str
    n_cells: int
    n_lambda: int
    n_sizes: int
    n_levels: int
    seed: int

    def grid(self) -> Grid:
        return make_species_grid(self.n_lambda, [2], self.n_sizes)

    def levels(self, grid: Grid):
        return fluct_levels(grid, self.n_levels)

    def cells(self) -> CellParams:
        return cell_params(self.n_cells, self.seed)


FLUCT_WORKLOADS = {
    # 65536 cells x 250 wavelengths x 16 very small grains x 64 levels
    "fluct-65536x250x16x64": FluctWorkload("fluct-65536x250x16x64", 65536, 250, 16, 64, 5),
}
