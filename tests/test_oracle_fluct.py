"""Pins of the oracle of thermally fluctuating grains (CPU only).

Nothing in the paper prints a distribution for any grain, so the oracle is
pinned to what the method and the mathematics fix:
  * the steady state of the full transition matrix, solved as a dense linear
    system on tiny inputs, with the matrix built here independently;
  * the closed form of a two-level grain;
  * normalisation, non-negativity, the zero field and non-finite fields;
  * energy balance: the power radiated over the distribution equals the
    power the discretised heating deposits, and equals Eq. 6's heating when
    the top level is out of reach;
  * the SED energy identity of the averaged emission;
  * the large-grain limit: a grain whose heat capacity dwarfs every photon
    sits at the equilibrium temperature of Eq. 7.
"""
import math

import numpy as np
import pytest

import oracle
import synth

H_PLANCK = 6.62607015e-34
C_LIGHT = 299792458.0


def _field(grid, n_cells, seed):
    """J[C, NL] in float64, the generator's field on the host."""
    import torch
    p = synth.cell_params(n_cells, seed)
    return synth.radiation_field(p, grid.lam, device="cpu").double().numpy()


def _rates(grid, J_row, s):
    eps = H_PLANCK * C_LIGHT / grid.lam
    return J_row * grid.c_abs[s] * grid.dlam / eps, eps


def _power(grid, s, T):
    return oracle.grain_power(grid.lam, grid.dlam, grid.c_abs[s], T)


def _dense_steady_state(grid, J_row, s, lev_T, lev_E):
    """The transition matrix of one pair, written out level pair by level
    pair, and its null vector with sum 1 from a dense least-squares solve."""
    M = lev_E.shape[0]
    R, eps = _rates(grid, J_row, s)
    A = np.zeros((M, M))
    for i in range(M - 1):
        for l in range(grid.n_lambda):
            e = lev_E[i] + eps[l]
            if e >= lev_E[-1]:
                A[M - 1, i] += R[l]
                continue
            f = int(np.searchsorted(lev_E, e, side="right") - 1)
            w = (e - lev_E[f]) / (lev_E[f + 1] - lev_E[f])
            if f > i:
                A[f, i] += (1 - w) * R[l]
            A[f + 1, i] += w * R[l]
    for j in range(1, M):
        A[j - 1, j] = _power(grid, s, lev_T[j]) / (lev_E[j] - lev_E[j - 1])
    Q = A - np.diag(A.sum(axis=0))  # dP/dt = Q P
    sysm = np.vstack([Q, np.ones((1, M))])
    rhs = np.zeros(M + 1)
    rhs[-1] = 1.0
    # scale the rows so that the solve sees comparable magnitudes
    scale = np.maximum(np.abs(sysm).max(axis=1), 1e-300)
    P, *_ = np.linalg.lstsq(sysm / scale[:, None], rhs / scale, rcond=None)
    return P


@pytest.fixture(scope="module")
def small():
    grid = synth.make_species_grid(24, [2], 3)
    lev_T, lev_E = synth.fluct_levels(grid, 9, t_lo=3.0, t_hi=1500.0)
    J = _field(grid, 4, 31)
    return grid, lev_T, lev_E, J


def test_recursion_equals_dense_solve(small):
    """The level-by-level flux balance is the exact steady state of the full
    matrix (its null vector), checked on every pair of a tiny problem."""
    grid, lev_T, lev_E, J = small
    P = oracle.fluct_distribution(J, grid, lev_T, lev_E)
    for c in range(J.shape[0]):
        for s in range(grid.n_grains):
            Pd = _dense_steady_state(grid, J[c], s, lev_T[s], lev_E[s])
            # a dense solve resolves each probability to about 1e-16 of the
            # largest (absolute), the recursion to relative FP64 rounding
            assert np.allclose(P[c, s], Pd, rtol=1e-9, atol=1e-14), (c, s)


def test_two_level_closed_form():
    """Two levels: P1 / P0 = (upward rate) / (cooling rate), with every photon
    reaching level 1 at least in part (fraction min(1, eps / E1))."""
    grid = synth.make_species_grid(40, [0], 2)
    J = _field(grid, 3, 7)
    for s in range(grid.n_grains):
        for E1, T1 in ((1e-19, 30.0), (5e-18, 400.0)):
            lev_T = np.array([[0.0, T1]] * grid.n_grains)
            lev_E = np.array([[0.0, E1]] * grid.n_grains)
            P = oracle.fluct_distribution(J, grid, lev_T, lev_E)
            for c in range(J.shape[0]):
                R, eps = _rates(grid, J[c], s)
                up = np.sum(R * np.minimum(1.0, eps / E1))
                down = _power(grid, s, T1) / E1
                assert P[c, s, 1] / P[c, s, 0] == pytest.approx(up / down, rel=1e-12)
                assert P[c, s].sum() == pytest.approx(1.0, rel=1e-15)


def test_normalised_nonnegative_and_special_fields(small):
    grid, lev_T, lev_E, J = small
    J = J.copy()
    J[1] = 0.0
    J[2, 5] = np.nan
    J[3, 7] = -1.0
    P = oracle.fluct_distribution(J, grid, lev_T, lev_E)
    assert np.allclose(P[0].sum(axis=1), 1.0, rtol=1e-14) and np.all(P[0] >= 0)
    # no field: the grain stays in the ground level
    assert np.all(P[1, :, 0] == 1.0) and np.all(P[1, :, 1:] == 0.0)
    # a NaN or negative intensity makes the whole distribution NaN
    assert np.all(np.isnan(P[2])) and np.all(np.isnan(P[3]))


def test_energy_balance():
    """Steady state conserves energy: the power radiated over the
    distribution equals the power the discretised heating deposits
    (photons above the top level stop there), and equals Eq. 6's heating
    when the top level is out of reach."""
    grid = synth.make_species_grid(60, [2], 4)
    J = _field(grid, 3, 11)
    lev_T, lev_E = synth.fluct_levels(grid, 48, t_lo=3.0, t_hi=2500.0)
    P = oracle.fluct_distribution(J, grid, lev_T, lev_E)
    H = oracle.heating(J, grid.c_abs, grid.dlam)
    for c in range(J.shape[0]):
        for s in range(grid.n_grains):
            radiated = sum(P[c, s, j] * _power(grid, s, lev_T[s, j]) for j in range(1, 48))
            R, eps = _rates(grid, J[c], s)
            deposited = sum(P[c, s, i] * np.sum(R * np.minimum(eps, lev_E[s, -1] - lev_E[s, i]))
                            for i in range(48))
            assert radiated == pytest.approx(deposited, rel=1e-10), (c, s)
            if P[c, s, -1] < 1e-30:
                assert radiated == pytest.approx(H[c, s], rel=1e-10), (c, s)


def test_sed_energy_identity(small):
    """sum_l L dlam = m sum_s w_s sum_j P_j P(T_j): the averaged emission
    carries exactly the radiated power of the distribution."""
    grid, lev_T, lev_E, J = small
    P = oracle.fluct_distribution(J, grid, lev_T, lev_E)
    m = np.array([0.5, 1.0, 2.0, 3.0])
    L = oracle.fluct_emission(P, grid, lev_T, m)
    for c in range(J.shape[0]):
        rhs = m[c] * sum(grid.weight[s] * sum(P[c, s, j] * _power(grid, s, lev_T[s, j])
                                              for j in range(lev_T.shape[1]))
                         for s in range(grid.n_grains))
        assert np.sum(L[c] * grid.dlam) == pytest.approx(rhs, rel=1e-12)
    # one grain in a cell of unit mass: the averaged Eq. 10 written out
    l = 7
    s = 1
    direct = grid.weight[s] * grid.c_abs[s, l] * sum(
        P[0, s, j] * oracle.planck(grid.lam[l], lev_T[s, j]) for j in range(lev_T.shape[1]))
    L1 = oracle.fluct_emission(P[:1, s:s + 1], synth.Grid(grid.lam, grid.dlam,
                                                          grid.c_abs[s:s + 1],
                                                          grid.weight[s:s + 1],
                                                          grid.size[s:s + 1],
                                                          grid.species[s:s + 1]),
                               lev_T[s:s + 1])
    assert L1[0, l] == pytest.approx(direct, rel=1e-13)


def test_large_grain_limit():
    """A grain whose heat capacity dwarfs every photon energy (a = 1 um,
    4.7e11 atoms of the Debye stand-in) on level grids around its Eq. 7
    temperature: the distribution collapses onto that temperature as the
    levels refine (mean off by about a tenth of a level spacing, shrinking in
    step with it; width set by the spacing, shrinking as its square root)."""
    grid = synth.make_species_grid(120, [0], 40)
    s = grid.n_grains - 1
    one = synth.Grid(grid.lam, grid.dlam, grid.c_abs[s:s + 1], grid.weight[s:s + 1],
                     grid.size[s:s + 1], grid.species[s:s + 1])
    J = _field(grid, 1, 3)
    H = oracle.heating(J, one.c_abs, one.dlam)
    Teq = oracle.temperature(H, one.lam, one.dlam, one.c_abs, one.size)[0, 0]
    res = []
    for n_levels in (129, 513):
        T1 = np.concatenate([[0.0], np.geomspace(0.8 * Teq, 1.25 * Teq, n_levels - 1)])
        E1 = synth.debye_enthalpy(T1, float(synth.grain_atoms(one.size[0])))
        P = oracle.fluct_distribution(J, one, T1[None, :], E1[None, :])[0, 0]
        mean = float(np.sum(P * T1))
        std = math.sqrt(float(np.sum(P * (T1 - mean) ** 2)))
        spacing = math.log(1.25 / 0.8) / (n_levels - 2)
        assert abs(mean / Teq - 1.0) < 0.5 * spacing
        assert std / Teq < 8.0 * math.sqrt(spacing)
        assert P[0] < 1e-12  # the ground level is emptied
        res.append((abs(mean / Teq - 1.0), std / Teq))
    assert res[1][0] < res[0][0] / 3.5 and res[1][1] < res[0][1] / 1.8


def test_small_grains_fluctuate():
    """The 0.35 nm grain (20 atoms of the Debye stand-in) in a typical field
    spends most of its time cold and is heated in spikes: a wide
    distribution, unlike the equilibrium of Eq. 7."""
    grid = synth.make_species_grid(120, [2], 4)
    lev_T, lev_E = synth.fluct_levels(grid, 64)
    J = _field(grid, 8, 13)
    P = oracle.fluct_distribution(J, grid, lev_T, lev_E)
    Tmean = np.sum(P[:, 0] * lev_T[0], axis=1)
    Tstd = np.sqrt(np.sum(P[:, 0] * (lev_T[0] - Tmean[:, None]) ** 2, axis=1))
    assert np.all(Tstd / Tmean > 0.5)
