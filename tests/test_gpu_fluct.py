"""GPU parity of thermally fluctuating grains: dust_fluct_solve_P and
dust_fluct_emit_sed through the C-ABI against the FP64 oracle (fluct_ref.c)
on the same seeded inputs, element by element.

Tolerances, from the arithmetic:
  * P: both sides solve the same flux balance in FP64; the GPU forms each
    upward rate from prefix sums over the wavelengths (differences of sums
    instead of sums, relative rounding a few 1e-16 times the ratio of the
    whole sum to the part), the recursion carries that through at most 255
    levels, and P leaves in FP32 (6e-8).  Bound: 1e-6 relative on every
    probability the oracle puts at or above 1e-30, and below 1e-29 where it
    puts less (FP32 keeps no relative precision near its underflow).
  * L: the averaged emission is an FP32 contraction over S M terms
    (products exact, sums of positive terms in FP32: at most S M 2^-24,
    about 1e-4 at S M = 2048; typically far less) from FP32 P and an FP32
    table, measured with the SED error of the equilibrium path (elements at
    or above 1e-6 of the cell's peak): 1e-3, the method's SED target.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import strided_rows
from oracle.compare import sed_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0907_3768_amd as dust  # noqa: E402

P_TOL = 1e-6
P_FLOOR = 1e-30
SED_TOL = 1e-3


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("these tests need an MI355X: torch.cuda.is_available() is False")
    dust.lib()
    return torch.device("cuda:0")


def _check_P(P, P_ref):
    P = np.asarray(P, dtype=np.float64)
    big = P_ref >= P_FLOOR
    rel = np.abs(P[big] - P_ref[big]) / P_ref[big]
    assert rel.max() <= P_TOL, rel.max()
    assert np.all(np.abs(P[~big]) <= 1e-29)
    return float(rel.max())


def _case(dev, n_cells, n_lambda, species, n_sizes, n_levels, seed, t_lo=2.0, t_hi=2500.0,
          ldj_pad=0):
    g = synth.make_species_grid(n_lambda, species, n_sizes)
    lev_T, lev_E = synth.fluct_levels(g, n_levels, t_lo, t_hi)
    p = synth.cell_params(n_cells, seed)
    if ldj_pad:
        buf = torch.full((n_cells, n_lambda + ldj_pad), -7.0, dtype=torch.float32, device=dev)
        synth.radiation_field(p, g.lam, device=dev, out=buf)
        J = buf[:, :n_lambda]
    else:
        J = synth.radiation_field(p, g.lam, device=dev)
    m = torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev)
    return g, lev_T, lev_E, p, J, m


@pytest.mark.parametrize("n_cells,n_lambda,species,n_sizes,n_levels", [
    (256, 120, [2], 8, 64),      # very small grains, one level per lane
    (77, 250, [2], 5, 100),      # two levels per lane, ragged
    (33, 33, [0, 2], 3, 256),    # four levels per lane, larger grains too
    (1, 8, [2], 1, 2),           # a two-level grain, one cell, 8 wavelengths
    (130, 65, [2], 3, 3),
])
def test_distribution_and_emission_match_oracle(dev, n_cells, n_lambda, species, n_sizes,
                                                n_levels):
    say(f"fluct C={n_cells} NL={n_lambda} species={species} sizes={n_sizes} M={n_levels}")
    g, lev_T, lev_E, p, J, m = _case(dev, n_cells, n_lambda, species, n_sizes, n_levels,
                                     900 + n_cells, ldj_pad=3)
    plan = dust.FluctPlan(g, lev_T, lev_E)
    S, M = g.n_grains, n_levels
    Pbuf = torch.full((n_cells, S * M + 5), -2.0, dtype=torch.float32, device=dev)
    Lbuf = torch.full((n_cells, n_lambda + 4), -3.0, dtype=torch.float32, device=dev)
    P, L = Pbuf[:, :S * M], Lbuf[:, :n_lambda]
    cnt = dust.new_counters(dev)
    plan.solve_P(J, P, counters=cnt)
    plan.emit(P, m, L)
    torch.cuda.synchronize()
    assert torch.all(Pbuf[:, S * M:] == -2.0) and torch.all(Lbuf[:, n_lambda:] == -3.0)
    Jh = _host(J).astype(np.float64)
    P_ref = oracle.fluct_distribution(Jh, g, lev_T, lev_E)
    err = _check_P(_host(P).reshape(n_cells, S, M), P_ref)
    L_ref = oracle.fluct_emission(P_ref, g, lev_T, p.m_dust)
    se = sed_errors(_host(L), L_ref, g.dlam)
    say(f"  P max rel {err:.3g}, SED {se}")
    assert se["max"] <= SED_TOL and se["energy_l1"] <= SED_TOL, se
    c = _host(cnt)
    assert c[0] == 0


def test_special_fields_and_counters(dev):
    """No radiation: the ground level.  A NaN or negative intensity: NaN for
    every level of every grain of that cell, counted per pair.  A level grid
    that ends too low for the field: counted as out of table."""
    g, lev_T, lev_E, p, J, m = _case(dev, 16, 120, [2], 4, 32, 41)
    J[3].zero_()
    J[5, 10] = float("nan")
    J[7, 2] = -1.0
    plan = dust.FluctPlan(g, lev_T, lev_E)
    cnt = dust.new_counters(dev)
    P = plan.solve_P(J, counters=cnt)
    L = plan.emit(P, m)
    torch.cuda.synchronize()
    Ph = _host(P).reshape(16, g.n_grains, 32)
    assert np.all(Ph[3, :, 0] == 1.0) and np.all(Ph[3, :, 1:] == 0.0)
    assert np.all(_host(L)[3] == 0.0)
    assert np.all(np.isnan(Ph[5])) and np.all(np.isnan(Ph[7]))
    assert int(_host(cnt)[0]) == 2 * g.n_grains
    keep = [c for c in range(16) if c not in (5, 7)]
    P_ref = oracle.fluct_distribution(_host(J)[keep].astype(np.float64), g, lev_T, lev_E)
    _check_P(Ph[keep], P_ref)
    # a short level grid: 2-30 K for grains that the field heats well above
    lev_T2, lev_E2 = synth.fluct_levels(g, 16, 2.0, 30.0)
    plan2 = dust.FluctPlan(g, lev_T2, lev_E2)
    cnt.zero_()
    P2 = plan2.solve_P(J[:3], counters=cnt)
    torch.cuda.synchronize()
    P2_ref = oracle.fluct_distribution(_host(J[:3]).astype(np.float64), g, lev_T2, lev_E2)
    _check_P(_host(P2).reshape(3, g.n_grains, 16), P2_ref)
    assert int(_host(cnt)[2]) == int(np.sum(P2_ref[:, :, -1] > 1e-6)) > 0


def test_emission_accumulates_and_energy_identity(dev):
    """accumulate adds the averaged emission onto L (here the equilibrium
    SED of the larger grains of the same cells from dust_run_fused); the
    SED carries the radiated power of the distributions:
    sum_l L dlam = m sum_s w_s sum_j P_j P(T_j)."""
    big = synth.make_grid(120, 2, 10)
    g, lev_T, lev_E, p, J, m = _case(dev, 64, 120, [2], 6, 64, 51)
    eq = dust.Plan(big, "mixed")
    T_eq, L = eq.fused(J, m)
    L0 = L.clone()
    fp = dust.FluctPlan(g, lev_T, lev_E)
    P = fp.solve_P(J)
    fp.emit(P, m, L, accumulate=True)
    L_alone = fp.emit(P, m)
    torch.cuda.synchronize()
    assert torch.allclose(L, L0 + L_alone, rtol=1e-6, atol=0)
    Ph = _host(P).reshape(64, g.n_grains, 64).astype(np.float64)
    power = np.array([[oracle.grain_power(g.lam, g.dlam, g.c_abs[s], lev_T[s, j])
                       for j in range(64)] for s in range(g.n_grains)])
    rhs = p.m_dust * np.einsum("csj,sj,s->c", Ph, power, g.weight)
    lhs = (_host(L_alone).astype(np.float64) * g.dlam).sum(axis=1)
    assert np.max(np.abs(lhs / rhs - 1.0)) < 1e-4


def test_fluct_workload_sampled(dev):
    """The fluctuating-grain workload at full size (65536 cells x 250
    wavelengths x 16 very small grains x 64 levels): strided cells against
    the oracle, properties on every output."""
    w = synth.FLUCT_WORKLOADS["fluct-65536x250x16x64"]
    g = w.grid()
    lev_T, lev_E = w.levels(g)
    p = w.cells()
    say("fluct workload: generating J")
    J = synth.radiation_field(p, g.lam, device=dev)
    m = torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev)
    plan = dust.FluctPlan(g, lev_T, lev_E)
    cnt = dust.new_counters(dev)
    P = plan.solve_P(J, counters=cnt)
    L = plan.emit(P, m)
    torch.cuda.synchronize()
    rows = strided_rows(w.n_cells, 64)
    idx = torch.as_tensor(rows, device=dev)
    say("fluct workload: oracle on 64 cells")
    P_ref = oracle.fluct_distribution(_host(J[idx]).astype(np.float64), g, lev_T, lev_E)
    S, M = g.n_grains, w.n_levels
    err = _check_P(_host(P[idx]).reshape(len(rows), S, M), P_ref)
    L_ref = oracle.fluct_emission(P_ref, g, lev_T, p.m_dust[rows])
    se = sed_errors(_host(L[idx]), L_ref, g.dlam)
    say(f"fluct workload: P max rel {err:.3g}, SED {se}")
    assert se["max"] <= SED_TOL and se["energy_l1"] <= SED_TOL
    sums = P.view(w.n_cells, S, M).sum(dim=2)
    assert bool(torch.isfinite(P).all()) and bool((P >= 0).all())
    assert torch.allclose(sums, torch.ones_like(sums), rtol=0, atol=1e-5)
    assert bool(torch.isfinite(L).all())
    assert int(_host(cnt)[0]) == 0


@pytest.mark.parametrize("pad", [0, 2, 1])
def test_emission_load_widths(dev, pad):
    """dust_fluct_emit_sed with P rows of S M + pad floats: float4 loads
    (pad 0, S M a multiple of 4), float2 (pad 2), single floats (pad 1);
    70 cells (a ragged last workgroup of 64), 200 wavelengths (a ragged last
    block of 128) and 5 x 12 grain-levels (a ragged last 32-k chunk)."""
    g, lev_T, lev_E, p, J, m = _case(dev, 70, 200, [2], 5, 12, 77)
    plan = dust.FluctPlan(g, lev_T, lev_E)
    K = g.n_grains * 12
    Pbuf = torch.full((70, K + pad), -2.0, dtype=torch.float32, device=dev)
    P = Pbuf[:, :K]
    plan.solve_P(J, P)
    Lbuf = torch.full((70, 200 + 3), -3.0, dtype=torch.float32, device=dev)
    L = Lbuf[:, :200]
    plan.emit(P, m, L)
    torch.cuda.synchronize()
    assert torch.all(Lbuf[:, 200:] == -3.0)
    P_ref = oracle.fluct_distribution(_host(J).astype(np.float64), g, lev_T, lev_E)
    _check_P(_host(P).reshape(70, g.n_grains, 12), P_ref)
    se = sed_errors(_host(L), oracle.fluct_emission(P_ref, g, lev_T, p.m_dust), g.dlam)
    say(f"fluct emission pad={pad}: SED {se}")
    assert se["max"] <= SED_TOL and se["energy_l1"] <= SED_TOL
