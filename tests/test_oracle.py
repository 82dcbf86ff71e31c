"""Pins of the FP64 oracle against what physics and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms (Stefan-Boltzmann, Wien displacement, grey and power-law grains in a
diluted blackbody field), BLAS, brute-force bisection written here from the
definition of the balance (Section 4, Eq. 7), and invariants (the SED energy
identity that follows from Eqs. 6, 7 and 10; monotonicity in J; invariance
under power-of-two rescaling of the cross-sections).  The Planck function used
on the test side is built from scipy's CODATA constants, independently of the
oracle's C source.
"""
import math

import numpy as np
import pytest
import scipy.constants as sc

import oracle
import synth
from conftest import read_golden

H_, C_, K_ = sc.h, sc.c, sc.k


def planck_indep(lam, T):
    """B_lambda(lam, T) from scipy's constants (test-side, numpy)."""
    lam = np.asarray(lam, dtype=np.float64)
    x = H_ * C_ / (K_ * lam * T)
    with np.errstate(over="ignore"):
        return 2.0 * H_ * C_ ** 2 / lam ** 5 / np.expm1(x)


def wide_grid(n=20000):
    # 1 nm .. 1 m: wide enough that truncation of the Planck integral is
    # below 1e-8 at 3 K and far below at >= 20 K.
    return synth.wavelength_grid(n, 1e-3, 1e6)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ----------------------------------------------------------------- Planck / quadrature

@pytest.mark.parametrize("T", [3.0, 20.0, 100.0, 1000.0, 10000.0])
def test_stefan_boltzmann(T):
    """P3: sum_l dlam B(lam_l, T) = sigma T^4 / pi (pins c1/c2^4 and the weights).

    The grid ends at 1 m; the tail beyond it, from the expansion
    1/(e^x - 1) = 1/x - 1/2 + O(x), is 2 c k T / (3 lam^3) - h c^2 / (4 lam^4)
    and is added back.  sigma is the value derived from the exact h, c, k (the
    fixture's 10-digit value is checked against it)."""
    sigma = sc.Stefan_Boltzmann
    assert read_golden("codata_2018.txt")["stefan_boltzmann"] == pytest.approx(sigma, rel=1e-9)
    lam, dlam = wide_grid()
    total = oracle.grain_power(lam, dlam, np.ones_like(lam), T)
    total += 2.0 * C_ * K_ * T / (3.0 * lam[-1] ** 3) - H_ * C_ ** 2 / (4.0 * lam[-1] ** 4)
    assert abs(total / (sigma * T ** 4 / math.pi) - 1.0) < 1e-12


@pytest.mark.parametrize("T", [3.0, 45.0, 530.0, 5800.0])
def test_wien_displacement(T):
    """The peak of the oracle's B_lambda sits at lambda T = b (pins c2 alone)."""
    b = read_golden("codata_2018.txt")["wien_displacement_b"]
    f = lambda x: -oracle.lib().dust_ref_planck(math.exp(x), T)
    lo, hi = math.log(0.2 * b / T), math.log(5.0 * b / T)
    g = (math.sqrt(5.0) - 1.0) / 2.0
    a_, b_ = lo, hi
    c_, d_ = b_ - g * (b_ - a_), a_ + g * (b_ - a_)
    for _ in range(200):
        if f(c_) < f(d_):
            b_ = d_
        else:
            a_ = c_
        c_, d_ = b_ - g * (b_ - a_), a_ + g * (b_ - a_)
    peak = math.exp(0.5 * (a_ + b_))
    assert abs(peak * T / b - 1.0) < 1e-7


def test_planck_matches_independent_form():
    lam = np.geomspace(1e-7, 1e-3, 50)
    for T in (2.7, 40.0, 3000.0):
        ours = oracle.planck(lam, T)
        ref = planck_indep(lam, T)
        m = ref > 1e-300
        np.testing.assert_allclose(ours[m], ref[m], rtol=1e-13)
    assert oracle.planck(1e-6, 0.0) == 0.0
    assert math.isnan(float(oracle.planck(1e-6, float("nan"))))
    # deep Wien tail underflows to exactly zero, never NaN
    assert oracle.planck(1e-8, 1.0) == 0.0


def test_planck_dT_is_derivative():
    lam = np.geomspace(1e-7, 1e-3, 20)
    for T in (5.0, 50.0, 500.0):
        h = T * 1e-6
        fd = (planck_indep(lam, T + h) - planck_indep(lam, T - h)) / (2 * h)
        ours = oracle.planck_dT(lam, T)
        m = fd > 1e-250
        np.testing.assert_allclose(ours[m], fd[m], rtol=1e-7)


# ----------------------------------------------------------------- heating (Eq. 6)

def test_heating_is_matrix_product():
    """P8: H = J @ (C dlam)^T, checked against BLAS."""
    g = synth.make_grid(120, 2, 10)
    p = synth.cell_params(64, 11)
    J = synth.radiation_field(p, g.lam).numpy()
    H = oracle.heating(J, g.c_abs, g.dlam)
    ref = J.astype(np.float64) @ (g.c_abs * g.dlam[None, :]).T
    np.testing.assert_allclose(H, ref, rtol=1e-13, atol=0)


def test_heating_brute_force_tiny():
    rng = np.random.default_rng(5)
    J = rng.uniform(0, 2, (3, 7))
    C = rng.uniform(0, 1, (2, 7))
    dl = rng.uniform(0.1, 1, 7)
    H = oracle.heating(J, C, dl)
    for c in range(3):
        for s in range(2):
            ref = math.fsum(J[c, l] * C[s, l] * dl[l] for l in range(7))
            assert abs(H[c, s] - ref) <= 1e-15 * abs(ref)


# ----------------------------------------------------------------- temperature (Eq. 7)

@pytest.mark.parametrize("W,Tstar", [(1e-10, 5800.0), (1e-8, 20000.0), (1e-6, 3000.0), (3e-9, 12000.0)])
def test_grey_grain_diluted_blackbody(W, Tstar):
    """P1: a grey grain in J = W B(T*) has T = W^(1/4) T* (Stefan-Boltzmann).
    Cases keep T >= 5 K so that the grid (up to 1 m) holds the grain's emission."""
    lam, dlam = wide_grid()
    C = np.full((1, lam.size), 1e-14)
    J = (W * planck_indep(lam, Tstar))[None, :]
    H = oracle.heating(J, C, dlam)
    T = oracle.temperature(H, lam, dlam, C, np.array([1e-7]))
    assert abs(T[0, 0] / (W ** 0.25 * Tstar) - 1.0) < 1e-9


@pytest.mark.parametrize("beta", [1.0, 1.5, 2.0])
@pytest.mark.parametrize("W", [1e-14, 1e-11])
def test_power_law_grain(beta, W):
    """P2: C ~ lambda^-beta gives T = W^(1/(4+beta)) T*, because
    int lambda^-beta B_lambda(T) dlambda is proportional to T^(4+beta)."""
    lam, dlam = wide_grid()
    Tstar = 8000.0
    C = (1e-14 * (lam / 1e-6) ** -beta)[None, :]
    J = (W * planck_indep(lam, Tstar))[None, :]
    H = oracle.heating(J, C, dlam)
    T = oracle.temperature(H, lam, dlam, C, np.array([1e-7]))
    assert abs(T[0, 0] / (W ** (1.0 / (4.0 + beta)) * Tstar) - 1.0) < 1e-9


def _bisect_root(H, lam, dlam, c_row, steps=200):
    """Brute force: bisection in ln T on [1e-2, 1e5] K with a test-side power."""
    def power(T):
        return math.fsum(c_row * dlam * planck_indep(lam, T))
    lo, hi = math.log(1e-2), math.log(1e5)
    assert power(math.exp(lo)) < H < power(math.exp(hi))
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if power(math.exp(mid)) < H:
            lo = mid
        else:
            hi = mid
    return math.exp(0.5 * (lo + hi))


def test_brute_force_bisection_tiny():
    """P7: 200-step bisection on a tiny grid (4 cells x 8 wavelengths x 3 grains)."""
    g = synth.make_grid(8, 2, [2, 1])
    p = synth.cell_params(4, 21)
    J = synth.radiation_field(p, g.lam).numpy().astype(np.float64)
    H = oracle.heating(J, g.c_abs, g.dlam)
    T, it = oracle.temperature(H, g.lam, g.dlam, g.c_abs, g.size, return_iters=True)
    for c in range(4):
        for s in range(3):
            ref = _bisect_root(H[c, s], g.lam, g.dlam, g.c_abs[s])
            assert abs(T[c, s] / ref - 1.0) < 2e-14, (c, s, T[c, s], ref)
    assert it.max() <= 40


def test_residual_machine_precision_small_workload():
    """P4: |P(T) - H| / H at the oracle's root is at rounding level."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g, p = w.grid(), w.cells()
    J = synth.radiation_field(p, g.lam).numpy()
    H, T, L, it = oracle.run(g, J, p.m_dust, return_iters=True)
    rng = np.random.default_rng(0)
    for c in rng.integers(0, w.n_cells, 40):
        for s in range(w.n_grains):
            P = math.fsum(g.c_abs[s] * g.dlam * planck_indep(g.lam, T[c, s]))
            assert abs(P / H[c, s] - 1.0) < 1e-13
    assert it.max() <= 20
    # the synthetic workload's temperature range (sanity of the generator)
    assert 2.0 < T.min() < 3.0 and 300.0 < T.max() < 700.0


def test_root_does_not_depend_on_guess():
    """The Eq. 11 guess only steers the iteration: rescaling the grain sizes
    (which moves the guess by orders of magnitude) leaves the root in place."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g, p = w.grid(), w.cells()
    J = synth.radiation_field(p.subset(slice(0, 128)), g.lam).numpy()
    H = oracle.heating(J, g.c_abs, g.dlam)
    T1 = oracle.temperature(H, g.lam, g.dlam, g.c_abs, g.size)
    T2 = oracle.temperature(H, g.lam, g.dlam, g.c_abs, g.size * 1e3)
    T3 = oracle.temperature(H, g.lam, g.dlam, g.c_abs, g.size * 1e-2)
    np.testing.assert_allclose(T2, T1, rtol=4e-15)
    np.testing.assert_allclose(T3, T1, rtol=4e-15)


def test_guess_floor_and_quality():
    k = read_golden("eq11_guess_constants.txt")
    assert oracle.guess(1e-60, 1e-7) == k["floor_K"]
    assert oracle.guess(0.0, 1e-7) == k["floor_K"]
    w = synth.WORKLOADS["small-1024x120x20"]
    g, p = w.grid(), w.cells()
    J = synth.radiation_field(p, g.lam).numpy()
    H, T, L = oracle.run(g, J, p.m_dust)
    dex = np.log10(oracle.guess(4 * math.pi * H, g.size[None, :]) / T)
    # the fit was made for other grains; it still lands within half a dex
    assert np.percentile(np.abs(dex), 99) < 0.5


def test_temperature_special_values():
    g = synth.make_grid(16, 1, 2)
    H = np.array([[0.0, float("nan")], [-1.0, float("inf")]])
    T = oracle.temperature(H, g.lam, g.dlam, g.c_abs, g.size)
    assert T[0, 0] == 0.0
    assert math.isnan(T[0, 1]) and math.isnan(T[1, 0]) and math.isnan(T[1, 1])


def test_monotone_in_J():
    """P6: T(alpha J) > T(J) for alpha > 1; grey grain: T(alpha J) = alpha^(1/4) T(J)."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g, p = w.grid(), w.cells()
    J = synth.radiation_field(p.subset(slice(0, 64)), g.lam).numpy().astype(np.float64)
    H1 = oracle.heating(J, g.c_abs, g.dlam)
    H2 = oracle.heating(1.5 * J, g.c_abs, g.dlam)
    T1 = oracle.temperature(H1, g.lam, g.dlam, g.c_abs, g.size)
    T2 = oracle.temperature(H2, g.lam, g.dlam, g.c_abs, g.size)
    assert np.all(T2 > T1)
    lam, dlam = wide_grid()
    C = np.full((1, lam.size), 3e-15)
    Jg = (1e-13 * planck_indep(lam, 9000.0))[None, :]
    Ta = oracle.temperature(oracle.heating(Jg, C, dlam), lam, dlam, C, np.array([1e-7]))
    Tb = oracle.temperature(oracle.heating(7.0 * Jg, C, dlam), lam, dlam, C, np.array([1e-7]))
    assert abs(Tb[0, 0] / Ta[0, 0] - 7.0 ** 0.25) < 1e-9


def test_power_of_two_rescaling_of_cross_sections():
    """P10: scaling C by 2^m scales both sides of Eq. 7 exactly; the root stays."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g, p = w.grid(), w.cells()
    J = synth.radiation_field(p.subset(slice(0, 64)), g.lam).numpy()
    T0 = oracle.temperature(oracle.heating(J, g.c_abs, g.dlam), g.lam, g.dlam, g.c_abs, g.size)
    for m in (-40, 37):
        Cs = g.c_abs * 2.0 ** m
        Ts = oracle.temperature(oracle.heating(J, Cs, g.dlam), g.lam, g.dlam, Cs, g.size)
        np.testing.assert_allclose(Ts, T0, rtol=4e-15)


# ----------------------------------------------------------------- emission (Eqs. 9-10)

def test_single_grain_single_cell_emission():
    """P9: with one grain and one cell the SED is m w C B(lambda, T)."""
    g = synth.make_grid(60, 1, 1)
    T = np.array([[37.5]])
    L = oracle.emission(T, g.lam, g.c_abs, g.weight, np.array([2.5]))
    ref = 2.5 * g.weight[0] * g.c_abs[0] * planck_indep(g.lam, 37.5)
    np.testing.assert_allclose(L[0], ref, rtol=1e-13, atol=1e-300)


def test_emission_sum_over_grains_brute_force():
    g = synth.make_grid(12, 2, 3)
    rng = np.random.default_rng(9)
    T = rng.uniform(5, 300, (2, 6))
    T[1, 2] = 0.0  # a grain with no heating emits nothing
    m = np.array([0.7, 3.0])
    L = oracle.emission(T, g.lam, g.c_abs, g.weight, m)
    for c in range(2):
        for l in range(12):
            ref = m[c] * math.fsum(g.weight[s] * g.c_abs[s, l] * planck_indep(g.lam[l], T[c, s])
                                   for s in range(6) if T[c, s] > 0)
            assert abs(L[c, l] - ref) <= 1e-13 * abs(ref) + 1e-300


def test_sed_energy_identity():
    """P5: sum_l L dlam = m sum_s w_s H_s whenever every T is a root of Eq. 7."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g, p = w.grid(), w.cells()
    J = synth.radiation_field(p, g.lam).numpy()
    H, T, L = oracle.run(g, J, p.m_dust)
    lhs = (L * g.dlam[None, :]).sum(1)
    rhs = p.m_dust * (H * g.weight[None, :]).sum(1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13)


def test_emission_nan_propagates():
    g = synth.make_grid(10, 1, 2)
    T = np.array([[float("nan"), 20.0]])
    L = oracle.emission(T, g.lam, g.c_abs, g.weight)
    assert np.all(np.isnan(L))


# ----------------------------------------------------------------- extra heating (Section 2)

@pytest.mark.parametrize("T", [20.0, 100.0, 1000.0])
def test_extra_heating_alone_grey_stefan_boltzmann(T):
    """A grey grain with no radiation field and heating Q from another source
    balances C sigma T^4 / pi = Q (Section 2: the heating need not be
    absorbed light)."""
    lam, dlam = wide_grid()
    C = 1e-14
    grid = synth.Grid(lam, dlam, np.full((1, lam.size), C), np.ones(1), np.array([1e-7]), np.zeros(1, int))
    Q = np.array([[C * sc.Stefan_Boltzmann * T ** 4 / math.pi]])
    _, Tq, _ = oracle.run(grid, np.zeros((1, lam.size)), Q=Q)
    assert abs(Tq[0, 0] / T - 1.0) < 1e-9


@pytest.mark.parametrize("beta", [1.0, 2.0])
@pytest.mark.parametrize("q", [0.0, 0.3, 5.0])
def test_extra_heating_power_law_grain(beta, q):
    """C ~ lambda^-beta: P ~ T^(4+beta), so adding Q = q H to the heating of a
    diluted blackbody raises T by (1 + q)^(1/(4+beta))."""
    lam, dlam = wide_grid()
    W, Tstar = 1e-12, 8000.0
    C = (1e-14 * (lam / 1e-6) ** -beta)[None, :]
    grid = synth.Grid(lam, dlam, C, np.ones(1), np.array([1e-7]), np.zeros(1, int))
    J = (W * planck_indep(lam, Tstar))[None, :]
    H0 = oracle.heating(J, C, dlam)
    H, T, _ = oracle.run(grid, J, Q=q * H0)
    assert H[0, 0] == pytest.approx((1.0 + q) * H0[0, 0], rel=1e-15)
    expect = (W * (1.0 + q)) ** (1.0 / (4.0 + beta)) * Tstar
    assert abs(T[0, 0] / expect - 1.0) < 1e-9


# ----------------------------------------------------------------- T table (Sections 2, 5)

def test_table_nodes_are_grain_power_at_even_temperatures():
    """The table holds Eq. 7's power at T_k = t_min + k (t_max - t_min)/(n-1);
    checked against a test-side sum with an independent Planck function, and
    for a grey grain against Stefan-Boltzmann."""
    g = synth.make_grid(40, 2, [2, 1])
    n, t0, t1 = 2000, 3.0, 1500.0
    P = oracle.table_build(g.lam, g.dlam, g.c_abs, n, t0, t1)
    assert P.shape == (g.c_abs.shape[0], n)
    step = (t1 - t0) / (n - 1)
    for s in range(P.shape[0]):
        for k in (0, 1, 17, 999, n - 1):
            Tk = t0 + k * step
            ref = math.fsum(g.c_abs[s] * g.dlam * planck_indep(g.lam, Tk))
            assert P[s, k] == pytest.approx(ref, rel=1e-13)
    lam, dlam = wide_grid()
    Pg = oracle.table_build(lam, dlam, np.ones((1, lam.size)), 11, 100.0, 1100.0)
    Tk = np.linspace(100.0, 1100.0, 11)
    np.testing.assert_allclose(Pg[0], sc.Stefan_Boltzmann * Tk ** 4 / math.pi, rtol=1e-11)


def test_table_interpolation_is_numpy_interp():
    """T(H) is piecewise-linear interpolation through (P_k, T_k), with the end
    temperatures outside the table: exactly what numpy.interp computes."""
    g = synth.make_grid(30, 2, [3, 2])
    n, t0, t1 = 2000, 3.0, 1500.0
    P = oracle.table_build(g.lam, g.dlam, g.c_abs, n, t0, t1)
    S = P.shape[0]
    rng = np.random.default_rng(7)
    H = np.exp(rng.uniform(np.log(P[:, 0].min() / 30), np.log(P[:, -1].max() * 30), size=(500, S)))
    H[0, :] = P[:, 5]            # exactly on a node
    H[1, :] = P[:, -1]           # exactly the last node: in range, t_max
    T, n_out = oracle.table_temperature(H, P, t0, t1)
    Tk = t0 + np.arange(n) * ((t1 - t0) / (n - 1))
    for s in range(S):
        ref = np.interp(H[:, s], P[s], Tk)
        np.testing.assert_allclose(T[:, s], ref, rtol=1e-13, atol=0)
    outside = (H < P[:, 0][None, :]) | (H > P[:, -1][None, :])
    assert n_out == int(outside.sum()) and n_out > 0
    assert np.all(T[0] == Tk[5]) and np.all(T[1] == t1)


def test_table_special_values_and_midpoints():
    g = synth.make_grid(20, 1, [2])
    n, t0, t1 = 50, 3.0, 1500.0
    P = oracle.table_build(g.lam, g.dlam, g.c_abs, n, t0, t1)
    step = (t1 - t0) / (n - 1)
    k = np.arange(n - 1)
    mid = 0.5 * (P[:, :-1] + P[:, 1:])               # [S, n-1]
    T, n_out = oracle.table_temperature(mid.T.copy(), P, t0, t1)
    np.testing.assert_allclose(T, (t0 + (k + 0.5) * step)[:, None].repeat(P.shape[0], 1),
                               rtol=1e-12)
    assert n_out == 0
    H = np.array([[0.0, np.nan], [-1.0, np.inf]])
    T, _ = oracle.table_temperature(H[:, :1].repeat(P.shape[0], 1), P, t0, t1)
    assert T[0, 0] == 0.0 and np.isnan(T[1, 0])


def test_table_underestimates_exact_root_within_one_step():
    """P(T) is convex on the table, so its inverse is concave and the chord
    lies below it: the table's T never exceeds the exact root and is within
    one table step of it (equal at the nodes)."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    J = synth.radiation_field(w.cells().subset(np.arange(256)), g.lam).numpy().astype(np.float64)
    H = oracle.heating(J, g.c_abs, g.dlam)
    T_exact = oracle.temperature(H, g.lam, g.dlam, g.c_abs, g.size)
    n, t0, t1 = 2000, 3.0, 1500.0
    P = oracle.table_build(g.lam, g.dlam, g.c_abs, n, t0, t1)
    T, _ = oracle.table_temperature(H, P, t0, t1)
    inside = (T_exact > t0) & (T_exact < t1)
    assert inside.mean() > 0.99
    d = T_exact[inside] - T[inside]
    assert np.all(d >= -1e-12 * T_exact[inside])
    assert np.all(d < (t1 - t0) / (n - 1))
    assert d.max() > 0.0


# ----------------------------------------------------------------- re-heating loop (Section 2)

def test_reheat_grey_grain_geometric_series():
    """One grey grain: the re-absorbed power of pass n is f H_n with
    f = g m w C, so H_n = H_0 (1 - f^(n+1)) / (1 - f) exactly."""
    lam, dlam = wide_grid(4000)
    Cg, w, m = 2e-14, 3.0, 0.7
    grid = synth.Grid(lam, dlam, np.full((1, lam.size), Cg), np.array([w]), np.array([1e-7]), np.zeros(1, int))
    J0 = np.stack([1e-10 * planck_indep(lam, 6000.0), 1e-13 * planck_indep(lam, 20000.0)])
    f = np.array([0.4, 0.15])
    coupling = f / (m * w * Cg)
    passes = oracle.reheat(grid, J0, np.full(2, m), coupling, 6)
    H0 = passes[0][0][:, 0]
    for n, (H, T, L) in enumerate(passes):
        expect = H0 * (1.0 - f ** (n + 1)) / (1.0 - f)
        np.testing.assert_allclose(H[:, 0], expect, rtol=1e-12)


def test_reheat_first_pass_and_monotone_convergence():
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    p = w.cells().subset(np.arange(64))
    J0 = synth.radiation_field(p, g.lam).numpy().astype(np.float64)
    coupling = synth.reheat_coupling(g, p.m_dust, 11)
    passes = oracle.reheat(g, J0, p.m_dust, coupling, 5)
    H, T, L = oracle.run(g, J0, p.m_dust)
    np.testing.assert_array_equal(passes[0][1], T)
    Ts = np.stack([t for _, t, _ in passes])
    dT = np.diff(Ts, axis=0)
    tiny = 1e-13 * Ts[-1]
    assert np.all(dT[0] > 0.0) and np.all(dT >= -tiny)
    # contraction: every later increment is smaller than the one before
    assert np.all(dT[1:] <= dT[:-1] + tiny)
    assert np.all(dT[-1] < 0.6 ** 3 * dT[0] + tiny)


def test_heating_sum_is_compensated():
    """Eq. 6's sum keeps the low-order bits a plain running sum drops: on
    terms spread over 16 decades it equals the correctly rounded sum
    (math.fsum) of the same products."""
    import math
    rng = np.random.default_rng(5)
    NL = 4000
    J = np.empty((1, NL))
    J[0, 0] = 1.0
    J[0, 1:] = rng.uniform(0.5, 1.5, NL - 1) * 1e-16
    c_abs = np.ones((1, NL))
    dlam = np.ones(NL)
    H = oracle.heating(J, c_abs, dlam)[0, 0]
    terms = [J[0, l] * c_abs[0, l] * dlam[l] for l in range(NL)]
    exact = math.fsum(terms)
    naive = 0.0
    for t in terms:
        naive += t
    assert abs(naive - exact) > 1e3 * abs(H - exact)  # a plain sum would not pass
    assert H == pytest.approx(exact, rel=2e-16, abs=0)
