"""GPU parity of the steps around the core path, through the C-ABI:

* the production variant of the temperature step (Sections 2 and 5): linear
  interpolation in a 2000-point table of the grain power, 3 K to 1500 K
  (mode DUST_TABLE_LINEAR), against the oracle's table variant;
* heating from sources other than the radiation field (Section 2), added to
  H before the balance is solved (dust_solve_ext.Q);
* the global iteration for dust that absorbs its own emission (Section 2):
  passes of the whole path with J updated from the previous pass's SED, the
  plain solve warm-started from the previous temperatures
  (dust_solve_ext.warm_start), against the oracle's iteration.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TABLE, T_TOL, check_against_oracle, oracle_on_rows, strided_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0907_3768_amd as dust  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("these tests need an MI355X: torch.cuda.is_available() is False")
    dust.lib()
    return torch.device("cuda:0")


def _inputs(grid, n_cells, seed, dev):
    p = synth.cell_params(n_cells, seed)
    J = synth.radiation_field(p, grid.lam, device=dev)
    m = torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev)
    return p, J, m


def _host(t):
    return t.detach().cpu().numpy()


def _run(plan, J, m, path, counters=None, Q=None, T=None, warm_start=False):
    if path == "separate":
        H, T, L = plan.run(J, m, counters=counters, Q=Q, T=T, warm_start=warm_start)
    else:
        H = None
        T, L = plan.fused(J, m, T=T, counters=counters, Q=Q, warm_start=warm_start)
    torch.cuda.synchronize()
    return H, T, L


# --------------------------------------------------------------------------- T table

@pytest.mark.parametrize("path", ["separate", "fused", "fused2"])
def test_table_small_full_compare(dev, path):
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    say(f"table-linear small-1024x120x20 path={path}")
    p, J, m = _inputs(g, w.n_cells, w.seed, dev)
    plan = dust.Plan(g, "table", fused_kernels=2 if path == "fused2" else 1)
    cnt = dust.new_counters(dev)
    H, T, L = _run(plan, J, m, "fused" if path == "fused2" else path, cnt)
    Jh, mh = _host(J), _host(m).astype(np.float64)
    res = check_against_oracle(g, Jh, mh, _host(T), _host(L), None if H is None else _host(H),
                               table=TABLE)
    say(res)
    # pairs outside the table: the same count as the oracle's, up to pairs
    # whose heating sits within rounding of a table end
    H_ref = oracle.heating(Jh, g.c_abs, g.dlam)
    P = oracle.table_build(g.lam, g.dlam, g.c_abs, *TABLE)
    _, n_out = oracle.table_temperature(H_ref, P, TABLE[1], TABLE[2])
    near = (np.abs(H_ref / P[:, 0][None, :] - 1) < 1e-5) | (np.abs(H_ref / P[:, -1][None, :] - 1) < 1e-5)
    c = _host(cnt)
    assert n_out > 0 and abs(int(c[2]) - n_out) <= int(near.sum())
    assert c[0] == 0 and c[1] == 0 and c[3] == 0
    # clamped pairs sit exactly at the end temperatures
    Th = _host(T)
    assert Th.min() == np.float32(3.0)


def test_table_never_above_exact_root(dev):
    """Linear interpolation of the concave T(H) lies below it: the table's T
    is at most the exact root (to the heating's rounding) and within a table
    step of it."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    p, J, m = _inputs(g, 512, 41, dev)
    T, L = dust.Plan(g, "table").fused(J, m)
    torch.cuda.synchronize()
    _, T_exact, _ = oracle_on_rows(g, _host(J), _host(m).astype(np.float64))
    Th = _host(T).astype(np.float64)
    inside = (T_exact > 3.0) & (T_exact < 1500.0)
    assert np.all(Th[inside] <= T_exact[inside] * (1.0 + 2e-6))
    assert np.all(T_exact[inside] - Th[inside] < (1500.0 - 3.0) / 1999 * (1.0 + 1e-6))
    rel = (T_exact[inside] - Th[inside]) / T_exact[inside]
    say(f"table-linear error vs exact root: max {rel.max():.3e}  median {np.median(rel):.3e}")


@pytest.mark.parametrize("shape", [(77, 33, 3, 5), (1, 8, 1, 1), (130, 250, 1, 17), (50, 80, 2, 9),
                                   (45, 200, 3, 5), (70, 300, 1, 23)])
def test_table_ragged(dev, shape):
    C, NL, ns, nz = shape
    g = synth.make_grid(NL, ns, nz)
    p, J, m = _inputs(g, C, 7 + C, dev)
    plan = dust.Plan(g, "table")
    for path in ("separate", "fused"):
        H, T, L = _run(plan, J, m, path)
        check_against_oracle(g, _host(J), _host(m).astype(np.float64), _host(T), _host(L),
                             None if H is None else _host(H), table=TABLE)


def test_table_other_ranges(dev):
    """ltab_n and the T range are options; 64 points over 10-400 K."""
    g = synth.make_grid(60, 2, 6)
    p, J, m = _inputs(g, 200, 13, dev)
    T, L = dust.Plan(g, "table", ltab_n=64, ltab_tmin=10.0, ltab_tmax=400.0).fused(J, m)
    torch.cuda.synchronize()
    check_against_oracle(g, _host(J), _host(m).astype(np.float64), _host(T), _host(L),
                         table=(64, 10.0, 400.0))


def test_table_full_size_sampled(dev):
    w = synth.WORKLOADS["plain-262144x250x80"]
    g = w.grid()
    say("table-linear full size plain-262144x250x80")
    p = w.cells()
    J = synth.radiation_field(p, g.lam, device=dev)
    m = torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev)
    T, L = dust.Plan(g, "table").fused(J, m)
    torch.cuda.synchronize()
    rows = strided_rows(w.n_cells, 128)
    idx = torch.as_tensor(rows, device=dev)
    check_against_oracle(g, _host(J[idx]), p.m_dust[rows], _host(T[idx]), _host(L[idx]),
                         table=TABLE)
    assert bool(((T >= 3.0) & (T <= 1500.0)).all())


# --------------------------------------------------------------------------- extra heating Q

@pytest.mark.parametrize("mode", ["plain", "mixed", "table"])
@pytest.mark.parametrize("path", ["separate", "fused", "fused2"])
def test_extra_heating(dev, mode, path):
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    C = 384
    say(f"extra heating mode={mode} path={path}")
    p, J, m = _inputs(g, C, 77, dev)
    J[5].zero_()  # a cell heated by Q alone
    Qh = synth.extra_heating(g, C, 78)
    Q = torch.as_tensor(Qh, device=dev)
    plan = dust.Plan(g, mode, fused_kernels=2 if path == "fused2" else 1)
    H, T, L = _run(plan, J, m, "fused" if path == "fused2" else path, Q=Q)
    check_against_oracle(g, _host(J), _host(m).astype(np.float64), _host(T), _host(L),
                         None if H is None else _host(H), Q=Qh,
                         table=TABLE if mode == "table" else None)
    assert np.all(_host(T)[5] > 0.0)


def test_extra_heating_strided_and_nan(dev):
    g = synth.make_grid(80, 2, 4)
    C, S = 96, g.n_grains
    p, J, m = _inputs(g, C, 5, dev)
    Qbuf = torch.full((C, S + 3), 7.0, dtype=torch.float32, device=dev)
    Qh = synth.extra_heating(g, C, 6)
    Qbuf[:, :S] = torch.as_tensor(Qh, device=dev)
    Qbuf[9, 1] = float("nan")
    plan = dust.Plan(g, "plain")
    cnt = dust.new_counters(dev)
    T, L = plan.fused(J, m, counters=cnt, Q=Qbuf[:, :S])
    torch.cuda.synchronize()
    Th = _host(T)
    assert np.isnan(Th[9, 1]) and int(_host(cnt)[0]) == 1
    keep = np.array([i for i in range(C) if i != 9])
    check_against_oracle(g, _host(J)[keep], _host(m)[keep].astype(np.float64), Th[keep],
                         _host(L)[keep], Q=Qh[keep])


def test_ext_argument_checks(dev):
    g = synth.make_grid(16, 1, 2)
    plan = dust.Plan(g, "plain")
    J = torch.ones((4, 16), dtype=torch.float32, device=dev)
    H = torch.ones((4, 2), dtype=torch.float32, device=dev)
    T = torch.ones((4, 2), dtype=torch.float32, device=dev)
    L = torch.ones((4, 16), dtype=torch.float32, device=dev)
    Q = torch.ones((4, 2), dtype=torch.float32, device=dev)
    Lb = dust.lib()
    vp = ctypes.c_void_p
    bad = [dust.SolveExt(None, 0, 0, 1),            # reserved must be 0
           dust.SolveExt(vp(Q.data_ptr()), 1, 0, 0),  # ldq < S
           dust.SolveExt(vp(Q.data_ptr() + 2), 2, 0, 0)]  # misaligned
    for x in bad:
        rc = Lb.dust_solve_T_ext(plan.handle, 4, vp(H.data_ptr()), 2, ctypes.byref(x),
                                 vp(T.data_ptr()), 2, None, None)
        assert rc == dust.DUST_EINVAL and len(dust.last_error()) > 0
        rc = Lb.dust_run_fused_ext(plan.handle, 4, vp(J.data_ptr()), 16, None, ctypes.byref(x),
                                   vp(T.data_ptr()), 2, vp(L.data_ptr()), 16, None, None)
        assert rc == dust.DUST_EINVAL
    torch.cuda.synchronize()
    assert bool((T == 1.0).all()) and bool((L == 1.0).all())  # nothing was launched


# --------------------------------------------------------------------------- warm start

@pytest.mark.parametrize("path", ["separate", "fused"])
def test_warm_start_from_solution_takes_one_evaluation(dev, path):
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    p, J, m = _inputs(g, 512, 19, dev)
    _, T_ref, _ = oracle_on_rows(g, _host(J), _host(m).astype(np.float64))
    plan = dust.Plan(g, "plain")
    cold = dust.new_counters(dev)
    _run(plan, J, m, path, cold)
    T = torch.as_tensor(T_ref.astype(np.float32), device=dev)
    warm = dust.new_counters(dev)
    H, T, L = _run(plan, J, m, path, warm, T=T, warm_start=True)
    check_against_oracle(g, _host(J), _host(m).astype(np.float64), _host(T), _host(L))
    pairs = int((T_ref > 0).sum())
    c_cold, c_warm = int(_host(cold)[3]), int(_host(warm)[3])
    say(f"Newton evaluations per pair: cold {c_cold / pairs:.2f}, warm {c_warm / pairs:.2f}")
    assert c_warm <= 1.02 * pairs < c_cold
    assert int(_host(warm)[1]) == 0


def test_warm_start_bad_values_fall_back(dev):
    """Entries that are not finite and > 0 start from the Eq. 11 guess."""
    g = synth.make_grid(120, 2, 5)
    p, J, m = _inputs(g, 64, 23, dev)
    plan = dust.Plan(g, "plain")
    T = torch.empty((64, g.n_grains), dtype=torch.float32, device=dev)
    vals = torch.tensor([0.0, -5.0, float("nan"), float("inf"), -float("inf"), 1e-30, 1e30,
                         0.3, 3e5, 1e9],
                        device=dev)
    T.copy_(vals[torch.arange(T.numel(), device=dev) % len(vals)].reshape(T.shape))
    cnt = dust.new_counters(dev)
    T, L = plan.fused(J, m, T=T, counters=cnt, warm_start=True)
    torch.cuda.synchronize()
    assert int(_host(cnt)[1]) == 0
    check_against_oracle(g, _host(J), _host(m).astype(np.float64), _host(T), _host(L))


@pytest.mark.parametrize("mode", ["mixed", "table"])
def test_warm_start_ignored_by_table_modes(dev, mode):
    g = synth.make_grid(120, 2, 5)
    p, J, m = _inputs(g, 64, 29, dev)
    plan = dust.Plan(g, mode)
    T0, L0 = plan.fused(J, m)
    T = torch.full_like(T0, 123.0)
    T1, L1 = plan.fused(J, m, T=T, warm_start=True)
    torch.cuda.synchronize()
    assert torch.equal(T0, T1) and torch.equal(L0, L1)


# --------------------------------------------------------------------------- re-heating loop

@pytest.mark.parametrize("mode,path", [("plain", "separate"), ("plain", "fused"),
                                       ("mixed", "fused"), ("table", "fused")])
def test_reheat_loop_matches_oracle(dev, mode, path):
    """Passes of the whole path with J_n = J0 + g L_{n-1}: the plain solve
    starts each pass from the previous pass's T; the last pass matches the
    oracle's iteration and the warm passes take fewer Newton evaluations."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    C, n_passes = 384, 4
    say(f"re-heating loop mode={mode} path={path}")
    p, J0, m = _inputs(g, C, 31, dev)
    coupling = synth.reheat_coupling(g, p.m_dust[:C], 32).astype(np.float32)
    gdev = torch.as_tensor(coupling, device=dev)[:, None]
    plan = dust.Plan(g, mode)
    T = torch.empty((C, g.n_grains), dtype=torch.float32, device=dev)
    L = None
    evals = []
    for n in range(n_passes):
        J = J0 if n == 0 else J0 + gdev * L
        cnt = dust.new_counters(dev)
        H, T, L = _run(plan, J, m, path, cnt, T=T, warm_start=n > 0)
        evals.append(int(_host(cnt)[3]))
    passes = oracle.reheat(g, _host(J0).astype(np.float64), _host(m).astype(np.float64),
                           coupling.astype(np.float64), n_passes,
                           table=TABLE if mode == "table" else None)
    H_ref, T_ref, L_ref = passes[-1]
    from oracle.compare import sed_errors, t_errors
    te = t_errors(_host(T), T_ref, H_ref)
    se = sed_errors(_host(L), L_ref, g.dlam)
    say({"T": te, "SED": se, "evals": evals})
    assert te["max"] <= T_TOL and te["zero_pairs_ok"]
    assert se["max"] <= 1e-3 and se["energy_l1"] <= 1e-3
    # the loop moved the temperatures: the last pass differs from the first
    assert float(np.max(T_ref / passes[0][1] - 1)) > 1e-3
    if mode == "plain":
        assert evals[-1] < evals[0]
