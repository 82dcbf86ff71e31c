"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Every case runs the kernels of libdust on cuda:0 and compares element by
element with the oracle on the same seeded inputs (the oracle consumes the
exact FP32 J the GPU consumed).  Full-size workloads run in the launch
configuration the benchmark times and are compared on strided samples of
cells.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import T_TOL, check_against_oracle, oracle_on_rows, strided_rows
from oracle.compare import sed_errors

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


def _inputs(grid, n_cells, seed, dev, ldj=None):
    p = synth.cell_params(n_cells, seed)
    NL = grid.n_lambda
    if ldj is None or ldj == NL:
        J = synth.radiation_field(p, grid.lam, device=dev)
    else:
        buf = torch.full((n_cells, ldj), -7.0, dtype=torch.float32, device=dev)
        synth.radiation_field(p, grid.lam, device=dev, out=buf)
        J = buf[:, :NL]
    m = torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev)
    return J, m


def _host(t):
    return t.detach().cpu().numpy()


def _run(plan, J, m, path, counters=None):
    if path == "separate":
        H, T, L = plan.run(J, m, counters=counters)
    else:
        H = None
        T, L = plan.fused(J, m, counters=counters)
    torch.cuda.synchronize()
    return H, T, L


# --------------------------------------------------------------------------- small, full compare

@pytest.mark.parametrize("mode", ["plain", "mixed", "mixed-f32", "mixed-polish"])
@pytest.mark.parametrize("path", ["separate", "fused", "fused2"])
def test_small_full_compare(dev, mode, path):
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    say(f"small-1024x120x20 mode={mode} path={path}")
    J, m = _inputs(g, w.n_cells, w.seed, dev)
    f32 = mode == "mixed-f32"
    polish = mode == "mixed-polish"
    mode = "mixed" if (f32 or polish) else mode
    plan = dust.Plan(g, mode, fused_kernels=2 if path == "fused2" else 1, f32_lookup=f32,
                     newton_polish=polish)
    path = "fused" if path == "fused2" else path
    cnt = dust.new_counters(dev)
    H, T, L = _run(plan, J, m, path, cnt)
    res = check_against_oracle(g, _host(J), _host(m).astype(np.float64), _host(T), _host(L),
                               None if H is None else _host(H))
    say(res)
    c = _host(cnt)
    assert c[0] == 0 and c[1] == 0  # no non-finite input, nothing unconverged
    # the workload has a few pairs below 2.7 K: the mixed path solves them exactly
    if mode == "mixed":
        assert c[2] > 0


# --------------------------------------------------------------------------- ragged shapes, strides

@pytest.mark.parametrize("mode", ["plain", "mixed"])
@pytest.mark.parametrize("path", ["separate", "fused", "fused2"])
@pytest.mark.parametrize("shape", [(1000, 117, 2, 7), (77, 33, 3, 5), (1, 8, 1, 1), (130, 250, 1, 17),
                                   (50, 80, 2, 9),
                                   # 5, 6 and 7 wavelength blocks of 32 (leftover blocks
                                   # shared by cells), and 10 (a second emission column of 2)
                                   (300, 150, 2, 6), (33, 190, 2, 4), (45, 200, 3, 5),
                                   (70, 300, 1, 23)])
def test_ragged_shapes_and_strides(dev, mode, path, shape):
    C, NL, ns, nz = shape
    say(f"ragged C={C} NL={NL} species={ns} sizes={nz} mode={mode} path={path}")
    g = synth.make_grid(NL, ns, nz)
    S = g.n_grains
    J, m = _inputs(g, C, 123 + C, dev, ldj=NL + 5)
    plan = dust.Plan(g, mode, fused_kernels=2 if path == "fused2" else 1)
    path = "fused" if path == "fused2" else path
    Tbuf = torch.full((C, S + 3), -3.0, dtype=torch.float32, device=dev)
    Lbuf = torch.full((C, NL + 7), -5.0, dtype=torch.float32, device=dev)
    T, L = Tbuf[:, :S], Lbuf[:, :NL]
    if path == "separate":
        Hbuf = torch.full((C, S + 2), -9.0, dtype=torch.float32, device=dev)
        H = Hbuf[:, :S]
        plan.absorb(J, H)
        plan.solve(H, T)
        plan.emit(T, m, L)
    else:
        plan.fused(J, m, T, L)
    torch.cuda.synchronize()
    # nothing written outside the rows
    assert torch.all(Tbuf[:, S:] == -3.0) and torch.all(Lbuf[:, NL:] == -5.0)
    if path == "separate":
        assert torch.all(Hbuf[:, S:] == -9.0)
    check_against_oracle(g, _host(J), _host(m).astype(np.float64), _host(T), _host(L),
                         _host(H) if path == "separate" else None)


def test_empty_input(dev):
    g = synth.make_grid(40, 1, 4)
    for mode in ("plain", "mixed"):
        plan = dust.Plan(g, mode)
        J = torch.empty((0, 40), dtype=torch.float32, device=dev)
        H, T, L = plan.run(J)
        T2, L2 = plan.fused(J)
        torch.cuda.synchronize()
        assert H.shape == (0, 4) and L.shape == (0, 40) and T2.shape == (0, 4)


def test_max_grains(dev):
    """The largest grain count the library takes (1024) in both modes."""
    C, NL = 40, 64
    g = synth.make_grid(NL, 2, 512)
    say("max grains S=1024")
    J, m = _inputs(g, C, 99, dev)
    for mode in ("plain", "mixed"):
        plan = dust.Plan(g, mode)
        for path in ("separate", "fused"):
            H, T, L = _run(plan, J, m, path)
            check_against_oracle(g, _host(J), _host(m).astype(np.float64), _host(T), _host(L),
                                 None if H is None else _host(H))


# --------------------------------------------------------------------------- special inputs

@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_zero_field_and_nan(dev, mode):
    g = synth.make_grid(120, 2, 10)
    J, m = _inputs(g, 64, 5, dev)
    J[3].zero_()
    J[7, 11] = float("nan")
    plan = dust.Plan(g, mode)
    for path in ("separate", "fused"):
        cnt = dust.new_counters(dev)
        H, T, L = _run(plan, J, m, path, cnt)
        Th, Lh = _host(T), _host(L)
        assert np.all(Th[3] == 0.0) and np.all(Lh[3] == 0.0)
        assert np.all(np.isnan(Th[7])) and np.all(np.isnan(Lh[7]))
        assert int(_host(cnt)[0]) == g.n_grains  # every pair of the NaN cell
        keep = np.array([i for i in range(64) if i != 7])
        check_against_oracle(g, _host(J)[keep], _host(m)[keep].astype(np.float64), Th[keep],
                             Lh[keep])


@pytest.mark.parametrize("f32,ltab_n,polish,bound", [(False, 0, False, 3e-7),
                                                      (True, 0, False, 4e-6),
                                                      (False, 4096, False, 3e-7),
                                                      (False, 1024, True, 2.5e-7),
                                                      (False, 4096, True, 2.5e-7)])
def test_mixed_lookup_precision(dev, f32, ltab_n, polish, bound):
    """The mixed temperature step alone: given the oracle's FP64 heating
    rounded to FP32, T must match the oracle's root of Eq. 7 for exactly that
    H to the lookup's own error (FP64 inverse table: interpolation ~1e-9,
    plus FP32 rounding of T; FP32 lookup: FP32 rounding of ln H').  With the
    default 1024 table temperatures and with 4096.  With the FP64 Newton
    polish on the forward table (interpolation error about 1e-11) what
    remains is the FP32 arithmetic of T = expf(head) (1 + tail): expf to
    about 1 ulp, the product and the final rounding half an ulp each, at most
    2 ulp = 2.4e-7 relative, and ln H' to about 4e-8 (a fifth of that in T)."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    J, _ = _inputs(g, 512, 23, dev)
    H64 = oracle.heating(_host(J).astype(np.float64), g.c_abs, g.dlam)
    H32 = H64.astype(np.float32)
    T_ref = oracle.temperature(H32.astype(np.float64), g.lam, g.dlam, g.c_abs, g.size)
    plan = dust.Plan(g, "mixed", f32_lookup=f32, ltab_n=ltab_n, newton_polish=polish)
    cnt = dust.new_counters(dev)
    T = plan.solve(torch.as_tensor(H32, device=dev), counters=cnt)
    torch.cuda.synchronize()
    err = np.abs(_host(T).astype(np.float64) / T_ref - 1.0)
    say(f"lookup f32={f32}: max rel T err {err.max():.3g}, out of table {int(_host(cnt)[2])}")
    assert err.max() <= bound


@pytest.mark.parametrize("f32,polish", [(False, False), (True, False), (False, True)])
def test_cold_cells_use_exact_fallback(dev, f32, polish):
    """Pairs colder than the table's 2.7 K take the exact FP64 solve."""
    g = synth.make_grid(120, 2, 10)
    p = synth.cell_params(32, 17)
    p.logw[:, :] = -22.0  # very weak fields: T well below 2.7 K for big grains
    J = synth.radiation_field(p, g.lam, device=dev)
    m = torch.ones(32, dtype=torch.float32, device=dev)
    plan = dust.Plan(g, "mixed", f32_lookup=f32, newton_polish=polish)
    cnt = dust.new_counters(dev)
    T, L = plan.fused(J, m, counters=cnt)
    torch.cuda.synchronize()
    assert int(_host(cnt)[2]) > 0 and int(_host(cnt)[1]) == 0
    assert float(_host(T).min()) < 2.7
    check_against_oracle(g, _host(J), np.ones(32), _host(T), _host(L))


@pytest.mark.parametrize("mode", ["plain", "mixed", "mixed-f32", "mixed-polish"])
def test_hot_cells_above_table(dev, mode):
    """Fields strong enough to heat grains above the table's 3000 K: the mixed
    path solves them exactly, the plain path by Newton as everywhere."""
    g = synth.make_grid(120, 2, 10)
    p = synth.cell_params(32, 19)
    p.logw[:, :] = -1.5
    J = synth.radiation_field(p, g.lam, device=dev)
    m = torch.ones(32, dtype=torch.float32, device=dev)
    f32 = mode == "mixed-f32"
    polish = mode == "mixed-polish"
    plan = dust.Plan(g, "mixed" if (f32 or polish) else mode, f32_lookup=f32,
                     newton_polish=polish)
    cnt = dust.new_counters(dev)
    T, L = plan.fused(J, m, counters=cnt)
    torch.cuda.synchronize()
    assert float(_host(T).max()) > 3000.0 and int(_host(cnt)[1]) == 0
    if mode != "plain":
        assert int(_host(cnt)[2]) > 0
    check_against_oracle(g, _host(J), np.ones(32), _host(T), _host(L))


def test_maxit_one_counts_unconverged(dev):
    g = synth.make_grid(120, 2, 10)
    J, m = _inputs(g, 64, 8, dev)
    plan = dust.Plan(g, "plain", maxit=1)
    cnt = dust.new_counters(dev)
    plan.run(J, m, counters=cnt)
    torch.cuda.synchronize()
    assert int(_host(cnt)[1]) > 0


def test_plain_tolerance_option(dev):
    """A looser stopping rule (the paper's 0.1 %) still lands within its bound."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    J, m = _inputs(g, 256, 3, dev)
    plan = dust.Plan(g, "plain", tol=1e-3)
    H, T, L = _run(plan, J, m, "separate")
    H_ref, T_ref, L_ref = oracle_on_rows(g, _host(J), _host(m).astype(np.float64))
    pos = H_ref > 0
    rel = np.abs(_host(T)[pos] - T_ref[pos]) / T_ref[pos]
    # a residual below 1e-3 after the last Newton step leaves T well inside 1e-3 / (d ln P / d ln T)
    assert rel.max() < 2.5e-4


def test_grey_grain_in_diluted_blackbody_gpu(dev):
    """Physics pin run on the GPU: T = W^(1/4) T* for a grey grain."""
    lam, dlam = synth.wavelength_grid(4000, 1e-2, 1e5)
    grid = synth.Grid(lam, dlam, np.full((1, lam.size), 1e-14), np.ones(1), np.array([1e-7]),
                      np.zeros(1, np.int32))
    W = np.array([1e-8, 1e-10, 3e-12])
    Ts = np.array([20000.0, 5800.0, 9000.0])
    c2 = 6.62607015e-34 * 299792458.0 / 1.380649e-23
    c1 = 2 * 6.62607015e-34 * 299792458.0 ** 2
    Jh = W[:, None] * c1 / lam[None, :] ** 5 / np.expm1(c2 / (lam[None, :] * Ts[:, None]))
    J = torch.as_tensor(Jh, dtype=torch.float32, device=dev)
    for mode in ("plain", "mixed"):
        plan = dust.Plan(grid, mode)
        T, L = plan.fused(J)
        torch.cuda.synchronize()
        rel = np.abs(_host(T)[:, 0] / (W ** 0.25 * Ts) - 1.0)
        assert rel.max() < 1e-4, (mode, rel)


# --------------------------------------------------------------------------- invariants

@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_sed_energy_identity_on_gpu(dev, mode):
    """sum_l L dlam = m sum_s w_s H_s (holds when every T solves Eq. 7)."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    J, m = _inputs(g, w.n_cells, w.seed, dev)
    plan = dust.Plan(g, mode)
    T, L = plan.fused(J, m)
    torch.cuda.synchronize()
    H_ref = oracle.heating(_host(J), g.c_abs, g.dlam)
    lhs = (_host(L).astype(np.float64) * g.dlam).sum(1)
    rhs = _host(m).astype(np.float64) * (H_ref * g.weight).sum(1)
    assert np.max(np.abs(lhs / rhs - 1)) < 1e-3


@pytest.mark.parametrize("NL", [250, 80])
def test_emission_forms_across_temperatures(dev, NL):
    """Eqs. 9-10 alone, element by element, on a sweep of temperatures from 3 K
    to 2000 K (grains of a cell within +-30 % of the cell's T), so that the
    emission's per-(grain group, cell, wavelength block) choices fall in every
    band of t = h c log2(e) / (k lam T) (each term is 1/(2^t - 1)): skipped,
    y, y + y^2 and the exact form (NL = 250: blocks of 32
    wavelengths and 16 grains; NL = 80, fewer than four blocks: chunks of 64
    wavelengths and 8 grains).
    Bound: t carries the rounding of u_l, 1/T and their product (<= 4 2^-24
    relative, i.e. <= ln 2 * 4 * 2^-24 * t relative in 2^-t), each form
    about 2^-24 of truncation, exp2 / rcp / the weights a few ulp,
    and the FP32 sum over S grains S 2^-24; over the elements at least 1e-6
    of their row's peak t stays below about 40, so 2e-5 holds with room."""
    g = synth.make_grid(NL, 2, 40)
    C, S = 600, g.n_grains
    rng = np.random.default_rng(11)
    Tc = 3.0 * (2000.0 / 3.0) ** (np.arange(C) / (C - 1))
    Th = (Tc[:, None] * rng.uniform(0.7, 1.3, size=(C, S))).astype(np.float32)
    mh = rng.uniform(0.5, 2.0, size=C).astype(np.float32)
    # the sweep reaches every band, with the choices taken as the kernel takes them
    u = 6.62607015e-34 * 299792458.0 / 1.380649e-23 * math.log2(math.e) / g.lam
    lw, gw = (32, 16) if -(-NL // 32) >= 4 else (64, 8)
    hot = (1.0 / Th.astype(np.float64)).reshape(C, S // gw, gw).min(axis=2)
    bands = set()
    for b in range(-(-NL // lw)):
        t = u[min(lw * b + lw - 1, NL - 1)] * hot
        bands |= set(np.digitize(t.ravel(), [12.0, 24.0, 150.0]).tolist())
    # (chunks of 64 end at long wavelengths, where no grain of the sweep is
    # cold enough to be skipped)
    assert bands >= ({0, 1, 2, 3} if lw == 32 else {0, 1, 2}), bands
    plan = dust.Plan(g, "mixed")
    T = torch.as_tensor(Th, device=dev)
    m = torch.as_tensor(mh, device=dev)
    L = plan.emit(T, m)
    torch.cuda.synchronize()
    L_ref = oracle.emission(Th, g.lam, g.c_abs, g.weight, mh)
    err = sed_errors(_host(L), L_ref, g.dlam)
    say(f"emission NL={NL}: {err}")
    assert err["max"] <= 2e-5, err


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_monotone_in_J(dev, mode):
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    J, m = _inputs(g, 256, 4, dev)
    plan = dust.Plan(g, mode)
    T1, _ = plan.fused(J, m)
    T2, _ = plan.fused(J * 1.01, m)
    torch.cuda.synchronize()
    assert torch.all(T2 > T1)


@pytest.mark.parametrize("mode", ["mixed", "table"])
def test_step_graph_replays_match_eager(dev, mode):
    """prepare + fused captured into a HIP graph (as the benchmark replays its
    step): every replay, with eager work and synchronisation between them,
    reproduces the eager launch bit for bit."""
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    J, m = _inputs(g, w.n_cells, w.seed, dev)
    plan = dust.Plan(g, mode)
    T0, L0 = plan.fused(J, m)
    torch.cuda.synchronize()
    T = torch.empty_like(T0)
    L = torch.empty_like(L0)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.prepare()
        plan.fused(J, m, T, L)
    for rep in range(3):
        T.fill_(-1.0)
        L.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(T, T0) and torch.equal(L, L0), f"replay {rep}"


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_deterministic_and_prepare(dev, mode):
    w = synth.WORKLOADS["small-1024x120x20"]
    g = w.grid()
    J, m = _inputs(g, w.n_cells, w.seed, dev)
    plan = dust.Plan(g, mode)
    a = [x.clone() for x in plan.fused(J, m)]
    plan.prepare()
    b = plan.fused(J, m)
    H, T, L = plan.run(J, m)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # the three-launch path agrees with the fused one to rounding
    assert torch.allclose(T, a[0], rtol=2e-6, atol=0)


# --------------------------------------------------------------------------- full sizes, sampled

# (workload, mode, table temperatures of the mixed form (0 = the default
# 1024), FP64 Newton polish).  The million-cell workload also runs as its
# configuration states it: 4096 log-spaced table temperatures and the polish;
# the 4M-cell workload also with the polish its configuration states.
FULL = [("plain-262144x250x80", "plain", 0, False), ("plain-262144x250x80", "mixed", 0, False),
        ("mixed-1048576x500x128", "mixed", 0, False),
        ("mixed-1048576x500x128", "mixed", 4096, True),
        ("full-4194304x1000x240", "mixed", 0, False),
        ("full-4194304x1000x240", "mixed", 0, True)]


@pytest.mark.parametrize("name,mode,ltab_n,polish", FULL)
def test_full_size_sampled(dev, name, mode, ltab_n, polish):
    w = synth.WORKLOADS[name]
    g = w.grid()
    say(f"full size {name} mode={mode} ltab_n={ltab_n} polish={polish}: generating J")
    p = w.cells()
    J = synth.radiation_field(p, g.lam, device=dev)
    m = torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev)
    plan = dust.Plan(g, mode, ltab_n=ltab_n, newton_polish=polish)
    cnt = dust.new_counters(dev)
    say(f"full size {name} mode={mode}: running")
    if mode == "plain":
        H, T, L = plan.run(J, m, counters=cnt)
    else:
        T, L = plan.fused(J, m, counters=cnt)
    torch.cuda.synchronize()
    # the 4096-cell strided subsample of the million-cell workloads, 192
    # cells of the others
    rows = strided_rows(w.n_cells, 4096 if w.n_cells >= (1 << 20) else 192)
    idx = torch.as_tensor(rows, device=dev)
    say(f"full size {name} mode={mode}: oracle on {len(rows)} cells")
    res = check_against_oracle(g, _host(J[idx]), p.m_dust[rows], _host(T[idx]), _host(L[idx]))
    say(res)
    c = _host(cnt)
    assert c[0] == 0 and c[1] == 0
    # properties that hold at any size, checked on every output
    assert bool(torch.isfinite(T).all()) and bool((T > 0).all())
    assert bool(torch.isfinite(L).all())


# --------------------------------------------------------------------------- streams

def test_calls_on_side_streams(dev):
    """One plan used from two side streams at once (the fused form on one,
    the three launches on the other, different inputs) gives the results of
    the same calls on the current stream, bit for bit."""
    g = synth.make_grid(250, 2, 40)
    Ja, ma = _inputs(g, 3000, 21, dev)
    Jb, mb = _inputs(g, 2000, 22, dev)
    plan = dust.Plan(g, "mixed")
    Ta_ref, La_ref = plan.fused(Ja, ma)
    _, Tb_ref, Lb_ref = plan.run(Jb, mb)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    Ta = torch.full_like(Ta_ref, -1.0)
    La = torch.full_like(La_ref, -1.0)
    Tb = torch.full_like(Tb_ref, -1.0)
    Lb = torch.full_like(Lb_ref, -1.0)
    Hb = torch.empty_like(Tb_ref)
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    for _ in range(3):
        plan.fused(Ja, ma, Ta, La, stream=s1)
        plan.absorb(Jb, Hb, stream=s2)
        plan.solve(Hb, Tb, stream=s2)
        plan.emit(Tb, mb, Lb, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(Ta, Ta_ref) and torch.equal(La, La_ref)
    assert torch.equal(Tb, Tb_ref) and torch.equal(Lb, Lb_ref)


# --------------------------------------------------------------------------- batched persistent launch

@pytest.mark.parametrize("autotune", [False, True])
def test_batch_small_and_odd_grids(dev, autotune):
    """A batch of grids that take the batched kernel's other paths: one grain,
    fewer than four wavelength blocks (the tile's cells split over the
    waves), an odd last 8-grain group, five wavelength blocks, ragged and
    single-cell grids.  Against the oracle, and bit for bit against the
    single-grid fused launch of each grid.  With autotune every candidate
    (16- and 32-cell tiles, one workgroup per item or a work queue) runs on
    these grids while the batch is made, and the chosen one is checked."""
    shapes = [(37, 8, 1, 1), (300, 33, 3, 5), (1, 80, 2, 9), (77, 117, 2, 7),
              (130, 250, 1, 23), (45, 150, 2, 6), (1000, 64, 1, 3)]
    plans, Js, ms, Ts, Ls, grids, params = [], [], [], [], [], [], []
    for k, (C, NL, ns, nz) in enumerate(shapes):
        g = synth.make_grid(NL, ns, nz)
        p = synth.cell_params(C, 500 + k)
        grids.append(g)
        params.append(p)
        plans.append(dust.Plan(g, "mixed"))
        Js.append(synth.radiation_field(p, g.lam, device=dev))
        ms.append(torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev))
        Ts.append(torch.zeros((C, g.n_grains), dtype=torch.float32, device=dev))
        Ls.append(torch.zeros((C, NL), dtype=torch.float32, device=dev))
    say(f"batch of small and odd grids: create (autotune={autotune})")
    b = dust.Batch(plans, Js, ms, Ts, Ls, autotune=autotune, refresh_plans=True)
    say("batch info", b.info())
    b.launch()
    torch.cuda.synchronize()
    for g, p, J, T, L in zip(grids, params, Js, Ts, Ls):
        check_against_oracle(g, _host(J), p.m_dust, _host(T), _host(L))
    for plan, J, m, T, L in zip(plans, Js, ms, Ts, Ls):
        T1, L1 = plan.fused(J, m)
        torch.cuda.synchronize()
        assert torch.equal(T1, T) and torch.equal(L1, L)
    b.close()


@pytest.mark.parametrize("refresh", [False, True])
def test_batch_matches_oracle_and_replays(dev, refresh):
    specs = synth.batch_specs(n_grids=12, scale=0.02)
    plans, Js, ms, Ts, Ls, grids, params = [], [], [], [], [], [], []
    for s in specs:
        g = s.grid()
        p = s.cells()
        grids.append(g)
        params.append(p)
        plans.append(dust.Plan(g, "mixed"))
        Js.append(synth.radiation_field(p, g.lam, device=dev))
        ms.append(torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev))
        Ts.append(torch.zeros((s.n_cells, g.n_grains), dtype=torch.float32, device=dev))
        Ls.append(torch.zeros((s.n_cells, g.n_lambda), dtype=torch.float32, device=dev))
    cnt = dust.new_counters(dev)
    say("batch: create (autotune + graph capture)")
    b = dust.Batch(plans, Js, ms, Ts, Ls, counters=cnt, autotune=True, refresh_plans=refresh)
    say("batch info", b.info())
    ref = None
    for rep in range(3):
        for t in Ts + Ls:
            t.zero_()
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        snap = [t.clone() for t in Ts + Ls]
        if ref is None:
            ref = snap
        else:
            for x, y in zip(ref, snap):
                assert torch.equal(x, y)
        _ = (Js[0] * 2).sum().item()  # unrelated eager work between replays
    for g, p, J, m, T, L in zip(grids, params, Js, ms, Ts, Ls):
        rows = strided_rows(J.shape[0], 48)
        idx = torch.as_tensor(rows, device=dev)
        check_against_oracle(g, _host(J[idx]), p.m_dust[rows], _host(T[idx]), _host(L[idx]))
    # batched results equal the single-grid fused launch bitwise
    for plan, J, m, T, L in zip(plans, Js, ms, Ts, Ls):
        T1, L1 = plan.fused(J, m)
        torch.cuda.synchronize()
        assert torch.equal(T1, T) and torch.equal(L1, L)
    b.close()


@pytest.mark.parametrize("name", ["plain-262144x250x80", "full-4194304x1000x240"])
def test_absorb_full_size_sampled(dev, name):
    """dust_absorb (mixed heating, the blocked kernel) at full size: strided
    rows of H against the oracle's Eq. 6 on the same FP32 J."""
    w = synth.WORKLOADS[name]
    g = w.grid()
    p = w.cells()
    say(f"absorb full size {name}: generating J")
    J = synth.radiation_field(p, g.lam, device=dev)
    plan = dust.Plan(g, "mixed")
    H = plan.absorb(J)
    torch.cuda.synchronize()
    rows = strided_rows(w.n_cells, 256)
    idx = torch.as_tensor(rows, device=dev)
    H_ref = oracle.heating(_host(J[idx]).astype(np.float64), g.c_abs, g.dlam)
    pos = H_ref > 0
    rel = np.abs(_host(H[idx]).astype(np.float64)[pos] - H_ref[pos]) / H_ref[pos]
    say(f"absorb {name}: max rel H err {rel.max():.3g}")
    assert rel.max() <= 1e-4
    assert bool(torch.isfinite(H).all()) and bool((H >= 0).all())


# (cells, wavelengths, species, sizes per species, row length of J, J's
# offset in floats).  The blocked heating kernel's load widths (4 floats: row
# length and start 16-byte aligned; 2: 8-byte aligned; 1: neither), ragged cell
# and wavelength counts, and grain counts of one to four passes of 16 tiles.
ABSORB_SHAPES = [(257, 100, [0], 5, 100, 0),       # float4 rows, 5 grains, 257 cells
                 (300, 250, [0, 1], 40, 250, 0),   # float2 rows (the 262k-cell shape)
                 (515, 250, [0, 1], 40, 253, 0),   # odd rows: scalar loads
                 (129, 200, [0, 1], 40, 204, 2),   # rows aligned to 8 bytes only
                 (70, 64, [0, 1, 2], 100, 64, 0),  # 300 grains: two passes (16 + 3 tiles)
                 (40, 96, [0, 1], 512, 96, 0),     # 1024 grains: four passes
                 # float4 rows, by the number of full 32-wavelength k-steps
                 (100, 20, [0], 30, 20, 0),        # none (NL < 32), 2 tiles
                 (300, 32, [0, 1], 40, 32, 0),     # one, 5 tiles
                 (600, 133, [0, 1, 2], 40, 136, 0),  # four + a ragged one, 8 tiles, 600 cells
                 (260, 160, [0, 1], 90, 160, 0),   # five, 12 tiles
                 (513, 192, [0, 1, 2], 80, 192, 0),  # six, 15 of 16 tiles, 513 cells
                 (1, 64, [0], 5, 64, 0),           # a single cell: 255 rows of the block past C
                 (17, 96, [0, 1], 40, 100, 0)]     # three full k-steps, no ragged one, padded rows


@pytest.mark.parametrize("path", ["separate", "fused"])
@pytest.mark.parametrize("seed", range(12))
def test_random_shapes_three_launches(dev, seed, path):
    """dust_absorb -> dust_solve_T -> dust_emit_sed, and dust_run_fused
    (mixed), on seeded random shapes -- cells 1-700, 8-300 wavelengths, 1-3 species of 1-60 sizes, J
    rows aligned to 16, 8 or 4 bytes by the row length and the start offset
    (so every J load width and both blocked heating kernels) -- against the
    oracle on every row, with nothing written past the rows."""
    rng = np.random.default_rng(4200 + seed)
    C = int(rng.integers(1, 701))
    NL = int(rng.integers(8, 301))
    species = sorted(rng.choice(3, size=int(rng.integers(1, 4)), replace=False).tolist())
    nz = int(rng.integers(1, 61))
    # J rows 16-byte aligned (direct loads into LDS), 8-byte, or 4-byte
    align = (4, 2, 1)[seed % 3]
    pad = (-NL) % align + align * int(rng.integers(0, 3))
    off = {4: 0, 2: 2 * int(rng.integers(0, 2)), 1: 1}[align]
    g = synth.make_species_grid(NL, species, nz)
    S = g.n_grains
    say(f"random seed={seed}: C={C} NL={NL} species={species} sizes={nz} pad={pad} off={off}")
    p = synth.cell_params(C, 5100 + seed)
    ldj = NL + pad
    buf = torch.full((C * ldj + off + 8,), -7.0, dtype=torch.float32, device=dev)
    J = buf[off:off + C * ldj].view(C, ldj)[:, :NL]
    synth.radiation_field(p, g.lam, device=dev, out=J)
    m = torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev)
    plan = dust.Plan(g, "mixed")
    Hbuf = torch.full((C, S + 2), -9.0, dtype=torch.float32, device=dev)
    Tbuf = torch.full((C, S + 3), -3.0, dtype=torch.float32, device=dev)
    Lbuf = torch.full((C, NL + 5), -5.0, dtype=torch.float32, device=dev)
    H, T, L = Hbuf[:, :S], Tbuf[:, :S], Lbuf[:, :NL]
    if path == "separate":
        plan.absorb(J, H)
        plan.solve(H, T)
        plan.emit(T, m, L)
    else:
        plan.fused(J, m, T, L)
    torch.cuda.synchronize()
    assert torch.all(Hbuf[:, S:] == -9.0) and torch.all(Tbuf[:, S:] == -3.0)
    assert torch.all(Lbuf[:, NL:] == -5.0)
    check_against_oracle(g, _host(J), _host(m).astype(np.float64), _host(T), _host(L),
                         _host(H) if path == "separate" else None)


@pytest.mark.parametrize("n_cells,n_lambda,ldj,species,n_sizes", [
    (300, 256, 256, [0, 1], 40),      # direct loads into LDS, eight full k-steps, 5 tiles
    (513, 200, 204, [0, 1, 2], 80),   # direct loads, six full k-steps + a ragged one, 15 tiles
    (257, 250, 250, [0, 1], 40),      # rows aligned to 8 bytes: staged through registers
    (70, 64, 64, [0, 1, 2], 100)])    # 300 grains: two passes
def test_absorb_matches_fused_heating(dev, n_cells, n_lambda, ldj, species, n_sizes):
    """dust_absorb followed by dust_solve_T gives the fused kernel's T bit for
    bit (mixed form): both heating kernels run the same bf16 split and the
    same MFMA products in the same order, and both solves the same lookup."""
    g = synth.make_species_grid(n_lambda, species, n_sizes)
    say(f"absorb vs fused C={n_cells} NL={n_lambda} ldj={ldj} S={g.n_grains}")
    J, m = _inputs(g, n_cells, 910 + n_cells, dev, ldj=ldj)
    plan = dust.Plan(g, "mixed")
    T_f, _ = plan.fused(J, m)
    H = plan.absorb(J)
    T_s = plan.solve(H)
    torch.cuda.synchronize()
    assert torch.equal(T_s, T_f)


@pytest.mark.parametrize("n_cells,n_lambda,species,n_sizes,ldj,off", ABSORB_SHAPES)
def test_absorb_load_widths_and_passes(dev, n_cells, n_lambda, species, n_sizes, ldj, off):
    """dust_absorb in the mixed form against the oracle's Eq. 6 on every row,
    H written to padded rows (the padding untouched)."""
    g = synth.make_species_grid(n_lambda, species, n_sizes)
    say(f"absorb C={n_cells} NL={n_lambda} S={g.n_grains} ldj={ldj} off={off}")
    p = synth.cell_params(n_cells, 700 + n_cells)
    buf = torch.full((n_cells * ldj + off + 8,), -7.0, dtype=torch.float32, device=dev)
    J = buf[off:off + n_cells * ldj].view(n_cells, ldj)[:, :n_lambda]
    synth.radiation_field(p, g.lam, device=dev, out=J)
    plan = dust.Plan(g, "mixed")
    Hbuf = torch.full((n_cells, g.n_grains + 3), -5.0, dtype=torch.float32, device=dev)
    H = Hbuf[:, :g.n_grains]
    plan.absorb(J, H)
    torch.cuda.synchronize()
    assert torch.all(Hbuf[:, g.n_grains:] == -5.0)
    H_ref = oracle.heating(_host(J).astype(np.float64), g.c_abs, g.dlam)
    pos = H_ref > 0
    rel = np.abs(_host(H).astype(np.float64)[pos] - H_ref[pos]) / H_ref[pos]
    say(f"  max rel H err {rel.max():.3g}")
    assert rel.max() <= 1e-4
    assert np.all(_host(H)[~pos] == 0.0)
