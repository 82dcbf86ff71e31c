"""GPU parity of the batched launches: every launch form the autotuner can
choose, the one-shot call, and the 64-grid batch at full scale.

Each batched result is compared with the FP64 oracle on the same seeded
inputs and bit for bit with the single-grid fused launch of every grid (the
batched kernels run the same tile body; only the order in which tiles are
handed out differs).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import SED_TOL, T_TOL, strided_rows
from oracle.compare import sed_errors, t_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0907_3768_amd as dust  # noqa: E402


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


# Grids that reach the batched kernel's other paths (one grain, fewer than
# four wavelength blocks, an odd last 8-grain group, ragged and single-cell
# grids) plus one of 150 grains, so that one, two and four grain tiles per
# wave are all candidate forms.
ODD_SHAPES = [(37, 8, 1, 1), (300, 33, 3, 5), (1, 80, 2, 9), (77, 117, 2, 7),
              (130, 250, 1, 23), (45, 150, 2, 6), (1000, 64, 1, 3), (200, 100, 3, 50)]


class Grids:
    """Plans, inputs, the single-grid fused results and the oracle's results."""

    def __init__(self, dev, shapes=None, specs=None, n_oracle=None):
        self.plans, self.J, self.m, self.grids, self.params = [], [], [], [], []
        self.T1, self.L1, self.ref = [], [], []
        items = shapes if shapes is not None else specs
        for k, it in enumerate(items):
            if shapes is not None:
                C, NL, ns, nz = it
                g = synth.make_grid(NL, ns, nz)
                p = synth.cell_params(C, 500 + k)
            else:
                g, p = it.grid(), it.cells()
            self.grids.append(g)
            self.params.append(p)
            self.plans.append(dust.Plan(g, "mixed"))
            self.J.append(synth.radiation_field(p, g.lam, device=dev))
            self.m.append(torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev))
        for plan, J, m in zip(self.plans, self.J, self.m):
            T1, L1 = plan.fused(J, m)
            self.T1.append(T1)
            self.L1.append(L1)
        torch.cuda.synchronize()
        for g, p, J in zip(self.grids, self.params, self.J):
            rows = strided_rows(J.shape[0], n_oracle) if n_oracle else np.arange(J.shape[0])
            idx = torch.as_tensor(rows, device=dev)
            H_ref, T_ref, L_ref = oracle.run(g, _host(J[idx]).astype(np.float64), p.m_dust[rows])
            self.ref.append((idx, H_ref, T_ref, L_ref))

    def outputs(self):
        T = [torch.full_like(t, -1.0) for t in self.T1]
        L = [torch.full_like(l, -1.0) for l in self.L1]
        return T, L

    def check(self, T, L):
        worst = 0.0
        for g, (idx, H_ref, T_ref, L_ref), Tb, Lb, T1, L1 in zip(self.grids, self.ref, T, L,
                                                                self.T1, self.L1):
            te = t_errors(_host(Tb[idx]), T_ref, H_ref)
            se = sed_errors(_host(Lb[idx]), L_ref, g.dlam)
            assert te["max"] <= T_TOL and te["zero_pairs_ok"], te
            assert se["max"] <= SED_TOL and se["energy_l1"] <= SED_TOL, se
            assert torch.equal(Tb, T1) and torch.equal(Lb, L1)
            worst = max(worst, te["max"])
        return worst


@pytest.fixture(scope="module")
def odd(dev):
    return Grids(dev, shapes=ODD_SHAPES)


CANDIDATES = [(tc, ntw, per_cu) for tc in (16, 32) for ntw in (1, 2, 4) for per_cu in (0, 2, 4, 6)]


@pytest.mark.parametrize("tc,ntw,per_cu", CANDIDATES)
def test_every_launch_form(dev, odd, monkeypatch, tc, ntw, per_cu):
    """Each candidate of the autotuner, pinned through the library's test hook,
    against the oracle and bit for bit against the single-grid launch."""
    monkeypatch.setenv("DUST_BATCH_CANDIDATE", f"{tc},{ntw},{per_cu}")
    T, L = odd.outputs()
    say(f"batch form tc={tc} ntw={ntw} per_cu={per_cu}")
    try:
        b = dust.Batch(odd.plans, odd.J, odd.m, T, L, autotune=True, refresh_plans=True)
    except dust.DustError as e:
        # forms whose LDS does not fit, or deeper than the largest grid needs
        assert e.code == dust.DUST_EUNSUPPORTED, e
        pytest.skip(f"form does not apply to this batch: {e}")
    assert b.form() == (tc, ntw, per_cu)
    for _ in range(2):  # the work-queue counter is reset by every replay
        b.launch()
        torch.cuda.synchronize()
        odd.check(T, L)
        for t in T + L:
            t.fill_(-1.0)
    b.close()


def test_malformed_candidate_is_refused(dev, odd, monkeypatch):
    monkeypatch.setenv("DUST_BATCH_CANDIDATE", "16,3,0")
    T, L = odd.outputs()
    with pytest.raises(dust.DustError) as ei:
        dust.Batch(odd.plans, odd.J, odd.m, T, L)
    assert ei.value.code == dust.DUST_EINVAL


def test_one_shot_batch_run(dev, odd):
    """dust_batch_run: the same results without a batch object, twice in a
    row (its work list is released after each call), and on a side stream."""
    T, L = odd.outputs()
    cnt = dust.new_counters(dev)
    dust.batch_run(odd.plans, odd.J, odd.m, T, L, counters=cnt)
    torch.cuda.synchronize()
    odd.check(T, L)
    assert int(_host(cnt)[0]) == 0 and int(_host(cnt)[1]) == 0
    for t in T + L:
        t.fill_(-1.0)
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream())
    dust.batch_run(odd.plans, odd.J, odd.m, T, L, stream=s)
    torch.cuda.synchronize()
    odd.check(T, L)


def test_one_shot_batch_run_with_empty_grids(dev, odd):
    """Grids of zero cells take no work items; an all-empty batch launches
    nothing."""
    J0 = torch.empty((0, odd.J[0].shape[1]), dtype=torch.float32, device=dev)
    T0 = torch.empty((0, odd.T1[0].shape[1]), dtype=torch.float32, device=dev)
    L0 = torch.empty((0, odd.L1[0].shape[1]), dtype=torch.float32, device=dev)
    dust.batch_run([odd.plans[0]], [J0], [None], [T0], [L0])
    T, L = odd.outputs()
    plans = [odd.plans[0]] + odd.plans[1:]
    Js = [J0] + odd.J[1:]
    ms = [None] + odd.m[1:]
    dust.batch_run(plans, Js, ms, [T0] + T[1:], [L0] + L[1:])
    torch.cuda.synchronize()
    for Tb, Lb, T1, L1 in zip(T[1:], L[1:], odd.T1[1:], odd.L1[1:]):
        assert torch.equal(Tb, T1) and torch.equal(Lb, L1)


def test_full_scale_batch(dev):
    """The 64 uneven grids at full size (1e3-2e5 cells, 100-600 wavelengths,
    10-240 grains), autotuned, with every plan's refresh in the graph:
    strided cells of every grid against the oracle, every grid bit for bit
    against its single-grid launch."""
    specs = synth.batch_specs()
    say(f"full-scale batch: {len(specs)} grids, {sum(s.n_cells for s in specs)} cells")
    G = Grids(dev, specs=specs, n_oracle=16)
    T, L = G.outputs()
    cnt = dust.new_counters(dev)
    b = dust.Batch(G.plans, G.J, G.m, T, L, counters=cnt, autotune=True, refresh_plans=True)
    say("full-scale batch form", b.form(), b.info())
    b.launch()
    torch.cuda.synchronize()
    worst = G.check(T, L)
    say(f"full-scale batch: worst relative T error {worst:.3g}")
    c = _host(cnt)
    assert c[0] == 0 and c[1] == 0
    b.close()
