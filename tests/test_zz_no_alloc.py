"""dust_batch_run_noalloc, the batched launch that allocates nothing, through
the C-ABI: the same results as dust_batch_run (which allocates its work list
on the stream) and as the FP64 oracle, on two calls in a row whose second
input is smaller than the first, so that the second reads a shorter work list
from the library's fixed array than the first one left there."""
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

FIRST = [(3000, 250, 2, 40), (777, 117, 3, 7), (1, 80, 2, 9), (200, 100, 3, 50)]
SECOND = [(500, 64, 1, 3), (33, 190, 2, 4)]


def _host(t):
    return t.detach().cpu().numpy()


def _grids(shapes, seed, dev):
    out = []
    for k, (C, NL, ns, nz) in enumerate(shapes):
        g = synth.make_grid(NL, ns, nz)
        p = synth.cell_params(C, seed + k)
        J = synth.radiation_field(p, g.lam, device=dev)
        m = torch.as_tensor(p.m_dust, dtype=torch.float32, device=dev)
        out.append((g, p, dust.Plan(g, "mixed"), J, m))
    return out


def _outputs(grids):
    T = [torch.full((J.shape[0], g.n_grains), -1.0, device=J.device) for g, _, _, J, _ in grids]
    L = [torch.full((J.shape[0], g.n_lambda), -1.0, device=J.device) for g, _, _, J, _ in grids]
    return T, L


def test_no_alloc_matches_allocating_run():
    if not torch.cuda.is_available():
        pytest.fail("this test needs an MI355X: torch.cuda.is_available() is False")
    dev = torch.device("cuda:0")
    for call, (shapes, seed) in enumerate(((FIRST, 700), (SECOND, 800))):
        print(f"no-alloc batch call {call}: {shapes}", file=sys.stderr, flush=True)
        grids = _grids(shapes, seed, dev)
        plans = [x[2] for x in grids]
        Js = [x[3] for x in grids]
        ms = [x[4] for x in grids]
        Ta, La = _outputs(grids)
        Tb, Lb = _outputs(grids)
        ca, cb = dust.new_counters(dev), dust.new_counters(dev)
        dust.batch_run(plans, Js, ms, Ta, La, counters=ca)
        dust.batch_run(plans, Js, ms, Tb, Lb, counters=cb, no_alloc=True)
        torch.cuda.synchronize()
        assert torch.equal(ca, cb)
        for (g, p, _, J, _), t_a, l_a, t_b, l_b in zip(grids, Ta, La, Tb, Lb):
            assert torch.equal(t_a, t_b) and torch.equal(l_a, l_b)
            rows = strided_rows(J.shape[0], 64)
            idx = torch.as_tensor(rows, device=dev)
            H_ref, T_ref, L_ref = oracle.run(g, _host(J[idx]).astype(np.float64), p.m_dust[rows])
            te = t_errors(_host(t_b[idx]), T_ref, H_ref)
            se = sed_errors(_host(l_b[idx]), L_ref, g.dlam)
            assert te["max"] <= T_TOL and te["zero_pairs_ok"], te
            assert se["max"] <= SED_TOL and se["energy_l1"] <= SED_TOL, se
