"""The seeded input generator: determinism, quadrature weights, normalisation."""
import math

import numpy as np

import synth


def test_cell_params_deterministic():
    a = synth.cell_params(500, 7)
    b = synth.cell_params(500, 7)
    for x, y in zip((a.n_bb, a.tau_v, a.tstar, a.logw, a.m_dust),
                    (b.n_bb, b.tau_v, b.tstar, b.logw, b.m_dust)):
        np.testing.assert_array_equal(x, y)
    assert set(np.unique(a.n_bb)) <= {1, 2, 3}
    assert a.tau_v.min() >= 0 and a.tau_v.max() <= 5
    assert a.tstar.min() >= 3000 and a.tstar.max() <= 30000
    assert a.logw.min() >= -16 and a.logw.max() <= -10


def test_wavelength_grid_weights():
    lam, dlam = synth.wavelength_grid(250)
    assert lam[0] == 0.09e-6 and abs(lam[-1] / 1000e-6 - 1) < 1e-15
    # ln-trapezoid: the weights divided by lambda sum to the ln range
    assert abs(np.sum(dlam / lam) - math.log(1000 / 0.09)) < 1e-12
    assert np.all(np.diff(lam) > 0)


def test_mrn_normalisation():
    g = synth.make_grid(50, 3, 17)
    for sp in range(3):
        m = g.species == sp
        vol = np.sum(g.weight[m] * 4 * math.pi / 3 * g.size[m] ** 3)
        assert abs(vol - 1) < 1e-12
    assert g.c_abs.shape == (51, 50)
    assert np.all(g.c_abs > 0)


def test_radiation_field_shape_and_range():
    g = synth.make_grid(120, 2, 10)
    p = synth.cell_params(256, 0)
    J = synth.radiation_field(p, g.lam).numpy()
    assert J.shape == (256, 120) and J.dtype == np.float32
    assert np.all(np.isfinite(J)) and np.all(J >= 0)
    assert J.max() < 1e8


def test_batch_specs():
    specs = synth.batch_specs()
    assert len(specs) == 64
    for s in specs:
        assert 1000 <= s.n_cells <= 200000
        assert 100 <= s.n_lambda <= 600
        assert 1 <= s.n_species <= 3 and 10 <= s.n_sizes <= 80
    assert specs == synth.batch_specs()
