"""Synthetic input generators: shapes, seeds and the geometric facts the paper states."""
import json
import math
import os

import numpy as np
import pytest

from paper_1303_2470_amd import inputs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_fcc_porosity_matches_paper():
    """Compact fcc packing: porosity 1 - pi/(3 sqrt 2) ~ 26 % (Sec. III, Fig. 4)."""
    g = GOLDEN["fcc"]
    m = inputs.fcc_mask(g["lattice_parameter"])
    phi = 1 - m.mean()
    assert abs(phi - (1 - math.pi / (3 * math.sqrt(2)))) < 5e-3
    assert abs(phi - g["porosity_approx"]) < 0.01


def test_sphere_pack_reaches_porosity_and_is_seeded():
    a = inputs.sphere_pack(48, 4, 0.5, seed=3)
    b = inputs.sphere_pack(48, 4, 0.5, seed=3)
    c = inputs.sphere_pack(48, 4, 0.5, seed=4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    phi = 1 - a.mean()
    assert 0.47 < phi <= 0.5


def test_slit_and_rates():
    m = inputs.slit_mask(4, 4, 24)
    assert m.shape == (24, 4, 4) and m[0].all() and m[-1].all() and not m[1:-1].any()
    ka, kd = inputs.loguniform_rates(64, 1e-4, 1e-1, seed=1)
    assert ka.shape == (64,) and (ka >= 1e-4).all() and (kd <= 1e-1).all()
    ka2, _ = inputs.loguniform_rates(64, 1e-4, 1e-1, seed=1)
    assert np.array_equal(ka, ka2)


def test_poiseuille_force_recipe():
    # g = 12 nu vbar / L^2 with nu = 1/6 at tau = 1
    g = inputs.poiseuille_force(10.0, 0.01, 64)
    assert abs(g - 12 * (1 / 6) * (10 * 0.01 / 64) / 64 ** 2) < 1e-20


def test_fcc_rates_invert_the_equilibrium_share():
    """k_a from f_a (fcc workload) reproduces f_a through the Eq. 11 weights."""
    from paper_1303_2470_amd import fcc
    nf, ni, kd = 260000, 60000, 1e-2
    f = np.array([0.0, 0.3, 0.79, 0.97])
    ka = fcc.adsorption_rates(f, nf, ni, kd)
    share = ni * ka / kd / (nf + ni * ka / kd)
    assert np.allclose(share, f, rtol=1e-13, atol=0)
    with pytest.raises(ValueError):
        fcc.adsorption_rates([1.0], nf, ni, kd)
