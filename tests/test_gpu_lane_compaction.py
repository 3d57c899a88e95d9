"""Lane compaction (variant 7: the haloed two-plane LDS-DMA block whose fluid
nodes are handed to its first threads, waves without a node skipping the
update) through the C-ABI.

Each node is updated by the same arithmetic with the same rounding bits as
in variant 4, so the fields agree bit for bit; the block sums group the
nodes differently, so the VACF series agree to rounding. Both are checked
against variant 4, and D(t) against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1303_2470_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1303_2470_amd import lbmp
    lbmp.load_library()
    return lbmp


def d_err(D, Dref, db):
    return float(np.max(np.abs(D - Dref) / np.maximum(np.abs(Dref), 1e-2 * db)))


def run(lb, monkeypatch, tile, flow, params, T, species=()):
    monkeypatch.setenv("LBMP_TILE", tile)
    mp = lb.mp_init(flow, params, 32, T)
    st = lb.mp_stats(mp, 0)
    lb.mp_step_n(mp, T)
    out = lb.mp_vacf(mp, 0)
    fields = [lb.mp_state(mp, 0, s) for s in species]
    mp.free()
    return st, out, fields


@pytest.mark.parametrize("shape,frac,seed", [((70, 9, 7), 0.3, 51), ((64, 17, 2), 0.6, 52), ((130, 5, 9), 0.8, 53)])
@pytest.mark.parametrize("gs", [1, 3, 5])
def test_lane_compaction_vs_block_and_oracle(lb, monkeypatch, shape, frac, seed, gs):
    """Random porous lattices (ragged in x, y and z; solid fractions 0.3-0.8,
    so blocks range from full to nearly empty), random velocity, five species
    (one without adsorption)."""
    m = inputs.random_mask(*shape, frac, seed=seed)
    u = inputs.random_velocity(m, 0.02, seed=seed + 100)
    ka = np.array([0.0, 0.02, 0.1, 0.005, 0.3])
    kd = np.array([0.1, 0.01, 0.2, 0.5, 0.9])
    params = {"D_b": 0.06, "k_a": ka, "k_d": kd}
    T = 150
    flow = lb.lb_flow_from_velocity(m, u)
    st, out, fields = run(lb, monkeypatch, f"7,2,{gs}", flow, params, T, species=(1, 4))
    assert (st["kernel_variant"], st["tile_k"], st["species_per_block"]) == (7, 2, gs)
    _, ref, ref_fields = run(lb, monkeypatch, f"4,2,{gs}", flow, params, T, species=(1, 4))
    for (X, Xa), (Xr, Xar) in zip(fields, ref_fields):
        assert np.array_equal(X, Xr) and np.array_equal(Xa, Xar)
    np.testing.assert_allclose(out["Z"], ref["Z"], rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(out["mass"], ref["mass"], rtol=1e-12)
    for s in range(5):
        r = oracle.vacf(m, u, 0.72, ka[s], kd[s], T)
        Dref = oracle.d_of_t(r["Z"], r["V"])
        assert d_err(out["D"][s], Dref, 0.06) < 1e-5, s
        assert np.allclose(out["mass"][s], r["mass"][:, -1], rtol=1e-5)


def test_lane_compaction_sphere_pack_full_group(lb, monkeypatch):
    """40^3 sphere pack (R = 5, porosity 0.4) with BGK-like random flow, 66
    species (a group of 64 and one of 2): fields equal to variant 4's, series
    to rounding, three species against the oracle."""
    m = inputs.sphere_pack(40, 5, 0.4, seed=54)
    u = inputs.random_velocity(m, 0.01, seed=55)
    ka, kd = inputs.loguniform_rates(66, 1e-3, 3e-1, seed=56)
    params = {"D_b": 0.05, "k_a": ka, "k_d": kd}
    T = 100
    flow = lb.lb_flow_from_velocity(m, u)
    st, out, fields = run(lb, monkeypatch, "7,2,64", flow, params, T, species=(0, 65))
    assert (st["kernel_variant"], st["species_per_block"]) == (7, 64)
    _, ref, ref_fields = run(lb, monkeypatch, "4,2,64", flow, params, T, species=(0, 65))
    for (X, Xa), (Xr, Xar) in zip(fields, ref_fields):
        assert np.array_equal(X, Xr) and np.array_equal(Xa, Xar)
    np.testing.assert_allclose(out["Z"], ref["Z"], rtol=1e-12, atol=1e-18)
    for s in (0, 31, 65):
        r = oracle.vacf(m, u, 0.6, ka[s], kd[s], T)
        Dref = oracle.d_of_t(r["Z"], r["V"])
        assert d_err(out["D"][s], Dref, 0.05) < 1e-5, s


def test_lane_compaction_refused(lb, monkeypatch):
    """Variant 7 needs FP32 storage and K = 2."""
    m = inputs.random_mask(20, 6, 4, 0.3, seed=57)
    fl = lb.lb_flow_from_velocity(m, np.zeros((3,) + m.shape))
    p = {"D_b": 0.06, "k_a": [0.01], "k_d": [0.02]}
    for tile, prec in (("7,1,1", 32), ("7,2,1", 64)):
        monkeypatch.setenv("LBMP_TILE", tile)
        with pytest.raises(lb.LbmpError) as e:
            lb.mp_init(fl, p, prec, 10)
        assert e.value.status == -1, tile
