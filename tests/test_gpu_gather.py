"""Gathered chunks (variant 8: a block updates up to 512 fluid nodes that are
consecutive in a tile-ordered compact storage, copying their values and their
halo's into LDS and reading each arrival at a precomputed slot) through the
C-ABI.

Every node sees the arithmetic and rounding bits of the LDS-DMA blocks, so the
fields equal variant 4's bit for bit (mp_state maps both storages back to
lattice order); the block sums group nodes differently, so the series agree
to rounding. D(t) is checked against the FP64 oracle (1e-5 relative, floor
1e-2 D_b).
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


def run(lb, monkeypatch, tile, flow, params, T, species=(), uptake=False):
    monkeypatch.setenv("LBMP_TILE", tile)
    mp = (lb.mp_uptake_init if uptake else lb.mp_init)(flow, params, 32, T)
    st = lb.mp_stats(mp, 0)
    lb.mp_step_n(mp, T)
    out = lb.mp_uptake(mp, 0) if uptake else lb.mp_vacf(mp, 0)
    fields = [lb.mp_state(mp, 0, s) for s in species]
    mp.free()
    return st, out, fields


@pytest.mark.parametrize("shape,frac,seed", [((70, 9, 7), 0.3, 61), ((21, 13, 11), 0.5, 62), ((130, 5, 9), 0.8, 63),
                                             ((16, 16, 16), 0.0, 64)])
@pytest.mark.parametrize("gs", [1, 3, 5])
@pytest.mark.parametrize("nh", [1, 2])
def test_gather_vs_block_and_oracle(lb, monkeypatch, shape, frac, seed, gs, nh):
    """Random porous lattices (ragged against the ordering tiles, solid
    fractions 0 to 0.8), random velocity, five species (one without
    adsorption); blocks of 256 and 512 threads."""
    monkeypatch.setenv("LBMP_GATHER_NH", str(nh))
    m = inputs.random_mask(*shape, frac, seed=seed)
    u = inputs.random_velocity(m, 0.02, seed=seed + 100)
    ka = np.array([0.0, 0.02, 0.1, 0.005, 0.3])
    kd = np.array([0.1, 0.01, 0.2, 0.5, 0.9])
    params = {"D_b": 0.06, "k_a": ka, "k_d": kd}
    T = 150
    flow = lb.lb_flow_from_velocity(m, u)
    st, out, fields = run(lb, monkeypatch, f"8,2,{gs}", flow, params, T, species=(1, 4))
    assert (st["kernel_variant"], st["tile_k"], st["species_per_block"]) == (8, 2, gs)
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


def test_gather_sphere_pack_full_group(lb, monkeypatch):
    """40^3 sphere pack (R = 5, porosity 0.4), 66 species (a group of 64 and
    one of 2): fields equal to variant 4's, three species against the oracle."""
    m = inputs.sphere_pack(40, 5, 0.4, seed=65)
    u = inputs.random_velocity(m, 0.01, seed=66)
    ka, kd = inputs.loguniform_rates(66, 1e-3, 3e-1, seed=67)
    params = {"D_b": 0.05, "k_a": ka, "k_d": kd}
    T = 100
    flow = lb.lb_flow_from_velocity(m, u)
    st, out, fields = run(lb, monkeypatch, "8,2,64", flow, params, T, species=(0, 65))
    assert (st["kernel_variant"], st["species_per_block"]) == (8, 64)
    _, ref, ref_fields = run(lb, monkeypatch, "4,2,64", flow, params, T, species=(0, 65))
    for (X, Xa), (Xr, Xar) in zip(fields, ref_fields):
        assert np.array_equal(X, Xr) and np.array_equal(Xa, Xar)
    np.testing.assert_allclose(out["Z"], ref["Z"], rtol=1e-12, atol=1e-18)
    for s in (0, 31, 65):
        r = oracle.vacf(m, u, 0.6, ka[s], kd[s], T)
        Dref = oracle.d_of_t(r["Z"], r["V"])
        assert d_err(out["D"][s], Dref, 0.05) < 1e-5, s


def test_gather_slits_with_poiseuille_flow(lb, monkeypatch):
    """Two slits in one launch (nx = 64, walls normal to z) with a BGK flow:
    the headline workload's structure at a small size, against the oracle."""
    flows, sps, masks, us = [], [], [], []
    for W, seed in ((16, 71), (10, 72)):
        m = inputs.slit_mask(64, 12, W + 2)
        g = inputs.poiseuille_force(10.0, 0.01, W)
        fl = lb.lb_flow_solve(m, 1.0, [g, 0, 0], 1e-10, 100000)
        ka, kd = inputs.loguniform_rates(4, 1e-3, 1e-1, seed=seed)
        flows.append(fl)
        sps.append({"D_b": 0.01, "k_a": ka, "k_d": kd})
        masks.append(m)
        col = oracle.bgk(inputs.slit_mask(1, 1, W + 2), 1.0, [g, 0, 0], 1e-10, 100000)
        us.append(np.broadcast_to(col["u"], (3, W + 2, 12, 64)).copy())
    monkeypatch.setenv("LBMP_TILE", "8,2,4")
    T = 300
    mp = lb.mp_init(flows, sps, 32, T)
    assert lb.mp_stats(mp, 0)["kernel_variant"] == 8
    lb.mp_step_n(mp, T)
    for gi in range(2):
        out = lb.mp_vacf(mp, gi)
        for s in (0, 3):
            r = oracle.vacf(masks[gi], us[gi], 0.12, sps[gi]["k_a"][s], sps[gi]["k_d"][s], T)
            Dref = oracle.d_of_t(r["Z"], r["V"])
            assert d_err(out["D"][s], Dref, 0.01) < 1e-5, (gi, s)
    mp.free()


def test_gather_uptake(lb, monkeypatch):
    """Out-of-equilibrium uptake (density only, irreversible adsorption
    allowed) on the gathered blocks: totals equal variant 4's."""
    m = inputs.sphere_pack(24, 3, 0.45, seed=81)
    u = inputs.random_velocity(m, 0.01, seed=82)
    flow = lb.lb_flow_from_velocity(m, u)
    params = {"D_b": 0.05, "k_a": [0.05, 0.02], "k_d": [0.0, 0.01]}
    _, out, _ = run(lb, monkeypatch, "8,2,2", flow, params, 80, uptake=True)
    _, ref, _ = run(lb, monkeypatch, "4,2,2", flow, params, 80, uptake=True)
    np.testing.assert_allclose(out["mobile"], ref["mobile"], rtol=1e-12)
    np.testing.assert_allclose(out["adsorbed"], ref["adsorbed"], rtol=1e-12, atol=1e-18)
    r = oracle.uptake(m, u, 0.6, 0.05, 0.0, 80)
    assert np.abs(out["mobile"][0] - r["mobile"][:80]).max() < 2e-6


def test_gather_refused_in_fp64(lb, monkeypatch):
    m = inputs.random_mask(20, 6, 4, 0.3, seed=83)
    fl = lb.lb_flow_from_velocity(m, np.zeros((3,) + m.shape))
    p = {"D_b": 0.06, "k_a": [0.01], "k_d": [0.02]}
    for tile, prec in (("8,1,1", 32), ("8,2,1", 64)):
        monkeypatch.setenv("LBMP_TILE", tile)
        with pytest.raises(lb.LbmpError) as e:
            lb.mp_init(fl, p, prec, 10)
        assert e.value.status == -1, tile
