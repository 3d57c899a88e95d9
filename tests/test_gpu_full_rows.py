"""Full-row LDS-DMA blocks (variants 5 and 6: the 64 x 8 one-plane and the
64 x 4 two-plane block on lattices one tile wide, nx = 64) through the C-ABI.

Their region has no x halo: rows are copied 16 bytes a lane, and the values at
x -+ 1 come from the neighbouring lanes of the wave that holds the periodic
row. The arithmetic and its order are those of variants 3 and 4, so the VACF
series and the fields must agree bit for bit with the haloed blocks (which
the oracle tests pin), and with the FP64 oracle to the FP32-storage bar.
"""
import numpy as np
import pytest

import oracle
from paper_1303_2470_amd import inputs

pytestmark = pytest.mark.gpu

HALOED = {5: 3, 6: 4}  # full-row variant -> the haloed block of the same tiles


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1303_2470_amd import lbmp
    lbmp.load_library()
    return lbmp


def d_err(D, Dref, db):
    """Largest |D - Dref| / max(|Dref|, 1e-2 D_b) (FP32 storage resolves D to
    about 2^-24 Z(0))."""
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


@pytest.mark.parametrize("shape,seed", [((64, 9, 7), 31), ((64, 3, 5), 32), ((64, 17, 2), 33)])
@pytest.mark.parametrize("tile", ["5,2,1", "5,2,3", "6,2,1", "6,2,3", "6,2,5"])
def test_full_rows_vs_haloed_and_oracle(lb, monkeypatch, tile, shape, seed):
    """Porous lattices 64 wide with ny and nz ragged against the block (ny = 3
    is shorter than the region, nz = 2 one plane pair), random velocity, five
    species (one without adsorption): row groups mix solid and fluid nodes,
    the solid ones being fetched as the zeros they hold."""
    m = inputs.random_mask(*shape, 0.3, seed=seed)
    u = inputs.random_velocity(m, 0.02, seed=seed + 100)
    ka = np.array([0.0, 0.02, 0.1, 0.005, 0.3])
    kd = np.array([0.1, 0.01, 0.2, 0.5, 0.9])
    params = {"D_b": 0.06, "k_a": ka, "k_d": kd}
    T = 150
    flow = lb.lb_flow_from_velocity(m, u)
    v, K, gs = (int(c) for c in tile.split(","))
    st, out, fields = run(lb, monkeypatch, tile, flow, params, T, species=(1, 4))
    assert (st["kernel_variant"], st["tile_k"], st["species_per_block"]) == (v, K, gs)
    _, ref_out, ref_fields = run(lb, monkeypatch, f"{HALOED[v]},{K},{gs}", flow, params, T, species=(1, 4))
    for key in ("Z", "mass", "vbar"):
        assert np.array_equal(out[key], ref_out[key]), key
    for (X, Xa), (Xr, Xar) in zip(fields, ref_fields):
        assert np.array_equal(X, Xr) and np.array_equal(Xa, Xar)
    for s in range(5):
        ref = oracle.vacf(m, u, 0.72, ka[s], kd[s], T)
        Dref = oracle.d_of_t(ref["Z"], ref["V"])
        assert d_err(out["D"][s], Dref, 0.06) < 1e-5, s
        assert np.allclose(out["mass"][s], ref["mass"][:, -1], rtol=1e-5)


@pytest.mark.parametrize("tile", ["5,2,64", "6,2,64"])
def test_full_rows_full_species_group(lb, monkeypatch, tile):
    """66 species (one group of 64 and one of 2) on a 64 x 10 x 9 porous
    lattice: bitwise equal to the haloed block, three species against the
    oracle."""
    m = inputs.random_mask(64, 10, 9, 0.3, seed=34)
    u = inputs.random_velocity(m, 0.02, seed=35)
    ka, kd = inputs.loguniform_rates(66, 1e-3, 3e-1, seed=36)
    params = {"D_b": 0.06, "k_a": ka, "k_d": kd}
    T = 100
    flow = lb.lb_flow_from_velocity(m, u)
    v = int(tile[0])
    st, out, _ = run(lb, monkeypatch, tile, flow, params, T)
    assert (st["kernel_variant"], st["species_per_block"]) == (v, 64)
    _, ref_out, _ = run(lb, monkeypatch, f"{HALOED[v]},2,64", flow, params, T)
    assert np.array_equal(out["Z"], ref_out["Z"]) and np.array_equal(out["mass"], ref_out["mass"])
    for s in (0, 63, 65):
        ref = oracle.vacf(m, u, 0.72, ka[s], kd[s], T)
        Dref = oracle.d_of_t(ref["Z"], ref["V"])
        assert d_err(out["D"][s], Dref, 0.06) < 1e-5, s


@pytest.mark.parametrize("tile", ["5,2,3", "6,2,3"])
def test_full_rows_slit_with_flow(lb, monkeypatch, tile):
    """Slit 64 x 8 x 22 with flow along x: bulk waves skip the sorption branch,
    wall waves take it; 400 steps against the full 3D oracle."""
    m = inputs.slit_mask(64, 8, 22)
    u = inputs.random_velocity(m, 0.02, seed=40)
    ka, kd = np.array([0.02, 0.0, 0.3]), np.array([0.01, 0.2, 0.6])
    T = 400
    flow = lb.lb_flow_from_velocity(m, u)
    st, out, _ = run(lb, monkeypatch, tile, flow, {"D_b": 0.05, "k_a": ka, "k_d": kd}, T)
    assert st["kernel_variant"] == int(tile[0])
    for s in range(3):
        ref = oracle.vacf(m, u, 0.6, ka[s], kd[s], T)
        Dref = oracle.d_of_t(ref["Z"], ref["V"])
        assert d_err(out["D"][s], Dref, 0.05) < 1e-5, s
        assert np.allclose(out["mass"][s], ref["mass"][:, -1], rtol=1e-5, atol=1e-9)


def test_full_rows_refused(lb, monkeypatch):
    """Full-row blocks need nx = 64 in every geometry, FP32 storage and K = 2."""
    m64 = inputs.random_mask(64, 6, 4, 0.3, seed=37)
    m70 = inputs.random_mask(70, 6, 4, 0.3, seed=38)
    f64 = lb.lb_flow_from_velocity(m64, np.zeros((3,) + m64.shape))
    f70 = lb.lb_flow_from_velocity(m70, np.zeros((3,) + m70.shape))
    p = {"D_b": 0.06, "k_a": [0.01], "k_d": [0.02]}
    for tile, flow, prec in (("6,2,1", f70, 32), ("5,2,1", f70, 32), ("6,2,1", f64, 64), ("5,1,1", f64, 32)):
        monkeypatch.setenv("LBMP_TILE", tile)
        with pytest.raises(lb.LbmpError) as e:
            lb.mp_init(flow, p, prec, 10)
        assert e.value.status == -1, tile
    monkeypatch.setenv("LBMP_TILE", "6,2,1")   # one geometry 70 wide refuses the batch
    with pytest.raises(lb.LbmpError):
        lb.mp_init([f64, f70], [p, p], 32, 10)


@pytest.mark.parametrize("shape,seed", [((64, 9, 7), 41), ((64, 3, 5), 42), ((64, 17, 2), 43), ((64, 6, 13), 44)])
@pytest.mark.parametrize("gs", [1, 3, 64])
def test_full_rows_four_planes(lb, monkeypatch, shape, seed, gs):
    """Full-row blocks of four planes (1,024 threads, variant 6 with K = 4):
    fields bitwise equal to the two-plane block's (same nodes, arithmetic and
    rounding bits), series to rounding (more, partly empty, reduction tiles),
    D(t) against the oracle; nz ragged against the four planes."""
    m = inputs.random_mask(*shape, 0.3, seed=seed)
    u = inputs.random_velocity(m, 0.02, seed=seed + 100)
    ka = np.array([0.0, 0.02, 0.1, 0.005, 0.3])
    kd = np.array([0.1, 0.01, 0.2, 0.5, 0.9])
    params = {"D_b": 0.06, "k_a": ka, "k_d": kd}
    T = 150
    flow = lb.lb_flow_from_velocity(m, u)
    st, out, fields = run(lb, monkeypatch, f"6,4,{gs}", flow, params, T, species=(1, 4))
    assert (st["kernel_variant"], st["tile_k"]) == (6, 4)
    _, ref_out, ref_fields = run(lb, monkeypatch, f"6,2,{gs}", flow, params, T, species=(1, 4))
    for (X, Xa), (Xr, Xar) in zip(fields, ref_fields):
        assert np.array_equal(X, Xr) and np.array_equal(Xa, Xar)
    np.testing.assert_allclose(out["Z"], ref_out["Z"], rtol=1e-12, atol=1e-18)
    for s in range(5):
        ref = oracle.vacf(m, u, 0.72, ka[s], kd[s], T)
        Dref = oracle.d_of_t(ref["Z"], ref["V"])
        assert d_err(out["D"][s], Dref, 0.06) < 1e-5, s
