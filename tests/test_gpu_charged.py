"""Charged tracers (Sec. II: the Q term of Eq. 8 and the excess chemical
potential beta mu^ex = beta q psi in the Eq. 11 weights) on the GPU through
mp_init_charged, against the FP64 oracle with the same potential.

Tolerance as elsewhere: FP64 storage 1e-10 relative on D(t); FP32 storage
1e-5 relative with the floor 1e-2 D_b (FP32 resolves D only to about
2^-24 Z(0)).
"""
import os

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


def d_err(D, Dref, db, floor):
    return float(np.max(np.abs(D - Dref) / np.maximum(np.abs(Dref), floor * db)))


def potential(mask, amp, seed):
    """A smooth random potential (a few Fourier modes) of amplitude ~amp."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = mask.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    b = np.zeros(mask.shape)
    for _ in range(4):
        k = rng.integers(0, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        b += np.cos(2 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + ph)
    return amp * b / 2


CASES = [(64, 1e-10, 1e-3), (32, 1e-5, 1e-2)]


@pytest.mark.parametrize("prec,tol,floor", CASES, ids=["fp64", "fp32"])
def test_porous_flow_potential_vs_oracle(lb, prec, tol, floor):
    """Random porous lattice with flow, sorption and a potential; three species
    and the opposite charge of the first on the same flow, one batched launch."""
    m = inputs.random_mask(20, 14, 11, 0.25, seed=51)
    u = inputs.random_velocity(m, 0.004, seed=52)
    bmu = potential(m, 1.0, seed=53)
    db, T = 0.03, 400
    ka, kd = np.array([0.02, 0.004, 0.0]), np.array([0.01, 0.05, 0.3])
    fl = lb.lb_flow_from_velocity(m, u)
    sp = [{"D_b": db, "k_a": ka, "k_d": kd}, {"D_b": db, "k_a": ka[:1], "k_d": kd[:1]}]
    mp = lb.mp_init([fl, fl], sp, prec, T, beta_mu_ex=[bmu, -bmu])
    lb.mp_step_n(mp, T)
    for gi, (b, k_a, k_d) in enumerate([(bmu, ka, kd), (-bmu, ka[:1], kd[:1])]):
        out = lb.mp_vacf(mp, gi)
        for s in range(len(k_a)):
            ref = oracle.vacf(m, u, 12 * db, k_a[s], k_d[s], T, bmu=b)
            Dref = oracle.d_of_t(ref["Z"], ref["V"])
            assert d_err(out["D"][s], Dref, db, floor) < tol, (gi, s)
            # FP32 storage keeps the link table in FP32: V from the rounded table
            assert np.allclose(out["vbar"][s], ref["V"], rtol=1e-9 if prec == 64 else 1e-6, atol=1e-16)
            assert np.allclose(out["mass"][s], ref["mass"][:, -1], rtol=1e-5 if prec == 32 else 1e-11,
                               atol=1e-9 if prec == 32 else 1e-14)
    mp.free()
    fl.free()


def test_boltzmann_weights_stay_at_rest(lb):
    """At rest the Eq. 11 weights with exp(-beta mu^ex) are the fixed point:
    after 200 FP64 steps the density fields equal them."""
    m = inputs.sphere_pack(24, 3, 0.5, seed=61)
    bmu = potential(m, 1.5, seed=62)
    pa, pd = 0.02, 0.01
    fl = lb.lb_flow_from_velocity(m, np.zeros((3,) + m.shape))
    mp = lb.mp_init(fl, {"D_b": 0.05, "k_a": [pa], "k_d": [pd]}, 64, 200, beta_mu_ex=[bmu])
    lb.mp_step_n(mp, 200)
    X, Xa = lb.mp_state(mp, 0, 0)
    cls = oracle.classify(m)
    w = np.where(cls > 0, np.exp(-bmu), 0.0)
    Z = w.sum() + (pa / pd) * w[cls == 2].sum()
    assert np.abs(X[0] - w / Z).max() <= 1e-12 * (w / Z).max()
    assert np.abs(Xa[0] - np.where(cls == 2, (pa / pd) * w / Z, 0.0)).max() <= 1e-12 * (w / Z).max()
    mp.free()
    fl.free()


def test_periodic_potential_effective_diffusion(lb):
    """Across a z-periodic potential in a bulk box the GPU's long-time D_z is
    the series-conductance (Lifson-Jackson) value of the one-dimensional
    detailed-balance chain, (lambda/12) / (<e^-mu> <e^((mu_z + mu_z+1)/2)>)."""
    nz, lam = 8, 0.9
    m = inputs.bulk_mask(64, 4, nz)
    z = np.arange(nz)
    mu = 1.2 * np.sin(2 * np.pi * z / nz) + 0.3 * np.cos(4 * np.pi * z / nz + 0.4)
    bmu = np.broadcast_to(mu[:, None, None], m.shape).copy()
    fl = lb.lb_flow_from_velocity(m, np.zeros((3,) + m.shape))
    mp = lb.mp_init(fl, {"D_b": lam / 12, "k_a": [0.0], "k_d": [0.5]}, 64, 800, beta_mu_ex=[bmu])
    lb.mp_step_n(mp, 800)
    D = lb.mp_vacf(mp, 0)["D"][0]
    lj = (lam / 12) / (np.mean(np.exp(-mu)) * np.mean(np.exp((mu + np.roll(mu, -1)) / 2)))
    assert abs(D[2, -1] / lj - 1) < 1e-12
    mp.free()
    fl.free()


@pytest.mark.parametrize("tile", ["3,1,2", "6,2,2", "7,2,2", "8,2,2"])
def test_lds_dma_kernels_with_potential(lb, tile):
    """The tuned FP32 step kernels (haloed, full-row, lane-compacted blocks)
    propagate the charged set-up like the oracle."""
    m = inputs.slit_mask(64, 8, 10) if tile.startswith("6") else inputs.sphere_pack(64, 4, 0.5, seed=71)[:12]
    u = inputs.random_velocity(m, 0.01, seed=72)
    bmu = potential(m, 0.8, seed=73)
    ka, kd = [0.02, 0.004], [0.01, 0.05]
    fl = lb.lb_flow_from_velocity(m, u)
    os.environ["LBMP_TILE"] = tile
    try:
        mp = lb.mp_init(fl, {"D_b": 0.05, "k_a": ka, "k_d": kd}, 32, 200, beta_mu_ex=[bmu])
    finally:
        del os.environ["LBMP_TILE"]
    assert lb.mp_stats(mp, 0)["kernel_variant"] == int(tile[0])
    lb.mp_step_n(mp, 200)
    out = lb.mp_vacf(mp, 0)
    for s in range(2):
        ref = oracle.vacf(np.ascontiguousarray(m), u, 0.6, ka[s], kd[s], 200, bmu=bmu)
        Dref = oracle.d_of_t(ref["Z"], ref["V"])
        assert d_err(out["D"][s], Dref, 0.05, 1e-2) < 1e-5, s
    mp.free()
    fl.free()


def test_charged_error_paths(lb):
    m = inputs.random_mask(6, 5, 4, 0.3, seed=81)
    fl = lb.lb_flow_from_velocity(m, np.zeros((3,) + m.shape))
    bad = np.zeros(m.shape)
    bad[m == 0] = np.nan
    with pytest.raises(lb.LbmpError) as e:
        lb.mp_init(fl, {"D_b": 0.05, "k_a": [0.01], "k_d": [0.01]}, 64, 10, beta_mu_ex=[bad])
    assert e.value.status == -1
    # a steep potential: Q factors push a stay probability below zero
    steep = np.where(np.indices(m.shape)[2] % 2 == 0, 0.0, 8.0)
    with pytest.raises(lb.LbmpError) as e:
        lb.mp_init(fl, {"Delta": 0.0, "k_a": [0.01], "k_d": [0.01]}, 64, 10, beta_mu_ex=[steep])
    assert e.value.status == -5
    fl.free()
