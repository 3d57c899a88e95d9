"""Out-of-equilibrium uptake (density propagated, irreversible adsorption
allowed) through the C-ABI vs the FP64 oracle and the two-state closed form."""
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


@pytest.mark.parametrize("prec,tol", [(64, 1e-13), (32, 2e-6)])
def test_two_layer_slit_closed_form(lb, prec, tol):
    """Every fluid node interfacial, uniform density stays uniform: the mobile
    share is m_eq + (1 - m_eq)(1 - p_a - p_d)^t (p_d = 0 included)."""
    m = inputs.slit_mask(64, 16, 4)
    pa, pd = np.array([0.05, 0.08, 0.3]), np.array([0.0, 0.02, 0.1])
    T = 200
    fl = lb.lb_flow_from_velocity(m, np.zeros((3,) + m.shape))
    mp = lb.mp_uptake_init(fl, {"Delta": 0.9, "k_a": pa, "k_d": pd}, prec, T)
    lb.mp_step_n(mp, T)
    out = lb.mp_uptake(mp, 0)
    t = np.arange(T)
    for s in range(3):
        meq = pd[s] / (pa[s] + pd[s])
        ref = meq + (1 - meq) * (1 - pa[s] - pd[s]) ** t
        assert np.abs(out["mobile"][s] - ref).max() < tol, s
        assert np.abs(out["mobile"][s] + out["adsorbed"][s] - 1).max() < tol, s
    mp.free()


@pytest.mark.parametrize("prec,tol", [(64, 1e-12), (32, 2e-6)])
def test_porous_flow_vs_oracle(lb, prec, tol):
    """40^3 sphere pack, random velocity, three species (one irreversible),
    400 steps, ragged tiles."""
    m = inputs.sphere_pack(40, 5, 0.5, seed=61)
    u = inputs.random_velocity(m, 0.01, seed=62)
    lam = 0.6
    ka, kd = np.array([0.02, 0.1, 0.004]), np.array([0.0, 0.05, 0.001])
    T = 400
    fl = lb.lb_flow_from_velocity(m, u)
    mp = lb.mp_uptake_init(fl, {"D_b": lam / 12, "k_a": ka, "k_d": kd}, prec, T)
    lb.mp_step_n(mp, T)
    out = lb.mp_uptake(mp, 0)
    for s in range(3):
        ref = oracle.uptake(m, u, lam, ka[s], kd[s], T)
        assert np.abs(out["mobile"][s] - ref["mobile"][:T]).max() < tol, s
        assert np.abs(out["adsorbed"][s] - ref["adsorbed"][:T]).max() < tol, s
    # irreversible: the adsorbed total never decreases (up to rounding)
    assert np.diff(out["adsorbed"][0]).min() > -tol
    part = lb.mp_uptake(mp, 0, 100, 50)
    assert np.array_equal(part["mobile"], out["mobile"][:, 100:150])
    mp.free()


def test_uptake_error_paths(lb):
    m = inputs.slit_mask(4, 4, 8)
    fl = lb.lb_flow_from_velocity(m, np.zeros((3, 8, 4, 4)))
    with pytest.raises(lb.LbmpError) as e:                  # k_d = 0 needs the uptake calls
        lb.mp_init(fl, {"Delta": 0.5, "k_a": [0.1], "k_d": [0.0]}, 32, 10)
    assert e.value.status == -1
    mp = lb.mp_uptake_init(fl, {"Delta": 0.5, "k_a": [0.1], "k_d": [0.0]}, 32, 10)
    lb.mp_step_n(mp, 5)
    with pytest.raises(lb.LbmpError) as e:                  # no VACF on an uptake handle
        lb.mp_vacf(mp, 0)
    assert e.value.status == -6
    with pytest.raises(lb.LbmpError) as e:                  # tau = 5 not recorded yet
        lb.mp_uptake(mp, 0, 0, 6)
    assert e.value.status == -1
    mp.free()
