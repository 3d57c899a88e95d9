"""Rates from D(t) (the converse use in the paper's conclusion): batched grid
refinement plus damped Gauss-Newton on the GPU path recovers (k_a, k_d) from
FP64 oracle curves of a slit at rest (normal direction, Sec. III set-up) and
of a random porous lattice with flow."""
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


@pytest.mark.parametrize("ka,kd", [(0.01, 0.004), (0.002, 0.02)])
def test_slit_rates_recovered(lb, ka, kd):
    """16-layer slit, D_b = 0.05, D_z(t) at log-spaced times to t = 3000. The
    second pair is weak sorption (f_a about 1 %), where the misfit valley of
    fixed k_a / k_d is long."""
    from paper_1303_2470_amd import inverse
    m = inputs.slit_mask(1, 1, 18)
    db = 0.05
    times = inverse.log_times(3000)
    ref = oracle.vacf(m, None, 12 * db, ka, kd, int(times.max()), qmask=8)
    Dt = oracle.d_of_t(ref["Z"], ref["V"])[2][times]
    fl = lb.lb_flow_from_velocity(m, np.zeros((3,) + m.shape))
    r = inverse.fit(lb, fl, db, times, Dt, directions=(2,))
    assert abs(r["k_a"] / ka - 1) < 1e-6 and abs(r["k_d"] / kd - 1) < 1e-6, r["history"]
    assert r["misfit"] < 1e-9
    ms = [h["misfit"] for h in r["history"]]
    assert all(b <= a for a, b in zip(ms, ms[1:]))


def test_porous_flow_rates_recovered(lb):
    """Random porous lattice with a random velocity field, D_x and D_y used;
    exact target, then the target with 0.1 % multiplicative noise."""
    from paper_1303_2470_amd import inverse
    m = inputs.random_mask(12, 10, 9, 0.3, seed=71)
    u = inputs.random_velocity(m, 0.01, seed=72)
    db, ka, kd = 0.04, 0.006, 0.009
    times = inverse.log_times(1500)
    ref = oracle.vacf(m, u, 12 * db, ka, kd, int(times.max()))
    Dt = oracle.d_of_t(ref["Z"], ref["V"])[:2][:, times]
    fl = lb.lb_flow_from_velocity(m, u)
    r = inverse.fit(lb, fl, db, times, Dt, directions=(0, 1))
    assert abs(r["k_a"] / ka - 1) < 1e-6 and abs(r["k_d"] / kd - 1) < 1e-6, r["history"]
    noisy = Dt * (1 + 1e-3 * np.random.default_rng(5).standard_normal(Dt.shape))
    r = inverse.fit(lb, fl, db, times, noisy, directions=(0, 1))
    assert abs(np.log(r["k_a"] / ka)) < 0.1 and abs(np.log(r["k_d"] / kd)) < 0.1, r["history"]
    assert r["misfit"] < 1.2e-3
