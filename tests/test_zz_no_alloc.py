"""lb_flow_solve_static (the flow solve with its scratch in the library's
static device array, for callers that cannot allocate) against lb_flow_solve
through the C-ABI: bitwise-equal velocities on two calls in a row, the second
on a smaller lattice, and the size limit refused on the host."""
import ctypes

import numpy as np
import pytest

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


def _solve_both(lb, mask, force, tol, max_steps):
    ref = lb.lb_flow_solve(mask, 1.0, force, tol, max_steps, allow_unconverged=True)
    new = lb.lb_flow_solve_static(mask, 1.0, force, tol, max_steps, allow_unconverged=True)
    out = (ref.velocity(), new.velocity(), ref.steps, new.steps, ref.residual, new.residual,
           ref.converged, new.converged)
    ref.free()
    new.free()
    return out


def test_static_solve_equals_workspace_solve_twice(lb):
    # first a porous lattice (large scratch), then a smaller slit: the second
    # call reuses the array the first one left behind
    cases = [(inputs.sphere_pack(40, 5, 0.5, seed=12), [2e-6, 1e-6, 0.0], 1e-9, 20000),
             (inputs.slit_mask(8, 6, 14), [1e-6, 0.0, 0.0], 1e-10, 20000)]
    assert cases[1][0].size < cases[0][0].size
    for mask, force, tol, ms in cases:
        u_ref, u_new, s_ref, s_new, r_ref, r_new, c_ref, c_new = _solve_both(lb, mask, force, tol, ms)
        assert c_ref and c_new
        assert s_ref == s_new and r_ref == r_new
        assert np.array_equal(u_ref, u_new)          # same kernels, same order: bitwise
        assert np.abs(u_ref).max() > 0


def test_static_solve_refuses_large_lattice_on_host(lb):
    nmax = lb.lb_flow_static_max_nodes()
    assert nmax >= 64 * 64 * 66                      # the Poiseuille slit of the flow workloads fits
    n = int(np.ceil((nmax + 1) ** (1 / 3))) + 1
    mask = np.zeros((n, n, n), np.uint8)
    with pytest.raises(lb.LbmpError) as e:
        lb.lb_flow_solve_static(mask, 1.0, [1e-6, 0, 0], 1e-8, 10)
    assert e.value.status == -3
