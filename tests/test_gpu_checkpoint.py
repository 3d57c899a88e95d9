"""Checkpoint and resume through the C-ABI (mp_save / mp_load).

A run stopped at step n, saved, loaded into a new handle of the same
workload and continued gives the same bits as an uninterrupted run: the VACF
series, D(t), the totals and the final fields, for the dense, compact
(lattice order) and gathered-chunk (tile order) field layouts, FP64 and FP32
storage, and the uptake mode. Loading into another workload, from a
truncated buffer or beyond the handle's recordable steps is refused on the
host.
"""
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


SPECIES = {"D_b": 0.05, "k_a": [0.0, 0.01, 0.05], "k_d": [0.1, 0.02, 0.004]}


def flow(lb, seed=31):
    m = inputs.random_mask(20, 12, 10, 0.3, seed=seed)
    return lb.lb_flow_from_velocity(m, inputs.random_velocity(m, 0.02, seed=seed + 1))


@pytest.mark.parametrize("tile,prec", [("0,1,1", 64), ("0,1,1", 32), ("4,2,2", 32), ("8,2,2", 32)])
def test_resume_equals_uninterrupted_run(lb, monkeypatch, tile, prec):
    monkeypatch.setenv("LBMP_TILE", tile)
    fl = flow(lb)
    T, n = 120, 50
    a = lb.mp_init(fl, SPECIES, prec, T)
    assert lb.mp_stats(a, 0)["kernel_variant"] == int(tile.split(",")[0])
    lb.mp_step_n(a, T)
    ra = lb.mp_vacf(a, 0)
    sa = [lb.mp_state(a, 0, s) for s in range(3)]
    a.free()
    b = lb.mp_init(fl, SPECIES, prec, T)
    lb.mp_step_n(b, n)
    buf = lb.mp_save(b)
    lb.mp_step_n(b, 7)                     # the handle moves on, the checkpoint does not
    b.free()
    c = lb.mp_init(fl, SPECIES, prec, T)
    lb.mp_load(c, buf)
    assert lb.mp_steps_done(c) == n
    lb.mp_step_n(c, T - n)
    rc = lb.mp_vacf(c, 0)
    for k in ("Z", "D", "mass", "vbar"):
        assert np.array_equal(ra[k], rc[k]), k
    for s in range(3):
        X, Xa = lb.mp_state(c, 0, s)
        assert np.array_equal(X, sa[s][0]) and np.array_equal(Xa, sa[s][1]), s
    c.free()
    fl.free()


def test_checkpoint_does_not_depend_on_the_field_layout(lb, monkeypatch):
    """Saved under the dense layout, loaded under the tile-ordered compact one:
    the restored state reads back the same (FP32 values are stored as they
    are)."""
    fl = flow(lb)
    monkeypatch.setenv("LBMP_TILE", "0,1,1")
    a = lb.mp_init(fl, SPECIES, 32, 40)
    lb.mp_step_n(a, 17)
    buf = lb.mp_save(a)
    sa = [lb.mp_state(a, 0, s) for s in range(3)]
    monkeypatch.setenv("LBMP_TILE", "8,2,2")
    b = lb.mp_init(fl, SPECIES, 32, 40)
    lb.mp_load(b, buf)
    for s in range(3):
        X, Xa = lb.mp_state(b, 0, s)
        assert np.array_equal(X, sa[s][0]) and np.array_equal(Xa, sa[s][1])
    assert np.array_equal(lb.mp_vacf(a, 0)["Z"], lb.mp_vacf(b, 0)["Z"])
    a.free()
    b.free()
    fl.free()


def test_uptake_resume(lb, monkeypatch):
    monkeypatch.setenv("LBMP_TILE", "4,2,2")
    fl = flow(lb)
    sp = {"D_b": 0.05, "k_a": [0.02, 0.05], "k_d": [0.0, 0.01]}
    a = lb.mp_uptake_init(fl, sp, 32, 60)
    lb.mp_step_n(a, 60)
    ra = lb.mp_uptake(a, 0)
    b = lb.mp_uptake_init(fl, sp, 32, 60)
    lb.mp_step_n(b, 25)
    c = lb.mp_uptake_init(fl, sp, 32, 60)
    lb.mp_load(c, lb.mp_save(b))
    lb.mp_step_n(c, 35)
    rc = lb.mp_uptake(c, 0)
    for k in ("mobile", "adsorbed"):
        assert np.array_equal(ra[k], rc[k]), k
    for h in (a, b, c):
        h.free()
    fl.free()


def test_load_refusals(lb, monkeypatch):
    monkeypatch.setenv("LBMP_TILE", "0,1,1")
    fl = flow(lb)
    a = lb.mp_init(fl, SPECIES, 32, 40)
    lb.mp_step_n(a, 30)
    buf = lb.mp_save(a)
    other = dict(SPECIES, k_a=[0.0, 0.01, 0.06])
    for make, status in ((lambda: lb.mp_init(fl, other, 32, 40), -1),        # other rates
                         (lambda: lb.mp_init(fl, SPECIES, 64, 40), -1),      # other precision
                         (lambda: lb.mp_init(fl, SPECIES, 32, 20), -6)):     # fewer recordable steps
        h = make()
        with pytest.raises(lb.LbmpError) as e:
            lb.mp_load(h, buf)
        assert e.value.status == status
        h.free()
    h = lb.mp_init(fl, SPECIES, 32, 40)
    with pytest.raises(lb.LbmpError) as e:
        lb.mp_load(h, buf[:-1])                                              # truncated
    assert e.value.status == -1
    with pytest.raises(lb.LbmpError) as e:
        lb.mp_load(h, np.zeros(64, np.uint8))                                # not a checkpoint
    assert e.value.status == -1
    h.free()
    a.free()
    fl.free()
