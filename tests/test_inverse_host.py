"""Host logic of the rate fit, on an analytic model: the mobile share of a
two-layer slit after a uniform mobile start, m(t) = m_eq + (1 - m_eq)
(1 - p_a - p_d)^t with m_eq = p_d / (p_a + p_d), where both rates are fixed
by the curve (plateau and relaxation rate)."""
import numpy as np

from paper_1303_2470_amd import inverse


def _model(t):
    def evaluate(pa, pd):
        meq = pd / (pa + pd)
        return (meq[:, None] + (1 - meq)[:, None] * (1 - pa - pd)[:, None] ** t[None])[:, None, :]
    return evaluate


def test_refine_recovers_two_state_rates():
    t = inverse.log_times(2000)
    ev = _model(t)
    for pa, pd in [(0.01, 0.004), (0.0003, 0.05), (0.08, 0.0002)]:
        target = ev(np.array([pa]), np.array([pd]))[0]
        r = inverse.refine(ev, target)
        assert abs(r["k_a"] / pa - 1) < 1e-7 and abs(r["k_d"] / pd - 1) < 1e-7, (pa, pd, r["history"])
        ms = [h["misfit"] for h in r["history"]]
        assert all(b <= a for a, b in zip(ms, ms[1:]))


def test_refine_stays_in_bounds():
    """A target outside the box ends on its edge, never beyond."""
    t = inverse.log_times(500)
    ev = _model(t)
    target = ev(np.array([0.5]), np.array([0.3]))[0]
    r = inverse.refine(ev, target, bounds=((1e-4, 1e-1), (1e-4, 1e-1)))
    assert 1e-4 <= r["k_a"] <= 1e-1 + 1e-15 and 1e-4 <= r["k_d"] <= 1e-1 + 1e-15


def test_log_times():
    t = inverse.log_times(3000)
    assert t[0] == 1 and t[-1] == 3000 and np.all(np.diff(t) > 0)


def test_porous_log_grid():
    from paper_1303_2470_amd import porous
    g = porous.log_grid(20000, 10)
    assert g[0] == 0 and g[1] == 1 and g[-1] == 20000 and np.all(np.diff(g) > 0)
    # about 10 points per decade once the integers thin out
    assert 9 <= np.sum((g >= 1000) & (g < 10000)) <= 11
