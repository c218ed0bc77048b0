"""Host logic of the adaptive Heun integrator (no GPU): convergence order and
step-size control on linear ODEs with closed-form solutions."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2108_03409_amd.driver import AdaptiveHeun  # noqa: E402


def test_heun_is_second_order():
    # y' = i w y: the local error of one Heun step is O(h^3)
    w = 2.0
    f = lambda y: 1j * w * y
    errs = []
    for h in [0.1, 0.05, 0.025]:
        y = AdaptiveHeun._heun(f, np.array([1.0 + 0j]), f(np.array([1.0 + 0j])), h)
        errs.append(abs(y[0] - np.exp(1j * w * h)))
    assert 7.0 < errs[0] / errs[1] < 9.0 and 7.0 < errs[1] / errs[2] < 9.0


def test_adaptive_heun_meets_tolerance_and_adapts():
    # a stiff-ish diagonal linear system: fast and slow modes
    lam = np.array([-1.0, -0.1 + 3j, 0.5j])
    f = lambda y: lam * y
    y0 = np.array([1.0, 1.0, 1.0], dtype=complex)
    st = AdaptiveHeun(dt=1e-4, tol=1e-6)
    t, y = 0.0, y0.copy()
    dts = []
    while t < 2.0 - 1e-12:
        st.dt = min(st.dt, 2.0 - t)
        t, y, h = st.step(t, f, y, lambda v: float(np.linalg.norm(v)))
        dts.append(h)
    exact = y0 * np.exp(lam * t)
    # the global error stays within the accumulated per-step tolerance
    assert np.linalg.norm(y - exact) < len(dts) * 1e-6
    assert max(dts) > 50 * dts[0]           # the step grew from the tiny initial value
    # a tighter tolerance takes more steps and is more accurate
    st2 = AdaptiveHeun(dt=1e-4, tol=1e-8)
    t2, y2, n2 = 0.0, y0.copy(), 0
    while t2 < 2.0 - 1e-12:
        st2.dt = min(st2.dt, 2.0 - t2)
        t2, y2, _ = st2.step(t2, f, y2, lambda v: float(np.linalg.norm(v)))
        n2 += 1
    assert n2 > len(dts)
    assert np.linalg.norm(y2 - y0 * np.exp(lam * t2)) < np.linalg.norm(y - exact)


def test_rejection_reduces_the_step():
    f = lambda y: -50.0 * y
    st = AdaptiveHeun(dt=0.5, tol=1e-6)
    t, y, h = st.step(0.0, f, np.array([1.0]), lambda v: float(np.abs(v).max()))
    assert st.n_rejected > 0 and h < 0.5
