"""Pins of the whole oracle step with a moving interface (geometry rebuilt by
warm-started redistancing every step): the insoluble expanding interface of
section 4.1, whose interfacial concentration falls as the area grows."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import analytic as A
from paper_2605_27534_amd import synth


@pytest.mark.parametrize("n,bound_avg,bound_peak", [(64, 0.015, 0.2), (128, 0.004, 0.08)])
def test_expanding_circle_gamma_times_radius(n, bound_avg, bound_peak):
    # 2D point source Q: R(t) = sqrt(R0^2 + Q t / pi), insoluble carrier, so
    # Gamma R = Gamma0 R0.  Interface average sum(psi)/sum(delta) (measured
    # 1.1% (64), 0.21% (128)) and delta-peak cells (14%, 5.8%).
    h = 1.0 / n
    R0, Q, g0 = 0.1, 0.05, 0.5
    prob = dict(dim=2, n=(n, n), h=h, bc=((2, 2), (2, 2)), bulk_enabled=0, D_s=1e-3)
    Rt = lambda t: math.sqrt(R0 ** 2 + Q * t / math.pi)
    chi = O.geometry(prob, synth.vof_ball((n, n), h, (0.5, 0.5, 0), R0, 2), 72)
    _, _, de = O.cell_geometry(prob, chi)
    P = g0 * de
    F = np.zeros_like(P)
    u = synth.u_source2d((n, n), h, (0.5, 0.5, 0), Q)
    dt = 0.004 if n == 64 else 0.002
    steps = int(round(0.6 / dt))
    vs = lambda k: synth.vof_ball((n, n), h, (0.5, 0.5, 0), Rt((k + 1) * dt), 2)
    chi2, _, P2, _, hist = O.run(prob, chi, u, F, P, dt, steps, vof_seq=vs, hj_iters=8)
    T = steps * dt
    assert hist[0][O.T_DTNEXT] > dt          # within the explicit stability bound
    assert abs(hist[-1][O.T_GAVG] * Rt(T) / (g0 * R0) - 1) < bound_avg
    _, _, de2 = O.cell_geometry(prob, chi2)
    peak = np.abs(chi2) < 0.5 * h
    assert np.max(np.abs(P2[peak] / de2[peak] * Rt(T) / (g0 * R0) - 1)) < bound_peak
    m0 = hist[0][O.T_MTOT]
    assert abs(hist[-1][O.T_MTOT] - m0) < 1e-13 * m0


def _sphere(n):
    h = 1.0 / n
    R0, K = 0.15, 1.0
    Df = K * (2 * R0) ** 2 / 16          # Pe_f = K d^2 / D_f = 16 (section 4.1)
    prob = dict(dim=3, n=(n, n, n), h=h, bc=((2, 2),) * 3, bulk_enabled=0, D_s=Df)
    c = (0.5, 0.5, 0.5)
    chi = O.geometry(prob, synth.vof_ball((n, n, n), h, c, R0, 3), 108)
    _, _, de = O.cell_geometry(prob, chi)
    P = 1.0 * de
    u = synth.u_expansion((n, n, n), h, c, K, 3)
    T = 0.6
    steps = int(math.ceil(T / (0.5 * h / (1.5 * K))))
    dt = T / steps
    vs = lambda k: synth.vof_ball((n, n, n), h, c, R0 * math.exp(K * (k + 1) * dt), 3)
    _, _, _, _, hist = O.run(prob, chi, u, np.zeros_like(P), P, dt, steps, vof_seq=vs,
                             hj_iters=16)
    t = (np.arange(steps) + 1) * dt
    err = np.max(np.abs(hist[:, O.T_GAVG] / A.expansion_gamma(t, K, 3) - 1))
    return err, hist


@pytest.mark.slow
def test_expanding_sphere_3d():
    # section 4.1: u = K r e_r, Gamma = Gamma0 exp(-2 K t) up to K t = 0.6;
    # interface-average errors measured 8.7% (32) and 6.1% (48), part of it
    # carrier leaving through the open box faces (accounted in the totals)
    e32, h32 = _sphere(32)
    e48, h48 = _sphere(48)
    assert e32 < 0.10 and e48 < 0.07 and e48 < e32
    for h in (h32, h48):
        assert abs(h[-1][O.T_MTOT] / h[0][O.T_MTOT] - 1) < 1e-13
