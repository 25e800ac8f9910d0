"""Pins of the oracle's hand-written discrete adjoint: gradients of the
surface-tension-history misfit L = mean_n (<sigma>^n - target^n)^2 with
respect to (k_a, k_d, D_b, D_s) and the initial bulk concentration field."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_27534_amd import synth


def setup_2d(kin=0, eos=1, bc=((0, 0), (2, 2))):
    n = 20
    h = 1.0 / n
    shp = (n, n - 3)
    prob = dict(dim=2, n=shp, h=h, bc=bc, eos=eos, eos_E=0.3, kinetics=kin)
    chi = O.geometry(prob, synth.vof_ball(shp, h, (0.5, 0.45, 0), 0.22, 2), 72)
    u = synth.u_rotation(shp, h, (0.5, 0.45, 0), 1.0)
    u = [u[0] + 0.2, u[1] - 0.1]
    c0 = 1 + 0.1 * synth.smooth_modes(shp, h, 4, dim=2)
    return prob, chi, u, c0, shp, h


def fd_check(prob, chi, u, c0, dt, N, theta, target, shp, h, dim=2, rel=1e-5):
    L, dth, gc0 = O.sigma_history_grad(prob, chi, u, c0, 0.2, dt, N, theta, target)
    for k in range(4):
        e = np.zeros(4)
        e[k] = theta[k] * 1e-5
        Lp = O.sigma_history_loss(prob, chi, u, c0, 0.2, dt, N, theta + e, target)
        Lm = O.sigma_history_loss(prob, chi, u, c0, 0.2, dt, N, theta - e, target)
        fd = (Lp - Lm) / (2 * e[k])
        # central differences at a 1e-5 relative step: ~1e-10 absolute noise
        assert abs(fd - dth[k]) <= rel * abs(fd) + 1e-10, (k, fd, dth[k])
    v = synth.smooth_modes(shp, h, 7, dim=dim)
    e = 1e-5
    Lp = O.sigma_history_loss(prob, chi, u, c0 + e * v, 0.2, dt, N, theta, target)
    Lm = O.sigma_history_loss(prob, chi, u, c0 - e * v, 0.2, dt, N, theta, target)
    fd = (Lp - Lm) / (2 * e)
    assert abs(fd - (gc0 * v).sum()) <= rel * abs(fd)


@pytest.mark.parametrize("kin,eos", [(0, 1), (1, 0), (0, 2)])
def test_adjoint_matches_central_differences_2d(kin, eos):
    prob, chi, u, c0, shp, h = setup_2d(kin, eos)
    dt = 0.1 * h * h / 1e-2
    N = 15
    theta = np.array([1.0, 1.0, 0.01, 0.001])
    fd_check(prob, chi, u, c0, dt, N, theta, np.linspace(0.95, 0.9, N), shp, h)


def test_adjoint_matches_central_differences_3d_periodic():
    n = (12, 10, 9)
    h = 1.0 / 12
    prob = dict(dim=3, n=n, h=h, bc=((0, 0), (2, 2), (1, 1)), eos=1, eos_E=0.3)
    chi = O.geometry(prob, synth.vof_ball(n, h, (0.5, 0.4, 0.35), 0.25, 3), 108)
    u = synth.u_hadamard(n, h, (0.5, 0.4, 0.35), 0.25, -0.2, 0.01)
    c0 = 1 + 0.1 * synth.smooth_modes(n, h, 4)
    dt = 0.08 * h * h / 1e-2
    N = 8
    theta = np.array([1.3, 0.7, 0.012, 0.0008])
    fd_check(prob, chi, u, c0, dt, N, theta, np.linspace(0.97, 0.93, N), n, h, dim=3)


def test_single_step_adjoint_is_the_transpose():
    # <mu, J v> (by central differences of one step) == <J^T mu, v>
    prob, chi, u, c0, shp, h = setup_2d()
    dt = 0.1 * h * h / 1e-2
    F, P = O.init_state(prob, chi, c0=c0, gamma0=0.3)
    # a generic state: in the far field psi = Gamma0 delta is exactly flat and
    # minmod sits on its kink at zero slope, where the frozen-branch adjoint is
    # a one-sided derivative; a smooth bump removes every flat region
    F = F + 0.01 * synth.smooth_modes(shp, h, 1, dim=2)
    P = P + 1e-3 * synth.smooth_modes(shp, h, 6, dim=2)
    mF, mP = synth.random_state(shp, 2, -1, 1)
    # a smooth direction: random cell noise would flip minmod branches in the
    # flat far field, where the step is only piecewise linear
    vF = synth.smooth_modes(shp, h, 3, dim=2)
    vP = 0.1 * synth.smooth_modes(shp, h, 5, dim=2)
    lF, lP, _ = O.adjoint_step(prob, chi, u, F, P, dt, mF, mP)
    e = 1e-6
    Fp, Pp, _, _ = O.step(prob, chi, u, F + e * vF, P + e * vP, dt)
    Fm, Pm, _, _ = O.step(prob, chi, u, F - e * vF, P - e * vP, dt)
    lhs = ((Fp - Fm) * mF + (Pp - Pm) * mP).sum() / (2 * e)
    rhs = (lF * vF + lP * vP).sum()
    assert abs(lhs - rhs) <= 1e-8 * abs(rhs)


def test_desorption_gradient_closed_form():
    # k_a = 0, uniform Gamma, linear EoS: <sigma>^n = sigma0 (1 - E Gamma0
    # (1 - k_d dt)^n / Gamma_inf), so dL/dk_d is a finite sum in closed form
    n = 32
    h = 1.0 / n
    prob = dict(dim=2, n=(n, n), h=h, bc=((0, 0), (0, 0)), eos=0, eos_E=0.4, sigma0=1.0)
    chi = O.geometry(prob, synth.vof_ball((n, n), h, (0.5, 0.5, 0), 0.25, 2), 72)
    dt = 0.1 * h * h / 1e-2
    N, kd, g0 = 25, 0.8, 0.6
    theta = np.array([0.0, kd, 0.01, 0.001])
    target = np.full(N, 0.8)
    L, dth, _ = O.sigma_history_grad(prob, chi, None, None, g0, dt, N, theta, target)
    s = [1.0 - 0.4 * g0 * (1 - kd * dt) ** k for k in range(1, N + 1)]
    dL = sum(2.0 / N * (s[k - 1] - 0.8) * 0.4 * g0 * k * (1 - kd * dt) ** (k - 1) * dt
             for k in range(1, N + 1))
    assert abs(dth[1] - dL) <= 1e-6 * abs(dL)
    assert abs(L - np.mean((np.array(s) - 0.8) ** 2)) <= 1e-6 * L
