"""Pins of the equation of state (sections 2.3, 5 and 6) and of the Marangoni
face force F = delta (I - n n) grad sigma (section 2.4)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_27534_amd import synth


def test_eos_special_values():
    base = dict(dim=2, n=(1, 1), h=1.0, sigma0=0.072, eos_E=0.3, gamma_inf=2.0)
    lin = O.eos(dict(base, eos=0), np.array([0.0, 2.0, 1.0]))
    assert np.allclose(lin, [0.072, 0.072 * 0.7, 0.072 * 0.85], rtol=0, atol=1e-17)
    # Langmuir: Gamma = Gamma_inf (1 - 1/e) gives ln(1/e) = -1 -> sigma0 (1 - E)
    g = 2.0 * (1 - math.exp(-1))
    lang = O.eos(dict(base, eos=1), np.array([0.0, g, 5.0]))
    assert abs(lang[0] - 0.072) < 1e-17
    assert abs(lang[1] - 0.072 * 0.7) < 1e-16
    assert abs(lang[2] - 0.072 * (1 + 0.3 * math.log(1e-6))) < 1e-12  # clamp at 1 - 1e-6
    # its low-concentration limit is the linear law (section 2.3)
    x = np.array([1e-4, 1e-3])
    rel = O.eos(dict(base, eos=1), 2.0 * x) / O.eos(dict(base, eos=0), 2.0 * x) - 1
    assert np.all(np.abs(rel) < 0.3 * x ** 2)
    # tanh law of section 6: E Gamma/Gamma_inf = atanh(1/2) halves sigma
    th = O.eos(dict(base, eos=2), np.array([2.0 * math.atanh(0.5) / 0.3]))
    assert abs(th[0] - 0.036) < 1e-16


def flat_prob(n):
    return dict(dim=2, n=(n, n), h=1.0 / n, bc=((1, 1), (0, 0)))


def test_force_vanishes_for_uniform_sigma():
    n = 32
    prob = dict(dim=3, n=(n, n - 4, n - 8), h=1.0 / n, bc=((0, 0), (1, 1), (2, 2)))
    chi = O.geometry(prob, synth.vof_ball((n, n - 4, n - 8), 1.0 / n, (0.5, 0.45, 0.4), 0.2, 3), 60)
    fs = O.force(prob, chi, np.full(O.shape(prob), 0.07))
    assert all(np.max(np.abs(f)) == 0.0 for f in fs)


def test_force_on_flat_interface():
    # interface y = 1/2 (grid face), sigma = a + b x: the x-faces carry
    # delta_face * b (tangential), y-faces nothing; integrated across the
    # interface the force is b * (integral of delta) ~ b
    n = 64
    h = 1.0 / n
    prob = flat_prob(n)
    f = synth.vof_flat((n, n), h, 0.5)
    chi = O.geometry(prob, f, 72)
    x, y, _ = synth.cell_centres((n, n), h)
    a, b = 0.07, -0.013
    sig = np.broadcast_to(a + b * x[None, None, :], O.shape(prob)).copy()
    fx, fy = O.force(prob, chi, sig)
    _, _, de = O.cell_geometry(prob, chi)
    dbar = 0.5 * (de[..., 1:] + de[..., :-1])       # interior x-faces 1..n-1
    # (the wrap face sees the jump of the non-periodic sigma and is left out)
    assert np.max(np.abs(fx[..., 1:n] - dbar * b)) < 1e-12 * np.max(np.abs(fx[..., 1:n]))
    assert np.max(np.abs(fy)) < 1e-18
    col = fx[0, :, 5].sum() * h
    assert abs(col / b - 1) < 2e-4
    # a normal gradient is projected out entirely wherever the normal is
    # defined (beyond the chi clamp grad chi = 0 and delta ~ 1e-4 is left
    # unprojected)
    sig2 = np.broadcast_to(a + b * y[None, :, None], O.shape(prob)).copy()
    fx2, fy2 = O.force(prob, chi, sig2)
    assert np.max(np.abs(fx2)) == 0.0
    yf = np.arange(n + 1) * h
    band = np.abs(yf - 0.5) < 16 * h
    assert np.max(np.abs(fy2[0, band, :])) < 1e-18


def test_force_tangential_on_circle():
    # sigma = a + b x around a circle: the force is tangent to the interface,
    # so at the faces crossing the top and bottom of the circle (normal along
    # y) the y-face force vanishes to O(h) while the x-face force is ~delta b
    n = 96
    h = 1.0 / n
    prob = dict(dim=2, n=(n, n), h=h, bc=((0, 0), (0, 0)))
    x, y, _ = synth.cell_centres((n, n), h)
    r = np.sqrt((x[None, None, :] - 0.5) ** 2 + (y[None, :, None] - 0.5) ** 2)
    chi = np.clip(0.3 - r, -18 * h, 18 * h)
    b = 0.02
    sig = np.broadcast_to(0.07 + b * x[None, None, :], O.shape(prob)).copy()
    fx, fy = O.force(prob, chi, sig)
    _, _, de = O.cell_geometry(prob, chi)
    j_top = int(0.8 / h)  # row crossing the top of the circle
    i_mid = n // 2
    assert abs(fx[0, j_top, i_mid] / (b * 0.5 * (de[0, j_top, i_mid] + de[0, j_top, i_mid - 1])) - 1) < 1e-2
    # total force integrates the surface gradient of sigma: for a closed
    # curve the integral of grad_s sigma over the interface vanishes by symmetry
    assert abs(fy.sum()) * h * h < 1e-12
