"""Pins of the interfacial-force oracle (section 2.4; oracle/capillary.py)
against facts it must reproduce:

- the PLIC line encloses the cell's volume fraction, and its chord is the
  exact one for axis-aligned and 45-degree lines;
- the PLIC interface length of straight 45-degree lines on a periodic box
  (volume fractions from the closed-form area of a half-plane in a square,
  the Youngs normal exact there by symmetry) is the exact length; a circle's
  is within about 1% of its perimeter (the Youngs normal is not exact on
  lines at other angles);
- the height-function curvature of a circle is -1/R (n points out of
  fluid 1), to second order;
- the capillary force of a circle with uniform sigma sums to zero over the
  faces, and across the circle it integrates to the Laplace jump sigma/R;
- the Marangoni force vanishes for uniform sigma and is d sigma/dx times the
  interface length on a flat interface."""
import math

import numpy as np
import pytest

from oracle import capillary as K
from oracle import oracle as O
from paper_2605_27534_amd import synth


def test_plic_line_encloses_the_volume_fraction():
    rng = np.random.default_rng(7)
    for _ in range(200):
        m = rng.normal(size=2)
        c = rng.uniform(0.001, 0.999)
        a = K.plic_alpha(m, c)
        assert abs(K._area(K._clip(K.SQUARE, m, a)[0]) - c) < 1e-14
    assert abs(K.plic_alpha((0.0, 1.0), 0.3) - 0.3) < 1e-15


def test_plic_chords():
    for c in (0.1, 0.5, 0.93):
        assert abs(K.plic_chord((0.0, -1.0), c) - 1.0) < 1e-14
        assert abs(K.plic_chord((2.0, 0.0), c) - 1.0) < 1e-14
    assert abs(K.plic_chord((1.0, 1.0), 0.5) - math.sqrt(2)) < 1e-14
    assert abs(K.plic_chord((1.0, 1.0), 0.125) - math.sqrt(2) / 2) < 1e-14
    assert abs(K.plic_chord((-1.0, 1.0), 0.875) - math.sqrt(2) / 2) < 1e-14
    assert K.plic_chord((1.0, 1.0), 1.0) == 0.0 and K.plic_chord((0.0, 0.0), 0.5) == 0.0


def below(t):
    """area of {x + y <= t} in the unit square, the closed form"""
    t = np.clip(t, 0.0, 2.0)
    return np.where(t <= 1.0, 0.5 * t * t, 1.0 - 0.5 * (2.0 - t) ** 2)


def diagonal_stripes(n):
    # cells of the unit torus, fluid 1 where (x + y) mod 1 lies in [1/4, 3/4]
    h = 1.0 / n
    i = np.arange(n)
    s = (i[None, :] + i[:, None]).astype(float)  # (x0 + y0) / h of each cell
    vof = np.zeros((n, n))
    for k in (-1, 0, 1, 2):
        vof += below((0.75 + k) / h - s) - below((0.25 + k) / h - s)
    return vof[None]


def test_straight_lines_have_their_exact_length():
    n = 32
    prob = dict(dim=2, n=(n, n), h=1.0 / n, bc=((1, 1), (1, 1)))
    vof = diagonal_stripes(n)
    dm = K.marangoni_delta(prob, vof)
    length = float(np.sum(dm)) * prob["h"] ** 2
    assert abs(length - 2 * math.sqrt(2)) < 1e-12, length
    # a horizontal interface: one chord h per cut cell
    vof = synth.vof_flat((n, n), 1.0 / n, 0.4 + 0.3 / n)
    prob = dict(dim=2, n=(n, n), h=1.0 / n, bc=((1, 1), (0, 0)))
    length = float(np.sum(K.marangoni_delta(prob, vof))) * prob["h"] ** 2
    assert abs(length - 1.0) < 1e-13


def circle(n, R, cen=(0.5, 0.5, 0)):
    h = 1.0 / n
    prob = dict(dim=2, n=(n, n), h=h, bc=((0, 0), (0, 0)))
    vof = synth.vof_disc((n, n), h, cen, R)
    chi = O.geometry(prob, vof, 80)
    return prob, vof, chi


def test_circle_perimeter():
    R = 0.3
    errs = []
    for n in (48, 96):
        prob, vof, _ = circle(n, R)
        length = float(np.sum(K.marangoni_delta(prob, vof))) * prob["h"] ** 2
        errs.append(abs(length - 2 * math.pi * R) / (2 * math.pi * R))
    # the Youngs normal reproduces straight lines only at 0, 45 and 90
    # degrees (pinned exactly above): elsewhere its bias of a degree or so
    # leaves the PLIC length about 1% off, at any h
    assert all(e < 1.5e-2 for e in errs), errs


def test_circle_curvature():
    R = 0.3
    errs = []
    for n in (48, 96):
        prob, vof, chi = circle(n, R)
        k = K.curvature(prob, vof, chi)[0]
        v = vof[0]
        cut = (v > 1e-6) & (v < 1 - 1e-6)
        errs.append(np.max(np.abs(k[cut] * R + 1.0)))
    assert errs[-1] < 1e-2 and errs[1] < 0.6 * errs[0], errs


def test_capillary_force_balance_and_laplace_jump():
    n, R, s0 = 64, 0.3, 0.7
    # centre on a grid node: the grid is symmetric about it
    prob, vof, chi = circle(n, R, cen=(0.5, 0.5, 0))
    sig = np.full(vof.shape, s0)
    cap, ma = K.forces(prob, vof, chi, sig)
    scale = np.max(np.abs(cap[0]))
    assert abs(np.sum(cap[0])) < 1e-12 * scale * cap[0].size
    assert abs(np.sum(cap[1])) < 1e-12 * scale * cap[1].size
    assert np.max(np.abs(ma[0])) == 0.0 and np.max(np.abs(ma[1])) == 0.0
    # across the right half of the centre rows: sum F h = -sigma / R
    h = prob["h"]
    for j in (n // 2 - 1, n // 2):
        jump = float(np.sum(cap[0][0, j, n // 2:])) * h
        assert abs(jump + s0 / R) < 0.02 * s0 / R, jump


def test_marangoni_force_on_a_flat_interface():
    n = 32
    h = 1.0 / n
    prob = dict(dim=2, n=(n, n), h=h, bc=((1, 1), (0, 0)))
    vof = synth.vof_flat((n, n), h, 0.5 + 0.25 * h)
    chi = O.geometry(prob, vof, 80)
    x = (np.arange(n) + 0.5) * h
    sig = np.broadcast_to((1.0 + 0.1 * np.sin(2 * math.pi * x))[None, None, :], (1, n, n)).copy()
    cap, ma = K.forces(prob, vof, chi, sig)
    # the x faces of the cut row carry delta_m (1/h) times the face
    # difference of sigma; summed with the face area h^2 over the periodic
    # row it telescopes to zero, and face by face it is the difference
    j = int(0.5 / h)
    fx = ma[0][0, j, :n]
    dsig = (sig[0, j, :] - np.roll(sig[0, j, :], 1)) / h
    assert np.max(np.abs(fx - dsig / h)) < 1e-12 * np.max(np.abs(dsig / h))
    assert np.max(np.abs(ma[1])) < 1e-12


# ---- axisymmetric rings
def test_axisym_cylinder_and_sphere():
    from tests import oracle_pins as PINS
    PINS.rings_capillary()
