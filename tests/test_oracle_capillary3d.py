"""Pins of the 3D interfacial-force oracle (section 2.4) against facts it
must reproduce, none of them a retyping of its formulas:

- the PLIC plane: exact areas of planes the geometry fixes (an axis-aligned
  plane, the regular hexagon of the cube's central diagonal section, the
  diagonal rectangle, the equilateral corner triangle), the 2D oracle's
  chord for a plane parallel to an axis, the complement symmetry, and the
  exact volume against a count of points on a fine lattice;
- a sphere: the sum of A_f over the cells converges to 4 pi R^2 and the
  height-function curvature to -2/R;
- a flat interface: delta_m = 1/h and kappa = 0 exactly, and the Marangoni
  force on the cut layer is delta_m times the face difference of sigma;
- uniform sigma on a sphere centred on a grid node: the capillary forces
  cancel by symmetry, the Marangoni force vanishes, and the force summed
  across the interface along an axis is the Laplace jump -2 sigma / R."""
import itertools
import math

import numpy as np
import pytest

from oracle import capillary as K2
from oracle import capillary3d as K3
from oracle import oracle as O
from paper_2605_27534_amd import synth


def test_plic_areas_fixed_by_the_geometry():
    for c in (0.1, 0.37, 0.9):
        assert K3.plic_area([0.0, 0.0, 2.0], c) == 1.0
        assert K3.plic_area([0.0, -3.0, 0.0], c) == 1.0
    assert abs(K3.plic_area([1.0, 1.0, 1.0], 0.5) - 3 * math.sqrt(3) / 4) < 1e-14
    assert abs(K3.plic_area([1.0, -1.0, 0.0], 0.5) - math.sqrt(2)) < 1e-14
    # the corner tetrahedron x + y + z <= a has volume a^3/6 and the
    # equilateral face sqrt(3) a^2 / 2
    for a in (0.1, 0.5, 0.9):
        c = a ** 3 / 6
        assert abs(K3.plic_area([2.0, 2.0, 2.0], c) - math.sqrt(3) * a * a / 2) < 1e-12


def test_plic_plane_parallel_to_an_axis_is_the_2d_chord():
    for m2 in ((1.0, 2.0), (0.3, -0.7), (-1.0, 0.2)):
        for c in (0.02, 0.2, 0.5, 0.77, 0.99):
            a3 = K3.plic_area([m2[0], m2[1], 0.0], c)
            a2 = K2.plic_chord(m2, c)
            assert abs(a3 - a2) < 1e-13 * a2, (m2, c, a3, a2)
            # and along the other axes
            assert abs(K3.plic_area([0.0, m2[0], m2[1]], c) - a2) < 1e-13 * a2


def test_plic_complement_and_permutations():
    rng = np.random.default_rng(11)
    for _ in range(20):
        m = list(rng.normal(size=3))
        c = float(rng.uniform(0.01, 0.99))
        a = K3.plic_area(m, c)
        assert abs(K3.plic_area([-v for v in m], 1.0 - c) - a) < 1e-12 * a
        for p in itertools.permutations(range(3)):
            assert abs(K3.plic_area([m[i] for i in p], c) - a) < 1e-12 * a


def test_plic_volume_against_a_lattice_count():
    # the exact volume below the plane against the fraction of 96^3 lattice
    # points below it (error of order the area / 96)
    rng = np.random.default_rng(12)
    g = (np.arange(96) + 0.5) / 96
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    for _ in range(6):
        m = rng.normal(size=3)
        lo = min(m[0] * x + m[1] * y + m[2] * z for x in (0, 1) for y in (0, 1) for z in (0, 1))
        hi = max(m[0] * x + m[1] * y + m[2] * z for x in (0, 1) for y in (0, 1) for z in (0, 1))
        alpha = float(rng.uniform(lo, hi))
        exact = float(K3.plic_volume(list(m), alpha))
        count = float(np.mean(m[0] * X + m[1] * Y + m[2] * Z <= alpha))
        assert abs(exact - count) < 2.5e-2, (m, alpha, exact, count)
        # and A_f = |m| dV/dalpha against a difference quotient of the count
        da = 0.02 * (hi - lo)
        dq = (np.mean(m[0] * X + m[1] * Y + m[2] * Z <= alpha + da) -
              np.mean(m[0] * X + m[1] * Y + m[2] * Z <= alpha - da)) / (2 * da)
        c = exact
        if K3.interfacial(c):
            area = K3.plic_area(list(m), c)
            assert abs(area - np.linalg.norm(m) * dq) < 0.1 * area + 0.05, (area, dq)


def sphere(n, R=0.3, cen=(0.5, 0.5, 0.5), sub=32):
    h = 1.0 / n
    prob = dict(dim=3, n=(n, n, n), h=h, bc=((0, 0), (0, 0), (0, 0)))
    vof = synth.vof_ball((n, n, n), h, cen, R, 3, sub=sub)
    chi = O.geometry(prob, vof, 100)
    return prob, vof, chi


def test_sphere_area_and_curvature():
    R = 0.3
    prob, vof, chi = sphere(24, R)
    h = prob["h"]
    kap, dm = K3.cell_fields(prob, vof, chi)
    area = float(np.sum(dm)) * h ** 3
    # the Youngs normal's bias leaves the PLIC area about 1% off at this h
    assert abs(area - 4 * math.pi * R * R) < 0.02 * 4 * math.pi * R * R, area
    cut = (vof > 1e-6) & (vof < 1 - 1e-6)
    err = np.abs(kap[cut] * R / 2 + 1.0)
    assert err.max() < 0.03 and err.mean() < 0.01, (err.max(), err.mean())


def test_flat_interface_marangoni():
    n = 12
    h = 1.0 / n
    prob = dict(dim=3, n=(n, n, n), h=h, bc=((1, 1), (1, 1), (0, 0)))
    z = (np.arange(n) + 0.5) * h
    zi = 0.5 + 0.25 * h  # the interface inside layer 6
    vof = np.clip((zi - (z - 0.5 * h)) / h, 0.0, 1.0)
    vof = np.broadcast_to(vof[:, None, None], (n, n, n)).copy()
    chi = O.geometry(prob, vof, 60)
    x = (np.arange(n) + 0.5) * h
    sig = (1.0 + 0.1 * np.sin(2 * math.pi * x)[None, None, :] +
           0.05 * np.cos(2 * math.pi * x)[None, :, None]) * np.ones((n, n, n))
    kap, dm = K3.cell_fields(prob, vof, chi)
    k = int(zi / h)
    assert np.all(dm[k] == 1.0 / h) and np.all(dm[:k] == 0.0) and np.all(dm[k + 1:] == 0.0)
    assert np.all(kap == 0.0)
    cap, ma = K3.forces(prob, vof, chi, sig)
    assert max(np.max(np.abs(f)) for f in cap) == 0.0
    # the x faces of the cut layer: delta_m (1/h) times the face difference
    fx = ma[0][k, :, :n]
    dsig = (sig[k] - np.roll(sig[k], 1, axis=1)) / h
    assert np.max(np.abs(fx - dsig / h)) < 1e-12 * np.max(np.abs(dsig / h))
    fy = ma[1][k, :n, :]
    dsig = (sig[k] - np.roll(sig[k], 1, axis=0)) / h
    assert np.max(np.abs(fy - dsig / h)) < 1e-12 * np.max(np.abs(dsig / h))
    assert np.max(np.abs(ma[2])) < 1e-12


def test_capillary_balance_and_laplace_jump():
    n, R, s0 = 24, 0.3, 0.7
    prob, vof, chi = sphere(n, R)
    h = prob["h"]
    sig = np.full(vof.shape, s0)
    cap, ma = K3.forces(prob, vof, chi, sig)
    for d in range(3):
        scale = np.max(np.abs(cap[d]))
        assert abs(np.sum(cap[d])) < 1e-12 * scale * cap[d].size
        assert np.max(np.abs(ma[d])) == 0.0
    # along the x axis through the centre: sum F h over the right half
    c = n // 2
    for j, k in ((c - 1, c - 1), (c, c - 1), (c - 1, c), (c, c)):
        jump = float(np.sum(cap[0][k, j, c:])) * h
        assert abs(jump + 2 * s0 / R) < 0.05 * 2 * s0 / R, jump


def test_face_force_matches_the_whole_box():
    # the face-by-face form (used on boxes too large for the whole-box one)
    # gives the same values, bit for bit, on a ragged box with a wall, an open
    # side and a periodic axis, for the faces next to the interface, the
    # boundary faces and random others
    n = (14, 12, 10)
    h = 1.0 / n[0]
    prob = dict(dim=3, n=n, h=h, bc=((0, 2), (1, 1), (2, 0)))
    vof = synth.vof_ball(n, h, (0.45, 0.5 * n[1] * h, 0.4 * n[2] * h), 0.28, 3)
    chi = O.geometry(prob, vof, 60)
    sig = 1.0 + 0.2 * synth.smooth_modes(n, h, 31, dim=3)
    cap, ma = K3.forces(prob, vof, chi, sig)
    rng = np.random.default_rng(32)
    for d in range(3):
        shp = cap[d].shape
        picks = [tuple(rng.integers(s) for s in shp) for _ in range(60)]
        kk, jj, ii = np.nonzero(cap[d] != 0.0)
        picks += list(zip(kk[::3], jj[::3], ii[::3]))
        picks += [(0, 0, 0), tuple(s - 1 for s in shp)]
        for (k, j, i) in picks:
            fc, fm = K3.face_force(prob, vof, chi, sig, d, (int(i), int(j), int(k)))
            assert fc == cap[d][k, j, i] and fm == ma[d][k, j, i], (d, i, j, k)
