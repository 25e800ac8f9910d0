"""Pins of the oracle's geometry stage: the phase field and regularised delta
(section 2.5 eq. (redistance), section 2.6 delta estimate) and the
Hamilton-Jacobi redistancing from VoF (section 2.5)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_27534_amd import synth


def column_prob(ny, h, chi_max_eps=12.0):
    return dict(dim=2, n=(1, ny), h=h, bc=((1, 1), (0, 0)), chi_max_eps=chi_max_eps)


@pytest.mark.parametrize("offset", [0.0, 0.13, 0.25, 0.5, 0.77])
def test_delta_integrates_to_one_across_planar_interface(offset):
    # P1: the integral of |grad phi| across a planar tanh profile is exactly 1;
    # with eps = 1.5 h the midpoint sum is 1 to ~1e-11 whatever the offset
    # (Poisson summation: the first alias term is ~ 2 pi^2 eps/h e^{-pi^2 eps/h}).
    ny, h = 400, 1.0
    prob = column_prob(ny, h, chi_max_eps=1e6)
    y = (np.arange(ny) + 0.5) * h
    chi = -(y - (200.0 + offset) * h)
    phi, om, de = O.cell_geometry(prob, chi.reshape(1, ny, 1))
    assert abs(de.sum() * h - 1.0) < 1e-10
    # phi is the tanh profile of eq. (redistance), and phi + (1 - phi) = 1
    eps = 1.5 * h
    assert np.allclose(phi.ravel(), 0.5 * (1 - np.tanh(chi / (2 * eps))), rtol=0, atol=1e-15)
    assert np.allclose((phi + om).ravel(), 1.0, atol=1e-15)
    # phi -> 0 in fluid 1 (chi > 0) and -> 1 in the liquid
    assert phi.ravel()[0] < 1e-12 and phi.ravel()[-1] > 1 - 1e-12


def test_delta_clamp_contribution():
    # each clamped cell contributes exactly h phi(chi_max)(1 - phi(chi_max))/eps
    ny, h = 200, 1.0
    prob = column_prob(ny, h)
    y = (np.arange(ny) + 0.5) * h
    chi_exact = -(y - 100.0 * h)
    chi = np.clip(chi_exact, -18 * h, 18 * h)
    _, _, de = O.cell_geometry(prob, chi.reshape(1, ny, 1))
    eps = 1.5 * h
    pm = 1 / (1 + math.exp(12.0))
    nclamp = int(np.sum(np.abs(chi_exact) >= 18 * h))
    unclamped = de.ravel()[np.abs(chi_exact) < 18 * h].sum() * h
    # the unclamped part integrates to 1 minus the two tails beyond 12 eps
    # (each tail is phi(chi_max)); the truncated midpoint sum carries an
    # end correction of order h^2 delta'/12 ~ 2e-7 here
    tail = 2 * pm
    assert abs(unclamped - (1 - tail)) < 5e-7
    assert abs(de.sum() * h - unclamped - nclamp * pm * (1 - pm) / eps * h) < 1e-15


def face_aligned_prob(n, dim):
    return dict(dim=dim, n=(n,) * dim, h=1.0 / n, bc=((0, 0),) * dim)


@pytest.mark.parametrize("dim", [2, 3])
def test_face_aligned_interface_gives_exact_distance(dim):
    # P2: an interface lying on grid faces pins the two adjacent cells to
    # +-h/2 exactly, and the Godunov sweeps propagate an exact distance.
    n = 48 if dim == 2 else 40
    h = 1.0 / n
    prob = face_aligned_prob(n, dim)
    k0 = n // 2
    shape = O.shape(prob)
    y = (np.arange(n) + 0.5) * h
    vof = np.zeros(shape)
    vof[..., :k0, :] = 1.0  # fluid 1 below the face y = k0 h
    iters = 72 if dim == 2 else 108
    chi = O.geometry(prob, vof, iters)
    exact = np.broadcast_to((k0 * h - y)[:, None], shape[-2:])
    exact = np.broadcast_to(exact, shape)
    chimax = 12 * (1.5 * h)
    # round-off exact within 4 eps; the Jacobi relaxation is still
    # converging geometrically towards the clamp after N_init sweeps
    near = np.abs(exact) < 4 * 1.5 * h
    assert np.max(np.abs(chi - exact)[near]) < 1e-12 * h
    band = np.abs(exact) < chimax - 1.5 * h
    assert np.max(np.abs(chi - exact)[band]) < 1e-4 * h
    assert np.all(np.abs(chi) <= chimax)


def test_russo_smereka_subcell_estimate_quarter_cut():
    # A planar cut a quarter of a cell above the lower face: the cut cell has
    # chi0 = -h/4, its lower neighbour +h/2, upper -h/2.  The estimate
    # h chi0 / Delta uses Delta = max(|centred difference|, largest jump) =
    # 3h/4, giving -h/3 and +2h/3 (a bias of h/12 in the zero level).
    n = 32
    h = 1.0 / n
    prob = dict(dim=2, n=(4, n), h=h, bc=((1, 1), (0, 0)))
    k = 16
    vof = synth.vof_flat((4, n), h, (k + 0.25) * h)
    pin, D = O.pin_data(prob, vof)
    col_pin = pin[0, :, 0]
    assert list(np.nonzero(col_pin)[0]) == [k - 1, k]
    assert abs(D[0, k, 0] - (-h / 3)) < 1e-17
    assert abs(D[0, k - 1, 0] - 2 * h / 3) < 1e-17


def test_geometry_antisymmetric_in_vof_bitwise():
    # swapping the phases (f -> 1 - f, exact for dyadic f) flips the sign of
    # chi bitwise: both Godunov branches and the pin rule are mirror images.
    n = 64
    h = 1.0 / n
    prob = dict(dim=2, n=(n, n), h=h, bc=((0, 0), (2, 2)))
    f = synth.vof_ball((n, n), h, (0.43, 0.52, 0), 0.21, 2)
    a = O.geometry(prob, f, 40)
    b = O.geometry(prob, 1.0 - f, 40)
    assert np.array_equal(a, -b)


def test_geometry_commutes_with_periodic_shift():
    n = 48
    h = 1.0 / n
    prob = dict(dim=2, n=(n, n), h=h, bc=((1, 1), (1, 1)))
    f = synth.vof_ball((n, n), h, (0.5, 0.5, 0), 0.2, 2)
    a = O.geometry(prob, f, 50)
    b = O.geometry(prob, np.roll(np.roll(f, 7, axis=2), -5, axis=1), 50)
    assert np.array_equal(np.roll(np.roll(a, 7, axis=2), -5, axis=1), b)


@pytest.mark.parametrize("n", [64, 128])
def test_circle_distance_accuracy(n):
    # measured accuracy of the VoF -> distance map on a circle: the first-order
    # subcell estimate leaves errors below 0.3 h within 6 eps of the interface
    h = 1.0 / n
    prob = dict(dim=2, n=(n, n), h=h, bc=((0, 0), (0, 0)))
    f = synth.vof_ball((n, n), h, (0.5, 0.5, 0), 0.25, 2)
    chi = O.geometry(prob, f, 72)
    x, y, _ = synth.cell_centres((n, n), h)
    r = np.sqrt((x[None, None, :] - 0.5) ** 2 + (y[None, :, None] - 0.5) ** 2)
    ex = 0.25 - r
    band = np.abs(ex) < 6 * 1.5 * h
    assert np.max(np.abs(chi - ex)[band]) < 0.3 * h
    # sign agrees with the VoF everywhere outside the cut cells
    assert np.all(np.sign(chi[f == 1.0]) > 0) and np.all(np.sign(chi[f == 0.0]) < 0)


def test_warm_start_from_converged_field_is_stationary():
    # a converged distance field is a fixed point of further sweeps
    n = 64
    h = 1.0 / n
    prob = face_aligned_prob(n, 2)
    vof = np.zeros(O.shape(prob))
    vof[..., : n // 2, :] = 1.0
    chi = O.geometry(prob, vof, 200)
    again = O.geometry(prob, vof, 8, chi=chi)
    assert np.max(np.abs(again - chi)) < 1e-15
