"""Pins of the ACDI oracle (section 2.5, the Phase-Field method) against
facts it must reproduce, none of them a retyping of its flux:

- the flux form conserves sum(phi) exactly with walls and periodic sides;
- phi -> 1 - phi commutes with the step (the equation is odd in phi - 1/2)
  without flow and under a uniform flow on a periodic box (where the
  advection keeps a constant field exactly);
- the step commutes with periodic shifts;
- with zeta = 0 it is the substep-1 advection of the surfactant fields;
- the equilibrium profile phi = 1/(1 + e^{x/eps}) is steady: the residual
  of the discrete flux divergence vanishes at second order in h;
- a profile twice too wide relaxes to the equilibrium width (interface
  measure sum phi (1 - phi)/eps h -> 1 per unit length);
- phi stays in [0, 1], up to the regularization constant 1e-6 that keeps s
  finite, over a full period of translation with zeta >= |u|, and returns
  close to its start;
- on axisymmetric rings (Appendix B): the integral of phi over the ring
  volumes is conserved exactly with walls and a periodic axis, and a
  profile that varies along the axis only (no radial flux) takes the same
  step as on the Cartesian grid."""
import math

import numpy as np
import pytest

from oracle import acdi as A
from oracle import oracle as O
from paper_2605_27534_amd import synth


def circle(n=(48, 40), bc=((0, 0), (1, 1)), R=0.22, cen=(0.47, 0.52, 0), eps_h=1.5):
    nx, ny = n
    h = 1.0 / nx
    prob = dict(dim=2, n=n, h=h, bc=bc, eps=eps_h * h)
    vof = synth.vof_ball(n, h, cen, R, 2)
    chi = O.geometry(prob, vof, 60)
    return prob, A.phi_of_chi(prob, chi)


@pytest.mark.parametrize("bc", [((0, 0), (0, 0)), ((1, 1), (0, 0)), ((1, 1), (1, 1))])
def test_conserves_phi(bc):
    prob, phi = circle(bc=bc)
    h = prob["h"]
    u = synth.u_source2d(prob["n"], h, (0.5, 0.5, 0), 0.05)
    out = phi
    for _ in range(5):
        out = A.acdi_step(prob, out, u, 0.2 * h, 0.5)
    before, after = math.fsum(phi.ravel()), math.fsum(out.ravel())
    assert abs(after - before) <= 1e-13 * before
    assert not np.allclose(out, phi)


def test_complement_symmetry():
    prob, phi = circle(bc=((1, 1), (1, 1)))
    h = prob["h"]
    u = synth.u_uniform(prob["n"], 2, (0.7, -0.4))
    a = A.acdi_step(prob, phi, u, 0.2 * h, 1.1)
    b = A.acdi_step(prob, 1.0 - phi, u, 0.2 * h, 1.1)
    assert np.max(np.abs(b - (1.0 - a))) < 1e-13
    # without flow as well
    a = A.acdi_step(prob, phi, None, 0.2 * h, 1.1)
    b = A.acdi_step(prob, 1.0 - phi, None, 0.2 * h, 1.1)
    assert np.max(np.abs(b - (1.0 - a))) < 1e-13


def test_commutes_with_periodic_shifts():
    prob, phi = circle(bc=((1, 1), (1, 1)))
    h = prob["h"]
    u = synth.u_uniform(prob["n"], 2, (0.4, -0.25))
    a = np.roll(A.acdi_step(prob, phi, u, 0.3 * h, 0.6), (3, -5), axis=(1, 2))
    b = A.acdi_step(prob, np.roll(phi, (3, -5), axis=(1, 2)), u, 0.3 * h, 0.6)
    assert np.max(np.abs(a - b)) < 1e-14


def test_zero_zeta_is_the_advection():
    prob, phi = circle()
    h = prob["h"]
    u = synth.u_source2d(prob["n"], h, (0.5, 0.5, 0), 0.05)
    a = A.acdi_step(prob, phi, u, 0.3 * h, 0.0)
    b, _ = O.advect(prob, u, phi, 0.3 * h)
    assert np.array_equal(a, b)


def flat_profile(nx, eps, ny=4, tilt=0.0):
    # two flat interfaces on a periodic box in x (a slab of fluid 1 in the
    # middle half); chi the signed distance, phi the equilibrium profile
    h = 1.0 / nx
    prob = dict(dim=2, n=(nx, ny), h=h, bc=((1, 1), (1, 1)), eps=eps)
    x = (np.arange(nx) + 0.5) * h
    chi = 0.25 - np.abs(x - 0.5)  # > 0 inside the slab
    chi = np.broadcast_to(chi[None, None, :], (1, ny, nx)).copy()
    phi = 1.0 / (1.0 + np.exp(chi / eps))
    return prob, phi


def test_equilibrium_profile_is_steady_to_second_order():
    eps = 0.02
    res = []
    for nx in (128, 256, 512):
        prob, phi = flat_profile(nx, eps)
        dt = 1e-3
        r = (A.regularize(prob, phi, dt, 1.0) - phi) / dt
        res.append(np.max(np.abs(r)))
    orders = [math.log2(res[i] / res[i + 1]) for i in range(2)]
    assert all(1.85 < o < 2.15 for o in orders), (res, orders)
    # against the size of each of the two terms of the flux divergence
    prob, phi = flat_profile(512, eps)
    h = prob["h"]
    lap = (np.roll(phi, -1, 2) - 2 * phi + np.roll(phi, 1, 2)) / h ** 2
    assert res[-1] < 1e-3 * eps * np.max(np.abs(lap))


def test_wide_profile_relaxes_to_the_equilibrium_width():
    nx, ny = 128, 4
    h = 1.0 / nx
    eps = 1.5 * h
    prob = dict(dim=2, n=(nx, ny), h=h, bc=((1, 1), (1, 1)), eps=eps)
    x = (np.arange(nx) + 0.5) * h
    chi = np.broadcast_to((0.25 - np.abs(x - 0.5))[None, None, :], (1, ny, nx)).copy()
    phi = 1.0 / (1.0 + np.exp(chi / (2 * eps)))  # twice the width
    per_len = 2 * ny * h  # two interfaces, each ny h long
    m0 = A.profile_thickness(prob, phi) / per_len
    assert abs(m0 - 2.0) < 0.02
    dt = 0.2 * h * h / eps  # zeta eps dt / h^2 = 0.2 at zeta = 1
    ms = []
    for _ in range(400):
        phi = A.regularize(prob, phi, dt, 1.0)
        ms.append(A.profile_thickness(prob, phi) / per_len)
    assert all(ms[i + 1] <= ms[i] + 1e-12 for i in range(len(ms) - 1))
    assert abs(ms[-1] - 1.0) < 0.03, ms[-1]


def test_bounded_over_a_period_of_translation():
    prob, phi = circle(n=(64, 64), bc=((1, 1), (1, 1)), R=0.2, cen=(0.5, 0.5, 0))
    h = prob["h"]
    U = (1.0, 0.0)
    u = synth.u_uniform(prob["n"], 2, U)
    zeta = 1.1
    dt = 0.25 * h
    nsteps = int(round(1.0 / dt))  # one period along x
    out = phi
    lo, hi = 1.0, 0.0
    for _ in range(nsteps):
        out = A.acdi_step(prob, out, u, dt, zeta)
        lo, hi = min(lo, out.min()), max(hi, out.max())
    assert lo > -A.VAREPS and hi < 1.0 + A.VAREPS, (lo, hi)
    assert abs(math.fsum(out.ravel()) - math.fsum(phi.ravel())) < 1e-11 * math.fsum(phi.ravel())
    # the shape survives: interface measure and position
    assert abs(A.profile_thickness(prob, out) / A.profile_thickness(prob, phi) - 1) < 0.05
    assert np.max(np.abs(out - phi)) < 0.25


def test_tilted_equilibrium_profile_is_steady():
    # a flat interface at an angle (lines x + 2y = const, periodic on the
    # unit torus): the face normal needs its transverse components; its
    # residual matches the axis-aligned profile's at the same h and eps
    eps, nx = 0.01, 256
    h = 1.0 / nx
    x = (np.arange(nx) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    g = np.mod(X + 2 * Y, 1.0)
    chi = (0.25 - np.abs(g - 0.5)) / math.sqrt(5.0)  # signed distance to the slab
    prob = dict(dim=2, n=(nx, nx), h=h, bc=((1, 1), (1, 1)), eps=eps)
    phi = (1.0 / (1.0 + np.exp(chi / eps)))[None]
    dt = 1e-3
    tilted = np.max(np.abs(A.regularize(prob, phi, dt, 1.0) - phi)) / dt
    p1, ph1 = flat_profile(nx, eps)
    aligned = np.max(np.abs(A.regularize(p1, ph1, dt, 1.0) - ph1)) / dt
    assert tilted < 3.0 * aligned, (tilted, aligned)
    # the size of one term alone, for scale
    assert aligned < 1e-2 * np.max(np.abs(ph1 * (1 - ph1))) / eps / h


@pytest.mark.parametrize("r0", [0.0, 0.3])
def test_axisymmetric_conserves_the_ring_integral(r0):
    # a sphere on the axis (r0 = 0) or a torus about it (r0 = 0.3), walls on
    # both radial sides, periodic along the axis; a flow with a radial part
    n = (40, 48)
    h = 1.0 / 40
    prob = dict(dim=2, n=n, h=h, bc=((0, 0), (1, 1)), eps=1.5 * h, axisym=1,
                origin=(r0, 0.0, 0.0))
    vof = synth.vof_ball(n, h, (0.0 if r0 == 0 else 0.35, 0.5, 0), 0.25, 2)
    phi = A.phi_of_chi(prob, O.geometry(prob, vof, 60))
    u = synth.u_source2d(n, h, (0.5, 0.5, 0), 0.05)
    # ring volumes written out from the geometry of the rings
    r = r0 + (np.arange(n[0]) + 0.5) * h
    vol = (2.0 * math.pi * r * h * h)[None, None, :]
    out = phi
    for _ in range(5):
        out = A.acdi_step(prob, out, u, 0.2 * h, 0.6)
    before, after = math.fsum((phi * vol).ravel()), math.fsum((out * vol).ravel())
    assert abs(after - before) <= 1e-13 * before, (before, after)
    assert not np.allclose(out, phi)
    # without the ring weights the same step does not conserve it
    cart = dict(prob, axisym=0)
    outc = phi
    for _ in range(5):
        outc = A.acdi_step(cart, outc, u, 0.2 * h, 0.6)
    assert abs(math.fsum((outc * vol).ravel()) - before) > 1e-9 * before


def test_axisymmetric_axial_profile_matches_the_cartesian_step():
    # phi varies along the axis only: radial fluxes vanish, the axial faces
    # carry weight 1, so the rings step as the Cartesian grid does
    n = (24, 48)
    h = 1.0 / 48
    z = (np.arange(n[1]) + 0.5) * h
    phi = 1.0 / (1.0 + np.exp((z - 0.37) / (2.0 * h)))
    phi = np.broadcast_to(phi[None, :, None], (1, n[1], n[0])).copy()
    for bc in (((0, 2), (0, 0)), ((0, 0), (1, 1))):
        prob = dict(dim=2, n=n, h=h, bc=bc, eps=1.5 * h, axisym=1, origin=(0.1, 0.0, 0.0))
        a = A.acdi_step(prob, phi, None, 0.2 * h, 0.8)
        b = A.acdi_step(dict(prob, axisym=0), phi, None, 0.2 * h, 0.8)
        assert np.max(np.abs(a - phi)) > 1e-6
        assert np.max(np.abs(a - b)) == 0.0
