"""Pins of the axisymmetric oracle (Appendix B: ring volumes, radial fluxes
weighted by the face radius) against facts it must reproduce:

- exact conservation of the total amount (ring volumes) with walls, in
  either flux form;
- a uniform field stays uniform under a flow that is divergence free in the
  axisymmetric sense (u_r = a r, u_z = -2 a z), which the Cartesian weights
  would not keep;
- the interface measure of a flat interface z = z0 over a disc of radius R
  is pi R^2 (each column carries sum delta h = 1);
- the Bessel mode J0(k r), J1(k R) = 0, decays at the rate D k^2 of the
  continuous cylindrical Laplacian, to second order in h."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import oracle as O
from paper_2605_27534_amd import synth


def axi_prob(nr, nz, R=1.0, bc=((0, 0), (0, 0)), **kw):
    h = R / nr
    return dict(dim=2, n=(nr, nz), h=h, bc=bc, axisym=1, **kw)


@pytest.mark.parametrize("form", [0, 1], ids=["weighted", "paper"])
def test_conserves_the_total_amount(form):
    prob = axi_prob(40, 48, bc=((0, 0), (0, 0)), eos=1, eos_E=0.3, k_a=1.5, k_d=0.7,
                    flux_form=form)
    h = prob["h"]
    z0 = 0.6
    vof = synth.vof_ball(prob["n"], h, (0.0, z0, 0), 0.35, 2)  # a sphere on the axis
    chi = O.geometry(prob, vof, 60)
    c0 = synth.uniform_field(prob["n"], 4, 0.8, 1.2)
    F, P = O.init_state(prob, chi, c0=c0, gamma0=0.4)
    u = synth.u_axisym_strain(prob["n"], h, 0.3, z0)
    tot = np.zeros(16)
    F1, P1, _, tot1 = O.step(prob, chi, None, F, P, 1e-4, tot.copy())
    m0 = tot1[O.T_MTOT]
    for _ in range(5):
        F1, P1, _, tot1 = O.step(prob, chi, u, F1, P1, 0.2 * h * h / 1e-2, tot1)
    assert abs(tot1[O.T_MTOT] - m0) <= 1e-13 * m0, (tot1[O.T_MTOT], m0)
    assert tot1[O.T_OUTCUM] == 0.0


def test_uniform_field_kept_by_an_axisymmetric_divergence_free_flow():
    prob = axi_prob(32, 40, bc=((0, 2), (2, 2)))
    h = prob["h"]
    u = synth.u_axisym_strain(prob["n"], h, 0.4, 0.7)
    xi = np.ones(O.shape(prob))
    xs, _ = O.advect(prob, u, xi, 0.3 * h)
    assert np.max(np.abs(xs - 1.0)) < 1e-14
    # the Cartesian balance of the same face values does not keep it
    xc, _ = O.advect(dict(prob, axisym=0), u, xi, 0.3 * h)
    assert np.max(np.abs(xc - 1.0)) > 1e-3


def test_flat_interface_measure_is_the_disc_area():
    R = 0.8
    prob = axi_prob(32, 64, R=R, bc=((0, 0), (0, 0)))
    h = prob["h"]
    vof = synth.vof_flat(prob["n"], h, 0.4 * 64 * h)
    chi = O.geometry(prob, vof, 80)
    F, P = O.init_state(prob, chi, c0=None, gamma0=0.0)
    _, _, _, tot = O.step(prob, chi, None, F, P, 1e-6, np.zeros(16))
    # per column sum delta h is 1 up to the clamp tails (pinned in the
    # Cartesian tests); the ring volumes turn the columns into pi R^2
    col = np.sum(O.cell_geometry(prob, chi)[2][0, :, 0]) * h
    assert abs(tot[O.T_SDELTA] - math.pi * R * R * col) <= 1e-12 * math.pi * R * R
    assert abs(col - 1.0) < 1e-3  # the clamp tails add about 1e-4


@pytest.mark.parametrize("dummy", [0])
def test_bessel_mode_decays_at_the_cylindrical_rate(dummy):
    R, D = 1.0, 1e-2
    k = special.jn_zeros(1, 1)[0] / R  # J0'(kR) = -J1(kR) = 0: no flux at r = R
    rates = []
    for nr in (32, 64, 128):
        prob = axi_prob(nr, 4, R=R, bc=((0, 0), (1, 1)), D_b=D, k_a=0.0, k_d=0.0)
        h = prob["h"]
        q = O.full(prob)
        chi = np.full(O.shape(prob), -q["chi_max_eps"] * q["eps"])  # all liquid
        r = (np.arange(nr) + 0.5) * h
        c = np.broadcast_to(special.j0(k * r)[None, None, :], O.shape(prob)).copy()
        phi, _, _ = O.cell_geometry(prob, chi)
        F = (phi + q["eta"]) * c
        P = np.zeros(O.shape(prob))
        dt = 1e-6
        F1, _, _, _ = O.step(prob, chi, None, F, P, dt, np.zeros(16))
        V = 2 * math.pi * r * h * h
        lam = np.sum(V * c * (F1 - F) / dt) / np.sum(V * c * F)
        rates.append(lam)
    exact = -D * k * k
    errs = [abs(x - exact) for x in rates]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-3 * abs(exact), (rates, exact)
    assert all(1.8 < o < 2.2 for o in orders), (errs, orders)
