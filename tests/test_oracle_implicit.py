"""Pins of the implicit substep-2 oracle (Appendix C, weighted flux form)
against facts it must reproduce, none of them a retyping of its assembly:

- the implicit equations hold for its result when evaluated with the
  explicit oracle's own flux and source code (an independent C routine);
- a Fourier mode in a uniform bulk decays by the closed-form implicit-Euler
  factor 1 / (1 + dt D lambda_m) of the discrete Laplacian;
- with walls and no flow, the total amount F + psi is conserved;
- it agrees with the explicit step to second order as dt -> 0.

Each also runs on axisymmetric rings (Appendix B), where the explicit
oracle's C routine carries the ring weights of its own, and the conserved
total is the integral over the ring volumes."""
import math

import numpy as np
import pytest

from oracle import implicit as I
from oracle import oracle as O
from paper_2605_27534_amd import synth


def circle_case(n=(40, 32), bc=((0, 0), (1, 1)), kinetics=0, axisym=False):
    nx, ny = n
    h = 1.0 / nx
    prob = dict(dim=2, n=n, h=h, bc=bc, kinetics=kinetics, eos=1, eos_E=0.3,
                D_b=1e-2, D_s=2e-3, k_a=2.0, k_d=0.7)
    cen = (0.48, 0.41, 0)
    if axisym:
        # a sphere on the axis: rings r in [0.05, 1.05] (x the radius), the
        # ball centred at r = 0.05
        prob.update(axisym=1, origin=(0.05, 0.0, 0.0))
        cen = (0.0, 0.41, 0)
    vof = synth.vof_ball(n, h, cen, 0.21, 2)
    chi = O.geometry(prob, vof, 60)
    c0 = synth.uniform_field(n, 4, 0.8, 1.2)
    F, P = O.init_state(prob, chi, c0=c0, gamma0=0.4)
    return prob, chi, F, P


@pytest.mark.parametrize("kinetics,axisym,form", [(0, False, 0), (1, False, 0), (0, True, 0),
                                                  (1, True, 0), (0, False, 1), (1, False, 1)])
def test_converged_picard_satisfies_the_implicit_equations(kinetics, axisym, form):
    prob, chi, F, P = circle_case(kinetics=kinetics, axisym=axisym)
    prob["flux_form"] = form
    h = prob["h"]
    dt = 20 * 0.2 * h * h / 1e-2  # twenty times the explicit diffusive step
    Fn, Pn, _, _ = I.implicit_step(prob, chi, None, F, P, dt, picard=60)
    # the explicit oracle advances (Fn, Pn) by dt' with div(flux) -/+ q
    # evaluated at (Fn, Pn): its increment over dt' is the right-hand side
    dtp = 1e-3
    Fe, Pe, _, _ = O.step(prob, chi, None, Fn, Pn, dtp)
    rhsF, rhsP = (Fe - Fn) / dtp, (Pe - Pn) / dtp
    lhsF, lhsP = (Fn - F) / dt, (Pn - P) / dt
    for lhs, rhs in ((lhsF, rhsF), (lhsP, rhsP)):
        err = np.max(np.abs(lhs - rhs)) / np.max(np.abs(lhs))
        assert err < 1e-9, err


def test_fourier_mode_decays_by_the_implicit_euler_factor():
    # phi uniform (chi at -chi_max everywhere), no exchange, periodic in x
    nx, ny = 48, 4
    h = 1.0 / nx
    prob = dict(dim=2, n=(nx, ny), h=h, bc=((1, 1), (1, 1)), D_b=1e-2, D_s=1e-3,
                k_a=0.0, k_d=0.0)
    q = O.full(prob)
    chi = np.full(O.shape(prob), -q["chi_max_eps"] * q["eps"])
    phi, _, _ = O.cell_geometry(prob, chi)
    m = 3
    x = (np.arange(nx) + 0.5) * h
    c0 = np.cos(2 * math.pi * m * x)[None, None, :] * np.ones(O.shape(prob))
    F = (phi + q["eta"]) * c0
    P = np.zeros(O.shape(prob))
    dt = 0.5
    Fn, _, _, _ = I.implicit_step(prob, chi, None, F, P, dt, picard=1)
    lam = 4.0 * math.sin(math.pi * m / nx) ** 2 / h ** 2
    ph = float(phi.ravel()[0])
    factor = 1.0 / (1.0 + dt * q["D_b"] * ph * lam / (ph + q["eta"]))
    err = np.max(np.abs(Fn - factor * F)) / np.max(np.abs(F))
    assert err < 1e-12, err


@pytest.mark.parametrize("kinetics,axisym,form", [(0, False, 0), (1, False, 0), (0, True, 0),
                                                  (1, True, 0), (0, False, 1), (1, False, 1)])
def test_total_amount_conserved_with_walls(kinetics, axisym, form):
    prob, chi, F, P = circle_case(bc=((0, 0), (0, 0)), kinetics=kinetics, axisym=axisym)
    prob["flux_form"] = form
    h = prob["h"]
    dt = 50 * 0.2 * h * h / 1e-2
    Fn, Pn, _, tot = I.implicit_step(prob, chi, None, F, P, dt, picard=60)
    if axisym:
        # ring volumes 2 pi r_i h^2, written out here from the geometry
        r = 0.05 + (np.arange(prob["n"][0]) + 0.5) * h
        vol = (2.0 * math.pi * r * h * h)[None, None, :]
    else:
        vol = h * h
    before = math.fsum((F * vol).ravel()) + math.fsum((P * vol).ravel())
    after = math.fsum((Fn * vol).ravel()) + math.fsum((Pn * vol).ravel())
    assert abs(after - before) <= 1e-12 * abs(before)
    assert tot[O.T_NBAD] == 0
    # the totals integrate over the same volumes
    assert abs(tot[O.T_MB] + tot[O.T_MS] - after) <= 1e-12 * abs(after)


@pytest.mark.parametrize("axisym,form", [(False, 0), (True, 0), (False, 1)])
def test_second_order_agreement_with_the_explicit_step(axisym, form):
    prob, chi, F, P = circle_case(bc=((0 if axisym else 2, 2), (1, 1)), axisym=axisym)
    prob["flux_form"] = form
    h = prob["h"]
    u = synth.u_source2d((40, 32), h, (0.48, 0.41, 0), 0.03)
    errs = []
    # dt small against the exchange rate k_a Gamma_inf / eps (~50 here)
    for dt in (0.01 * h * h / 1e-2, 0.005 * h * h / 1e-2):
        Fi, Pi, _, ti = I.implicit_step(prob, chi, u, F, P, dt, picard=60)
        Fe, Pe, _, te = O.step(prob, chi, u, F, P, dt)
        errs.append(max(np.max(np.abs(Fi - Fe)), np.max(np.abs(Pi - Pe))))
        # substep 1 is the same explicit advection in both: the same outflow
        # and the same largest cell-mean velocity
        assert abs(ti[O.T_OUT] - te[O.T_OUT]) <= 1e-12 * (abs(te[O.T_MB]) + abs(te[O.T_MS]))
        assert abs(ti[O.T_SU] - te[O.T_SU]) <= 1e-14 * te[O.T_SU]
    order = math.log2(errs[0] / errs[1])
    assert 1.85 < order < 2.15, (errs, order)
