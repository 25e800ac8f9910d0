"""Pins of the oracle's exchange kinetics on the flat-interface problems of
section 4.3 (no flow, bulk diffusion plus adsorption/desorption), run as a
4-cell-wide periodic strip across [-4, 4] with the liquid above y = 0.
Scalings: Gamma_inf = F_inf = D_b = 1, so Da = k_a, Bi = k_d, t is the
paper's dimensionless time and y its dimensionless distance."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import analytic as A
from paper_2605_27534_amd import synth


def flat(N, kin, ka, kd, F0, G0, T):
    h = 8.0 / N
    nx = 4
    prob = dict(dim=2, n=(nx, N), h=h, bc=((1, 1), (0, 0)), kinetics=kin, k_a=ka,
                k_d=kd, D_b=1.0, D_s=1.0, gamma_inf=1.0)
    org = (0.0, -4.0, 0.0)
    f = synth.vof_flat((nx, N), h, 0.0, origin=org)
    chi = O.geometry(prob, f, 72)
    _, y, _ = synth.cell_centres((nx, N), h, org)
    phi, _, de = O.cell_geometry(prob, chi)
    F, P = F0 * phi, G0 * de
    eps = 1.5 * h
    lam = (3 + math.cosh(1 / 1.5)) / h ** 2 + ka / eps + ka + kd
    dt = 0.8 / lam
    steps = int(math.ceil(T / dt))
    dt = T / steps
    _, F2, P2, _, hist = O.run(prob, chi, None, F, P, dt, steps)
    G = hist[:, O.T_MS] / (nx * h)           # interfacial amount per unit length
    t = (np.arange(steps) + 1) * dt
    c = (F2 / (phi + 1e-12))[0, :, 0]
    mtot = hist[:, O.T_MTOT]
    return t, G, y, c, mtot


def test_reference_solver_reproduces_henry_closed_form():
    # the 1D sharp-interface reference (used below for Langmuir) reproduces the
    # closed form of section 4.3.1 when the saturation factor is dropped
    t = np.array([0.1, 0.5, 1.0])
    g, _, _ = A.langmuir_1d_reference(1.0, 0.0, t, length=6.0, n=1200, saturation=False)
    assert np.max(np.abs(g - A.henry_gamma(t, 1.0))) < 2e-4


def test_henry_closed_form_identities():
    # dGamma/dt = Da F(0, t) and F solves the Robin problem F_y(0) = Da F(0)
    Da, t, e = 0.5, 0.7, 1e-5
    dG = (A.henry_gamma(t + e, Da) - A.henry_gamma(t - e, Da)) / (2 * e)
    assert abs(dG - Da * A.henry_bulk(0.0, t, Da)) < 1e-8
    dF = (A.henry_bulk(e, t, Da) - A.henry_bulk(-e, t, Da)) / (2 * e)
    assert abs(dF - Da * A.henry_bulk(0.0, t, Da)) < 1e-8


@pytest.mark.parametrize("N,bound_g,bound_f", [(64, 0.05, 0.02), (128, 0.016, 0.007)])
def test_constant_adsorption_flux_converges(N, bound_g, bound_f):
    # section 4.3.1, Da = 1: Gamma(t) and the bulk profile approach the erf
    # closed forms; measured Gamma errors at t = 1: 0.106 (32), 0.040 (64),
    # 0.0129 (128); bulk 0.029, 0.015, 0.0055
    t, G, y, c, mtot = flat(N, 1, 1.0, 0.0, 1.0, 0.0, 1.0)
    assert abs(G[-1] - A.henry_gamma(t[-1], 1.0)) < bound_g
    m = y > 0.5
    assert np.max(np.abs(c[m] - A.henry_bulk(y[m], t[-1], 1.0))) < bound_f
    assert abs(mtot[-1] - mtot[0]) < 1e-13 * mtot[0]


@pytest.mark.parametrize("N,bound_f", [(64, 0.016), (128, 0.0035)])
def test_pure_desorption_converges(N, bound_f):
    # section 4.3.2, Bi = 1: Gamma = e^{-t}; bulk enrichment follows the
    # integral closed form; measured bulk errors 0.053 (32), 0.013 (64),
    # 0.0027 (128) -- second order
    t, G, y, c, _ = flat(N, 0, 0.0, 1.0, 0.0, 1.0, 1.0)
    assert np.max(np.abs(G - A.desorption_gamma(t, 1.0))) < 1e-3
    m = (y > 0.5) & (y < 3.0)
    assert np.max(np.abs(c[m] - A.desorption_bulk(y[m], t[-1], 1.0))) < bound_f


@pytest.mark.parametrize("N,bound", [(64, 0.016), (128, 0.006)])
def test_langmuir_against_1d_reference(N, bound):
    # section 4.3.3, Da = Bi = 1: Gamma(t) against the 1D second-order FV +
    # BDF reference over t in [0, 2]; measured 0.030 (32), 0.013 (64),
    # 0.0046 (128)
    t, G, y, c, _ = flat(N, 0, 1.0, 1.0, 1.0, 0.0, 2.0)
    ref, _, _ = A.langmuir_1d_reference(1.0, 1.0, t[::10], length=4.0)
    assert np.max(np.abs(G[::10] - ref)) < bound
    # heading for the section 4.3.3 equilibrium Da/(Da+Bi), reduced by depletion
    assert 0.38 < G[-1] < A.langmuir_gamma_eq(1.0, 1.0)
