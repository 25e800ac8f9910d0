"""Parity of the axisymmetric (r, z) path (Appendix B; k_col2d with ring
weights, through the C ABI) with the FP64 oracle on the same seeded inputs:
fields relative max-norm (FP64 1e-12, FP32 2e-5) and the totals, which are
volume and area integrals over the rings."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_27534_amd import synth
from tests.harness import compare_totals, rel_max, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

F64, F32 = 1, 0
TOL = {F64: 1e-12, F32: 2e-5}


def compare(o, g, prec, bulk=True):
    chi_o, F_o, P_o, S_o, H_o = o
    chi_g, F_g, P_g, S_g, H_g, s = g
    pairs = [("chi", chi_g, chi_o), ("psi", P_g, P_o), ("sigma", S_g, S_o)]
    if bulk:
        pairs.append(("F", F_g, F_o))
    errs = {n: rel_max(a, b) for n, a, b in pairs}
    tol = TOL[prec]
    assert all(v <= tol for v in errs.values()), sorted(errs.items())
    compare_totals(H_g[-1], H_o[-1], tol, F_o if bulk else None, P_o)
    assert s.status() == 0
    return errs


@pytest.mark.parametrize("prec", [F64, F32])
def test_axisym_static_sphere(prec):
    n = (150, 131)
    h = 1.0 / 150
    prob = dict(dim=2, n=n, h=h, bc=((0, 2), (0, 0)), axisym=1, eos=0, eos_E=0.3,
                k_a=1.5, k_d=0.7)
    z0 = 0.47
    vof = synth.vof_ball(n, h, (0.0, z0, 0), 0.3, 2)
    dt = 0.2 * h * h / 1e-2
    c0 = synth.uniform_field(n, 4, 0.8, 1.2)
    o = run_oracle(prob, vof, 12, dt, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 12, dt, prec, c0=c0, gamma0=0.4)
    compare(o, g, prec)


@pytest.mark.parametrize("prec", [F64, F32])
def test_axisym_strain_flow_open_sides(prec):
    n = (130, 140)
    h = 1.0 / 130
    z0 = 0.55
    prob = dict(dim=2, n=n, h=h, bc=((0, 2), (2, 2)), axisym=1, eos=0, eos_E=0.2,
                k_a=1.0, k_d=0.5, origin=(0.0, 0.0, 0.0))
    vof = synth.vof_ball(n, h, (0.0, z0, 0), 0.25, 2)
    u = synth.u_axisym_strain(n, h, 0.3, z0)
    dt = 0.15 * h * h / 1e-2
    c0 = synth.uniform_field(n, 6, 0.8, 1.2)
    o = run_oracle(prob, vof, 10, dt, u=u, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 10, dt, prec, u=u, c0=c0, gamma0=0.4)
    compare(o, g, prec)
    assert o[4][-1][O.T_OUTCUM] != 0.0  # the open sides carried surfactant


@pytest.mark.parametrize("prec", [F64, F32])
def test_axisym_translating_sphere_moving_geometry(prec):
    # a sphere on the axis carried along it by a uniform axial flow, the
    # VoF recomputed every step (the moving 2D geometry path), an annular
    # domain starting off the axis is not needed: the rings start at r = 0
    n = (96, 160)
    h = 1.0 / 96
    U = 0.4
    dt = 0.15 * h * h / 1e-2
    z0 = 0.45
    prob = dict(dim=2, n=n, h=h, bc=((0, 2), (2, 2)), axisym=1, eos=0, eos_E=0.2,
                k_a=1.0, k_d=0.5)
    vof = synth.vof_ball(n, h, (0.0, z0, 0), 0.22, 2)
    seq = lambda k: synth.vof_ball(n, h, (0.0, z0 + U * (k + 1) * dt, 0), 0.22, 2)
    u = synth.u_uniform(n, 2, (0.0, U))
    c0 = synth.uniform_field(n, 9, 0.8, 1.2)
    o = run_oracle(prob, vof, 8, dt, u=u, vof_seq=seq, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 8, dt, prec, u=u, vof_seq=seq, c0=c0, gamma0=0.4)
    compare(o, g, prec)


@pytest.mark.parametrize("prec", [F64, F32])
@pytest.mark.parametrize("flow", [False, True], ids=["static", "strain"])
def test_axisym_paper_form(flow, prec):
    # the paper's flux form on the rings (k_step2d with ring weights): a
    # sphere on the axis, walls or open sides, with and without the strain
    # flow (ragged 64 x 16 tiles in both directions)
    n = (100, 121)
    h = 1.0 / 100
    z0 = 0.55
    prob = dict(dim=2, n=n, h=h, bc=((0, 2), (2, 2) if flow else (0, 0)), axisym=1,
                flux_form=1, eos=1, eos_E=0.2, k_a=1.0, k_d=0.5)
    vof = synth.vof_ball(n, h, (0.0, z0, 0), 0.27, 2)
    u = synth.u_axisym_strain(n, h, 0.3, z0) if flow else None
    dt = 0.1 * h * h / 1e-2
    c0 = synth.uniform_field(n, 7, 0.8, 1.2)
    o = run_oracle(prob, vof, 10, dt, u=u, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 10, dt, prec, u=u, c0=c0, gamma0=0.4)
    compare(o, g, prec)
    if flow:
        assert o[4][-1][O.T_OUTCUM] != 0.0


@pytest.mark.parametrize("prec", [F64, F32])
def test_axisym_paper_form_moving_geometry(prec):
    # the paper form on the rings with the VoF recomputed every step (FP32:
    # the fused tile step with its in-tile redistancing; FP64: the geometry
    # kernels, then the static tile step), an annular box off the axis
    n = (80, 130)
    h = 1.0 / 96
    U = 0.4
    dt = 0.1 * h * h / 1e-2
    z0 = 0.5
    r0 = 0.1
    prob = dict(dim=2, n=n, h=h, bc=((0, 2), (2, 2)), axisym=1, flux_form=1, eos=0,
                eos_E=0.2, k_a=1.0, k_d=0.5, origin=(r0, 0.0, 0.0))
    ball = lambda zc: synth.vof_ball(n, h, (0.45, zc, 0), 0.2, 2, origin=(r0, 0.0, 0.0))
    vof = ball(z0)
    seq = lambda k: ball(z0 + U * (k + 1) * dt)
    u = synth.u_uniform(n, 2, (0.0, U))
    c0 = synth.uniform_field(n, 10, 0.8, 1.2)
    o = run_oracle(prob, vof, 8, dt, u=u, vof_seq=seq, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 8, dt, prec, u=u, vof_seq=seq, c0=c0, gamma0=0.4)
    compare(o, g, prec)


@pytest.mark.parametrize("prec", [F64, F32])
@pytest.mark.parametrize("variant", [(1, 0), (0, 1), (1, 1)], ids=["mc", "transverse", "mc-transverse"])
def test_axisym_advection_variants(variant, prec):
    # the substep-1 variants on the rings (Cartesian face values, ring
    # weights on the divergence), under the straining flow with open sides
    lim, tr = variant
    n = (130, 140)
    h = 1.0 / 130
    z0 = 0.55
    prob = dict(dim=2, n=n, h=h, bc=((0, 2), (2, 2)), axisym=1, eos=0, eos_E=0.2,
                k_a=1.0, k_d=0.5, limiter=lim, bcg_transverse=tr)
    vof = synth.vof_ball(n, h, (0.0, z0, 0), 0.25, 2)
    u = synth.u_axisym_strain(n, h, 0.3, z0)
    dt = 0.15 * h * h / 1e-2
    c0 = synth.uniform_field(n, 6, 0.8, 1.2)
    o = run_oracle(prob, vof, 10, dt, u=u, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 10, dt, prec, u=u, c0=c0, gamma0=0.4)
    compare(o, g, prec)


# The implicit substep 2 (Appendix C) on the rings: the CG rows scaled by the
# ring radius (a symmetric matrix), substep 1 with the ring weights
@pytest.mark.parametrize("prec", [F64, F32])
@pytest.mark.parametrize("flow", ["strain", "axial"])
@pytest.mark.parametrize("form", [0, 1], ids=["weighted", "paper"])
def test_axisym_implicit(form, flow, prec):
    # form 1: the paper's flux, BiCGSTAB with the radial faces weighted
    from oracle import implicit as I
    from tests.harness import default_hj_init
    from tests.test_gpu_implicit import CG, CG_P, compare_paper
    n = (130, 140)
    h = 1.0 / 130
    z0 = 0.55
    if flow == "strain":
        bc = ((0, 2), (2, 2))
        u = synth.u_axisym_strain(n, h, 0.3, z0)
        eos = 1  # Langmuir
    else:
        # walls and a periodic axis: this case drives Gamma to within 1e-3 of
        # Gamma_inf, where the Langmuir EoS multiplies Gamma's FP32 rounding
        # by Gamma_inf / (Gamma_inf - Gamma); the tanh EoS is well conditioned
        bc = ((0, 0), (1, 1))
        u = synth.u_uniform(n, 2, (0.0, 0.3))
        eos = 2
    prob = dict(dim=2, n=n, h=h, bc=bc, axisym=1, eos=eos, eos_E=0.3, kinetics=0,
                D_b=1e-2, D_s=2e-3, k_a=1.5, k_d=0.7, substep2=1, flux_form=form,
                **(CG_P if form else CG)[prec])
    vof = synth.vof_ball(n, h, (0.0, z0, 0), 0.25, 2)
    c0 = synth.uniform_field(n, 6, 0.8, 1.2)
    dt = 10 * 0.2 * h * h / 1e-2  # ten times the explicit diffusive step
    q = O.full(prob)
    chi = O.geometry(prob, vof, default_hj_init(q))
    F, P = O.init_state(prob, chi, c0=c0, gamma0=0.4)
    o = I.run(prob, chi, u, F, P, dt, 4, picard=3)
    g = run_gpu(prob, vof, 4, dt, prec, u=u, c0=c0, gamma0=0.4)
    if form:
        compare_paper(o, g, prec, 1.5 * h)
    else:
        compare(o, g, prec)
    if flow == "strain":
        assert o[4][-1][O.T_OUTCUM] != 0.0  # the open sides carried surfactant


# The ACDI interface (section 2.5) on the rings, with either substep 2: a
# sphere carried along the axis, re-initialized from the VoF at step 3
@pytest.mark.parametrize("prec", [F64, F32])
@pytest.mark.parametrize("substep2", [0, 1, "paper"], ids=["explicit", "implicit", "paper"])
def test_axisym_acdi(substep2, prec):
    from tests.test_gpu_acdi import compare as acdi_compare
    from tests.test_gpu_acdi import run_both
    from tests.test_gpu_implicit import CG
    n = (96, 160)
    h = 1.0 / 96
    U = 0.4
    z0 = 0.45
    u = synth.u_uniform(n, 2, (0.0, U))
    # implicit: above the explicit surfactant bound, below the ACDI one;
    # "paper": the paper's flux form, explicit, at a smaller step
    paper = substep2 == "paper"
    substep2 = 0 if paper else substep2
    dt = 0.15 * h * h / 1e-2 * (1.5 if substep2 else (0.7 if paper else 1))
    prob = dict(dim=2, n=n, h=h, bc=((0, 2), (1, 1)), axisym=1, eos=1, eos_E=0.2,
                k_a=1.0, k_d=0.5, acdi_zeta=1.1 * U, substep2=substep2,
                flux_form=1 if paper else 0, **(CG[prec] if substep2 else {}))
    ball = lambda t: synth.vof_ball(n, h, (0.0, z0 + U * t, 0), 0.22, 2)
    reinit = lambda k: ball(k * dt) if k == 3 else None
    o, g = run_both(prob, ball(0.0), 7, dt, prec, u=u, reinit=reinit,
                    c0=synth.uniform_field(n, 8, 0.8, 1.2))
    delta_tol = None
    if prec == F32:
        # phi is stored in FP32 and the liquid around the bubble has phi near
        # 1, where a float resolves 1 - phi only to 2^-24: every ACDI step
        # since the re-initialization (and the initialization) may move
        # 1 - phi, and with it delta ~ (1 - phi)/eps, by that much in every
        # cell.  On the rings the far field holds most of the volume, so the
        # integral of delta can move by (k + 1) 2^-24 V / eps (k = 3 steps,
        # V the volume of the box), relative to the oracle's integral
        q = O.full(prob)
        V = math.pi * ((n[0] * h) ** 2) * (n[1] * h)
        delta_tol = TOL[F32] + 4 * 2.0 ** -24 * V / q["eps"] / o[5][-1][O.T_SDELTA]
    acdi_compare(o, g, prec, 1.5 * h, delta_tol=delta_tol)
