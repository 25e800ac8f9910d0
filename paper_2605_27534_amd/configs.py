"""The five benchmark workloads as plain problem descriptions.

Each function returns a dict with the problem (the keys of the library's
parameter structs), the time step, the step count and callables producing the
seeded inputs (FP64 NumPy from `synth`; the 3D sphere also has the same
inputs generated on a torch device, from `synth_dev`).  Time steps are fixed numbers
chosen at or below the explicit stability bound of the split step (the bound
is the library's SURF_T_DT_NEXT; the values below were read from it for the
analytic velocity fields and rounded down).
"""
from __future__ import annotations

import math

import numpy as np

from . import synth, synth_dev


def c0_static_circle():
    """128^2 FP64, unit box, walls, static circle R = 0.25, u = 0, Langmuir
    kinetics k_a = k_d = Gamma_inf = 1, D_b = 1e-2, D_s = 1e-3, linear EoS
    sigma = 1 - 0.5 Gamma; F0 = phi (c = 1 in the liquid), psi0 = 0;
    200 steps at dt = 0.2 h^2 / D_b."""
    n = 128
    h = 1.0 / n
    prob = dict(dim=2, n=(n, n), h=h, bc=((0, 0), (0, 0)), eos=0, eos_E=0.5, sigma0=1.0,
                k_a=1.0, k_d=1.0, gamma_inf=1.0, D_b=1e-2, D_s=1e-3)
    return dict(name="static circle 128^2 fp64", prob=prob, precision=1,
                dt=0.2 * h * h / 1e-2, steps=200,
                vof0=lambda: synth.vof_ball((n, n), h, (0.5, 0.5, 0), 0.25, 2),
                vof_seq=None, u=None, c0=None, c0_const=1.0, gamma0=0.0, hj_step=8)


def c1_expanding_circle(n=1024, soluble=True, dt=None, extra=None, name=None):
    """1024^2 FP32, open box, circle R(t) = sqrt(R0^2 + Q t / pi), R0 = 0.1,
    Q = 0.05, centred, under the 2D source flow (core radius 0.02); VoF at
    t^{n+1} each step; Gamma0 = 0.5; c0 ~ U[0.8, 1.2] (seed 1) in the liquid;
    Langmuir EoS sigma0 = 1, E = 0.2; kinetics and diffusivities as the static
    circle; 2000 steps.  The insoluble variant switches the bulk off."""
    h = 1.0 / n
    R0, Q = 0.1, 0.05
    prob = dict(dim=2, n=(n, n), h=h, bc=((2, 2), (2, 2)), eos=1, eos_E=0.2, sigma0=1.0,
                k_a=1.0, k_d=1.0, gamma_inf=1.0, D_b=1e-2, D_s=1e-3,
                bulk_enabled=1 if soluble else 0)
    # explicit bound at 1024^2: substep 2 limits (soluble 1.776e-5, insoluble 1.803e-4)
    if dt is None:
        dt = (1.77e-5 if soluble else 1.80e-4) * (1024.0 / n) ** 2
    prob.update(extra or {})
    Rt = lambda t: math.sqrt(R0 ** 2 + Q * t / math.pi)
    return dict(name=name or "expanding circle %d^2 fp32 %s" % (n, "soluble" if soluble else "insoluble"),
                prob=prob, precision=0, dt=dt, steps=2000, R=Rt,
                vof0=lambda: synth.vof_ball((n, n), h, (0.5, 0.5, 0), R0, 2),
                vof_seq=lambda k: synth.vof_ball((n, n), h, (0.5, 0.5, 0), Rt((k + 1) * dt), 2),
                u=lambda: synth.u_source2d((n, n), h, (0.5, 0.5, 0), Q),
                c0=lambda: synth.uniform_field((n, n), 1, 0.8, 1.2) if soluble else None,
                c0_const=1.0, gamma0=0.5, hj_step=8)


def c1_implicit(n=1024, steps=100):
    """The soluble expanding circle with substep 2 implicit (section 3,
    Appendix C): dt = 8.5e-4 at 1024^2 (48 times the explicit step; the
    advective bound 0.5 h / S_u with S_u = 0.562 is 8.69e-4), 3 Picard sweeps,
    each linear solve to ||M^-1 r|| <= 1e-9 ||x||, at most 400 CG iterations;
    100 steps."""
    dt = 8.5e-4 * (1024.0 / n)
    cfg = c1_expanding_circle(n, soluble=True, dt=dt,
                              extra=dict(substep2=1, picard_iters=3, cg_tol=1e-9,
                                         cg_max_iters=400),
                              name="expanding circle %d^2 fp32 soluble implicit" % n)
    cfg["steps"] = steps
    return cfg


def c1_acdi(n=1024, reinit_every=50):
    """The soluble expanding circle with the ACDI interface (section 2.5): phi
    advanced by one ACDI step per step with zeta = 0.46 (the paper's 1.1 times
    the largest speed; the source flow's largest face value is 0.418, at the
    core), re-initialized from the VoF every 50 steps; the rest as C1,
    2000 steps.  The ACDI bound 1/(zeta (4 eps/h^2 + sqrt(2)/h)) = 2.9e-4 is
    far above dt."""
    cfg = c1_expanding_circle(n, soluble=True, extra=dict(interface=1, acdi_zeta=0.46),
                              name="expanding circle %d^2 fp32 soluble acdi" % n)
    cfg["reinit_every"] = reinit_every
    return cfg


def c1_variants(n=1024):
    """The soluble expanding circle with the substep-1 variants of the unsplit
    BCG scheme (section 3.1): the monotonized central limiter and the
    transverse term of the predictor; the rest as C1."""
    return c1_expanding_circle(n, soluble=True, extra=dict(limiter=1, bcg_transverse=1),
                               name="expanding circle %d^2 fp32 soluble mc-transverse" % n)


def c1_forces(n=1024):
    """The soluble expanding circle with the interfacial forces of the flow
    coupling (section 2.4) evaluated after every step: capillary and Marangoni
    forces on the faces from the step's VoF and the sigma it returns; the rest
    as C1."""
    cfg = c1_expanding_circle(n, soluble=True,
                              name="expanding circle %d^2 fp32 soluble forces" % n)
    cfg["forces"] = True
    return cfg


def c2_translating_sphere(n=256):
    """256^3 FP32, periodic in z, open in x and y; sphere R = 0.15 with centre
    (0.5, 0.5, 0.25 + U t), U = 0.5, VoF each step; lab-frame
    Hadamard-Rybczynski flow (viscosity ratio 0.01, sphere-frame stream -U)
    plus U along z, nearest periodic image; bubble-scaled parameters with
    d = 0.3: D_b = U d / Pe_b (Pe_b = 100), D_s = U d / Pe_s (Pe_s = 1000),
    k_d = Bi U / d (Bi = 1), k_a = Da U / (d c0) (Da = 0.1), Langmuir EoS with
    E = 0.3, c0 = 1, Gamma0 = 0; 1000 steps."""
    h = 1.0 / n
    U, R, d = 0.5, 0.15, 0.3
    prob = dict(dim=3, n=(n, n, n), h=h, bc=((2, 2), (2, 2), (1, 1)), eos=1, eos_E=0.3,
                sigma0=1.0, gamma_inf=1.0, D_b=U * d / 100, D_s=U * d / 1000,
                k_d=1.0 * U / d, k_a=0.1 * U / d, hj_iters_step=16)
    dt = 1.24e-3 * (256.0 / n) ** 2
    zc = lambda t: (0.25 + U * t) % 1.0
    cen = lambda t: (0.5, 0.5, zc(t))
    return dict(name="translating sphere %d^3 fp32" % n, prob=prob, precision=0, dt=dt,
                steps=1000,
                vof0=lambda: synth.vof_ball((n, n, n), h, cen(0.0), R, 3, period_z=1.0),
                vof_seq=lambda k: synth.vof_ball((n, n, n), h, cen((k + 1) * dt), R, 3,
                                                 period_z=1.0),
                u_seq=lambda k: synth.u_hadamard((n, n, n), h, cen(k * dt), R, -U, 0.01,
                                                 frame_shift=U, period_z=1.0),
                # the same inputs generated on a torch device
                vof_seq_dev=lambda k, dev: synth_dev.vof_ball((n, n, n), h, cen((k + 1) * dt), R,
                                                              period_z=1.0, device=dev),
                u_seq_dev=lambda k, dev: synth_dev.u_hadamard((n, n, n), h, cen(k * dt), R, -U,
                                                              0.01, frame_shift=U, period_z=1.0,
                                                              device=dev),
                vof0_dev=lambda dev: synth_dev.vof_ball((n, n, n), h, cen(0.0), R, period_z=1.0,
                                                        device=dev),
                c0=None, c0_const=1.0, gamma0=0.0, hj_step=16)


def c2_forces(n=256):
    """The translating sphere of C2 with the interfacial forces of the flow
    coupling (section 2.4) evaluated after every step, in 3D: capillary and
    Marangoni forces on the three face sets from the step's VoF and the sigma
    it returns; the rest as C2."""
    cfg = dict(c2_translating_sphere(n))
    cfg["name"] = "translating sphere %d^3 fp32 forces" % n
    cfg["forces"] = True
    return cfg


def c2_acdi(n=256, reinit_every=50):
    """The translating sphere of C2 on the ACDI interface (section 2.5): phi
    advanced by one ACDI step per step with zeta = 0.82 (1.1 times the
    largest face speed of the flow, 0.747), re-initialized from the VoF
    every 50 steps; the rest as C2.  The explicit regularization bounds the
    step: 1/(zeta (6 eps/h^2 + sqrt(3)/h)) = 4.5e-4 at 256^3, so
    dt = 3.5e-4 (256/n)."""
    cfg = c2_translating_sphere(n)
    cfg = dict(cfg)
    cfg["prob"] = dict(cfg["prob"], interface=1, acdi_zeta=0.82)
    cfg["dt"] = 3.5e-4 * (256.0 / n)
    cfg["name"] = "translating sphere %d^3 fp32 acdi" % n
    cfg["reinit_every"] = reinit_every
    dt, U, R = cfg["dt"], 0.5, 0.15
    zc = lambda t: (0.25 + U * t) % 1.0
    cen = lambda t: (0.5, 0.5, zc(t))
    h = 1.0 / n
    cfg["vof_seq"] = lambda k: synth.vof_ball((n, n, n), h, cen((k + 1) * dt), R, 3, period_z=1.0)
    cfg["u_seq"] = lambda k: synth.u_hadamard((n, n, n), h, cen(k * dt), R, -U, 0.01,
                                              frame_shift=U, period_z=1.0)
    cfg["vof_seq_dev"] = lambda k, dev: synth_dev.vof_ball((n, n, n), h, cen((k + 1) * dt), R,
                                                           period_z=1.0, device=dev)
    cfg["u_seq_dev"] = lambda k, dev: synth_dev.u_hadamard((n, n, n), h, cen(k * dt), R, -U, 0.01,
                                                           frame_shift=U, period_z=1.0, device=dev)
    return cfg


def c2_axisymmetric(nr=512, nz=1024):
    """The translating sphere of C2 on axisymmetric rings (Appendix B): r in
    [0, 0.5] (wall on the axis, open outside), z in [0, 1] periodic, h = 1/1024,
    FP32; sphere R = 0.15 on the axis at z = 0.25 + U t, U = 0.5, VoF each
    step; the Hadamard-Rybczynski flow plus U along z, nearest periodic image;
    the bubble-scaled parameters of C2; 1000 steps at dt = 1.2e-3 (256/1024)^2."""
    h = 1.0 / nz
    U, R, d = 0.5, 0.15, 0.3
    prob = dict(dim=2, n=(nr, nz), h=h, bc=((0, 2), (1, 1)), axisym=1, eos=1, eos_E=0.3,
                sigma0=1.0, gamma_inf=1.0, D_b=U * d / 100, D_s=U * d / 1000,
                k_d=1.0 * U / d, k_a=0.1 * U / d, hj_iters_step=16)
    dt = 1.2e-3 * (256.0 / nz) ** 2
    zc = lambda t: (0.25 + U * t) % 1.0
    n = (nr, nz)

    def vof(t):
        # the meridional disc of the sphere and its periodic images in z
        f = synth.vof_ball(n, h, (0.0, zc(t), 0), R, 2)
        for s in (-1.0, 1.0):
            f = np.maximum(f, synth.vof_ball(n, h, (0.0, zc(t) + s, 0), R, 2))
        return f

    return dict(name="translating sphere axisymmetric %dx%d fp32" % (nr, nz), prob=prob,
                precision=0, dt=dt, steps=1000,
                vof0=lambda: vof(0.0),
                vof_seq=lambda k: vof((k + 1) * dt),
                u_seq=lambda k: synth.u_hadamard_axi(n, h, zc(k * dt), R, -U, 0.01,
                                                     frame_shift=U, period_z=1.0),
                c0=None, c0_const=1.0, gamma0=0.0, hj_step=16)


def c3_ensemble(seed=3, count=64):
    """64 independent 2D static-circle instances: n ~ choice{128, 256, 512,
    1024}, R ~ U[0.15, 0.3] centred, Bi, Da ~ 10^U[-2, 2] (drawn in the order
    n, R, Bi, Da), flat-interface scalings with D_b = 1e-2: k_a = 1e-2 Da,
    k_d = 1e-2 Bi; the rest as the static circle but FP32; 500 steps at
    dt = 0.2 h^2 / D_b each."""
    rng = np.random.default_rng(seed)
    ns = rng.choice([128, 256, 512, 1024], size=count)
    Rs = rng.uniform(0.15, 0.3, size=count)
    Bi = 10.0 ** rng.uniform(-2, 2, size=count)
    Da = 10.0 ** rng.uniform(-2, 2, size=count)
    out = []
    for i in range(count):
        n = int(ns[i])
        h = 1.0 / n
        prob = dict(dim=2, n=(n, n), h=h, bc=((0, 0), (0, 0)), eos=0, eos_E=0.5, sigma0=1.0,
                    gamma_inf=1.0, D_b=1e-2, D_s=1e-3, k_a=1e-2 * Da[i], k_d=1e-2 * Bi[i])
        R = float(Rs[i])
        out.append(dict(prob=prob, dt=0.2 * h * h / 1e-2, steps=500, precision=0, R=R,
                        vof0=(lambda n=n, h=h, R=R: synth.vof_ball((n, n), h, (0.5, 0.5, 0), R, 2)),
                        c0_const=1.0, gamma0=0.0))
    return out


def c4_adjoint(n=128):
    """128^3 FP32 (FP64 oracle), static sphere R = 0.2 at the centre, walls in
    x and y, open in z, sphere-frame Hadamard-Rybczynski flow with stream
    V = -0.2 and viscosity ratio 0.01; nominal (k_a, k_d, D_b, D_s) =
    (1, 1, 0.01, 0.001), target run at (1.3, 0.7, 0.012, 0.0008); Langmuir EoS
    E = 0.3, Gamma0 = 0; c0 = 1 + 0.1 s(x) with s a seeded sum of 8 cosine
    modes (seed 4); 500 steps, checkpoint every 50."""
    h = 1.0 / n
    prob = dict(dim=3, n=(n, n, n), h=h, bc=((0, 0), (0, 0), (2, 2)), eos=1, eos_E=0.3,
                sigma0=1.0, gamma_inf=1.0, k_a=1.0, k_d=1.0, D_b=0.01, D_s=0.001)
    dt = 5.97e-4 * (128.0 / n) ** 2
    c = (0.5, 0.5, 0.5)
    return dict(name="adjoint sphere %d^3 fp32" % n, prob=prob, precision=0, dt=dt, steps=500,
                checkpoint=50, theta_nominal=(1.0, 1.0, 0.01, 0.001),
                theta_target=(1.3, 0.7, 0.012, 0.0008),
                vof0=lambda: synth.vof_ball((n, n, n), h, c, 0.2, 3),
                u=lambda: synth.u_hadamard((n, n, n), h, c, 0.2, -0.2, 0.01),
                c0=lambda: 1.0 + 0.1 * synth.smooth_modes((n, n, n), h, 4),
                gamma0=0.0)
