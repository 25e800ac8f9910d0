"""Parity of the substep-1 variants (section 3.1: the monotonized central
limiter and the transverse term of the unsplit BCG predictor; the HIP path
through the C ABI) with the FP64 oracle on the same seeded inputs: chi, F,
psi, sigma and the totals after 20 steps on ragged 2D grids with walls, open
and periodic sides, and the expanding-circle workload at full size.
Tolerances: FP64 1e-12 and FP32 2e-5, relative max-norm field by field."""
import math

import numpy as np
import pytest

from paper_2605_27534_amd import synth
from tests.harness import run_gpu, run_oracle
from tests.test_gpu_parity import F32, F64, compare, flow_2d

pytestmark = pytest.mark.gpu

VARIANTS = [(1, 0), (0, 1), (1, 1)]  # (limiter, transverse)
CASES = [
    # name, bc, kinetics, eos, bulk, flow
    ("walls-rot", ((0, 0), (0, 0)), 0, 0, 1, "rot"),
    ("open-source-insoluble", ((2, 2), (2, 2)), 0, 1, 0, "source"),
    ("periodic-shift", ((1, 1), (1, 1)), 1, 2, 1, "shift"),
    ("periodic-x-open-y", ((1, 1), (2, 2)), 0, 1, 1, "shift"),
]


@pytest.mark.parametrize("prec", [F64, F32])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("variant", VARIANTS, ids=["mc", "transverse", "mc-transverse"])
def test_variants_2d(variant, case, prec):
    lim, tr = variant
    name, bc, kin, eos, bulk, flow = case
    n = (200, 136)  # 4 strips of 58 columns, 17 row chunks: ragged both ways
    h = 1.0 / 200
    prob = dict(dim=2, n=n, h=h, bc=bc, kinetics=kin, eos=eos, bulk_enabled=bulk, eos_E=0.3,
                D_b=1e-2, D_s=2e-3, k_a=1.5, k_d=0.7, limiter=lim, bcg_transverse=tr)
    vof = synth.vof_ball(n, h, (0.47, 0.33, 0), 0.17, 2)
    u = flow_2d(flow, n, h)
    c0 = synth.uniform_field(n, 7, 0.8, 1.2)
    dt = 0.15 * h * h / 1e-2
    o = run_oracle(prob, vof, 20, dt, u=u, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 20, dt, prec, u=u, c0=c0, gamma0=0.4)
    fields = ("chi", "F", "psi", "sigma") if bulk else ("chi", "psi", "sigma")
    print(variant, name, prec, compare(o, g, prec, fields=fields), flush=True)


@pytest.mark.parametrize("variant", VARIANTS, ids=["mc", "transverse", "mc-transverse"])
def test_variants_change_the_result(variant):
    # the variants are not the default scheme: on the same inputs the fields
    # differ well above rounding
    lim, tr = variant
    n = (96, 80)
    h = 1.0 / 96
    base = dict(dim=2, n=n, h=h, bc=((1, 1), (1, 1)), eos=1, eos_E=0.3)
    vof = synth.vof_ball(n, h, (0.47, 0.43, 0), 0.2, 2)
    u = flow_2d("shift", n, h)
    dt = 0.15 * h * h / 1e-2
    g0 = run_gpu(base, vof, 10, dt, F64, u=u, gamma0=0.4)
    g1 = run_gpu(dict(base, limiter=lim, bcg_transverse=tr), vof, 10, dt, F64, u=u, gamma0=0.4)
    assert np.max(np.abs(g1[2] - g0[2])) > 1e-6 * np.max(np.abs(g0[2]))


def test_expanding_circle_full_size_mc_transverse():
    # the 1024^2 expanding circle (VoF recomputed each step, the pipelined
    # geometry not used here) with both variants, FP32, 4 steps, element by
    # element against the oracle
    from paper_2605_27534_amd import configs as C
    cfg = C.c1_expanding_circle(extra=dict(limiter=1, bcg_transverse=1))
    prob = dict(cfg["prob"])
    vof0 = cfg["vof0"]()
    u = cfg["u"]()
    c0 = cfg["c0"]()
    nsteps = 4
    o = run_oracle(prob, vof0, nsteps, cfg["dt"], u=u, vof_seq=cfg["vof_seq"], c0=c0,
                   gamma0=cfg["gamma0"])
    g = run_gpu(prob, vof0, nsteps, cfg["dt"], F32, u=u, vof_seq=cfg["vof_seq"], c0=c0,
                gamma0=cfg["gamma0"])
    print(compare(o, g, F32), flush=True)


# Explicit 3D (the tile transport k_step takes the variants): a ragged grid
# (40 x 36 x 28 cells in 16 x 8 x 8 tiles), the Hadamard-Rybczynski flow of
# a sphere, closed, open and periodic sides; the moving case rebuilds the
# level set from a translated VoF field every step
CASES_3D = [
    # name, bc, kinetics, eos, moving
    ("walls", ((0, 0), (0, 0), (0, 0)), 0, 1, False),
    ("open-x-periodic-z", ((2, 2), (0, 0), (1, 1)), 1, 2, False),
    ("periodic-z-moving", ((0, 0), (2, 2), (1, 1)), 0, 0, True),
]


@pytest.mark.parametrize("prec", [F64, F32])
@pytest.mark.parametrize("case", CASES_3D, ids=[c[0] for c in CASES_3D])
@pytest.mark.parametrize("variant", VARIANTS, ids=["mc", "transverse", "mc-transverse"])
def test_variants_3d_explicit(variant, case, prec):
    lim, tr = variant
    name, bc, kin, eos, moving = case
    n = (40, 36, 28)
    h = 1.0 / 40
    Lz = n[2] * h
    prob = dict(dim=3, n=n, h=h, bc=bc, kinetics=kin, eos=eos, eos_E=0.3, D_b=1e-2, D_s=2e-3,
                k_a=1.5, k_d=0.7, limiter=lim, bcg_transverse=tr)
    cen = (0.5, 0.44, 0.36)
    per_z = Lz if bc[2][0] == 1 else None
    U = 0.3
    u = synth.u_hadamard(n, h, cen, 0.2, -U, 0.01, frame_shift=U if moving else 0.0,
                         period_z=per_z)
    dt = 0.15 * h * h / 1e-2
    vof = synth.vof_ball(n, h, cen, 0.2, 3, period_z=per_z)
    seq = None
    if moving:
        seq = lambda k: synth.vof_ball(n, h, (cen[0], cen[1], cen[2] + U * (k + 1) * dt), 0.2, 3,
                                       period_z=per_z)
    c0 = synth.uniform_field(n, 9, 0.8, 1.2)
    o = run_oracle(prob, vof, 8, dt, u=u, vof_seq=seq, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 8, dt, prec, u=u, vof_seq=seq, c0=c0, gamma0=0.4)
    print(variant, name, prec, compare(o, g, prec), flush=True)
