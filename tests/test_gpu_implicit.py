"""Parity of the implicit substep 2 (the HIP path through the C ABI) with the
FP64 oracle of `oracle/implicit.py` on the same seeded inputs, at time steps
above the explicit diffusive bound.  Tolerances: FP64 1e-12 and FP32 2e-5,
relative max-norm field by field; totals in FP64.  The FP64 runs solve each
linear problem to ||M^-1 r|| <= 1e-15 ||x|| (M the Jacobi diagonal), the FP32
runs to 1e-12 (the solver's vectors are FP64 in both)."""
import math

import numpy as np
import pytest

from oracle import implicit as I
from oracle import oracle as O
from paper_2605_27534_amd import synth
from tests.harness import default_hj_init, rel_max, run_gpu

pytestmark = pytest.mark.gpu

F64, F32 = 1, 0
TOL = {F64: 1e-12, F32: 2e-5}
CG = {F64: dict(cg_tol=1e-15, cg_max_iters=1500), F32: dict(cg_tol=1e-12, cg_max_iters=1500)}


def run_oracle_implicit(prob, vof, nsteps, dt, u=None, vof_seq=None, c0=None, gamma0=0.0,
                        picard=3):
    q = O.full(prob)
    chi = O.geometry(prob, vof, default_hj_init(q))
    F, P = O.init_state(prob, chi, c0=c0, gamma0=gamma0)
    return I.run(prob, chi, u, F, P, dt, nsteps, vof_seq=vof_seq, hj_iters=8, picard=picard)


def compare(o, g, prec, fields=("chi", "F", "psi", "sigma")):
    chi_o, F_o, P_o, S_o, H_o = o
    chi_g, F_g, P_g, S_g, H_g, s = g
    errs = {}
    for name, a, b in (("chi", chi_g, chi_o), ("F", F_g, F_o), ("psi", P_g, P_o),
                       ("sigma", S_g, S_o)):
        if name in fields and a is not None:
            errs[name] = rel_max(a, b)
    tol = TOL[prec]
    assert all(v <= tol for v in errs.values()), errs
    for slot in (O.T_MB, O.T_MS, O.T_SDELTA, O.T_SSIGD, O.T_MTOT, O.T_GAVG, O.T_SAVG, O.T_OUTCUM):
        a, b = H_g[-1][slot], H_o[-1][slot]
        assert abs(a - b) <= tol * max(abs(b), 1e-300) + 1e-300, (slot, a, b)
    assert H_g[-1][O.T_T] == pytest.approx(H_o[-1][O.T_T], rel=1e-14)
    # no stability flag: substep 2 has no bound when implicit
    assert s.status() == 0
    return errs


CASES_2D = [
    # name, bc, kinetics, bulk, flow
    ("walls-periodic-langmuir", ((0, 0), (1, 1)), 0, 1, "source"),
    ("open-henry", ((2, 2), (2, 0)), 1, 1, "source"),
    ("insoluble-noflow", ((0, 0), (0, 0)), 0, 0, None),
]


@pytest.mark.parametrize("prec", [F64, F32])
@pytest.mark.parametrize("case", CASES_2D, ids=[c[0] for c in CASES_2D])
def test_implicit_2d(case, prec):
    name, bc, kin, bulk, flow = case
    n = (150, 131)
    h = 1.0 / 150
    prob = dict(dim=2, n=n, h=h, bc=bc, kinetics=kin, bulk_enabled=bulk, eos=1, eos_E=0.3,
                D_b=1e-2, D_s=2e-3, k_a=1.5, k_d=0.7, substep2=1, **CG[prec])
    cen = (0.47, 0.43, 0)
    vof = synth.vof_ball(n, h, cen, 0.2, 2)
    u = synth.u_source2d(n, h, cen, 0.04) if flow else None
    c0 = synth.uniform_field(n, 7, 0.8, 1.2)
    dt = 10 * 0.2 * h * h / 1e-2  # ten times the explicit diffusive step
    o = run_oracle_implicit(prob, vof, 4, dt, u=u, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 4, dt, prec, u=u, c0=c0, gamma0=0.4)
    compare(o, g, prec, fields=("chi", "F", "psi", "sigma") if bulk else ("chi", "psi", "sigma"))


@pytest.mark.parametrize("prec", [F64, F32])
def test_implicit_2d_moving_interface(prec):
    n = (130, 120)
    h = 1.0 / 130
    prob = dict(dim=2, n=n, h=h, bc=((2, 2), (2, 2)), eos=1, eos_E=0.2, substep2=1,
                **CG[prec])
    cen = (0.5, 0.46, 0)
    R0, Q = 0.15, 0.05
    dt = 8 * 0.2 * h * h / 1e-2
    Rt = lambda t: math.sqrt(R0 ** 2 + Q * t / math.pi)
    vof = synth.vof_ball(n, h, cen, R0, 2)
    seq = lambda k: synth.vof_ball(n, h, cen, Rt((k + 1) * dt), 2)
    u = synth.u_source2d(n, h, cen, Q)
    c0 = synth.uniform_field(n, 3, 0.8, 1.2)
    o = run_oracle_implicit(prob, vof, 4, dt, u=u, vof_seq=seq, c0=c0, gamma0=0.5)
    g = run_gpu(prob, vof, 4, dt, prec, u=u, vof_seq=seq, c0=c0, gamma0=0.5)
    compare(o, g, prec)


@pytest.mark.parametrize("prec", [F64, F32])
def test_implicit_3d(prec):
    # small enough for the oracle's sparse direct solves (fill-in grows fast in 3D)
    n = (28, 24, 16)
    h = 1.0 / 28
    prob = dict(dim=3, n=n, h=h, bc=((2, 2), (0, 0), (1, 1)), eos=1, eos_E=0.3, D_b=1e-2,
                D_s=2e-3, k_a=1.5, k_d=0.7, substep2=1, **CG[prec])
    cen = (0.45, 0.42, 0.28)
    vof = synth.vof_ball(n, h, cen, 0.15, 3)
    u = synth.u_hadamard(n, h, cen, 0.15, -0.3, 0.01)
    c0 = synth.uniform_field(n, 8, 0.8, 1.2)
    dt = 6 * 0.1 * h * h / 1e-2
    o = run_oracle_implicit(prob, vof, 3, dt, u=u, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 3, dt, prec, u=u, c0=c0, gamma0=0.4)
    compare(o, g, prec)
