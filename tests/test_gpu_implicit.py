"""Parity of the implicit substep 2 (the HIP path through the C ABI) with the
FP64 oracle of `oracle/implicit.py` on the same seeded inputs, at time steps
above the explicit diffusive bound.  Tolerances: FP64 1e-12 and FP32 2e-5,
relative max-norm field by field; totals in FP64.  The FP64 runs solve each
linear problem to ||M^-1 r|| <= 1e-15 ||x|| (M the Jacobi diagonal), the FP32
runs to 1e-9 (the solver's vectors are FP64 in both)."""
import math

import numpy as np
import pytest

from oracle import implicit as I
from oracle import oracle as O
from paper_2605_27534_amd import surf as S
from paper_2605_27534_amd import synth
from tests.harness import compare_totals, default_hj_init, rel_max, run_gpu

pytestmark = pytest.mark.gpu

F64, F32 = 1, 0
TOL = {F64: 1e-12, F32: 2e-5}
# FP32 at the benchmark's solver tolerance
CG = {F64: dict(cg_tol=1e-15, cg_max_iters=1500), F32: dict(cg_tol=1e-9, cg_max_iters=1500)}


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
    compare_totals(H_g[-1], H_o[-1], tol, F_o if "F" in fields else None, P_o)
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


def test_solver_records_and_cap():
    # every solve of the step reports its iteration count; a cap too small
    # to meet the test raises the SOLVE status bit (every launch still ends
    # normally: the cap only bounds the number of launches)
    n = (150, 131)
    h = 1.0 / 150
    base = dict(dim=2, n=n, h=h, bc=((0, 0), (1, 1)), eos=1, eos_E=0.3, D_b=1e-2, D_s=2e-3,
                k_a=1.5, k_d=0.7, substep2=1, picard_iters=3, cg_tol=1e-10, cg_max_iters=600)
    cen = (0.47, 0.43, 0)
    vof = synth.vof_ball(n, h, cen, 0.2, 2)
    dt = 10 * 0.2 * h * h / 1e-2
    res = {}
    for cap in (600, 3):
        s = S.Surf(dict(base, cg_max_iters=cap), dt, S.SURF_F64)
        s.set_geometry(s.tensor(vof), full=True)
        F, P = s.init_state(s.tensor(synth.uniform_field(n, 7, 0.8, 1.2)), 1.0, 0.4)
        F2, P2 = s.empty(), s.empty()
        with pytest.raises(S.SurfError):
            s.solver_iterations()  # no implicit step yet
        s.step(F, P, F2, P2)
        its = s.solver_iterations()
        assert len(its) == 6  # (interface, bulk) x 3 sweeps
        assert all(0 <= k <= cap for k in its), its
        res[cap] = (its, s.status())
    its, st = res[600]
    assert st == 0 and max(its) < 600 and its[0] > 0, res
    # the last sweep starts from nearly converged iterates
    assert its[4] < its[0] and its[5] < its[1], its
    its, st = res[3]
    assert st & S.STATUS_SOLVE and its == [3] * 6, res


def test_graph_replay_equals_paced_eager():
    # eagerly the host paces the CG launches and stops enqueuing once a solve
    # has met its test; a captured graph holds every capped launch, those
    # after convergence returning at once.  The device decides convergence
    # in both, so the results are bitwise equal, on every replay.
    import torch
    n = (150, 131)
    h = 1.0 / 150
    prob = dict(dim=2, n=n, h=h, bc=((2, 2), (2, 0)), eos=1, eos_E=0.3, D_b=1e-2, D_s=2e-3,
                k_a=1.5, k_d=0.7, substep2=1, cg_tol=1e-9, cg_max_iters=150)
    cen = (0.47, 0.43, 0)
    dt = 10 * 0.2 * h * h / 1e-2
    vof = synth.vof_ball(n, h, cen, 0.2, 2)
    vofs = [synth.vof_ball(n, h, cen, 0.2 + 0.002 * (k + 1), 2) for k in range(3)]
    u = synth.u_source2d(n, h, cen, 0.04)
    c0 = synth.uniform_field(n, 7, 0.8, 1.2)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = S.Surf(prob, dt, S.SURF_F32)
        T = s.tensor
        vof_d, vofs_d, u_d, c0_d = T(vof), [T(v) for v in vofs], [T(x) for x in u], T(c0)
        bufs = [[s.empty(), s.empty()] for _ in range(2)]
        sig = s.empty()

        def reset():
            s.set_geometry(vof_d, full=True)
            F, P = s.init_state(c0_d, 1.0, 0.4)
            bufs[0][0].copy_(F)
            bufs[0][1].copy_(P)

        def steps():
            for k in range(3):
                a, b = bufs[k % 2], bufs[(k + 1) % 2]
                s.step(a[0], a[1], b[0], b[1], u=u_d, vof_next=vofs_d[k], sigma_out=sig)

        def result():
            torch.cuda.synchronize()
            return [x.clone() for x in bufs[1]] + [sig.clone()]

        reset()
        steps()
        ref = result()
        ref_iters = s.solver_iterations()
        assert max(ref_iters) < 150 and s.status() == 0, ref_iters
        reset()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            steps()
        for rep in range(2):
            reset()
            torch.cuda.synchronize()
            g.replay()
            got = result()
            for name, a, b in zip(("F", "psi", "sigma"), got, ref):
                assert torch.equal(a, b), (rep, name)
            assert s.solver_iterations() == ref_iters


@pytest.mark.parametrize("prec", [F64, F32])
@pytest.mark.parametrize("dim", [2, 3])
def test_implicit_with_unsplit_bcg(dim, prec):
    # the paper's integrator: the implicit substep 2 after the unsplit BCG
    # advection (MC limiter and transverse term)
    if dim == 2:
        n = (150, 131)
        h = 1.0 / 150
        bc = ((2, 2), (1, 1))
        cen = (0.47, 0.43, 0)
        # a rotation plus a shift, slow enough for the advective bound at
        # ten times the explicit diffusive step
        u = synth.u_rotation(n, h, cen, 0.5)
        u = [u[0] + 0.1, u[1] - 0.05]
        vof = synth.vof_ball(n, h, cen, 0.2, 2)
        dt = 10 * 0.2 * h * h / 1e-2
        steps = 4
    else:
        n = (28, 24, 16)
        h = 1.0 / 28
        bc = ((2, 2), (0, 0), (1, 1))
        cen = (0.45, 0.42, 0.28)
        u = synth.u_hadamard(n, h, cen, 0.15, -0.3, 0.01)
        vof = synth.vof_ball(n, h, cen, 0.15, 3)
        dt = 6 * 0.1 * h * h / 1e-2
        steps = 3
    prob = dict(dim=dim, n=n, h=h, bc=bc, eos=1, eos_E=0.3, D_b=1e-2, D_s=2e-3, k_a=1.5,
                k_d=0.7, substep2=1, limiter=1, bcg_transverse=1, **CG[prec])
    c0 = synth.uniform_field(n, 8, 0.8, 1.2)
    o = run_oracle_implicit(prob, vof, steps, dt, u=u, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, steps, dt, prec, u=u, c0=c0, gamma0=0.4)
    print(compare(o, g, prec), flush=True)


# The paper's flux form (the upwind anti-diffusion makes each problem
# non-symmetric): BiCGSTAB with the Jacobi preconditioner, FP64 solves to
# ||M^-1 r|| <= 1e-16 ||x|| on the recursively updated residual (the error
# itself levels off near rounding; far from the interface, where psi is
# small, it is small against psi only at such a tolerance)
CG_P = {F64: dict(cg_tol=1e-16, cg_max_iters=1500), F32: dict(cg_tol=1e-9, cg_max_iters=1500)}


def compare_paper(o, g, prec, eps, bulk=True):
    """As compare, except sigma: here the unknown is psi itself, and the stop
    test bounds its error against ||psi||, not cell by cell; Gamma = psi /
    (delta + eta/eps) multiplies that error by 1/delta far from the
    interface.  So sigma is compared as sigma delta (what the interface
    averages and the force take), and as sigma itself where delta is above
    1e-3 of its peak.  Likewise c_max = max F/(phi + eta) in the totals."""
    chi_o, F_o, P_o, S_o, H_o = o
    chi_g, F_g, P_g, S_g, H_g, s = g
    ph = 1.0 / (1.0 + np.exp(chi_o / eps))
    de = ph * (1.0 - ph)
    band = de > 1e-3 * de.max()
    pairs = [("chi", chi_g, chi_o), ("psi", P_g, P_o), ("sigma delta", S_g * de, S_o * de),
             ("sigma in the band", S_g[band], S_o[band])]
    if bulk:
        pairs.append(("F", F_g, F_o))
    errs = {nm: rel_max(a, b) for nm, a, b in pairs}
    tol = TOL[prec]
    assert all(v <= tol for v in errs.values()), errs
    slot_tol = None
    if bulk:
        # c_max = max F/(phi + eta) with F the unknown: the field check bounds
        # F's error by tol ||F||, so c_max's relative error by tol ||F|| over
        # F at the cell of c_max (small where phi is)
        c = F_o / (ph + 1e-12)
        k = np.unravel_index(np.argmax(c), c.shape)
        slot_tol = {O.T_CMAX: tol * max(1.0, np.max(np.abs(F_o)) / abs(F_o[k]))}
    compare_totals(H_g[-1], H_o[-1], tol, F_o if bulk else None, P_o, slot_tol=slot_tol)
    assert s.status() == 0
    return errs


@pytest.mark.parametrize("prec", [F64, F32])
@pytest.mark.parametrize("case", CASES_2D, ids=[c[0] for c in CASES_2D])
def test_implicit_paper_form_2d(case, prec):
    name, bc, kin, bulk, flow = case
    n = (150, 131)
    h = 1.0 / 150
    prob = dict(dim=2, n=n, h=h, bc=bc, kinetics=kin, bulk_enabled=bulk, eos=1, eos_E=0.3,
                D_b=1e-2, D_s=2e-3, k_a=1.5, k_d=0.7, substep2=1, flux_form=1, **CG_P[prec])
    cen = (0.47, 0.43, 0)
    vof = synth.vof_ball(n, h, cen, 0.2, 2)
    u = synth.u_source2d(n, h, cen, 0.04) if flow else None
    c0 = synth.uniform_field(n, 7, 0.8, 1.2)
    dt = 10 * 0.2 * h * h / 1e-2  # ten times the explicit diffusive step
    o = run_oracle_implicit(prob, vof, 4, dt, u=u, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 4, dt, prec, u=u, c0=c0, gamma0=0.4)
    print(name, prec, compare_paper(o, g, prec, 1.5 * h, bulk=bool(bulk)), flush=True)
    rec = g[5].solver_iterations()
    assert rec[0] > 0 and all(0 <= r < CG_P[prec]["cg_max_iters"] for r in rec), rec


@pytest.mark.parametrize("prec", [F64, F32])
def test_implicit_paper_form_3d(prec):
    n = (28, 24, 16)
    h = 1.0 / 28
    prob = dict(dim=3, n=n, h=h, bc=((2, 2), (0, 0), (1, 1)), eos=1, eos_E=0.3, D_b=1e-2,
                D_s=2e-3, k_a=1.5, k_d=0.7, substep2=1, flux_form=1, **CG_P[prec])
    cen = (0.45, 0.42, 0.28)
    vof = synth.vof_ball(n, h, cen, 0.15, 3)
    u = synth.u_hadamard(n, h, cen, 0.15, -0.3, 0.01)
    c0 = synth.uniform_field(n, 8, 0.8, 1.2)
    dt = 6 * 0.1 * h * h / 1e-2
    o = run_oracle_implicit(prob, vof, 3, dt, u=u, c0=c0, gamma0=0.4)
    g = run_gpu(prob, vof, 3, dt, prec, u=u, c0=c0, gamma0=0.4)
    compare(o, g, prec)
