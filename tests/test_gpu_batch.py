"""The batched form (one persistent launch over the tiles of many instances,
one HIP graph per call) against the single-problem path and the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_27534_amd import synth
from tests.harness import rel_max, run_oracle, to_np

pytestmark = pytest.mark.gpu


def instances():
    # ragged sizes (not multiples of the 64 x 16 tile), mixed boundaries,
    # kinetics, equations of state and flux forms
    specs = [((96, 80), ((0, 0), (0, 0)), dict(kinetics=0, eos=1, eos_E=0.3), 0.22),
             ((130, 70), ((1, 1), (0, 0)), dict(kinetics=1, eos=0, eos_E=0.5, flux_form=1), 0.2),
             ((64, 64), ((2, 2), (0, 0)), dict(kinetics=0, eos=2, eos_E=0.4, k_a=3.0), 0.25),
             ((40, 150), ((0, 0), (1, 1)), dict(kinetics=0, eos=1, eos_E=0.2, k_d=0.3), 0.15)]
    out = []
    for (nx, ny), bc, kw, R in specs:
        h = 1.0 / max(nx, ny)
        prob = dict(dim=2, n=(nx, ny), h=h, bc=bc)
        prob.update(kw)
        vof = synth.vof_ball((nx, ny), h, (0.5 * nx * h, 0.5 * ny * h, 0), R * min(nx, ny) * h, 2)
        c0 = 1 + 0.1 * synth.smooth_modes((nx, ny), h, 11 + len(out), dim=2)
        out.append((prob, 0.2 * h * h / 1e-2, vof, c0))
    return out


def run_batch(insts, prec, steps, tune=False, side_stream=False):
    import torch
    if side_stream:
        # on a non-null stream every call is recorded once into a HIP graph
        # and replayed
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            out = run_batch(insts, prec, steps, tune)
        torch.cuda.synchronize()
        return out
    from paper_2605_27534_amd.batch import Batch
    b = Batch([p for p, _, _, _ in insts], [dt for _, dt, _, _ in insts], prec)
    for i, (p, dt, vof, c0) in enumerate(insts):
        b.set_geometry(i, torch.as_tensor(vof).to("cuda", b.dtype).reshape(b.shapes[i]).contiguous())
        b.init_state(i, torch.as_tensor(c0).to("cuda", b.dtype).reshape(b.shapes[i]).contiguous(),
                     1.0, 0.1)
    if tune:
        b.tune()
    tot = torch.zeros((len(insts), 16), dtype=torch.float64, device="cuda")
    for k in steps:
        b.step(k, tot)
    torch.cuda.synchronize()
    res = []
    for i in range(len(insts)):
        F, P = b.state(i)
        res.append((to_np(F), to_np(P), to_np(b.sigma[i]), tot[i].cpu().numpy()))
    b.close()
    return res


def run_single(prob, dt, vof, c0, prec, nsteps):
    import torch
    from paper_2605_27534_amd import surf as S
    s = S.Surf(prob, dt, prec)
    s.set_geometry(s.tensor(vof), full=True)
    F, P = s.init_state(s.tensor(c0), 1.0, 0.1)
    F2, P2, sig = s.empty(), s.empty(), s.empty()
    tot = torch.zeros(16, dtype=torch.float64, device="cuda")
    for _ in range(nsteps):
        s.step(F, P, F2, P2, sigma_out=sig, totals=tot)
        F, F2, P, P2 = F2, F, P2, P
    torch.cuda.synchronize()
    return to_np(F), to_np(P), to_np(sig), tot.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_matches_single_problem_path(prec):
    # the batched kernel (64 x 16 tiles) and the single-problem path (column
    # streaming for the weighted form) order and contract the same arithmetic
    # differently, so they agree to rounding level, not bitwise; each is
    # checked against the FP64 oracle on its own
    insts = instances()
    N = 9
    got = run_batch(insts, prec, [4, 5])
    ftol, ttol = (1e-13, 1e-12) if prec == 1 else (2e-6, 2e-6)
    for i, (p, dt, vof, c0) in enumerate(insts):
        ref = run_single(p, dt, vof, c0, prec, N)
        for name, a, b in zip(("F", "psi", "sigma"), got[i][:3], ref[:3]):
            assert rel_max(a, b) <= ftol, (i, name, rel_max(a, b))
        for slot in range(16):
            x, y = got[i][3][slot], ref[3][slot]
            assert abs(x - y) <= ttol * max(abs(y), 1e-300), (i, slot, x, y)


def test_batch_fp64_matches_oracle():
    insts = instances()[:3]
    N = 25
    got = run_batch(insts, 1, [N])
    for i, (p, dt, vof, c0) in enumerate(insts):
        chi, F, P, S, hist = run_oracle(p, vof, N, dt, c0=c0, gamma0=0.1)
        for name, a, b in (("F", got[i][0], F), ("psi", got[i][1], P), ("sigma", got[i][2], S)):
            assert rel_max(a.reshape(b.shape), b) <= 1e-12, (i, name)
        for slot in (O.T_MB, O.T_MS, O.T_SDELTA, O.T_SSIGD, O.T_MTOT, O.T_GAVG, O.T_SAVG):
            assert abs(got[i][3][slot] - hist[-1][slot]) <= 1e-12 * abs(hist[-1][slot]), (i, slot)
        assert got[i][3][O.T_T] == pytest.approx(hist[-1][O.T_T], rel=1e-14)


def ring_instances():
    # axisymmetric rings (Appendix B) beside a Cartesian instance: a sphere
    # on the axis (open outer side), an annulus off the axis with a ring of
    # fluid (walls), and a Cartesian disc
    out = []
    specs = [((90, 120), ((0, 2), (0, 0)), (0.0, 0.0, 0.0), (0.0, 0.55), 0.3),
             ((70, 64), ((0, 0), (1, 1)), (0.2, 0.0, 0.0), (0.6, 0.5), 0.2)]
    for (nx, ny), bc, org, (cx, cz), R in specs:
        h = 1.0 / max(nx, ny)
        prob = dict(dim=2, n=(nx, ny), h=h, bc=bc, axisym=1, origin=org, eos=1, eos_E=0.3,
                    k_a=1.5, k_d=0.7)
        vof = synth.vof_ball((nx, ny), h, (cx, cz, 0), R, 2, origin=org)
        c0 = synth.uniform_field((nx, ny), 20 + len(out), 0.8, 1.2)
        out.append((prob, 0.2 * h * h / 1e-2, vof, c0))
    return out + [instances()[0]]


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_with_rings(prec):
    # the ring instances take the ring variant of the column waves in the
    # same persistent launch as the Cartesian one: against the single-problem
    # path (k_col2d's ring instance) and, in FP64, against the oracle
    insts = ring_instances()
    N = 9
    got = run_batch(insts, prec, [4, 5])
    ftol, ttol = (1e-13, 1e-12) if prec == 1 else (2e-6, 2e-6)
    for i, (p, dt, vof, c0) in enumerate(insts):
        ref = run_single(p, dt, vof, c0, prec, N)
        for name, a, b in zip(("F", "psi", "sigma"), got[i][:3], ref[:3]):
            assert rel_max(a, b) <= ftol, (i, name, rel_max(a, b))
        for slot in range(16):
            x, y = got[i][3][slot], ref[3][slot]
            assert abs(x - y) <= ttol * max(abs(y), 1e-300), (i, slot, x, y)
        if prec == 1:
            chi, F, P, S, hist = run_oracle(p, vof, N, dt, c0=c0, gamma0=0.1)
            for name, a, b in (("F", got[i][0], F), ("psi", got[i][1], P), ("sigma", got[i][2], S)):
                assert rel_max(a.reshape(b.shape), b) <= 1e-12, (i, name)
            for slot in (O.T_MB, O.T_MS, O.T_SDELTA, O.T_SSIGD, O.T_MTOT, O.T_GAVG, O.T_SAVG):
                assert abs(got[i][3][slot] - hist[-1][slot]) <= 1e-12 * abs(hist[-1][slot]), (i, slot)


def test_tuned_launch_shape_and_step_split_leave_results_unchanged():
    # the autotuner's choice changes only the launch shape; the fields are
    # per-cell and must not change, the totals only by reduction order
    insts = instances()
    a = run_batch(insts, 0, [7])
    b = run_batch(insts, 0, [1, 2, 4], tune=True)
    for x, y in zip(a, b):
        for u, v in zip(x[:3], y[:3]):
            assert np.array_equal(u, v)
        assert np.allclose(x[3], y[3], rtol=1e-13, atol=0)


def make_batch(insts, prec):
    import torch
    from paper_2605_27534_amd.batch import Batch
    b = Batch([p for p, _, _, _ in insts], [dt for _, dt, _, _ in insts], prec)
    for i, (p, dt, vof, c0) in enumerate(insts):
        b.set_geometry(i, torch.as_tensor(vof).to("cuda", b.dtype).reshape(b.shapes[i]).contiguous())
        b.init_state(i, torch.as_tensor(c0).to("cuda", b.dtype).reshape(b.shapes[i]).contiguous(),
                     1.0, 0.1)
    return b


def test_graph_replays_match_eager_launches():
    # a batch on a side stream records each distinct (step count, parity,
    # totals) call once as a HIP graph and replays it; every replay is
    # checked against the same steps launched eagerly on the null stream,
    # with eager work and synchronisations in between
    import torch
    insts = instances()
    eager = make_batch(insts, 0)
    te = torch.zeros((len(insts), 16), dtype=torch.float64, device="cuda")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        graph = make_batch(insts, 0)
        tg = torch.zeros((len(insts), 16), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    for k in (1, 2, 2, 2, 3, 2, 1):
        eager.step(k, te)
        with torch.cuda.stream(st):
            graph.step(k, tg)
        torch.cuda.synchronize()
        assert eager.parity == graph.parity
        for i in range(len(insts)):
            for x, y in zip(eager.state(i), graph.state(i)):
                assert torch.equal(x, y), (k, i)
            assert torch.equal(eager.sigma[i], graph.sigma[i])
        assert torch.equal(te, tg)
    eager.close()
    graph.close()


def test_ensemble_sample_runs_and_conserves():
    # the first four instances of the 64-instance static-circle ensemble at
    # their drawn sizes (no flow: total surfactant is conserved exactly up
    # to rounding with walls all round)
    import torch
    from paper_2605_27534_amd import configs
    from paper_2605_27534_amd.batch import Batch
    ens = configs.c3_ensemble()
    pick = ens[:4]
    b = Batch([e["prob"] for e in pick], [e["dt"] for e in pick], 0)
    for i, e in enumerate(pick):
        b.set_geometry(i, torch.as_tensor(e["vof0"]()).to("cuda", torch.float32)
                       .reshape(b.shapes[i]).contiguous())
        b.init_state(i, None, e["c0_const"], e["gamma0"])
    t0 = torch.zeros((4, 16), dtype=torch.float64, device="cuda")
    t1 = torch.zeros((4, 16), dtype=torch.float64, device="cuda")
    b.step(1, t0)
    b.step(50, t1)
    torch.cuda.synchronize()
    t0, t1 = t0.cpu().numpy(), t1.cpu().numpy()
    for i in range(4):
        assert abs(t1[i][O.T_MTOT] / t0[i][O.T_MTOT] - 1) < 2e-6
        assert t1[i][O.T_NBAD] == 0
        assert t1[i][O.T_MS] > t0[i][O.T_MS]   # adsorption from the bulk
    b.close()
