"""The pipelined moving interface (surf_prepare_geometry): the next step's
geometry on an auxiliary stream while the current transport runs.  The
kernels and their arguments are those of plain surf_step calls, so the
results must be bitwise equal, eagerly and replayed from a HIP graph that
spans both streams."""
import math

import numpy as np
import pytest

from paper_2605_27534_amd import surf as S
from paper_2605_27534_amd import synth
from tests.harness import to_np

pytestmark = pytest.mark.gpu

F64, F32 = 1, 0


def circle_case(n, precision, R0=0.12):
    # the expanding circle (source flow, VoF recomputed every step) with a
    # ragged grid so that boundary strips and rows are exercised
    nx, ny = n
    h = 1.0 / max(nx, ny)
    Q = 0.05
    dt = 0.15 * h * h / 1e-2
    prob = dict(dim=2, n=n, h=h, bc=((2, 2), (2, 0)), eos=1, eos_E=0.2,
                hj_iters_step=8)
    cen = (0.5 * nx * h, 0.47 * ny * h, 0)
    Rt = lambda t: math.sqrt(R0 ** 2 + Q * t / math.pi)
    vof0 = synth.vof_ball(n, h, cen, R0, 2)
    vofs = [synth.vof_ball(n, h, cen, Rt((k + 1) * dt), 2) for k in range(24)]
    u = synth.u_source2d(n, h, cen, Q)
    c0 = synth.uniform_field(n, 5, 0.8, 1.2)
    return prob, dt, vof0, vofs, u, c0


class Runner:
    """One context on its own stream, with ping-pong state buffers."""

    def __init__(self, case, precision):
        import torch
        prob, dt, vof0, vofs, u, c0 = case
        self.main = torch.cuda.Stream()
        self.aux = torch.cuda.Stream()
        with torch.cuda.stream(self.main):
            self.s = S.Surf(prob, dt, precision)
            T = self.s.tensor
            self.vof0 = T(vof0)
            self.vofs = [T(v) for v in vofs]
            self.u = [T(x) for x in u]
            self.c0 = T(c0)
            self.bufs = [[self.s.empty(), self.s.empty()] for _ in range(2)]
            self.sig = self.s.empty()
            self.hist = torch.zeros((len(vofs), 16), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()

    def reset(self):
        import torch
        with torch.cuda.stream(self.main):
            self.s.set_geometry(self.vof0, full=True)
            F, P = self.s.init_state(self.c0, 1.0, 0.3)
            self.bufs[0][0].copy_(F)
            self.bufs[0][1].copy_(P)
        torch.cuda.synchronize()

    def steps(self, k0, k1, pipelined, forces=None):
        """Steps k0 .. k1-1 on the context's stream (current stream = main);
        with `forces` (a list), the interfacial forces of each step are taken
        between the step and the next prepared geometry and appended."""
        for k in range(k0, k1):
            a, b = self.bufs[k % 2], self.bufs[(k + 1) % 2]
            # with pipelined, the geometry of step k > k0 was prepared on the
            # auxiliary stream during step k-1
            self.s.step(a[0], a[1], b[0], b[1], u=self.u, vof_next=self.vofs[k],
                        sigma_out=self.sig, totals=self.hist[k])
            if forces is not None:
                cap, ma = self.s.interface_force(self.vofs[k], self.sig)
                forces.append(cap + ma + self.s.force(self.sig))
            if pipelined and k + 1 < k1:
                self.s.prepare_geometry(self.vofs[k + 1], self.aux)

    def result(self, k1):
        import torch
        torch.cuda.synchronize()
        F, P = self.bufs[k1 % 2]
        return (to_np(self.s.levelset()), to_np(F), to_np(P), to_np(self.sig),
                self.hist.cpu().numpy()[:k1].copy())


def assert_same(a, b):
    for name, x, y in zip(("chi", "F", "psi", "sigma", "totals"), a, b):
        assert np.array_equal(x, y), (name, float(np.max(np.abs(x - y))))


@pytest.mark.parametrize("prec", [F32, F64])
def test_pipelined_equals_plain(prec):
    import torch
    case = circle_case((150, 131), prec)
    K = 20
    plain = Runner(case, prec)
    plain.reset()
    with torch.cuda.stream(plain.main):
        plain.steps(0, K, pipelined=False)
    ref = plain.result(K)
    pipe = Runner(case, prec)
    pipe.reset()
    with torch.cuda.stream(pipe.main):
        pipe.steps(0, K, pipelined=True)
    assert_same(pipe.result(K), ref)
    assert pipe.s.status() == plain.s.status() == 0


@pytest.mark.parametrize("prec", [F32, F64])
def test_interface_forces_between_pipelined_steps(prec):
    # the force kernels (interfacial, and the Marangoni force from the level
    # set) read the current level set while the next step's geometry is
    # prepared into the other buffer: forces and fields equal those of the
    # unpipelined run bit for bit
    import torch
    case = circle_case((150, 131), prec)
    K = 12
    runs = []
    for pipelined in (False, True):
        r = Runner(case, prec)
        r.reset()
        f = []
        with torch.cuda.stream(r.main):
            r.steps(0, K, pipelined=pipelined, forces=f)
        runs.append((r.result(K), [[to_np(x) for x in fk] for fk in f], r.s.status()))
    (ref, fref, st0), (got, fgot, st1) = runs
    assert_same(got, ref)
    assert st0 == st1 == 0
    assert len(fgot) == len(fref) == K
    for k in range(K):
        for x, y in zip(fgot[k], fref[k]):
            assert np.array_equal(x, y), k
    assert max(np.max(np.abs(x)) for x in fref[-1]) > 0


def test_pipelined_equals_plain_full_size():
    # 1024^2: the live-tile pass no longer fits the GPU at once next to the
    # transport, so its workgroups start at different times; every one must
    # still rank the same live tiles (a tile missed would keep stale values
    # and raise the interface-jump status bit on the next step)
    import torch
    case = circle_case((1024, 1024), F32, R0=0.2)
    K = 24
    plain = Runner(case, F32)
    plain.reset()
    with torch.cuda.stream(plain.main):
        plain.steps(0, K, pipelined=False)
    ref = plain.result(K)
    pipe = Runner(case, F32)
    pipe.reset()
    with torch.cuda.stream(pipe.main):
        pipe.steps(0, K, pipelined=True)
    assert_same(pipe.result(K), ref)
    assert pipe.s.status() == plain.s.status() == 0


def test_pipelined_graph_replays():
    # K steps captured once (the auxiliary stream joins the capture through
    # the events), replayed three times from the same start with eager work
    # and synchronisations in between; every replay equals the eager run
    import torch
    case = circle_case((150, 131), F32)
    K0, K = 2, 12
    eager = Runner(case, F32)
    eager.reset()
    with torch.cuda.stream(eager.main):
        eager.steps(0, K0 + K, pipelined=True)
    ref = eager.result(K0 + K)

    r = Runner(case, F32)
    r.reset()
    with torch.cuda.stream(r.main):
        r.steps(0, K0, pipelined=True)
    torch.cuda.synchronize()
    # the level set and state after K0 steps, to restart each replay from
    chi0 = r.s.levelset().clone()
    F0, P0 = [x.clone() for x in r.bufs[K0 % 2]]
    t0 = r.hist[K0 - 1, S.T_T:S.T_T + 1].clone()  # the running time after K0 steps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=r.main):
        r.steps(K0, K0 + K, pipelined=True)
    torch.cuda.synchronize()
    for rep in range(3):
        with torch.cuda.stream(r.main):
            r.s.set_levelset(chi0)
            # the replay starts from the level set, the state and the running
            # time after K0 steps (the time keys the FP32 stochastic
            # rounding); the cumulative totals restart
            r.s.init_state(r.c0, 1.0, 0.3)
            r.s.set_time(t0)
            r.bufs[K0 % 2][0].copy_(F0)
            r.bufs[K0 % 2][1].copy_(P0)
            r.hist.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(r.main):
            g.replay()
        torch.cuda.synchronize()
        got = r.result(K0 + K)
        for name, x, y in zip(("chi", "F", "psi", "sigma"), got[:4], ref[:4]):
            assert np.array_equal(x, y), (rep, name, float(np.max(np.abs(x - y))))
        # per-step totals except the running time and cumulative sums, which
        # restart at the replay's first step
        cols = [S.T_MB, S.T_MS, S.T_SDELTA, S.T_SSIGD, S.T_SU, S.T_MINPSI, S.T_GAVG, S.T_SAVG]
        assert np.array_equal(got[4][K0:, cols], ref[4][K0:, cols]), rep


def test_prepare_errors():
    import torch
    case = circle_case((96, 96), F32)
    r = Runner(case, F32)
    r.reset()
    with torch.cuda.stream(r.main):
        a, b = r.bufs[0], r.bufs[1]
        r.s.step(a[0], a[1], b[0], b[1], u=r.u, vof_next=r.vofs[0], sigma_out=r.sig)
        r.s.prepare_geometry(r.vofs[1], r.aux)
        # a second prepare, a different VoF and the level-set calls are refused
        for call in (lambda: r.s.prepare_geometry(r.vofs[2], r.aux),
                     lambda: r.s.step(b[0], b[1], a[0], a[1], u=r.u, vof_next=r.vofs[2],
                                      sigma_out=r.sig),
                     lambda: r.s.set_geometry(r.vofs[2], full=True),
                     lambda: r.s.levelset()):
            with pytest.raises(S.SurfError):
                call()
        # the pending geometry is consumed by the step with its VoF
        r.s.step(b[0], b[1], a[0], a[1], u=r.u, vof_next=r.vofs[1], sigma_out=r.sig)
    torch.cuda.synchronize()
    # a 3D paper-form context does not take the pipelined path
    n = (20, 18, 16)
    s3 = S.Surf(dict(dim=3, n=n, h=1.0 / 20, bc=((0, 0), (0, 0), (0, 0)), flux_form=1), 1e-4,
                F32)
    vof = s3.tensor(synth.vof_ball(n, 1.0 / 20, (0.5, 0.45, 0.4), 0.2, 3))
    s3.set_geometry(vof, full=True)
    with pytest.raises(S.SurfError):
        s3.prepare_geometry(vof, torch.cuda.Stream())


@pytest.mark.parametrize("dim", [2, 3])
def test_time_transport_matches_step(dim):
    # the measurement entry runs the step's own transport kernel: its outputs
    # equal those of surf_step with the same inputs, and the running state
    # (time, totals of the next step) is left alone
    import torch
    if dim == 2:
        n, h = (150, 131), 1.0 / 150
        prob = dict(dim=2, n=n, h=h, bc=((2, 2), (1, 1)), eos=1, eos_E=0.3)
        cen = (0.5, 0.42, 0)
        u = synth.u_source2d(n, h, cen, 0.05)
    else:
        n, h = (70, 40, 20), 1.0 / 70
        prob = dict(dim=3, n=n, h=h, bc=((2, 2), (0, 0), (1, 1)), eos=1, eos_E=0.3)
        cen = (0.5, 0.28, 0.14)
        u = synth.u_hadamard(n, h, cen, 0.1, -0.3, 0.01)
    vof = synth.vof_ball(n, h, cen, 0.1, dim)
    c0 = synth.uniform_field(n, 3, 0.8, 1.2)
    dt = 0.1 * h * h / 1e-2
    s = S.Surf(prob, dt, F32)
    T = s.tensor
    s.set_geometry(T(vof), full=True)
    F, P = s.init_state(T(c0), 1.0, 0.4)
    ud = [T(x) for x in u]
    F1, P1, S1 = s.empty(), s.empty(), s.empty()
    F2, P2, S2 = s.empty(), s.empty(), s.empty()
    tot1 = torch.zeros(16, dtype=torch.float64, device="cuda")
    tot2 = torch.zeros(16, dtype=torch.float64, device="cuda")
    ms = s.time_transport(F, P, F2, P2, u=ud, sigma_out=S2, reps=3)
    assert ms > 0
    s.step(F, P, F1, P1, u=ud, sigma_out=S1, totals=tot1)
    torch.cuda.synchronize()
    for a, b in ((F1, F2), (P1, P2), (S1, S2)):
        assert torch.equal(a, b)
    # a second context without the timing call gives the same first step
    s2 = S.Surf(prob, dt, F32)
    s2.set_geometry(T(vof), full=True)
    Fb, Pb = s2.init_state(T(c0), 1.0, 0.4)
    s2.step(Fb, Pb, F2, P2, u=ud, sigma_out=S2, totals=tot2)
    torch.cuda.synchronize()
    assert torch.equal(tot1, tot2)


def sphere_case(n, precision, K=16, steps=12):
    # a sphere translating along periodic z through open x and y sides,
    # carried by a uniform flow, VoF recomputed every step, K warm-start
    # sweeps per step
    nx, ny, nz = n
    h = 1.0 / nx
    U, R = 0.5, 0.2
    dt = 0.1 * h * h / 1e-2  # below the 3D explicit bound (about 0.128 h^2 / D_b here)
    prob = dict(dim=3, n=n, h=h, bc=((2, 2), (2, 2), (1, 1)), eos=1, eos_E=0.2,
                hj_iters_step=K)
    Lz = nz * h
    cen = lambda t: (0.5 * nx * h, 0.47 * ny * h, (0.3 * Lz + U * t) % Lz)
    vof0 = synth.vof_ball(n, h, cen(0.0), R, 3, period_z=Lz)
    vofs = [synth.vof_ball(n, h, cen((k + 1) * dt * 60), R, 3, period_z=Lz)
            for k in range(steps)]
    u = synth.u_uniform(n, 3, (0.0, 0.0, U))
    c0 = synth.uniform_field(n, 6, 0.8, 1.2)
    return prob, dt, vof0, vofs, u, c0


@pytest.mark.parametrize("prec", [F32, F64])
def test_pipelined_equals_plain_3d(prec):
    # 3D: the next geometry sweeps both level-set buffers on the auxiliary
    # stream while the transport reads the snapshot; bitwise equal to plain
    # steps (the sphere moves 60 steps' worth per step so that tiles turn
    # live and quiescent)
    import torch
    case = sphere_case((72, 64, 80), prec)
    K = 12
    plain = Runner(case, prec)
    plain.reset()
    with torch.cuda.stream(plain.main):
        plain.steps(0, K, pipelined=False)
    ref = plain.result(K)
    pipe = Runner(case, prec)
    pipe.reset()
    with torch.cuda.stream(pipe.main):
        pipe.steps(0, K, pipelined=True)
    assert_same(pipe.result(K), ref)
    # the interface outruns the flow here (F stays where phi drops), so the
    # negative and unstable bits are raised; both runs raise the same ones
    assert pipe.s.status() == plain.s.status()


def test_pipelined_3d_graph_replay():
    import torch
    case = sphere_case((72, 64, 80), F32)
    K0, K = 1, 10
    eager = Runner(case, F32)
    eager.reset()
    with torch.cuda.stream(eager.main):
        eager.steps(0, K0 + K, pipelined=True)
    ref = eager.result(K0 + K)
    r = Runner(case, F32)
    r.reset()
    with torch.cuda.stream(r.main):
        r.steps(0, K0, pipelined=True)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=r.main):
        r.steps(K0, K0 + K, pipelined=True)
    g.replay()
    assert_same(r.result(K0 + K), ref)
