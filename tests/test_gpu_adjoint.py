"""The GPU discrete adjoint (through the C ABI and the autograd wrapper)
against the FP64 oracle adjoint and against central differences."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_27534_amd import synth

pytestmark = pytest.mark.gpu


def problem(dim):
    if dim == 2:
        n = (40, 34)
        h = 1.0 / 40
        prob = dict(dim=2, n=n, h=h, bc=((0, 0), (2, 2)), eos=1, eos_E=0.3)
        chi = O.geometry(prob, synth.vof_ball(n, h, (0.5, 0.45, 0), 0.22, 2), 72)
        u = synth.u_rotation(n, h, (0.5, 0.45, 0), 1.0)
        u = [u[0] + 0.2, u[1] - 0.1]
        c0 = 1 + 0.1 * synth.smooth_modes(n, h, 4, dim=2)
        dt = 0.1 * h * h / 1e-2
    else:
        n = (16, 14, 12)
        h = 1.0 / 16
        prob = dict(dim=3, n=n, h=h, bc=((0, 0), (0, 0), (2, 2)), eos=1, eos_E=0.3)
        chi = O.geometry(prob, synth.vof_ball(n, h, (0.5, 0.45, 0.4), 0.25, 3), 108)
        u = synth.u_hadamard(n, h, (0.5, 0.45, 0.4), 0.25, -0.2, 0.01)
        c0 = 1 + 0.1 * synth.smooth_modes(n, h, 4)
        dt = 0.08 * h * h / 1e-2
    return prob, chi, u, c0, dt, n, h


def gpu_grad(prob, chi, u, c0, dt, N, theta, target, precision, K):
    import torch
    from paper_2605_27534_amd.adjoint import Rollout, SurfRollout
    ro = Rollout(prob, dt, precision, chi=chi, u=u, gamma0=0.2, nsteps=N, checkpoint=K)
    th = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
    c = torch.tensor(c0, dtype=ro.s.dtype, device="cuda", requires_grad=True)
    tg = torch.tensor(target, dtype=torch.float64, device="cuda")
    loss = SurfRollout.apply(th, c, ro, tg)
    gth, gc = torch.autograd.grad(loss, (th, c))
    return float(loss), gth.cpu().numpy(), gc.double().cpu().numpy()


@pytest.mark.parametrize("dim", [2, 3])
def test_fp64_adjoint_matches_oracle(dim):
    prob, chi, u, c0, dt, n, h = problem(dim)
    N = 12
    theta = np.array([1.3, 0.7, 0.012, 0.0008])
    target = np.linspace(0.97, 0.93, N)
    Lo, dto, gco = O.sigma_history_grad(prob, chi, u, c0, 0.2, dt, N, theta, target)
    Lg, dtg, gcg = gpu_grad(prob, chi, u, c0, dt, N, theta, target, 1, 5)
    assert abs(Lg - Lo) <= 1e-12 * Lo
    assert np.max(np.abs(dtg - dto) / np.abs(dto)) <= 1e-10, (dtg, dto)
    assert np.max(np.abs(gcg - gco)) <= 1e-10 * np.max(np.abs(gco))


@pytest.mark.parametrize("dim", [2, 3])
def test_fp32_adjoint_against_fp64_oracle(dim):
    # FP32 forward + adjoint against the FP64 oracle: the loss and the
    # gradients (each dtheta component relative to itself, dL/dc0 against its
    # max-norm) within 2e-5, the bar of the FP32 field comparisons
    prob, chi, u, c0, dt, n, h = problem(dim)
    N = 12
    theta = np.array([1.3, 0.7, 0.012, 0.0008])
    target = np.linspace(0.97, 0.93, N)
    Lo, dto, gco = O.sigma_history_grad(prob, chi, u, c0, 0.2, dt, N, theta, target)
    Lg, dtg, gcg = gpu_grad(prob, chi, u, c0, dt, N, theta, target, 0, 4)
    print("dim %d: loss %.3g, dtheta %s, dc0 %.3g" % (
        dim, abs(Lg - Lo) / Lo, np.abs(dtg - dto) / np.abs(dto),
        np.max(np.abs(gcg - gco)) / np.max(np.abs(gco))), flush=True)
    assert abs(Lg - Lo) <= 2e-5 * Lo
    assert np.max(np.abs(dtg - dto) / np.abs(dto)) <= 2e-5, (dtg, dto)
    assert np.max(np.abs(gcg - gco)) <= 2e-5 * np.max(np.abs(gco))


def test_checkpoint_interval_does_not_change_gradients():
    prob, chi, u, c0, dt, n, h = problem(2)
    N = 11
    theta = np.array([1.0, 1.0, 0.01, 0.001])
    target = np.linspace(0.97, 0.93, N)
    ref = gpu_grad(prob, chi, u, c0, dt, N, theta, target, 0, N)
    for K in (1, 3, 5):
        g = gpu_grad(prob, chi, u, c0, dt, N, theta, target, 0, K)
        assert g[0] == ref[0]
        assert np.array_equal(g[1], ref[1]) and np.array_equal(g[2], ref[2])


def test_gradients_match_central_differences_fp64():
    # GPU FP64 forward differences on the four scalars and 8 seeded smooth
    # directions of c0 against the adjoint
    import torch
    from paper_2605_27534_amd.adjoint import Rollout
    prob, chi, u, c0, dt, n, h = problem(2)
    N = 10
    theta = np.array([1.3, 0.7, 0.012, 0.0008])
    target = np.linspace(0.97, 0.93, N)
    _, dtg, gcg = gpu_grad(prob, chi, u, c0, dt, N, theta, target, 1, 4)
    ro = Rollout(prob, dt, 1, chi=chi, u=u, gamma0=0.2, nsteps=N, checkpoint=N)
    tg = torch.tensor(target, dtype=torch.float64, device="cuda")

    def L(th, c):
        loss, _, _, _ = ro.forward(torch.tensor(th, device="cuda", dtype=torch.float64),
                                   torch.tensor(c, device="cuda", dtype=torch.float64), tg)
        return float(loss)

    for k in range(4):
        e = np.zeros(4)
        e[k] = 1e-4 * theta[k]
        fd = (L(theta + e, c0) - L(theta - e, c0)) / (2 * e[k])
        assert abs(fd - dtg[k]) <= 1e-5 * abs(fd) + 1e-10, (k, fd, dtg[k])
    for seed in range(44, 52):
        v = synth.smooth_modes(n, h, seed, dim=2)
        e = 1e-4
        fd = (L(theta, c0 + e * v) - L(theta, c0 - e * v)) / (2 * e)
        assert abs(fd - (gcg * v).sum()) <= 1e-5 * abs(fd) + 1e-10, seed


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("flow", [True, False])
def test_step_advected_state(prec, flow):
    # surf_step_advected: the outputs and totals of surf_step bit for bit, and
    # the advected state against the oracle's substep 1 (section 2.2) on the
    # same input state
    import torch
    from paper_2605_27534_amd import surf as S
    from tests.harness import rel_max, to_np
    prob, chi, u, c0, dt, n, h = problem(3)
    outs = []
    for keep in (False, True):  # a fresh context each (the totals accumulate)
        s = S.Surf(dict(prob), dt, prec)
        s.set_levelset(s.tensor(chi))
        F, P = s.init_state(s.tensor(c0), 1.0, 0.2)
        ug = [s.tensor(x) for x in u] if flow else None
        star = (s.empty(), s.empty()) if keep else None
        Fo, Po, sg = s.empty(), s.empty(), s.empty()
        tot = torch.zeros(16, dtype=torch.float64, device="cuda")
        s.step(F, P, Fo, Po, u=ug, sigma_out=sg, totals=tot, star=star)
        outs.append((Fo, Po, sg, tot, star))
    torch.cuda.synchronize()
    a, b = outs
    for x, y in zip(a[:4], b[:4]):
        assert torch.equal(x, y)
    Fs, Ps = (to_np(x) for x in b[4])
    if flow:
        Fo, _ = O.advect(prob, u, to_np(F), dt)
        Po, _ = O.advect(prob, u, to_np(P), dt)
        tol = 1e-13 if prec == 1 else 2e-6
        eF, eP = rel_max(Fs, Fo), rel_max(Ps, Po)
        print("advected state: F %.3g, psi %.3g" % (eF, eP), flush=True)
        assert eF <= tol and eP <= tol
    else:
        assert np.array_equal(Fs, to_np(F)) and np.array_equal(Ps, to_np(P))


@pytest.mark.parametrize("prec", [1, 0])
def test_backward_with_and_without_the_advected_state(prec):
    # the 3D backward pass reads the advected state the recomputation keeps;
    # the same gradients as the adjoint steps that advect again
    import torch
    from paper_2605_27534_amd.adjoint import Rollout, SurfRollout
    prob, chi, u, c0, dt, n, h = problem(3)
    N = 9
    theta = [1.3, 0.7, 0.012, 0.0008]
    target = torch.tensor(np.linspace(0.97, 0.93, N), dtype=torch.float64, device="cuda")
    res = []
    for keep in (None, False):
        ro = Rollout(prob, dt, prec, chi=chi, u=u, gamma0=0.2, nsteps=N, checkpoint=4)
        ro.keep_advected = keep
        th = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
        c = torch.tensor(c0, dtype=ro.s.dtype, device="cuda", requires_grad=True)
        loss = SurfRollout.apply(th, c, ro, target)
        gth, gc = torch.autograd.grad(loss, (th, c))
        res.append((gth.cpu().numpy(), gc.double().cpu().numpy()))
        assert ro.keep_advected is (True if keep is None else False)
    (t1, c1), (t2, c2) = res
    tol = 1e-12 if prec == 1 else 1e-5
    assert np.max(np.abs(t1 - t2) / np.abs(t2)) <= tol, (t1, t2)
    assert np.max(np.abs(c1 - c2)) <= tol * np.max(np.abs(c2))


def test_advected_state_entry_points_validation():
    import torch
    from paper_2605_27534_amd import surf as S
    prob, chi, u, c0, dt, n, h = problem(3)
    s = S.Surf(dict(prob, adjoint=1), dt, 1)
    s.set_levelset(s.tensor(chi))
    F, P = s.init_state(s.tensor(c0), 1.0, 0.2)
    Fo, Po, Fs, Ps = (s.empty() for _ in range(4))
    for star in ((Fs, Po), (Fo, Ps), (F, Ps), (Fs, P)):  # aliased outputs
        with pytest.raises(S.SurfError) as e:
            s.step(F, P, Fo, Po, star=star)
        assert e.value.code == -1
    s.step(F, P, Fo, Po, star=(Fs, Ps))
    lF, lP, mF, mP = (s.empty() for _ in range(4))
    dth = torch.zeros(4, dtype=torch.float64, device="cuda")
    for out in ((Fs, lP), (lF, Ps)):  # an adjoint output on the advected state
        with pytest.raises(S.SurfError) as e:
            s.adjoint_step(F, P, mF, mP, out[0], out[1], dth, star=(Fs, Ps))
        assert e.value.code == -1
    # a 2D context has no such step; the rollout falls back to the plain one
    p2, chi2, u2, c02, dt2, _, _ = problem(2)
    s2 = S.Surf(dict(p2), dt2, 1)
    s2.set_levelset(s2.tensor(chi2))
    F2, P2 = s2.init_state(s2.tensor(c02), 1.0, 0.2)
    with pytest.raises(S.SurfError) as e:
        s2.step(F2, P2, s2.empty(), s2.empty(), star=(s2.empty(), s2.empty()))
    assert e.value.code == -1
    torch.cuda.synchronize()
