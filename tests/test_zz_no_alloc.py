"""surf_step_static, the allocation-free step (for callers that cannot
allocate device memory), against surf_step on the same inputs: two calls in
a row on one device, the second on a smaller grid, in 2D and 3D, FP32 and
FP64.  The two entry points run the same kernels, so the fields and the
totals must agree bit for bit."""
import numpy as np
import pytest
import torch

from paper_2605_27534_amd import surf as S
from paper_2605_27534_amd import synth

pytestmark = pytest.mark.gpu


def step_static(prob, dt, prec, chi, u, F, P, F2, P2, sig, tot):
    return S.step_static(prob, dt, prec, chi, F, P, F2, P2, u=u, sigma_out=sig, totals=tot)


def case(dim, big):
    if dim == 2:
        n = (300, 212) if big else (130, 75)
        h = 1.0 / n[0]
        prob = dict(dim=2, n=n, h=h, bc=((2, 2), (1, 1)), eos=1, eos_E=0.3, k_a=1.5, k_d=0.7)
        cen = (0.47, 0.33, 0)
        vof = synth.vof_ball(n, h, cen, 0.17 if big else 0.2, 2)
        u = synth.u_source2d(n, h, cen, 0.05)
    else:
        n = (70, 64, 50) if big else (40, 36, 20)
        h = 1.0 / n[0]
        prob = dict(dim=3, n=n, h=h, bc=((2, 2), (0, 0), (1, 1)), eos=1, eos_E=0.3, k_a=1.5,
                    k_d=0.7)
        cen = (0.45, 0.42, 0.25)
        vof = synth.vof_ball(n, h, cen, 0.17, 3, period_z=n[2] * h)
        u = synth.u_hadamard(n, h, cen, 0.17, -0.3, 0.01)
    c0 = synth.uniform_field(n, 7, 0.8, 1.2)
    dt = 0.1 * h * h / 1e-2
    return prob, vof, u, c0, dt


@pytest.mark.parametrize("prec", [S.SURF_F64, S.SURF_F32])
@pytest.mark.parametrize("dim", [2, 3])
def test_static_step_matches_surf_step(dim, prec):
    for big in (True, False):
        prob, vof, u, c0, dt = case(dim, big)
        s = S.Surf(prob, dt, prec)
        T = s.tensor
        s.set_geometry(T(vof), full=True)
        chi = s.levelset().contiguous()
        F, P = s.init_state(T(c0), 1.0, 0.3)
        ud = [T(x) for x in u]
        # three steps through each entry point from the same state
        Fa, Pa = F.clone(), P.clone()
        Fb, Pb = F.clone(), P.clone()
        ta = torch.zeros((3, 16), dtype=torch.float64, device="cuda")
        tb = torch.zeros((3, 16), dtype=torch.float64, device="cuda")
        sa, sb = s.empty(), s.empty()
        for k in range(3):
            Fn, Pn = s.empty(), s.empty()
            s.step(Fa, Pa, Fn, Pn, u=ud, sigma_out=sa, totals=ta[k])
            Fa, Pa = Fn, Pn
            Fm, Pm = s.empty(), s.empty()
            if k > 0:
                tb[k].copy_(tb[k - 1])  # running time and outflow from the previous call
            rc = step_static(prob, dt, prec, chi, ud, Fb, Pb, Fm, Pm, sb, tb[k])
            assert rc == 0, rc
            Fb, Pb = Fm, Pm
        torch.cuda.synchronize()
        for x, y in ((Fa, Fb), (Pa, Pb), (sa, sb)):
            assert torch.equal(x, y)
        assert torch.equal(ta, tb), (ta - tb).abs().max()
        s.close()


def test_static_step_rejects_oversized_and_unsupported():
    prob, vof, u, c0, dt = case(2, False)
    s = S.Surf(prob, dt, S.SURF_F32)
    T = s.tensor
    s.set_geometry(T(vof), full=True)
    chi = s.levelset().contiguous()
    F, P = s.init_state(T(c0), 1.0, 0.3)
    F2, P2 = s.empty(), s.empty()
    # the paper flux form runs another kernel: not offered here
    assert step_static(dict(prob, flux_form=1), dt, S.SURF_F32, chi, None, F, P, F2, P2, None,
                       None) == -1
    # a grid needing more than 4096 transport workgroups (58-column strips
    # by 32-row groups): rejected before any launch
    big = dict(prob, n=(58 * 64, 32 * 65))
    assert step_static(big, dt, S.SURF_F32, chi, None, F, P, F2, P2, None, None) == -2
    s.close()
