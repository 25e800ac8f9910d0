"""Parity of the interfacial forces (section 2.4; the HIP path through the C
ABI, surf_interface_force) with the FP64 oracle of `oracle/capillary.py` on
the same seeded inputs: the capillary and the Marangoni force on the x and y
faces.  The level set is the oracle's (installed with surf_set_levelset), so
the comparison isolates the force kernel.  Tolerances: FP64 1e-12 and FP32
2e-5, relative max-norm per face array; at 1024^2 on sampled faces, each
against the largest force of its array."""
import math

import numpy as np
import pytest

from oracle import capillary as K
from oracle import oracle as O
from paper_2605_27534_amd import surf as S
from paper_2605_27534_amd import synth
from tests.harness import rel_max, to_np
from tests.test_oracle_capillary import diagonal_stripes

pytestmark = pytest.mark.gpu

F64, F32 = 1, 0
TOL = {F64: 1e-12, F32: 2e-5}


def rounded(a, prec):
    a = np.asarray(a, dtype=np.float64)
    return a.astype(np.float32).astype(np.float64) if prec == F32 else a


def gpu_forces(prob, vof, chi, sig, prec, cap=True, ma=True):
    s = S.Surf(dict(prob), 1e-4, prec)
    T = s.tensor
    s.set_levelset(T(chi))
    c, m = s.interface_force(T(vof), T(sig), cap=cap, ma=ma)
    import torch
    torch.cuda.synchronize()
    return ([to_np(x) for x in c] if c is not None else None,
            [to_np(x) for x in m] if m is not None else None)


def compare(prob, vof, chi, sig, prec, curved=True):
    vof, chi, sig = (rounded(a, prec) for a in (vof, chi, sig))
    cap_o, ma_o = K.forces(prob, vof, chi, sig)
    cap_g, ma_g = gpu_forces(prob, vof, chi, sig, prec)
    for d in range(2):
        assert cap_g[d].shape == cap_o[d].shape
        e1 = rel_max(cap_g[d], cap_o[d])
        e2 = rel_max(ma_g[d], ma_o[d])
        print("prec %d axis %d: capillary %.3g, Marangoni %.3g" % (prec, d, e1, e2), flush=True)
        assert e1 <= TOL[prec], ("capillary", d, e1)
        assert e2 <= TOL[prec], ("marangoni", d, e2)
        assert np.max(np.abs(cap_o[d])) > 0 or not curved
    assert max(np.max(np.abs(m)) for m in ma_o) > 0
    return cap_o, ma_o, cap_g, ma_g


def disc_case(n, h, centre, R, bc, seed, images=()):
    prob = dict(dim=2, n=n, h=h, bc=bc)
    vof = synth.vof_disc(n, h, centre, R)
    for off in images:  # periodic images of the disc
        vof = vof + synth.vof_disc(n, h, (centre[0] + off[0], centre[1] + off[1], 0), R)
    chi = O.geometry(prob, vof, 80)
    sig = 1.0 + 0.2 * synth.smooth_modes(n, h, seed, dim=2)
    return prob, vof, chi, sig


@pytest.mark.parametrize("prec", [F64, F32])
def test_disc_between_walls(prec):
    # 64 x 48 (13 workgroups of nodes, a ragged last one), walls, an
    # off-centre disc with a varying sigma
    prob, vof, chi, sig = disc_case((64, 48), 1.0 / 64, (0.47, 0.39, 0), 0.21,
                                    ((0, 0), (0, 0)), seed=11)
    compare(prob, vof, chi, sig, prec)


@pytest.mark.parametrize("prec", [F64, F32])
def test_disc_across_the_periodic_side_and_near_a_wall(prec):
    # periodic in x (the disc wraps round it), walls in y with the disc two
    # cells from the bottom: mirrored height columns fall back to the level
    # set; open top side
    n, h = (70, 40), 1.0 / 64
    Lx = n[0] * h
    prob, vof, chi, sig = disc_case(n, h, (0.06, 0.17, 0), 0.14, ((1, 1), (0, 2)), seed=12,
                                    images=((Lx, 0.0),))
    assert vof.max() <= 1.0 + 1e-12
    compare(prob, vof, chi, sig, prec)


def rings_case(n, h, centre, R, bc, seed, r0=0.0):
    prob = dict(dim=2, n=n, h=h, bc=bc, axisym=1, origin=(r0, 0.0, 0.0))
    vof = synth.vof_disc(n, h, centre, R, origin=(r0, 0.0, 0.0))
    chi = O.geometry(prob, vof, 80)
    sig = 1.0 + 0.2 * synth.smooth_modes(n, h, seed, dim=2, origin=(r0, 0.0, 0.0))
    return prob, vof, chi, sig


@pytest.mark.parametrize("prec", [F64, F32])
def test_rings_sphere_on_the_axis(prec):
    # axisymmetric rings: a sphere of fluid 1 on the axis (wall at r = 0, open
    # outside, periodic z); the azimuthal curvature and the swept-area delta
    prob, vof, chi, sig = rings_case((40, 72), 1.0 / 72, (0.0, 0.5, 0), 0.27,
                                     ((0, 2), (1, 1)), seed=14)
    cap_o, ma_o, cap_g, ma_g = compare(prob, vof, chi, sig, prec)


@pytest.mark.parametrize("prec", [F64, F32])
def test_rings_torus_off_the_axis(prec):
    # an annular box (r from 0.2, walls on both radial sides, open in z) with
    # a ring of fluid 1 (a torus in 3D) away from the axis
    prob, vof, chi, sig = rings_case((48, 40), 1.0 / 64, (0.55, 0.3, 0), 0.16,
                                     ((0, 0), (2, 2)), seed=15, r0=0.2)
    compare(prob, vof, chi, sig, prec)


def test_diagonal_stripes_fp64():
    # 45-degree lines on a periodic box: exact Youngs normals, ties between
    # the column directions, the PLIC chord through cell corners
    n = 40
    prob = dict(dim=2, n=(n, n), h=1.0 / n, bc=((1, 1), (1, 1)))
    vof = diagonal_stripes(n)
    chi = O.geometry(prob, vof, 80)
    sig = 1.0 + 0.2 * synth.smooth_modes((n, n), 1.0 / n, 13, dim=2)
    cap_o, _, cap_g, _ = compare(prob, vof, chi, sig, F64, curved=False)
    assert max(np.max(np.abs(c)) for c in cap_g) == 0.0  # straight lines


def test_flat_interface_and_uniform_sigma_fp64():
    n = 32
    h = 1.0 / n
    prob = dict(dim=2, n=(n, n), h=h, bc=((1, 1), (0, 0)))
    vof = synth.vof_flat((n, n), h, 0.5 + 0.25 * h)
    chi = O.geometry(prob, vof, 80)
    x = (np.arange(n) + 0.5) * h
    sig = np.broadcast_to((1.0 + 0.1 * np.sin(2 * math.pi * x))[None, None, :], (1, n, n)).copy()
    cap_o, ma_o, cap_g, ma_g = compare(prob, vof, chi, sig, F64, curved=False)
    # a flat interface has no curvature; uniform sigma has no Marangoni force
    assert max(np.max(np.abs(c)) for c in cap_g) < 1e-10
    prob2, vof2, chi2, _ = disc_case((48, 48), 1.0 / 48, (0.52, 0.49, 0), 0.3,
                                     ((0, 0), (0, 0)), seed=14)
    _, ma = gpu_forces(prob2, vof2, chi2, np.full(vof2.shape, 0.7), F64, cap=False)
    assert max(np.max(np.abs(m)) for m in ma) < 1e-12


def test_one_pair_only_and_validation():
    prob, vof, chi, sig = disc_case((32, 32), 1.0 / 32, (0.5, 0.5, 0), 0.3, ((0, 0), (0, 0)), 15)
    cap, ma = gpu_forces(prob, vof, chi, sig, F64, ma=False)
    assert ma is None and cap is not None
    cap_o, _ = K.forces(prob, vof, chi, sig)
    assert rel_max(cap[0], cap_o[0]) <= 1e-12
    s = S.Surf(dict(prob), 1e-4, F64)
    T = s.tensor
    with pytest.raises(S.SurfError) as e:  # no level set yet
        s.interface_force(T(vof), T(sig))
    assert e.value.code == -4
    s.set_levelset(T(chi))
    with pytest.raises(S.SurfError) as e:
        s.interface_force(T(vof), T(sig), cap=False, ma=False)
    assert e.value.code == -1


@pytest.mark.parametrize("prec", [F32])
def test_expanding_circle_size_sampled(prec):
    # the 1024^2 expanding-circle workload (the VoF of its first step, 8x8
    # subsamples per cell) with the circle's clamped signed distance as the
    # level set; faces next to the interface and random others, against the
    # oracle face by face
    from paper_2605_27534_amd import configs as C
    import torch
    cfg = C.c1_expanding_circle()
    prob = dict(cfg["prob"], hj_iters_step=8)
    n = prob["n"]
    s = S.Surf(prob, cfg["dt"], prec)
    T = s.tensor
    vof = rounded(cfg["vof0"](), prec)
    sig = rounded(1.0 + 0.2 * synth.smooth_modes(n, prob["h"], 16, dim=2), prec)
    q = O.full(prob)
    chi = rounded(synth.distance_ball(n, prob["h"], (0.5, 0.5, 0), 0.1,
                                      q["chi_max_eps"] * q["eps"]), prec)
    s.set_levelset(T(chi))
    c, m = s.interface_force(T(vof), T(sig))
    torch.cuda.synchronize()
    cap_g, ma_g = [to_np(x) for x in c], [to_np(x) for x in m]
    rng = np.random.default_rng(17)
    v = vof[0]
    cut = (v > K.CUT) & (v < 1 - K.CUT)
    jj, ii = np.nonzero(cut)
    for d in range(2):
        faces = set()
        for j, i in zip(jj, ii):  # the two faces of each interfacial cell along d
            faces.add((j, i))
            faces.add((j + (d == 1), i + (d == 0)))
        faces = sorted(faces)
        pick = [faces[k] for k in rng.choice(len(faces), size=min(400, len(faces)),
                                             replace=False)]
        shp = cap_g[d].shape[1:]
        pick += [(int(rng.integers(shp[0])), int(rng.integers(shp[1]))) for _ in range(100)]
        scale_c = np.max(np.abs(cap_g[d]))
        scale_m = np.max(np.abs(ma_g[d]))
        assert scale_c > 0 and scale_m > 0
        worst_c = worst_m = 0.0
        for (j, i) in pick:
            fc, fm = K.face_force(prob, vof, chi, sig, d, j, i)
            worst_c = max(worst_c, abs(cap_g[d][0, j, i] - fc) / scale_c)
            worst_m = max(worst_m, abs(ma_g[d][0, j, i] - fm) / scale_m)
        print("axis %d: %d faces, capillary %.3g, Marangoni %.3g" % (d, len(pick), worst_c,
                                                                     worst_m), flush=True)
        assert worst_c <= TOL[prec] and worst_m <= TOL[prec]
