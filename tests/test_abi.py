"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "surf.h")).read()
    return sorted(set(re.findall(r"\b(surf_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2605_27534_amd import surf as S
    L = S.lib()
    syms = header_symbols()
    assert "surf_step" in syms and "surf_force" in syms
    for name in syms:
        assert hasattr(L, name), name
    assert set(S.EXPORTS) >= set(syms)
    assert L.surf_version().startswith(b"surf")


def _structs(**over):
    from paper_2605_27534_amd import surf as S
    prob = dict(dim=2, n=(32, 24), h=1.0 / 32, bc=((0, 0), (1, 1)))
    prob.update(over)
    return S.make_structs(prob, 1e-3, S.SURF_F32)


def test_workspace_bytes_and_init_validate_arguments():
    from paper_2605_27534_amd import surf as S
    L = S.lib()
    g, p, _ = _structs()
    nb = ctypes.c_size_t(0)
    assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
    assert nb.value >= 3 * 32 * 24 * 4
    # a host buffer stands in for the workspace: init issues no device work
    buf = ctypes.create_string_buffer(nb.value + 512)
    base = (ctypes.addressof(buf) + 255) // 256 * 256
    ctx = ctypes.c_void_p()
    assert L.surf_init(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p),
                       ctypes.c_void_p(base), nb, None) == 0
    # call-order checks happen before any launch
    assert L.surf_init_state(ctx, None, ctypes.c_double(1.0), ctypes.c_double(0.0),
                             ctypes.c_void_p(base), ctypes.c_void_p(base)) == -4
    assert L.surf_set_geometry(ctx, ctypes.c_void_p(base), 0) == -4
    assert L.surf_step(ctx, None, None, None, None, None, None, None, None) == -1
    # the step that keeps its advected state: 3D plane-marching contexts only;
    # the adjoint step that reads it: adjoint contexts only
    q = [ctypes.c_void_p(base + 256 * k) for k in range(8)]
    assert L.surf_step_advected(ctx, None, q[0], q[1], q[2], q[3], None, None, q[4], q[5]) == -1
    assert L.surf_step_advected(ctx, None, q[0], None, q[2], q[3], None, None, q[4], q[5]) == -1
    assert L.surf_adjoint_step_advected(None, None, q[0], q[1], q[2], q[3], q[4], q[5], None,
                                        q[6], q[7], q[0]) == -1
    assert L.surf_adjoint_step_advected(ctx, None, q[0], q[1], q[2], q[3], q[4], q[5], None,
                                        q[6], q[7], q[0]) == -4
    assert L.surf_set_dt(ctx, ctypes.c_double(-1.0)) == -1
    assert L.surf_destroy(ctx) == 0
    # too small a workspace, misaligned workspace
    ctx2 = ctypes.c_void_p()
    assert L.surf_init(ctypes.byref(ctx2), ctypes.byref(g), ctypes.byref(p),
                       ctypes.c_void_p(base), ctypes.c_size_t(nb.value - 1), None) == -2
    assert L.surf_init(ctypes.byref(ctx2), ctypes.byref(g), ctypes.byref(p),
                       ctypes.c_void_p(base + 8), nb, None) == -1


@pytest.mark.parametrize("over", [
    dict(dim=4), dict(n=(3, 24)), dict(bc=((1, 0), (0, 0))), dict(h=0.0),
    dict(n=(32, 24, 2)),
])
def test_bad_grids_rejected(over):
    from paper_2605_27534_amd import surf as S
    L = S.lib()
    g, p, _ = _structs(**over)
    nb = ctypes.c_size_t(0)
    assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == -1


def test_bad_params_rejected():
    from paper_2605_27534_amd import surf as S
    L = S.lib()
    for field, val in (("precision", 7), ("eos", 3), ("eps", 0.0), ("dt", 0.0),
                       ("gamma_inf", -1.0), ("k_a", -1.0)):
        g, p, _ = _structs()
        setattr(p, field, val)
        nb = ctypes.c_size_t(0)
        assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == -1, field


def test_strerror():
    from paper_2605_27534_amd import surf as S
    L = S.lib()
    assert L.surf_strerror(0) == b"ok"
    assert L.surf_strerror(-2) == b"workspace too small"


def test_batch_workspace_validates_instances():
    from paper_2605_27534_amd import surf as S
    from paper_2605_27534_amd.batch import _bind
    L = _bind(S.lib())
    probs = [dict(dim=2, n=(96, 80), h=1 / 96.0), dict(dim=2, n=(130, 70), h=1 / 130.0,
                                                       bc=((1, 1), (0, 0)))]
    grids = (S.Grid * 2)()
    params = (S.Params * 2)()
    for i, p in enumerate(probs):
        grids[i], params[i], _ = S.make_structs(p, 1e-4, S.SURF_F32)
    nb = ctypes.c_size_t(0)
    assert L.surf_batch_workspace_bytes(2, grids, params, ctypes.byref(nb)) == 0
    # two level sets and the per-tile records at least
    assert nb.value >= (96 * 80 + 130 * 70) * 4
    assert L.surf_batch_workspace_bytes(0, grids, params, ctypes.byref(nb)) == -1
    # mixed precision and a 3D instance are rejected
    params[1].precision = S.SURF_F64
    assert L.surf_batch_workspace_bytes(2, grids, params, ctypes.byref(nb)) == -1
    params[1].precision = S.SURF_F32
    g3, p3, _ = S.make_structs(dict(dim=3, n=(16, 16, 16), h=1 / 16.0), 1e-4, S.SURF_F32)
    grids[1], params[1] = g3, p3
    assert L.surf_batch_workspace_bytes(2, grids, params, ctypes.byref(nb)) == -1
    # rings: the weighted form (the column kernel) only
    ring = dict(dim=2, n=(64, 64), h=1 / 64.0, bc=((0, 2), (0, 0)), axisym=1)
    grids[1], params[1], _ = S.make_structs(ring, 1e-4, S.SURF_F32)
    assert L.surf_batch_workspace_bytes(2, grids, params, ctypes.byref(nb)) == 0
    grids[1], params[1], _ = S.make_structs(dict(ring, flux_form=1), 1e-4, S.SURF_F32)
    assert L.surf_batch_workspace_bytes(2, grids, params, ctypes.byref(nb)) == -1
    # creation needs device buffers: a null handle array is rejected first
    h = ctypes.c_void_p()
    assert L.surf_batch_create(ctypes.byref(h), 2, grids, params, None, None, None, None, 0,
                               None) == -1


def test_params_struct_matches_the_header():
    # the binding's surf_params mirrors include/surf.h: 8 int32, 13 doubles,
    # 4 int32, 1 double, 2 int32, 2 doubles, 2 int32, naturally aligned
    import ctypes
    from paper_2605_27534_amd import surf as S
    assert ctypes.sizeof(S.Params) == 8 * 4 + 13 * 8 + 4 * 4 + 8 + 2 * 4 + 2 * 8 + 2 * 4
    assert S.Params.cg_tol.offset == 8 * 4 + 13 * 8 + 4 * 4
    assert S.Params.acdi_vareps.offset == ctypes.sizeof(S.Params) - 16
    assert S.Params.transverse.offset == ctypes.sizeof(S.Params) - 4


def test_implicit_substep2_validation():
    import ctypes
    from paper_2605_27534_amd import surf as S
    L = S.lib()
    nb = ctypes.c_size_t(0)
    base = dict(dim=2, n=(32, 32), h=1 / 32, bc=((0, 0), (0, 0)), substep2=1)
    g, p, _ = S.make_structs(base, 1e-3, S.SURF_F32)
    assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
    ws_imp = nb.value
    g, p, _ = S.make_structs(dict(base, substep2=0), 1e-3, S.SURF_F32)
    assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
    assert ws_imp >= nb.value + 15 * 32 * 32 * 8  # the FP64 work arrays
    # the paper form solves by BiCGSTAB, with its coefficient B per axis
    g, p, _ = S.make_structs(dict(base, flux_form=1), 1e-3, S.SURF_F32)
    assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
    assert nb.value >= ws_imp + 2 * 32 * 32 * 8
    for bad in (dict(adjoint=1), dict(substep2=2), dict(picard_iters=-1),
                dict(picard_iters=33), dict(cg_tol=-1.0), dict(cg_max_iters=-1)):
        g, p, _ = S.make_structs(dict(base, **bad), 1e-3, S.SURF_F32)
        assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == -1, bad


def test_acdi_validation():
    import ctypes
    from paper_2605_27534_amd import surf as S
    L = S.lib()
    nb = ctypes.c_size_t(0)
    base = dict(dim=2, n=(32, 32), h=1 / 32, bc=((0, 0), (0, 0)), interface=1, acdi_zeta=0.5)
    g, p, _ = S.make_structs(base, 1e-3, S.SURF_F32)
    assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
    ws_acdi = nb.value
    g, p, _ = S.make_structs(dict(base, interface=0), 1e-3, S.SURF_F32)
    assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
    assert ws_acdi >= nb.value + 3 * 32 * 32 * 4  # phi, phi* and s
    for bad in (dict(acdi_zeta=0.0), dict(acdi_zeta=-1.0), dict(acdi_zeta=float("inf")),
                dict(acdi_vareps=-1e-6), dict(acdi_vareps=0.5), dict(interface=2),
                dict(adjoint=1)):
        g, p, _ = S.make_structs(dict(base, **bad), 1e-3, S.SURF_F32)
        assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == -1, bad


def test_axisym_validation():
    import ctypes
    from paper_2605_27534_amd import surf as S
    L = S.lib()
    nb = ctypes.c_size_t(0)
    base = dict(dim=2, n=(64, 64), h=1 / 64, bc=((0, 2), (0, 0)), axisym=1)
    g, p, _ = S.make_structs(base, 1e-3, S.SURF_F32)
    assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
    for bad in (dict(axisym=2), dict(bc=((1, 1), (0, 0))), dict(adjoint=1),
                dict(origin=(-0.1, 0.0, 0.0)),
                dict(dim=3, n=(64, 64, 8), bc=((0, 2), (0, 0), (0, 0)))):
        g, p, _ = S.make_structs(dict(base, **bad), 1e-3, S.SURF_F32)
        assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == -1, bad
    # the implicit substep, the ACDI interface and the paper form run on the
    # rings too
    for good in (dict(substep2=1), dict(interface=1, acdi_zeta=0.5),
                 dict(substep2=1, interface=1, acdi_zeta=0.5), dict(flux_form=1),
                 dict(flux_form=1, interface=1, acdi_zeta=0.5), dict(flux_form=1, substep2=1)):
        g, p, _ = S.make_structs(dict(base, **good), 1e-3, S.SURF_F32)
        assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0, good


def test_interface_force_validation():
    """surf_interface_force rejects missing inputs and half-given output sets
    before touching the device, and asks for a level set first (2D, rings
    and 3D)."""
    import ctypes
    from paper_2605_27534_amd import surf as S
    L = S.lib()

    def ctx_of(prob):
        g, p, _ = S.make_structs(prob, 1e-3, S.SURF_F32)
        nb = ctypes.c_size_t(0)
        assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
        buf = ctypes.create_string_buffer(nb.value + 512)
        base = (ctypes.addressof(buf) + 255) // 256 * 256
        ctx = ctypes.c_void_p()
        assert L.surf_init(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p),
                           ctypes.c_void_p(base), nb, None) == 0
        return ctx, buf, base

    two = dict(dim=2, n=(32, 24), h=1.0 / 32, bc=((0, 0), (1, 1)))
    ctx, buf, base = ctx_of(two)
    p = ctypes.c_void_p(base)
    pair = (ctypes.c_void_p * 2)(base, base)
    half = (ctypes.c_void_p * 2)(base, None)
    assert L.surf_interface_force(ctx, p, p, pair, pair) == -4  # no level set
    assert L.surf_interface_force(ctx, p, p, pair, None) == -4
    assert L.surf_interface_force(ctx, p, p, None, None) == -1
    assert L.surf_interface_force(ctx, None, p, pair, pair) == -1
    assert L.surf_interface_force(ctx, p, None, pair, pair) == -1
    assert L.surf_interface_force(ctx, p, p, half, pair) == -1
    assert L.surf_interface_force(ctx, p, p, pair, half) == -1
    assert L.surf_interface_force(None, p, p, pair, pair) == -1
    assert L.surf_destroy(ctx) == 0
    ctx, buf, base = ctx_of(dict(axisym=1, **dict(two, bc=((0, 2), (0, 0)))))
    assert L.surf_interface_force(ctx, p, p, pair, pair) == -4  # rings: no level set yet
    assert L.surf_interface_force(ctx, p, p, half, pair) == -1
    assert L.surf_destroy(ctx) == 0
    cube = dict(dim=3, n=(16, 16, 16), h=1.0 / 16, bc=((0, 0), (0, 0), (1, 1)))
    ctx, buf, base = ctx_of(cube)
    trip = (ctypes.c_void_p * 3)(base, base, base)
    part = (ctypes.c_void_p * 3)(base, base, None)
    assert L.surf_interface_force(ctx, p, p, trip, trip) == -4  # no level set
    assert L.surf_interface_force(ctx, p, p, None, trip) == -4
    assert L.surf_interface_force(ctx, p, p, trip, part) == -1
    assert L.surf_interface_force(ctx, p, p, None, None) == -1
    assert L.surf_destroy(ctx) == 0


def test_advection_variant_validation():
    """The MC limiter and the transverse term: the weighted form, no adjoint,
    no batch; either substep 2 in 2D (Cartesian or axisymmetric, the VoF or
    the ACDI interface) and in 3D."""
    import ctypes
    from paper_2605_27534_amd import surf as S
    L = S.lib()
    nb = ctypes.c_size_t(0)
    base = dict(dim=2, n=(64, 48), h=1 / 64, bc=((1, 1), (0, 2)), limiter=1, bcg_transverse=1)
    for ok in (dict(), dict(limiter=0), dict(bcg_transverse=0)):
        g, p, _ = S.make_structs(dict(base, **ok), 1e-3, S.SURF_F32)
        assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0, ok
    cube = dict(dim=3, n=(16, 16, 16), bc=((1, 1), (0, 2), (0, 0)))
    for ok in (dict(substep2=1), dict(cube, substep2=1), cube,
               dict(cube, interface=1, acdi_zeta=0.5)):
        g, p, _ = S.make_structs(dict(base, **ok), 1e-3, S.SURF_F32)
        assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0, ok
    g, p, _ = S.make_structs(dict(base, interface=1, acdi_zeta=0.5), 1e-3, S.SURF_F32)
    assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
    for bad in (dict(limiter=2), dict(bcg_transverse=-1), dict(flux_form=1), dict(adjoint=1),
                dict(cube, flux_form=1)):
        g, p, _ = S.make_structs(dict(base, **bad), 1e-3, S.SURF_F32)
        assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == -1, bad
    # on axisymmetric rings too
    g, p, _ = S.make_structs(dict(base, axisym=1, bc=((0, 2), (0, 0))), 1e-3, S.SURF_F32)
    assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
    g, p, _ = S.make_structs(base, 1e-3, S.SURF_F32)
    nbb = ctypes.c_size_t(0)
    assert L.surf_batch_workspace_bytes(1, ctypes.byref(g), ctypes.byref(p),
                                        ctypes.byref(nbb)) == -1


def test_prepare_phase_validation():
    """surf_prepare_phase: ACDI contexts on the weighted-form explicit path
    (2D or 3D), every velocity component, and a level set first; checked
    before any device work."""
    import ctypes
    from paper_2605_27534_amd import surf as S
    L = S.lib()

    def ctx_of(prob):
        g, p, _ = S.make_structs(prob, 1e-3, S.SURF_F32)
        nb = ctypes.c_size_t(0)
        assert L.surf_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == 0
        buf = ctypes.create_string_buffer(nb.value + 512)
        base = (ctypes.addressof(buf) + 255) // 256 * 256
        ctx = ctypes.c_void_p()
        assert L.surf_init(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p),
                           ctypes.c_void_p(base), nb, None) == 0
        return ctx, buf, base

    fake_stream = ctypes.c_void_p(1)  # never used: every check fails first
    acdi = dict(dim=2, n=(32, 32), h=1 / 32, bc=((0, 0), (0, 0)), interface=1, acdi_zeta=0.5)
    ctx, buf, base = ctx_of(acdi)
    assert L.surf_prepare_phase(ctx, None, None) == -1
    assert L.surf_prepare_phase(ctx, None, fake_stream) == -4  # no level set yet
    half = (ctypes.c_void_p * 3)(base, None, None)
    assert L.surf_prepare_phase(ctx, half, fake_stream) == -1
    assert L.surf_destroy(ctx) == 0
    cube = dict(dim=3, n=(16, 16, 16), bc=((0, 0), (0, 0), (0, 0)))
    ctx, buf, base = ctx_of(dict(acdi, **cube))
    assert L.surf_prepare_phase(ctx, None, fake_stream) == -4  # no level set yet
    two = (ctypes.c_void_p * 3)(base, base, None)
    assert L.surf_prepare_phase(ctx, two, fake_stream) == -1  # no z velocity
    assert L.surf_destroy(ctx) == 0
    for bad in (dict(interface=0), dict(flux_form=1), dict(cube, flux_form=1),
                dict(substep2=1)):
        ctx, buf, base = ctx_of(dict(acdi, **bad))
        assert L.surf_prepare_phase(ctx, None, fake_stream) == -1, bad
        assert L.surf_destroy(ctx) == 0
