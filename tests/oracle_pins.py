"""Checks that pin parts of the FP64 oracle to what the paper and the
mathematics fix, written as plain functions so that the same check runs on
the oracle itself (tests/test_oracle_pins_*.py) and on copies of the oracle
with one mistake planted (tests/test_oracle_mutations.py), where it must
fail.  Each function raises AssertionError when its pin does not hold and
returns the measured figures otherwise."""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O

ETA = 1e-12


# ------------------------------------------------------------------ helpers
def _phi_of(prob, chi):
    phi, _, de = O.cell_geometry(prob, chi)
    return phi, de


def _tendency(prob, chi, F, P, dt):
    """(F+ - F)/dt and (psi+ - psi)/dt of one oracle step with u = 0."""
    Fo, Po, _, tot = O.step(prob, chi, None, F, P, dt)
    return (Fo - F) / dt, (Po - P) / dt, tot


def _flat_chi(prob, axis, x0):
    """Signed distance of the plane x_axis = x0 with fluid 1 (chi > 0) below."""
    q = O.full(prob)
    x, y, z = [(np.arange(m) + 0.5) * q["h"] for m in q["n"]]
    coord = (x, y, z)[axis]
    shp = [1, 1, 1]
    shp[2 - axis] = coord.size
    return np.broadcast_to((x0 - coord).reshape(shp), O.shape(prob)).copy()


# ------------------------------------------------- paper form: zero flux
def paper_form_zero_flux_residuals(dim=2, axis=0, eps=0.05, ratios=(2, 4, 8, 16), axisym=False):
    """The paper-form fluxes of substep 2 (section 2.6: D grad xi + B xi with
    B_F = -D (1 - phi) n / eps and B_psi = -D (1 - 2 phi) n / eps) vanish
    for F = c phi and psi = Gamma delta with c and Gamma uniform, whenever
    |grad phi| = phi (1 - phi)/eps, i.e. for the tanh profile of a plane.
    At fixed eps the discrete tendency of that state must therefore go to
    zero as h -> 0 (first order: the anti-diffusive flux is upwinded).

    Returns, per resolution h = eps / r, the max-norm tendency of F and psi
    scaled by D c / eps^2 and D Gamma / eps^3 (the size of the separate
    terms).

    axisym (dim 2, axis 0): the same on the rings of Appendix B with the
    plane r = 0.5, a cylinder of fluid 1 about the axis (the box's low x side
    on the axis): the fluxes vanish pointwise whatever weights their
    divergence takes, so the tendency goes to zero in the same way."""
    out = []
    D_b, D_s, c, G = 0.01, 0.002, 0.7, 0.4
    for r in ratios:
        h = eps / r
        N = int(round(1.0 / h))
        n = [4] * dim
        n[axis] = N
        bc = [(1, 1)] * dim
        bc[axis] = (0, 0)
        prob = dict(dim=dim, n=tuple(n), h=h, bc=tuple(bc), eps=eps, flux_form=1,
                    k_a=0.0, k_d=0.0, D_b=D_b, D_s=D_s)
        if axisym:
            assert dim == 2 and axis == 0
            prob["axisym"] = 1
        chi = _flat_chi(prob, axis, 0.5)
        assert np.max(np.abs(chi)) < 12 * eps  # no cell at the clamp
        phi, de = _phi_of(prob, chi)
        F = c * phi
        P = G * de
        dt = 1e-3 * h * h / D_b
        tF, tP, _ = _tendency(prob, chi, F, P, dt)
        out.append((np.max(np.abs(tF)) / (D_b * c / eps ** 2),
                    np.max(np.abs(tP)) / (D_s * G / eps ** 3)))
    out = np.array(out)
    # first order: each halving of h roughly halves the residual, and at
    # h = eps/16 it is a few per cent of the separate terms
    for k in range(len(ratios) - 1):
        assert 1.6 < out[k, 0] / out[k + 1, 0] < 2.5, out
        assert 1.6 < out[k, 1] / out[k + 1, 1] < 2.5, out
    assert out[-1, 0] < 0.05 and out[-1, 1] < 0.05, out
    return out


def paper_form_upwind_positivity(eps_over_h=0.5, dt_frac=0.5):
    """The anti-diffusive flux is a convective flux with velocity -B,
    upwinded (section 3.2).  With central diffusion and upwinded
    convection every off-diagonal coefficient of the explicit update is
    non-negative at any cell Peclet number |B| h / D; taken on the other
    side it turns negative once |B| h / D > 1.  At eps = h/2 that number
    reaches 2, so from a state of isolated non-negative spikes (stride 3, so
    that a cell next to a spike has a zero on its other side) one step of
    the upwinded form keeps every value non-negative (the diagonal is
    non-negative below the step bound) and a downwinded one does not.

    Returns the most negative value over the step, relative to the spike."""
    n = 48
    h = 1.0 / n
    eps = eps_over_h * h
    prob = dict(dim=2, n=(n, n), h=h, bc=((0, 0), (0, 0)), eps=eps, flux_form=1,
                k_a=0.0, k_d=0.0, D_b=1e-2, D_s=1e-2, cfl_diff=1.0)
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    chi = (0.3 - np.sqrt((X - 0.5) ** 2 + (Y - 0.47) ** 2))[None]
    chi = np.clip(chi, -12 * eps, 12 * eps)
    worst = 0.0
    dt = None
    for ox in range(3):
        for oy in range(3):
            F = np.zeros(O.shape(prob))
            F[0, oy::3, ox::3] = 1.0
            if dt is None:
                _, _, _, tot = O.step(prob, chi, None, F, F, 1e-12)
                dt = dt_frac * tot[O.T_DTNEXT]
            Fo, Po, _, _ = O.step(prob, chi, None, F, F, dt)
            worst = min(worst, Fo.min(), Po.min())
    assert worst >= -1e-15, worst
    return worst


# ------------------------------------------- the explicit step bound
def _stride2_patterns(dim):
    offs = [(0,), (1,)]
    for _ in range(dim - 1):
        offs = [o + (a,) for o in offs for a in (0, 1)]
    return offs


def _spike(prob, off):
    a = np.zeros(O.shape(prob))
    q = O.full(prob)
    if q["dim"] == 2:
        a[0, off[1]::2, off[0]::2] = 1.0
    else:
        a[off[2]::2, off[1]::2, off[0]::2] = 1.0
    return a


def diagonal_decrements(prob, chi, field, F_base=None, P_base=None, scale=1.0):
    """Per cell (1 - A_ii)/dt, A the linear map of one explicit step of
    `field` ('F' or 'psi') about the base state, from spikes on the 2^dim
    stride-2 sublattices (no two spikes share a face, and every stencil of
    the step reaches face neighbours only).  Also returns 1 / T_DTNEXT (the
    oracle's bound with cfl_diff = 1)."""
    q = O.full(prob)
    assert q["cfl_diff"] == 1.0
    Fb = np.zeros(O.shape(prob)) if F_base is None else F_base
    Pb = np.zeros(O.shape(prob)) if P_base is None else P_base
    _, _, _, tot = O.step(prob, chi, None, Fb, Pb, 1e-30)
    lam = 1.0 / tot[O.T_DTNEXT]
    dt = 0.5 / lam
    F0, P0, _, _ = O.step(prob, chi, None, Fb, Pb, dt)
    dec = np.zeros(O.shape(prob))
    for off in _stride2_patterns(q["dim"]):
        s = _spike(prob, off) * scale
        if field == "F":
            F1, _, _, _ = O.step(prob, chi, None, Fb + s, Pb, dt)
            resp = F1 - F0
        else:
            _, P1, _, _ = O.step(prob, chi, None, Fb, Pb + s, dt)
            resp = P1 - P0
        m = s > 0
        dec[m] = (1.0 - resp[m] / s[m]) / dt
    return dec, lam


def max_diagonal_decrement(prob, chi, field, **kw):
    dec, lam = diagonal_decrements(prob, chi, field, **kw)
    return float(dec.max()), lam


def _near_clamp(chi, chimax):
    """Cells at the clamp or with a face neighbour at it."""
    c = np.abs(chi) >= chimax * (1 - 1e-14)
    out = c.copy()
    for ax in range(chi.ndim):
        if chi.shape[ax] > 1:
            out |= np.roll(c, 1, ax) | np.roll(c, -1, ax)
    return out


def bound_weighted_diffusion(dim):
    """Weighted form (section 3.2 with the confinement weights phi and
    delta): the diagonal of the explicit diffusion of F is
    1 - dt D/h^2 sum_faces phibar_f / phi_i.  Along a grid-aligned normal,
    deep on the side where phi -> 0, neighbouring phi differ by e^{+-h/eps},
    so the sum is 2 dim - 2 + 1 + cosh(h/eps): inside the unclamped band the
    bound must be that, attained and never exceeded.  At the clamp edge the
    outer neighbour sits at the clamp, its weight equal to the cell's, and
    the normal axis contributes 1 + (1 + e^{h/eps})/2 instead: there the
    decrement exceeds the bound by at most (1 - e^{-h/eps})/2 over the sum."""
    n = 64 if dim == 2 else 40
    h = 1.0 / n
    nn = (n, 4) if dim == 2 else (n, 4, 4)
    bc = ((0, 0), (1, 1)) if dim == 2 else ((0, 0), (1, 1), (1, 1))
    prob = dict(dim=dim, n=nn, h=h, bc=bc, k_a=0.0, k_d=0.0, D_b=1e-2, D_s=1e-2,
                cfl_diff=1.0)
    chimax = 12 * 1.5 * h
    chi = np.clip(_flat_chi(prob, 0, 0.5), -chimax, chimax)
    edge = _near_clamp(chi, chimax)
    a = h / (1.5 * h)
    excess = (1 - math.exp(-a)) / 2 / (2 * dim - 1 + math.cosh(a))
    res = []
    for field in ("F", "psi"):
        dec, lam = diagonal_decrements(prob, chi, field)
        band, rim = dec[~edge].max(), dec[edge].max()
        assert band <= lam * (1 + 1e-12), (field, band, lam)
        assert band >= 0.99 * lam, (field, band, lam)
        assert rim <= lam * (1 + excess) * (1 + 1e-12), (field, rim, lam, excess)
        res.append((band / lam, rim / lam))
    return res


def _oblique_stripe_chi(prob, width=0.5):
    """Signed distance to a periodic stripe of fluid 1 between the planes
    sum_d x_d = 0.25 and 0.25 + width (mod 1), normal (1, .., 1)/sqrt(dim)."""
    q = O.full(prob)
    dim = q["dim"]
    cs = [(np.arange(m) + 0.5) * q["h"] for m in q["n"][:dim]]
    grids = np.meshgrid(*cs[::-1], indexing="ij")  # z, y, x (or y, x)
    s = np.mod(sum(grids), 1.0)
    c1, c2 = 0.25, 0.25 + width
    inside = (s > c1) & (s < c2)
    d_in = np.minimum(s - c1, c2 - s)
    d_out = np.minimum(np.mod(c1 - s, 1.0), np.mod(s - c2, 1.0))
    chi = np.where(inside, d_in, -d_out) / math.sqrt(dim)
    return chi.reshape(O.shape(prob))


def bound_paper_diffusion(dim):
    """Paper form: central diffusion (diagonal 2 dim D/h^2) plus the upwinded
    anti-diffusive flux, whose diagonal is sum over the faces the cell is
    upwind of |B_f|/h <= D sum_d |n_d| /(eps h) <= D sqrt(dim)/(eps h).  A
    plane with normal (1, .., 1)/sqrt(dim), deep in its tails (|1 - phi|,
    |1 - 2 phi| -> 1), attains it.  eps = 0.75 h, the paper's own choice."""
    n = 64 if dim == 2 else 48
    h = 1.0 / n
    eps = 0.75 * h
    prob = dict(dim=dim, n=(n,) * dim, h=h, bc=((1, 1),) * dim, eps=eps, flux_form=1,
                k_a=0.0, k_d=0.0, D_b=1e-2, D_s=1e-2, cfl_diff=1.0)
    chi = np.clip(_oblique_stripe_chi(prob), -12 * eps, 12 * eps)
    rF, lam = max_diagonal_decrement(prob, chi, "F")
    rP, _ = max_diagonal_decrement(prob, chi, "psi")
    assert rF <= lam * (1 + 1e-12) and rP <= lam * (1 + 1e-12), (rF, rP, lam)
    assert rF >= 0.99 * lam and rP >= 0.99 * lam, (rF, rP, lam)
    return rF / lam, rP / lam


def bound_adsorption():
    """Exchange source (section 2.6): with psi = 0 the bulk loses
    dt k_a c Gamma_inf delta = dt k_a Gamma_inf (delta/phi) F per step, and
    delta/phi = (1 - phi)/eps -> 1/eps where phi -> 0.  With no diffusion
    and a bulk far below saturation, the bound is k_a Gamma_inf/eps (+ the
    tiny k_a c_max), attained deep in fluid 1."""
    n = 64
    h = 1.0 / n
    prob = dict(dim=2, n=(n, 4), h=h, bc=((0, 0), (1, 1)), k_a=3.0, k_d=0.0,
                D_b=0.0, D_s=0.0, gamma_inf=2.0, cfl_diff=1.0)
    chi = np.clip(_flat_chi(prob, 0, 0.5), -18 * h, 18 * h)
    phi, _ = _phi_of(prob, chi)
    # F = 1e-6 phi: c = 1e-6 everywhere, so k_a c_max is negligible
    rF, lam = max_diagonal_decrement(prob, chi, "F", F_base=1e-6 * phi, scale=1e-9)
    assert rF <= lam * (1 + 1e-12), (rF, lam)
    assert rF >= 0.99 * lam, (rF, lam)
    return rF / lam


def bound_desorption():
    """Exchange source, interfacial side: psi loses dt (k_a c + k_d) psi per
    step (Langmuir), so with the bulk at c = c0 the bound must hold
    k_a c_max + k_d; with Gamma_inf tiny the k_a Gamma_inf/eps term drops
    out and it is attained everywhere."""
    n = 32
    h = 1.0 / n
    prob = dict(dim=2, n=(n, n), h=h, bc=((0, 0), (0, 0)), k_a=2.0, k_d=0.5,
                D_b=0.0, D_s=0.0, gamma_inf=1e-9, cfl_diff=1.0)
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    chi = np.clip(0.25 - np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2), -18 * h, 18 * h)[None]
    phi, _ = _phi_of(prob, chi)
    c0 = 1.7
    rP, lam = max_diagonal_decrement(prob, chi, "psi", F_base=c0 * (phi + ETA),
                                     P_base=np.zeros(O.shape(prob)), scale=1e-6 * phi.min())
    assert rP <= lam * (1 + 1e-9), (rP, lam)
    assert rP >= 0.99 * lam, (rP, lam)
    return rP / lam


# --------------------------------------------- Marangoni face force
def force_stencil_exact_for_quadratics(dim):
    """Section 2.4: F = delta (grad sigma - n (n . grad sigma)) on every face,
    n = grad chi / |grad chi|.  The face gradient (compact normal difference,
    the transverse centred differences of the two cells averaged) is exact
    for quadratic fields at the face centre, so with chi and sigma quadratic
    (with every cross term) the discrete force equals the closed form built
    from the exact gradients at the face centres, at every face whose
    stencil stays inside the box."""
    n = (20, 17, 14)[:dim]
    h = 1.0 / 20
    prob = dict(dim=dim, n=n, h=h, bc=((0, 0),) * dim)
    rng = np.random.default_rng(11)
    A = rng.normal(size=(dim, dim))
    A = 0.5 * (A + A.T)
    b = rng.normal(size=dim)
    S = rng.normal(size=(dim, dim))
    S = 0.5 * (S + S.T)
    g = rng.normal(size=dim)

    def field(M, v, c0, pts):
        return c0 + pts @ v + 0.5 * np.einsum("...i,ij,...j->...", pts, M, pts)

    cs = [(np.arange(m) + 0.5) * h - 0.5 for m in n]
    mesh = np.meshgrid(*cs[::-1], indexing="ij")
    pts = np.stack(mesh[::-1], axis=-1)  # (..., dim) in x, y, z order
    chi = 0.1 * field(A, b, 0.01, pts).reshape(O.shape(prob))
    sig = (0.07 + 0.01 * field(S, g, 0.0, pts)).reshape(O.shape(prob))
    fs = O.force(prob, chi, sig)
    _, _, de = O.cell_geometry(prob, chi)
    worst = 0.0
    for d in range(dim):
        # faces 2 .. n_d - 2 along d, cells 1 .. n_e - 2 across
        sl = [slice(1, m - 1) for m in n]
        sl[d] = slice(2, n[d] - 1)
        fc = [(np.arange(m) + 0.5) * h - 0.5 for m in n]
        fc[d] = np.arange(n[d] + 1) * h - 0.5
        fmesh = np.meshgrid(*fc[::-1], indexing="ij")
        fpts = np.stack(fmesh[::-1], axis=-1)
        gchi = 0.1 * (b + fpts @ A)
        gsig = 0.01 * (g + fpts @ S)
        nrm = np.linalg.norm(gchi, axis=-1, keepdims=True)
        nv = gchi / np.maximum(nrm, 1e-6)
        proj = gsig - nv * np.sum(nv * gsig, axis=-1, keepdims=True)
        # mean delta of the two cells of each face (the regularised delta
        # of section 2.6 is pinned on its own)
        dd = de.reshape([m for m in n][::-1])
        lo = [slice(None)] * dim
        hi = [slice(None)] * dim
        ax = dim - 1 - d
        lo[ax] = slice(0, n[d] - 1)
        hi[ax] = slice(1, n[d])
        dbar = 0.5 * (dd[tuple(lo)] + dd[tuple(hi)])
        pad = [(0, 0)] * dim
        pad[ax] = (1, 1)
        dbar = np.pad(dbar, pad)
        exp = (dbar * proj[..., d]).reshape(fs[d].shape)
        sel = tuple([slice(None)] * (3 - dim) + sl[::-1]) if dim == 3 else (slice(None),) + tuple(sl[::-1])
        err = np.max(np.abs(fs[d][sel] - exp[sel])) / np.max(np.abs(exp[sel]))
        worst = max(worst, err)
    assert worst < 1e-11, worst
    return worst


# ------------------------------------- periodic axes: the last face
def periodic_last_face_unread():
    """On a periodic axis face n_d is the same face as face 0.  The oracle
    reads face 0 wherever it needs it (fluxes, the transverse predictor,
    the cell-mean velocity of the step bound), so a different value in the
    array's last face changes nothing, totals included."""
    n = (24, 20, 16)
    h = 1.0 / 24
    prob = dict(dim=3, n=n, h=h, bc=((1, 1), (2, 2), (1, 1)), bcg_transverse=1, limiter=1)
    rng = np.random.default_rng(5)
    F = rng.uniform(0.5, 1.5, O.shape(prob))
    P = rng.uniform(0.0, 0.3, O.shape(prob))
    x = (np.arange(24) + 0.5) * h
    chi = np.broadcast_to(np.clip(0.4 - x, -0.5, 0.5), O.shape(prob)).copy()
    u = [rng.uniform(-1, 1, O.face_shape(prob, d)) for d in range(3)]
    u[0][..., 24] = u[0][..., 0]
    u[2][16] = u[2][0]
    a = O.step(prob, chi, u, F, P, 0.1 * h)
    ub = [v.copy() for v in u]
    ub[0][..., 24] = 50.0
    ub[2][16] = -50.0
    b = O.step(prob, chi, ub, F, P, 0.1 * h)
    for x1, x2 in zip(a[:3], b[:3]):
        assert np.array_equal(x1, x2)
    assert np.array_equal(a[3], b[3]), (a[3], b[3])
    return True


# ------------------------------------- implicit substep 2, paper form
def paper_implicit_residual(I=None, kinetics=1, axisym=False):
    """The implicit paper-form step (Appendix C with the paper's flux), with
    the Picard sweeps converged, satisfies its implicit equations when they
    are evaluated by the explicit C oracle: advancing the result by a tiny
    dt' with O.step gives (xi' - xi)/dt' = the right-hand side at xi, which
    must equal (xi - xi*)/dt.  A flipped anti-diffusive term or the wrong
    upwind cell in the implicit operator leaves a residual of the size of
    that term.  I: the implicit oracle module (a planted copy in the
    mutation tests).  axisym: on the rings of Appendix B (a sphere on the
    axis), where the explicit step is pinned by conservation and by the
    equilibrium profile about a cylinder, so that a missing or misplaced
    ring weight in the implicit operator leaves a residual too."""
    if I is None:
        from oracle import implicit as I
    from paper_2605_27534_amd import synth
    n = (40, 32)
    h = 1.0 / 40
    prob = dict(dim=2, n=n, h=h, bc=((0, 0), (1, 1)), kinetics=kinetics, eos=1, eos_E=0.3,
                D_b=1e-2, D_s=2e-3, k_a=2.0, k_d=0.7, flux_form=1)
    centre = (0.48, 0.41, 0)
    if axisym:
        prob["axisym"] = 1
        centre = (0.0, 0.41, 0)
    chi = O.geometry(prob, synth.vof_ball(n, h, centre, 0.21, 2), 60)
    F, P = O.init_state(prob, chi, c0=synth.uniform_field(n, 4, 0.8, 1.2), gamma0=0.4)
    dt = 20 * 0.2 * h * h / 1e-2
    Fn, Pn, _, _ = I.implicit_step(prob, chi, None, F, P, dt, picard=60)
    dtp = 1e-3
    Fe, Pe, _, _ = O.step(prob, chi, None, Fn, Pn, dtp)
    worst = 0.0
    for lhs, rhs in (((Fn - F) / dt, (Fe - Fn) / dtp), ((Pn - P) / dt, (Pe - Pn) / dtp)):
        worst = max(worst, float(np.max(np.abs(lhs - rhs)) / np.max(np.abs(lhs))))
    assert worst < 1e-9, worst
    return worst


def _rings_case(n, centre_z, R, cylinder=False):
    from paper_2605_27534_amd import synth
    nr, nz = n
    h = 1.0 / nz
    prob = dict(dim=2, n=(nr, nz), h=h, bc=((0, 2), (1, 1)), axisym=1)
    if cylinder:
        r = (np.arange(nr) + 0.5) * h
        c = np.clip((R - r) / h + 0.5, 0.0, 1.0)  # the interface r = R inside one ring
        vof = np.broadcast_to(c[None, :], (nz, nr)).copy()[None]
    else:
        vof = synth.vof_ball((nr, nz), h, (0.0, centre_z, 0), R, 2, sub=64)
    return prob, vof, O.geometry(prob, vof, 72)


def rings_capillary(K=None):
    """The interfacial forces on axisymmetric rings against the geometry of
    surfaces of revolution: a cylinder of fluid 1 about the axis has, in
    each ring layer, delta_m times the ring volumes equal to the lateral
    area 2 pi R h (the chord is the layer's height at r = R), and kappa = the
    azimuthal -1/r at the cell centre; a sphere on the axis has delta_m
    times the volumes summing to 4 pi R^2 (1%) and kappa = -2/R (2% mean)."""
    if K is None:
        from oracle import capillary as K
    nr, nz, R = 16, 12, 0.37
    prob, vof, chi = _rings_case((nr, nz), 0.0, R, cylinder=True)
    h = prob["h"]
    dm = K.marangoni_delta(prob, vof)[0]
    kap = K.curvature(prob, vof, chi)[0]
    rmid = (np.arange(nr) + 0.5) * h
    vol = 2 * math.pi * rmid * h * h
    for j in range(nz):
        assert abs(np.sum(dm[j] * vol) - 2 * math.pi * R * h) < 1e-13
    i = int(R / h)
    assert np.all(np.abs(kap[:, i] + 1.0 / rmid[i]) < 1e-12)
    nr, nz, R = 48, 96, 0.3
    prob, vof, chi = _rings_case((nr, nz), 0.5, R)
    h = prob["h"]
    dm = K.marangoni_delta(prob, vof)[0]
    rmid = (np.arange(nr) + 0.5) * h
    area = float(np.sum(dm * (2 * math.pi * rmid * h * h)[None, :]))
    assert abs(area - 4 * math.pi * R * R) < 0.01 * 4 * math.pi * R * R, area
    kap = K.curvature(prob, vof, chi)[0]
    v = vof[0]
    cut = (v > K.CUT) & (v < 1 - K.CUT)
    err = np.abs(kap[cut] * R / 2 + 1.0)
    assert err.mean() < 0.02 and np.median(err) < 0.01, (err.mean(), np.median(err))
    # without the rings the same cells give the circle's -1/R
    k2 = K.curvature(dict(prob, axisym=0), vof, chi)[0]
    assert abs(np.median(k2[cut] * R) + 1.0) < 0.02
