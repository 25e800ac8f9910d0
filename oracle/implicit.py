"""FP64 oracle of the implicit substep 2 (section 3, second substep of the
split; Appendix C), in the weighted flux form and in the paper's own form.

TEST INFRASTRUCTURE ONLY: the tests and the CPU-baseline leg of the
benchmark may import this module; the product path never does.  It shares no
code with the HIP library; it reuses the C oracle (``oracle.py``) for the
cell geometry and the explicit advection of substep 1.

The step (section 3: Lie split; Appendix C: implicit Euler for substep 2):

    xi*     = advection of xi^n over dt                         (substep 1)
    (xi^{n+1} - xi*) / dt = div(flux(xi^{n+1})) +/- q^{n+1}     (substep 2)

with the weighted-form flux through a face, D wbar (r_R - r_L) / h, where
r = xi / (w + eta_w) is the carrier quotient (c = F/(phi + eta) for the
bulk, Gamma = psi/(delta + eta/eps) for the interface), wbar the mean of w
over the face (w = phi or delta), and no diffusive flux through walls and
open sides.  In terms of r the flux divergence is -K r with K the symmetric
face-weighted graph Laplacian

    K[L,L] += k, K[R,R] += k, K[L,R] -= k, K[R,L] -= k,  k = D wbar / h^2

for every face that carries flux.  The source q = k_a c (Gamma_inf delta -
psi) - k_d psi (Langmuir; Henry drops psi in the adsorption term) couples the
two fields; Appendix C recasts each equation as a linear elliptic problem
whose reaction coefficient holds the other field at t^{n+1}.  Those two
problems are solved alternately (Picard sweeps, the interfacial one first):

    interface:  [ (delta+eta/eps)(1/dt + kl k_a c + k_d) + K_s ] Gamma
                    = psi*/dt + k_a c Gamma_inf delta
    bulk:       [ (phi+eta)/dt + k_a (Gamma_inf delta - kl psi) + K_b ] c
                    = F*/dt + k_d psi

(kl = 1 Langmuir, 0 Henry), starting from c = c*.  Each linear problem is
solved exactly (a sparse direct solve).  After `picard` sweeps:
F = (phi+eta) c, psi = (delta+eta/eps) Gamma, sigma = sigma(psi/(delta+eta/eps)).

On axisymmetric rings (Appendix B) the balance of cell i is divided by its
volume 2 pi r_i h^2, so a radial face's flux enters cell i with the weight
r_face / r_i (an axial face's with 1): face f between L and R adds
k r_f / r_L to row L and k r_f / r_R to row R, and the totals integrate over
the ring volumes.

In the paper's form (sections 2.6, 3.2, Appendix A) the unknowns are F and
psi themselves and the flux through a face is D (xi_R - xi_L)/h + Bbar xi_up:
the centred diffusion plus the anti-diffusive transport at velocity -B, B
the face mean of the cell values B_F = -D_b (1 - phi) n_d / eps (bulk) and
B_psi = -D_s (1 - 2 phi) n_d / eps (carrier), n = -grad chi / |grad chi|
from centred differences (|grad chi| bounded below by 1e-6), xi_up the cell
upwind of -Bbar (L when Bbar < 0).  Its divergence is -P xi with P a
non-symmetric matrix, and the two problems read

    interface:  [ 1/dt + kl k_a c + k_d + P_s ] psi = psi*/dt + k_a c Gamma_inf delta
    bulk:       [ 1/dt + k_a (Gamma_inf delta - kl psi)/(phi + eta) + P_b ] F
                    = F*/dt + k_d psi

with c = F/(phi + eta) at its latest value.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import oracle as O


def radii(q):
    """Axisymmetric rings: (r_i, r_{i+1/2}) of every cell as [nz][ny][nx]
    arrays (the mid radius and the radius of the high radial face)."""
    nx, ny, nz = q["n"]
    r0 = float(q.get("origin", (0.0, 0.0, 0.0))[0])
    i = np.arange(nx, dtype=np.float64)
    rmid = np.broadcast_to(r0 + (i + 0.5) * q["h"], (nz, ny, nx))
    rhi = np.broadcast_to(r0 + (i + 1.0) * q["h"], (nz, ny, nx))
    return rmid, rhi


def cell_volumes(q):
    """h^dim, or 2 pi r_i h^2 on axisymmetric rings."""
    if q["axisym"]:
        rmid, _ = radii(q)
        return 2.0 * math.pi * rmid * q["h"] ** 2
    return np.full(O.shape(q), q["h"] ** q["dim"])


def laplacian(q, w, D):
    """K (N x N, CSR) for face weights w (cell field, [nz][ny][nx]): each
    face's coefficient k enters its two cells' rows with their divergence
    weights (1, or r_face / r_i for a radial face of a ring)."""
    nx, ny, nz = q["n"]
    N = nx * ny * nz
    idx = np.arange(N).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    bc = list(q["bc"]) + [(0, 0)] * (3 - len(q["bc"]))
    rmid, rhi = radii(q) if q["axisym"] else (None, None)
    for d in range(q["dim"]):
        ax = 2 - d  # numpy axis of grid axis d
        per = bc[d][0] == O.BC_PERIODIC
        L = idx
        R = np.roll(idx, -1, axis=ax)  # right neighbour (wrapped)
        wL = w
        wR = np.roll(w, -1, axis=ax)
        k = D * 0.5 * (wL + wR) / (q["h"] ** 2)
        if q["axisym"] and d == 0:
            # the face is the high face of L and the low face of R
            kL = k * rhi / rmid
            kR = k * rhi / np.roll(rmid, -1, axis=ax)
        else:
            kL, kR = k, k
        if not per:
            # the face between the last cell and the wrapped first one is a
            # side: no flux
            sl = [slice(None)] * 3
            sl[ax] = slice(0, q["n"][d] - 1)
            L, R = L[tuple(sl)], R[tuple(sl)]
            kL, kR = kL[tuple(sl)], kR[tuple(sl)]
        L, R, kL, kR = L.ravel(), R.ravel(), kL.ravel(), kR.ravel()
        rows += [L, R, L, R]
        cols += [L, R, R, L]
        vals += [kL, kR, -kL, -kR]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def _nbr(a, d, off, per, n):
    """a shifted so that entry i holds a[i + off] along grid axis d: wrapped
    on a periodic axis, mirrored about the boundary face otherwise."""
    ax = 2 - d
    idx = np.arange(n) + off
    if per:
        idx = np.mod(idx, n)
    else:
        idx = np.where(idx < 0, -1 - idx, idx)
        idx = np.where(idx >= n, 2 * n - 1 - idx, idx)
    return np.take(a, idx, axis=ax)


def paper_B(q, chi, phi, om, bulk_field):
    """The paper-form coefficient of every cell along each axis."""
    bc = list(q["bc"]) + [(0, 0)] * (3 - len(q["bc"]))
    per = [bc[d][0] == O.BC_PERIODIC for d in range(3)]
    n = q["n"]
    g = [(_nbr(chi, e, 1, per[e], n[e]) - _nbr(chi, e, -1, per[e], n[e])) / (2.0 * q["h"])
         for e in range(q["dim"])]
    nrm = np.sqrt(sum(x * x for x in g))
    nrm = np.maximum(nrm, 1e-6)
    D = q["D_b"] if bulk_field else q["D_s"]
    w = om if bulk_field else om - phi
    return [-D * w / q["eps"] * (-g[d] / nrm) for d in range(q["dim"])]


def paper_operator(q, chi, phi, om, bulk_field):
    """P (N x N, CSR): minus the paper-form flux divergence, -(1/h) sum_d
    (flux_hi - flux_lo), as a matrix acting on xi (on rings the radial
    fluxes weighted by r_face / r_i, as in the explicit step)."""
    nx, ny, nz = q["n"]
    N = nx * ny * nz
    h = q["h"]
    D = q["D_b"] if bulk_field else q["D_s"]
    idx = np.arange(N).reshape(nz, ny, nx)
    B = paper_B(q, chi, phi, om, bulk_field)
    bc = list(q["bc"]) + [(0, 0)] * (3 - len(q["bc"]))
    rmid, rhi = radii(q) if q["axisym"] else (None, None)
    rows, cols, vals = [], [], []
    for d in range(q["dim"]):
        ax = 2 - d
        per = bc[d][0] == O.BC_PERIODIC
        L = idx
        R = np.roll(idx, -1, axis=ax)
        Bf = 0.5 * (B[d] + np.roll(B[d], -1, axis=ax))
        if q["axisym"] and d == 0:
            # rings: the face enters row L with r_face / r_L and row R with
            # r_face / r_R (it is L's high face and R's low face)
            wL = rhi / rmid
            wR = rhi / np.roll(rmid, -1, axis=ax)
        else:
            wL = wR = np.ones(O.shape(q))
        if not per:
            sl = [slice(None)] * 3
            sl[ax] = slice(0, q["n"][d] - 1)
            L, R, Bf = L[tuple(sl)], R[tuple(sl)], Bf[tuple(sl)]
            wL, wR = wL[tuple(sl)], wR[tuple(sl)]
        L, R, Bf, wL, wR = L.ravel(), R.ravel(), Bf.ravel(), wL.ravel(), wR.ravel()
        up = np.where(Bf < 0.0, L, R)
        # flux = D (xi_R - xi_L)/h + Bf xi_up through the high face of L and
        # the low face of R: minus the divergence takes -flux/h in row L and
        # +flux/h in row R
        k = D / (h * h)
        rows += [L, L, R, R, L, R]
        cols += [L, R, R, L, up, up]
        vals += [k * wL, -k * wL, k * wR, -k * wR, -Bf / h * wL, Bf / h * wR]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def implicit_step(prob, chi, u, F, psi, dt, picard=3, totals=None):
    """One step with substep 2 implicit.  Returns (F, psi, sigma, totals);
    totals follow the explicit step's layout, with the next stable dt taken
    from the advective bound only (substep 2 has none)."""
    q = O.full(prob)
    paper = q["flux_form"] == 1
    shp = O.shape(prob)
    N = int(np.prod(shp))
    phi, om, de = O.cell_geometry(prob, chi)
    bulk = bool(q["bulk_enabled"])
    if u is not None:
        Fs, outF = O.advect(prob, u, F, dt) if bulk else (np.array(F, dtype=np.float64), 0.0)
        Ps, outP = O.advect(prob, u, psi, dt)
    else:
        Fs, outF = np.array(F, dtype=np.float64), 0.0
        Ps, outP = np.array(psi, dtype=np.float64), 0.0
    dF = phi + q["eta"]
    dP = de + q["eta"] / q["eps"]
    kl = 1.0 if q["kinetics"] == 0 else 0.0
    ka, kd, ginf = (q["k_a"], q["k_d"], q["gamma_inf"]) if bulk else (0.0, 0.0, 0.0)
    c = (Fs / dF).ravel()
    G = (Ps / dP).ravel()
    dFv, dPv, dev = dF.ravel(), dP.ravel(), de.ravel()
    Fsv, Psv = Fs.ravel(), Ps.ravel()
    if paper:
        Pb = paper_operator(q, chi, phi, om, True)
        Ps_ = paper_operator(q, chi, phi, om, False)
        Fv, Pv = Fsv.copy(), Psv.copy()
        for _ in range(max(1, picard) if bulk else 1):
            cF = Fv / dFv if bulk else np.zeros_like(Fv)
            A = Ps_ + sp.diags(1.0 / dt + kl * ka * cF + kd)
            Pv = spla.spsolve(A.tocsc(), Psv / dt + ka * cF * ginf * dev)
            if not bulk:
                break
            A = Pb + sp.diags(1.0 / dt + ka * (ginf * dev - kl * Pv) / dFv)
            Fv = spla.spsolve(A.tocsc(), Fsv / dt + kd * Pv)
        Fo = Fv.reshape(shp) if bulk else np.array(F, dtype=np.float64)
        Po = Pv.reshape(shp)
    else:
        Kb = laplacian(q, phi, q["D_b"])
        Ks = laplacian(q, de, q["D_s"])
        for _ in range(max(1, picard) if bulk else 1):
            # interfacial problem with c at its latest value
            A = Ks + sp.diags(dPv * (1.0 / dt + kl * ka * c + kd))
            G = spla.spsolve(A.tocsc(), Psv / dt + ka * c * ginf * dev)
            if not bulk:
                break
            psi_new = dPv * G
            # bulk problem with the new psi
            A = Kb + sp.diags(dFv / dt + ka * (ginf * dev - kl * psi_new))
            c = spla.spsolve(A.tocsc(), Fsv / dt + kd * psi_new)
        Fo = (dFv * c).reshape(shp) if bulk else np.array(F, dtype=np.float64)
        Po = (dPv * G).reshape(shp)
    S = O.eos(prob, Po / dP)
    tot = np.zeros(16) if totals is None else np.array(totals, dtype=np.float64)
    vol = cell_volumes(q)
    mb = math.fsum((Fo * vol).ravel()) if bulk else 0.0
    ms = math.fsum((Po * vol).ravel())
    sd = math.fsum((de * vol).ravel())
    ssd = math.fsum((S * de * vol).ravel())
    su = 0.0
    if u is not None:
        s = np.zeros(shp)
        for d in range(q["dim"]):
            ud = np.asarray(u[d], dtype=np.float64)
            ax = 2 - d
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[ax] = slice(0, q["n"][d])
            hi[ax] = slice(1, q["n"][d] + 1)
            uh = ud[tuple(hi)].copy()
            if q["bc"][d][1] == O.BC_PERIODIC:
                # face n_d of a periodic axis is face 0
                last = [slice(None)] * 3
                last[ax] = slice(q["n"][d] - 1, q["n"][d])
                first = [slice(None)] * 3
                first[ax] = slice(0, 1)
                uh[tuple(last)] = ud[tuple(first)]
            ul = ud[tuple(lo)]
            if q["axisym"] and d == 0:
                # the radial mean weights each face by r_face / r_i
                rmid, rhi = radii(q)
                ul = ul * (rhi - q["h"]) / rmid
                uh = uh * rhi / rmid
            s += np.abs(0.5 * (ul + uh))
        su = float(s.max())
    out = outF + outP
    outcum = tot[O.T_OUTCUM] + out
    dta = q["cfl_adv"] * q["h"] / su if su > 0 else math.inf
    cc = Fo / dF
    tot[O.T_MB] = mb
    tot[O.T_MS] = ms
    tot[O.T_OUT] = out
    tot[O.T_OUTCUM] = outcum
    tot[O.T_SDELTA] = sd
    tot[O.T_SSIGD] = ssd
    tot[O.T_SU] = su
    tot[O.T_DTNEXT] = dta
    tot[O.T_MINF] = float(Fo.min()) if bulk else 0.0
    tot[O.T_MINPSI] = float(Po.min())
    tot[O.T_NBAD] = float(np.count_nonzero(~np.isfinite(Fo) | ~np.isfinite(Po) | ~np.isfinite(S)))
    tot[O.T_T] = tot[O.T_T] + dt
    tot[O.T_GAVG] = ms / sd
    tot[O.T_SAVG] = ssd / sd
    tot[O.T_MTOT] = mb + ms + outcum
    tot[O.T_CMAX] = float(cc.max()) if bulk else 0.0
    return Fo, Po, S, tot


def run(prob, chi, u, F, psi, dt, nsteps, vof_seq=None, hj_iters=8, picard=3):
    """nsteps implicit steps (the level set warm-started from vof_seq(n)
    before step n when given).  Returns (chi, F, psi, sigma, totals history)."""
    tot = np.zeros(16)
    hist = []
    S = None
    for n in range(nsteps):
        if vof_seq is not None:
            chi = O.geometry(prob, vof_seq(n), hj_iters, chi=chi)
        F, psi, S, tot = implicit_step(prob, chi, u, F, psi, dt, picard=picard, totals=tot)
        hist.append(tot.copy())
    return chi, F, psi, S, np.array(hist)
