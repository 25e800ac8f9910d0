"""FP64 oracle of the phase field evolved by ACDI (section 2.5, the
Phase-Field method), in place of a level set rebuilt from the VoF every step.

TEST INFRASTRUCTURE ONLY: the tests and the CPU-baseline leg of the
benchmark may import this module; the product path never does.  It shares no
code with the HIP library; it reuses the C oracle (``oracle.py``) for the
advection of substep 1, the cell geometry, the level set from the VoF and the
surfactant step.

The paper evolves phi by the Allen-Cahn-type ACDI equation

    d phi/dt + div(u phi) = div( zeta [ eps grad phi
                                        - 1/4 (1 - tanh^2(s / (2 eps))) grad s / |grad s| ] )

with the auxiliary signed-distance-like field s = eps ln((phi + ve) / (1 - phi + ve))
(the paper calls it psi; here psi is the interfacial carrier), ve = 1e-6, and
the velocity scale zeta at least the largest speed.  Readings (they are the
HIP library's readings too):

* the same Lie split as the surfactant fields: phi* = the advection of phi by
  the substep-1 scheme (BCG face values with the minmod limiter, flux form),
  then phi^{n+1} = phi* + dt div G(phi*);
* G through a face along d: zeta [ eps (phi_R - phi_L)/h - 1/4 (1 - T^2) n_d ],
  T = tanh(s_f / (2 eps)) with s_f the mean of s over the two cells, and n the
  unit vector of the face gradient of s: normal component (s_R - s_L)/h, each
  transverse component the mean of the two cells' centred differences (ghost
  cells mirror at walls and open sides, wrap on periodic axes),
  n = g / max(|g|, 1/2).  Continuously phi (1 - phi) grad s = eps grad phi, so
  the flux is zeta eps grad phi (1 - 1/|grad s|): diffusion where the profile
  is too thin, anti-diffusion where it is too wide, nothing at the equilibrium
  |grad s| = 1.  Where s flattens (the tails, and the plateau the level-set
  clamp leaves), a unit normal would make that anti-diffusion unbounded and
  turn rounding into exponentially growing noise; the bound 1/2 caps it at
  zeta eps |grad phi|, the size of the diffusion, and leaves every profile up
  to twice the equilibrium width unchanged;
* no regularization flux through walls and open sides;
* s is evaluated on phi clamped into [0, 1] (so that it stays finite when
  rounding leaves phi a little outside);
* phi from a level set: phi = (1 - tanh(chi / (2 eps)))/2 = 1/(1 + e^{chi/eps}),
  the cell-geometry phi of the surfactant path;
* the level set the surfactant transport sees: chi = -s(phi), clamped to
  |chi| <= chi_max (the transport's own phi of it is then (phi + ve)/(1 + 2 ve));
* re-initialization from a VoF field: the warm-started level set (hj sweeps
  from the current chi), then phi from it;
* on axisymmetric rings (Appendix B) the fluxes are the same expressions in
  (r, z) (the azimuthal component vanishes by symmetry), and the balance of
  ring i, divided by its volume 2 pi r_i h^2, takes a radial face's flux
  with the weight r_face / r_i, as the surfactant fields do.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O

VAREPS = 1e-6


def s_of_phi(prob, phi, vareps=VAREPS):
    """The auxiliary field s = eps ln((phi + ve)/(1 - phi + ve)), phi clamped
    into [0, 1]."""
    q = O.full(prob)
    p = np.clip(np.asarray(phi, dtype=np.float64), 0.0, 1.0)
    return q["eps"] * np.log((p + vareps) / (1.0 - p + vareps))


def chi_of_phi(prob, phi, vareps=VAREPS):
    q = O.full(prob)
    cm = q["chi_max_eps"] * q["eps"]
    return np.clip(-s_of_phi(prob, phi, vareps), -cm, cm)


def phi_of_chi(prob, chi):
    phi, _, _ = O.cell_geometry(prob, chi)
    return phi


def _axes(q):
    bc = list(q["bc"]) + [(0, 0)] * (3 - len(q["bc"]))
    return [bc[d][0] == O.BC_PERIODIC for d in range(3)]


def _nb(a, d, off, per, n):
    """a shifted so that entry i holds a[i + off] along grid axis d: wrapped
    on a periodic axis, mirrored (ghost = the cell itself, then its
    neighbours) otherwise."""
    ax = 2 - d
    idx = np.arange(n) + off
    if per:
        idx = np.mod(idx, n)
    else:
        idx = np.where(idx < 0, -1 - idx, idx)
        idx = np.where(idx >= n, 2 * n - 1 - idx, idx)
        idx = np.clip(idx, 0, n - 1)
    return np.take(a, idx, axis=ax)


def regularization_fluxes(prob, phi, zeta, vareps=VAREPS):
    """G on the high face of every cell along each axis (entry i: the face
    between cells i and i+1, wrapped on periodic axes); zero where the face
    is a wall or an open side."""
    q = O.full(prob)
    h, eps = q["h"], q["eps"]
    per = _axes(q)
    n = q["n"]
    s = s_of_phi(prob, phi, vareps)
    # centred differences of s in every cell, per axis
    cd = [(_nb(s, t, 1, per[t], n[t]) - _nb(s, t, -1, per[t], n[t])) / (2.0 * h)
          for t in range(q["dim"])]
    G = []
    for d in range(q["dim"]):
        sR = _nb(s, d, 1, per[d], n[d])
        phR = _nb(phi, d, 1, per[d], n[d])
        gn = (sR - s) / h
        g2 = gn * gn
        for t in range(q["dim"]):
            if t == d:
                continue
            gt = 0.5 * (cd[t] + _nb(cd[t], d, 1, per[d], n[d]))
            g2 = g2 + gt * gt
        nd = gn / np.maximum(np.sqrt(g2), 0.5)
        T = np.tanh(0.5 * (s + sR) / (2.0 * eps))
        Gd = zeta * (eps * (phR - phi) / h - 0.25 * (1.0 - T * T) * nd)
        if not per[d]:
            sl = [slice(None)] * 3
            sl[2 - d] = slice(n[d] - 1, n[d])
            Gd[tuple(sl)] = 0.0  # the high side of the box
        G.append(Gd)
    return G


def regularize(prob, phi, dt, zeta, vareps=VAREPS):
    """phi + dt div G(phi)."""
    q = O.full(prob)
    per = _axes(q)
    n = q["n"]
    G = regularization_fluxes(prob, phi, zeta, vareps)
    div = np.zeros_like(phi, dtype=np.float64)
    for d in range(q["dim"]):
        Glo = _nb(G[d], d, -1, per[d], n[d])
        if not per[d]:
            sl = [slice(None)] * 3
            sl[2 - d] = slice(0, 1)
            Glo[tuple(sl)] = 0.0  # the low side of the box
        if q["axisym"] and d == 0:
            # ring i between r_lo = r0 + i h and r_hi = r_lo + h, mid radius r_i
            r0 = float(q.get("origin", (0.0, 0.0, 0.0))[0])
            r_lo = r0 + np.arange(n[0], dtype=np.float64) * q["h"]
            r_mid = r_lo + 0.5 * q["h"]
            div = div + (G[d] * ((r_lo + q["h"]) / r_mid) - Glo * (r_lo / r_mid))
        else:
            div = div + (G[d] - Glo)
    return phi + dt * div / q["h"]


def acdi_step(prob, phi, u, dt, zeta, vareps=VAREPS):
    """One ACDI step: advection (when u is given), then regularization."""
    ps = np.array(phi, dtype=np.float64) if u is None else O.advect(prob, u, phi, dt)[0]
    return regularize(prob, ps, dt, zeta, vareps)


def run(prob, chi, u, F, psi, dt, nsteps, zeta, vof_seq=None, hj_iters=8, totals=None,
        implicit=False, picard=3):
    """nsteps surfactant steps on an ACDI interface.  vof_seq(n) -> a VoF
    field to re-initialize from before step n, or None to advance phi by
    ACDI.  Returns (chi, phi, F, psi, sigma, totals history)."""
    from . import implicit as I
    tot = np.zeros(16) if totals is None else totals
    # the regularization step is explicit: a diffusion of coefficient
    # zeta eps and a transport at speed up to zeta, whose explicit bound
    # (2 dim zeta eps/h^2 + zeta sqrt(dim)/h) joins the next stable step
    q = O.full(prob)
    lam = zeta * (2.0 * q["dim"] * q["eps"] / q["h"] ** 2 + math.sqrt(q["dim"]) / q["h"])
    phi = phi_of_chi(prob, chi)
    hist = []
    S = None
    for k in range(nsteps):
        v = vof_seq(k) if vof_seq is not None else None
        if v is not None:
            chi = O.geometry(prob, v, hj_iters, chi=chi)
            phi = phi_of_chi(prob, chi)
        else:
            phi = acdi_step(prob, phi, u, dt, zeta)
            chi = chi_of_phi(prob, phi)
        if implicit:
            F, psi, S, tot = I.implicit_step(prob, chi, u, F, psi, dt, picard=picard, totals=tot)
        else:
            F, psi, S, tot = O.step(prob, chi, u, F, psi, dt, tot)
        tot[O.T_DTNEXT] = min(tot[O.T_DTNEXT], q["cfl_diff"] / lam)
        hist.append(tot.copy())
    return chi, phi, F, psi, S, np.array(hist)


def ring_volumes(prob):
    """The cell volumes: h^dim, or 2 pi r_i h^2 on axisymmetric rings."""
    q = O.full(prob)
    if not q["axisym"]:
        return np.full(O.shape(prob), q["h"] ** q["dim"])
    r0 = float(q.get("origin", (0.0, 0.0, 0.0))[0])
    r = r0 + (np.arange(q["n"][0], dtype=np.float64) + 0.5) * q["h"]
    return np.broadcast_to(2.0 * math.pi * r * q["h"] ** 2, O.shape(prob)).copy()


def profile_thickness(prob, phi):
    """sum phi (1 - phi) / eps h^dim over the box: the interface measure the
    equilibrium profile gives (1 per unit area of a flat interface)."""
    q = O.full(prob)
    return float(math.fsum((phi * (1.0 - phi) / q["eps"]).ravel()) * q["h"] ** q["dim"])
