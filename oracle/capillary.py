"""FP64 oracle of the interfacial forces of the flow coupling (section 2.4):
the capillary force sigma kappa delta_s n and the Marangoni force
delta_m grad_s sigma with the PLIC interface area per cell volume, in 2D.

TEST INFRASTRUCTURE ONLY: the tests may import this module; the product path
never does.  It shares no code with the HIP library.

Notation: c the VoF fraction of fluid 1, chi the signed distance (> 0 in
fluid 1), phi the phase field (0 in fluid 1), n = grad phi / |grad phi| the
unit normal, pointing out of fluid 1.  Readings (the HIP library takes the same):

* kappa = -div n by height functions (Cummins, Francois and Kothe, Comput.
  Struct. 83, 2005) in each cell with 0 < c < 1: along the axis of the
  larger component of the Youngs normal (below), the fluid-1 heights
  H_k = sum_{l=-3..3} c in the three columns k = -1, 0, 1 through the cell
  and its neighbours, H' = (H_1 - H_-1)/2, H'' = (H_1 - 2 H_0 + H_-1)/h,
  kappa = H'' / (1 + H'^2)^(3/2) (negative for a convex blob of fluid 1),
  in each interfacial cell.
  A column whose end cells are not full on the fluid-1 side and empty on the
  other (to 1e-6) makes the stencil inconsistent; such a cell takes the
  level-set curvature instead: div(grad chi / |grad chi|) by central
  differences, moved to the interface with kappa / (1 - chi kappa), |grad
  chi| bounded below by 1e-6.  On a face, kappa is the mean over its
  interfacial cells (0 if neither is);
* delta_s n = |grad c| n = -grad c (c decreases along n), so the capillary
  force is -sigma kappa grad c, evaluated on the faces of the velocity grid:
  -sigma_f kappa_f (c_R - c_L)/h, sigma_f and kappa_f the means over the two
  cells (the balanced-force placement of the VoF gradient);
* a cell is interfacial when 1e-6 < c < 1 - 1e-6 (fractions within 1e-6 of 0
  or 1 count as empty or full);
* delta_m = A_f / V_c from a PLIC reconstruction in each interfacial cell: the Youngs normal m = -grad c from the 3x3 stencil (weights
  1, 2, 1 across the difference direction), the line m.x = alpha placed so
  that the part of the cell on the side m.x <= alpha has area c h^2, A_f the
  length of the line inside the cell; other cells, and cells with m = 0,
  have none; on a face, the mean of the two cells;
* grad_s sigma on a face: the face gradient of sigma (compact normal
  difference, the two cells' centred transverse differences averaged) minus
  its normal part, n from the same face gradient of chi bounded below by
  1e-6 (the rule of the regularized Marangoni force);
* faces on walls and open sides carry no force.

On axisymmetric rings (Appendix B; x the radius r, y the axis z, ring i at
r_i = r0 + (i + 1/2) h) the interface is a surface of revolution, so:

* kappa adds the azimuthal principal curvature to the meridional one: with
  n = m / |m| (the Youngs normal, out of fluid 1), kappa = kappa_2D - n_r/r_i
  (-2/R on a sphere of fluid 1, -1/R on a cylinder of radius R about the
  axis); the level-set fallback adds (d chi / dr) / (|grad chi| r_i) to the
  2D divergence and moves the sum to the interface with kappa / (1 - chi
  kappa / 2) (exact on a sphere);
* delta_m = A_f / V_c with A_f the area the PLIC chord sweeps about the axis,
  2 pi r_m |chord| (r_m the radius of the chord's midpoint), and V_c = 2 pi
  r_i h^2: delta_m = (|chord| / h^2) r_m / r_i.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O


def _axes(q):
    bc = list(q["bc"]) + [(0, 0)] * (3 - len(q["bc"]))
    return [bc[d][0] == O.BC_PERIODIC for d in range(3)]


def _at(a, j, i, q, per):
    """a[j, i] of a 2D cell field with mirror / wrap ghosts."""
    nx, ny = q["n"][0], q["n"][1]

    def m(v, n, p):
        if p:
            return v % n
        if v < 0:
            v = -1 - v
        if v >= n:
            v = 2 * n - 1 - v
        return min(max(v, 0), n - 1)
    return a[m(j, ny, per[1]), m(i, nx, per[0])]


def ring_radius(q, i):
    """r_i of ring column i (axisymmetric)."""
    return float(q.get("origin", (0.0, 0.0, 0.0))[0]) + (i + 0.5) * q["h"]


def levelset_curvature(prob, chi, j, i):
    q = O.full(prob)
    per = _axes(q)
    h = q["h"]
    ch = np.asarray(chi, dtype=np.float64)[0]
    c = lambda dj, di: _at(ch, j + dj, i + di, q, per)
    cx = (c(0, 1) - c(0, -1)) / (2 * h)
    cy = (c(1, 0) - c(-1, 0)) / (2 * h)
    cxx = (c(0, 1) - 2 * c(0, 0) + c(0, -1)) / (h * h)
    cyy = (c(1, 0) - 2 * c(0, 0) + c(-1, 0)) / (h * h)
    cxy = (c(1, 1) - c(1, -1) - c(-1, 1) + c(-1, -1)) / (4 * h * h)
    g = max(math.sqrt(cx * cx + cy * cy), 1e-6)
    kc = (cxx * cy * cy - 2 * cx * cy * cxy + cyy * cx * cx) / g ** 3
    if q["axisym"]:
        # div(grad chi / |grad chi|) in (r, z) adds (d chi / dr) / (|grad chi| r)
        kc += cx / (g * ring_radius(q, i))
        return kc / (1.0 - c(0, 0) * kc / 2.0)
    return kc / (1.0 - c(0, 0) * kc)


def cell_curvature(prob, vof, chi, j, i):
    """kappa of cell (j, i) (assumed interfacial), 2D."""
    q = O.full(prob)
    per = _axes(q)
    h = q["h"]
    v = np.asarray(vof, dtype=np.float64)[0]
    mx, my = youngs_normal(v, j, i, q, per)
    vert = abs(my) >= abs(mx)  # columns along y
    out = my if vert else mx   # the normal's component along the columns
    H = []
    ok = True
    for kk in (-1, 0, 1):
        col = []
        for l in range(-3, 4):
            col.append(_at(v, j + l, i + kk, q, per) if vert else
                       _at(v, j + kk, i + l, q, per))
        # fluid 1 lies against the normal: at the low end when the normal
        # points to +, at the high end otherwise
        full, empty = (col[0], col[-1]) if out > 0 else (col[-1], col[0])
        if not (full >= 1.0 - CUT and empty <= CUT):
            ok = False
        H.append(sum(col))
    if ok:
        d1 = 0.5 * (H[2] - H[0])
        d2 = (H[2] - 2.0 * H[1] + H[0]) / h
        kap = d2 / (1.0 + d1 * d1) ** 1.5
        if q["axisym"] and (mx != 0.0 or my != 0.0):
            # the azimuthal curvature -n_r / r_i, n the unit Youngs normal
            kap -= mx / math.hypot(mx, my) / ring_radius(q, i)
        return kap
    return levelset_curvature(prob, chi, j, i)


def curvature(prob, vof, chi):
    """kappa in every cell with 0 < c < 1 (0 elsewhere), 2D."""
    v = np.asarray(vof, dtype=np.float64)[0]
    ny, nx = v.shape
    k = np.zeros_like(v)
    for j in range(ny):
        for i in range(nx):
            if interfacial(v[j, i]):
                k[j, i] = cell_curvature(prob, vof, chi, j, i)
    return k[None]


# ---- PLIC in the unit square, by clipping and bisection

def _clip(poly, m, alpha):
    """The part of a convex polygon (list of (x, y)) where m.x <= alpha, and
    the points where its boundary crosses the line (Sutherland-Hodgman with
    one half-plane)."""
    out, cuts = [], []
    for a, b in zip(poly, poly[1:] + poly[:1]):
        fa = m[0] * a[0] + m[1] * a[1] - alpha
        fb = m[0] * b[0] + m[1] * b[1] - alpha
        if fa <= 0:
            out.append(a)
        if (fa < 0 < fb) or (fb < 0 < fa):
            t = fa / (fa - fb)
            p = (a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1]))
            out.append(p)
            cuts.append(p)
    return out, cuts


def _area(poly):
    s = 0.0
    for a, b in zip(poly, poly[1:] + poly[:1]):
        s += a[0] * b[1] - b[0] * a[1]
    return 0.5 * abs(s)


SQUARE = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]
CUT = 1e-6  # interfacial cells: CUT < c < 1 - CUT


def interfacial(c):
    return CUT < c < 1.0 - CUT


def plic_alpha(m, c):
    """alpha with area{x in the unit square : m.x <= alpha} = c."""
    lo = min(m[0] * x + m[1] * y for x, y in SQUARE)
    hi = max(m[0] * x + m[1] * y for x, y in SQUARE)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        a = _area(_clip(SQUARE, m, mid)[0])
        if a < c:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def plic_segment(m, c):
    """The end points of the PLIC line inside the unit square (None when the
    cell is full, empty or m = 0)."""
    if not interfacial(c) or (m[0] == 0.0 and m[1] == 0.0):
        return None
    alpha = plic_alpha(m, c)
    _, cuts = _clip(SQUARE, m, alpha)
    if len(cuts) < 2:
        # the line runs along an edge or through a corner: its points on the
        # square are the polygon's vertices lying on it
        pts = [p for p in SQUARE if abs(m[0] * p[0] + m[1] * p[1] - alpha) < 1e-14]
        cuts = cuts + pts
        if len(cuts) < 2:
            return None
    return cuts[0], cuts[1]


def plic_chord(m, c):
    """Length of the PLIC line inside the unit square (0 when the cell is
    full, empty or m = 0)."""
    seg = plic_segment(m, c)
    if seg is None:
        return 0.0
    (x0, y0), (x1, y1) = seg
    return math.hypot(x1 - x0, y1 - y0)


def youngs_normal(vof, j, i, q, per):
    f = lambda dj, di: _at(vof, j + dj, i + di, q, per)
    mx = -((f(1, 1) + 2 * f(0, 1) + f(-1, 1)) - (f(1, -1) + 2 * f(0, -1) + f(-1, -1)))
    my = -((f(1, 1) + 2 * f(1, 0) + f(1, -1)) - (f(-1, 1) + 2 * f(-1, 0) + f(-1, -1)))
    return mx, my


def cell_delta(prob, vof, j, i):
    """delta_m = A_f / V_c of cell (j, i), 2D (0 unless interfacial)."""
    q = O.full(prob)
    per = _axes(q)
    v = np.asarray(vof, dtype=np.float64)[0]
    c = v[j, i]
    if not interfacial(c):
        return 0.0
    m = youngs_normal(v, j, i, q, per)
    if q["axisym"]:
        seg = plic_segment(m, c)
        if seg is None:
            return 0.0
        (x0, y0), (x1, y1) = seg
        rm = float(q.get("origin", (0.0, 0.0, 0.0))[0]) + (i + 0.5 * (x0 + x1)) * q["h"]
        return math.hypot(x1 - x0, y1 - y0) / q["h"] * rm / ring_radius(q, i)
    return plic_chord(m, c) / q["h"]


def marangoni_delta(prob, vof):
    """delta_m = A_f / V_c per cell (2D)."""
    v = np.asarray(vof, dtype=np.float64)[0]
    ny, nx = v.shape
    out = np.zeros_like(v)
    for j in range(ny):
        for i in range(nx):
            if interfacial(v[j, i]):
                out[j, i] = cell_delta(prob, vof, j, i)
    return out[None]


def face_force(prob, vof, chi, sigma, d, j, i, kap=None, dm=None):
    """(capillary, Marangoni) on face (j, i) of the faces along d (layouts
    [ny][nx+1] and [ny+1][nx]).  kap and dm: the per-cell curvature and
    delta_m fields when already computed, else the two cells' values are
    computed here."""
    q = O.full(prob)
    per = _axes(q)
    h = q["h"]
    nx, ny = q["n"][0], q["n"][1]
    v = np.asarray(vof, dtype=np.float64)[0]
    ch = np.asarray(chi, dtype=np.float64)[0]
    sg = np.asarray(sigma, dtype=np.float64)[0]
    f = (i, j)[d]
    nd = (nx, ny)[d]
    if (f == 0 or f == nd) and not per[d]:
        return 0.0, 0.0
    # cells L and R of the face (the last face of a periodic axis is the first)
    if d == 0:
        iR, jR = i % nx, j
        iL, jL = (i - 1) % nx, j
    else:
        iR, jR = i, j % ny
        iL, jL = i, (j - 1) % ny
    cutL = interfacial(v[jL, iL])
    cutR = interfacial(v[jR, iR])
    kapc = (lambda jj, ii: kap[0][jj, ii]) if kap is not None else \
        (lambda jj, ii: cell_curvature(prob, vof, chi, jj, ii))
    dmc = (lambda jj, ii: dm[0][jj, ii]) if dm is not None else \
        (lambda jj, ii: cell_delta(prob, vof, jj, ii))
    sf = 0.5 * (sg[jL, iL] + sg[jR, iR])
    if cutL and cutR:
        kf = 0.5 * (kapc(jL, iL) + kapc(jR, iR))
    else:
        kf = kapc(jL, iL) if cutL else (kapc(jR, iR) if cutR else 0.0)
    cap = -sf * kf * (v[jR, iR] - v[jL, iL]) / h

    def face_grad(a):
        g = [0.0, 0.0]
        g[d] = (a[jR, iR] - a[jL, iL]) / h
        t = 1 - d
        dl = [0, 0]
        dl[t] = 1
        for (jj, ii) in ((jL, iL), (jR, iR)):
            g[t] += 0.5 * (_at(a, jj + dl[1], ii + dl[0], q, per) -
                           _at(a, jj - dl[1], ii - dl[0], q, per)) / (2 * h)
        return g
    gs = face_grad(sg)
    gc = face_grad(ch)
    nrm = max(math.hypot(gc[0], gc[1]), 1e-6)
    n = (gc[0] / nrm, gc[1] / nrm)
    ndot = n[0] * gs[0] + n[1] * gs[1]
    dL = dmc(jL, iL) if cutL else 0.0
    dR = dmc(jR, iR) if cutR else 0.0
    dmf = 0.5 * (dL + dR)
    return cap, dmf * (gs[d] - n[d] * ndot)


def forces(prob, vof, chi, sigma):
    """(capillary [fx, fy], Marangoni [fx, fy]) on the faces (2D, face
    layouts [ny][nx+1] and [ny+1][nx])."""
    q = O.full(prob)
    nx, ny = q["n"][0], q["n"][1]
    kap = curvature(prob, vof, chi)
    dm = marangoni_delta(prob, vof)
    cap = [np.zeros((1, ny, nx + 1)), np.zeros((1, ny + 1, nx))]
    ma = [np.zeros((1, ny, nx + 1)), np.zeros((1, ny + 1, nx))]
    for d in range(2):
        m = [nx, ny]
        m[d] += 1
        for j in range(m[1]):
            for i in range(m[0]):
                cap[d][0, j, i], ma[d][0, j, i] = face_force(prob, vof, chi, sigma, d, j, i,
                                                             kap, dm)
    return cap, ma
