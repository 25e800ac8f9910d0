"""FP64 oracle of the interfacial forces of the flow coupling (section 2.4)
in 3D: the capillary force sigma kappa delta_s n and the Marangoni force
delta_m grad_s sigma with the PLIC interface area per cell volume.

TEST INFRASTRUCTURE ONLY: the tests may import this module; the product path
never does.  It shares no code with the HIP library.

The readings are those of the 2D oracle (capillary.py), carried to 3D:

* a cell is interfacial when 1e-6 < c < 1 - 1e-6;
* the Youngs normal m = -grad c from the 3x3x3 stencil: along each axis the
  difference of the two neighbouring planes, each summed over its 3x3 cells
  with the weights (1, 2, 1) x (1, 2, 1);
* kappa by height functions (Cummins, Francois and Kothe 2005): along an
  axis a, the fluid-1 heights H(p, q) = sum_{l=-4..4} c of the nine columns
  through the cell and its neighbours (p, q) in the other two axes b < c;
  H_b, H_c the centred first differences, H_bb, H_cc the second differences
  over h, H_bc the mixed one over 4h, and
  kappa = (H_bb (1 + H_c^2) + H_cc (1 + H_b^2) - 2 H_bc H_b H_c)
          / (1 + H_b^2 + H_c^2)^(3/2)
  (twice the mean curvature, negative for a convex blob of fluid 1, the 2D
  expression when nothing varies along c).  The columns are nine cells
  long (seven in 2D): in 3D the interface can rise by a cell along each of
  two transverse axes.  The axes are tried in the order of m's components,
  largest first (ties to the higher axis), skipping zero ones, and the first
  whose nine columns all close (end cells full on the fluid-1 side and
  empty on the other, to 1e-6) gives kappa.  A cell where none closes takes
  the mean of the height curvatures of the interfacial cells of its 3x3x3
  block that have one, and where there is none, the level set's curvature
  div(grad chi / |grad chi|) by central differences (|grad chi| bounded
  below by 1e-6), moved to the interface with kappa / (1 - chi kappa / 2)
  (exact on a sphere, whose principal curvatures are kappa / 2 each).  The
  level set's second differences carry its O(h^2) error as an O(1) error
  in kappa, so it is the last resort;
* delta_m = A_f / V_c: the plane m.x = alpha that leaves the volume fraction
  c of the unit cube on its side m.x <= alpha, and A_f the area of the plane
  inside the cube, divided by h.  The volume of {x in the unit cube : m.x <=
  alpha} is written out exactly: with the components made positive by
  reflecting the axes (x_i -> 1 - x_i where m_i < 0) and the zero ones
  dropped (the volume does not depend on them), d components left,
  V = sum over subsets S of the d axes of (-1)^|S| (alpha - sum_S m)_+^d
      / (d! prod m),
  the corner simplex less the parts beyond the faces x_i = 1 (inclusion and
  exclusion); it is evaluated in exact rational arithmetic, alpha is found
  by bisection on V = c, and A_f = |m| dV/dalpha;
* on a face: the capillary force -sigma_f kappa_f (c_R - c_L)/h with
  sigma_f the mean of the two cells and kappa_f the mean over the
  interfacial ones; the Marangoni force delta_m,f (grad sigma - n (n . grad
  sigma))_d with delta_m,f the mean of the two cells, grad the face
  gradient (compact normal difference, each transverse component the mean
  of the two cells' centred differences) and n the same face gradient of
  chi over max(|.|, 1e-6); faces on walls and open sides carry no force, on
  a periodic axis the last face repeats the first.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np

from . import oracle as O

CUT = 1e-6
HL = 4  # height columns reach HL cells on each side of the cell


def interfacial(c):
    return CUT < c < 1.0 - CUT


def _axes(q):
    bc = list(q["bc"]) + [(0, 0)] * (3 - len(q["bc"]))
    return [bc[d][0] == O.BC_PERIODIC for d in range(3)]


def _map(v, n, per):
    if per:
        return v % n
    if v < 0:
        v = -1 - v
    if v >= n:
        v = 2 * n - 1 - v
    return min(max(v, 0), n - 1)


def _at(a, x, q, per):
    """a at cell x = (i, j, k) with mirror / wrap ghosts (a is [nz][ny][nx])."""
    n = q["n"]
    return a[_map(x[2], n[2], per[2]), _map(x[1], n[1], per[1]), _map(x[0], n[0], per[0])]


def _off(x, d, s):
    y = list(x)
    y[d] += s
    return y


# ---- the Youngs normal
def youngs(v, x, q, per):
    w = (1.0, 2.0, 1.0)
    m = [0.0, 0.0, 0.0]
    for d in range(3):
        b, c = [e for e in range(3) if e != d]
        s = 0.0
        for p in (-1, 0, 1):
            for r in (-1, 0, 1):
                y = list(x)
                y[b] += p
                y[c] += r
                s += w[p + 1] * w[r + 1] * (_at(v, _off(y, d, 1), q, per) -
                                             _at(v, _off(y, d, -1), q, per))
        m[d] = -s
    return m


# ---- PLIC in the unit cube, exactly
def _fr(x):
    return Fraction(x)  # exact: every float is a dyadic rational


def plic_volume(m, alpha):
    """The exact volume (a Fraction) of {x in [0,1]^3 : m.x <= alpha}."""
    a = _fr(alpha)
    mp = []
    for mi in m:
        f = _fr(mi)
        if f < 0:
            a -= f  # reflect the axis: m_i x_i = m_i - |m_i| x_i'
            f = -f
        if f != 0:
            mp.append(f)
    d = len(mp)
    if d == 0:
        return Fraction(1) if a >= 0 else Fraction(0)
    num = Fraction(0)
    for k in range(d + 1):
        for S in itertools.combinations(range(d), k):
            t = a - sum((mp[i] for i in S), Fraction(0))
            if t > 0:
                num += (-1) ** k * t ** d
    den = Fraction(math.factorial(d))
    for f in mp:
        den *= f
    return num / den


def plic_dvolume(m, alpha):
    """dV/dalpha of plic_volume, exactly."""
    a = _fr(alpha)
    mp = []
    for mi in m:
        f = _fr(mi)
        if f < 0:
            a -= f
            f = -f
        if f != 0:
            mp.append(f)
    d = len(mp)
    if d == 0:
        return Fraction(0)
    num = Fraction(0)
    for k in range(d + 1):
        for S in itertools.combinations(range(d), k):
            t = a - sum((mp[i] for i in S), Fraction(0))
            if t > 0:
                num += (-1) ** k * t ** (d - 1)
    den = Fraction(math.factorial(d - 1))
    for f in mp:
        den *= f
    return num / den


def plic_alpha(m, c):
    """alpha with volume{x : m.x <= alpha} = c, by bisection."""
    corners = [m[0] * x + m[1] * y + m[2] * z
               for x in (0.0, 1.0) for y in (0.0, 1.0) for z in (0.0, 1.0)]
    lo, hi = min(corners), max(corners)
    cf = _fr(c)
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if plic_volume(m, mid) < cf:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def plic_area(m, c):
    """Area of the PLIC plane inside the unit cube (0 when the cell is not
    interfacial or m = 0)."""
    if not interfacial(c) or (m[0] == 0.0 and m[1] == 0.0 and m[2] == 0.0):
        return 0.0
    alpha = plic_alpha(m, c)
    return math.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2) * float(plic_dvolume(m, alpha))


def cell_delta(prob, vof, x):
    q = O.full(prob)
    per = _axes(q)
    v = np.asarray(vof, dtype=np.float64)
    c = _at(v, x, q, per)
    if not interfacial(c):
        return 0.0
    return plic_area(youngs(v, x, q, per), c) / q["h"]


# ---- curvature
def levelset_curvature(prob, chi, x):
    q = O.full(prob)
    per = _axes(q)
    h = q["h"]
    ch = np.asarray(chi, dtype=np.float64)

    def c(*o):
        return _at(ch, [x[0] + o[0], x[1] + o[1], x[2] + o[2]], q, per)
    e = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    g = [(c(*e[d]) - c(*[-v for v in e[d]])) / (2 * h) for d in range(3)]
    c0 = c(0, 0, 0)
    H = [[0.0] * 3 for _ in range(3)]
    for d in range(3):
        H[d][d] = (c(*e[d]) - 2 * c0 + c(*[-v for v in e[d]])) / (h * h)
    for a in range(3):
        for b in range(a + 1, 3):
            pp = [e[a][i] + e[b][i] for i in range(3)]
            pm = [e[a][i] - e[b][i] for i in range(3)]
            H[a][b] = H[b][a] = (c(*pp) - c(*pm) - c(*[-v for v in pm]) +
                                 c(*[-v for v in pp])) / (4 * h * h)
    gm = max(math.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2), 1e-6)
    num = (H[0][0] * (g[1] ** 2 + g[2] ** 2) + H[1][1] * (g[0] ** 2 + g[2] ** 2) +
           H[2][2] * (g[0] ** 2 + g[1] ** 2) -
           2 * (g[0] * g[1] * H[0][1] + g[0] * g[2] * H[0][2] + g[1] * g[2] * H[1][2]))
    kc = num / gm ** 3
    return kc / (1.0 - c0 * kc / 2.0)


def height_curvature(prob, vof, x):
    """kappa of interfacial cell x = (i, j, k) by height functions, or None
    when no axis gives nine closed columns."""
    q = O.full(prob)
    per = _axes(q)
    h = q["h"]
    v = np.asarray(vof, dtype=np.float64)
    m = youngs(v, x, q, per)
    for a in sorted(range(3), key=lambda d: (abs(m[d]), d), reverse=True):
        if m[a] == 0.0:
            continue
        b, cc = [e for e in range(3) if e != a]
        ok = True
        H = {}
        for p in (-1, 0, 1):
            for r in (-1, 0, 1):
                col = []
                for l in range(-HL, HL + 1):
                    y = list(x)
                    y[a] += l
                    y[b] += p
                    y[cc] += r
                    col.append(_at(v, y, q, per))
                full, empty = (col[0], col[-1]) if m[a] > 0 else (col[-1], col[0])
                if not (full >= 1.0 - CUT and empty <= CUT):
                    ok = False
                H[p, r] = sum(col)
        if not ok:
            continue
        Hb = 0.5 * (H[1, 0] - H[-1, 0])
        Hc = 0.5 * (H[0, 1] - H[0, -1])
        Hbb = (H[1, 0] - 2 * H[0, 0] + H[-1, 0]) / h
        Hcc = (H[0, 1] - 2 * H[0, 0] + H[0, -1]) / h
        Hbc = (H[1, 1] - H[1, -1] - H[-1, 1] + H[-1, -1]) / (4 * h)
        return ((Hbb * (1 + Hc * Hc) + Hcc * (1 + Hb * Hb) - 2 * Hbc * Hb * Hc) /
                (1 + Hb * Hb + Hc * Hc) ** 1.5)
    return None


def cell_fields(prob, vof, chi):
    """(kappa, delta_m) of every cell: 0 away from the interfacial ones."""
    q = O.full(prob)
    per = _axes(q)
    v = np.asarray(vof, dtype=np.float64)
    nz, ny, nx = v.shape
    kh = np.full_like(v, np.nan)  # height curvature where it closes
    dm = np.zeros_like(v)
    cut = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if interfacial(v[k, j, i]):
                    cut.append((i, j, k))
                    kk = height_curvature(prob, vof, (i, j, k))
                    if kk is not None:
                        kh[k, j, i] = kk
                    dm[k, j, i] = cell_delta(prob, vof, (i, j, k))
    kap = np.zeros_like(v)
    for (i, j, k) in cut:
        if np.isfinite(kh[k, j, i]):
            kap[k, j, i] = kh[k, j, i]
            continue
        # the mean over the block's interfacial cells with a height curvature,
        # in the order dz, dy, dx = -1, 0, 1
        s, cnt = 0.0, 0
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dx == 0 and dy == 0 and dz == 0:
                        continue
                    y = (i + dx, j + dy, k + dz)
                    if not interfacial(_at(v, y, q, per)):
                        continue
                    val = _at(kh, y, q, per)
                    if np.isfinite(val):
                        s += val
                        cnt += 1
        kap[k, j, i] = s / cnt if cnt else levelset_curvature(prob, chi, (i, j, k))
    return kap, dm


def forces(prob, vof, chi, sigma):
    """(capillary [fx, fy, fz], Marangoni [fx, fy, fz]) on the faces."""
    q = O.full(prob)
    per = _axes(q)
    h = q["h"]
    n = q["n"]
    v = np.asarray(vof, dtype=np.float64)
    ch = np.asarray(chi, dtype=np.float64)
    sg = np.asarray(sigma, dtype=np.float64)
    kap, dm = cell_fields(prob, vof, chi)
    cap, ma = [], []
    for d in range(3):
        shp = [n[2], n[1], n[0]]
        shp[2 - d] += 1
        fc = np.zeros(shp)
        fm = np.zeros(shp)
        for k in range(shp[0]):
            for j in range(shp[1]):
                for i in range(shp[2]):
                    f = (i, j, k)[d]
                    if (f == 0 or f == n[d]) and not per[d]:
                        continue
                    R = [i, j, k]
                    R[d] = f % n[d]
                    L = list(R)
                    L[d] = (f - 1) % n[d]
                    kR, jR, iR = R[2], R[1], R[0]
                    kL, jL, iL = L[2], L[1], L[0]
                    cutL = interfacial(v[kL, jL, iL])
                    cutR = interfacial(v[kR, jR, iR])
                    sf = 0.5 * (sg[kL, jL, iL] + sg[kR, jR, iR])
                    if cutL and cutR:
                        kf = 0.5 * (kap[kL, jL, iL] + kap[kR, jR, iR])
                    else:
                        kf = kap[kL, jL, iL] if cutL else (kap[kR, jR, iR] if cutR else 0.0)
                    fc[k, j, i] = -sf * kf * (v[kR, jR, iR] - v[kL, jL, iL]) / h

                    def face_grad(a):
                        g = [0.0, 0.0, 0.0]
                        g[d] = (a[kR, jR, iR] - a[kL, jL, iL]) / h
                        for t in range(3):
                            if t == d:
                                continue
                            for X in (L, R):
                                g[t] += 0.5 * (_at(a, _off(X, t, 1), q, per) -
                                               _at(a, _off(X, t, -1), q, per)) / (2 * h)
                        return g
                    gs = face_grad(sg)
                    gc = face_grad(ch)
                    nrm = max(math.sqrt(gc[0] ** 2 + gc[1] ** 2 + gc[2] ** 2), 1e-6)
                    nn = [gc[e] / nrm for e in range(3)]
                    ndot = nn[0] * gs[0] + nn[1] * gs[1] + nn[2] * gs[2]
                    dmf = 0.5 * (dm[kL, jL, iL] + dm[kR, jR, iR])
                    fm[k, j, i] = dmf * (gs[d] - nn[d] * ndot)
        cap.append(fc)
        ma.append(fm)
    return cap, ma


# ---- one face at a time (for sampled comparisons on large boxes)
def cell_kappa(prob, vof, chi, x):
    """kappa of interfacial cell x: its height curvature, else the mean of
    the height curvatures of the interfacial cells of its 3x3x3 block (dz,
    dy, dx from -1 to 1), else the level-set curvature moved to the
    interface."""
    kk = height_curvature(prob, vof, x)
    if kk is not None:
        return kk
    q = O.full(prob)
    per = _axes(q)
    v = np.asarray(vof, dtype=np.float64)
    s, cnt = 0.0, 0
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == 0 and dy == 0 and dz == 0:
                    continue
                y = [x[0] + dx, x[1] + dy, x[2] + dz]
                if not interfacial(_at(v, y, q, per)):
                    continue
                y = [_map(y[e], q["n"][e], per[e]) for e in range(3)]
                val = height_curvature(prob, vof, y)
                if val is not None:
                    s += val
                    cnt += 1
    return s / cnt if cnt else levelset_curvature(prob, chi, x)


def face_force(prob, vof, chi, sigma, d, face):
    """(capillary, Marangoni) on the face along d with index face = (i, j, k)
    in the face layout (coordinate d runs to n_d), as forces() gives it."""
    q = O.full(prob)
    per = _axes(q)
    h = q["h"]
    n = q["n"]
    f = face[d]
    if (f == 0 or f == n[d]) and not per[d]:
        return 0.0, 0.0
    v = np.asarray(vof, dtype=np.float64)
    sg = np.asarray(sigma, dtype=np.float64)
    ch = np.asarray(chi, dtype=np.float64)
    R = list(face)
    R[d] = f % n[d]
    L = list(R)
    L[d] = (f - 1) % n[d]
    cL, cR = v[L[2], L[1], L[0]], v[R[2], R[1], R[0]]
    cutL, cutR = interfacial(cL), interfacial(cR)
    kL = cell_kappa(prob, vof, chi, L) if cutL else 0.0
    kR = cell_kappa(prob, vof, chi, R) if cutR else 0.0
    kf = 0.5 * (kL + kR) if cutL and cutR else (kL if cutL else (kR if cutR else 0.0))
    sf = 0.5 * (sg[L[2], L[1], L[0]] + sg[R[2], R[1], R[0]])
    cap = -sf * kf * (cR - cL) / h

    def grad(a):
        g = [0.0, 0.0, 0.0]
        g[d] = (a[R[2], R[1], R[0]] - a[L[2], L[1], L[0]]) / h
        for t in range(3):
            if t != d:
                for X in (L, R):
                    g[t] += 0.5 * (_at(a, _off(X, t, 1), q, per) -
                                   _at(a, _off(X, t, -1), q, per)) / (2 * h)
        return g
    gs, gc = grad(sg), grad(ch)
    nrm = max(math.sqrt(gc[0] ** 2 + gc[1] ** 2 + gc[2] ** 2), 1e-6)
    nn = [gc[e] / nrm for e in range(3)]
    ndot = nn[0] * gs[0] + nn[1] * gs[1] + nn[2] * gs[2]
    dmf = 0.5 * (cell_delta(prob, vof, L) + cell_delta(prob, vof, R))
    return cap, dmf * (gs[d] - nn[d] * ndot)
