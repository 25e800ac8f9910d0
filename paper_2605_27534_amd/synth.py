"""Seeded synthetic inputs: VoF fractions and face velocities.

This module holds no step arithmetic: it only produces the prescribed inputs
(interfaces, velocity fields, random initial concentrations) that both the
HIP library and the CPU oracle consume.  Everything is FP64 NumPy; FP32 runs
cast the arrays.  Shapes follow the library layout: cells [nz][ny][nx] with
x fastest; faces along axis d carry n_d + 1 entries along d.

Geometry convention: fluid 1 (the bubble / disperse phase) is the inside of
the circle or sphere, so vof = 1 there and the liquid is outside.
"""
from __future__ import annotations

import math

import numpy as np


def cell_centres(n, h, origin=(0.0, 0.0, 0.0)):
    nx, ny, nz = (list(n) + [1, 1])[:3]
    x = origin[0] + (np.arange(nx) + 0.5) * h
    y = origin[1] + (np.arange(ny) + 0.5) * h
    z = origin[2] + (np.arange(nz) + 0.5) * h
    return x, y, z


def _subcell_offsets(sub, dim, h):
    s = (np.arange(sub) + 0.5) / sub - 0.5
    if dim == 2:
        ox, oy = np.meshgrid(s, s, indexing="xy")
        return ox.ravel() * h, oy.ravel() * h, np.zeros(sub * sub)
    oz, oy, ox = np.meshgrid(s, s, s, indexing="ij")
    return ox.ravel() * h, oy.ravel() * h, oz.ravel() * h


def vof_ball(n, h, centre, R, dim, sub=8, origin=(0.0, 0.0, 0.0), period_z=None):
    """Fraction of sub^dim subcell centres inside a circle (dim 2) or sphere
    (dim 3) of radius R.  Values are k / sub^dim, exact in binary for
    sub = 8.  `period_z` (box length) takes the nearest periodic image in z.
    Only the cells of the ball's bounding box are visited."""
    x, y, z = cell_centres(n, h, origin)
    nx, ny, nz = len(x), len(y), len(z)
    f = np.zeros((nz, ny, nx))
    pad = R + h

    def span(coord, c):
        lo = np.searchsorted(coord, c - pad, side="left")
        hi = np.searchsorted(coord, c + pad, side="right")
        return slice(int(lo), int(hi))

    sx, sy = span(x, centre[0]), span(y, centre[1])
    if dim == 3:
        zs = [centre[2]]
        if period_z is not None:
            zs = [centre[2] - period_z, centre[2], centre[2] + period_z]
        szs = [(span(z, zc), zc) for zc in zs]
    else:
        szs = [(slice(0, nz), None)]
    half_diag = 0.5 * h * math.sqrt(dim) * (1 + 1e-9)
    ox, oy, oz = _subcell_offsets(sub, dim, h)
    for sz, zc in szs:
        xs, ys, zz = x[sx], y[sy], z[sz]
        if xs.size == 0 or ys.size == 0 or zz.size == 0:
            continue
        dx = xs - centre[0]
        dy = ys - centre[1]
        dz = (zz - zc) if dim == 3 else np.zeros(zz.size)
        r = np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
        block = np.zeros(r.shape)
        block[r <= R - half_diag] = 1.0
        cut = np.nonzero(np.abs(r - R) < half_diag)
        if cut[0].size:
            px = dx[cut[2]][:, None] + ox[None, :]
            py = dy[cut[1]][:, None] + oy[None, :]
            pz = dz[cut[0]][:, None] + oz[None, :]
            inside = (px * px + py * py + pz * pz) < R * R
            block[cut] = inside.sum(axis=1) / float(sub ** dim)
        f[sz, sy, sx] = np.maximum(f[sz, sy, sx], block)
    return f


def distance_ball(n, h, centre, R, clamp, origin=(0.0, 0.0, 0.0), period_z=None):
    """Signed distance R - |x - centre| to a sphere, or a circle for a 2D n
    (positive inside), cut to [-clamp, clamp], at the cell centres of an
    (nz, ny, nx) box; `period_z` (box length) takes the nearest periodic
    image in z."""
    x, y, z = cell_centres(n, h, origin)
    dz = z - centre[2] if len(n) == 3 else np.zeros(1)
    if period_z is not None:
        dz = dz - period_z * np.round(dz / period_z)
    dy = y - centre[1]
    dx = x - centre[0]
    out = np.empty((len(z), len(y), len(x)))
    for k in range(len(z)):  # a plane at a time: no full-box temporaries
        r = np.sqrt(dz[k] ** 2 + dy[:, None] ** 2 + dx[None, :] ** 2)
        out[k] = np.clip(R - r, -clamp, clamp)
    return out


def vof_disc(n, h, centre, R, samples=256, origin=(0.0, 0.0, 0.0)):
    """2D fraction of each cell inside a circle, integrated along x with the
    midpoint rule (`samples` points per cell) over the exact covered length
    in y: relative errors of order (1/samples)^2, against 1/64 for the
    subcell count of vof_ball (what curvature from volume fractions needs)."""
    nx, ny = n[0], n[1]
    x0 = origin[0] + np.arange(nx) * h
    y0 = origin[1] + np.arange(ny) * h
    t = (np.arange(samples) + 0.5) / samples * h
    f = np.zeros((1, ny, nx))
    for i in range(nx):
        xs = x0[i] + t - centre[0]
        s = np.sqrt(np.maximum(R * R - xs * xs, 0.0))
        lo = np.maximum(y0[:, None], centre[1] - s[None, :])
        hi = np.minimum(y0[:, None] + h, centre[1] + s[None, :])
        f[0, :, i] = np.mean(np.clip(hi - lo, 0.0, h), axis=1) / h
    # full and empty cells exactly (the sums above round)
    f[f > 1.0 - 1e-13] = 1.0
    f[f < 1e-13] = 0.0
    return f


def vof_flat(n, h, y0, origin=(0.0, 0.0, 0.0)):
    """Flat interface at y = y0, fluid 1 below: f = fraction of the cell
    below y0 (exact)."""
    nx, ny, nz = (list(n) + [1, 1])[:3]
    ylo = origin[1] + np.arange(ny) * h
    frac = np.clip((y0 - ylo) / h, 0.0, 1.0)
    return np.broadcast_to(frac[None, :, None], (nz, ny, nx)).copy()


def face_centres(n, h, d, origin=(0.0, 0.0, 0.0)):
    """Coordinates (x, y, z) broadcastable to the face array along axis d."""
    nx, ny, nz = (list(n) + [1, 1])[:3]
    m = [nx, ny, nz]
    m[d] += 1
    coords = []
    for e in range(3):
        if e == d:
            c = origin[e] + np.arange(m[e]) * h
        else:
            c = origin[e] + (np.arange(m[e]) + 0.5) * h
        coords.append(c)
    X = coords[0][None, None, :]
    Y = coords[1][None, :, None]
    Z = coords[2][:, None, None]
    return X, Y, Z


def zeros_faces(n, dim):
    nx, ny, nz = (list(n) + [1, 1])[:3]
    out = []
    for d in range(dim):
        m = [nz, ny, nx]
        m[2 - d] += 1
        out.append(np.zeros(m))
    return out


def u_rotation(n, h, centre, omega, origin=(0.0, 0.0, 0.0)):
    """2D solid-body rotation u = omega (-(y - yc), x - xc).  Face-normal
    components are independent of the normal coordinate, so the face values
    are exact averages and the field is discretely divergence free."""
    X, Y, _ = face_centres(n, h, 0, origin)
    ux = np.broadcast_to(-omega * (Y - centre[1]) + 0 * X, face_centres_shape(n, 0)).copy()
    X, Y, _ = face_centres(n, h, 1, origin)
    uy = np.broadcast_to(omega * (X - centre[0]) + 0 * Y, face_centres_shape(n, 1)).copy()
    return [ux, uy]


def u_uniform(n, dim, U):
    """The same velocity U[d] on every face along d."""
    out = zeros_faces(n, dim)
    for d in range(dim):
        out[d][...] = U[d]
    return out


def u_axisym_strain(n, h, a, z0, origin=(0.0, 0.0, 0.0)):
    """Axisymmetric straining flow on an (r, z) grid (x the radius): u_r = a r,
    u_z = -2 a (z - z0), at the face centres.  r_face u_r differences over a
    ring balance the axial ones exactly, so the field is discretely
    divergence free in the axisymmetric sense."""
    X, Y, _ = face_centres(n, h, 0, origin)
    ur = np.broadcast_to(a * X + 0 * Y, face_centres_shape(n, 0)).copy()
    X, Y, _ = face_centres(n, h, 1, origin)
    uz = np.broadcast_to(-2.0 * a * (Y - z0) + 0 * X, face_centres_shape(n, 1)).copy()
    return [ur, uz]


def face_centres_shape(n, d):
    nx, ny, nz = (list(n) + [1, 1])[:3]
    m = [nz, ny, nx]
    m[2 - d] += 1
    return tuple(m)


def u_expansion(n, h, centre, K, dim, origin=(0.0, 0.0, 0.0)):
    """Uniform radial expansion u = K (x - xc): face averages are exact."""
    out = []
    for d in range(dim):
        X, Y, Z = face_centres(n, h, d, origin)
        c = (X, Y, Z)[d]
        out.append(np.broadcast_to(K * (c - centre[d]), face_centres_shape(n, d)).copy())
    return out


def u_source2d(n, h, centre, Q, r_core=0.02, origin=(0.0, 0.0, 0.0)):
    """2D point source of strength Q, u = Q r_hat / (2 pi r), regularised to
    the linear field Q x / (2 pi r_core^2) inside r_core.  Away from the core
    each face value is the exact mean normal velocity over the face
    (Q times the subtended angle over 2 pi, divided by h), so the field is
    discretely divergence free there."""
    out = []
    for d in range(2):
        X, Y, _ = face_centres(n, h, d, origin)
        Xc = np.broadcast_to(X - centre[0], face_centres_shape(n, d))
        Yc = np.broadcast_to(Y - centre[1], face_centres_shape(n, d))
        if d == 0:  # normal x, segment along y
            A, B0, B1 = Xc, Yc - 0.5 * h, Yc + 0.5 * h
        else:       # normal y, segment along x
            A, B0, B1 = Yc, Xc - 0.5 * h, Xc + 0.5 * h
        with np.errstate(divide="ignore", invalid="ignore"):
            exact = Q / (2 * math.pi) * (np.arctan(B1 / A) - np.arctan(B0 / A)) / h
        point = Q * A / (2 * math.pi * r_core ** 2)
        r = np.sqrt(Xc ** 2 + Yc ** 2)
        near = r < r_core + h
        out.append(np.where(near, point, np.nan_to_num(exact)))
    return out


def _hr_velocity(x, y, z, a, V, lam):
    """Hadamard-Rybczynski creeping flow past a fluid sphere of radius a
    (viscosity ratio lam) with far-field velocity V along z, sphere at the
    origin.  Stream function Psi = A(r) sin^2(theta);
    u_r = 2 A cos(theta) / r^2, u_theta = -A' sin(theta) / r."""
    r = np.sqrt(x * x + y * y + z * z)
    r = np.maximum(r, 1e-300)
    rho = np.sqrt(x * x + y * y)
    cth = z / r
    sth = rho / r
    k1 = (2 + 3 * lam) / (2 * (1 + lam))
    k2 = lam / (2 * (1 + lam))
    outside = r >= a
    Ao = 0.5 * V * (r * r - k1 * a * r + k2 * a ** 3 / r)
    dAo = 0.5 * V * (2 * r - k1 * a - k2 * a ** 3 / (r * r))
    ci = -V / (4 * (1 + lam))
    Ai = ci * (r * r - r ** 4 / (a * a))
    dAi = ci * (2 * r - 4 * r ** 3 / (a * a))
    A = np.where(outside, Ao, Ai)
    dA = np.where(outside, dAo, dAi)
    ur = 2 * A * cth / (r * r)
    ut = -dA * sth / r
    # unit vectors: e_r = (x, y, z)/r ; e_theta = (cos th cos ph, cos th sin ph, -sin th)
    with np.errstate(invalid="ignore", divide="ignore"):
        cph = np.where(rho > 0, x / np.maximum(rho, 1e-300), 1.0)
        sph = np.where(rho > 0, y / np.maximum(rho, 1e-300), 0.0)
    ux = ur * sth * cph + ut * cth * cph
    uy = ur * sth * sph + ut * cth * sph
    uz = ur * cth - ut * sth
    return ux, uy, uz


def u_hadamard(n, h, centre, a, V, lam, frame_shift=0.0, origin=(0.0, 0.0, 0.0),
               period_z=None):
    """Face-centre values of the Hadamard-Rybczynski flow around a sphere at
    `centre` (sphere-frame far-field velocity V along z), plus `frame_shift`
    added to the z component (lab frame of a sphere moving at -V)."""
    out = []
    for d in range(3):
        X, Y, Z = face_centres(n, h, d, origin)
        shp = face_centres_shape(n, d)
        Xc = np.broadcast_to(X - centre[0], shp)
        Yc = np.broadcast_to(Y - centre[1], shp)
        Zc = np.broadcast_to(Z - centre[2], shp)
        if period_z is not None:
            Zc = Zc - period_z * np.round(Zc / period_z)
        ux, uy, uz = _hr_velocity(Xc, Yc, Zc, a, V, lam)
        out.append(np.ascontiguousarray((ux, uy, uz + frame_shift)[d]))
    return out


def u_hadamard_axi(n, h, zc, a, V, lam, frame_shift=0.0, origin=(0.0, 0.0, 0.0),
                   period_z=None):
    """The Hadamard-Rybczynski flow of `u_hadamard` on an axisymmetric (r, z)
    grid (x the radius from origin[0], y the axis), the sphere on the axis at
    z = zc: u_r on the radial faces, u_z (+ frame_shift) on the axial faces."""
    out = []
    for d in range(2):
        X, Y, _ = face_centres(n, h, d, origin)
        shp = face_centres_shape(n, d)
        R = np.broadcast_to(X, shp)
        Zc = np.broadcast_to(Y - zc, shp)
        if period_z is not None:
            Zc = Zc - period_z * np.round(Zc / period_z)
        ur, _, uz = _hr_velocity(R, np.zeros(shp), Zc, a, V, lam)
        out.append(np.ascontiguousarray(ur if d == 0 else uz + frame_shift))
    return out


def smooth_modes(n, h, seed, nmodes=8, kmax=3, dim=3, origin=(0.0, 0.0, 0.0)):
    """Sum of `nmodes` cosine modes with integer wave vectors |k|_inf <= kmax
    and random phases, normalised to max |s| = 1 (seeded)."""
    rng = np.random.default_rng(seed)
    x, y, z = cell_centres(n, h, origin)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    s = np.zeros_like(X)
    for _ in range(nmodes):
        k = rng.integers(-kmax, kmax + 1, size=3)
        if dim == 2:
            k[2] = 0
        ph = rng.uniform(0, 2 * math.pi)
        amp = rng.uniform(0.5, 1.0)
        s += amp * np.cos(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
    return s / np.max(np.abs(s))


def uniform_field(n, seed, lo, hi):
    """Per-cell U[lo, hi] values (seeded)."""
    nx, ny, nz = (list(n) + [1, 1])[:3]
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(nz, ny, nx))


def random_state(n, seed, lo=0.0, hi=1.0):
    """Two seeded random cell fields (used by brute-force checks)."""
    nx, ny, nz = (list(n) + [1, 1])[:3]
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(nz, ny, nx)), rng.uniform(lo, hi, size=(nz, ny, nx))


def random_faces(n, dim, seed, scale):
    rng = np.random.default_rng(seed)
    return [rng.uniform(-scale, scale, size=face_centres_shape(n, d)) for d in range(dim)]
