"""Device-side (torch) versions of the large seeded inputs of synth.py.

The translating-sphere workload needs a new VoF field and a new face
velocity field at every step of a 256^3 grid; generating those on the host
takes seconds per step.  These functions compute the same fields with the
same formulas in FP64 torch ops on any device (a GPU for the benchmark, the
CPU for the tests that check them against synth.py).  Like synth.py they
hold no step arithmetic: they only produce prescribed inputs.
"""
from __future__ import annotations

import math

import torch


def _axis(n, h, origin, faces, device):
    off = 0.0 if faces else 0.5
    return origin + (torch.arange(n + (1 if faces else 0), dtype=torch.float64, device=device) + off) * h


def vof_ball(n, h, centre, R, sub=8, origin=(0.0, 0.0, 0.0), period_z=None, device="cpu"):
    """Fraction of sub^3 subcell centres inside the sphere of radius R (3D
    only), the nearest periodic image in z when `period_z` is given; the same
    values as synth.vof_ball (k / sub^3, exact in binary for sub = 8)."""
    nx, ny, nz = n
    x = _axis(nx, h, origin[0], False, device)
    y = _axis(ny, h, origin[1], False, device)
    z = _axis(nz, h, origin[2], False, device)
    f = torch.zeros((nz, ny, nx), dtype=torch.float64, device=device)
    pad = R + h

    def span(c, cc):
        lo = int(torch.searchsorted(c, torch.tensor(cc - pad, dtype=torch.float64, device=device),
                                    right=False))
        hi = int(torch.searchsorted(c, torch.tensor(cc + pad, dtype=torch.float64, device=device),
                                    right=True))
        return slice(lo, hi)

    sx, sy = span(x, centre[0]), span(y, centre[1])
    zs = [centre[2]] if period_z is None else [centre[2] - period_z, centre[2], centre[2] + period_z]
    half_diag = 0.5 * h * math.sqrt(3) * (1 + 1e-9)
    s = (torch.arange(sub, dtype=torch.float64, device=device) + 0.5) / sub - 0.5
    oz, oy, ox = torch.meshgrid(s, s, s, indexing="ij")
    ox, oy, oz = ox.reshape(-1) * h, oy.reshape(-1) * h, oz.reshape(-1) * h
    for zc in zs:
        sz = span(z, zc)
        xs, ys, zz = x[sx], y[sy], z[sz]
        if xs.numel() == 0 or ys.numel() == 0 or zz.numel() == 0:
            continue
        dx, dy, dz = xs - centre[0], ys - centre[1], zz - zc
        r = torch.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
        block = torch.zeros_like(r)
        block[r <= R - half_diag] = 1.0
        cut = torch.nonzero(torch.abs(r - R) < half_diag, as_tuple=True)
        if cut[0].numel():
            cnt = torch.zeros(cut[0].numel(), dtype=torch.float64, device=device)
            for k0 in range(0, ox.numel(), 64):
                px = dx[cut[2]][:, None] + ox[None, k0:k0 + 64]
                py = dy[cut[1]][:, None] + oy[None, k0:k0 + 64]
                pz = dz[cut[0]][:, None] + oz[None, k0:k0 + 64]
                cnt += ((px * px + py * py + pz * pz) < R * R).sum(dim=1).to(torch.float64)
            block[cut] = cnt / float(sub ** 3)
        f[sz, sy, sx] = torch.maximum(f[sz, sy, sx], block)
    return f


def _hr_velocity(x, y, z, a, V, lam):
    """Hadamard-Rybczynski creeping flow past a fluid sphere of radius a at
    the origin (viscosity ratio lam, far-field V along z): the formulas of
    synth._hr_velocity."""
    r = torch.sqrt(x * x + y * y + z * z).clamp_min(1e-300)
    rho = torch.sqrt(x * x + y * y)
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
    A = torch.where(outside, Ao, Ai)
    dA = torch.where(outside, dAo, dAi)
    ur = 2 * A * cth / (r * r)
    ut = -dA * sth / r
    rs = rho.clamp_min(1e-300)
    cph = torch.where(rho > 0, x / rs, torch.ones_like(x))
    sph = torch.where(rho > 0, y / rs, torch.zeros_like(y))
    return (ur * sth * cph + ut * cth * cph, ur * sth * sph + ut * cth * sph, ur * cth - ut * sth)


def u_hadamard(n, h, centre, a, V, lam, frame_shift=0.0, origin=(0.0, 0.0, 0.0), period_z=None,
               device="cpu", dtype=torch.float64):
    """Face-centre values of the flow of synth.u_hadamard (x, y, z face
    arrays), computed in FP64 and returned in `dtype`."""
    nx, ny, nz = n
    out = []
    for d in range(3):
        X = _axis(nx, h, origin[0], d == 0, device)[None, None, :] - centre[0]
        Y = _axis(ny, h, origin[1], d == 1, device)[None, :, None] - centre[1]
        Z = _axis(nz, h, origin[2], d == 2, device)[:, None, None] - centre[2]
        if period_z is not None:
            Z = Z - period_z * torch.round(Z / period_z)
        shp = (Z.shape[0], Y.shape[1], X.shape[2])
        ux, uy, uz = _hr_velocity(X.expand(shp), Y.expand(shp), Z.expand(shp), a, V, lam)
        out.append(((ux, uy, uz + frame_shift)[d]).to(dtype).contiguous())
    return out
