"""Shared helpers of the parity tests: run the same seeded inputs through the
FP64 oracle and through libsurf, and compare them."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def rel_max(a, b):
    """||a - b||_inf / ||b||_inf (field by field; 0 when both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    num = np.max(np.abs(a - b))
    if den == 0:
        return float(num)
    return float(num / den)


def to_np(t):
    return t.detach().to("cpu").double().numpy()


def run_oracle(prob, vof0, nsteps, dt, u=None, u_seq=None, vof_seq=None, chi=None,
               c0=None, c0_const=1.0, gamma0=0.0, hj_init=None, hj_step=8):
    q = O.full(prob)
    if chi is None:
        iters = hj_init if hj_init is not None else default_hj_init(q)
        chi = O.geometry(prob, vof0, iters)
    F, P = O.init_state(prob, chi, c0=c0, c0_const=c0_const, gamma0=gamma0)
    chi, F, P, S, hist = O.run(prob, chi, u, F, P, dt, nsteps, vof_seq=vof_seq,
                               hj_iters=hj_step, u_seq=u_seq)
    return chi, F, P, S, hist


def default_hj_init(q):
    import math
    chimax = q["chi_max_eps"] * q["eps"]
    dtau = q["h"] / q["dim"]
    return 2 * int(math.ceil(chimax / dtau - 1e-9))


def run_gpu(prob, vof0, nsteps, dt, precision, u=None, u_seq=None, vof_seq=None, chi=None,
            c0=None, c0_const=1.0, gamma0=0.0, hj_step=8):
    import torch
    from paper_2605_27534_amd import surf as S
    p = dict(prob)
    p["hj_iters_step"] = hj_step
    s = S.Surf(p, dt, precision)
    if chi is None:
        s.set_geometry(s.tensor(vof0), full=True)
    else:
        s.set_levelset(s.tensor(chi))
    F, P = s.init_state(None if c0 is None else s.tensor(c0), c0_const, gamma0)
    hist = torch.zeros((max(nsteps, 1), 16), dtype=torch.float64, device="cuda")
    F2 = s.empty() if F is not None else None
    P2 = s.empty()
    sig = s.empty()
    ud = None if u is None else [s.tensor(v) for v in u]
    for n in range(nsteps):
        un = ud if u_seq is None else [s.tensor(v) for v in u_seq(n)]
        vn = None if vof_seq is None else s.tensor(vof_seq(n))
        s.step(F, P, F2, P2, u=un, vof_next=vn, sigma_out=sig, totals=hist[n])
        F, F2 = F2, F
        P, P2 = P2, P
    torch.cuda.synchronize()
    chi_out = to_np(s.levelset())
    out = (chi_out, None if F is None else to_np(F), to_np(P), to_np(sig),
           hist.cpu().numpy()[:nsteps], s)
    return out


def compare_totals(tg, to, tt, F_o, P_o, slot_tol=None):
    """Every slot of one step's totals against the oracle's: the sums, the
    interface averages, the stable step and the largest cell-mean speed
    relative to themselves; the open-side budget relative to the total
    surfactant; the minima relative to their field's max-norm (a minimum
    near zero has no relative size of its own); the count of non-finite
    values exactly.  slot_tol: a relative tolerance per slot in place of tt
    for those slots (each caller states its derivation)."""
    slot_tol = slot_tol or {}
    for slot in (O.T_MB, O.T_MS, O.T_SDELTA, O.T_SSIGD, O.T_MTOT, O.T_GAVG, O.T_SAVG,
                 O.T_SU, O.T_DTNEXT, O.T_CMAX):
        a, b = tg[slot], to[slot]
        if a == b:  # equal, infinities included (no flow: no advective bound)
            continue
        assert abs(a - b) <= slot_tol.get(slot, tt) * max(abs(b), 1e-300), (slot, a, b)
    scale = abs(to[O.T_MB]) + abs(to[O.T_MS])
    for slot in (O.T_OUT, O.T_OUTCUM):
        assert abs(tg[slot] - to[slot]) <= tt * scale, (slot, tg[slot], to[slot])
    if F_o is not None:
        Fs = np.max(np.abs(F_o))
        assert abs(tg[O.T_MINF] - to[O.T_MINF]) <= tt * Fs, (tg[O.T_MINF], to[O.T_MINF])
    Ps = np.max(np.abs(P_o))
    assert abs(tg[O.T_MINPSI] - to[O.T_MINPSI]) <= tt * Ps, (tg[O.T_MINPSI], to[O.T_MINPSI])
    assert tg[O.T_NBAD] == to[O.T_NBAD]
    assert abs(tg[O.T_T] - to[O.T_T]) <= 1e-14 * abs(to[O.T_T])
