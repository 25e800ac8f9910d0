"""Python face of the FP64 CPU oracle (``surf_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product path never does.  It
shares no code with the HIP library.

A problem is described by a plain dict (the same keys the library's
parameter structs use):

    dim, n=(nx, ny, nz), h, bc=((xlo, xhi), (ylo, yhi), (zlo, zhi)),
    flux_form, kinetics, eos, bulk_enabled, eps, D_b, D_s, k_a, k_d,
    gamma_inf, sigma0, eos_E, eta, chi_max_eps, cfl_adv, cfl_diff

Arrays are float64 numpy arrays in [nz][ny][nx] order (x fastest); face
arrays along axis d have n_d + 1 entries along d.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "surf_oracle.c")
_OUT = os.path.join(_HERE, "_build", "liboracle.so")

# totals slots (16 doubles)
T_MB, T_MS, T_OUT, T_OUTCUM, T_SDELTA, T_SSIGD, T_SU, T_DTNEXT = range(8)
T_MINF, T_MINPSI, T_NBAD, T_T, T_GAVG, T_SAVG, T_MTOT, T_CMAX = range(8, 16)

BC_WALL, BC_PERIODIC, BC_OPEN = 0, 1, 2

DEFAULTS = dict(
    flux_form=0, kinetics=0, eos=0, bulk_enabled=1, D_b=1e-2, D_s=1e-3,
    k_a=1.0, k_d=1.0, gamma_inf=1.0, sigma0=1.0, eos_E=0.5, eta=1e-12,
    chi_max_eps=12.0, cfl_adv=0.5, cfl_diff=0.8, axisym=0, limiter=0, bcg_transverse=0,
)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math; OpenMP over the
    independent cell and face loops, every sum in a fixed serial order)."""
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    if force or not os.path.exists(_OUT) or os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
        tmp = _OUT + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-fno-fast-math", "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _OUT)
    return _OUT


_lib = None
_gomp = None
_max_threads = None


_forced_threads = None


def _threads_for(ncell):
    """One thread for small grids (a parallel region costs more than their
    loops), all of them otherwise, unless set_threads fixed the count; the
    arithmetic does not depend on it."""
    global _gomp, _max_threads
    if _gomp is None:
        try:
            _gomp = ctypes.CDLL("libgomp.so.1")
            _max_threads = int(_gomp.omp_get_max_threads())
        except OSError:
            _gomp = False
    if _gomp:
        if _forced_threads:
            _gomp.omp_set_num_threads(_forced_threads)
        else:
            _gomp.omp_set_num_threads(1 if ncell < 65536 else _max_threads)


def set_threads(n=None):
    """Run every following call on n threads (None: the size rule above).
    Returns the thread count the oracle then uses on a large grid."""
    global _forced_threads
    lib()
    _threads_for(0)
    _forced_threads = int(n) if n else None
    return _forced_threads or (_max_threads if _gomp else 1)


def lib():
    global _lib
    if _lib is None:
        # idle threads wait asleep: the oracle shares the host with the tests
        os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")
        _lib = ctypes.CDLL(build())
        # keep freed work arrays in the heap (glibc): the oracle allocates its
        # field-sized temporaries per call, and fresh pages for each call
        # would cost more than the loops at the larger sizes
        try:
            libc = ctypes.CDLL("libc.so.6")
            libc.mallopt(-3, 32 << 20)  # M_MMAP_THRESHOLD (glibc's largest)
            libc.mallopt(-1, 1 << 30)   # M_TRIM_THRESHOLD
        except OSError:
            pass
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def full(prob: dict) -> dict:
    q = dict(DEFAULTS)
    q.update(prob)
    n = list(q["n"]) + [1] * (3 - len(q["n"]))
    q["n"] = tuple(int(v) for v in n)
    if "eps" not in q:
        q["eps"] = 1.5 * q["h"]
    return q


def pack(prob: dict):
    q = full(prob)
    lib()
    _threads_for(q["n"][0] * q["n"][1] * q["n"][2])
    bc = q.get("bc", ((0, 0), (0, 0), (0, 0)))
    bc = [tuple(b) for b in bc] + [(0, 0)] * (3 - len(bc))
    for b in bc:
        assert (b[0] == BC_PERIODIC) == (b[1] == BC_PERIODIC), "periodic axes wrap on both sides"
    ip = np.array([q["dim"], *q["n"], bc[0][0], bc[0][1], bc[1][0], bc[1][1],
                   bc[2][0], bc[2][1], q["flux_form"], q["kinetics"], q["eos"],
                   q["bulk_enabled"], int(q["axisym"]), int(q["limiter"]),
                   int(q["bcg_transverse"])], dtype=np.int32)
    r0 = float(q.get("origin", (0.0, 0.0, 0.0))[0])
    dp = np.array([q["h"], q["eps"], q["D_b"], q["D_s"], q["k_a"], q["k_d"],
                   q["gamma_inf"], q["sigma0"], q["eos_E"], q["eta"],
                   q["chi_max_eps"], q["cfl_adv"], q["cfl_diff"], r0, 0, 0],
                  dtype=np.float64)
    return ip, dp


def shape(prob: dict):
    q = full(prob)
    nx, ny, nz = q["n"]
    return (nz, ny, nx)


def face_shape(prob: dict, d: int):
    nz, ny, nx = shape(prob)
    s = [nz, ny, nx]
    s[2 - d] += 1
    return tuple(s)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def geometry(prob, vof, iters, chi=None):
    """chi from vof by `iters` HJ sweeps; warm start from `chi` if given."""
    ip, dp = pack(prob)
    vof = _f64(vof)
    out = np.zeros(shape(prob)) if chi is None else _f64(chi).copy()
    rc = lib().or_geometry(_p(ip), _p(dp), _p(vof), _p(out), ctypes.c_int(iters),
                           ctypes.c_int(0 if chi is None else 1))
    assert rc == 0
    return out


def pin_data(prob, vof):
    ip, dp = pack(prob)
    pin = np.zeros(shape(prob), dtype=np.uint8)
    D = np.zeros(shape(prob))
    rc = lib().or_pin_data(_p(ip), _p(dp), _p(_f64(vof)), _p(pin), _p(D))
    assert rc == 0
    return pin.astype(bool), D


def cell_geometry(prob, chi):
    ip, dp = pack(prob)
    phi, om, de = (np.zeros(shape(prob)) for _ in range(3))
    lib().or_cell_geometry(_p(ip), _p(dp), _p(_f64(chi)), _p(phi), _p(om), _p(de))
    return phi, om, de


def eos(prob, G):
    ip, dp = pack(prob)
    G = _f64(G)
    out = np.zeros_like(G)
    lib().or_eos(_p(ip), _p(dp), _p(G), ctypes.c_long(G.size), _p(out))
    return out


def init_state(prob, chi, c0=None, c0_const=1.0, gamma0=0.0):
    ip, dp = pack(prob)
    F, psi = np.zeros(shape(prob)), np.zeros(shape(prob))
    c0a = None if c0 is None else _f64(c0)
    lib().or_init_state(_p(ip), _p(dp), _p(_f64(chi)), _p(c0a),
                        ctypes.c_double(c0_const), ctypes.c_double(gamma0),
                        _p(F), _p(psi))
    return F, psi


def advect(prob, u, xi, dt):
    ip, dp = pack(prob)
    us = [None if v is None else _f64(v) for v in (list(u) + [None] * 3)[:3]]
    xs = np.zeros(shape(prob))
    out = ctypes.c_double(0.0)
    rc = lib().or_advect(_p(ip), _p(dp), _p(us[0]), _p(us[1]), _p(us[2]),
                         _p(_f64(xi)), ctypes.c_double(dt), _p(xs), ctypes.byref(out))
    assert rc == 0
    return xs, out.value


def step(prob, chi, u, F, psi, dt, totals=None):
    """One step.  Returns (F, psi, sigma, totals)."""
    ip, dp = pack(prob)
    us = [None] * 3 if u is None else [None if v is None else _f64(v)
                                       for v in (list(u) + [None] * 3)[:3]]
    Fo, Po, S = (np.zeros(shape(prob)) for _ in range(3))
    tot = np.zeros(16) if totals is None else np.array(totals, dtype=np.float64)
    rc = lib().or_step(_p(ip), _p(dp), _p(_f64(chi)), _p(us[0]), _p(us[1]), _p(us[2]),
                       _p(_f64(F)), _p(_f64(psi)), ctypes.c_double(dt),
                       _p(Fo), _p(Po), _p(S), _p(tot))
    assert rc == 0
    return Fo, Po, S, tot


def force(prob, chi, sigma):
    ip, dp = pack(prob)
    q = full(prob)
    outs = [np.zeros(face_shape(prob, d)) for d in range(q["dim"])] + [None] * (3 - q["dim"])
    lib().or_force(_p(ip), _p(dp), _p(_f64(chi)), _p(_f64(sigma)),
                   _p(outs[0]), _p(outs[1]), _p(outs[2]))
    return outs[:q["dim"]]


def run(prob, chi, u, F, psi, dt, nsteps, vof_seq=None, hj_iters=8, totals=None,
        u_seq=None):
    """nsteps steps.  vof_seq(n) -> vof at t^{n+1} (moving geometry: chi is
    warm-started with hj_iters sweeps before each step); u_seq(n) -> u^n."""
    tot = np.zeros(16) if totals is None else totals
    hist = []
    for n in range(nsteps):
        if vof_seq is not None:
            chi = geometry(prob, vof_seq(n), hj_iters, chi=chi)
        un = u_seq(n) if u_seq is not None else u
        F, psi, S, tot = step(prob, chi, un, F, psi, dt, tot)
        hist.append(tot.copy())
    return chi, F, psi, S, np.array(hist)


# ---------------------------------------------------------------- adjoint
def adjoint_step(prob, chi, u, F, psi, dt, mF, mP):
    """lambda^n from lambda^{n+1} = (mF, mP) for the step from (F, psi);
    returns (lF, lP, dtheta[4]) with dtheta = d/d(k_a, k_d, D_b, D_s)."""
    ip, dp = pack(prob)
    us = [None] * 3 if u is None else [None if v is None else _f64(v)
                                       for v in (list(u) + [None] * 3)[:3]]
    lF, lP = np.zeros(shape(prob)), np.zeros(shape(prob))
    dth = np.zeros(4)
    rc = lib().or_adjoint_step(_p(ip), _p(dp), _p(_f64(chi)), _p(us[0]), _p(us[1]), _p(us[2]),
                               _p(_f64(F)), _p(_f64(psi)), ctypes.c_double(dt),
                               _p(_f64(mF)), _p(_f64(mP)), _p(lF), _p(lP), _p(dth))
    assert rc == 0
    return lF, lP, dth


def loss_grad(prob, chi, psi, w):
    ip, dp = pack(prob)
    g = np.zeros(shape(prob))
    lib().or_loss_grad(_p(ip), _p(dp), _p(_f64(chi)), _p(_f64(psi)), ctypes.c_double(w), _p(g))
    return g


def with_theta(prob, theta):
    q = dict(prob)
    q["k_a"], q["k_d"], q["D_b"], q["D_s"] = (float(v) for v in theta)
    return q


def rollout(prob, chi, u, c0, gamma0, dt, nsteps, theta):
    """Forward run from F0 = c0 phi, psi0 = gamma0 delta at parameters theta;
    returns the states [x^0 .. x^N] and <sigma>^n for n = 1..N."""
    q = with_theta(prob, theta)
    F, P = init_state(q, chi, c0=c0, gamma0=gamma0)
    states = [(F, P)]
    sig = []
    tot = np.zeros(16)
    for _ in range(nsteps):
        F, P, _, tot = step(q, chi, u, F, P, dt, tot)
        states.append((F, P))
        sig.append(tot[T_SAVG])
    return states, np.array(sig)


def sigma_history_loss(prob, chi, u, c0, gamma0, dt, nsteps, theta, target):
    """L = mean over steps n = 1..N of (<sigma>^n - target^n)^2."""
    _, sig = rollout(prob, chi, u, c0, gamma0, dt, nsteps, theta)
    return float(np.mean((sig - target) ** 2))


def sigma_history_grad(prob, chi, u, c0, gamma0, dt, nsteps, theta, target):
    """Loss and its gradient with respect to theta (4) and the initial bulk
    concentration field c0, by the discrete adjoint (all states stored)."""
    q = with_theta(prob, theta)
    states, sig = rollout(prob, chi, u, c0, gamma0, dt, nsteps, theta)
    loss = float(np.mean((sig - target) ** 2))
    phi, _, de = cell_geometry(q, chi)
    sd = de.sum() * q["h"] ** q["dim"]
    vol = q["h"] ** q["dim"]
    # d<sigma>/dpsi_i = sigma'(Gamma_i) delta_i vol / (sum delta vol (delta_i + eta/eps))
    w = lambda n: 2.0 / nsteps * (sig[n - 1] - target[n - 1]) * vol / sd
    lF = np.zeros(shape(q))
    lP = loss_grad(q, chi, states[nsteps][1], w(nsteps))
    dth = np.zeros(4)
    for n in range(nsteps - 1, -1, -1):
        F, P = states[n]
        lF, lP, d = adjoint_step(q, chi, u, F, P, dt, lF, lP)
        dth += d
        if n >= 1:
            lP = lP + loss_grad(q, chi, P, w(n))
    gc0 = lF * phi
    return loss, dth, gc0
