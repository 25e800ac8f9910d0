"""Python binding of libsurf (include/surf.h): argument marshalling only.

Every step of the surfactant path runs in the HIP kernels of libsurf.so;
torch tensors serve as device buffers and torch's current HIP stream as the
stream.  Importing this module loads the library and raises if it is missing
(there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsurf.so")

SURF_F32, SURF_F64 = 0, 1
SURF_SUBSTEP2_EXPLICIT, SURF_SUBSTEP2_IMPLICIT = 0, 1
SURF_IFACE_VOF, SURF_IFACE_ACDI = 0, 1
FLUX_WEIGHTED, FLUX_PAPER = 0, 1
KIN_LANGMUIR, KIN_HENRY = 0, 1
EOS_LINEAR, EOS_LANGMUIR, EOS_TANH = 0, 1, 2
BC_WALL, BC_PERIODIC, BC_OPEN = 0, 1, 2
STATUS_NONFINITE, STATUS_NEGATIVE, STATUS_UNSTABLE, STATUS_GEOMETRY, STATUS_SOLVE = 1, 2, 4, 8, 16

# totals slots
T_MB, T_MS, T_OUT, T_OUTCUM, T_SDELTA, T_SSIGD, T_SU, T_DTNEXT = range(8)
T_MINF, T_MINPSI, T_NBAD, T_T, T_GAVG, T_SAVG, T_MTOT, T_CMAX = range(8, 16)

ERRORS = {0: "ok", -1: "invalid argument", -2: "workspace too small",
          -3: "HIP runtime error", -4: "call-order violation", -5: "unstable"}

EXPORTS = [
    "surf_workspace_bytes", "surf_init", "surf_set_geometry", "surf_set_levelset",
    "surf_get_levelset", "surf_get_phase", "surf_init_state", "surf_step", "surf_prepare_geometry",
    "surf_prepare_phase",
    "surf_time_transport", "surf_force", "surf_interface_force", "surf_set_dt",
    "surf_get_status", "surf_clear_status", "surf_solver_iterations", "surf_time_solver", "surf_time_acdi",
    "surf_destroy", "surf_strerror", "surf_version",
    "surf_profile_enable", "surf_profile_read", "surf_set_kinetics", "surf_loss_weights",
    "surf_adjoint_seed", "surf_adjoint_step", "surf_adjoint_c0",
    "surf_batch_workspace_bytes", "surf_batch_create", "surf_batch_set_geometry",
    "surf_batch_init_state", "surf_batch_step", "surf_batch_parity", "surf_batch_tune",
    "surf_batch_destroy", "surf_step_static", "surf_set_time", "surf_step_advected",
    "surf_adjoint_step_advected",
]


class SurfError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed: %s (%d)" % (what, ERRORS.get(code, "?"), code))
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3),
                ("bc", (ctypes.c_int32 * 2) * 3), ("axisym", ctypes.c_int32),
                ("h", ctypes.c_double), ("origin", ctypes.c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("flux_form", ctypes.c_int32),
                ("kinetics", ctypes.c_int32), ("eos", ctypes.c_int32),
                ("bulk_enabled", ctypes.c_int32), ("hj_iters_init", ctypes.c_int32),
                ("hj_iters_step", ctypes.c_int32), ("adjoint", ctypes.c_int32),
                ("eps", ctypes.c_double), ("D_b", ctypes.c_double), ("D_s", ctypes.c_double),
                ("k_a", ctypes.c_double), ("k_d", ctypes.c_double),
                ("gamma_inf", ctypes.c_double), ("sigma0", ctypes.c_double),
                ("eos_E", ctypes.c_double), ("eta", ctypes.c_double),
                ("chi_max_eps", ctypes.c_double), ("cfl_adv", ctypes.c_double),
                ("cfl_diff", ctypes.c_double), ("dt", ctypes.c_double),
                ("substep2", ctypes.c_int32), ("picard_iters", ctypes.c_int32),
                ("cg_max_iters", ctypes.c_int32), ("pad2_", ctypes.c_int32),
                ("cg_tol", ctypes.c_double), ("interface", ctypes.c_int32),
                ("pad3_", ctypes.c_int32), ("acdi_zeta", ctypes.c_double),
                ("acdi_vareps", ctypes.c_double), ("limiter", ctypes.c_int32),
                ("transverse", ctypes.c_int32)]


_lib = None


def lib():
    """Load libsurf.so (built by paper_2605_27534_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsurf.so is not built (%s); run "
                               "`python -m paper_2605_27534_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int
        L.surf_workspace_bytes.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
        L.surf_init.argtypes = [ctypes.POINTER(vp), vp, vp, vp, ctypes.c_size_t, vp]
        L.surf_set_geometry.argtypes = [vp, vp, i32]
        L.surf_set_levelset.argtypes = [vp, vp]
        L.surf_get_levelset.argtypes = [vp, vp]
        L.surf_get_phase.argtypes = [vp, vp]
        L.surf_init_state.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, vp, vp]
        L.surf_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.surf_force.argtypes = [vp, vp, vp]
        L.surf_interface_force.argtypes = [vp, vp, vp, vp, vp]
        L.surf_prepare_geometry.argtypes = [vp, vp, vp]
        L.surf_prepare_phase.argtypes = [vp, vp, vp]
        L.surf_time_transport.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double)]
        L.surf_set_dt.argtypes = [vp, ctypes.c_double]
        L.surf_set_time.argtypes = [vp, vp]
        L.surf_get_status.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
        L.surf_clear_status.argtypes = [vp]
        L.surf_time_solver.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_double)]
        L.surf_time_acdi.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_double)]
        L.surf_solver_iterations.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), i32,
                                             ctypes.POINTER(ctypes.c_int32)]
        L.surf_destroy.argtypes = [vp]
        L.surf_strerror.argtypes = [i32]
        L.surf_strerror.restype = ctypes.c_char_p
        L.surf_version.restype = ctypes.c_char_p
        L.surf_profile_enable.argtypes = [vp, i32]
        d = ctypes.c_double
        L.surf_set_kinetics.argtypes = [vp, d, d, d, d]
        L.surf_loss_weights.argtypes = [vp, vp, ctypes.c_int64, vp, ctypes.c_int32, vp, vp]
        L.surf_adjoint_seed.argtypes = [vp, vp, vp, vp, vp]
        L.surf_adjoint_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.surf_adjoint_c0.argtypes = [vp, vp, vp]
        L.surf_step_advected.argtypes = [vp] * 10
        L.surf_adjoint_step_advected.argtypes = [vp] * 12
        L.surf_profile_read.argtypes = [vp, vp, vp, vp, vp]
        L.surf_step_static.argtypes = [vp, vp, ctypes.c_double, vp, vp, vp, vp, vp, vp, vp, vp,
                                       vp]
        _lib = L
    return _lib


DEFAULTS = dict(flux_form=0, kinetics=0, eos=0, bulk_enabled=1, D_b=1e-2, D_s=1e-3,
                k_a=1.0, k_d=1.0, gamma_inf=1.0, sigma0=1.0, eos_E=0.5, eta=1e-12,
                chi_max_eps=12.0, cfl_adv=0.5, cfl_diff=0.8, hj_iters_init=0,
                hj_iters_step=0, adjoint=0, substep2=0, picard_iters=0, cg_max_iters=0,
                cg_tol=0.0, interface=0, acdi_zeta=0.0, acdi_vareps=0.0, limiter=0,
                bcg_transverse=0)


def make_structs(prob: dict, dt: float, precision: int):
    q = dict(DEFAULTS)
    q.update(prob)
    n = list(q["n"]) + [1] * (3 - len(q["n"]))
    bc = [tuple(b) for b in q.get("bc", ())] + [(0, 0)] * 3
    g = Grid()
    g.dim = q["dim"]
    for d in range(3):
        g.n[d] = int(n[d])
        g.bc[d][0], g.bc[d][1] = bc[d]
    g.h = q["h"]
    g.axisym = int(q.get("axisym", 0))
    org = q.get("origin", (0.0, 0.0, 0.0))
    for d in range(3):
        g.origin[d] = org[d] if d < len(org) else 0.0
    p = Params()
    p.precision = precision
    for k in ("flux_form", "kinetics", "eos", "bulk_enabled", "hj_iters_init", "hj_iters_step",
              "adjoint", "substep2", "picard_iters", "cg_max_iters", "interface"):
        setattr(p, k, int(q[k]))
    for k in ("D_b", "D_s", "k_a", "k_d", "gamma_inf", "sigma0", "eos_E", "eta",
              "chi_max_eps", "cfl_adv", "cfl_diff", "cg_tol", "acdi_zeta", "acdi_vareps"):
        setattr(p, k, float(q[k]))
    p.limiter = int(q["limiter"])
    p.transverse = int(q["bcg_transverse"])
    p.eps = float(q.get("eps", 1.5 * q["h"]))
    p.dt = float(dt)
    return g, p, q


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Surf:
    """One surfactant problem on the current CUDA/HIP device and stream."""

    def __init__(self, prob: dict, dt: float, precision: int = SURF_F32, device="cuda"):
        self.L = lib()
        self.grid, self.params, self.prob = make_structs(prob, dt, precision)
        self.dtype = torch.float64 if precision == SURF_F64 else torch.float32
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        nb = ctypes.c_size_t(0)
        self._check(self.L.surf_workspace_bytes(ctypes.byref(self.grid), ctypes.byref(self.params),
                                                ctypes.byref(nb)), "surf_workspace_bytes")
        self.workspace = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        ws_ptr = self.workspace.data_ptr() + off
        self.stream = torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        self._check(self.L.surf_init(ctypes.byref(ctx), ctypes.byref(self.grid),
                                     ctypes.byref(self.params), ctypes.c_void_p(ws_ptr),
                                     ctypes.c_size_t(int(nb.value)),
                                     ctypes.c_void_p(self.stream.cuda_stream)), "surf_init")
        self.ctx = ctx
        n = list(self.prob["n"]) + [1] * 3
        self.shape = (int(n[2]), int(n[1]), int(n[0]))
        self.dim = int(self.prob["dim"])

    # -- helpers
    def _check(self, rc, what):
        if rc != 0:
            raise SurfError(rc, what)

    def face_shape(self, d):
        s = list(self.shape)
        s[2 - d] += 1
        return tuple(s)

    def empty(self):
        return torch.empty(self.shape, dtype=self.dtype, device=self.device)

    def tensor(self, a):
        return torch.as_tensor(a).to(device=self.device, dtype=self.dtype).contiguous()

    def _cell(self, t, name):
        if t is None:
            return None
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() \
                or tuple(t.shape) != self.shape:
            raise ValueError("%s: expected contiguous %s %s on %s" % (name, self.dtype, self.shape,
                                                                    self.device))
        return t

    def _faces(self, u, name):
        if u is None:
            return None
        for d in range(self.dim):
            t = u[d]
            if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() \
                    or tuple(t.shape) != self.face_shape(d):
                raise ValueError("%s[%d]: expected contiguous %s %s" % (name, d, self.dtype,
                                                                       self.face_shape(d)))
        arr = (ctypes.c_void_p * 3)(*[u[d].data_ptr() if d < self.dim else None for d in range(3)])
        return arr

    # -- API
    def set_geometry(self, vof, full=True):
        self._check(self.L.surf_set_geometry(self.ctx, _ptr(self._cell(vof, "vof")), int(full)),
                    "surf_set_geometry")

    def set_levelset(self, chi):
        self._check(self.L.surf_set_levelset(self.ctx, _ptr(self._cell(chi, "chi"))),
                    "surf_set_levelset")

    def phase(self):
        """The ACDI phase field phi (ACDI contexts)."""
        out = self.empty()
        self._check(self.L.surf_get_phase(self.ctx, _ptr(out)), "surf_get_phase")
        return out

    def levelset(self):
        out = self.empty()
        self._check(self.L.surf_get_levelset(self.ctx, _ptr(out)), "surf_get_levelset")
        return out

    def init_state(self, c0=None, c0_const=1.0, gamma0=0.0):
        F = self.empty() if self.params.bulk_enabled else None
        psi = self.empty()
        self._check(self.L.surf_init_state(self.ctx, _ptr(self._cell(c0, "c0")),
                                           float(c0_const), float(gamma0), _ptr(F), _ptr(psi)),
                    "surf_init_state")
        return F, psi

    def step(self, F_in, psi_in, F_out, psi_out, u=None, vof_next=None, sigma_out=None,
             totals=None, star=None):
        """One step; with star = (F_star, psi_star) (static level set only) the
        advected state of the step is written there too."""
        ua = self._faces(u, "u")
        if totals is not None and (totals.dtype != torch.float64 or totals.numel() < 16
                                   or totals.device != self.device):
            raise ValueError("totals: 16 float64 on the device")
        if star is not None:
            if vof_next is not None:
                raise ValueError("star: static level set only")
            self._check(self.L.surf_step_advected(
                self.ctx, ua, _ptr(self._cell(F_in, "F_in")), _ptr(self._cell(psi_in, "psi_in")),
                _ptr(self._cell(F_out, "F_out")), _ptr(self._cell(psi_out, "psi_out")),
                _ptr(self._cell(sigma_out, "sigma_out")), _ptr(totals),
                _ptr(self._cell(star[0], "F_star")), _ptr(self._cell(star[1], "psi_star"))),
                "surf_step_advected")
            return
        self._check(self.L.surf_step(self.ctx, _ptr(self._cell(vof_next, "vof_next")), ua,
                                     _ptr(self._cell(F_in, "F_in")),
                                     _ptr(self._cell(psi_in, "psi_in")),
                                     _ptr(self._cell(F_out, "F_out")),
                                     _ptr(self._cell(psi_out, "psi_out")),
                                     _ptr(self._cell(sigma_out, "sigma_out")), _ptr(totals)),
                    "surf_step")

    def prepare_geometry(self, vof_next, stream):
        """Enqueues the next step's geometry on `stream` (a torch stream other
        than the context's); the next step() must get the same vof_next."""
        self._check(self.L.surf_prepare_geometry(self.ctx, _ptr(self._cell(vof_next, "vof_next")),
                                                 ctypes.c_void_p(stream.cuda_stream)),
                    "surf_prepare_geometry")

    def prepare_phase(self, u, stream):
        """ACDI: enqueues the next step's ACDI step on `stream` (a torch stream
        other than the context's); the next step() gets vof_next=None and
        the same u."""
        self._check(self.L.surf_prepare_phase(self.ctx, self._faces(u, "u"),
                                              ctypes.c_void_p(stream.cuda_stream)),
                    "surf_prepare_phase")

    def time_transport(self, F_in, psi_in, F_out, psi_out, u=None, sigma_out=None, reps=100):
        """Mean milliseconds of one transport-kernel launch over `reps`
        back-to-back launches (outputs overwritten; state untouched)."""
        ua = self._faces(u, "u")
        ms = ctypes.c_double(0.0)
        self._check(self.L.surf_time_transport(self.ctx, ua, _ptr(self._cell(F_in, "F_in")),
                                               _ptr(self._cell(psi_in, "psi_in")),
                                               _ptr(self._cell(F_out, "F_out")),
                                               _ptr(self._cell(psi_out, "psi_out")),
                                               _ptr(self._cell(sigma_out, "sigma_out")),
                                               int(reps), ctypes.byref(ms)),
                    "surf_time_transport")
        return ms.value

    def force(self, sigma, out=None):
        if out is None:
            out = [torch.empty(self.face_shape(d), dtype=self.dtype, device=self.device)
                   for d in range(self.dim)]
        arr = (ctypes.c_void_p * 3)(*[out[d].data_ptr() if d < self.dim else None
                                      for d in range(3)])
        self._check(self.L.surf_force(self.ctx, _ptr(self._cell(sigma, "sigma")), arr),
                    "surf_force")
        return out

    def interface_force(self, vof, sigma, cap=True, ma=True, out=None):
        """(capillary [fx, fy(, fz)], Marangoni [fx, fy(, fz)]) on the faces;
        a set not asked for is None.  `out` = (cap, ma) reuses caller arrays."""
        if out is None:
            mk = lambda: [torch.empty(self.face_shape(d), dtype=self.dtype, device=self.device)
                          for d in range(self.dim)]
            out = (mk() if cap else None, mk() if ma else None)
        arrs = [None if o is None else self._faces(o, "force") for o in out]
        self._check(self.L.surf_interface_force(self.ctx, _ptr(self._cell(vof, "vof")),
                                                _ptr(self._cell(sigma, "sigma")), arrs[0],
                                                arrs[1]),
                    "surf_interface_force")
        return out

    def set_dt(self, dt):
        self._check(self.L.surf_set_dt(self.ctx, float(dt)), "surf_set_dt")

    def set_time(self, t=None):
        """Running time from a one-element float64 device tensor (None: 0)."""
        if t is not None and (t.dtype != torch.float64 or t.device != self.device):
            raise ValueError("time: a float64 device tensor")
        self._check(self.L.surf_set_time(self.ctx, _ptr(t)), "surf_set_time")

    def status(self):
        b = ctypes.c_uint32(0)
        self._check(self.L.surf_get_status(self.ctx, ctypes.byref(b)), "surf_get_status")
        return int(b.value)

    def clear_status(self):
        self._check(self.L.surf_clear_status(self.ctx), "surf_clear_status")

    def time_acdi(self, u=None, reps=100):
        """Mean ms of one ACDI step (both kernels), the state unchanged."""
        ms = ctypes.c_double(0.0)
        self._check(self.L.surf_time_acdi(self.ctx, self._faces(u, "u"), int(reps), ctypes.byref(ms)),
                    "surf_time_acdi")
        return ms.value

    def time_solver(self, field, reps):
        """Mean ms of one CG iteration launch (implicit contexts)."""
        ms = ctypes.c_double(0.0)
        self._check(self.L.surf_time_solver(self.ctx, int(field), int(reps), ctypes.byref(ms)),
                    "surf_time_solver")
        return ms.value

    def solver_iterations(self):
        """CG iterations of each linear solve of the last implicit step."""
        buf = (ctypes.c_int32 * 64)()
        n = ctypes.c_int32(0)
        self._check(self.L.surf_solver_iterations(self.ctx, buf, 64, ctypes.byref(n)),
                    "surf_solver_iterations")
        return [int(buf[i]) for i in range(n.value)]

    # -- adjoint
    def set_kinetics(self, k_a, k_d, D_b, D_s):
        self._check(self.L.surf_set_kinetics(self.ctx, float(k_a), float(k_d), float(D_b),
                                             float(D_s)), "surf_set_kinetics")

    def loss_weights(self, totals_hist, target, w_out, loss_out=None):
        n = int(target.numel())
        self._check(self.L.surf_loss_weights(self.ctx, _ptr(totals_hist),
                                             ctypes.c_int64(totals_hist.stride(0)),
                                             _ptr(target), ctypes.c_int32(n), _ptr(w_out),
                                             _ptr(loss_out)), "surf_loss_weights")

    def adjoint_seed(self, psi, w, lamF, lamP):
        self._check(self.L.surf_adjoint_seed(self.ctx, _ptr(self._cell(psi, "psi")), _ptr(w),
                                             _ptr(self._cell(lamF, "lamF")),
                                             _ptr(self._cell(lamP, "lamP"))), "surf_adjoint_seed")

    def adjoint_step(self, F, psi, mF, mP, lF, lP, dtheta, u=None, w=None, star=None):
        """lambda^n from lambda^{n+1} = (mF, mP); star = (F_star, psi_star) from
        step(..., star=...) on the same state skips the advection's
        recomputation."""
        ua = self._faces(u, "u")
        if star is not None:
            self._check(self.L.surf_adjoint_step_advected(
                self.ctx, ua, _ptr(self._cell(F, "F")), _ptr(self._cell(psi, "psi")),
                _ptr(self._cell(star[0], "F_star")), _ptr(self._cell(star[1], "psi_star")),
                _ptr(self._cell(mF, "mF")), _ptr(self._cell(mP, "mP")), _ptr(w),
                _ptr(self._cell(lF, "lF")), _ptr(self._cell(lP, "lP")), _ptr(dtheta)),
                "surf_adjoint_step_advected")
            return
        self._check(self.L.surf_adjoint_step(self.ctx, ua, _ptr(self._cell(F, "F")),
                                             _ptr(self._cell(psi, "psi")),
                                             _ptr(self._cell(mF, "mF")), _ptr(self._cell(mP, "mP")),
                                             _ptr(w), _ptr(self._cell(lF, "lF")),
                                             _ptr(self._cell(lP, "lP")), _ptr(dtheta)),
                    "surf_adjoint_step")

    def adjoint_c0(self, lF0):
        out = self.empty()
        self._check(self.L.surf_adjoint_c0(self.ctx, _ptr(self._cell(lF0, "lF0")), _ptr(out)),
                    "surf_adjoint_c0")
        return out

    def profile(self, enable=True):
        self._check(self.L.surf_profile_enable(self.ctx, int(enable)), "surf_profile_enable")

    def profile_read(self):
        """(transport ms, transport launches, redistancing ms, sweeps)."""
        a, c = ctypes.c_double(0), ctypes.c_double(0)
        b, d = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self.L.surf_profile_read(self.ctx, ctypes.byref(a), ctypes.byref(b),
                                             ctypes.byref(c), ctypes.byref(d)),
                    "surf_profile_read")
        return a.value, b.value, c.value, d.value

    def close(self):
        if getattr(self, "ctx", None):
            self.L.surf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, F, psi, nsteps, u=None, vof_seq=None, sigma=None, totals_hist=None):
        """nsteps steps with ping-pong buffers; returns (F, psi, sigma).
        vof_seq(n) gives the VoF at t^{n+1} (device tensor) or None.
        totals_hist: float64 device tensor [nsteps, 16] or None."""
        F2 = self.empty() if F is not None else None
        P2 = self.empty()
        S = sigma if sigma is not None else self.empty()
        for n in range(nsteps):
            v = vof_seq(n) if vof_seq is not None else None
            tot = totals_hist[n] if totals_hist is not None else None
            self.step(F, psi, F2, P2, u=u, vof_next=v, sigma_out=S, totals=tot)
            F, F2 = F2, F
            psi, P2 = P2, psi
        return F, psi, S


def step_static(prob: dict, dt: float, precision: int, chi, F_in, psi_in, F_out, psi_out,
                u=None, sigma_out=None, totals=None, stream=None):
    """surf_step_static: one step with no context and no workspace (the
    library's file-scope device array holds the reduction records).  Tensors
    are device buffers of the problem's precision; totals (16 float64) is
    read for the running time and outflow and rewritten.  Returns the
    library's return code (0 on success)."""
    L = lib()
    g, p, _ = make_structs(prob, dt, precision)
    ua = None
    if u is not None:
        arr = (ctypes.c_void_p * 3)(*([ctypes.c_void_p(x.data_ptr()) for x in u] +
                                      [None] * (3 - len(u))))
        ua = ctypes.cast(arr, ctypes.c_void_p)
    st = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    return int(L.surf_step_static(ctypes.byref(g), ctypes.byref(p), float(dt), _ptr(chi), ua,
                                  _ptr(F_in), _ptr(psi_in), _ptr(F_out), _ptr(psi_out),
                                  _ptr(sigma_out), _ptr(totals), ctypes.c_void_p(st)))
