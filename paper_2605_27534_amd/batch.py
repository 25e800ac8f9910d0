"""Python binding of libsurf's batched form (surf_batch_* in include/surf.h):
many independent static-interface 2D problems of different sizes advanced by
one persistent kernel launch per step and one HIP graph per call.

Argument marshalling only: the geometry build, the initial state, every step
and every per-instance total are libsurf kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import surf as S

BATCH_EXPORTS = [
    "surf_batch_workspace_bytes", "surf_batch_create", "surf_batch_set_geometry",
    "surf_batch_init_state", "surf_batch_step", "surf_batch_parity", "surf_batch_tune",
    "surf_batch_destroy",
]


def _bind(L):
    if getattr(L, "_batch_bound", False):
        return L
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    L.surf_batch_workspace_bytes.argtypes = [i32, vp, vp, ctypes.POINTER(ctypes.c_size_t)]
    L.surf_batch_create.argtypes = [ctypes.POINTER(vp), i32, vp, vp, vp, vp, vp, vp,
                                    ctypes.c_size_t, vp]
    L.surf_batch_set_geometry.argtypes = [vp, i32, vp]
    L.surf_batch_init_state.argtypes = [vp, i32, vp, ctypes.c_double, ctypes.c_double]
    L.surf_batch_step.argtypes = [vp, i32, vp]
    L.surf_batch_parity.argtypes = [vp]
    L.surf_batch_tune.argtypes = [vp, ctypes.POINTER(i32), vp, i32]
    L.surf_batch_destroy.argtypes = [vp]
    L._batch_bound = True
    return L


class Batch:
    """probs: list of problem dicts (2D, one precision), dts: per-instance dt.

    The state of instance i lives in F[i][parity], psi[i][parity] (two
    buffers each); `state(i)` returns the current pair."""

    def __init__(self, probs, dts, precision=S.SURF_F32, device="cuda", sigma=True):
        self.L = _bind(S.lib())
        n = len(probs)
        self.n = n
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.dtype = torch.float64 if precision == S.SURF_F64 else torch.float32
        grids = (S.Grid * n)()
        params = (S.Params * n)()
        self.shapes = []
        for i, (p, dt) in enumerate(zip(probs, dts)):
            g, q, full = S.make_structs(p, dt, precision)
            grids[i] = g
            params[i] = q
            self.shapes.append((1, int(full["n"][1]), int(full["n"][0])))
        self.grids, self.params = grids, params
        nb = ctypes.c_size_t(0)
        self._check(self.L.surf_batch_workspace_bytes(n, grids, params, ctypes.byref(nb)),
                    "surf_batch_workspace_bytes")
        self.workspace = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=dev)
        ws = self.workspace.data_ptr() + (-self.workspace.data_ptr()) % 256
        self.F = [[torch.zeros(s, dtype=self.dtype, device=dev) for _ in range(2)]
                  for s in self.shapes]
        self.P = [[torch.zeros(s, dtype=self.dtype, device=dev) for _ in range(2)]
                  for s in self.shapes]
        self.sigma = [torch.zeros(s, dtype=self.dtype, device=dev) for s in self.shapes] \
            if sigma else None
        Fp = (ctypes.c_void_p * (2 * n))(*[t.data_ptr() for pair in self.F for t in pair])
        Pp = (ctypes.c_void_p * (2 * n))(*[t.data_ptr() for pair in self.P for t in pair])
        Sp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.sigma]) if sigma else None
        self.stream = torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        self._check(self.L.surf_batch_create(ctypes.byref(h), n, grids, params, Fp, Pp, Sp,
                                             ctypes.c_void_p(ws), ctypes.c_size_t(int(nb.value)),
                                             ctypes.c_void_p(self.stream.cuda_stream)),
                    "surf_batch_create")
        self.h = h

    def _check(self, rc, what):
        if rc != 0:
            raise S.SurfError(rc, what)

    def _cell(self, i, t, name):
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() \
                or tuple(t.shape) != self.shapes[i]:
            raise ValueError("%s: expected contiguous %s %s" % (name, self.dtype, self.shapes[i]))
        return t

    def set_geometry(self, i, vof):
        vof = self._cell(i, vof, "vof")
        self._check(self.L.surf_batch_set_geometry(self.h, i, ctypes.c_void_p(vof.data_ptr())),
                    "surf_batch_set_geometry")

    def init_state(self, i, c0=None, c0_const=1.0, gamma0=0.0):
        p = None if c0 is None else ctypes.c_void_p(self._cell(i, c0, "c0").data_ptr())
        self._check(self.L.surf_batch_init_state(self.h, i, p, float(c0_const), float(gamma0)),
                    "surf_batch_init_state")

    def step(self, nsteps=1, totals=None):
        """Advance every instance nsteps steps; totals [n, 16] float64 receives
        each instance's totals of the last step."""
        if totals is not None:
            if totals.dtype != torch.float64 or tuple(totals.shape) != (self.n, 16) \
                    or not totals.is_contiguous() or totals.device != self.device:
                raise ValueError("totals: expected contiguous float64 [%d, 16]" % self.n)
        p = None if totals is None else ctypes.c_void_p(totals.data_ptr())
        self._check(self.L.surf_batch_step(self.h, int(nsteps), p), "surf_batch_step")

    @property
    def parity(self):
        return int(self.L.surf_batch_parity(self.h))

    def state(self, i):
        k = self.parity
        return self.F[i][k], self.P[i][k]

    def tune(self):
        choice = ctypes.c_int32(-1)
        times = (ctypes.c_double * 16)()
        self._check(self.L.surf_batch_tune(self.h, ctypes.byref(choice), times, 16),
                    "surf_batch_tune")
        return int(choice.value), list(times)

    def close(self):
        if getattr(self, "h", None):
            self.L.surf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
