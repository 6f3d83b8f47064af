"""Python binding of the building-cube projection library (argument marshalling only).

Every step of the path runs in the HIP kernels of libbcm.so; torch provides device memory
(fields and the workspace) and the stream.  Names follow include/bcm.h.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L


class BCMError(RuntimeError):
    def __init__(self, status, where):
        lib = L.load()
        msg = lib.bcm_last_error().decode(errors="replace")
        name = lib.bcm_status_string(status).decode()
        super().__init__(f"{where}: {name} ({status}): {msg}")
        self.status = status


def _check(status, where, allow_warning=True):
    if status < 0 or (status > 0 and not allow_warning):
        raise BCMError(status, where)
    return status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mesh:
    """A validated building-cube mesh (host copy inside the library).

    Accepts any object with the attributes n, root_edge, origin [n_c,3] float64, level [n_c]
    int8, nbr [n_c,6,4] int32, face_bc [n_c,6] int8 (for example bcm_inputs.Mesh)."""

    def __init__(self, desc):
        self._lib = L.load()
        self.n = int(desc.n)
        self.n_cubes = int(desc.origin.shape[0])
        self.n_cells = self.n_cubes * self.n ** 3
        self._origin = np.ascontiguousarray(desc.origin, dtype=np.float64)
        self._level = np.ascontiguousarray(desc.level, dtype=np.int8)
        self._nbr = np.ascontiguousarray(desc.nbr, dtype=np.int32)
        self._face_bc = np.ascontiguousarray(desc.face_bc, dtype=np.int8)
        d = L.MeshDesc(self.n_cubes, self.n,
                       self._origin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       self._level.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                       float(desc.root_edge),
                       self._nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                       self._face_bc.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
        h = ctypes.c_void_p()
        _check(self._lib.bcm_mesh_create(ctypes.byref(d), ctypes.byref(h)), "bcm_mesh_create",
               allow_warning=False)
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.bcm_mesh_destroy(self.handle)
            self.handle = None


@dataclass
class SolveReport:
    status: int
    n_outer: int
    n_inner: int
    final_rel_res: float
    history: list = field(default_factory=list)


def _report(cap=4096):
    hist = (ctypes.c_double * cap)()
    r = L.Report(0, 0, 0, 0.0, ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)), cap, 0)
    return r, hist


def _unpack(r, hist):
    return SolveReport(r.status, r.n_outer, r.n_inner, r.final_rel_res,
                       [hist[i] for i in range(r.history_len)])


def default_opts():
    o = L.SolverOpts()
    L.load().bcm_default_opts(ctypes.byref(o))
    return o


class Plan:
    """Solver plan bound to a torch-allocated device workspace.

    precision: "fp64", "mixed" or "mixed_f32fields"; other keyword arguments override the
    fields of bcm_solver_opts (tol, max_iter, max_outer, inner_tol, pre_sweeps, post_sweeps,
    coarse_iters, krylov, coarse_solver, coarse_cycles, graph_split, prolong, check_every)."""

    def __init__(self, mesh: Mesh, precision="fp64", device="cuda", **opts):
        self._lib = L.load()
        self.mesh = mesh
        o = default_opts()
        o.precision = L.PRECISIONS[precision]
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown solver option {k}")
            setattr(o, k, v)
        self.opts = o
        self.precision = precision
        self.field_dtype = torch.float32 if precision == "mixed_f32fields" else torch.float64
        h = ctypes.c_void_p()
        nbytes = ctypes.c_size_t()
        _check(self._lib.bcm_plan_create(mesh.handle, ctypes.byref(o), ctypes.byref(h),
                                         ctypes.byref(nbytes)), "bcm_plan_create",
               allow_warning=False)
        self.handle = h
        self.workspace_bytes = nbytes.value
        self.device = torch.device(device)
        self.workspace = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8,
                                     device=self.device)
        _check(self._lib.bcm_plan_bind(self.handle, _ptr(self.workspace), self.workspace_bytes,
                                       _stream()), "bcm_plan_bind", allow_warning=False)

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.bcm_plan_destroy(self.handle)
            self.handle = None

    # -- helpers -----------------------------------------------------------------------------
    def _field(self, t, name, dtype=None):
        dtype = dtype or self.field_dtype
        if t is None:
            return None
        if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()
                and t.numel() == self.mesh.n_cells):
            raise ValueError(f"{name}: expected a contiguous {dtype} CUDA tensor of "
                             f"{self.mesh.n_cells} values")
        return t

    def empty(self, dtype=None):
        return torch.empty(self.mesh.n_cells, dtype=dtype or self.field_dtype,
                           device=self.device)

    def _face_shape(self, d):
        n = self.mesh.n
        return self.mesh.n_cubes * (n + 1) * n * n

    # -- entry points --------------------------------------------------------------------------
    def project(self, u, alpha, U_in, dt, rho, us=(0.0, 0.0, 0.0), p0=None, face_u=False,
                out=None, history=4096, want_b=False):
        """One projection step; returns dict(u_new=[3], p, report, face_u=[3] or None,
        b = the solved Poisson right-hand side or None)."""
        u = [self._field(x, f"u[{d}]") for d, x in enumerate(u)]
        alpha = self._field(alpha, "alpha")
        us_t = [self._field(x, "us") if torch.is_tensor(x) else None for x in us]
        usc = [0.0 if torch.is_tensor(x) else float(x) for x in us]
        if out is None:
            out = dict(u_new=[self.empty() for _ in range(3)],
                       p=self.empty(torch.float64))
        p0 = self._field(p0, "p0", torch.float64)
        fu = [torch.empty(self._face_shape(d), dtype=self.field_dtype, device=self.device)
              for d in range(3)] if face_u else [None] * 3
        pin = L.ProjectIn((ctypes.c_void_p * 3)(*[x.data_ptr() for x in u]), _ptr(alpha).value,
                          (ctypes.c_void_p * 3)(*[t.data_ptr() if t is not None else None
                                                  for t in us_t]),
                          (ctypes.c_double * 3)(*usc), float(U_in), float(dt), float(rho),
                          _ptr(p0).value)
        b = self.empty(torch.float64) if want_b else None
        pout = L.ProjectOut((ctypes.c_void_p * 3)(*[x.data_ptr() for x in out["u_new"]]),
                            out["p"].data_ptr(),
                            (ctypes.c_void_p * 3)(*[t.data_ptr() if t is not None else None
                                                    for t in fu]), _ptr(b).value)
        rep, hist = _report(history)
        st = self._lib.bcm_project(self.handle, ctypes.byref(pin), ctypes.byref(pout),
                                   ctypes.byref(rep), _stream())
        _check(st, "bcm_project")
        out = dict(out)
        out["report"] = _unpack(rep, hist)
        out["face_u"] = fu if face_u else None
        out["b"] = b
        return out

    def project_recompute(self, u, alpha, p, U_in, dt, rho, us=(0.0, 0.0, 0.0), out=None):
        """Forcing + correction with a given pressure (no solve); returns u_new [3]."""
        u = [self._field(x, f"u[{d}]") for d, x in enumerate(u)]
        alpha = self._field(alpha, "alpha")
        p = self._field(p, "p", torch.float64)
        us_t = [self._field(x, "us") if torch.is_tensor(x) else None for x in us]
        usc = [0.0 if torch.is_tensor(x) else float(x) for x in us]
        out = out or [self.empty() for _ in range(3)]
        pin = L.ProjectIn((ctypes.c_void_p * 3)(*[x.data_ptr() for x in u]), _ptr(alpha).value,
                          (ctypes.c_void_p * 3)(*[t.data_ptr() if t is not None else None
                                                  for t in us_t]),
                          (ctypes.c_double * 3)(*usc), float(U_in), float(dt), float(rho), None)
        pout = L.ProjectOut((ctypes.c_void_p * 3)(*[x.data_ptr() for x in out]), None,
                            (ctypes.c_void_p * 3)(None, None, None))
        _check(self._lib.bcm_project_recompute(self.handle, ctypes.byref(pin), _ptr(p),
                                               ctypes.byref(pout), _stream()),
               "bcm_project_recompute", allow_warning=False)
        return out

    def project_adjoint(self, u, alpha, g_u_new, U_in, dt, rho, us=(0.0, 0.0, 0.0), g_p=None,
                        want_lambda=False, history=4096, g_alpha=None, g_U_in=0.0,
                        accumulate=False):
        """Reverse-mode derivative of project; returns (g_u [3], g_alpha, g_U_in, report,
        lambda or None).  With accumulate=True the step's cotangents of alpha and U_in are
        added (in the library) to the given g_alpha field and g_U_in value."""
        u = [self._field(x, f"u[{d}]") for d, x in enumerate(u)]
        alpha = self._field(alpha, "alpha")
        g = [self._field(x, f"g_u_new[{d}]") for d, x in enumerate(g_u_new)]
        g_p = self._field(g_p, "g_p", torch.float64)
        us_t = [self._field(x, "us") if torch.is_tensor(x) else None for x in us]
        usc = [0.0 if torch.is_tensor(x) else float(x) for x in us]
        g_u = [self.empty() for _ in range(3)]
        if alpha is None:
            g_alpha = None
        elif g_alpha is None:
            if accumulate:
                raise ValueError("accumulate=True needs the g_alpha field to add to")
            g_alpha = self.empty()
        else:
            g_alpha = self._field(g_alpha, "g_alpha")
        lam = self.empty(torch.float64) if want_lambda else None
        ain = L.AdjointIn((ctypes.c_void_p * 3)(*[x.data_ptr() for x in u]), _ptr(alpha).value,
                          (ctypes.c_void_p * 3)(*[t.data_ptr() if t is not None else None
                                                  for t in us_t]),
                          (ctypes.c_double * 3)(*usc), float(U_in), float(dt), float(rho),
                          (ctypes.c_void_p * 3)(*[x.data_ptr() for x in g]), _ptr(g_p).value)
        aout = L.AdjointOut((ctypes.c_void_p * 3)(*[x.data_ptr() for x in g_u]),
                            _ptr(g_alpha).value, float(g_U_in) if accumulate else 0.0,
                            _ptr(lam).value, 1 if accumulate else 0)
        rep, hist = _report(history)
        st = self._lib.bcm_project_adjoint(self.handle, ctypes.byref(ain), ctypes.byref(aout),
                                           ctypes.byref(rep), _stream())
        _check(st, "bcm_project_adjoint")
        return g_u, g_alpha, float(aout.g_U_in), _unpack(rep, hist), lam

    def momentum(self, u, U_in, dt, nu, scheme="cn", h_prev=None, want_h=False, cn_tol=0.0,
                 cn_max_iter=0, out=None, history=4096):
        """Momentum sub-step u^n -> u~ (scheme "euler", "ab2" or "cn"); returns dict(u_tilde=[3],
        h=[3] = H(u^n) or None, report)."""
        u = [self._field(x, f"u[{d}]") for d, x in enumerate(u)]
        hp = [self._field(x, f"h_prev[{d}]") for d, x in enumerate(h_prev)] if h_prev else None
        ut = out or [self.empty() for _ in range(3)]
        h = [self.empty() for _ in range(3)] if want_h else None
        mi = L.MomentumIn((ctypes.c_void_p * 3)(*[x.data_ptr() for x in u]),
                          (ctypes.c_void_p * 3)(*([x.data_ptr() for x in hp] if hp else
                                                  [None] * 3)),
                          float(U_in), float(dt), float(nu), L.SCHEMES[scheme], float(cn_tol),
                          int(cn_max_iter))
        mo = L.MomentumOut((ctypes.c_void_p * 3)(*[x.data_ptr() for x in ut]),
                           (ctypes.c_void_p * 3)(*([x.data_ptr() for x in h] if h else
                                                   [None] * 3)))
        rep, hist = _report(history)
        st = self._lib.bcm_momentum(self.handle, ctypes.byref(mi), ctypes.byref(mo),
                                    ctypes.byref(rep), _stream())
        _check(st, "bcm_momentum")
        return dict(u_tilde=ut, h=h, report=_unpack(rep, hist))

    def ib_force(self, u, X, dt, rho, dV=None, Us=(0.0, 0.0, 0.0), want_UF=False, out=None):
        """Lagrangian-particle forcing u~ -> u*; X, dV, Us: contiguous device float64 tensors
        (3n, n and 3n values, particle-major) or Us a constant triple.  Returns dict(u_star=[3], U_p, F_p ([n, 3] or None))."""
        u = [self._field(x, f"u[{d}]") for d, x in enumerate(u)]
        n = int(X.numel()) // 3 if X is not None else 0
        if X is not None and X.numel() != 3 * n:
            raise ValueError("X: expected 3 coordinates per particle")
        for t, name in ((X, "X"), (dV, "dV")) + (((Us, "Us"),) if torch.is_tensor(Us) else ()):
            if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError(f"{name}: expected a contiguous float64 CUDA tensor")
        usc = (0.0, 0.0, 0.0) if torch.is_tensor(Us) else tuple(float(v) for v in Us)
        pt = L.Particles(n, _ptr(X).value, _ptr(dV).value,
                         _ptr(Us).value if torch.is_tensor(Us) else None,
                         (ctypes.c_double * 3)(*usc))
        us = out or [self.empty() for _ in range(3)]
        Up = torch.empty((n, 3), dtype=torch.float64, device=self.device) if want_UF else None
        Fp = torch.empty((n, 3), dtype=torch.float64, device=self.device) if want_UF else None
        st = self._lib.bcm_ib_force(self.handle, ctypes.byref(pt),
                                    (ctypes.c_void_p * 3)(*[x.data_ptr() for x in u]),
                                    (ctypes.c_void_p * 3)(*[x.data_ptr() for x in us]),
                                    float(dt), float(rho), _ptr(Up), _ptr(Fp), _stream())
        _check(st, "bcm_ib_force", allow_warning=False)
        return dict(u_star=us, U_p=Up, F_p=Fp)

    def compress_bound(self):
        """Worst-case size in bytes of a compressed field of this mesh."""
        bound = ctypes.c_size_t()
        _check(self._lib.bcm_compress_bound(self.handle, ctypes.byref(bound)),
               "bcm_compress_bound", allow_warning=False)
        return bound.value

    def compress(self, field, step, out=None):
        """Wavelet-compress an FP64 cell field; returns the stream as a device uint8 tensor (a
        view of `out` when given, else of a buffer of the worst-case size)."""
        field = self._field(field, "field", torch.float64)
        buf = out if out is not None else torch.empty(self.compress_bound(), dtype=torch.uint8,
                                                      device=self.device)
        n = ctypes.c_size_t()
        _check(self._lib.bcm_compress(self.handle, _ptr(field), float(step), _ptr(buf),
                                      buf.numel(), ctypes.byref(n), _stream()),
               "bcm_compress", allow_warning=False)
        return buf[:n.value]

    def decompress(self, stream, out=None):
        """Decode a stream (device uint8 tensor) into an FP64 cell field."""
        out = self.empty(torch.float64) if out is None else self._field(out, "out", torch.float64)
        _check(self._lib.bcm_decompress(self.handle, _ptr(stream), stream.numel(), _ptr(out),
                                        _stream()), "bcm_decompress", allow_warning=False)
        return out

    def kinetic_energy(self, u, rho, g_scale=None, want_J=True):
        """J = (rho/2) sum_i V_i |u_i|^2 (host float, or None with want_J=False) and, when
        g_scale is given, the seed cotangent g_scale * rho * V * u (three fields; else None)."""
        u = [self._field(x, f"u[{d}]") for d, x in enumerate(u)]
        seed = [self.empty() for _ in range(3)] if g_scale is not None else None
        J = ctypes.c_double(0.0)
        st = self._lib.bcm_kinetic_energy(
            self.handle, (ctypes.c_void_p * 3)(*[x.data_ptr() for x in u]), float(rho),
            float(g_scale) if g_scale is not None else 0.0,
            ctypes.byref(J) if want_J else None,
            (ctypes.c_void_p * 3)(*[x.data_ptr() for x in seed]) if seed else None, _stream())
        _check(st, "bcm_kinetic_energy", allow_warning=False)
        return (J.value if want_J else None), seed

    def poisson_solve(self, b, p=None, use_guess=False, history=4096):
        """Solve A p = b (FP64 fields); returns (p, report)."""
        b = self._field(b, "b", torch.float64)
        p = self.empty(torch.float64) if p is None else self._field(p, "p", torch.float64)
        rep, hist = _report(history)
        st = self._lib.bcm_poisson_solve(self.handle, _ptr(b), _ptr(p), int(bool(use_guess)),
                                         ctypes.byref(rep), _stream())
        _check(st, "bcm_poisson_solve")
        return p, _unpack(rep, hist)

    def apply_laplacian(self, p, out=None):
        p = self._field(p, "p", torch.float64)
        out = self.empty(torch.float64) if out is None else out
        _check(self._lib.bcm_apply_laplacian(self.handle, _ptr(p), _ptr(out), _stream()),
               "bcm_apply_laplacian", allow_warning=False)
        return out

    def timing_enable(self, kernel_class, every=1):
        """Time launches of a kernel class with HIP events (None: off); every > 1 times only
        one launch in each run of `every`, which keeps the events' own stream stalls out of
        the rest of a timed region."""
        _check(self._lib.bcm_timing_enable(
            self.handle, kernel_class.encode() if kernel_class else None),
            "bcm_timing_enable", allow_warning=False)
        if kernel_class and every != 1:
            _check(self._lib.bcm_timing_sample(self.handle, int(every)),
                   "bcm_timing_sample", allow_warning=False)

    def timing_read(self):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(self._lib.bcm_timing_read(self.handle, ctypes.byref(n), ctypes.byref(ms)),
               "bcm_timing_read", allow_warning=False)
        return int(n.value), float(ms.value)


def timing_names():
    lib = L.load()
    out, i = [], 0
    while True:
        s = lib.bcm_timing_name(i)
        if not s:
            return out
        out.append(s.decode())
        i += 1
