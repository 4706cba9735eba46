"""Python binding of the tpt library (tensor-product--Thomas direct solver for
constant-coefficient Poisson/Helmholtz equations on stretched staggered grids,
arXiv 2603.09528 §2.2, on one MI355X).

Argument marshalling only: every step of a solve runs in the HIP kernels of
``libtpt.so`` (built in-tree by ``python -m paper_2603_09528_amd.build``).
PyTorch supplies device memory and streams; fields are float64 CUDA tensors
of shape (Nz, Ny, Nx) (x fastest), or (nrhs, Nz, Ny, Nx).

Boundary conditions per direction are pairs of 'P' (periodic), 'N'
(Neumann) or 'D' (Dirichlet); locations are 'C' (cell centre) or 'F' (face).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpt.so")

FP64, MIXED_FP32, MIXED_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": MIXED_FP32, "bf16x3": MIXED_BF16X3}
_BC = {"P": 0, "N": 1, "D": 2}
_LOC = {"C": 0, "F": 1}
_KIND = {"poisson": 0, "helmholtz": 1}
_IMPLICIT = {"xyz": 0, "yz": 1, "z": 2}
OK, PENDING = 0, 1


class TptError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tpt error {code}: {msg}")
        self.code = code


class _Desc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3),
        ("faces", ctypes.POINTER(ctypes.c_double) * 3),
        ("bc", (ctypes.c_int * 2) * 3),
        ("loc", ctypes.c_int * 3),
        ("kind", ctypes.c_int),
        ("alpha", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("rtol", ctypes.c_double),
        ("max_refine", ctypes.c_int),
        ("fixed_refine", ctypes.c_int),
        ("nrhs", ctypes.c_int),
        ("flags", ctypes.c_int),
        ("implicit", ctypes.c_int),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("rel_correction", ctypes.c_double),
        ("rel_residual", ctypes.c_double),
        ("null_line", ctypes.c_int),
        ("compat_defect", ctypes.c_double),
        ("nonfinite", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded libtpt.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_09528_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        dp = ctypes.POINTER(ctypes.c_double)
        sig = {
            "tpt_plan_desc_init": (None, [ctypes.POINTER(_Desc)]),
            "tpt_plan_create": (i, [ctypes.POINTER(_Desc), ctypes.POINTER(vp)]),
            "tpt_plan_destroy": (i, [vp]),
            "tpt_plan_shape": (i, [vp, ctypes.POINTER(ctypes.c_int)]),
            "tpt_plan_workspace_bytes": (i, [vp, ctypes.POINTER(sz)]),
            "tpt_plan_eigen": (i, [vp, i, dp, dp]),
            "tpt_plan_operator": (i, [vp, i, dp, dp, dp, dp]),
            "tpt_plan_transforms": (i, [vp, ctypes.POINTER(ctypes.c_int)]),
            "tpt_plan_fused": (i, [vp, ctypes.POINTER(ctypes.c_int)]),
            "tpt_solve": (i, [vp, vp, vp, vp, sz, vp]),
            "tpt_solve_info": (i, [vp, ctypes.POINTER(Info)]),
            "tpt_solve_noalloc": (i, [vp, vp, vp, vp]),
            "tpt_residual": (i, [vp, vp, vp, vp, vp]),
            "tpt_static_workspace_capacity": (sz, []),
            "tpt_divergence": (i, [vp, vp, vp, vp, vp, vp]),
            "tpt_gradient_update": (i, [vp, vp, vp, vp, vp, vp]),
            "tpt_project_workspace_bytes": (i, [vp, ctypes.POINTER(sz)]),
            "tpt_project": (i, [vp, vp, vp, vp, vp, vp, sz, vp]),
            "tpt_ns_create": (i, [vp, d, d, i, ctypes.POINTER(vp)]),
            "tpt_ns_destroy": (i, [vp]),
            "tpt_ns_workspace_bytes": (i, [vp, ctypes.POINTER(sz)]),
            "tpt_ns_substep": (i, [vp, i, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
            "tpt_batch_create": (i, [i, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
            "tpt_batch_destroy": (i, [vp]),
            "tpt_batch_workspace_bytes": (i, [vp, ctypes.POINTER(sz)]),
            "tpt_batch_solve": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, sz, vp, i]),
            "tpt_batch_info": (i, [vp, i, ctypes.POINTER(Info)]),
            "tpt_autotune": (i, [i, ctypes.POINTER(vp), vp]),
            "tpt_autotune_save": (i, [ctypes.c_char_p]),
            "tpt_autotune_load": (i, [ctypes.c_char_p]),
            "tpt_server_create": (i, [sz, i, ctypes.POINTER(vp)]),
            "tpt_server_submit": (i, [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_ulonglong)]),
            "tpt_server_poll": (i, [vp, ctypes.c_ulonglong, ctypes.POINTER(Info), dp, dp, dp]),
            "tpt_server_drain": (i, [vp]),
            "tpt_server_destroy": (i, [vp]),
            "tpt_thomas": (i, [i, i, i, i, vp, vp, vp, vp, vp, i, d, d, i, vp, vp, vp, i, vp]),
            "tpt_gemm": (i, [i, i, i, i, i, i, i, vp, ctypes.c_longlong, vp, ctypes.c_longlong, vp,
                             ctypes.c_longlong, vp]),
            "tpt_timing_enable": (i, [i]),
            "tpt_timing_collect": (i, [ctypes.POINTER(ctypes.c_int), ctypes.c_char_p, sz, dp,
                                       ctypes.POINTER(ctypes.c_longlong)]),
            "tpt_last_error": (ctypes.c_char_p, []),
            "tpt_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


EXPORTED = ("tpt_plan_desc_init", "tpt_plan_create", "tpt_plan_destroy", "tpt_plan_shape",
            "tpt_plan_workspace_bytes", "tpt_plan_eigen", "tpt_plan_operator", "tpt_plan_transforms", "tpt_plan_fused", "tpt_solve",
            "tpt_solve_info", "tpt_solve_noalloc", "tpt_residual", "tpt_static_workspace_capacity", "tpt_divergence", "tpt_gradient_update",
            "tpt_project_workspace_bytes", "tpt_project", "tpt_ns_create", "tpt_ns_destroy",
            "tpt_ns_workspace_bytes", "tpt_ns_substep", "tpt_batch_create", "tpt_batch_destroy", "tpt_batch_workspace_bytes",
            "tpt_batch_solve", "tpt_batch_info", "tpt_autotune", "tpt_autotune_save", "tpt_autotune_load",
            "tpt_server_create", "tpt_server_submit", "tpt_server_poll", "tpt_server_drain",
            "tpt_server_destroy", "tpt_thomas", "tpt_gemm", "tpt_timing_enable", "tpt_timing_collect",
            "tpt_last_error", "tpt_version")


def _check(rc):
    if rc < 0:
        msg = lib().tpt_last_error()
        raise TptError(rc, msg.decode() if msg else "")
    return rc


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _require_f64_cuda(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != int(np.prod(shape)):
        raise ValueError(f"{name} has {t.numel()} elements, expected {int(np.prod(shape))}")


class Plan:
    """A solver plan for one grid, boundary-condition set and operator.

    n: cells (nx, ny, nz); faces: three arrays of n+1 face coordinates;
    bc: three (lower, upper) pairs; loc: three of 'C'/'F'; kind 'poisson' or
    'helmholtz' with alpha; implicit 'xyz', 'yz' or 'z' (Helmholtz: the
    directions in the implicit operator); precision 'fp64', 'fp32' or 'bf16x3';
    fixed_refine >= 0 runs that many corrections without host synchronisation;
    dense_x / dense_y force the dense GEMM for a direction where a fast
    transform (FFT, DCT-II, DST-II of a uniform direction) would apply;
    fuse_xy runs the x fast transform and the y GEMM of an FP64 solve as
    one fused pass per direction (see `fused`; slower on gfx950 than the
    separate passes, so off by default); seq_thomas solves the z lines with
    the sequential kernel instead of the partitioned one; check=False skips
    the right-hand-side check (Info.compat_defect, Info.nonfinite).
    """

    def __init__(self, n, faces, bc, loc=("C", "C", "C"), kind="poisson", alpha=0.0, precision="fp64",
                 rtol=1e-12, max_refine=8, fixed_refine=-1, nrhs=1, host_only=False, dense_x=False,
                 dense_y=False, fuse_xy=False, seq_thomas=False, check=True, implicit="xyz"):
        L = lib()
        d = _Desc()
        L.tpt_plan_desc_init(ctypes.byref(d))
        self._faces = [np.ascontiguousarray(np.asarray(f, dtype=np.float64)) for f in faces]
        for k in range(3):
            d.n[k] = int(n[k])
            d.faces[k] = self._faces[k].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.bc[k][0] = _BC[bc[k][0]]
            d.bc[k][1] = _BC[bc[k][1]]
            d.loc[k] = _LOC[loc[k]]
        d.kind = _KIND[kind]
        d.alpha = float(alpha)
        d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        d.rtol = float(rtol)
        d.max_refine = int(max_refine)
        d.fixed_refine = int(fixed_refine)
        d.nrhs = int(nrhs)
        d.implicit = _IMPLICIT[implicit]
        d.flags = ((1 if host_only else 0) | (2 if dense_x else 0) | (4 if dense_y else 0)
                   | (8 if fuse_xy else 0) | (16 if seq_thomas else 0) | (0 if check else 32))
        h = ctypes.c_void_p()
        _check(L.tpt_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._bc = tuple(tuple(b) for b in bc)
        self.nrhs = int(nrhs)
        self.precision = precision
        s = (ctypes.c_int * 3)()
        _check(L.tpt_plan_shape(h, s))
        self.nxyz = (s[0], s[1], s[2])
        self._ws = None

    @classmethod
    def from_problem(cls, p, **kw):
        """Plan for an object with n, faces, bc, loc, kind, alpha (and
        optionally implicit) attributes."""
        kw.setdefault("implicit", getattr(p, "implicit", "xyz"))
        return cls(p.n, p.faces, p.bc, p.loc, p.kind, p.alpha, **kw)

    @property
    def handle(self):
        return self._h

    @property
    def shape(self):
        nx, ny, nz = self.nxyz
        return (nz, ny, nx) if self.nrhs == 1 else (self.nrhs, nz, ny, nx)

    @property
    def dof(self):
        nx, ny, nz = self.nxyz
        return nx * ny * nz

    @property
    def transforms(self):
        """How x and y are transformed: each of 'gemm', 'fft', 'dct', 'dst',
        or 'none' for a direction the plan leaves explicit."""
        v = (ctypes.c_int * 2)()
        _check(lib().tpt_plan_transforms(self._h, v))
        names = ("gemm", "fft", "dct", "dst", "none")
        return names[v[0]], names[v[1]]

    @property
    def fused(self):
        """True when an FP64 solve runs the x fast transform inside the y
        GEMM's loads (one pass each way instead of two)."""
        v = ctypes.c_int()
        _check(lib().tpt_plan_fused(self._h, ctypes.byref(v)))
        return bool(v.value)

    @property
    def x_fft(self) -> bool:
        """True if the x eigenbasis is applied by a fast transform."""
        return self.transforms[0] not in ("gemm", "none")

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().tpt_plan_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    def eigen(self, direction: int):
        n = self.nxyz[direction]
        lam = np.empty(n)
        Qt = np.empty((n, n))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().tpt_plan_eigen(self._h, direction, lam.ctypes.data_as(dp), Qt.ctypes.data_as(dp)))
        return lam, Qt

    def operator(self, direction: int):
        n = self.nxyz[direction]
        arrs = [np.empty(n) for _ in range(4)]
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().tpt_plan_operator(self._h, direction, *[a.ctypes.data_as(dp) for a in arrs]))
        return tuple(arrs)

    def workspace(self):
        """A torch workspace tensor of the right size (cached on the plan)."""
        import torch
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes(), dtype=torch.uint8, device="cuda")
        return self._ws

    def solve(self, rhs, out=None, workspace=None, stream=None):
        """Solve for rhs (float64 CUDA tensor of self.shape); returns out."""
        import torch
        _require_f64_cuda(rhs, self.shape, "rhs")
        if out is None:
            out = torch.empty_like(rhs)
        _require_f64_cuda(out, self.shape, "out")
        ws = self.workspace() if workspace is None else workspace
        _check(lib().tpt_solve(self._h, _ptr(rhs), _ptr(out), _ptr(ws), ws.numel() * ws.element_size(),
                               _stream(stream)))
        return out

    def solve_noalloc(self, rhs, out, stream=None):
        """Solve with the library's static device workspace (no allocation;
        see tpt_solve_noalloc); out must be given."""
        _require_f64_cuda(rhs, self.shape, "rhs")
        _require_f64_cuda(out, self.shape, "out")
        _check(lib().tpt_solve_noalloc(self._h, _ptr(rhs), _ptr(out), _stream(stream)))
        return out

    def info(self) -> Info:
        inf = Info()
        _check(lib().tpt_solve_info(self._h, ctypes.byref(inf)))
        return inf

    def residual(self, x, f, r=None, stream=None):
        """r = f - A x of the plan's operator in FP64, stored as float32
        (see tpt_residual); x, f float64 CUDA tensors of self.shape."""
        import torch
        _require_f64_cuda(x, self.shape, "x")
        _require_f64_cuda(f, self.shape, "f")
        if r is None:
            r = torch.empty(x.shape, dtype=torch.float32, device=x.device)
        if not isinstance(r, torch.Tensor) or r.dtype != torch.float32 or r.device != x.device \
                or not r.is_contiguous() or r.numel() != x.numel():
            raise ValueError("r must be a contiguous float32 tensor on x's device with x's size")
        _check(lib().tpt_residual(self._h, _ptr(x), _ptr(f), _ptr(r), _stream(stream)))
        return r

    # ---- projection step (pressure plans: cell-centred, periodic / Neumann) ----
    def velocity_shapes(self):
        """Shapes of u, v, w on the faces of this pressure grid."""
        nx, ny, nz = self.nxyz
        b = self._bc
        nf = [n if b[d][0] == "P" else n - 1 for d, n in enumerate((nx, ny, nz))]
        return (nz, ny, nf[0]), (nz, nf[1], nx), (nf[2], ny, nx)

    def _check_velocity(self, u, v, w):
        for t, s, name in zip((u, v, w), self.velocity_shapes(), "uvw"):
            _require_f64_cuda(t, s, name)

    def divergence(self, u, v, w, out=None, stream=None):
        import torch
        self._check_velocity(u, v, w)
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        _require_f64_cuda(out, self.shape, "div")
        _check(lib().tpt_divergence(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(out), _stream(stream)))
        return out

    def gradient_update(self, phi, u, v, w, stream=None):
        """(u, v, w) -= G phi in place."""
        self._check_velocity(u, v, w)
        _require_f64_cuda(phi, self.shape, "phi")
        _check(lib().tpt_gradient_update(self._h, _ptr(phi), _ptr(u), _ptr(v), _ptr(w), _stream(stream)))

    def project(self, u, v, w, phi=None, workspace=None, stream=None):
        """Project (u, v, w) in place onto the divergence-free fields;
        returns the pressure correction phi."""
        import torch
        self._check_velocity(u, v, w)
        if phi is None:
            phi = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        _require_f64_cuda(phi, self.shape, "phi")
        if workspace is None:
            b = ctypes.c_size_t()
            _check(lib().tpt_project_workspace_bytes(self._h, ctypes.byref(b)))
            workspace = torch.empty(b.value, dtype=torch.uint8, device="cuda")
        _check(lib().tpt_project(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(phi), _ptr(workspace),
                                 workspace.numel(), _stream(stream)))
        return phi

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.tpt_plan_destroy(h)
            self._h = None


class NavierStokes:
    """Runge-Kutta substeps of the incompressible Navier-Stokes solver
    (§2.1, Eq. rk3) on the grid of a pressure plan (see tpt_ns_create and
    tpt_ns_substep): kinematic viscosity nu, time step dt, implicit
    directions 'none', 'z', 'yz' or 'xyz'.  Velocities in the face layouts
    of Plan.velocity_shapes(), pressure in the plan's shape."""

    def __init__(self, pressure: "Plan", nu: float, dt: float, implicit: str = "xyz"):
        imp = dict(_IMPLICIT, none=3)[implicit]
        h = ctypes.c_void_p()
        _check(lib().tpt_ns_create(pressure.handle, float(nu), float(dt), imp, ctypes.byref(h)))
        self._h = h
        self.pressure = pressure
        self.nu, self.dt, self.implicit = float(nu), float(dt), implicit
        self._ws = None
        self._e = None

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().tpt_ns_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    def workspace(self):
        import torch
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes(), dtype=torch.uint8, device="cuda")
        return self._ws

    def substep(self, k, u, v, w, e, p, phi=None, workspace=None, stream=None):
        """Substep k (1, 2, 3) in place: (u, v, w) u^k -> u^{k+1}; e = (eu, ev,
        ew) E^{k-1} -> E^k; p P^{k-1/2} -> P^{k+1/2}.  Returns phi."""
        import torch
        P = self.pressure
        P._check_velocity(u, v, w)
        for t, s_, name in zip(e, P.velocity_shapes(), ("eu", "ev", "ew")):
            _require_f64_cuda(t, s_, name)
        _require_f64_cuda(p, P.shape, "p")
        if phi is None:
            phi = torch.empty(P.shape, dtype=torch.float64, device="cuda")
        _require_f64_cuda(phi, P.shape, "phi")
        ws = self.workspace() if workspace is None else workspace
        _check(lib().tpt_ns_substep(self._h, int(k), _ptr(u), _ptr(v), _ptr(w), _ptr(e[0]), _ptr(e[1]),
                                    _ptr(e[2]), _ptr(p), _ptr(phi), _ptr(ws), ws.numel() * ws.element_size(),
                                    _stream(stream)))
        return phi

    def step(self, u, v, w, p, phi=None, stream=None):
        """One full time step (substeps 1, 2, 3) in place; returns the last
        substep's phi."""
        import torch
        if self._e is None:
            self._e = tuple(torch.empty(s_, dtype=torch.float64, device="cuda")
                            for s_ in self.pressure.velocity_shapes())
        for k in (1, 2, 3):
            phi = self.substep(k, u, v, w, self._e, p, phi=phi, stream=stream)
        return phi

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.tpt_ns_destroy(h)
            self._h = None


class Batch:
    """Many independent plans solved with one launch per stage."""

    def __init__(self, plans: Sequence[Plan]):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().tpt_batch_create(len(self.plans), arr, ctypes.byref(h)))
        self._h = h
        self._ws = None

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().tpt_batch_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    def solve(self, rhs, outs, use_graph=True, stream=None, workspace=None):
        import torch
        if len(rhs) != len(self.plans) or len(outs) != len(self.plans):
            raise ValueError("one rhs and one out per plan")
        for p, r, o in zip(self.plans, rhs, outs):
            _require_f64_cuda(r, p.shape, "rhs")
            _require_f64_cuda(o, p.shape, "out")
        if workspace is None:
            if self._ws is None:
                self._ws = torch.empty(self.workspace_bytes(), dtype=torch.uint8, device="cuda")
            workspace = self._ws
        n = len(self.plans)
        ra = (ctypes.c_void_p * n)(*[_ptr(r) for r in rhs])
        oa = (ctypes.c_void_p * n)(*[_ptr(o) for o in outs])
        _check(lib().tpt_batch_solve(self._h, ra, oa, _ptr(workspace), workspace.numel(), _stream(stream),
                                     1 if use_graph else 0))
        return outs

    def info(self, index: int) -> Info:
        """Info of problem `index` of the last solve (after synchronising)."""
        inf = Info()
        _check(lib().tpt_batch_info(self._h, int(index), ctypes.byref(inf)))
        return inf

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.tpt_batch_destroy(h)
            self._h = None


def autotune(plans: Sequence[Plan], stream=None):
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    _check(lib().tpt_autotune(len(plans), arr, _stream(stream)))


def autotune_save(path: str):
    _check(lib().tpt_autotune_save(path.encode()))


def autotune_load(path: str):
    _check(lib().tpt_autotune_load(path.encode()))


class Server:
    """Continuous-batching serving loop (see tpt_server_* in include/tpt.h)."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 4):
        h = ctypes.c_void_p()
        _check(lib().tpt_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, plan: Plan, rhs, out) -> int:
        _require_f64_cuda(rhs, plan.shape, "rhs")
        _require_f64_cuda(out, plan.shape, "out")
        t = ctypes.c_ulonglong()
        _check(lib().tpt_server_submit(self._h, plan.handle, _ptr(rhs), _ptr(out), ctypes.byref(t)))
        self._keep[t.value] = (plan, rhs, out)
        return t.value

    def poll(self, ticket: int):
        """None if pending, else (info, t_submit, t_start, t_done)."""
        inf = Info()
        ts, t0, t1 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = _check(lib().tpt_server_poll(self._h, ticket, ctypes.byref(inf), ctypes.byref(ts), ctypes.byref(t0),
                                          ctypes.byref(t1)))
        if rc == PENDING:
            return None
        self._keep.pop(ticket, None)
        return inf, ts.value, t0.value, t1.value

    def drain(self):
        _check(lib().tpt_server_drain(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.tpt_server_destroy(h)
            self._h = None


# partitioned Thomas configurations (lines per block, segments, planes per
# segment), variants 1..
THOMAS_PARTS = ((64, 4, 8), (64, 8, 8), (32, 8, 8), (64, 8, 16), (32, 8, 16), (16, 8, 16), (64, 16, 16),
                (32, 16, 16), (16, 16, 16), (64, 8, 32), (32, 8, 32), (16, 8, 32), (16, 32, 16), (32, 16, 32),
                (16, 16, 32), (16, 64, 16), (16, 32, 32))


def thomas(nx, ny, nz, nsys, lamx, lamy, az, bz, cz, sigma, tau, pin_line, f, x, scratch, stream=None,
           periodic_z=False, variant=-1):
    """Kernel-level batched Thomas solve on explicit device inputs (cyclic
    lines with periodic_z); variant -1 automatic, 0 sequential, 1.. the
    partitioned configurations THOMAS_PARTS."""
    _check(lib().tpt_thomas(nx, ny, nz, nsys, _ptr(lamx), _ptr(lamy), _ptr(az), _ptr(bz), _ptr(cz),
                            1 if periodic_z else 0, float(sigma), float(tau), int(pin_line), _ptr(f), _ptr(x),
                            _ptr(scratch), int(variant), _stream(stream)))
    return x


def gemm(prec, A, B, C, M, N, K, batch=1, sA=0, sB=0, sC=0, b_nk=False, variant=-1, stream=None):
    """Kernel-level strided-batched GEMM with the MFMA kernels: C = A B
    (B stored K x N) or, with b_nk, C = A B^T (B stored N x K)."""
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    _check(lib().tpt_gemm(p, 1 if b_nk else 0, int(variant), M, N, K, batch, _ptr(A), sA, _ptr(B), sB, _ptr(C), sC,
                          _stream(stream)))
    return C


def timing_enable(on: bool = True):
    _check(lib().tpt_timing_enable(1 if on else 0))


def timing_collect():
    """{kernel name: (total ms, launches)} since the last collect."""
    cap = 64
    cnt = ctypes.c_int(cap)
    names = ctypes.create_string_buffer(4096)
    ms = (ctypes.c_double * cap)()
    n = (ctypes.c_longlong * cap)()
    _check(lib().tpt_timing_collect(ctypes.byref(cnt), names, 4096, ms, n))
    keys = [k.decode() for k in names.raw.split(b"\0")][: min(cnt.value, cap)]
    return {k: (ms[i], n[i]) for i, k in enumerate(keys)}


def version() -> str:
    return lib().tpt_version().decode()
