"""Python binding of the HIP library libgks.so (argument marshalling only).

Every step of the scheme runs in the library's HIP kernels; this module only
converts problem descriptions and arrays to the C ABI of include/gks.h and
back.  It fails loudly when the library is missing: there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgks.so")

GKS_OK, GKS_EINVAL, GKS_ENOMEM, GKS_EDEVICE, GKS_ENONPHYS, GKS_ESTATE = 0, -1, -2, -3, -4, -5
PREC_FP64, PREC_FP32_MIXED = 0, 1
KERNEL_FLUX, KERNEL_ROW, KERNEL_CELL = 0, 1, 2
BC_PERIODIC, BC_EXTRAP, BC_REFLECT, BC_INFLOW, BC_SPLIT, BC_CHAR = 0, 1, 2, 3, 4, 5


class GksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class gks_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("xlo", C.c_double), ("xhi", C.c_double), ("ylo", C.c_double), ("yhi", C.c_double),
                ("gamma", C.c_double), ("mu", C.c_double), ("cfl", C.c_double), ("dt_fixed", C.c_double),
                ("t_end", C.c_double), ("order", C.c_int32), ("recon", C.c_int32), ("bc", C.c_int32 * 4),
                ("bc_state", C.c_double * 32), ("bc_split", C.c_double * 8), ("bc_beyond", C.c_int32 * 4)]


_lib = None


def lib():
    """Load libgks.so (built by paper_1901_00261_amd/build.py); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run python paper_1901_00261_amd/build.py)")
        # PyTorch ships its own HIP runtime under the same soname.  Loaded
        # first, it is the runtime this library binds to, so the process has
        # one runtime and PyTorch's device buffers and streams are valid here;
        # loaded after this library, PyTorch would start a second runtime,
        # whose GPU initialisation fails.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        pp = C.POINTER(C.POINTER(C.c_double))
        hnd = C.c_void_p
        L.gks_init.argtypes = [C.POINTER(gks_problem), C.c_int32, C.c_int32, pp, pp, pp, C.c_void_p, C.POINTER(hnd)]
        L.gks_init_device.argtypes = L.gks_init.argtypes
        L.gks_step.argtypes = [hnd, C.c_int32, C.POINTER(C.c_int32)]
        L.gks_state.argtypes = [hnd, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                C.POINTER(C.c_int64)]
        L.gks_state_device.argtypes = [hnd, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.gks_problem_status.argtypes = [hnd, C.c_int32, C.POINTER(C.c_int32)]
        L.gks_free.argtypes = [hnd]
        L.gks_last_error.argtypes = [hnd]
        L.gks_last_error.restype = C.c_char_p
        L.gks_kernel_timing.argtypes = [hnd, C.c_int32]
        L.gks_kernel_time.argtypes = [hnd, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.gks_cell_updates.argtypes = [hnd, C.POINTER(C.c_int64)]
        L.gks_launch_config.argtypes = [hnd]
        L.gks_launch_config.restype = C.c_char_p
        L.gks_run1d_noalloc.argtypes = [C.POINTER(gks_problem), C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                        C.c_double, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                        C.POINTER(C.c_int32)]
        _lib = L
    return _lib


EXPORTED = ("gks_init", "gks_init_device", "gks_step", "gks_state", "gks_state_device", "gks_problem_status",
            "gks_free", "gks_last_error", "gks_kernel_timing", "gks_kernel_time", "gks_cell_updates",
            "gks_launch_config", "gks_run1d_noalloc")


def to_struct(p) -> gks_problem:
    s = gks_problem()
    s.dim, s.nx, s.ny = p.dim, p.nx, (p.ny if p.dim == 2 else 1)
    s.xlo, s.xhi, s.ylo, s.yhi = p.xlo, p.xhi, p.ylo, p.yhi
    s.gamma, s.mu, s.cfl, s.dt_fixed, s.t_end = p.gamma, p.mu, p.cfl, p.dt_fixed, p.t_end
    s.order, s.recon = p.order, p.recon
    for k in range(4):
        s.bc[k] = int(p.bc[k])
    st = getattr(p, "bc_state", None)
    sp = getattr(p, "bc_split", None)
    be = getattr(p, "bc_beyond", None)
    if st is not None:
        for i, v in enumerate(np.asarray(st, dtype=np.float64).ravel()[:32]):
            s.bc_state[i] = float(v)
    if sp is not None:
        for i, v in enumerate(np.asarray(sp, dtype=np.float64).ravel()[:8]):
            s.bc_split[i] = float(v)
    for k in range(4):
        s.bc_beyond[k] = int(be[k]) if be is not None else BC_REFLECT
    return s


class Solver:
    """A handle of the library holding one 2-D problem or a batch of 1-D
    problems (objects with the fields of workloads.Problem)."""

    def __init__(self, problems, precision=PREC_FP64, stream=None, device_arrays=None):
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self.dim = self.problems[0].dim
        L = lib()
        n = len(self.problems)
        arr = (gks_problem * n)(*[to_struct(p) for p in self.problems])
        PD = C.POINTER(C.c_double)
        if device_arrays is None:
            self._keep = []
            ptrs = []
            for name in ("W", "Wx", "Wy"):
                row = []
                for p in self.problems:
                    a = getattr(p, name)
                    if a is None:
                        row.append(PD())
                        continue
                    a = np.ascontiguousarray(a, dtype=np.float64)
                    self._keep.append(a)
                    row.append(a.ctypes.data_as(PD))
                ptrs.append((PD * n)(*row))
            init = L.gks_init
        else:
            # device_arrays: list over problems of (W, Wx, Wy) device addresses (ints)
            ptrs = [(PD * n)(*[C.cast(C.c_void_p(d[k]) if d[k] else None, PD) for d in device_arrays])
                    for k in range(3)]
            init = L.gks_init_device
        h = C.c_void_p()
        st = init(arr, n, precision, ptrs[0], ptrs[1], ptrs[2], C.c_void_p(stream) if stream else None,
                  C.byref(h))
        if st != GKS_OK:
            raise GksError(st, L.gks_last_error(None).decode())
        self.h = h

    def _check(self, st):
        if st != GKS_OK:
            raise GksError(st, lib().gks_last_error(self.h).decode())

    def step(self, max_steps=1, raise_on_error=True):
        na = C.c_int32(0)
        st = lib().gks_step(self.h, int(max_steps), C.byref(na))
        if raise_on_error:
            self._check(st)
        return na.value if st == GKS_OK else st

    def state(self, p=0):
        pr = self.problems[p]
        nv = pr.dim + 2
        shape = (pr.nx, nv) if pr.dim == 1 else (pr.ny, pr.nx, nv)
        W = np.empty(shape)
        Wx = np.empty(shape)
        Wy = np.empty(shape) if pr.dim == 2 else None
        t = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(lib().gks_state(self.h, p, W.ctypes.data, Wx.ctypes.data,
                                    Wy.ctypes.data if Wy is not None else None, C.byref(t), C.byref(n)))
        return W, Wx, Wy, t.value, n.value

    def state_device(self, p, W_ptr, Wx_ptr, Wy_ptr=None):
        """Copy problem p into caller-owned device buffers (addresses as ints,
        layout as the host arrays of state())."""
        self._check(lib().gks_state_device(self.h, p, C.c_void_p(W_ptr), C.c_void_p(Wx_ptr),
                                           C.c_void_p(Wy_ptr) if Wy_ptr else None))

    def status(self, p=0):
        s = C.c_int32(0)
        self._check(lib().gks_problem_status(self.h, p, C.byref(s)))
        return s.value

    def timing(self, enable=True):
        self._check(lib().gks_kernel_timing(self.h, 1 if enable else 0))

    def kernel_time(self, kernel_id):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(lib().gks_kernel_time(self.h, kernel_id, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def cell_updates(self):
        c = C.c_int64(0)
        self._check(lib().gks_cell_updates(self.h, C.byref(c)))
        return c.value

    def launch_config(self):
        return lib().gks_launch_config(self.h).decode()

    def close(self):
        if getattr(self, "h", None):
            lib().gks_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def run1d_noalloc(problem, W_ptr, Wx_ptr, nsteps, t0=0.0, precision=PREC_FP64, stream=None, sync=True):
    """gks_run1d_noalloc: advance one 1-D problem in place in caller-owned
    device arrays (addresses as ints, [nx][3] float64).  With sync, returns
    (t, steps, status); otherwise only enqueues the kernels."""
    s = to_struct(problem)
    t = C.c_double(0.0)
    n = C.c_int64(0)
    stv = C.c_int32(0)
    st = lib().gks_run1d_noalloc(C.byref(s), precision, C.c_void_p(W_ptr), C.c_void_p(Wx_ptr), int(nsteps),
                                 float(t0), C.c_void_p(stream) if stream else None,
                                 C.byref(t) if sync else None, C.byref(n) if sync else None,
                                 C.byref(stv) if sync else None)
    if st != GKS_OK:
        raise GksError(st, lib().gks_last_error(None).decode())
    return (t.value, n.value, stv.value) if sync else None
