"""ctypes binding of the C oracle (gks_oracle.c).

TEST INFRASTRUCTURE ONLY.  Shares nothing with the HIP library: its own C
source, its own build, its own argument marshalling.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

PERIODIC, EXTRAP, REFLECT, INFLOW, SPLIT, CHAR = 0, 1, 2, 3, 4, 5
LINEAR, WENOZ = 0, 1


class OracleError(RuntimeError):
    def __init__(self, code, msg, t=None, nsteps=None):
        super().__init__(msg)
        self.code = code
        self.t = t            # time reached (run() failures)
        self.nsteps = nsteps  # steps completed before the failure


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = C.CDLL(_build.LIB)
        d = C.POINTER(C.c_double)
        i = C.POINTER(C.c_int)
        _lib.orc_run.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                 C.c_int, C.c_int, i, d, d, i, d, d, d, d, C.POINTER(C.c_long)]
        _lib.orc_linear_map.argtypes = [C.c_int, d]
        _lib.orc_candidate_map.argtypes = [C.c_int, d]
        _lib.orc_weno.argtypes = [C.c_int, d, d, d, d, d]
        _lib.orc_set_weno_eps.argtypes = [C.c_double]
        _lib.orc_tangential_map.argtypes = [d]
        _lib.orc_euler_R.argtypes = [C.c_int, C.c_double, d, d]
        _lib.orc_raw_moment.argtypes = [C.c_int, C.c_double, d, C.c_int, C.c_int, C.c_int, C.c_int, d]
        _lib.orc_micro_solve.argtypes = [C.c_int, C.c_double, d, d, d]
        _lib.orc_psi_moments_lin.argtypes = [C.c_int, C.c_double, d, d, C.c_int, d]
        _lib.orc_gks_point.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, d, d]
        _lib.orc_exp_fit.argtypes = [C.c_double, C.c_double, d]
        _lib.orc_threads.argtypes = []
        _lib.orc_kinetic_average.argtypes = [C.c_int, C.c_double, d, d, d]
        _lib.orc_tangential_weno.argtypes = [C.c_int, d, d]
        _lib.orc_tangential_weno_weights.argtypes = [d]
        _lib.orc_tangential_weno_detail.argtypes = [C.c_int, d, d]
        _lib.orc_fallbacks.argtypes = []
        _lib.orc_fallbacks.restype = C.c_long
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a.copy()


def run(dim, W, Wx, Wy=None, *, xlo, xhi, ylo=0.0, yhi=1.0, gamma=1.4, mu=0.0, cfl=0.3,
        dt_fixed=0.0, t_end, max_steps=0, order=8, recon=WENOZ, bc=(PERIODIC,) * 4, t0=0.0,
        bc_state=None, bc_split=None, bc_beyond=None):
    """Advance (W, Wx[, Wy]) with the oracle.  Arrays: [nx, nv] (1-D) or
    [ny, nx, nv] (2-D), conservative averages and cell-averaged gradients.
    Boundary data for INFLOW / SPLIT sides: bc_state [4 sides][2 states][4]
    (conservative, 4 slots), bc_split [4][2] (switch position at t = 0 and
    its speed), bc_beyond [4] (INFLOW of state B or REFLECT beyond the
    switch).  Returns (W, Wx, Wy, t, nsteps).  Raises OracleError on
    failure."""
    W = _f64(W)
    Wx = _f64(Wx)
    if dim == 1:
        nx, ny = W.shape[0], 1
        Wy = np.zeros(1)
    else:
        ny, nx = W.shape[0], W.shape[1]
        Wy = _f64(Wy)
    bca = (C.c_int * 4)(*bc)
    bstate = _f64(np.zeros(32) if bc_state is None else bc_state, 32)
    bsplit = _f64(np.zeros(8) if bc_split is None else bc_split, 8)
    bbey = (C.c_int * 4)(*((REFLECT,) * 4 if bc_beyond is None else bc_beyond))
    t = C.c_double(t0)
    n = C.c_long(0)
    st = lib().orc_run(dim, nx, ny, xlo, xhi, ylo, yhi, gamma, mu, cfl, dt_fixed, t_end, max_steps,
                       order, recon, bca, _p(bstate), _p(bsplit), bbey, _p(W), _p(Wx), _p(Wy), C.byref(t),
                       C.byref(n))
    if st != 0:
        raise OracleError(st, f"oracle run failed with status {st} at t={t.value} after {n.value} steps",
                          t=t.value, nsteps=n.value)
    return W, Wx, (Wy if dim == 2 else None), t.value, n.value


def linear_map(order):
    out = np.zeros((3, 8))
    lib().orc_linear_map(order, _p(out))
    return out


def candidate_map(k):
    out = np.zeros((5, 8))
    lib().orc_candidate_map(k, _p(out))
    return out


def weno(order, Wk, Dk):
    """Scalar WENO-Z: returns (left value, dx*left derivative, right value,
    dx*right derivative), delta[7], beta[7] (left state)."""
    Wk = _f64(Wk, 4)
    Dk = _f64(Dk, 4)
    res = np.zeros(4)
    delta = np.zeros(7)
    beta = np.zeros(7)
    lib().orc_weno(order, _p(Wk), _p(Dk), _p(res), _p(delta), _p(beta))
    return res, delta, beta


def set_weno_eps(eps):
    lib().orc_set_weno_eps(eps)


def tangential_map():
    out = np.zeros((3, 3, 5))
    lib().orc_tangential_map(_p(out))
    return out


def euler_R(dim, gamma, W):
    W = _f64(W, 4) if len(W) == 4 else np.concatenate([_f64(W), np.zeros(4 - len(W))])
    nv = dim + 2
    R = np.zeros(16)
    st = lib().orc_euler_R(dim, gamma, _p(W), _p(R))
    if st:
        raise OracleError(st, "non-physical state")
    return R[: nv * nv].reshape(nv, nv)


def _pad4(v):
    out = np.zeros(4)
    v = np.asarray(v, dtype=np.float64).ravel()
    out[: len(v)] = v
    return out


def raw_moment(dim, gamma, W, a, b, c, half=0):
    W = _pad4(W)
    out = C.c_double(0.0)
    st = lib().orc_raw_moment(dim, gamma, _p(W), a, b, c, half, C.byref(out))
    if st:
        raise OracleError(st, "non-physical state")
    return out.value


def micro_solve(dim, gamma, W, b):
    W = _pad4(W)
    b = _pad4(b)
    a = np.zeros(4)
    st = lib().orc_micro_solve(dim, gamma, _p(W), _p(b), _p(a))
    if st:
        raise OracleError(st, "non-physical state")
    return a[: dim + 2]


def psi_moments_lin(dim, gamma, W, a, half=0):
    W = _pad4(W)
    a = _pad4(a)
    out = np.zeros(4)
    st = lib().orc_psi_moments_lin(dim, gamma, _p(W), _p(a), half, _p(out))
    if st:
        raise OracleError(st, "non-physical state")
    return out[: dim + 2]


GP_FIELDS = ("W0", "W0x", "W0y", "W0xx", "W0xy", "W0yy", "Wl", "Wlx", "Wly", "Wr", "Wrx", "Wry")


def gks_point(dim, gamma, mu, dt, **fields):
    """Interface-point evaluation.  Keyword arrays named as GP_FIELDS (missing
    ones are zero).  Returns dict FL, FdL, S0, S1, S2."""
    buf = np.zeros(48)
    for q, name in enumerate(GP_FIELDS):
        if name in fields:
            buf[4 * q: 4 * q + 4] = _pad4(fields[name])
    out = np.zeros(20)
    st = lib().orc_gks_point(dim, gamma, mu, dt, _p(buf), _p(out))
    if st:
        raise OracleError(st, "non-physical state")
    nv = dim + 2
    return {k: out[4 * q: 4 * q + nv].copy() for q, k in enumerate(("FL", "FdL", "S0", "S1", "S2"))}


def exp_fit(tau_n, dt):
    out = np.zeros(4)
    lib().orc_exp_fit(tau_n, dt, _p(out))
    return out


def threads():
    return lib().orc_threads()


def set_threads(n):
    """Number of OpenMP threads for later runs."""
    lib().orc_set_threads.argtypes = [C.c_int]
    lib().orc_set_threads(int(n))


def kinetic_average(dim, gamma, Wl, Wr):
    Wl = _pad4(Wl)
    Wr = _pad4(Wr)
    out = np.zeros(4)
    st = lib().orc_kinetic_average(dim, gamma, _p(Wl), _p(Wr), _p(out))
    if st:
        raise OracleError(st, "non-physical state")
    return out[: dim + 2]


def tangential_weno(g, q):
    q = _f64(q, 5)
    out = C.c_double(0.0)
    lib().orc_tangential_weno(g, _p(q), C.byref(out))
    return out.value


def tangential_weno_weights():
    out = np.zeros((3, 3))
    lib().orc_tangential_weno_weights(_p(out))
    return out


def tangential_weno_detail(g, q):
    """Tangential WENO-Z at Gauss point g: (value, beta[3], candidate values[3])."""
    q = _f64(q, 5)
    out = np.zeros(7)
    lib().orc_tangential_weno_detail(g, _p(q), _p(out))
    return out[0], out[1:4].copy(), out[4:7].copy()


def fallbacks():
    """Positivity fallbacks (reading A21) taken by the last run(): face-row
    WENO-Z states replaced by the adjacent cell average plus Gauss-point
    states replaced by their face-row line value."""
    return int(lib().orc_fallbacks())
