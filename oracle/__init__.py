"""CPU oracle for dense time-independent Lindblad propagation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the library itself
never does, and nothing here imports the library.

The arithmetic lives in ``oracle.c`` (plain FP64 C99 loops, long-double
brute-force references); this module compiles it with gcc on first use,
loads it with ctypes and adds the numpy error metrics.  Paper: arXiv
2603.18052 -- Eq. (1) (Lindblad equation), Eqs. (2)-(3) (vectorised step),
Alg. 1 (Pade [13/13] build), Alg. 2 (row-major matvec), Alg. 3 (batch of
independent states).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# FP64 reference: no -ffast-math; portable x86-64-v3 so the library built
# here also runs on other hosts.
CFLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=gnu11"]

THETA = 0.25  # Alg. 1 threshold (the paper's choice, not Higham's 5.37)
OK, ENOMEM, ESINGULAR, ENONFINITE = 0, -3, -5, -6


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        p, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        sig = {
            "orc_lindblad_rhs": (None, [i, p, i, p, p, p]),
            "orc_liouvillian": (None, [i, p, i, p, p]),
            "orc_matvec": (None, [i, p, p, p]),
            "orc_propagate": (None, [i, p, i, p, ll, i]),
            "orc_norm1": (d, [i, p]),
            "orc_scaling_exponent": (i, [d, d]),
            "orc_pade13_coefficients": (None, [p]),
            "orc_lu_solve": (i, [i, p, p, i]),
            "orc_expm_pade13": (i, [i, p, d, p, p]),
            "orc_propagators": (i, [i, i, p, p, d, p, p]),
            "orc_expm_taylor_ld": (None, [i, p, p]),
            "orc_rk4_ld": (None, [i, p, i, p, p, d, ll, i]),
            "orc_taylor_steps_ld": (None, [i, p, i, p, p, d, ll]),
            "orc_expm_frechet_blocktri": (i, [i, p, p, d, p, p]),
            "orc_grape": (i, [i, i, i, p, p, p, d, d, p, p, p, p, p]),
            "orc_max_threads": (i, []),
            "orc_quantize_q15": (None, [ll, p, p, p]),
            "orc_propagate_q15": (None, [i, p, p, i, p, p, ll]),
            "orc_quantize_q31": (None, [ll, p, p, p]),
            "orc_propagate_q31": (None, [i, p, p, i, p, p, ll]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _c(a, dtype=np.complex128):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != OK:
        raise OracleError(f"{what}: status {rc}")


# --------------------------------------------------------------- wrappers
def lindblad_rhs(H, Lk, rho):
    """Eq. (1) applied to one d x d matrix."""
    H, Lk, rho = _c(H), _c(Lk), _c(rho)
    out = np.empty_like(rho)
    lib().orc_lindblad_rhs(H.shape[0], _p(H), Lk.shape[0], _p(Lk), _p(rho), _p(out))
    return out


def liouvillian(H, Lk):
    """Row-major superoperator of Eq. (1): (d^2, d^2) complex128."""
    H, Lk = _c(H), _c(Lk)
    d = H.shape[0]
    out = np.empty((d * d, d * d), dtype=np.complex128)
    lib().orc_liouvillian(d, _p(H), Lk.shape[0], _p(Lk), _p(out))
    return out


def norm1(A):
    A = _c(A)
    return lib().orc_norm1(A.shape[0], _p(A))


def scaling_exponent(norm, theta=THETA):
    return lib().orc_scaling_exponent(float(norm), float(theta))


def pade13_coefficients():
    b = np.empty(14)
    lib().orc_pade13_coefficients(_p(b))
    return b


def lu_solve(A, B):
    A, B = _c(A).copy(), _c(B).copy()
    nrhs = 1 if B.ndim == 1 else B.shape[1]
    _check(lib().orc_lu_solve(A.shape[0], _p(A), _p(B), nrhs), "lu_solve")
    return B


def expm(A, theta=THETA, return_s=False):
    """Alg. 1 on an already scaled generator A = L dt."""
    A = _c(A)
    n = A.shape[0]
    P = np.empty_like(A)
    s = ctypes.c_int(0)
    _check(lib().orc_expm_pade13(n, _p(A), float(theta), _p(P), ctypes.byref(s)), "expm_pade13")
    return (P, s.value) if return_s else P


def propagator(L, dt, theta=THETA, return_s=False):
    return expm(np.asarray(L) * dt, theta, return_s)


def propagators(L, dt, theta=THETA):
    """Batched builds: L (M, n, n), dt scalar or (M,) -> (P (M, n, n), s (M,))."""
    L = _c(L)
    M, n = L.shape[0], L.shape[1]
    dts = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (M,)))
    P = np.empty_like(L)
    s = np.empty(M, dtype=np.int32)
    _check(lib().orc_propagators(n, M, _p(L), _p(dts), float(theta), _p(P), _p(s)), "propagators")
    return P, s


def expm_taylor_ld(A):
    A = _c(A)
    P = np.empty_like(A)
    lib().orc_expm_taylor_ld(A.shape[0], _p(A), _p(P))
    return P


def matvec(P, x):
    P, x = _c(P), _c(x)
    y = np.empty_like(x)
    lib().orc_matvec(P.shape[0], _p(P), _p(x), _p(y))
    return y


def propagate(P, rho, nsteps, nthreads=0):
    """Alg. 3 over Alg. 2: rho (B, n) or (B, d, d); returns the new states."""
    P = _c(P)
    n = P.shape[0]
    x = _c(rho).copy()
    shape = x.shape
    B = x.size // n
    lib().orc_propagate(n, _p(P), B, _p(x), int(nsteps), int(nthreads))
    return x.reshape(shape)


def rk4_ld(H, Lk, rho, dt, nsteps, sub=64):
    H, Lk = _c(H), _c(Lk)
    x = _c(rho).copy()
    lib().orc_rk4_ld(H.shape[0], _p(H), Lk.shape[0], _p(Lk), _p(x), float(dt), int(nsteps), int(sub))
    return x


def taylor_steps_ld(H, Lk, rho, dt, nsteps):
    """Eq. (1) stepped by its own Taylor series in long double."""
    H, Lk = _c(H), _c(Lk)
    x = _c(rho).copy()
    lib().orc_taylor_steps_ld(H.shape[0], _p(H), Lk.shape[0], _p(Lk), _p(x), float(dt), int(nsteps))
    return x


def expm_frechet(A, E, theta=THETA):
    """(exp(A), L(A, E)) from the block-triangular identity."""
    A, E = _c(A), _c(E)
    n = A.shape[0]
    eA, Lf = np.empty_like(A), np.empty_like(A)
    _check(lib().orc_expm_frechet_blocktri(n, _p(A), _p(E), float(theta), _p(eA), _p(Lf)), "frechet")
    return eA, Lf


def grape(L0, Lc, u, dt, x0, w, slices=None, theta=THETA, want_grad=True):
    """Fidelity F = Re<w, x_M> and its gradient (M, C) w.r.t. u.

    ``slices``: iterable of slice indices whose gradient rows are computed
    (None = all); other rows are NaN."""
    L0, Lc, u, x0, w = _c(L0), _c(Lc), _c(u, np.float64), _c(x0), _c(w)
    n = L0.shape[0]
    M, C = u.shape
    F = ctypes.c_double(0.0)
    grad = np.full((M, C), np.nan)
    mask = None
    if slices is not None:
        mask = np.zeros(M, dtype=np.uint8)
        mask[list(slices)] = 1
    rc = lib().orc_grape(n, M, C, _p(L0), _p(Lc), _p(u), float(dt), float(theta), _p(x0.reshape(-1)),
                         _p(w.reshape(-1)), ctypes.byref(F), _p(grad) if want_grad else None,
                         _p(mask) if mask is not None else None)
    _check(rc, "grape")
    return F.value, grad


def max_threads():
    return lib().orc_max_threads()


# ------------------------------------------------------------ Alg. 5 (Q1.15)
def quantize_q15(z):
    """Q1.15 codes (re, im) of complex values: round to nearest, saturate."""
    z = _c(z)
    re = np.empty(z.shape, dtype=np.int16)
    im = np.empty(z.shape, dtype=np.int16)
    lib().orc_quantize_q15(z.size, _p(z), _p(re), _p(im))
    return re, im


def propagate_q15(P, rho, nsteps):
    """Alg. 5 fixed-point chain: P and rho (B, n) or (B, d, d) complex are
    quantised to Q1.15, nsteps exact-integer steps with floor truncation and
    saturation run, and the codes (re, im) int16 (B, n) are returned."""
    P = _c(P)
    n = P.shape[0]
    x = _c(rho).reshape(-1, n)
    Pr, Pi = quantize_q15(P)
    xr, xi = quantize_q15(x)
    lib().orc_propagate_q15(n, _p(Pr), _p(Pi), x.shape[0], _p(xr), _p(xi), int(nsteps))
    return xr, xi


def from_q15(re, im):
    return (np.asarray(re, dtype=np.float64) + 1j * np.asarray(im, dtype=np.float64)) / 32768.0


# ------------------------------------------------------------ Alg. 5 (Q1.31)
def quantize_q31(z):
    """Q1.31 codes (re, im) int32 of complex values: round to nearest, saturate."""
    z = _c(z)
    re = np.empty(z.shape, dtype=np.int32)
    im = np.empty(z.shape, dtype=np.int32)
    lib().orc_quantize_q31(z.size, _p(z), _p(re), _p(im))
    return re, im


def propagate_q31(P, rho, nsteps):
    """The fixed-point chain at 31 fractional bits: P and rho (B, n) or
    (B, d, d) quantised to Q1.31, nsteps exact-integer steps (128-bit sums)
    with floor truncation and saturation; returns the codes (re, im) int32."""
    P = _c(P)
    n = P.shape[0]
    x = _c(rho).reshape(-1, n)
    Pr, Pi = quantize_q31(P)
    xr, xi = quantize_q31(x)
    lib().orc_propagate_q31(n, _p(Pr), _p(Pi), x.shape[0], _p(xr), _p(xi), int(nsteps))
    return xr, xi


def from_q31(re, im):
    return (np.asarray(re, dtype=np.float64) + 1j * np.asarray(im, dtype=np.float64)) / 2147483648.0


# ------------------------------------------------------------ error metrics
def herm(X):
    return 0.5 * (X + np.conj(np.swapaxes(X, -1, -2)))


def trace_distance(rho, sigma):
    """T = 1/2 sum |eig(Herm(rho - sigma))|, batched over leading axes."""
    D = herm(np.asarray(rho) - np.asarray(sigma))
    return 0.5 * np.abs(np.linalg.eigvalsh(D)).sum(axis=-1)


def rel_fro(X, Xref):
    X, Xref = np.asarray(X), np.asarray(Xref)
    return np.linalg.norm((X - Xref).ravel()) / np.linalg.norm(Xref.ravel())


def rel_per_state(X, Xref, X0=None):
    """Largest relative 2-norm error over the states of a batch: the rows of
    (B, n) arrays ((B, d, d) batches and single (n,) states are accepted), so
    one bad state cannot hide among good ones as it can in one Frobenius
    norm over the batch.  A zero reference state counts its absolute error.

    With X0 (the initial states) each error is taken relative to the larger
    of the state's initial and final norms.  A chain under a contraction
    that is not trace preserving (random test matrices) can shrink a state
    by many orders of magnitude; its forward error is bounded by N times the
    per-step rounding times the initial norm, not the final one."""
    X, Xref = np.asarray(X), np.asarray(Xref)
    B = 1 if X.ndim == 1 else X.shape[0]
    D = (X - Xref).reshape(B, -1)
    den = np.linalg.norm(Xref.reshape(B, -1), axis=1)
    if X0 is not None:
        den = np.maximum(den, np.linalg.norm(np.asarray(X0).reshape(B, -1), axis=1))
    den = np.where(den > 0, den, 1.0)
    return float((np.linalg.norm(D, axis=1) / den).max())


def state_report(rho):
    """Drift metrics of a batch of density matrices (B, d, d)."""
    rho = np.asarray(rho)
    tr = np.trace(rho, axis1=-2, axis2=-1)
    anti = np.abs(rho - np.conj(np.swapaxes(rho, -1, -2))).max(axis=(-1, -2))
    lam = np.linalg.eigvalsh(herm(rho)).min(axis=-1)
    return dict(trace_err=np.abs(tr - 1.0), antiherm=anti, lambda_min=lam)
