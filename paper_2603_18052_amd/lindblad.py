"""ctypes binding of liblindblad.so (C-ABI in include/lindblad.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Tensors are torch CUDA (ROCm) tensors; the work is enqueued on
torch's current stream.  If the library is missing or fails to load, every
call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblindblad.so")

OK, EINVAL, ESHAPE, ENOMEM, EHIP, ESINGULAR, ENONFINITE, ENOTSUP = 0, -1, -2, -3, -4, -5, -6, -7
C128, C64, BF16_HILO, BF16_SLICED, Q15, I8_SLICED, Q31, I8_HERM = 0, 1, 2, 3, 4, 5, 6, 7
PRECISIONS = {"c128": C128, "c64": C64, "bf16_hilo": BF16_HILO, "bf16_sliced": BF16_SLICED, "q15": Q15,
              "i8_sliced": I8_SLICED, "q31": Q31, "i8_herm": I8_HERM}

SYMBOLS = {
    # name: (restype, argtypes)
    "lb_workspace_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]),
    "lb_workspace_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "lb_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "lindblad_last_error": (ctypes.c_char_p, []),
    "lindblad_liouvillian": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "lindblad_generators": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lindblad_propagator": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "lindblad_propagator_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p]),
    "lindblad_propagator_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "lindblad_propagator_stages": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lindblad_propagate": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p, ctypes.c_void_p]),
    "lindblad_propagate_baseline": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                                   ctypes.c_longlong, ctypes.c_void_p, ctypes.c_void_p]),
    "grape_gradient": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "lindblad_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "lindblad_chain_variants": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                               ctypes.c_int, ctypes.c_void_p]),
    "lindblad_chain_variant": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "lindblad_propagate_variant": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int, ctypes.c_void_p,
                                                  ctypes.c_void_p]),
    "lindblad_tune": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_longlong, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "lindblad_tune_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "lindblad_batch_set_window": (ctypes.c_int, [ctypes.c_size_t]),
    "lindblad_batch_enqueue": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lindblad_expmv": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_longlong, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "lindblad_expmv_params": (ctypes.c_int, [ctypes.c_double, ctypes.POINTER(ctypes.c_int),
                                             ctypes.POINTER(ctypes.c_int)]),
}

# Chain variant families (id = family * 100 + tile parameter).
VARIANT_FAMILIES = {1: "baseline", 2: "wave", 3: "fused", 4: "bf16_fused", 5: "gemm", 6: "matvec32", 7: "planes",
                    8: "fused_balanced", 9: "q15", 10: "fused_tail", 11: "gemm_tiled", 12: "planes_tiled",
                    13: "i8_fused", 14: "fx_i8", 15: "i8_gemm"}


GRAPH_VARIANT = 50  # added to a per-step family: steps replayed from a captured HIP graph


def variant_name(v: int) -> str:
    fam, prm = divmod(int(v), 100)
    name = VARIANT_FAMILIES.get(fam, f"family{fam}")
    graph = fam in (1, 5, 6, 7, 9, 11, 12, 15) and prm >= GRAPH_VARIANT
    prm = prm % GRAPH_VARIANT if fam in (1, 5, 6, 7, 9, 11, 12, 15) else prm
    if fam == 3:
        name = f"{name}(k{prm})"
    elif fam == 5:
        name = f"{name}(w{prm})"
    elif fam == 9:
        name = f"{name}_{'wave' if prm == 0 else 'matvec'}"
    elif fam == 11:
        name = {1: f"{name}(ring)", 2: f"{name}(ring+splitk)"}.get(prm, f"{name}(w{prm})")
    elif fam == 12 and prm in (1, 2):
        name = f"{name}({'ring' if prm == 1 else 'ring+splitk'})"
    elif fam == 10 and prm in (1, 2, 3):
        name = f"{name}({('w16', 'tiles', 'tiles+presum')[prm - 1]})"
    elif fam == 13 and prm in (0, 1, 2):
        name = f"{name}({('w8', 'w4', 'w8+progress')[prm]})"
    elif fam == 15 and prm in (0, 1, 2, 3):
        name = f"{name}({('96x64', '96x32', '64x16', '96x32 pair')[prm]})"
    return name + "+graph" if graph else name


class LindbladError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    """struct lb_problem of the C-ABI."""
    _fields_ = [("d", ctypes.c_int), ("L", ctypes.c_void_p), ("dt", ctypes.c_double),
                ("nsteps", ctypes.c_longlong), ("rho", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_18052_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().lindblad_last_error().decode()


def _check(rc):
    if rc != OK:
        raise LindbladError(rc, last_error())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype=torch.complex128, name="tensor") -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (ROCm) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Workspace:
    """Library-owned device scratch with a byte cap (lb_workspace)."""

    def __init__(self, max_bytes: int = 64 << 30):
        h = ctypes.c_void_p()
        _check(lib().lb_workspace_create(int(max_bytes), ctypes.byref(h)))
        self.handle = h

    @property
    def nbytes(self) -> int:
        return lib().lb_workspace_bytes(self.handle)

    def close(self):
        if self.handle is not None:
            _check(lib().lb_workspace_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ws(ws):
    return ws.handle if ws is not None else None


# ------------------------------------------------------------ entry points
def liouvillian(H: torch.Tensor, Lk: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Eq. (1) superoperator, row-major vectorisation: (d^2, d^2) complex128."""
    H = _dev(H, name="H")
    d = H.shape[0]
    K = 0 if Lk is None else Lk.shape[0]
    if K:
        Lk = _dev(Lk, name="Lk")
    if out is None:
        out = torch.empty((d * d, d * d), dtype=torch.complex128, device=H.device)
    _check(lib().lindblad_liouvillian(d, _ptr(H), K, _ptr(Lk) if K else None, _ptr(out), _stream()))
    return out


def generators(L0: torch.Tensor, Lc: torch.Tensor, u: torch.Tensor, out: torch.Tensor | None = None):
    """Eq. (5) slice generators: out[m] = L0 + sum_c u[m, c] Lc[c]."""
    L0 = _dev(L0, name="L0")
    u = _dev(u, torch.float64, "u")
    n = L0.shape[0]
    M, C = u.shape
    if C:
        Lc = _dev(Lc, name="Lc")
    if out is None:
        out = torch.empty((M, n, n), dtype=torch.complex128, device=L0.device)
    _check(lib().lindblad_generators(n, M, C, _ptr(L0), _ptr(Lc) if C else None, _ptr(u), _ptr(out), _stream()))
    return out


def propagator(L: torch.Tensor, dt, theta: float = 0.25, ws: Workspace | None = None, return_s: bool = False,
               status: torch.Tensor | None = None):
    """Alg. 1: P = exp(L dt).  L is (n, n) or (M, n, n); dt a float or M floats.

    The library call is stream-ordered (s and the status word stay on the
    device).  Without `status` this wrapper then reads the status word back
    (one synchronisation) and raises LindbladError on a non-finite norm, a
    zero pivot or an s beyond the squaring cap; with a caller's int32
    `status` tensor (set to 0 beforehand) it returns at once and the caller
    checks the word when it wants.  return_s: also return s (ints; a device
    tensor when `status` is given)."""
    L = _dev(L, name="L")
    single = L.dim() == 2
    Lb = L.unsqueeze(0) if single else L
    M, n = Lb.shape[0], Lb.shape[1]
    dts = (ctypes.c_double * M)(*([float(dt)] * M if isinstance(dt, (int, float)) else [float(x) for x in dt]))
    s_dev = torch.empty(M, dtype=torch.int32, device=Lb.device) if return_s else None
    own = status is None
    if own:
        status = torch.zeros(1, dtype=torch.int32, device=Lb.device)
    P = torch.empty_like(Lb)
    _check(lib().lindblad_propagator(n, M, _ptr(Lb), dts, float(theta), _ptr(P),
                                     _ptr(s_dev) if return_s else None, _ptr(status), _ws(ws), _stream()))
    if own:
        code = int(status.item())
        if code != OK:
            what = {ENONFINITE: "||L dt||_1 is not finite", ESINGULAR: "zero pivot in the Pade denominator V - U",
                    ENOTSUP: "scaling exponent above the squaring cap"}.get(code, "device status")
            raise LindbladError(code, f"lindblad_propagator: {what} (status {code})")
    P = P[0] if single else P
    if return_s:
        s = s_dev.tolist() if own else s_dev
        return P, (s[0] if single and own else s)
    return P


def propagator_stages(L: torch.Tensor, dt, theta: float = 0.25, ws: Workspace | None = None):
    """lindblad_propagator_stages: the build timed by stage.  Returns
    (P, s list, {"solve", "pade_products", "squarings", "other"} in ms);
    synchronises."""
    L = _dev(L, name="L")
    Lb = L.unsqueeze(0) if L.dim() == 2 else L
    M, n = Lb.shape[0], Lb.shape[1]
    dts = (ctypes.c_double * M)(*([float(dt)] * M if isinstance(dt, (int, float)) else [float(x) for x in dt]))
    s_host = (ctypes.c_int * M)()
    ms = (ctypes.c_double * 4)()
    P = torch.empty_like(Lb)
    _check(lib().lindblad_propagator_stages(n, M, _ptr(Lb), dts, float(theta), _ptr(P), s_host, ms, _ws(ws),
                                            _stream()))
    stages = dict(zip(("solve", "pade_products", "squarings", "other"), list(ms)))
    return (P[0] if L.dim() == 2 else P), list(s_host), stages


def propagator_noalloc(L: torch.Tensor, dt, P: torch.Tensor, theta: float = 0.25,
                       s_used: torch.Tensor | None = None, status: torch.Tensor | None = None) -> None:
    """lindblad_propagator_noalloc: the build into a caller-provided P (same
    shape as L) on the library's fixed device scratch; allocates nothing.
    `s_used` (int32, M) and `status` (int32, 1, set to 0 beforehand) are
    optional device tensors; the call returns without synchronising."""
    L = _dev(L, name="L")
    Lb = L.unsqueeze(0) if L.dim() == 2 else L
    M, n = Lb.shape[0], Lb.shape[1]
    if P.shape != L.shape or P.dtype != torch.complex128 or not P.is_contiguous():
        raise ValueError("P must be a contiguous complex128 tensor shaped like L")
    dts = (ctypes.c_double * M)(*([float(dt)] * M if isinstance(dt, (int, float)) else [float(x) for x in dt]))
    _check(lib().lindblad_propagator_noalloc(n, M, _ptr(Lb), dts, float(theta), _ptr(P),
                                             _ptr(s_used) if s_used is not None else None,
                                             _ptr(status) if status is not None else None, _stream()))


def noalloc_scratch_bytes() -> int:
    return int(lib().lindblad_propagator_noalloc_scratch_bytes())


def propagate(P: torch.Tensor, rho: torch.Tensor, nsteps: int, precision="c128", ws: Workspace | None = None):
    """rho (B, n) or (B, d, d) complex128, updated in place: rho <- P^nsteps rho."""
    P = _dev(P, name="P")
    rho = _dev(rho, name="rho")
    n = P.shape[0]
    B = rho.numel() // n
    _check(lib().lindblad_propagate(n, _ptr(P), _prec(precision), B, _ptr(rho), int(nsteps), _ws(ws), _stream()))
    return rho


def _prec(precision) -> int:
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def chain_variants(n: int, precision="c128", B: int = 1) -> list[int]:
    """Variant ids that exist for (n, precision, B)."""
    ids = (ctypes.c_int * 32)()
    cnt = ctypes.c_int()
    _check(lib().lindblad_chain_variants(int(n), _prec(precision), int(B), ids, 32, ctypes.byref(cnt)))
    return list(ids[:min(cnt.value, 32)])


def chain_variant(n: int, precision="c128", B: int = 1) -> int:
    """The variant lindblad_propagate runs for (n, precision, B) right now."""
    v = ctypes.c_int()
    _check(lib().lindblad_chain_variant(int(n), _prec(precision), int(B), ctypes.byref(v)))
    return v.value


def propagate_variant(P: torch.Tensor, rho: torch.Tensor, nsteps: int, variant: int, precision="c128",
                      ws: Workspace | None = None):
    P = _dev(P, name="P")
    rho = _dev(rho, name="rho")
    n = P.shape[0]
    B = rho.numel() // n
    _check(lib().lindblad_propagate_variant(n, _ptr(P), _prec(precision), B, _ptr(rho), int(nsteps), int(variant),
                                            _ws(ws), _stream()))
    return rho


def tune(P: torch.Tensor, rho: torch.Tensor, precision="c128", probe_steps: int = 32, repeats: int = 3,
         ws: Workspace | None = None):
    """Time every chain variant for this shape on a copy of rho and keep the
    fastest for the process.  Returns (variant id, ms per probe run)."""
    P = _dev(P, name="P")
    rho = _dev(rho, name="rho")
    n = P.shape[0]
    B = rho.numel() // n
    v, ms = ctypes.c_int(), ctypes.c_float()
    _check(lib().lindblad_tune(n, _ptr(P), _prec(precision), B, _ptr(rho), int(probe_steps), int(repeats), _ws(ws),
                               _stream(), ctypes.byref(v), ctypes.byref(ms)))
    return v.value, ms.value


def tune_set(n: int, precision, B: int, variant: int):
    """Record a variant for (n, precision, B) without timing; 0 clears."""
    _check(lib().lindblad_tune_set(int(n), _prec(precision), int(B), int(variant)))


def propagate_baseline(P: torch.Tensor, rho: torch.Tensor, nsteps: int, ws: Workspace | None = None):
    P = _dev(P, name="P")
    rho = _dev(rho, name="rho")
    n = P.shape[0]
    B = rho.numel() // n
    _check(lib().lindblad_propagate_baseline(n, _ptr(P), B, _ptr(rho), int(nsteps), _ws(ws), _stream()))
    return rho


def expmv(L: torch.Tensor, rho: torch.Tensor, t: float, nsteps: int = 1, ws: Workspace | None = None) -> int:
    """rho <- (e^{tL})^nsteps rho without forming the propagator (in place);
    returns the number of products L V per step."""
    L = _dev(L, name="L")
    rho = _dev(rho, name="rho")
    n = L.shape[0]
    B = rho.numel() // n
    prods = ctypes.c_int(0)
    _check(lib().lindblad_expmv(n, _ptr(L), float(t), B, _ptr(rho), int(nsteps), ctypes.byref(prods), _ws(ws),
                                _stream()))
    return prods.value


def expmv_params(a: float):
    """(s, m) of lindblad_expmv for ||t (L - mu I)||_1 = a (host only)."""
    s, m = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().lindblad_expmv_params(float(a), ctypes.byref(s), ctypes.byref(m)))
    return s.value, m.value


def grape_gradient(L0, Lc, u, dt, x0, w, theta=0.25, checkpoint_bytes=0, ws: Workspace | None = None):
    """Returns (F, grad (M, C) float64 on the device)."""
    L0 = _dev(L0, name="L0")
    Lc = _dev(Lc, name="Lc")
    u = _dev(u, torch.float64, "u")
    x0 = _dev(x0, name="x0")
    w = _dev(w, name="w")
    n = L0.shape[0]
    M, C = u.shape
    F = ctypes.c_double(0.0)
    grad = torch.empty((M, C), dtype=torch.float64, device=u.device)
    _check(lib().grape_gradient(n, M, C, _ptr(L0), _ptr(Lc), _ptr(u), float(dt), float(theta), _ptr(x0), _ptr(w),
                                ctypes.byref(F), _ptr(grad), int(checkpoint_bytes), _ws(ws), _stream()))
    return F.value, grad


def batch_set_window(nbytes: int = 0):
    """Propagator byte budget of the mixed batch's sliding window (0 = default)."""
    _check(lib().lindblad_batch_set_window(int(nbytes)))


def _problems(problems):
    arr = (Problem * len(problems))()
    for i, p in enumerate(problems):
        arr[i].d = int(p["d"])
        arr[i].L = _dev(p["L"], name="L").data_ptr()
        arr[i].dt = float(p["dt"])
        arr[i].nsteps = int(p["nsteps"])
        arr[i].rho = _dev(p["rho"], name="rho").data_ptr()
    return arr


def batch_run(problems, precision="c64", theta: float = 0.25, ws: Workspace | None = None):
    """problems: list of dicts with d, L (n x n tensor), dt, nsteps, rho (n tensor, updated in place)."""
    arr = _problems(problems)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().lindblad_batch_run(arr, len(problems), prec, float(theta), _ws(ws), _stream()))


def batch_enqueue(problems, precision="c64", theta: float = 0.25, status: torch.Tensor | None = None,
                  ws: Workspace | None = None):
    """lindblad_batch_enqueue: the mixed batch without host synchronisation
    (capturable into a graph); `status` an int32 device tensor set to 0 first."""
    arr = _problems(problems)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().lindblad_batch_enqueue(arr, len(problems), prec, float(theta),
                                        _ptr(status) if status is not None else None, _ws(ws), _stream()))


class GrapeFidelity(torch.autograd.Function):
    """F(u) = Re <w, x_M> with the hand-written adjoint gradient of grape_gradient."""

    @staticmethod
    def forward(ctx, u, L0, Lc, dt, x0, w, theta=0.25):
        F, grad = grape_gradient(L0, Lc, u.detach().contiguous(), dt, x0, w, theta)
        ctx.save_for_backward(grad)
        return torch.tensor(F, dtype=torch.float64, device=u.device)

    @staticmethod
    def backward(ctx, gF):
        (grad,) = ctx.saved_tensors
        return gF * grad, None, None, None, None, None, None
