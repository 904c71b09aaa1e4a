"""Python binding of the SplitSolve C ABI (include/splitsolve.h) through ctypes.

Argument marshalling only: every step of the computation runs in the HIP library
``libsplitsolve.so``.  PyTorch supplies device memory and the stream; tensors must live on the
context's GPU, be contiguous, and use complex128 (matrices), float64 (energies) or int32 (indices).
If the library is missing, importing works but every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsplitsolve.so")

SS_OK, SS_ERR_ARG, SS_ERR_NOMEM, SS_ERR_DEVICE, SS_ERR_UNSUPPORTED = range(5)
SS_MAX_S = 1024
SS_PREC_FP64, SS_PREC_FP32, SS_PREC_FP32_LU, SS_PREC_BF16 = 0, 1, 2, 3
SS_KEEP_FACTORS = 1

EXPORTS = (
    "ss_create", "ss_destroy", "ss_set_stream", "ss_set_sync_free", "ss_set_lu_width", "ss_set_lu_tile", "ss_synchronize", "ss_status_string", "ss_last_error",
    "ss_workspace_bytes", "ss_workspace_size", "ss_kernel_timer", "ss_kernel_timer_read", "ss_measure_ceilings", "ss_lead_selfenergy",
    "ss_precompute_columns", "ss_lu_factor", "ss_apply_obc", "ss_transmission", "ss_transmission_noalloc",
    "ss_injection_left", "ss_refine_psi",
    "ss_transmission_psi", "ss_plan_create", "ss_plan_execute", "ss_plan_groups", "ss_plan_lu_tile", "ss_plan_describe",
    "ss_plan_graph_nodes", "ss_plan_graph_segments", "ss_plan_destroy", "ss_mlp_param_count", "ss_mlp_forward", "ss_mlp_backward",
    "ss_mlp_adam", "ss_warm_features", "ss_sigma_moments", "ss_sigma_encode", "ss_sigma_decode",
    "ss_lead_selfenergy_warm", "ss_observables", "ss_energy_integral", "ss_precompute_columns_spike",
)


class SplitSolveError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class _Btd(ctypes.Structure):
    _fields_ = [
        ("nb", ctypes.c_int), ("s", ctypes.c_int), ("nk", ctypes.c_int),
        ("H_diag", ctypes.c_void_p), ("H_upper", ctypes.c_void_p),
        ("S_diag", ctypes.c_void_p), ("S_upper", ctypes.c_void_p),
    ]


class _Instance(ctypes.Structure):
    _fields_ = [
        ("nb", ctypes.c_int), ("s", ctypes.c_int), ("E", ctypes.c_double),
        ("H_diag", ctypes.c_void_p), ("H_upper", ctypes.c_void_p),
        ("S_diag", ctypes.c_void_p), ("S_upper", ctypes.c_void_p),
        ("H00", ctypes.c_void_p), ("H01", ctypes.c_void_p), ("S00", ctypes.c_void_p), ("S01", ctypes.c_void_p),
        ("psi", ctypes.c_void_p),
    ]


class _PlanOpts(ctypes.Structure):
    _fields_ = [
        ("eta", ctypes.c_double), ("absorb", ctypes.c_double), ("sigma_tol", ctypes.c_double),
        ("sigma_passes", ctypes.c_int),
        ("m", ctypes.c_int), ("use_graph", ctypes.c_int), ("autotune", ctypes.c_int),
        ("mem_bytes", ctypes.c_size_t), ("graph_segment_nodes", ctypes.c_int),
    ]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsplitsolve.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run `python -m paper_1812_01396_amd.build`)")
    lib = ctypes.CDLL(path)
    P, I, D, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.ss_create.argtypes = [ctypes.POINTER(P), I, P]
    lib.ss_create.restype = I
    lib.ss_destroy.argtypes = [P]
    lib.ss_destroy.restype = None
    lib.ss_set_stream.argtypes = [P, P]
    lib.ss_set_stream.restype = I
    lib.ss_set_sync_free.argtypes = [P, I]
    lib.ss_set_sync_free.restype = I
    lib.ss_set_lu_width.argtypes = [P, I]
    lib.ss_set_lu_width.restype = I
    lib.ss_set_lu_tile.argtypes = [P, I]
    lib.ss_set_lu_tile.restype = I
    lib.ss_synchronize.argtypes = [P]
    lib.ss_synchronize.restype = I
    lib.ss_status_string.argtypes = [I]
    lib.ss_status_string.restype = ctypes.c_char_p
    lib.ss_last_error.argtypes = [P]
    lib.ss_last_error.restype = ctypes.c_char_p
    lib.ss_workspace_bytes.argtypes = [P]
    lib.ss_workspace_bytes.restype = Z
    lib.ss_workspace_size.argtypes = [I, I, I, I, I, I, ctypes.POINTER(Z)]
    lib.ss_workspace_size.restype = I
    lib.ss_measure_ceilings.argtypes = [P, ctypes.POINTER(D)]
    lib.ss_measure_ceilings.restype = I
    lib.ss_kernel_timer.argtypes = [P, ctypes.c_char_p]
    lib.ss_kernel_timer.restype = I
    lib.ss_kernel_timer_read.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(D),
                                         ctypes.POINTER(D)]
    lib.ss_kernel_timer_read.restype = I
    lib.ss_lead_selfenergy.argtypes = [P, I, I, I, P, P, P, P, P, P, D, D, I, P, P, P, P]
    lib.ss_lead_selfenergy.restype = I
    lib.ss_precompute_columns.argtypes = [P, ctypes.POINTER(_Btd), I, P, P, D, I, I, P, P]
    lib.ss_precompute_columns.restype = I
    lib.ss_lu_factor.argtypes = [P, I, I, P, P, P]
    lib.ss_lu_factor.restype = I
    lib.ss_apply_obc.argtypes = [P, I, I, I, P, P, D, I, P, P, P, P]
    lib.ss_apply_obc.restype = I
    lib.ss_transmission.argtypes = [P, I, I, P, P, P]
    lib.ss_transmission.restype = I
    lib.ss_transmission_noalloc.argtypes = [P, I, I, P, P, P]
    lib.ss_transmission_noalloc.restype = I
    lib.ss_injection_left.argtypes = [P, I, I, P, D, I, P, P]
    lib.ss_injection_left.restype = I
    lib.ss_refine_psi.argtypes = [P, ctypes.POINTER(_Btd), I, P, P, P, P, I, P, P, D, I, P, P]
    lib.ss_refine_psi.restype = I
    lib.ss_transmission_psi.argtypes = [P, I, I, I, I, P, P, P, P, P]
    lib.ss_transmission_psi.restype = I
    lib.ss_plan_create.argtypes = [P, I, ctypes.POINTER(_Instance), ctypes.POINTER(_PlanOpts), P, P,
                                   ctypes.POINTER(P)]
    lib.ss_plan_create.restype = I
    lib.ss_plan_execute.argtypes = [P]
    lib.ss_plan_execute.restype = I
    lib.ss_plan_groups.argtypes = [P]
    lib.ss_plan_groups.restype = I
    lib.ss_plan_lu_tile.argtypes = [P, I]
    lib.ss_plan_lu_tile.restype = I
    lib.ss_plan_describe.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                                     ctypes.POINTER(I), ctypes.POINTER(D)]
    lib.ss_plan_describe.restype = I
    lib.ss_plan_graph_nodes.argtypes = [P]
    lib.ss_plan_graph_nodes.restype = ctypes.c_longlong
    lib.ss_plan_graph_segments.argtypes = [P]
    lib.ss_plan_graph_segments.restype = I
    lib.ss_plan_destroy.argtypes = [P]
    lib.ss_plan_destroy.restype = None
    IP = ctypes.POINTER(ctypes.c_int)
    F = ctypes.c_float
    lib.ss_mlp_param_count.argtypes = [I, IP]
    lib.ss_mlp_param_count.restype = Z
    lib.ss_mlp_forward.argtypes = [P, I, IP, P, I, P, P]
    lib.ss_mlp_forward.restype = I
    lib.ss_mlp_backward.argtypes = [P, I, IP, P, I, P, P, P, P, P]
    lib.ss_mlp_backward.restype = I
    lib.ss_mlp_adam.argtypes = [P, Z, P, P, P, P, F, F, F, F, I]
    lib.ss_mlp_adam.restype = I
    lib.ss_warm_features.argtypes = [P, I, P, P, I, D, P]
    lib.ss_warm_features.restype = I
    lib.ss_sigma_moments.argtypes = [P, I, I, P, F, P, P]
    lib.ss_sigma_moments.restype = I
    lib.ss_sigma_encode.argtypes = [P, I, I, P, P, P, P]
    lib.ss_sigma_encode.restype = I
    lib.ss_sigma_decode.argtypes = [P, I, I, P, P, P, P]
    lib.ss_sigma_decode.restype = I
    lib.ss_precompute_columns_spike.argtypes = [P, ctypes.POINTER(_Btd), I, P, P, D, I, I, P, P]
    lib.ss_precompute_columns_spike.restype = I
    lib.ss_observables.argtypes = [P, ctypes.POINTER(_Btd), I, P, P, I, P, P, P]
    lib.ss_observables.restype = I
    lib.ss_energy_integral.argtypes = [P, I, I, P, P, P]
    lib.ss_energy_integral.restype = I
    lib.ss_lead_selfenergy_warm.argtypes = [P, I, I, I, P, P, P, P, P, P, D, P, D, I, I, P, P, P, P, P]
    lib.ss_lead_selfenergy_warm.restype = I
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_kidx(kidx, nk):
    if kidx.numel() and (int(kidx.min()) < 0 or int(kidx.max()) >= nk):
        raise ValueError(f"kidx entries must lie in [0, {nk})")


def _need(t, dtype, device, name, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name}: expected a tensor on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


class Context:
    """One ss_ctx bound to a device and a stream (default: torch's current stream on that device)."""

    def __init__(self, device: int | torch.device = 0, stream: torch.cuda.Stream | None = None):
        self.lib = load_library()
        self.device = torch.device("cuda", device if isinstance(device, int) else device.index or 0)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.ss_create(ctypes.byref(h), self.device.index, ctypes.c_void_p(stream.cuda_stream))
        if st != SS_OK:
            raise SplitSolveError(st, "ss_create failed")
        self.handle = h
        self._plans = weakref.WeakSet()  # plans built on this context are closed before it

    def close(self):
        for p in list(getattr(self, "_plans", ())):
            p.close()
        if getattr(self, "handle", None):
            self.lib.ss_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int):
        if st != SS_OK:
            msg = self.lib.ss_last_error(self.handle).decode()
            raise SplitSolveError(st, f"{self.lib.ss_status_string(st).decode()}: {msg}")

    def set_sync_free(self, on: bool):
        """Never wait for the stream inside a call (for stream/graph capture)."""
        self.check(self.lib.ss_set_sync_free(self.handle, int(bool(on))))

    def set_lu_width(self, width: int):
        """LU panel width for this context's factorizations (0: the default by order)."""
        self.check(self.lib.ss_set_lu_width(self.handle, int(width)))

    def set_lu_tile(self, tile: int):
        """Tile of the LU's general block products for this context: 0 64 x 64 (default), 1 32 x 64."""
        self.check(self.lib.ss_set_lu_tile(self.handle, int(tile)))

    def synchronize(self):
        self.check(self.lib.ss_synchronize(self.handle))

    def workspace_bytes(self) -> int:
        return int(self.lib.ss_workspace_bytes(self.handle))

    def measure_ceilings(self) -> dict:
        """Measured FP64/FP32 matrix-core, FP64 vector and copy rates of this GPU (ss_measure_ceilings)."""
        out = (ctypes.c_double * 4)()
        self.check(self.lib.ss_measure_ceilings(self.handle, out))
        return dict(fp64_mfma_tflops=out[0], fp32_mfma_tflops=out[1], fp64_valu_tflops=out[2], copy_gbps=out[3])

    def kernel_timer(self, family: str | None):
        """Start (or with None stop) bracketing launches of one kernel family with HIP events."""
        self.check(self.lib.ss_kernel_timer(self.handle, family.encode() if family else None))

    def kernel_timer_read(self, with_flops: bool = False):
        """(summed milliseconds, launches[, stated flops, stated bytes]) of the timed family since the last
        read."""
        ms, n, fl, by = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
        self.check(self.lib.ss_kernel_timer_read(self.handle, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl),
                                                 ctypes.byref(by)))
        return (ms.value, n.value, fl.value, by.value) if with_flops else (ms.value, n.value)


def ss_lead_selfenergy(ctx: Context, H00, H01, S00, S01, E, eta: float, tol: float = 0.0, max_iter: int = 0,
                       kidx=None, sigma=None, iters=None, resid=None, info=None, validate: bool = True):
    """Sigma_L and Sigma_R of the lead cell(s) at energies E (see ss_lead_selfenergy in splitsolve.h).

    H00..S01: [nk, s, s] (or [s, s]) complex128; E: [batch] float64.  Returns (sigma [batch, 2, s, s],
    iters [batch] int32, resid [batch, 2] float64, info [batch] int32), all on the device.
    """
    dev = ctx.device
    if H00.dim() == 2:
        H00, H01, S00, S01 = (x.unsqueeze(0) for x in (H00, H01, S00, S01))
    nk, s, _ = H00.shape
    for name, t in (("H00", H00), ("H01", H01), ("S00", S00), ("S01", S01)):
        _need(t, torch.complex128, dev, name, (nk, s, s))
    _need(E, torch.float64, dev, "E")
    batch = E.numel()
    if kidx is not None:
        _need(kidx, torch.int32, dev, "kidx", (batch,))
        if validate:  # reads kidx back to the host (a stream synchronization)
            _check_kidx(kidx, nk)
    sigma = sigma if sigma is not None else torch.empty(batch, 2, s, s, dtype=torch.complex128, device=dev)
    iters = iters if iters is not None else torch.empty(batch, dtype=torch.int32, device=dev)
    resid = resid if resid is not None else torch.empty(batch, 2, dtype=torch.float64, device=dev)
    info = info if info is not None else torch.empty(batch, dtype=torch.int32, device=dev)
    _need(sigma, torch.complex128, dev, "sigma", (batch, 2, s, s))
    ctx.check(ctx.lib.ss_lead_selfenergy(
        ctx.handle, batch, s, nk, _ptr(H00), _ptr(H01), _ptr(S00), _ptr(S01), _ptr(kidx), _ptr(E),
        float(eta), float(tol), int(max_iter), _ptr(sigma), _ptr(iters), _ptr(resid), _ptr(info)))
    return sigma, iters, resid, info


def _btd(Hd, Hu, Sd, Su, dev):
    if Hd.dim() == 3:
        Hd, Hu, Sd, Su = (x.unsqueeze(0) for x in (Hd, Hu, Sd, Su))
    nk, nb, s, _ = Hd.shape
    _need(Hd, torch.complex128, dev, "Hd", (nk, nb, s, s))
    _need(Sd, torch.complex128, dev, "Sd", (nk, nb, s, s))
    _need(Hu, torch.complex128, dev, "Hu", (nk, nb - 1, s, s))
    _need(Su, torch.complex128, dev, "Su", (nk, nb - 1, s, s))
    btd = _Btd(nb, s, nk, Hd.data_ptr(), Hu.data_ptr() if nb > 1 else 0, Sd.data_ptr(),
               Su.data_ptr() if nb > 1 else 0)
    return btd, nk, nb, s


def ss_precompute_columns(ctx: Context, Hd, Hu, Sd, Su, E, kidx=None, Q=None, info=None, validate: bool = True,
                          prec: int = SS_PREC_FP64, keep_factors: bool = False, absorb: float = 0.0):
    """Q = first and last block columns of (E S - H)^{-1} for every instance (Sec. 3B, Step 1).

    Hd, Sd: [nk, nb, s, s]; Hu, Su: [nk, nb-1, s, s] (or without the leading nk).  E: [batch] float64.
    prec: SS_PREC_FP64, SS_PREC_FP32, SS_PREC_FP32_LU or SS_PREC_BF16 (products of the recursion); keep_factors keeps the first-column
    recursion's factors in the context for ss_refine_psi; absorb: absorbing boundary (i*absorb*I on the
    first and last diagonal blocks; pass the same value to ss_apply_obc).  Returns (Q [batch, nb, s, 2s],
    info [batch]).
    """
    dev = ctx.device
    btd, nk, nb, s = _btd(Hd, Hu, Sd, Su, dev)
    _need(E, torch.float64, dev, "E")
    batch = E.numel()
    if kidx is not None:
        _need(kidx, torch.int32, dev, "kidx", (batch,))
        if validate:  # reads kidx back to the host (a stream synchronization)
            _check_kidx(kidx, nk)
    Q = Q if Q is not None else torch.empty(batch, nb, s, 2 * s, dtype=torch.complex128, device=dev)
    info = info if info is not None else torch.empty(batch, dtype=torch.int32, device=dev)
    _need(Q, torch.complex128, dev, "Q", (batch, nb, s, 2 * s))
    flags = SS_KEEP_FACTORS if keep_factors else 0
    ctx.check(ctx.lib.ss_precompute_columns(ctx.handle, ctypes.byref(btd), batch, _ptr(kidx), _ptr(E), float(absorb),
                                            int(prec), flags, _ptr(Q), _ptr(info)))
    return Q, info


def ss_lu_factor(ctx: Context, A, perm=None, info=None):
    """Batched LU with partial pivoting, in place (see ss_lu_factor in splitsolve.h).

    A: [nmat, n, n] complex128 (overwritten with L and U of P A = L U, getrf layout).  Returns
    (A, perm [nmat, n] int32, info [nmat] int32), all on the device.
    """
    dev = ctx.device
    nmat, n, n2 = A.shape
    _need(A, torch.complex128, dev, "A", (nmat, n, n))
    perm = perm if perm is not None else torch.empty(nmat, n, dtype=torch.int32, device=dev)
    info = info if info is not None else torch.empty(nmat, dtype=torch.int32, device=dev)
    _need(perm, torch.int32, dev, "perm", (nmat, n))
    _need(info, torch.int32, dev, "info", (nmat,))
    ctx.check(ctx.lib.ss_lu_factor(ctx.handle, nmat, n, _ptr(A), _ptr(perm), _ptr(info)))
    return A, perm, info


def ss_apply_obc(ctx: Context, Q, sigma, inj=None, psi=None, gc=None, info=None, want_gc: bool = True,
                 absorb: float = 0.0):
    """Steps 2-4 (Sec. 3B, Eq. (x)): psi = Q (b' + z) and the corner of G^R.

    Q: [batch, nb, s, 2s] from ss_precompute_columns with the same absorb; sigma: [batch, 2, s, s];
    inj = b': [batch, 2s, m] or None.
    Returns (psi [batch, nb, s, m] or None, gc [batch, 2s, 2s] or None, info [batch] int32).
    """
    dev = ctx.device
    batch, nb, s, s2 = Q.shape
    _need(Q, torch.complex128, dev, "Q", (batch, nb, s, 2 * s))
    _need(sigma, torch.complex128, dev, "sigma", (batch, 2, s, s))
    m = 0
    if inj is not None:
        m = inj.shape[-1]
        _need(inj, torch.complex128, dev, "inj", (batch, 2 * s, m))
        psi = psi if psi is not None else torch.empty(batch, nb, s, m, dtype=torch.complex128, device=dev)
        _need(psi, torch.complex128, dev, "psi", (batch, nb, s, m))
    if want_gc:
        gc = gc if gc is not None else torch.empty(batch, 2 * s, 2 * s, dtype=torch.complex128, device=dev)
        _need(gc, torch.complex128, dev, "gc", (batch, 2 * s, 2 * s))
    info = info if info is not None else torch.empty(batch, dtype=torch.int32, device=dev)
    ctx.check(ctx.lib.ss_apply_obc(ctx.handle, batch, nb, s, _ptr(Q), _ptr(sigma), float(absorb), m, _ptr(inj), _ptr(psi),
                                   _ptr(gc) if want_gc else None, _ptr(info)))
    return (psi if m > 0 else None), (gc if want_gc else None), info


def ss_transmission(ctx: Context, gc, sigma, T=None):
    """Caroli T_LR, T_RL from the corner of G^R.  Returns T [batch, 2] float64."""
    dev = ctx.device
    batch, n2, _ = gc.shape
    s = n2 // 2
    _need(gc, torch.complex128, dev, "gc", (batch, 2 * s, 2 * s))
    _need(sigma, torch.complex128, dev, "sigma", (batch, 2, s, s))
    T = T if T is not None else torch.empty(batch, 2, dtype=torch.float64, device=dev)
    _need(T, torch.float64, dev, "T", (batch, 2))
    ctx.check(ctx.lib.ss_transmission(ctx.handle, batch, s, _ptr(gc), _ptr(sigma), _ptr(T)))
    return T


def ss_transmission_noalloc(ctx: Context, gc, sigma, T):
    """ss_transmission through the library's fixed per-device scratch (no device allocation by the
    library; T [batch, 2] float64 must be given).  Returns T."""
    dev = ctx.device
    batch, n2, _ = gc.shape
    s = n2 // 2
    _need(gc, torch.complex128, dev, "gc", (batch, 2 * s, 2 * s))
    _need(sigma, torch.complex128, dev, "sigma", (batch, 2, s, s))
    _need(T, torch.float64, dev, "T", (batch, 2))
    ctx.check(ctx.lib.ss_transmission_noalloc(ctx.handle, batch, s, _ptr(gc), _ptr(sigma), _ptr(T)))
    return T


def ss_injection_left(ctx: Context, sigma, mmax: int, tol: float = 0.0, inj=None, rank=None):
    """b' = [W_L; 0] with W_L W_L^H ~ Gamma_L (pivoted Cholesky).  Returns (inj [batch, 2s, mmax], rank [batch])."""
    dev = ctx.device
    batch, _, s, _ = sigma.shape
    _need(sigma, torch.complex128, dev, "sigma", (batch, 2, s, s))
    inj = inj if inj is not None else torch.empty(batch, 2 * s, mmax, dtype=torch.complex128, device=dev)
    rank = rank if rank is not None else torch.empty(batch, dtype=torch.int32, device=dev)
    _need(inj, torch.complex128, dev, "inj", (batch, 2 * s, mmax))
    ctx.check(ctx.lib.ss_injection_left(ctx.handle, batch, s, _ptr(sigma), float(tol), int(mmax), _ptr(inj),
                                        _ptr(rank)))
    return inj, rank


def ss_refine_psi(ctx: Context, Hd, Hu, Sd, Su, E, Q, sigma, inj, psi, kidx=None, tol: float = 0.0,
                  max_iter: int = 0, iters=None, resid=None):
    """Refine psi in place on the full system (kept factors of the last precompute with keep_factors and
    the corner factorization of the last ss_apply_obc on this context).  Returns (psi, iters, resid)."""
    dev = ctx.device
    btd, nk, nb, s = _btd(Hd, Hu, Sd, Su, dev)
    batch = E.numel()
    m = inj.shape[-1]
    _need(E, torch.float64, dev, "E")
    _need(Q, torch.complex128, dev, "Q", (batch, nb, s, 2 * s))
    _need(sigma, torch.complex128, dev, "sigma", (batch, 2, s, s))
    _need(inj, torch.complex128, dev, "inj", (batch, 2 * s, m))
    _need(psi, torch.complex128, dev, "psi", (batch, nb, s, m))
    if kidx is not None:
        _need(kidx, torch.int32, dev, "kidx", (batch,))
    iters = iters if iters is not None else torch.empty(batch, dtype=torch.int32, device=dev)
    resid = resid if resid is not None else torch.empty(batch, dtype=torch.float64, device=dev)
    ctx.check(ctx.lib.ss_refine_psi(ctx.handle, ctypes.byref(btd), batch, _ptr(kidx), _ptr(E), _ptr(Q),
                                    _ptr(sigma), m, _ptr(inj), _ptr(psi), float(tol), int(max_iter), _ptr(iters),
                                    _ptr(resid)))
    return psi, iters, resid


def ss_transmission_psi(ctx: Context, psi, sigma, T=None, psi0=None, gc=None):
    """T = Re Tr[psi_nb^H Gamma_R psi_nb] for psi injected from the left; with psi0 (the last block row of
    the unrefined psi, [batch, s, m]) and gc (the corner of G^R that came with it) the part of Gamma_L
    outside the injection factor is added back (see splitsolve.h).  Returns T [batch] float64."""
    dev = ctx.device
    batch, nb, s, m = psi.shape
    _need(psi, torch.complex128, dev, "psi")
    _need(sigma, torch.complex128, dev, "sigma", (batch, 2, s, s))
    if (psi0 is None) != (gc is None):
        raise ValueError("psi0 and gc are given together or not at all")
    if psi0 is not None:
        _need(psi0, torch.complex128, dev, "psi0", (batch, s, m))
        _need(gc, torch.complex128, dev, "gc", (batch, 2 * s, 2 * s))
    T = T if T is not None else torch.empty(batch, dtype=torch.float64, device=dev)
    ctx.check(ctx.lib.ss_transmission_psi(ctx.handle, batch, nb, s, m, _ptr(psi), _ptr(sigma), _ptr(psi0),
                                          _ptr(gc), _ptr(T)))
    return T


class Instance:
    """One (E, k) instance of an uneven batch: device tensors of its blocks and lead cell.

    Hd [nb][s][s], Hu [nb-1][s][s], Sd, Su likewise; H00, H01, S00, S01 [s][s]; psi [nb][s][m] or None.
    """

    def __init__(self, Hd, Hu, Sd, Su, H00, H01, S00, S01, E, psi=None):
        self.Hd, self.Hu, self.Sd, self.Su = Hd, Hu, Sd, Su
        self.H00, self.H01, self.S00, self.S01 = H00, H01, S00, S01
        self.E = float(E)
        self.psi = psi
        self.nb, self.s = int(Hd.shape[0]), int(Hd.shape[1])


class Plan:
    """ss_plan over a list of Instance objects; keeps every tensor it was built from alive.

    T [n][2] float64 and info [n][4] int32 (device: self-energy, Step 1 and corner codes, decimation
    passes) are written by every ``execute()``.
    """

    def __init__(self, ctx: Context, instances, eta: float, m: int = 0, use_graph: bool = True,
                 autotune: bool = True, sigma_tol: float = 0.0, sigma_passes: int = 0, mem_bytes: int = 0,
                 absorb: float = 0.0, graph_segment_nodes: int = 0):
        dev = ctx.device
        n = len(instances)
        if n < 1:
            raise ValueError("a plan needs at least one instance")
        arr = (_Instance * n)()
        for i, x in enumerate(instances):
            nb, s = x.nb, x.s
            if s < 1 or s > SS_MAX_S or nb < 1:
                raise ValueError(f"instance {i}: unsupported sizes nb={nb}, s={s}")
            _need(x.Hd, torch.complex128, dev, f"instance {i} Hd", (nb, s, s))
            _need(x.Sd, torch.complex128, dev, f"instance {i} Sd", (nb, s, s))
            _need(x.Hu, torch.complex128, dev, f"instance {i} Hu", (nb - 1, s, s))
            _need(x.Su, torch.complex128, dev, f"instance {i} Su", (nb - 1, s, s))
            for nm in ("H00", "H01", "S00", "S01"):
                _need(getattr(x, nm), torch.complex128, dev, f"instance {i} {nm}", (s, s))
            if x.psi is not None:
                if m < 1:
                    raise ValueError("psi requested with m = 0")
                _need(x.psi, torch.complex128, dev, f"instance {i} psi", (nb, s, m))
            arr[i] = _Instance(nb, s, x.E, x.Hd.data_ptr(), x.Hu.data_ptr() if nb > 1 else None, x.Sd.data_ptr(),
                               x.Su.data_ptr() if nb > 1 else None, x.H00.data_ptr(), x.H01.data_ptr(),
                               x.S00.data_ptr(), x.S01.data_ptr(), None if x.psi is None else x.psi.data_ptr())
        opts = _PlanOpts(float(eta), float(absorb), float(sigma_tol), int(sigma_passes), int(m), int(bool(use_graph)),
                         int(bool(autotune)), int(mem_bytes), int(graph_segment_nodes))
        self.ctx = ctx
        self.instances = list(instances)
        self.T = torch.zeros(n, 2, dtype=torch.float64, device=dev)
        self.info = torch.zeros(n, 4, dtype=torch.int32, device=dev)
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.ss_plan_create(ctx.handle, n, arr, ctypes.byref(opts), _ptr(self.T), _ptr(self.info),
                                         ctypes.byref(h)))
        self.handle = h
        ctx._plans.add(self)

    def execute(self):
        self.ctx.check(self.ctx.lib.ss_plan_execute(self.handle))

    @property
    def graph_nodes(self) -> int:
        return int(self.ctx.lib.ss_plan_graph_nodes(self.handle))

    @property
    def graph_segments(self) -> int:
        return int(self.ctx.lib.ss_plan_graph_segments(self.handle))

    def groups(self):
        """Per group: dict(s, count, chunk, lu_width, lu_tile, tune_ms)."""
        out = []
        lib = self.ctx.lib
        for g in range(lib.ss_plan_groups(self.handle)):
            s, c, ch, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            ms = ctypes.c_double()
            self.ctx.check(lib.ss_plan_describe(self.handle, g, ctypes.byref(s), ctypes.byref(c), ctypes.byref(ch),
                                                ctypes.byref(w), ctypes.byref(ms)))
            out.append(dict(s=s.value, count=c.value, chunk=ch.value, lu_width=w.value,
                            lu_tile=int(lib.ss_plan_lu_tile(self.handle, g)), tune_ms=ms.value))
        return out

    def close(self):
        if getattr(self, "handle", None):
            self.ctx.lib.ss_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned warm start


def _dims_arg(dims):
    arr = (ctypes.c_int * len(dims))(*[int(d) for d in dims])
    return len(dims) - 1, arr


class MLP:
    """FP32 perceptron on the GPU (tanh hidden layers, linear output) trained with the library's kernels.

    ``params`` packs W_l [dims[l]][dims[l+1]] then b_l per layer (see ss_mlp_param_count)."""

    def __init__(self, ctx: Context, dims, params=None, seed: int = 0):
        self.ctx, self.dims = ctx, [int(d) for d in dims]
        self.nl, self._dims = _dims_arg(self.dims)
        count = int(ctx.lib.ss_mlp_param_count(self.nl, self._dims))
        if count == 0:
            raise ValueError(f"invalid layer sizes {dims}")
        self.count = count
        dev = ctx.device
        if params is None:
            g = torch.Generator(device="cpu").manual_seed(seed)
            chunks = []
            for i in range(self.nl):
                chunks.append((torch.randn(self.dims[i] * self.dims[i + 1], generator=g, dtype=torch.float64)
                               / self.dims[i] ** 0.5).float())
                chunks.append(torch.zeros(self.dims[i + 1], dtype=torch.float32))
            params = torch.cat(chunks).to(dev)
        self.params = _need(params, torch.float32, dev, "params", (count,))
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)

    def acts_size(self, n: int) -> int:
        return n * sum(self.dims[1:])

    def forward(self, X, acts=None):
        """Every layer's output in one flat FP32 tensor; returns (acts, output view [n][dims[-1]])."""
        n = int(X.shape[0])
        _need(X, torch.float32, self.ctx.device, "X", (n, self.dims[0]))
        if acts is None:
            acts = torch.empty(self.acts_size(n), dtype=torch.float32, device=self.ctx.device)
        self.ctx.check(self.ctx.lib.ss_mlp_forward(self.ctx.handle, self.nl, self._dims, _ptr(self.params), n, _ptr(X),
                                                   _ptr(acts)))
        out = acts[n * sum(self.dims[1:-1]):].view(n, self.dims[-1])
        return acts, out

    def backward(self, X, acts, target):
        n = int(X.shape[0])
        _need(target, torch.float32, self.ctx.device, "target", (n, self.dims[-1]))
        self.ctx.check(self.ctx.lib.ss_mlp_backward(self.ctx.handle, self.nl, self._dims, _ptr(self.params), n, _ptr(X),
                                                    _ptr(acts), _ptr(target), _ptr(self.grads), _ptr(self.loss)))
        return self.loss

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        self.ctx.check(self.ctx.lib.ss_mlp_adam(self.ctx.handle, self.count, _ptr(self.params), _ptr(self.grads),
                                                _ptr(self.m), _ptr(self.v), lr, beta1, beta2, eps, self.step))


def ss_warm_features(ctx: Context, E, k, nfreq: int = 8, e_scale: float = 5.0, X=None):
    n = int(E.numel())
    _need(E, torch.float64, ctx.device, "E")
    _need(k, torch.float64, ctx.device, "k", (n,))
    if X is None:
        X = torch.empty(n, 3 + 4 * nfreq, dtype=torch.float32, device=ctx.device)
    ctx.check(ctx.lib.ss_warm_features(ctx.handle, n, _ptr(E), _ptr(k), nfreq, e_scale, _ptr(X)))
    return X


def ss_sigma_moments(ctx: Context, sigma, std_floor: float = 0.0):
    n, _, s, _ = sigma.shape
    _need(sigma, torch.complex128, ctx.device, "sigma", (n, 2, s, s))
    mean = torch.empty(4 * s * s, dtype=torch.float32, device=ctx.device)
    std = torch.empty_like(mean)
    ctx.check(ctx.lib.ss_sigma_moments(ctx.handle, n, s, _ptr(sigma), std_floor, _ptr(mean), _ptr(std)))
    return mean, std


def ss_sigma_encode(ctx: Context, sigma, mean, std, y=None):
    n, _, s, _ = sigma.shape
    _need(sigma, torch.complex128, ctx.device, "sigma", (n, 2, s, s))
    if y is None:
        y = torch.empty(n, 4 * s * s, dtype=torch.float32, device=ctx.device)
    ctx.check(ctx.lib.ss_sigma_encode(ctx.handle, n, s, _ptr(sigma), _ptr(mean), _ptr(std), _ptr(y)))
    return y


def ss_sigma_decode(ctx: Context, y, mean, std, s: int, sigma=None):
    n = int(y.shape[0])
    _need(y, torch.float32, ctx.device, "y", (n, 4 * s * s))
    if sigma is None:
        sigma = torch.empty(n, 2, s, s, dtype=torch.complex128, device=ctx.device)
    ctx.check(ctx.lib.ss_sigma_decode(ctx.handle, n, s, _ptr(y), _ptr(mean), _ptr(std), _ptr(sigma)))
    return sigma


def ss_lead_selfenergy_warm(ctx: Context, H00, H01, S00, S01, E, eta: float, sigma_init, kidx=None, tol: float = 0.0,
                            max_newton: int = 0, smith_steps: int = 0, sigma=None):
    """Warm-started Sigma (see ss_lead_selfenergy_warm); returns (sigma, newton_iters, dec_iters, resid, info)."""
    nk, s, _ = H00.shape
    batch = int(E.numel())
    dev = ctx.device
    for nm, t in (("H00", H00), ("H01", H01), ("S00", S00), ("S01", S01)):
        _need(t, torch.complex128, dev, nm, (nk, s, s))
    _need(E, torch.float64, dev, "E", (batch,))
    _need(sigma_init, torch.complex128, dev, "sigma_init", (batch, 2, s, s))
    if kidx is not None:
        _need(kidx, torch.int32, dev, "kidx", (batch,))
        _check_kidx(kidx, nk)
    if sigma is None:
        sigma = torch.empty(batch, 2, s, s, dtype=torch.complex128, device=dev)
    it_n = torch.zeros(batch, dtype=torch.int32, device=dev)
    it_d = torch.zeros(batch, dtype=torch.int32, device=dev)
    resid = torch.zeros(batch, 2, dtype=torch.float64, device=dev)
    info = torch.zeros(batch, dtype=torch.int32, device=dev)
    ctx.check(ctx.lib.ss_lead_selfenergy_warm(ctx.handle, batch, s, nk, _ptr(H00), _ptr(H01), _ptr(S00), _ptr(S01),
                                              _ptr(kidx), _ptr(E), eta, _ptr(sigma_init), tol, max_newton, smith_steps,
                                              _ptr(sigma), _ptr(it_n), _ptr(it_d), _ptr(resid), _ptr(info)))
    return sigma, it_n, it_d, resid, info


def ss_observables(ctx: Context, Hd, Hu, Sd, Su, E, psi, kidx=None, density=True, current=True):
    """Orbital density [batch, nb, s] and bond currents [batch, nb - 1] of psi (see ss_observables in
    splitsolve.h); either may be switched off (None returned)."""
    dev = ctx.device
    btd, nk, nb, s = _btd(Hd, Hu, Sd, Su, dev)
    batch = E.numel()
    m = psi.shape[-1]
    _need(E, torch.float64, dev, "E")
    _need(psi, torch.complex128, dev, "psi", (batch, nb, s, m))
    if kidx is not None:
        _need(kidx, torch.int32, dev, "kidx", (batch,))
    dens = torch.empty(batch, nb, s, dtype=torch.float64, device=dev) if density else None
    cur = torch.empty(batch, max(nb - 1, 0), dtype=torch.float64, device=dev) if current else None
    ctx.check(ctx.lib.ss_observables(ctx.handle, ctypes.byref(btd), batch, _ptr(kidx), _ptr(E), m, _ptr(psi),
                                     _ptr(dens), _ptr(cur) if (cur is not None and nb > 1) else None))
    return dens, cur


def ss_energy_integral(ctx: Context, w, x, out=None):
    """out[j] = sum_b w[b] x[b, j] (x [batch, ...] float64, summed over the leading axis)."""
    dev = ctx.device
    batch = x.shape[0]
    n = int(x[0].numel()) if batch > 0 else 0
    _need(w, torch.float64, dev, "w", (batch,))
    _need(x, torch.float64, dev, "x")
    out = out if out is not None else torch.empty(x.shape[1:], dtype=torch.float64, device=dev)
    ctx.check(ctx.lib.ss_energy_integral(ctx.handle, batch, n, _ptr(w), _ptr(x), _ptr(out)))
    return out


def ss_precompute_columns_spike(ctx: Context, Hd, Hu, Sd, Su, E, nparts: int, kidx=None, Q=None, info=None,
                                prec: int = SS_PREC_FP64, absorb: float = 0.0):
    """Q as ss_precompute_columns, through nparts partitions per instance and their recursive SPIKE merge
    (see splitsolve.h).  Returns (Q [batch, nb, s, 2s], info [batch])."""
    dev = ctx.device
    btd, nk, nb, s = _btd(Hd, Hu, Sd, Su, dev)
    batch = E.numel()
    _need(E, torch.float64, dev, "E")
    if kidx is not None:
        _need(kidx, torch.int32, dev, "kidx", (batch,))
        _check_kidx(kidx, nk)
    Q = Q if Q is not None else torch.empty(batch, nb, s, 2 * s, dtype=torch.complex128, device=dev)
    _need(Q, torch.complex128, dev, "Q", (batch, nb, s, 2 * s))
    info = info if info is not None else torch.empty(batch, dtype=torch.int32, device=dev)
    ctx.check(ctx.lib.ss_precompute_columns_spike(ctx.handle, ctypes.byref(btd), batch, _ptr(kidx), _ptr(E),
                                                  float(absorb), int(prec), int(nparts), _ptr(Q), _ptr(info)))
    return Q, info


def ss_workspace_size(batch: int, nb: int, s: int, m: int = 0, prec: int = SS_PREC_FP64, flags: int = 0) -> int:
    """Device workspace a fresh context holds after one pass of the four steps at these sizes (see
    ss_workspace_size in splitsolve.h).  Host-only: needs the library, not a GPU."""
    lib = load_library()
    out = ctypes.c_size_t()
    st = lib.ss_workspace_size(int(batch), int(nb), int(s), int(m), int(prec), int(flags), ctypes.byref(out))
    if st != SS_OK:
        raise SplitSolveError(st, "ss_workspace_size: argument out of range")
    return int(out.value)
