"""Python binding of libannkin.so (ctypes).

Argument marshalling only: every step of the source-term evaluation runs in
the library's HIP kernels.  PyTorch provides device memory (CUDA/HIP tensors)
and the current stream.  There is no CPU fallback: if the library or a GPU is
missing, these functions raise.

Layouts follow the C ABI (``include/annkin.h``): T and P are [n] tensors, Y
and omega are [NS, n] tensors with the cell index fastest (row stride = the
leading dimension ld >= n).
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libannkin.so")

AK_FP64 = 0
AK_FP32 = 1
_ERRORS = {-1: "AK_EINVAL", -2: "AK_EDEVICE", -3: "AK_ENOMEM", -4: "AK_E2BIG",
           -5: "AK_ETIMEDOUT", -6: "AK_ECANCELED", -7: "AK_EUNSUPPORTED"}

_lib = None


class AnnkinError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class MechanismDesc(C.Structure):
    _fields_ = [
        ("n_species", C.c_int32), ("n_reactions", C.c_int32),
        ("W", C.c_void_p), ("nu_f", C.c_void_p), ("nu_r", C.c_void_p),
        ("ln_A", C.c_void_p), ("beta", C.c_void_p), ("Ea", C.c_void_p),
        ("nasa_low", C.c_void_p), ("nasa_high", C.c_void_p), ("T_mid", C.c_void_p),
        ("reversible", C.c_void_p), ("rtype", C.c_void_p), ("efficiency", C.c_void_p),
        ("low_ln_A", C.c_void_p), ("low_beta", C.c_void_p), ("low_Ea", C.c_void_p),
        ("troe", C.c_void_p),
    ]


class KcNetDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("n_hidden", C.c_int32), ("n_out", C.c_int32),
                ("pad", C.c_int32), ("weights", C.c_void_p), ("biases", C.c_void_p),
                ("x_mean", C.c_double), ("x_std", C.c_double), ("y_mean", C.c_void_p),
                ("y_std", C.c_void_p)]


class ServerConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_inflight", C.c_int32),
                ("max_batch_requests", C.c_int32), ("batching", C.c_int32),
                ("max_batch_cells", C.c_int64), ("arena_bytes", C.c_size_t),
                ("small_request_cells", C.c_int64), ("arena", C.c_void_p)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("cancelled", C.c_int64),
                ("failed", C.c_int64), ("batches", C.c_int64), ("launches", C.c_int64),
                ("cells", C.c_int64), ("queue_depth", C.c_int64), ("inflight", C.c_int32),
                ("pad", C.c_int32), ("arena_bytes", C.c_size_t), ("arena_used", C.c_size_t),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("max_ms", C.c_double), ("cells_per_s", C.c_double)]


def lib():
    """Load libannkin.so (fails loudly if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2008_08483_amd.build`")
        h = C.CDLL(LIB_PATH)
        h.ak_last_error.restype = C.c_char_p
        h.ak_version.restype = C.c_char_p
        h.ak_load_mechanism.argtypes = [C.POINTER(MechanismDesc), C.c_int, C.POINTER(C.c_void_p)]
        h.ak_load_mechanism_ex.argtypes = [C.POINTER(MechanismDesc), C.c_int, C.c_int,
                                           C.POINTER(C.c_void_p)]
        h.ak_mechanism_compiled.argtypes = [C.c_void_p, C.c_int]
        h.ak_jit_source.argtypes = [C.POINTER(MechanismDesc), C.c_int, C.c_char_p, C.c_size_t,
                                    C.POINTER(C.c_size_t)]
        h.ak_jit_tables.argtypes = [C.POINTER(MechanismDesc), C.c_int, C.c_void_p, C.c_size_t,
                                    C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t),
                                    C.POINTER(C.c_size_t)]
        h.ak_jit_jacobian_source.argtypes = [C.POINTER(MechanismDesc), C.c_int, C.c_int,
                                             C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
        h.ak_jit_jacobian_tables.argtypes = [C.POINTER(MechanismDesc), C.c_void_p, C.c_size_t,
                                             C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t),
                                             C.POINTER(C.c_size_t)]
        h.ak_integrate_euler.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_int64, C.c_int64, C.c_double, C.c_int,
                                         C.c_void_p]
        h.ak_integrate_implicit.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_int64, C.c_int64, C.c_double,
                                            C.c_int, C.c_void_p]
        h.ak_free_mechanism.argtypes = [C.c_void_p]
        h.ak_mechanism_n_species.argtypes = [C.c_void_p]
        h.ak_mechanism_n_reactions.argtypes = [C.c_void_p]
        h.ak_eval_source.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
        h.ak_error_count.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]
        h.ak_mechanism_compiled_jacobian.argtypes = [C.c_void_p, C.c_int]
        h.ak_eval_jacobian_interleaved.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                                   C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                                   C.c_int64, C.c_void_p]
        h.ak_eval_jacobian.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
        h.ak_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]
        h.ak_server_submit.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                                       C.POINTER(C.c_void_p)]
        h.ak_request_wait.argtypes = [C.c_void_p, C.c_double]
        h.ak_request_cancel.argtypes = [C.c_void_p]
        h.ak_request_free.argtypes = [C.c_void_p]
        h.ak_server_get_stats.argtypes = [C.c_void_p, C.POINTER(ServerStats)]
        h.ak_server_reset_stats.argtypes = [C.c_void_p]
        h.ak_server_destroy.argtypes = [C.c_void_p]
        h.ak_eval_vjp.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                  C.c_int64, C.c_void_p, C.c_void_p]
        h.ak_eval_lnkc.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int64, C.c_void_p,
                                   C.c_int64, C.c_void_p]
        h.ak_load_kcnet.argtypes = [C.POINTER(KcNetDesc), C.c_int, C.POINTER(C.c_void_p)]
        h.ak_free_kcnet.argtypes = [C.c_void_p]
        h.ak_kcnet_n_out.argtypes = [C.c_void_p]
        h.ak_eval_lnkc_net.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int64, C.c_void_p,
                                       C.c_int64, C.c_void_p]
        h.ak_eval_source_lnkc.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                          C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
        h.ak_eval_production.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                         C.c_void_p, C.c_int64, C.c_void_p]
        h.ak_eval_source_net.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                         C.c_void_p, C.c_int64, C.c_void_p]
        h.ak_integrate_euler_net.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                             C.c_double, C.c_int, C.c_void_p]
        _lib = h
    return _lib


def _check(rc: int):
    if rc != 0:
        raise AnnkinError(rc, lib().ak_last_error().decode())


def _torch():
    import torch
    return torch


AK_KERNEL_AUTO = 0
AK_KERNEL_TABLE = 1
_KERNELS = {"auto": AK_KERNEL_AUTO, "table": AK_KERNEL_TABLE}


def _desc(src):
    """(MechanismDesc, arrays it points into) for a mechanism-like object.
    Pressure-dependent reactions (Sec. 2.4) come from the optional
    attributes rtype, eff, low_ln_A, low_beta, low_Ea and troe."""
    nr, ns = int(src.nu_f.shape[0]), int(src.W.shape[0])
    keep = {
        "W": np.ascontiguousarray(src.W, np.float64),
        "nu_f": np.ascontiguousarray(src.nu_f, np.int8),
        "nu_r": np.ascontiguousarray(src.nu_r, np.int8),
        "ln_A": np.ascontiguousarray(src.ln_A, np.float64),
        "beta": np.ascontiguousarray(src.beta, np.float64),
        "Ea": np.ascontiguousarray(src.Ea, np.float64),
        "nasa_low": np.ascontiguousarray(src.nasa_low, np.float64),
        "nasa_high": np.ascontiguousarray(src.nasa_high, np.float64),
        "T_mid": np.ascontiguousarray(src.T_mid, np.float64),
        "reversible": np.ascontiguousarray(src.reversible, np.uint8),
    }
    opt = {"rtype": ("rtype", np.uint8, (nr,)), "efficiency": ("eff", np.float64, (nr, ns)),
           "low_ln_A": ("low_ln_A", np.float64, (nr,)),
           "low_beta": ("low_beta", np.float64, (nr,)),
           "low_Ea": ("low_Ea", np.float64, (nr,)), "troe": ("troe", np.float64, (nr, 4))}
    for name, (attr, dt, shape) in opt.items():
        v = getattr(src, attr, None)
        if v is not None:
            v = np.ascontiguousarray(v, dt)
            if v.shape != shape:
                raise ValueError(f"{attr} must have shape {shape}")
        keep[name] = v

    def ptr(k):
        return None if keep[k] is None else keep[k].ctypes.data

    d = MechanismDesc(ns, nr, *(ptr(k) for k in (
        "W", "nu_f", "nu_r", "ln_A", "beta", "Ea", "nasa_low", "nasa_high", "T_mid",
        "reversible", "rtype", "efficiency", "low_ln_A", "low_beta", "low_Ea", "troe")))
    return d, keep


def jit_source(src, precision: str = "fp32") -> str:
    """HIP source text the library generates for a mechanism (no GPU needed)."""
    d, keep = _desc(src)
    prec = {"fp32": AK_FP32, "fp64": AK_FP64}[precision]
    need = C.c_size_t()
    _check(lib().ak_jit_source(C.byref(d), prec, None, 0, C.byref(need)))
    buf = C.create_string_buffer(need.value)
    _check(lib().ak_jit_source(C.byref(d), prec, buf, need.value, C.byref(need)))
    return buf.value.decode()


def jit_tables(src, precision: str = "fp32"):
    """(species table, reaction table) the generated kernels read (no GPU
    needed; a diagnostic beside jit_source)."""
    d, keep = _desc(src)
    prec = {"fp32": AK_FP32, "fp64": AK_FP64}[precision]
    nsp, nrx = C.c_size_t(), C.c_size_t()
    _check(lib().ak_jit_tables(C.byref(d), prec, None, 0, None, 0, C.byref(nsp), C.byref(nrx)))
    sp = np.zeros(nsp.value)
    rx = np.zeros(nrx.value)
    _check(lib().ak_jit_tables(C.byref(d), prec, sp.ctypes.data_as(C.c_void_p), sp.size,
                               rx.ctypes.data_as(C.c_void_p), rx.size, C.byref(nsp),
                               C.byref(nrx)))
    return sp, rx


def jit_jacobian_source(src, precision: str = "fp64", interleaved: bool = False,
                        vjp: bool = False) -> str:
    """HIP source text of the state Jacobian compiled for a mechanism (no GPU
    needed); ``interleaved`` for the cell-minor output layout, ``vjp`` for
    the vector-Jacobian product instead."""
    d, keep = _desc(src)
    prec = {"fp32": AK_FP32, "fp64": AK_FP64}[precision]
    il = 2 if vjp else int(bool(interleaved))
    need = C.c_size_t()
    _check(lib().ak_jit_jacobian_source(C.byref(d), prec, il, None, 0, C.byref(need)))
    buf = C.create_string_buffer(need.value)
    _check(lib().ak_jit_jacobian_source(C.byref(d), prec, il, buf, need.value, C.byref(need)))
    return buf.value.decode()


def jit_jacobian_tables(src):
    """(species table, reaction table) of the compiled Jacobian (no GPU
    needed)."""
    d, keep = _desc(src)
    nsp, nrx = C.c_size_t(), C.c_size_t()
    _check(lib().ak_jit_jacobian_tables(C.byref(d), None, 0, None, 0, C.byref(nsp),
                                        C.byref(nrx)))
    sp = np.zeros(nsp.value)
    rx = np.zeros(nrx.value)
    _check(lib().ak_jit_jacobian_tables(C.byref(d), sp.ctypes.data_as(C.c_void_p), sp.size,
                                        rx.ctypes.data_as(C.c_void_p), rx.size, C.byref(nsp),
                                        C.byref(nrx)))
    return sp, rx


class Mechanism:
    """A mechanism uploaded to one GPU.  ``src`` is any object with the
    attributes of ``synth.Mechanism`` (W, nu_f, nu_r, ln_A, beta, Ea,
    nasa_low, nasa_high, T_mid, reversible).  ``kernels="auto"`` compiles
    the mechanism into its own source-term kernels where it fits them;
    ``"table"`` uses the table-driven kernels only."""

    def __init__(self, src, device: int | None = None, kernels: str = "auto"):
        torch = _torch()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        self.n_species = int(src.W.shape[0])
        self.n_reactions = int(src.nu_f.shape[0])
        d, self._keep = _desc(src)
        h = C.c_void_p()
        _check(lib().ak_load_mechanism_ex(C.byref(d), self.device, _KERNELS[kernels], C.byref(h)))
        self._h = h
        self.name = getattr(src, "name", "mechanism")

    @classmethod
    def from_file(cls, path, device: int | None = None, kernels: str = "auto"):
        """Read a CHEMKIN-II mechanism file (ELEMENTS, SPECIES, THERMO and
        REACTIONS blocks in one file) and upload it.  Parsing is host work
        in ``chemkin``; the result goes through the same loader as any other
        mechanism."""
        from . import chemkin
        return cls(chemkin.load(path), device=device, kernels=kernels)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ak_free_mechanism(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def compiled(self, dtype) -> bool:
        """Whether eval_source runs the mechanism-compiled kernel for the
        precision of ``dtype`` (torch.float32 or torch.float64)."""
        rc = lib().ak_mechanism_compiled(self._h, _prec(dtype))
        if rc < 0:
            _check(rc)
        return rc == 1

    def compiled_jacobian(self, dtype) -> bool:
        """Whether the mechanism has a compiled state Jacobian (eval_jacobian
        runs it unless AK_JIT_JACOBIAN=0; eval_jacobian_interleaved needs
        it)."""
        rc = lib().ak_mechanism_compiled_jacobian(self._h, _prec(dtype))
        if rc < 0:
            _check(rc)
        return rc == 1

    def error_count(self, stream=None) -> int:
        """Read and reset the device-side bad-cell counter (synchronises)."""
        n = C.c_int64()
        _check(lib().ak_error_count(self._h, _stream_ptr(stream), C.byref(n)))
        return int(n.value)


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _prec(dtype):
    torch = _torch()
    if dtype == torch.float32 or dtype is np.float32 or dtype == np.dtype(np.float32):
        return AK_FP32
    if dtype == torch.float64 or dtype is np.float64 or dtype == np.dtype(np.float64):
        return AK_FP64
    raise TypeError(f"unsupported dtype {dtype}: use float32 or float64")


def _check_state(mech, T, P, Y):
    torch = _torch()
    for name, t in (("T", T), ("P", P), ("Y", Y)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a GPU tensor")
    if T.dtype != P.dtype or T.dtype != Y.dtype:
        raise TypeError("T, P and Y must share one dtype")
    n = T.shape[0]
    if T.dim() != 1 or P.shape != (n,) or not T.is_contiguous() or not P.is_contiguous():
        raise ValueError("T and P must be contiguous [n] tensors")
    if Y.dim() != 2 or Y.shape[0] != mech.n_species or Y.shape[1] != n or Y.stride(1) != 1:
        raise ValueError(f"Y must be [NS={mech.n_species}, n={n}] with unit cell stride")
    return n


def eval_source(mech: Mechanism, T, P, Y, out=None, stream=None):
    """omega [NS, n] (kmol m^-3 s^-1) for states T [n] (K), P [n] (Pa),
    Y [NS, n]; float32 tensors select the FP32 path, float64 the FP64 path.
    Asynchronous on ``stream`` (default: torch's current stream)."""
    torch = _torch()
    n = _check_state(mech, T, P, Y)
    if out is None:
        out = torch.empty((mech.n_species, n), dtype=T.dtype, device=T.device)
    elif (out.shape != (mech.n_species, n) or out.dtype != T.dtype or out.stride(1) != 1
          or not out.is_cuda):
        raise ValueError("out must be a GPU [NS, n] tensor of the state dtype")
    ldY = Y.stride(0) if mech.n_species > 1 else n
    ldO = out.stride(0) if mech.n_species > 1 else n
    _check(lib().ak_eval_source(mech.handle, _prec(T.dtype), T.data_ptr(), P.data_ptr(),
                                Y.data_ptr(), ldY, n, out.data_ptr(), ldO, _stream_ptr(stream)))
    return out


def eval_jacobian(mech: Mechanism, T, P, Y, out=None, stream=None):
    """Dense Jacobian [n, NS+1, NS+1] of (omega, omega_T) with respect to
    (Y_1..Y_NS, T) at fixed P (row-major per cell).  Asynchronous."""
    torch = _torch()
    n = _check_state(mech, T, P, Y)
    nv = mech.n_species + 1
    if out is None:
        out = torch.empty((n, nv, nv), dtype=T.dtype, device=T.device)
    elif (out.shape != (n, nv, nv) or out.dtype != T.dtype or not out.is_cuda
          or out.stride(2) != 1 or out.stride(1) != nv):
        raise ValueError("out must be a GPU [n, NS+1, NS+1] tensor, rows contiguous")
    ldY = Y.stride(0) if mech.n_species > 1 else n
    ldJ = out.stride(0) if n > 1 else nv * nv
    _check(lib().ak_eval_jacobian(mech.handle, _prec(T.dtype), T.data_ptr(), P.data_ptr(),
                                  Y.data_ptr(), ldY, n, out.data_ptr(), ldJ,
                                  _stream_ptr(stream)))
    return out


def eval_jacobian_interleaved(mech: Mechanism, T, P, Y, out=None, stream=None):
    """The same Jacobian in the interleaved layout [NS+1, NS+1, n] (cells
    innermost, like Y): out[r, c, i] = d x_r' / d x_c of cell i.  Always the
    kernel compiled for the mechanism.  Asynchronous."""
    torch = _torch()
    n = _check_state(mech, T, P, Y)
    nv = mech.n_species + 1
    if out is None:
        out = torch.empty((nv, nv, n), dtype=T.dtype, device=T.device)
    elif (out.shape != (nv, nv, n) or out.dtype != T.dtype or not out.is_cuda
          or out.stride(2) != 1 or out.stride(0) != nv * out.stride(1)):
        raise ValueError("out must be a GPU [NS+1, NS+1, n] tensor, cells contiguous")
    ldY = Y.stride(0) if mech.n_species > 1 else n
    ldJ = out.stride(1) if nv * nv > 1 else n
    _check(lib().ak_eval_jacobian_interleaved(mech.handle, _prec(T.dtype), T.data_ptr(),
                                              P.data_ptr(), Y.data_ptr(), ldY, n,
                                              out.data_ptr(), ldJ, _stream_ptr(stream)))
    return out


def eval_vjp(mech: Mechanism, T, P, Y, g_omega, stream=None):
    """(g_Y [NS, n], g_T [n]) = (g_omega^T d omega/dY, g_omega^T d omega/dT)."""
    torch = _torch()
    n = _check_state(mech, T, P, Y)
    if (g_omega.shape != (mech.n_species, n) or g_omega.dtype != T.dtype
            or not g_omega.is_cuda or g_omega.stride(1) != 1):
        raise ValueError("g_omega must be a GPU [NS, n] tensor of the state dtype")
    gY = torch.empty((mech.n_species, n), dtype=T.dtype, device=T.device)
    gT = torch.empty((n,), dtype=T.dtype, device=T.device)
    ldY = Y.stride(0) if mech.n_species > 1 else n
    ldG = g_omega.stride(0) if mech.n_species > 1 else n
    _check(lib().ak_eval_vjp(mech.handle, _prec(T.dtype), T.data_ptr(), P.data_ptr(),
                             Y.data_ptr(), ldY, n, g_omega.data_ptr(), ldG, gY.data_ptr(),
                             n, gT.data_ptr(), _stream_ptr(stream)))
    return gY, gT


def integrate_euler(mech: Mechanism, T, P, Y, dt: float, n_steps: int, stream=None):
    """Advance (T [n], Y [NS, n]) in place by n_steps forward-Euler steps of
    dt seconds of the 0-D constant-pressure reactor at fixed P [n]
    (Sec. 3.1).  float32 tensors select the FP32 path, float64 the FP64 path.
    Asynchronous on ``stream`` (default: torch's current stream)."""
    n = _check_state(mech, T, P, Y)
    _check(lib().ak_integrate_euler(mech.handle, _prec(T.dtype), T.data_ptr(), P.data_ptr(),
                                    Y.data_ptr(), Y.stride(0), n, float(dt), int(n_steps),
                                    _stream_ptr(stream)))
    return T, Y


# ---------------------------------------------------------------------------
# ln K_c alone and the approximate network in its place (Sec. 2.3)

def _check_T(T):
    torch = _torch()
    if not isinstance(T, torch.Tensor) or not T.is_cuda:
        raise TypeError("T must be a GPU tensor")
    if T.dim() != 1 or not T.is_contiguous():
        raise ValueError("T must be a contiguous [n] tensor")
    _prec(T.dtype)
    return T.shape[0]


def _lnk_out(out, nr, n, T):
    torch = _torch()
    if out is None:
        return torch.empty((nr, n), dtype=T.dtype, device=T.device)
    if (out.shape != (nr, n) or out.dtype != T.dtype or not out.is_cuda
            or out.stride(1) != 1):
        raise ValueError("out must be a GPU [NR, n] tensor of T's dtype, cells contiguous")
    return out


def eval_lnkc(mech: Mechanism, T, out=None, stream=None):
    """ln K_c [NR, n] (Eq. 8 through the Gibbs and stoichiometric layers,
    Eqs. 9-11) at temperatures T [n].  Asynchronous."""
    n = _check_T(T)
    out = _lnk_out(out, mech.n_reactions, n, T)
    ldK = out.stride(0) if mech.n_reactions > 1 else n
    _check(lib().ak_eval_lnkc(mech.handle, _prec(T.dtype), T.data_ptr(), n, out.data_ptr(),
                              ldK, _stream_ptr(stream)))
    return out


class KcNet:
    """The approximate ln K_c network of Sec. 2.3 (Architecture 2) uploaded
    to one GPU.  ``net`` has ``weights`` (N_L + 1 matrices [1, N_H],
    [N_H, N_H] ..., [N_H, N_R]), ``biases``, ``x_mean``, ``x_std``,
    ``y_mean`` and ``y_std`` (for instance ``kcnet.KcNetWeights``)."""

    def __init__(self, net, device: int | None = None):
        torch = _torch()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        W = [np.ascontiguousarray(w, dtype=np.float64) for w in net.weights]
        B = [np.ascontiguousarray(b, dtype=np.float64).reshape(-1) for b in net.biases]
        if len(W) < 2 or len(W) != len(B):
            raise ValueError("a network needs at least one hidden layer and a readout")
        nh = W[0].shape[1]
        nr = W[-1].shape[1]
        if W[0].shape != (1, nh) or any(w.shape != (nh, nh) for w in W[1:-1]) \
                or W[-1].shape != (nh, nr) or any(b.shape != (w.shape[1],) for w, b in zip(W, B)):
            raise ValueError("inconsistent layer shapes")
        self.n_layers, self.n_hidden, self.n_out = len(W) - 1, nh, nr
        self._w = np.concatenate([w.reshape(-1) for w in W])
        self._b = np.concatenate(B)
        self._ym = np.ascontiguousarray(net.y_mean, dtype=np.float64).reshape(-1)
        self._ys = np.ascontiguousarray(net.y_std, dtype=np.float64).reshape(-1)
        if self._ym.shape != (nr,) or self._ys.shape != (nr,):
            raise ValueError("y_mean and y_std must have one entry per output")
        d = KcNetDesc(self.n_layers, nh, nr, 0, self._w.ctypes.data, self._b.ctypes.data,
                      float(net.x_mean), float(net.x_std), self._ym.ctypes.data,
                      self._ys.ctypes.data)
        h = C.c_void_p()
        _check(lib().ak_load_kcnet(C.byref(d), self.device, C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ak_free_kcnet(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_lnkc_net(net: KcNet, T, out=None, stream=None):
    """ln K_c [N_R, n] from the network at temperatures T [n].  Asynchronous."""
    n = _check_T(T)
    out = _lnk_out(out, net.n_out, n, T)
    ldK = out.stride(0) if net.n_out > 1 else n
    _check(lib().ak_eval_lnkc_net(net.handle, _prec(T.dtype), T.data_ptr(), n, out.data_ptr(),
                                  ldK, _stream_ptr(stream)))
    return out


def eval_source_lnkc(mech: Mechanism, T, P, Y, lnK, out=None, stream=None):
    """omega [NS, n] with ln K_c of reaction j in cell i taken from
    lnK [NR, n] in place of Eq. 8.  Asynchronous."""
    torch = _torch()
    n = _check_state(mech, T, P, Y)
    if (not isinstance(lnK, torch.Tensor) or not lnK.is_cuda or lnK.dtype != T.dtype
            or lnK.shape != (mech.n_reactions, n) or lnK.stride(1) != 1):
        raise ValueError("lnK must be a GPU [NR, n] tensor of the state dtype, cells contiguous")
    if out is None:
        out = torch.empty((mech.n_species, n), dtype=T.dtype, device=T.device)
    elif (out.shape != (mech.n_species, n) or out.dtype != T.dtype or out.stride(1) != 1
          or not out.is_cuda):
        raise ValueError("out must be a GPU [NS, n] tensor of the state dtype")
    ldY = Y.stride(0) if mech.n_species > 1 else n
    ldO = out.stride(0) if mech.n_species > 1 else n
    ldK = lnK.stride(0) if mech.n_reactions > 1 else n
    _check(lib().ak_eval_source_lnkc(mech.handle, _prec(T.dtype), T.data_ptr(), P.data_ptr(),
                                     Y.data_ptr(), ldY, n, lnK.data_ptr(), ldK, out.data_ptr(),
                                     ldO, _stream_ptr(stream)))
    return out


def eval_production(mech: Mechanism, rates, out=None, stream=None):
    """omega = nu r [NS, n] (FP32) from rates of progress r [NR, n] (FP32,
    cells contiguous), contracted on the matrix cores in split bfloat16.
    Asynchronous."""
    torch = _torch()
    if (not isinstance(rates, torch.Tensor) or not rates.is_cuda
            or rates.dtype != torch.float32 or rates.dim() != 2
            or rates.shape[0] != mech.n_reactions or rates.stride(1) != 1):
        raise ValueError("rates must be a GPU float32 [NR, n] tensor, cells contiguous")
    n = rates.shape[1]
    if out is None:
        out = torch.empty((mech.n_species, n), dtype=torch.float32, device=rates.device)
    elif (out.shape != (mech.n_species, n) or out.dtype != torch.float32
          or out.stride(1) != 1 or not out.is_cuda):
        raise ValueError("out must be a GPU float32 [NS, n] tensor")
    ldR = rates.stride(0) if mech.n_reactions > 1 else n
    ldO = out.stride(0) if mech.n_species > 1 else n
    _check(lib().ak_eval_production(mech.handle, rates.data_ptr(), ldR, n, out.data_ptr(),
                                    ldO, _stream_ptr(stream)))
    return out


def eval_source_net(mech: Mechanism, net: KcNet, T, P, Y, out=None, stream=None):
    """omega [NS, n] with the network's ln K_c in place of Eq. 8 (the
    drop-in of Sec. 2.3).  Asynchronous."""
    torch = _torch()
    n = _check_state(mech, T, P, Y)
    if out is None:
        out = torch.empty((mech.n_species, n), dtype=T.dtype, device=T.device)
    elif (out.shape != (mech.n_species, n) or out.dtype != T.dtype or out.stride(1) != 1
          or not out.is_cuda):
        raise ValueError("out must be a GPU [NS, n] tensor of the state dtype")
    ldY = Y.stride(0) if mech.n_species > 1 else n
    ldO = out.stride(0) if mech.n_species > 1 else n
    _check(lib().ak_eval_source_net(mech.handle, net.handle, _prec(T.dtype), T.data_ptr(),
                                    P.data_ptr(), Y.data_ptr(), ldY, n, out.data_ptr(), ldO,
                                    _stream_ptr(stream)))
    return out


def integrate_implicit(mech: Mechanism, T, P, Y, dt: float, n_steps: int, stream=None):
    """Advance (T [n], Y [NS, n]) in place by n_steps linearly implicit
    Euler steps of dt seconds ((I - dt Jf) dx = dt f, Jf from the state
    Jacobian; Sec. 4's stiff integration) at fixed P [n].  Asynchronous."""
    n = _check_state(mech, T, P, Y)
    _check(lib().ak_integrate_implicit(mech.handle, _prec(T.dtype), T.data_ptr(), P.data_ptr(),
                                       Y.data_ptr(), Y.stride(0), n, float(dt), int(n_steps),
                                       _stream_ptr(stream)))
    return T, Y


def integrate_euler_net(mech: Mechanism, net: KcNet, T, P, Y, dt: float, n_steps: int,
                        stream=None):
    """integrate_euler with the network's ln K_c in place of Eq. 8 at every
    step (Sec. 3.1's a-posteriori test).  In place, asynchronous."""
    n = _check_state(mech, T, P, Y)
    _check(lib().ak_integrate_euler_net(mech.handle, net.handle, _prec(T.dtype), T.data_ptr(),
                                        P.data_ptr(), Y.data_ptr(), Y.stride(0), n, float(dt),
                                        int(n_steps), _stream_ptr(stream)))
    return T, Y


def _source_function():
    torch = _torch()

    class SourceTerm(torch.autograd.Function):
        """omega(T, P, Y), differentiable in T and Y through the library's
        hand-written VJP kernel (P is treated as a constant)."""

        @staticmethod
        def forward(ctx, mech, T, P, Y):
            Tc, Pc, Yc = T.contiguous(), P.contiguous(), Y.contiguous()
            ctx.mech = mech
            ctx.save_for_backward(Tc, Pc, Yc)
            return eval_source(mech, Tc, Pc, Yc)

        @staticmethod
        def backward(ctx, g):
            T, P, Y = ctx.saved_tensors
            gY, gT = eval_vjp(ctx.mech, T, P, Y, g.contiguous())
            return None, gT, None, gY

    return SourceTerm


_SOURCE_FN = None


def source_term(mech: Mechanism, T, P, Y):
    """Differentiable omega (see SourceTerm)."""
    global _SOURCE_FN
    if _SOURCE_FN is None:
        _SOURCE_FN = _source_function()
    return _SOURCE_FN.apply(mech, T, P, Y)


def jacobian(mech: Mechanism, T, P, Y):
    """Alias of eval_jacobian."""
    return eval_jacobian(mech, T, P, Y)


# ---------------------------------------------------------------------------
# serving

def _host_ptr(a):
    """Address of a host buffer: a CPU torch tensor or a numpy array."""
    if hasattr(a, "data_ptr"):
        if a.is_cuda:
            raise TypeError("server requests take host buffers")
        return a.data_ptr()
    return a.ctypes.data


def _host_info(a):
    """(element type "float32" / "float64" / other, shape, strides in elements)
    of a CPU torch tensor or a numpy array."""
    if hasattr(a, "data_ptr"):
        name, shape, strides = str(a.dtype), tuple(a.shape), tuple(a.stride())
    else:
        name, shape, strides = str(a.dtype), tuple(a.shape), tuple(
            s // a.itemsize for s in a.strides)
    kind = "float32" if "float32" in name else "float64" if "float64" in name else name
    return kind, shape, strides


class Request:
    """One submitted request.  Keeps its host buffers alive until it has
    completed (or been cancelled) and been freed; dropping a pending request
    cancels it if it is still queued and otherwise waits for it, so that no
    copy into its buffers outlives them."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    def wait(self, timeout: float = -1.0) -> None:
        _check(lib().ak_request_wait(self._h, float(timeout)))

    def cancel(self) -> bool:
        """True if the request was still queued and is now cancelled."""
        return lib().ak_request_cancel(self._h) == 0

    def free(self) -> None:
        if self._h is not None and self._h.value:
            _check(lib().ak_request_free(self._h))
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            if self._h is not None and self._h.value:
                if lib().ak_request_cancel(self._h) != 0:
                    lib().ak_request_wait(self._h, -1.0)   # admitted: let its copies finish
                lib().ak_request_free(self._h)
                self._h = None
                self._keep = None
        except Exception:
            pass


class Server:
    """Continuous-batching source-term server on one GPU (see annkin.h)."""

    def __init__(self, device: int | None = None, max_inflight: int = 3,
                 max_batch_requests: int = 64, batching: bool = True,
                 max_batch_cells: int = 1 << 16, arena_bytes: int = 1 << 30,
                 small_request_cells: int = 4096, arena=None):
        """``arena``: optionally a caller-owned GPU tensor (any dtype,
        contiguous, 256-byte aligned) that the server stages requests in
        instead of allocating its own; its size in bytes replaces
        ``arena_bytes`` and it must outlive the server."""
        if device is None:
            device = _torch().cuda.current_device()
        ptr = None
        if arena is not None:
            if not arena.is_cuda or not arena.is_contiguous():
                raise ValueError("arena must be a contiguous GPU tensor")
            arena_bytes = arena.numel() * arena.element_size()
            ptr = arena.data_ptr()
            self._arena = arena
        cfg = ServerConfig(int(device), int(max_inflight), int(max_batch_requests),
                           1 if batching else 0, int(max_batch_cells), int(arena_bytes),
                           int(small_request_cells), ptr)
        h = C.c_void_p()
        _check(lib().ak_server_create(C.byref(cfg), C.byref(h)))
        self._h = h

    def submit(self, mech: Mechanism, T, P, Y, out) -> Request:
        """Queue one request: host T [n], P [n], Y [NS, ldY-strided], results
        into host out [NS, ldO-strided]; all float32 or all float64.  T and P
        must be contiguous; Y and out need unit cell stride."""
        dt, shp, st = _host_info(Y)
        if len(shp) != 2:
            raise ValueError("Y must be [NS, n]")
        n = shp[1]
        ns = mech.n_species
        if shp[0] != ns or st[1] != 1:
            raise ValueError("Y must be [NS, n] with unit cell stride")
        prec = {"float32": AK_FP32, "float64": AK_FP64}.get(dt)
        if prec is None:
            raise TypeError("float32 or float64 buffers")
        for what, a in (("T", T), ("P", P)):
            adt, ashp, ast = _host_info(a)
            if adt != dt:
                raise TypeError(f"{what} must have Y's dtype {dt}, not {adt}")
            if tuple(ashp) != (n,) or (n > 1 and ast[0] != 1):
                raise ValueError(f"{what} must be a contiguous [n={n}] buffer")
        odt, oshp, ost = _host_info(out)
        if odt != dt:
            raise TypeError(f"out must have Y's dtype {dt}, not {odt}")
        if tuple(oshp) != (ns, n) or ost[1] != 1:
            raise ValueError("out must be [NS, n] with unit cell stride")
        ldY = st[0] if ns > 1 else n
        ldO = ost[0] if ns > 1 else n
        h = C.c_void_p()
        _check(lib().ak_server_submit(self._h, mech.handle, prec, _host_ptr(T), _host_ptr(P),
                                      _host_ptr(Y), ldY, n, _host_ptr(out), ldO, C.byref(h)))
        return Request(h, (T, P, Y, out, mech))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().ak_server_get_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_ if f != "pad"}

    def reset_stats(self) -> None:
        _check(lib().ak_server_reset_stats(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ak_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
