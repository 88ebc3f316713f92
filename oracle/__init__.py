"""Test oracle: plain CPU evaluation of the chemical source term.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP library
never loads it and shares no code with it.

What it computes (Barwey & Raman, Sec. 2) in the classical form, cell by
cell: concentrations from the ideal-gas state, Arrhenius forward rate
constants (Eq. 5), equilibrium constants from NASA-7 enthalpy and entropy
changes (Eq. 8), reverse constants k_r = k_f / K_c (Eq. 7), rates of progress
as products of concentrations (Eq. 3), and net production rates (Eq. 2).
``source(..., precision="ld")`` evaluates in x86 extended precision.
``lnkc`` gives ln K_c alone, ``source_lnkc`` the source term with a given
ln K_c in place of Eq. 8, ``production`` the stoichiometric contraction
omega = nu r of given rates of progress, and ``kcnet`` the approximate ln K_c network of
Sec. 2.3 (Architecture 2) written out in numpy float64.

Pins (``tests/test_oracle_pins.py``): two hand-worked reactions in closed
form, detailed balance at a constructed equilibrium state, atom and mass
conservation, degree-0 homogeneity in Y, thermodynamic identities
(dH/dT = cp, dS/dT = cp/T, van 't Hoff), the Arrhenius special case, brute
force at 50 digits on tiny mechanisms, and for the Jacobian central finite
differences and conservation of elements.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ("oracle.c", "oracle.h", "oracle_impl.h")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
           "-o", tmp, os.path.join(_HERE, "oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Mech(C.Structure):
    _fields_ = [
        ("ns", C.c_int), ("nr", C.c_int),
        ("W", C.c_void_p), ("nu_f", C.c_void_p), ("nu_r", C.c_void_p),
        ("ln_A", C.c_void_p), ("beta", C.c_void_p), ("Ea", C.c_void_p),
        ("nasa_low", C.c_void_p), ("nasa_high", C.c_void_p), ("T_mid", C.c_void_p),
        ("reversible", C.c_void_p),
        ("rtype", C.c_void_p), ("eff", C.c_void_p),
        ("low_ln_A", C.c_void_p), ("low_beta", C.c_void_p), ("low_Ea", C.c_void_p),
        ("troe", C.c_void_p),
    ]


_LD = np.longdouble
assert np.finfo(_LD).nmant >= 63, "the oracle's extended precision needs x86 long double"


def _lib_handle():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = C.CDLL(_LIB_PATH)
        for sfx in ("f64", "ld"):
            getattr(lib, f"ora_thermo_{sfx}").argtypes = [C.c_void_p, C.c_double, C.c_void_p,
                                                          C.c_void_p, C.c_void_p]
            getattr(lib, f"ora_rates_{sfx}").argtypes = [C.c_void_p, C.c_double, C.c_double,
                                                         C.c_void_p] + [C.c_void_p] * 5
            getattr(lib, f"ora_source_{sfx}").argtypes = [
                C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int]
            getattr(lib, f"ora_temp_source_{sfx}").argtypes = [
                C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                C.c_void_p, C.c_int]
            getattr(lib, f"ora_integrate_euler_{sfx}").argtypes = [
                C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                C.c_double, C.c_int, C.c_int]
            getattr(lib, f"ora_jacobian_{sfx}").argtypes = [
                C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                C.c_void_p, C.c_int64, C.c_int]
            getattr(lib, f"ora_jacobian_scaled_{sfx}").argtypes = [
                C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                C.c_void_p, C.c_void_p, C.c_int64, C.c_int]
            getattr(lib, f"ora_integrate_implicit_{sfx}").argtypes = [
                C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                C.c_double, C.c_int]
            getattr(lib, f"ora_lnkc_{sfx}").argtypes = [C.c_void_p, C.c_int64, C.c_void_p,
                                                        C.c_void_p, C.c_int64]
            getattr(lib, f"ora_source_lnkc_{sfx}").argtypes = [
                C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int]
        _lib = lib
    return _lib


class OracleMechanism:
    """Holds contiguous copies of a mechanism's arrays and the C view of them.

    ``mech`` is any object with the attributes of ``synth.Mechanism``."""

    def __init__(self, mech):
        self.ns = int(mech.W.shape[0])
        self.nr = int(mech.nu_f.shape[0])
        self._keep = {
            "W": np.ascontiguousarray(mech.W, dtype=np.float64),
            "nu_f": np.ascontiguousarray(mech.nu_f, dtype=np.int8),
            "nu_r": np.ascontiguousarray(mech.nu_r, dtype=np.int8),
            "ln_A": np.ascontiguousarray(mech.ln_A, dtype=np.float64),
            "beta": np.ascontiguousarray(mech.beta, dtype=np.float64),
            "Ea": np.ascontiguousarray(mech.Ea, dtype=np.float64),
            "nasa_low": np.ascontiguousarray(mech.nasa_low, dtype=np.float64),
            "nasa_high": np.ascontiguousarray(mech.nasa_high, dtype=np.float64),
            "T_mid": np.ascontiguousarray(mech.T_mid, dtype=np.float64),
            "reversible": np.ascontiguousarray(mech.reversible, dtype=np.uint8),
        }
        assert self._keep["nu_f"].shape == (self.nr, self.ns)
        # pressure-dependent reactions (optional attributes; None = absent)
        opt = {"rtype": (np.uint8, (self.nr,)), "eff": (np.float64, (self.nr, self.ns)),
               "low_ln_A": (np.float64, (self.nr,)), "low_beta": (np.float64, (self.nr,)),
               "low_Ea": (np.float64, (self.nr,)), "troe": (np.float64, (self.nr, 4))}
        for name, (dt, shape) in opt.items():
            v = getattr(mech, name, None)
            if v is not None:
                v = np.ascontiguousarray(v, dtype=dt)
                assert v.shape == shape, (name, v.shape)
            self._keep[name] = v
        k = self._keep

        def ptr(n):
            return None if k[n] is None else k[n].ctypes.data

        self._c = _Mech(self.ns, self.nr, *(ptr(n) for n in (
            "W", "nu_f", "nu_r", "ln_A", "beta", "Ea", "nasa_low", "nasa_high", "T_mid",
            "reversible", "rtype", "eff", "low_ln_A", "low_beta", "low_Ea", "troe")))

    @property
    def ptr(self):
        return C.addressof(self._c)


def _as_mech(m):
    return m if isinstance(m, OracleMechanism) else OracleMechanism(m)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dtype(precision):
    if precision == "f64":
        return np.float64
    if precision == "ld":
        return _LD
    raise ValueError(precision)


def thermo(mech, T: float, precision: str = "f64"):
    """(h/RT, s/R, cp/R) per species at temperature T."""
    m = _as_mech(mech)
    dt = _dtype(precision)
    h, s, cp = (np.zeros(m.ns, dt) for _ in range(3))
    getattr(_lib_handle(), f"ora_thermo_{precision}")(m.ptr, float(T), h.ctypes.data,
                                                      s.ctypes.data, cp.ctypes.data)
    return h, s, cp


def rates(mech, T: float, P: float, Y, precision: str = "f64"):
    """One cell: dict of C [NS] and kf, Kc, qf, qr [NR] (SI-kmol units)."""
    m = _as_mech(mech)
    dt = _dtype(precision)
    Yc = _f64(Y)
    assert Yc.shape == (m.ns,)
    out = {"C": np.zeros(m.ns, dt)}
    for n in ("kf", "Kc", "qf", "qr"):
        out[n] = np.zeros(m.nr, dt)
    rc = getattr(_lib_handle(), f"ora_rates_{precision}")(
        m.ptr, float(T), float(P), Yc.ctypes.data, out["C"].ctypes.data,
        out["kf"].ctypes.data, out["Kc"].ctypes.data, out["qf"].ctypes.data,
        out["qr"].ctypes.data)
    if rc:
        raise RuntimeError("oracle rates failed")
    return out


def source(mech, T, P, Y, precision: str = "f64", scales: bool = False, n_threads: int = 0):
    """Net production rates omega [NS, n] (kmol m^-3 s^-1) for states
    T [n] (K), P [n] (Pa), Y [NS, n].  With ``scales`` also returns the gross
    scale S and net scale N (same shape)."""
    m = _as_mech(mech)
    dt = _dtype(precision)
    T, P = _f64(T), _f64(P)
    Y = _f64(Y)
    n = T.shape[0]
    assert P.shape == (n,) and Y.shape == (m.ns, n)
    om = np.zeros((m.ns, n), dt)
    S = np.zeros((m.ns, n), dt) if scales else None
    N = np.zeros((m.ns, n), dt) if scales else None
    rc = getattr(_lib_handle(), f"ora_source_{precision}")(
        m.ptr, n, T.ctypes.data, P.ctypes.data, Y.ctypes.data, n, om.ctypes.data,
        S.ctypes.data if scales else None, N.ctypes.data if scales else None, n,
        int(n_threads))
    if rc:
        raise RuntimeError("oracle source failed")
    return (om, S, N) if scales else om


def integrate_implicit(mech, T, P, Y, dt: float, n_steps: int, precision: str = "f64"):
    """0-D constant-pressure reactor, n_steps linearly implicit Euler steps of
    dt: (I - dt Jf) dx = dt f(x) with f = (W omega / rho, omega_T) and Jf from
    the analytic Jacobian, rho held at the step's start (Sec. 4's stiff
    integration).  Returns new (T [n], Y [NS, n]); P [n] is held fixed."""
    m = _as_mech(mech)
    _dtype(precision)
    T = np.array(T, dtype=np.float64, copy=True)
    P = _f64(P)
    Y = np.array(Y, dtype=np.float64, copy=True, order="C")
    n = T.shape[0]
    assert P.shape == (n,) and Y.shape == (m.ns, n)
    rc = getattr(_lib_handle(), f"ora_integrate_implicit_{precision}")(
        m.ptr, n, T.ctypes.data, P.ctypes.data, Y.ctypes.data, n, float(dt), int(n_steps))
    if rc == -2:
        raise NotImplementedError("oracle Jacobian of third-body and falloff reactions")
    if rc:
        raise RuntimeError(f"oracle integrate_implicit failed ({rc})")
    return T, Y


def integrate_euler_lnkc(mech, lnk_of, T, P, Y, dt: float, n_steps: int):
    """The forward-Euler 0-D reactor of ``integrate_euler`` with ln K_c from
    ``lnk_of(T) -> [NR, n]`` in place of Eq. 8 at every step (a trained
    ln K_c as a drop-in, Sec. 3.1's a-posteriori use), in float64, composed
    from ``source_lnkc`` and ``thermo``:
        Y_k += dt W_k omega_k / rho,  T += dt omega_T,
        omega_T = -sum_k H_k omega_k / sum_k C_k cp_k,  rho = sum_k C_k W_k.
    Returns new (T [n], Y [NS, n])."""
    m = _as_mech(mech)
    W = np.asarray(mech.W, np.float64)
    T = np.array(T, dtype=np.float64, copy=True)
    P = _f64(P)
    Y = np.array(Y, dtype=np.float64, copy=True)
    n = T.shape[0]
    ru = 8314.46261815324
    for _ in range(n_steps):
        om = source_lnkc(mech, T, P, Y, lnk_of(T))
        for i in range(n):
            h, _, cp = thermo(m, T[i])
            yc = np.maximum(Y[:, i], 0.0)
            C = P[i] / (ru * T[i]) * (yc / W) / (yc / W).sum()
            rho = float((C * W).sum())
            omT = -float((ru * T[i] * h * om[:, i]).sum()) / float((C * ru * cp).sum())
            Y[:, i] += dt * W * om[:, i] / rho
            T[i] += dt * omT
    return T, Y


def lnkc(mech, T, precision: str = "f64"):
    """ln K_c (Eq. 8) [NR, n] of every reaction (file order) at temperatures T [n]."""
    m = _as_mech(mech)
    dt = _dtype(precision)
    T = _f64(T)
    n = T.shape[0]
    out = np.zeros((m.nr, n), dt)
    rc = getattr(_lib_handle(), f"ora_lnkc_{precision}")(m.ptr, n, T.ctypes.data,
                                                         out.ctypes.data, n)
    if rc:
        raise RuntimeError("oracle lnkc failed")
    return out


def source_lnkc(mech, T, P, Y, lnK, precision: str = "f64", scales: bool = False,
                n_threads: int = 0):
    """As ``source``, with ln K_c of reaction j in cell i taken from
    ``lnK[j, i]`` (a trained ln K_c as a drop-in, Sec. 2.3)."""
    m = _as_mech(mech)
    dt = _dtype(precision)
    T, P, Y = _f64(T), _f64(P), _f64(Y)
    lnK = _f64(lnK)
    n = T.shape[0]
    assert P.shape == (n,) and Y.shape == (m.ns, n) and lnK.shape == (m.nr, n)
    om = np.zeros((m.ns, n), dt)
    S = np.zeros((m.ns, n), dt) if scales else None
    N = np.zeros((m.ns, n), dt) if scales else None
    rc = getattr(_lib_handle(), f"ora_source_lnkc_{precision}")(
        m.ptr, n, T.ctypes.data, P.ctypes.data, Y.ctypes.data, n, lnK.ctypes.data, n,
        om.ctypes.data, S.ctypes.data if scales else None, N.ctypes.data if scales else None,
        n, int(n_threads))
    if rc:
        raise RuntimeError("oracle source_lnkc failed")
    return (om, S, N) if scales else om


def _elu(x):
    return np.where(x >= 0.0, x, np.expm1(np.minimum(x, 0.0)))


def kcnet(net, T, bound: bool = False):
    """The approximate ln K_c network of Sec. 2.3, Architecture 2, in float64:
    input the standardized log temperature, N_L hidden layers
    X_{l+1} = elu(X_l W_l + B_l) (Eqs. 12 and 14), then a linear output layer
    to the N_R standardized outputs, mapped back by the training set's
    standard deviation and mean.  ``net`` has ``weights`` (N_L + 1 matrices,
    [1, N_H], [N_H, N_H] ..., [N_H, N_R]), ``biases``, ``x_mean``, ``x_std``
    (scalars) and ``y_mean``, ``y_std`` ([N_R]).  Returns ln K_c [N_R, n].

    With ``bound``, also returns the running magnitude of the same
    computation (every product and sum taken in absolute value, elu by its
    slope bound 1), the scale a rounding-error bound of another evaluation
    is proportional to."""
    W = [np.asarray(w, np.float64) for w in net.weights]
    B = [np.asarray(b, np.float64) for b in net.biases]
    x = (np.log(np.asarray(T, np.float64)) - float(net.x_mean)) / float(net.x_std)
    X = x[:, None]
    Xa = np.abs(X)
    for l in range(len(W) - 1):
        X = _elu(X @ W[l] + B[l])
        Xa = Xa @ np.abs(W[l]) + np.abs(B[l])
    out = X @ W[-1] + B[-1]
    ys, ym = np.asarray(net.y_std, np.float64), np.asarray(net.y_mean, np.float64)
    lnk = (out * ys + ym).T.copy()
    if not bound:
        return lnk
    mag = ((Xa @ np.abs(W[-1]) + np.abs(B[-1])) * np.abs(ys) + np.abs(ym)).T.copy()
    return lnk, mag


def production(mech, r):
    """Net production rates omega = nu r [NS, n] (Eq. 2) from given rates of
    progress r [NR, n] (r_j = q_f,j - q_r,j, file order), in float64, with
    nu = nu'' - nu' (products minus reactants).  The reduced-precision
    contraction (the single/half-precision future work of Sec. 4) is checked
    against this exact product."""
    nu = (np.asarray(mech.nu_r, np.float64) - np.asarray(mech.nu_f, np.float64)).T
    r = np.asarray(r, np.float64)
    assert r.ndim == 2 and r.shape[0] == nu.shape[1]
    return nu @ r


def temp_source(mech, T, P, Y, precision: str = "f64", n_threads: int = 0):
    """Constant-pressure temperature source omega_T [n] in K/s."""
    m = _as_mech(mech)
    dt = _dtype(precision)
    T, P, Y = _f64(T), _f64(P), _f64(Y)
    n = T.shape[0]
    out = np.zeros(n, dt)
    rc = getattr(_lib_handle(), f"ora_temp_source_{precision}")(
        m.ptr, n, T.ctypes.data, P.ctypes.data, Y.ctypes.data, n, out.ctypes.data,
        int(n_threads))
    if rc:
        raise RuntimeError("oracle temp_source failed")
    return out


def jacobian(mech, T, P, Y, precision: str = "f64", scales: bool = False, n_threads: int = 0):
    """Analytic Jacobian [n, NS+1, NS+1] of (omega, omega_T) w.r.t. (Y, T).
    With ``scales`` also returns the gross scale of every entry (each
    chain-rule term replaced by its absolute value)."""
    m = _as_mech(mech)
    dt = _dtype(precision)
    T, P, Y = _f64(T), _f64(P), _f64(Y)
    n = T.shape[0]
    nv = m.ns + 1
    J = np.zeros((n, nv, nv), dt)
    Ja = np.zeros((n, nv, nv), dt) if scales else None
    rc = getattr(_lib_handle(), f"ora_jacobian_scaled_{precision}")(
        m.ptr, n, T.ctypes.data, P.ctypes.data, Y.ctypes.data, n, J.ctypes.data,
        Ja.ctypes.data if scales else None, nv * nv, int(n_threads))
    if rc == -2:
        raise NotImplementedError("oracle Jacobian of third-body and falloff reactions")
    if rc:
        raise RuntimeError("oracle jacobian failed")
    return (J, Ja) if scales else J


def integrate_euler(mech, T, P, Y, dt: float, n_steps: int, precision: str = "f64",
                    n_threads: int = 0):
    """0-D constant-pressure reactor, n_steps forward-Euler steps of dt
    (Sec. 3.1): returns new (T [n], Y [NS, n]); P [n] is held fixed."""
    m = _as_mech(mech)
    _dtype(precision)
    T = np.array(T, dtype=np.float64, copy=True)
    P = _f64(P)
    Y = np.array(Y, dtype=np.float64, copy=True, order="C")
    n = T.shape[0]
    assert P.shape == (n,) and Y.shape == (m.ns, n)
    rc = getattr(_lib_handle(), f"ora_integrate_euler_{precision}")(
        m.ptr, n, T.ctypes.data, P.ctypes.data, Y.ctypes.data, n, float(dt), int(n_steps),
        int(n_threads))
    if rc:
        raise RuntimeError("oracle integrate_euler failed")
    return T, Y
