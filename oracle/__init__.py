"""FP64 CPU oracle for the rotating spin-1 SO/Rabi-coupled SSCN step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP library; the C source (``gp_spin1_oracle.c``) holds the
arithmetic, this module only marshals numpy arrays through ctypes.

Parameters are passed as a plain mapping with the keys
``nx, ny, dx, dy, x0, y0, dt, c0, c2, gamma, eta, rabi, omega`` (explicit grid
origins: x_i = x0 + i dx, y_j = y0 + j dy) and the optional keys ``gx, gy``
(trap frequencies, default 1), ``split`` (0 Lie, 1 Strang), ``fix_m`` and
``magnetization`` (imaginary-time projection to a fixed magnetisation).  Wave functions are complex128
arrays of shape (3, ny, nx), components ordered m = +1, 0, -1.

Every function cites the passage of arXiv:2105.10517 it follows; the C file
header lists the readings taken where the paper is silent.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")

PARAM_KEYS = ("nx", "ny", "dx", "dy", "x0", "y0", "dt", "c0", "c2", "gamma", "eta", "rabi", "omega")
OPTIONAL_KEYS = {"gx": 1.0, "gy": 1.0, "split": 0, "fix_m": 0, "magnetization": 0.0}


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("dt", ctypes.c_double),
                ("c0", ctypes.c_double), ("c2", ctypes.c_double), ("gamma", ctypes.c_double),
                ("eta", ctypes.c_int32), ("rabi", ctypes.c_double), ("omega", ctypes.c_double),
                ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("split", ctypes.c_int32),
                ("fix_m", ctypes.c_int32), ("magnetization", ctypes.c_double)]


class _Obs(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double * 3), ("norm_total", ctypes.c_double),
                ("magnetization", ctypes.c_double), ("energy", ctypes.c_double),
                ("e_kin", ctypes.c_double), ("e_trap", ctypes.c_double), ("e_int", ctypes.c_double),
                ("e_rot", ctypes.c_double), ("e_so", ctypes.c_double), ("e_rabi", ctypes.c_double),
                ("lz", ctypes.c_double), ("mu", ctypes.c_double * 3), ("mu_total", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIBPATH)
        P = ctypes.POINTER(_Params)
        vp = ctypes.c_void_p
        for name, args in [("orc_pointwise", [P, vp, ctypes.c_int]),
                           ("orc_sweep_x", [P, vp, ctypes.c_int]),
                           ("orc_sweep_y", [P, vp, ctypes.c_int]),
                           ("orc_normalize", [P, vp]),
                           ("orc_step", [P, vp, ctypes.c_int64, ctypes.c_int]),
                           ("orc_apply_h", [P, vp, vp]),
                           ("orc_local_matrix", [P, vp, ctypes.c_double, ctypes.c_double, vp]),
                           ("orc_observables", [P, vp, ctypes.POINTER(_Obs)]),
                           ("orc_set_threads", [ctypes.c_int])]:
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = None
        lib.orc_norm.argtypes = [P, vp]
        lib.orc_norm.restype = ctypes.c_double
        lib.orc_get_threads.argtypes = []
        lib.orc_get_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _params(p) -> _Params:
    missing = [k for k in PARAM_KEYS if k not in p]
    if missing:
        raise KeyError(f"oracle parameters missing {missing}")
    return _Params(int(p["nx"]), int(p["ny"]), float(p["dx"]), float(p["dy"]), float(p["x0"]),
                   float(p["y0"]), float(p["dt"]), float(p["c0"]), float(p["c2"]), float(p["gamma"]),
                   int(p["eta"]), float(p["rabi"]), float(p["omega"]),
                   float(p.get("gx", 1.0)), float(p.get("gy", 1.0)), int(p.get("split", 0)),
                   int(bool(p.get("fix_m", 0))), float(p.get("magnetization", 0.0)))


def _checked(p, psi):
    a = np.ascontiguousarray(np.array(psi, dtype=np.complex128, copy=True))
    if a.shape != (3, int(p["ny"]), int(p["nx"])):
        raise ValueError(f"psi shape {a.shape} != (3, ny, nx)")
    return a


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def pointwise(p, psi, imag: bool):
    """Local substep exp(-i dt H_loc) / exp(-dt H_loc) (Eqs. S.1-S.3, S.5)."""
    a = _checked(p, psi)
    _load().orc_pointwise(ctypes.byref(_params(p)), a.ctypes.data, int(bool(imag)))
    return a


def sweep_x(p, psi, imag: bool):
    """Crank-Nicolson x sweep with the x parts of -Omega L_z and of the SO term."""
    a = _checked(p, psi)
    _load().orc_sweep_x(ctypes.byref(_params(p)), a.ctypes.data, int(bool(imag)))
    return a


def sweep_y(p, psi, imag: bool):
    """Crank-Nicolson y sweep with the y parts of -Omega L_z and of the SO term."""
    a = _checked(p, psi)
    _load().orc_sweep_y(ctypes.byref(_params(p)), a.ctypes.data, int(bool(imag)))
    return a


def normalize(p, psi):
    """psi / sqrt(dx dy sum |psi|^2): the normalisation condition after Eq. (S.5)."""
    a = _checked(p, psi)
    _load().orc_normalize(ctypes.byref(_params(p)), a.ctypes.data)
    return a


def norm(p, psi) -> float:
    a = _checked(p, psi)
    return float(_load().orc_norm(ctypes.byref(_params(p)), a.ctypes.data))


def step(p, psi, nsteps: int, imag: bool):
    """nsteps SSCN steps (local, x, y, and renormalisation in imaginary time)."""
    a = _checked(p, psi)
    _load().orc_step(ctypes.byref(_params(p)), a.ctypes.data, int(nsteps), int(bool(imag)))
    return a


def apply_h(p, psi):
    """Right-hand sides of Eqs. (S.1)-(S.2) on the grid (zero ghost points)."""
    a = _checked(p, psi)
    out = np.empty_like(a)
    _load().orc_apply_h(ctypes.byref(_params(p)), a.ctypes.data, out.ctypes.data)
    return out


def local_matrix(p, v, x: float, y: float):
    """3x3 H_loc = (V + c0 rho) I + c2 F.Sigma + R Sigma_x at one point."""
    vv = np.ascontiguousarray(np.array(v, dtype=np.complex128).reshape(3))
    H = np.zeros(9, dtype=np.complex128)
    _load().orc_local_matrix(ctypes.byref(_params(p)), vv.ctypes.data, float(x), float(y), H.ctypes.data)
    return H.reshape(3, 3)


def observables(p, psi) -> dict:
    """Norms, magnetisation, the Eq. (S.6) energy and its parts, <L_z>, mu_m, mu."""
    a = _checked(p, psi)
    o = _Obs()
    _load().orc_observables(ctypes.byref(_params(p)), a.ctypes.data, ctypes.byref(o))
    return {"norm": list(o.norm), "norm_total": o.norm_total, "magnetization": o.magnetization,
            "energy": o.energy, "e_kin": o.e_kin, "e_trap": o.e_trap, "e_int": o.e_int, "e_rot": o.e_rot,
            "e_so": o.e_so, "e_rabi": o.e_rabi, "lz": o.lz, "mu": list(o.mu), "mu_total": o.mu_total}


# Bohr radius in metres (CODATA 2018).
BOHR_RADIUS_M = 5.29177210903e-11


def couplings(n_atoms: float, a0_bohr: float, a2_bohr: float, l0_over_sqrt_kappa_m: float):
    """c0, c2 of Eq. (S.4): c0 = 2 N sqrt(2 pi kappa) (a0 + 2 a2) / (3 l0),
    c2 = 2 N sqrt(2 pi kappa) (a2 - a0) / (3 l0); the length l0/sqrt(kappa) is
    passed directly (the paper quotes it, 4 micrometres)."""
    pref = 2.0 * n_atoms * math.sqrt(2.0 * math.pi) / (3.0 * l0_over_sqrt_kappa_m)
    return (pref * (a0_bohr + 2.0 * a2_bohr) * BOHR_RADIUS_M,
            pref * (a2_bohr - a0_bohr) * BOHR_RADIUS_M)
