"""ORACLE (test infrastructure): Python side of the quadrature element.

Builds oracle/element.c with gcc on first use (or from the build step) and
calls it through ctypes.  Arrays cross as host float64/int32 AoS arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .quadrature import tet_rule

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "element.c")
_LIB = os.path.join(_HERE, "liboracle_element.so")
_lib = None

NDOF = 19


def build(force: bool = True) -> str:
    """Compile the oracle's C element with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_element.restype = ctypes.c_int
        lib.oracle_element.argtypes = [ctypes.c_int64, ip, dp, dp, dp, dp, dp, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp,
                                       ctypes.c_int, dp, dp, dp, dp]
        _lib = lib
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def element_residual_tangent(xyz, tets, u, beta, nu, dt=0.0, u_prev=None, body=None,
                             bubble_scale=1.0, with_tangent=True, n_quad=7, picard=False, advect=None):
    """Element residuals R [E, 19] and tangents K [E, 19, 19] (K None if not requested).

    xyz [n_nodes, 3], tets [E, 4], u [n_nodes, 4] = (v, p), beta [E, 3],
    nu kinematic viscosity, dt <= 0 for steady (u_prev ignored), body
    [n_nodes, 3] P1 nodal body force or None.  picard: the fixed-point tangent
    (advecting velocity held fixed) instead of Newton's.  advect = (u_adv, beta_adv):
    the advecting velocity of the residual's convective term from that state (tests of
    the fixed-point tangent); None: the state itself.
    """
    lib = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    u = np.ascontiguousarray(u, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    E = tets.shape[0]
    transient = dt is not None and dt > 0
    up = np.ascontiguousarray(u_prev, dtype=np.float64) if transient else None
    if transient and up is None:
        raise ValueError("transient run needs u_prev")
    f = None if body is None else np.ascontiguousarray(body, dtype=np.float64)
    lam, w = tet_rule(n_quad)
    lam = np.ascontiguousarray(lam)
    w = np.ascontiguousarray(w)
    ua = ba = None
    if advect is not None:
        ua = np.ascontiguousarray(advect[0], dtype=np.float64)
        ba = np.ascontiguousarray(advect[1], dtype=np.float64)
        assert ua.shape == u.shape and ba.shape == beta.shape
    R = np.zeros((E, NDOF))
    K = np.zeros((E, NDOF, NDOF)) if with_tangent else None
    rc = lib.oracle_element(E, _ptr(tets, ctypes.c_int32), _ptr(xyz, ctypes.c_double),
                            _ptr(u, ctypes.c_double), _ptr(up, ctypes.c_double),
                            _ptr(beta, ctypes.c_double), _ptr(f, ctypes.c_double),
                            float(nu), (1.0 / dt) if transient else 0.0, float(bubble_scale),
                            1 if picard else 0, _ptr(ua, ctypes.c_double), _ptr(ba, ctypes.c_double),
                            int(lam.shape[0]), _ptr(lam, ctypes.c_double), _ptr(w, ctypes.c_double),
                            _ptr(R, ctypes.c_double), _ptr(K, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"degenerate element {rc - 1} (det J <= 0)")
    return R, K
