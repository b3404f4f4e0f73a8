"""ORACLE (test infrastructure only): build and load the plain C oracle code."""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stepping.c")
_LIB = os.path.join(_HERE, "_stepping.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile stepping.c with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        _lib.pd_oracle_step_1d.argtypes = [ctypes.c_int, ctypes.c_int,
                                           ctypes.c_double] + [dp] * 9
        _lib.pd_oracle_step_1d.restype = ctypes.c_int
    return _lib
