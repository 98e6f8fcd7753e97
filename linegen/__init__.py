"""Seeded synthetic line lists shaped like the paper's workloads (input recipe only).

Both the oracle side (host twin, ``generate``/``select``) and the GPU side (device twin,
``generate_device``) draw their inputs here; the arithmetic is in ``linegen_core.h`` and
the two twins are bit-identical. This module holds none of the opacity method.
"""
import ctypes
import os
import subprocess

import numpy as np

from .configs import CONFIGS, Workload, workload  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_CORE = os.path.join(_HERE, "linegen_core.h")
_CPU_SRC = os.path.join(_HERE, "linegen_cpu.c")
_GPU_SRC = os.path.join(_HERE, "linegen_gpu.hip")
_CPU_LIB = os.path.join(_HERE, "liblinegen_cpu.so")
_GPU_LIB = os.path.join(_HERE, "liblinegen_gpu.so")


def _stale(lib, *srcs):
    return not os.path.exists(lib) or any(os.path.getmtime(lib) < os.path.getmtime(s) for s in srcs)


def build_cpu(force=False):
    if force or _stale(_CPU_LIB, _CPU_SRC, _CORE):
        tmp = _CPU_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _CPU_SRC, "-lm"])
        os.replace(tmp, _CPU_LIB)
    return _CPU_LIB


def build_gpu(force=False):
    if force or _stale(_GPU_LIB, _GPU_SRC, _CORE):
        tmp = _GPU_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["hipcc", "-O3", "--offload-arch=gfx950", "-ffp-contract=off",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-fPIC", "-shared", "-o", tmp, _GPU_SRC],
                              stderr=subprocess.DEVNULL if os.environ.get("HK_QUIET_BUILD") else None)
        os.replace(tmp, _GPU_LIB)
    return _GPU_LIB


class Recipe(ctypes.Structure):
    _fields_ = [("nu_law", ctypes.c_int32), ("e_law", ctypes.c_int32), ("s_reading", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("nu_lo", ctypes.c_double), ("nu_hi", ctypes.c_double),
                ("s_lo", ctypes.c_double), ("s_hi", ctypes.c_double), ("e_par", ctypes.c_double),
                ("g_lo", ctypes.c_double), ("g_hi", ctypes.c_double), ("n_lo", ctypes.c_double),
                ("n_hi", ctypes.c_double), ("T_ref", ctypes.c_double)]


_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_cpu = None
_gpu = None
FIELDS = ("nu", "S_ref", "E", "gamma_ref", "n")


def _cpu_lib():
    global _cpu
    if _cpu is None:
        lib = ctypes.CDLL(build_cpu())
        R = ctypes.POINTER(Recipe)
        lib.lg_generate.argtypes = [R, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, _D, _D, _D, _D, _D]
        lib.lg_select_par.argtypes = [R, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int64, _I64, _D, _D, _D, _D, _D, _I64, ctypes.c_int]
        lib.lg_select_par.restype = ctypes.c_int64
        lib.lg_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _D]
        lib.lg_math.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D]
        _cpu = lib
    return _cpu


def _gpu_lib():
    global _gpu
    if _gpu is None:
        if not os.path.exists(_GPU_LIB):
            raise RuntimeError("linegen: %s is not built (run __graft_entry__.build())" % _GPU_LIB)
        lib = ctypes.CDLL(_GPU_LIB)
        lib.lg_generate_device.argtypes = [ctypes.POINTER(Recipe), ctypes.c_uint64, ctypes.c_int64,
                                           ctypes.c_int64] + [ctypes.c_void_p] * 5 + [ctypes.c_void_p]
        lib.lg_generate_device.restype = ctypes.c_int
        _gpu = lib
    return _gpu


def _p(a):
    return a.ctypes.data_as(_D)


def generate(recipe, seed, N, i0=0):
    """Host twin: lines i0 .. i0+N-1 as a dict of float64 arrays."""
    out = {k: np.empty(N) for k in FIELDS}
    _cpu_lib().lg_generate(ctypes.byref(recipe), seed, i0, N, *[_p(out[k]) for k in FIELDS])
    return out


def select(recipe, seed, N, nu_lo, nu_hi, cap=None):
    """Host twin: the lines of [0, N) with nu in [nu_lo, nu_hi), in index order.

    Returns (idx, lines). Raises if more than ``cap`` lines fall in the interval."""
    cap = int(cap if cap is not None else 1 << 22)
    idx = np.empty(cap, np.int64)
    out = {k: np.empty(cap) for k in FIELDS}
    nb = 256
    scratch = np.empty(nb, np.int64)
    tot = _cpu_lib().lg_select_par(ctypes.byref(recipe), seed, N, nu_lo, nu_hi, cap,
                                   idx.ctypes.data_as(_I64), *[_p(out[k]) for k in FIELDS],
                                   scratch.ctypes.data_as(_I64), nb)
    if tot > cap:
        raise ValueError("linegen.select: %d lines in [%g, %g) exceed cap %d" % (tot, nu_lo, nu_hi, cap))
    return idx[:tot].copy(), {k: v[:tot].copy() for k, v in out.items()}


def uniforms(seed, i0, count, f):
    out = np.empty(count)
    _cpu_lib().lg_uniforms(seed, i0, count, f, _p(out))
    return out


def math_helper(which, x):
    """The generator's own exp (0), expm1 (1) or log (2) on the host (for its tests)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    _cpu_lib().lg_math({"exp": 0, "expm1": 1, "log": 2}[which], x.size, _p(x), _p(y))
    return y


def generate_device(recipe, seed, N, ptrs, stream=0, i0=0):
    """Device twin: fill five device float64 arrays (pointers, in FIELDS order) with lines i0..i0+N-1."""
    rc = _gpu_lib().lg_generate_device(ctypes.byref(recipe), seed, i0, N, *[ctypes.c_void_p(p) for p in ptrs],
                                       ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError("lg_generate_device failed with HIP error %d" % rc)
