"""FP64 CPU oracle for the line-by-line opacity hot path (HELIOS-K 2.0, arXiv:2101.02005).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``. The product package never imports it.

The arithmetic lives in ``oracle.c`` (plain C, IEEE double, OpenMP over output points);
this module only builds that file with gcc and marshals numpy arrays through ctypes.
Definitions followed (see the header of oracle.c for the full list):

* S(T): Sec. 2.2.2 eq. (S) in the form of eq. (S1) with S' (Sec. 2.4.3, step 1).
* alpha: inverse of eq. (alphaD); gamma: the ExoMol Lorentz width of Sec. 2.2 without
  the natural-broadening term.
* V = Re w(x+iy)/(sqrt(pi) alpha), x, y as in Sec. 2.4.2.
* k_j = sum of S_i V over lines with |nu_j - nu_i| <= cut (Sec. 2.4.3, step 4).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile oracle.c with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Species(ctypes.Structure):
    _fields_ = [("mass_amu", ctypes.c_double), ("T_ref", ctypes.c_double),
                ("P_ref_atm", ctypes.c_double), ("q_a", ctypes.c_double), ("q_b", ctypes.c_double)]


_lib = None
GH_NODES = 32  # Gauss-Hermite nodes of the far-wing profile derivatives
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64, dbl, sp = ctypes.c_int64, ctypes.c_double, ctypes.POINTER(Species)
        lib.or_faddeeva_arr.argtypes = [i64, _D, _D, _D, _D]
        lib.or_voigt_arr.argtypes = [i64, _D, _D, _D, _D]
        lib.or_line_params.argtypes = [i64, _D, _D, _D, _D, _D, sp, dbl, dbl, _D, _D, _D]
        lib.or_opacity.argtypes = [i64, _D, _D, _D, _D, _D, sp, dbl, dbl, dbl, dbl, dbl, i64, _I64, _D]
        lib.or_opacity.restype = ctypes.c_int
        lib.or_gradient.argtypes = [i64, _D, _D, _D, _D, _D, sp, dbl, dbl, dbl, dbl, i64, dbl, _D, i64,
                                    _I64, _D, _D, _D, _D, _D, _D, _D, _D]
        lib.or_gradient.restype = ctypes.c_int
        lib.or_line_functional.argtypes = [i64, _D, _D, _D, _D, _D, sp, dbl, dbl, dbl, dbl, i64, dbl,
                                           _D, _D]
        lib.or_count_evals.argtypes = [i64, _D, dbl, dbl, i64, dbl]
        lib.or_count_evals.restype = ctypes.c_int64
        lib.or_jranges.argtypes = [i64, _D, dbl, dbl, i64, dbl, _I64, _I64]
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_voigt_derivs_arr.argtypes = [i64, _D, _D, _D, _D, _D, _D]
        ci = ctypes.c_int
        lib.or_opacity_ex.argtypes = [i64, _D, _D, _D, _D, _D, sp, dbl, dbl, dbl, dbl, dbl, ci, ci, ci, i64,
                                      _I64, _D]
        lib.or_opacity_ex.restype = ctypes.c_int
        lib.or_gradient_ex.argtypes = [i64, _D, _D, _D, _D, _D, sp, dbl, dbl, dbl, dbl, i64, dbl, ci, ci, _D,
                                       i64, _I64, _D, _D, _D, _D, _D, _D, _D, _D]
        lib.or_gradient_ex.restype = ctypes.c_int
        lib.or_cut_lengths.argtypes = [i64, _D, _D, _D, sp, dbl, dbl, ci, dbl, _D]
        lib.or_opacity_hitran.argtypes = [i64, _D, _D, _D, _D, _D, _D, _D, sp, dbl, dbl, dbl, dbl, dbl, dbl, ci,
                                          ci, ci, i64, _I64, _D]
        lib.or_opacity_hitran.restype = ctypes.c_int
        lib.or_set_gauss_hermite.argtypes = [ctypes.c_int, _D, _D]
        lib.or_set_gauss_hermite.restype = ctypes.c_int
        t, w = np.polynomial.hermite.hermgauss(GH_NODES)
        t, w = _d(t), _d(w)
        if lib.or_set_gauss_hermite(GH_NODES, _p(t), _p(w)) != 0:
            raise RuntimeError("or_set_gauss_hermite failed")
        _lib = lib
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _pi(a):
    return a.ctypes.data_as(_I64) if a is not None else None


def species(mass_amu, T_ref=296.0, P_ref_atm=1.0, q_a=0.05, q_b=1.5):
    return Species(mass_amu, T_ref, P_ref_atm, q_a, q_b)


def num_threads():
    return int(_load().or_num_threads())


def faddeeva(x, y):
    """w(x + i y) for y >= 0 (complex128 array)."""
    x, y = np.broadcast_arrays(_d(x), _d(y))
    x, y = _d(x).ravel(), _d(y).ravel()
    re, im = np.empty_like(x), np.empty_like(x)
    _load().or_faddeeva_arr(x.size, _p(x), _p(y), _p(re), _p(im))
    return re + 1j * im


def voigt(delta, alpha, gamma):
    """Unit-area Voigt profile V(delta; alpha, gamma) = Re w((delta + i gamma)/alpha)/(sqrt(pi) alpha)."""
    d, a, g = np.broadcast_arrays(_d(delta), _d(alpha), _d(gamma))
    d, a, g = _d(d).ravel(), _d(a).ravel(), _d(g).ravel()
    out = np.empty_like(d)
    _load().or_voigt_arr(d.size, _p(d), _p(a), _p(g), _p(out))
    return out


def voigt_derivs(delta, alpha, gamma, with_delta=False):
    """(dV/dgamma, dV/dalpha[, dV/ddelta]) of the unit-area Voigt profile (closed form near the
    centre, Gauss-Hermite quadrature of the convolution integral for |z| >= 10)."""
    d, a, g = np.broadcast_arrays(_d(delta), _d(alpha), _d(gamma))
    d, a, g = _d(d).ravel(), _d(a).ravel(), _d(g).ravel()
    dg, da, dd = np.empty_like(d), np.empty_like(d), np.empty_like(d)
    _load().or_voigt_derivs_arr(d.size, _p(d), _p(a), _p(g), _p(dg), _p(da), _p(dd))
    return (dg, da, dd) if with_delta else (dg, da)


def line_params(lines, sp, T, P):
    """(S(T), alpha, gamma) per line."""
    nu, S, E, g, n = (_d(lines[k]) for k in ("nu", "S_ref", "E", "gamma_ref", "n"))
    N = nu.size
    o = [np.empty(N) for _ in range(3)]
    _load().or_line_params(N, _p(nu), _p(S), _p(E), _p(g), _p(n), ctypes.byref(sp), T, P,
                           _p(o[0]), _p(o[1]), _p(o[2]))
    return o


def opacity(lines, sp, T, P, nu_start, dnu, cut, pts):
    """FP64 k at the grid indices ``pts`` (cut = inf: no cut)."""
    nu, S, E, g, n = (_d(lines[k]) for k in ("nu", "S_ref", "E", "gamma_ref", "n"))
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.empty(pts.size)
    rc = _load().or_opacity(nu.size, _p(nu), _p(S), _p(E), _p(g), _p(n), ctypes.byref(sp), T, P,
                            nu_start, dnu, cut, pts.size, _pi(pts), _p(out))
    if rc != 0:
        raise ValueError("or_opacity: invalid arguments (%d)" % rc)
    return out


def gradient(lines, sp, T, P, nu_start, dnu, n_grid, cut, g, sel=None):
    """Analytic FP64 adjoint of L = sum_j g_j k_j for the lines ``sel`` (default: all).

    Returns a dict of per-line arrays: GS, Gg, Ga, dS_ref, dgamma_ref, dn, dT_part, dlnP_part."""
    nu, S, E, gr, n = (_d(lines[k]) for k in ("nu", "S_ref", "E", "gamma_ref", "n"))
    gg = _d(g)
    assert gg.size == n_grid
    sel = np.arange(nu.size, dtype=np.int64) if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    names = ("GS", "Gg", "Ga", "dS_ref", "dgamma_ref", "dn", "dT_part", "dlnP_part")
    out = {k: np.empty(sel.size) for k in names}
    rc = _load().or_gradient(nu.size, _p(nu), _p(S), _p(E), _p(gr), _p(n), ctypes.byref(sp), T, P,
                             nu_start, dnu, n_grid, cut, _p(gg), sel.size, _pi(sel),
                             *[_p(out[k]) for k in names])
    if rc != 0:
        raise ValueError("or_gradient: invalid arguments (%d)" % rc)
    return out


def line_functional(lines, sp, T, P, nu_start, dnu, n_grid, cut, g):
    """Per-line L_i = sum_j g_j S_i V_ij."""
    nu, S, E, gr, n = (_d(lines[k]) for k in ("nu", "S_ref", "E", "gamma_ref", "n"))
    gg = _d(g)
    out = np.empty(nu.size)
    _load().or_line_functional(nu.size, _p(nu), _p(S), _p(E), _p(gr), _p(n), ctypes.byref(sp), T, P,
                               nu_start, dnu, n_grid, cut, _p(gg), _p(out))
    return out


def count_evals(nu, nu_start, dnu, n_grid, cut):
    """Number of (line, grid point) pairs with |nu_j - nu_i| <= cut."""
    nu = _d(nu)
    return int(_load().or_count_evals(nu.size, _p(nu), nu_start, dnu, n_grid, cut))


def jranges(nu, nu_start, dnu, n_grid, cut):
    """Per-line inclusive grid-index range of the cut (j1 < j0: empty)."""
    nu = _d(nu)
    j0, j1 = np.empty(nu.size, np.int64), np.empty(nu.size, np.int64)
    _load().or_jranges(nu.size, _p(nu), nu_start, dnu, n_grid, cut, _pi(j0), _pi(j1))
    return j0, j1


# Options of the extended forward (profiles of Sec. 2.1, plinth of Sec. 2.1.1, cut modes of
# Sec. 2.4.3 step 4): the same codes as the library's options.
PROFILE_VOIGT, PROFILE_LORENTZ, PROFILE_DOPPLER, PROFILE_BINNED_GAUSS = 0, 1, 2, 3
CUT_FIXED, CUT_DOPPLER, CUT_LORENTZ = 0, 1, 2


def opacity_ex(lines, sp, T, P, nu_start, dnu, cut, pts, cut_mode=CUT_FIXED, profile=PROFILE_VOIGT, plinth=False):
    """FP64 k at the grid indices ``pts`` with a line profile, a cut mode (cut is then a multiple of
    the Doppler or Lorentz half-width) and optional plinth removal."""
    nu, S, E, g, n = (_d(lines[k]) for k in ("nu", "S_ref", "E", "gamma_ref", "n"))
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.empty(pts.size)
    rc = _load().or_opacity_ex(nu.size, _p(nu), _p(S), _p(E), _p(g), _p(n), ctypes.byref(sp), T, P,
                               nu_start, dnu, cut, int(cut_mode), int(profile), int(bool(plinth)), pts.size,
                               _pi(pts), _p(out))
    if rc != 0:
        raise ValueError("or_opacity_ex: invalid arguments (%d)" % rc)
    return out


def gradient_ex(lines, sp, T, P, nu_start, dnu, n_grid, cut, g, cut_mode=CUT_FIXED, plinth=False, sel=None):
    """As gradient(), for the Voigt profile with a cut mode and optional plinth removal."""
    nu, S, E, gr, n = (_d(lines[k]) for k in ("nu", "S_ref", "E", "gamma_ref", "n"))
    gg = _d(g)
    assert gg.size == n_grid
    sel = np.arange(nu.size, dtype=np.int64) if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    names = ("GS", "Gg", "Ga", "dS_ref", "dgamma_ref", "dn", "dT_part", "dlnP_part")
    out = {k: np.empty(sel.size) for k in names}
    rc = _load().or_gradient_ex(nu.size, _p(nu), _p(S), _p(E), _p(gr), _p(n), ctypes.byref(sp), T, P,
                                nu_start, dnu, n_grid, cut, int(cut_mode), int(bool(plinth)), _p(gg), sel.size,
                                _pi(sel), *[_p(out[k]) for k in names])
    if rc != 0:
        raise ValueError("or_gradient_ex: invalid arguments (%d)" % rc)
    return out


def cut_lengths(lines, sp, T, P, cut_mode, cut):
    """Per-line cutting length at (T, P) in cm^-1."""
    nu, g, n = (_d(lines[k]) for k in ("nu", "gamma_ref", "n"))
    out = np.empty(nu.size)
    _load().or_cut_lengths(nu.size, _p(nu), _p(g), _p(n), ctypes.byref(sp), T, P, int(cut_mode), cut, _p(out))
    return out


def opacity_hitran(lines, sp, T, P, P_self, nu_start, dnu, cut, pts, cut_mode=CUT_FIXED, profile=PROFILE_VOIGT,
                   plinth=False):
    """FP64 k at the grid indices ``pts`` for a HITRAN-style list: ``lines`` holds nu, S_ref, E,
    gamma_air, gamma_self, n and delta (the pressure shift, cm^-1/atm); the Lorentz half-width is
    eq. (gammaL) without the natural term and the centre is shifted to nu + delta P / P_ref."""
    f = [_d(lines[k]) for k in ("nu", "S_ref", "E", "gamma_air", "gamma_self", "n", "delta")]
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.empty(pts.size)
    rc = _load().or_opacity_hitran(f[0].size, *[_p(a) for a in f], ctypes.byref(sp), T, P, P_self, nu_start, dnu,
                                   cut, int(cut_mode), int(profile), int(bool(plinth)), pts.size, _pi(pts), _p(out))
    if rc != 0:
        raise ValueError("or_opacity_hitran: invalid arguments (%d)" % rc)
    return out
