"""ctypes binding of libhk.so (include/hk.h). Argument marshalling only: every step of the
computation runs in the library's HIP kernels. Device arrays are torch tensors on the
current GPU; the stream is torch's current stream unless one is given."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhk.so")

HK_OK, HK_EINVAL, HK_ENOMEM, HK_EDEVICE, HK_EUNSUPPORTED = 0, 1, 2, 3, 4
_NAMES = {0: "HK_OK", 1: "HK_EINVAL", 2: "HK_ENOMEM", 3: "HK_EDEVICE", 4: "HK_EUNSUPPORTED"}


class HkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_NAMES.get(status, status), msg))
        self.status = status


class Species(ctypes.Structure):
    _fields_ = [("mass_amu", ctypes.c_double), ("T_ref", ctypes.c_double), ("P_ref_atm", ctypes.c_double),
                ("q_a", ctypes.c_double), ("q_b", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("nu_start", ctypes.c_double), ("dnu", ctypes.c_double), ("n", ctypes.c_int64)]


class LineOverride(ctypes.Structure):
    _fields_ = [("S_ref", ctypes.c_void_p), ("gamma_ref", ctypes.c_void_p), ("n_exp", ctypes.c_void_p)]


class Timings(ctypes.Structure):
    _fields_ = [("prep_ms", ctypes.c_double), ("worklist_ms", ctypes.c_double), ("voigt_ms", ctypes.c_double),
                ("combine_ms", ctypes.c_double), ("backward_ms", ctypes.c_double), ("bin_ms", ctypes.c_double),
                ("tile_width", ctypes.c_int32), ("lines_per_batch", ctypes.c_int32),
                ("chunk_lines", ctypes.c_int32), ("n_items", ctypes.c_int32), ("core_ms", ctypes.c_double),
                ("core_evals", ctypes.c_int64), ("far_ms", ctypes.c_double),
                ("wing_evals", ctypes.c_int64), ("class_evals", ctypes.c_int64 * 8), ("status", ctypes.c_int32),
                ("backward_evals", ctypes.c_int64)]


# evaluation classes of Timings.class_evals
CLASS_NAMES = ("direct", "far", "very_far", "middle", "masked", "tile_far", "tile_far8", "core")

PROFILE_VOIGT, PROFILE_LORENTZ, PROFILE_DOPPLER, PROFILE_BINNED_GAUSS = 0, 1, 2, 3
CUT_FIXED, CUT_DOPPLER, CUT_LORENTZ = 0, 1, 2


class Options(ctypes.Structure):
    _fields_ = [("profile", ctypes.c_int32), ("cut_mode", ctypes.c_int32), ("plinth", ctypes.c_int32),
                ("direct", ctypes.c_int32)]


_lib = None
_vp, _i64, _i32, _dbl, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t


def load():
    """Load libhk.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhk.so is not built at %s: run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    sig = {
        "hk_prepare_lines": ([_vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(Species), _vp, ctypes.POINTER(_vp)], st),
        "hk_release_lines": ([_vp], st),
        "hk_empty_cache": ([], st),
        "hk_lines_count": ([_vp], _i64),
        "hk_workspace_size": ([_vp, ctypes.c_int, _i32, _i32, ctypes.POINTER(Grid), _dbl, ctypes.POINTER(_sz)], st),
        "hk_opacity": ([_vp, ctypes.POINTER(LineOverride), _dbl, _dbl, Grid, _dbl, _vp, _vp, _sz, _vp], st),
        "hk_opacity_batched": ([_vp, _i32, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), ctypes.POINTER(Grid),
                                ctypes.POINTER(_i64), _dbl, _vp, _vp, _sz, _vp], st),
        "hk_opacity_backward": ([_vp, ctypes.POINTER(LineOverride), _dbl, _dbl, Grid, _dbl, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _sz, _vp], st),
        "hk_debug_cut_bounds": ([_vp, Grid, _dbl, _vp, _vp, _vp], st),
        "hk_debug_sorted": ([_vp, _vp, _vp, _vp], st),
        "hk_debug_line_params": ([_vp, _dbl, _dbl, _vp, _vp, _vp, _vp], st),
        "hk_get_timings": ([ctypes.POINTER(Timings)], st),
        "hk_workspace_size_ex": ([_vp, ctypes.c_int, _i32, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl),
                                  ctypes.POINTER(Grid), _dbl, ctypes.POINTER(Options), _vp, ctypes.POINTER(_sz)], st),
        "hk_opacity_ex": ([_vp, ctypes.POINTER(LineOverride), _dbl, _dbl, Grid, _dbl, ctypes.POINTER(Options), _vp,
                           _vp, _sz, _vp], st),
        "hk_opacity_batched_ex": ([_vp, _i32, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), ctypes.POINTER(Grid),
                                   ctypes.POINTER(_i64), _dbl, ctypes.POINTER(Options), _vp, _vp, _sz, _vp], st),
        "hk_opacity_noalloc": ([_vp, ctypes.POINTER(LineOverride), _dbl, _dbl, Grid, _dbl, _vp, _vp], st),
        "hk_noalloc_max_bytes": ([], _sz),
        "hk_prepare_lines_hitran": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(Species), _vp,
                                     ctypes.POINTER(_vp)], st),
        "hk_workspace_size_hitran": ([_vp, _dbl, _dbl, _dbl, Grid, _dbl, ctypes.POINTER(Options), _vp,
                                      ctypes.POINTER(_sz)], st),
        "hk_opacity_hitran": ([_vp, _dbl, _dbl, _dbl, Grid, _dbl, ctypes.POINTER(Options), _vp, _vp, _sz, _vp], st),
        "hk_opacity_stream": ([_vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(Species), _dbl, _dbl, Grid, _dbl,
                               ctypes.POINTER(Options), _i64, _vp, _vp], st),
        "hk_debug_grid_records": ([_vp, _dbl, _dbl, Grid, _dbl, ctypes.POINTER(Options), _vp, _sz, _vp, _vp, _vp,
                                   _vp], st),
        "hk_last_error": ([], ctypes.c_char_p),
        "hk_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(status):
    if status != HK_OK:
        raise HkError(status, load().hk_last_error().decode())


def _stream(stream):
    """The HIP stream handle of `stream` (a torch.cuda.Stream, a raw handle, or None for torch's
    current stream)."""
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def _keep_for_stream(stream, *tensors):
    """Tensors allocated here on torch's current stream but used by kernels enqueued on another
    stream: tell torch's caching allocator not to hand their memory out again before that stream's
    work has reached this point."""
    if stream is None:
        return
    import torch
    h = int(getattr(stream, "cuda_stream", stream))
    if h == torch.cuda.current_stream().cuda_stream:
        return
    ts = stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.ExternalStream(h)
    for t in tensors:
        if t is not None:
            t.record_stream(ts)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Lines:
    """Owner of an hk_lines handle (the binned line list on the GPU)."""

    def __init__(self, handle, n_lines, species):
        self.handle = handle
        self.n_lines = n_lines
        self.species = species

    def release(self):
        if self.handle:
            h, self.handle = self.handle, None
            _check(load().hk_release_lines(h))

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.release()


def species(mass_amu, T_ref=296.0, P_ref_atm=1.0, q_a=0.05, q_b=1.5):
    return Species(mass_amu, T_ref, P_ref_atm, q_a, q_b)


def grid(nu_start, dnu, n):
    return Grid(nu_start, dnu, n)


def hk_prepare_lines(nu, S_ref, E_low, gamma_ref, n_exp, sp, stream=None):
    """Bin a device line list (float64 tensors, equal length). Returns a Lines handle."""
    n = int(nu.numel())
    for t in (nu, S_ref, E_low, gamma_ref, n_exp):
        if t.numel() != n or not t.is_contiguous():
            raise ValueError("line arrays must be contiguous and of equal length")
    h = ctypes.c_void_p()
    _check(load().hk_prepare_lines(_ptr(nu), _ptr(S_ref), _ptr(E_low), _ptr(gamma_ref), _ptr(n_exp), n,
                                   ctypes.byref(sp), _stream(stream), ctypes.byref(h)))
    return Lines(h.value, n, sp)


def hk_prepare_lines_hitran(nu, S_ref, E_low, gamma_air, gamma_self, n_exp, delta_air, sp, stream=None):
    """Bin a HITRAN-style device line list (float64 tensors: the five fields of hk_prepare_lines
    with gamma_air as the width, plus gamma_self and the pressure shift delta_air)."""
    n = int(nu.numel())
    for t in (nu, S_ref, E_low, gamma_air, gamma_self, n_exp, delta_air):
        if t.numel() != n or not t.is_contiguous():
            raise ValueError("line arrays must be contiguous and of equal length")
    h = ctypes.c_void_p()
    _check(load().hk_prepare_lines_hitran(_ptr(nu), _ptr(S_ref), _ptr(E_low), _ptr(gamma_air), _ptr(gamma_self),
                                          _ptr(n_exp), _ptr(delta_air), n, ctypes.byref(sp), _stream(stream),
                                          ctypes.byref(h)))
    return Lines(h.value, n, sp)


def hk_opacity_hitran(lines, T, P_atm, P_self, grd, cutoff, k=None, ws=None, opts=None, stream=None):
    """k (float32 tensor of grd.n) of a HITRAN-style list at (T, P, P_self)."""
    import torch
    new_k = k is None
    if new_k:
        k = torch.empty(grd.n, dtype=torch.float32, device="cuda")
    need = ctypes.c_size_t()
    _check(load().hk_workspace_size_hitran(ctypes.c_void_p(lines.handle), float(T), float(P_atm), float(P_self), grd,
                                           float(cutoff), _opts(opts), _stream(stream), ctypes.byref(need)))
    need = need.value
    new_ws = ws is None or ws.numel() < need + 256
    if new_ws:
        ws = _workspace(need, k.device)
    _check(load().hk_opacity_hitran(ctypes.c_void_p(lines.handle), float(T), float(P_atm), float(P_self), grd,
                                    float(cutoff), _opts(opts), _ptr(k), ctypes.c_void_p(_aligned(ws)), need,
                                    _stream(stream)))
    _keep_for_stream(stream, k if new_k else None, ws if new_ws else None)
    return k


def hk_opacity_stream(nu, S_ref, E_low, gamma_ref, n_exp, sp, T, P_atm, grd, cutoff, chunk_lines, k=None,
                      opts=None, stream=None):
    """k of a line list in host memory (contiguous float64 numpy arrays or CPU tensors, ideally
    pinned), processed in chunks of chunk_lines lines with the copies overlapping the work."""
    import numpy as np
    import torch
    arrs = []
    for a in (nu, S_ref, E_low, gamma_ref, n_exp):
        if isinstance(a, torch.Tensor):
            if a.is_cuda or a.dtype != torch.float64 or not a.is_contiguous():
                raise ValueError("host arrays must be contiguous float64 CPU tensors")
            arrs.append(ctypes.c_void_p(a.data_ptr()))
        else:
            a = np.ascontiguousarray(a, dtype=np.float64)
            arrs.append((a, ctypes.c_void_p(a.ctypes.data)))
    ptrs = [x[1] if isinstance(x, tuple) else x for x in arrs]
    n = len(nu)
    if k is None:
        k = torch.empty(grd.n, dtype=torch.float32, device="cuda")
    _check(load().hk_opacity_stream(*ptrs, n, ctypes.byref(sp), float(T), float(P_atm), grd, float(cutoff), _opts(opts),
                                    int(chunk_lines), _ptr(k), _stream(stream)))
    return k


def hk_release_lines(lines):
    lines.release()


def hk_empty_cache():
    """Return the library's cached device blocks (released handles, binning temporaries)."""
    _check(load().hk_empty_cache())


def hk_workspace_size(lines, mode, grids, cutoff, n_temps=None):
    grids = list(grids)
    arr = (Grid * len(grids))(*grids)
    out = ctypes.c_size_t()
    _check(load().hk_workspace_size(ctypes.c_void_p(lines.handle), mode, len(grids),
                                    len(grids) if n_temps is None else n_temps, arr, cutoff, ctypes.byref(out)))
    return out.value


def _workspace(nbytes, device=None):
    import torch
    return torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device or "cuda")


def _aligned(ws):
    p = ws.data_ptr()
    return p + ((256 - p % 256) % 256)


def _override(ovr):
    if ovr is None:
        return None
    S, g, n = ovr
    return ctypes.byref(LineOverride(_ptr(S).value, _ptr(g).value, _ptr(n).value))


def options(profile=0, cut_mode=0, plinth=0, direct=0):
    return Options(int(profile), int(cut_mode), int(plinth), int(direct))


def _opts(opts):
    if opts is None:
        return None
    if isinstance(opts, dict):
        opts = options(**opts)
    return ctypes.byref(opts)


def hk_workspace_size_ex(lines, mode, T, P_atm, grids, cutoff, opts=None, stream=None):
    grids = list(grids)
    n = len(grids)
    Ta = (ctypes.c_double * n)(*[float(t) for t in T]) if T is not None else None
    Pa = (ctypes.c_double * n)(*[float(p) for p in P_atm]) if P_atm is not None else None
    out = ctypes.c_size_t()
    _check(load().hk_workspace_size_ex(ctypes.c_void_p(lines.handle), mode, n, Ta, Pa, (Grid * n)(*grids),
                                       float(cutoff), _opts(opts), _stream(stream), ctypes.byref(out)))
    return out.value


def hk_opacity(lines, T, P_atm, grd, cutoff, k=None, ws=None, ovr=None, stream=None, opts=None):
    """k (float32 tensor of grd.n) at one (T, P). ovr: optional (S_ref, gamma_ref, n) float64 tensors.
    opts: None (the defaults, hk_opacity) or an Options / dict of its fields (hk_opacity_ex)."""
    import torch
    new_k = k is None
    if new_k:
        k = torch.empty(grd.n, dtype=torch.float32, device="cuda")
    if opts is None:
        need = hk_workspace_size(lines, 0, [grd], cutoff)
    else:
        need = hk_workspace_size_ex(lines, 0, [T], [P_atm], [grd], cutoff, opts, stream)
    new_ws = ws is None or ws.numel() < need + 256
    if new_ws:
        ws = _workspace(need, k.device)
    if opts is None:
        _check(load().hk_opacity(ctypes.c_void_p(lines.handle), _override(ovr), float(T), float(P_atm), grd,
                                 float(cutoff), _ptr(k), ctypes.c_void_p(_aligned(ws)), need, _stream(stream)))
    else:
        _check(load().hk_opacity_ex(ctypes.c_void_p(lines.handle), _override(ovr), float(T), float(P_atm), grd,
                                    float(cutoff), _opts(opts), _ptr(k), ctypes.c_void_p(_aligned(ws)), need,
                                    _stream(stream)))
    _keep_for_stream(stream, k if new_k else None, ws if new_ws else None)
    return k


def hk_opacity_noalloc(lines, T, P_atm, grd, cutoff, k, ovr=None, stream=None):
    """hk_opacity with the library's fixed scratch array as workspace: nothing is allocated (k is
    the caller's float32 tensor of grd.n)."""
    _check(load().hk_opacity_noalloc(ctypes.c_void_p(lines.handle), _override(ovr), float(T), float(P_atm), grd,
                                     float(cutoff), _ptr(k), _stream(stream)))
    return k


def hk_noalloc_max_bytes():
    return int(load().hk_noalloc_max_bytes())


def hk_debug_grid_records(lines, T, P_atm, grd, cutoff, opts=None, stream=None):
    """(j_lo, j_hi, plinth) per line in caller order, as an options call decides them."""
    import torch
    N = lines.n_lines
    lo = torch.empty(N, dtype=torch.int32, device="cuda")
    hi = torch.empty(N, dtype=torch.int32, device="cuda")
    pl = torch.empty(N, dtype=torch.float32, device="cuda")
    need = 28 * N + 768
    ws = _workspace(need)
    _check(load().hk_debug_grid_records(ctypes.c_void_p(lines.handle), float(T), float(P_atm), grd, float(cutoff),
                                        _opts(opts), ctypes.c_void_p(_aligned(ws)), need, _ptr(lo), _ptr(hi),
                                        _ptr(pl), _stream(stream)))
    _keep_for_stream(stream, lo, hi, pl, ws)
    return lo, hi, pl


def hk_opacity_batched(lines, T, P_atm, grids, cutoff, out_offset=None, k=None, ws=None, stream=None, opts=None):
    """k for several (T, P, grid) pairs in one launch; pair p writes k[out_offset[p]:][:grids[p].n]."""
    import torch
    n_pairs = len(T)
    grids = list(grids)
    if out_offset is None:
        out_offset, o = [], 0
        for g in grids:
            out_offset.append(o)
            o += g.n
    total = max(int(o_ + g.n) for o_, g in zip(out_offset, grids))
    new_k = k is None
    if new_k:
        k = torch.empty(total, dtype=torch.float32, device="cuda")
    if opts is None:
        need = hk_workspace_size(lines, 1, grids, cutoff, n_temps=len(set(float(t) for t in T)))
    else:
        need = hk_workspace_size_ex(lines, 1, T, P_atm, grids, cutoff, opts, stream)
    new_ws = ws is None or ws.numel() < need + 256
    if new_ws:
        ws = _workspace(need, k.device)
    Ta = (ctypes.c_double * n_pairs)(*[float(t) for t in T])
    Pa = (ctypes.c_double * n_pairs)(*[float(p) for p in P_atm])
    Ga = (Grid * n_pairs)(*grids)
    Oa = (ctypes.c_int64 * n_pairs)(*[int(o) for o in out_offset])
    if opts is None:
        _check(load().hk_opacity_batched(ctypes.c_void_p(lines.handle), n_pairs, Ta, Pa, Ga, Oa, float(cutoff),
                                         _ptr(k), ctypes.c_void_p(_aligned(ws)), need, _stream(stream)))
    else:
        _check(load().hk_opacity_batched_ex(ctypes.c_void_p(lines.handle), n_pairs, Ta, Pa, Ga, Oa, float(cutoff),
                                            _opts(opts), _ptr(k), ctypes.c_void_p(_aligned(ws)), need,
                                            _stream(stream)))
    _keep_for_stream(stream, k if new_k else None, ws if new_ws else None)
    return k


def hk_opacity_backward(lines, T, P_atm, grd, cutoff, dL_dk, ws=None, ovr=None, stream=None):
    """Returns (dL/dT_lnP float64[2], dL/dS_ref float64[N], dL/dgamma_ref float32[N], dL/dn float32[N])."""
    import torch
    N = lines.n_lines
    dev = dL_dk.device
    out2 = torch.empty(2, dtype=torch.float64, device=dev)
    dS = torch.empty(N, dtype=torch.float64, device=dev)
    dg = torch.empty(N, dtype=torch.float32, device=dev)
    dn = torch.empty(N, dtype=torch.float32, device=dev)
    need = hk_workspace_size(lines, 2, [grd], cutoff)
    new_ws = ws is None or ws.numel() < need + 256
    if new_ws:
        ws = _workspace(need, dev)
    _check(load().hk_opacity_backward(ctypes.c_void_p(lines.handle), _override(ovr), float(T), float(P_atm), grd,
                                      float(cutoff), _ptr(dL_dk), _ptr(out2), _ptr(dS), _ptr(dg), _ptr(dn),
                                      ctypes.c_void_p(_aligned(ws)), need, _stream(stream)))
    _keep_for_stream(stream, out2, dS, dg, dn, ws if new_ws else None)
    return out2, dS, dg, dn


def hk_debug_cut_bounds(lines, grd, cutoff, stream=None):
    import torch
    lo = torch.empty(lines.n_lines, dtype=torch.int32, device="cuda")
    hi = torch.empty(lines.n_lines, dtype=torch.int32, device="cuda")
    _check(load().hk_debug_cut_bounds(ctypes.c_void_p(lines.handle), grd, float(cutoff), _ptr(lo), _ptr(hi),
                                      _stream(stream)))
    _keep_for_stream(stream, lo, hi)
    return lo, hi


def hk_debug_sorted(lines, stream=None):
    import torch
    keys = torch.empty(lines.n_lines, dtype=torch.int32, device="cuda")
    perm = torch.empty(lines.n_lines, dtype=torch.int32, device="cuda")
    _check(load().hk_debug_sorted(ctypes.c_void_p(lines.handle), _ptr(keys), _ptr(perm), _stream(stream)))
    return keys, perm


def hk_debug_line_params(lines, T, P_atm, stream=None):
    import torch
    outs = [torch.empty(lines.n_lines, dtype=torch.float64, device="cuda") for _ in range(3)]
    _check(load().hk_debug_line_params(ctypes.c_void_p(lines.handle), float(T), float(P_atm),
                                       *[_ptr(o) for o in outs], _stream(stream)))
    return outs


def hk_get_timings():
    t = Timings()
    _check(load().hk_get_timings(ctypes.byref(t)))
    return t
