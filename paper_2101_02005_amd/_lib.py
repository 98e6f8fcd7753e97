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
                ("wing_evals", ctypes.c_int64)]


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
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


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


def hk_opacity(lines, T, P_atm, grd, cutoff, k=None, ws=None, ovr=None, stream=None):
    """k (float32 tensor of grd.n) at one (T, P). ovr: optional (S_ref, gamma_ref, n) float64 tensors."""
    import torch
    if k is None:
        k = torch.empty(grd.n, dtype=torch.float32, device="cuda")
    need = hk_workspace_size(lines, 0, [grd], cutoff)
    if ws is None or ws.numel() < need + 256:
        ws = _workspace(need, k.device)
    _check(load().hk_opacity(ctypes.c_void_p(lines.handle), _override(ovr), float(T), float(P_atm), grd,
                             float(cutoff), _ptr(k), ctypes.c_void_p(_aligned(ws)), need, _stream(stream)))
    return k


def hk_opacity_batched(lines, T, P_atm, grids, cutoff, out_offset=None, k=None, ws=None, stream=None):
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
    if k is None:
        k = torch.empty(total, dtype=torch.float32, device="cuda")
    need = hk_workspace_size(lines, 1, grids, cutoff, n_temps=len(set(float(t) for t in T)))
    if ws is None or ws.numel() < need + 256:
        ws = _workspace(need, k.device)
    Ta = (ctypes.c_double * n_pairs)(*[float(t) for t in T])
    Pa = (ctypes.c_double * n_pairs)(*[float(p) for p in P_atm])
    Ga = (Grid * n_pairs)(*grids)
    Oa = (ctypes.c_int64 * n_pairs)(*[int(o) for o in out_offset])
    _check(load().hk_opacity_batched(ctypes.c_void_p(lines.handle), n_pairs, Ta, Pa, Ga, Oa, float(cutoff), _ptr(k),
                                     ctypes.c_void_p(_aligned(ws)), need, _stream(stream)))
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
    if ws is None or ws.numel() < need + 256:
        ws = _workspace(need, dev)
    _check(load().hk_opacity_backward(ctypes.c_void_p(lines.handle), _override(ovr), float(T), float(P_atm), grd,
                                      float(cutoff), _ptr(dL_dk), _ptr(out2), _ptr(dS), _ptr(dg), _ptr(dn),
                                      ctypes.c_void_p(_aligned(ws)), need, _stream(stream)))
    return out2, dS, dg, dn


def hk_debug_cut_bounds(lines, grd, cutoff, stream=None):
    import torch
    lo = torch.empty(lines.n_lines, dtype=torch.int32, device="cuda")
    hi = torch.empty(lines.n_lines, dtype=torch.int32, device="cuda")
    _check(load().hk_debug_cut_bounds(ctypes.c_void_p(lines.handle), grd, float(cutoff), _ptr(lo), _ptr(hi),
                                      _stream(stream)))
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
