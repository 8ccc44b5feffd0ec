"""ctypes binding of include/fcc_dct.h.  Same names as the C ABI; the only work
done here is argument marshalling (torch tensors or raw device pointers to
integers, status codes to exceptions)."""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfccdct.so")

FCC_OK = 0
FCC_PREC_FP64, FCC_PREC_FP32, FCC_PREC_SPLIT_BF16, FCC_PREC_SPLIT_FP16 = 0, 1, 2, 3
FCC_REAL_INPUT, FCC_STAGES_FP32, FCC_STAGES_FP64, FCC_LEVEL0_FP32 = 1, 2, 4, 8
FCC_TRANSPOSED, FCC_HERMITIAN_PACKED, FCC_FOLD_FFT, FCC_FOLD_BASE = 16, 32, 64, 128
(FCC_MAP_XCD, FCC_MAP_F_INNER, FCC_MAP_NODES8, FCC_MAP_NODES64, FCC_MAP_SPLIT, FCC_MAP_BALANCE, FCC_MAP_XCD16,
 FCC_MAP_CLUSTER, FCC_MAP_ORBIT) = 1, 2, 4, 8, 16, 32, 64, 128, 256
_MAX_LEVELS = 10

# torch is loaded first so that libfccdct.so binds to the HIP runtime torch
# already carries (same soname): one HIP/HSA runtime per process.
import torch  # noqa: E402,F401

if not os.path.exists(_LIB_PATH):
    raise ImportError("libfccdct.so is not built: run `python -m paper_1807_10058_amd.build` "
                      "(or __graft_entry__.build())")
_lib = ctypes.CDLL(_LIB_PATH)


class _LevelTables(ctypes.Structure):
    _fields_ = [("nl", ctypes.c_int), ("m", ctypes.c_int), ("nmono", ctypes.c_int), ("npoly", ctypes.c_int),
                ("mono", ctypes.POINTER(ctypes.c_int)), ("poly", ctypes.POINTER(ctypes.c_double)),
                ("b_rowptr", ctypes.POINTER(ctypes.c_int)), ("b_src", ctypes.POINTER(ctypes.c_uint)),
                ("b_pid", ctypes.POINTER(ctypes.c_ushort)),
                ("c_rowptr", ctypes.POINTER(ctypes.c_int)), ("c_src", ctypes.POINTER(ctypes.c_uint)),
                ("c_pid", ctypes.POINTER(ctypes.c_ushort)),
                ("cube_block", ctypes.POINTER(ctypes.c_int)), ("kappa_block", ctypes.POINTER(ctypes.c_int))]


class _OrbitTemplate(ctypes.Structure):
    _fields_ = [("nc", ctypes.c_int), ("w", ctypes.POINTER(ctypes.c_int)),
                ("b_rowptr", ctypes.POINTER(ctypes.c_int)), ("b_ent", ctypes.POINTER(ctypes.c_ushort)),
                ("c_rowptr", ctypes.POINTER(ctypes.c_int)), ("c_ent", ctypes.POINTER(ctypes.c_ushort)),
                ("nrep", ctypes.c_int), ("rep", ctypes.POINTER(ctypes.c_uint))]


class _OrbitBlocks(ctypes.Structure):
    _fields_ = [("nl", ctypes.c_int), ("m", ctypes.c_int), ("npoly", ctypes.c_int), ("nconst", ctypes.c_int),
                ("ntempl", ctypes.c_int), ("poly", ctypes.POINTER(ctypes.c_double)),
                ("group", ctypes.POINTER(ctypes.c_int)), ("templ", _OrbitTemplate * 16)]


class _Tuning(ctypes.Structure):
    _fields_ = [("tail_levels", ctypes.c_int * 2), ("tile", ((ctypes.c_int * 3) * 2) * 2),
                ("map", (ctypes.c_uint * _MAX_LEVELS) * 2)]


def _tuning_to_c(t):
    c = _Tuning()
    for d in range(2):
        c.tail_levels[d] = int(t["tail_levels"][d])
        for L in range(2):
            for a in range(3):
                c.tile[d][L][a] = int(t["tile"][d][L][a])
        maps = list(t["map"][d])
        for L in range(_MAX_LEVELS):
            c.map[d][L] = int(maps[L]) if L < len(maps) else 0
    return c


def _tuning_from_c(c):
    return {"tail_levels": [c.tail_levels[0], c.tail_levels[1]],
            "tile": [[[c.tile[d][L][a] for a in range(3)] for L in range(2)] for d in range(2)],
            "map": [[c.map[d][L] for L in range(_MAX_LEVELS)] for d in range(2)]}


class _LaunchInfo(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("points", ctypes.c_longlong),
                ("in_bytes", ctypes.c_int), ("out_bytes", ctypes.c_int)]


_vp = ctypes.c_void_p
_lib.fcc_dct_plan.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                              ctypes.c_uint, _vp]
_lib.fcc_dct_plan_tuned.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                    ctypes.c_uint, ctypes.POINTER(_Tuning), _vp]
_lib.fcc_dct_get_tuning.argtypes = [_vp, ctypes.POINTER(_Tuning)]
_lib.fcc_dct_autotune.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_uint,
                                  ctypes.c_int, ctypes.POINTER(_Tuning), _vp]
_lib.fcc_dct_forward.argtypes = [_vp, _vp, _vp, _vp]
_lib.fcc_dct_inverse.argtypes = [_vp, _vp, _vp, _vp]
_lib.fcc_dct_forward_static.argtypes = [_vp, _vp, _vp, _vp]
_lib.fcc_dct_batched.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 ctypes.c_int, _vp]
_lib.fcc_dct_destroy.argtypes = [_vp]
_lib.fcc_dct_batched_release.argtypes = []
_lib.fcc_dct_packed_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_longlong)]
_lib.fcc_fold_unfold_tables.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), _vp, _vp,
                                        ctypes.POINTER(ctypes.c_int)]
_lib.fcc_spectrum_quantise.argtypes = [_vp, ctypes.c_longlong, ctypes.c_float, ctypes.c_float, _vp, _vp, _vp, _vp]
_lib.fcc_dct_describe_launches.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(_LaunchInfo), ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int)]
_lib.fcc_dct_batched_time_launches.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp),
                                               ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_LaunchInfo),
                                               ctypes.c_int, ctypes.POINTER(ctypes.c_int), _vp]
_lib.fcc_dct_roundtrip_residual.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_double), _vp]
_lib.fcc_dct_time_launches.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float),
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_int), _vp]
_lib.fcc_status_string.argtypes = [ctypes.c_int]
_lib.fcc_status_string.restype = ctypes.c_char_p
_lib.fcc_asp_tables.argtypes = [ctypes.c_int, ctypes.POINTER(_LevelTables)]
_lib.fcc_asp_orbit_blocks.argtypes = [ctypes.c_int, ctypes.POINTER(_OrbitBlocks)]
for _f in ("fcc_dct_plan", "fcc_dct_plan_tuned", "fcc_dct_get_tuning", "fcc_dct_autotune", "fcc_dct_forward", "fcc_dct_forward_static", "fcc_dct_inverse", "fcc_dct_batched", "fcc_dct_destroy", "fcc_dct_batched_release",
           "fcc_dct_describe_launches", "fcc_dct_batched_time_launches", "fcc_spectrum_quantise", "fcc_dct_packed_size", "fcc_fold_unfold_tables",
           "fcc_asp_tables", "fcc_asp_orbit_blocks", "fcc_dct_time_launches", "fcc_dct_roundtrip_residual"):
    getattr(_lib, _f).restype = ctypes.c_int


def lib_path():
    return _LIB_PATH


class FccError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s" % (where, fcc_status_string(status)))


def fcc_status_string(status):
    return _lib.fcc_status_string(int(status)).decode()


def _check(status, where):
    if status != FCC_OK:
        raise FccError(status, where)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()  # torch tensor


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Plan:
    """Owns an fcc_plan_t; destroyed with fcc_dct_destroy."""

    def __init__(self, handle, n, prec, flags):
        self.handle, self.n, self.prec, self.flags = handle, n, prec, flags

    def __del__(self):
        try:
            if self.handle:
                _lib.fcc_dct_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def fcc_dct_plan(n, rst=None, prec=FCC_PREC_FP32, flags=FCC_REAL_INPUT, stream=None):
    h = _vp()
    r = None if rst is None else (ctypes.c_double * 3)(*[float(v) for v in rst])
    st = _stream(stream) if stream is not None or _torch_cuda() else None
    _check(_lib.fcc_dct_plan(ctypes.byref(h), int(n), r, int(prec), int(flags), st), "fcc_dct_plan")
    return Plan(h.value, int(n), int(prec), int(flags))


def fcc_dct_plan_tuned(n, rst=None, prec=FCC_PREC_FP32, flags=FCC_REAL_INPUT, tuning=None, stream=None):
    """fcc_dct_plan with an explicit schedule: a dict with keys tail_levels [fwd, inv],
    tile [dir][level][3] (log2 sizes) and map [dir][level] (FCC_MAP_* bits), or None."""
    h = _vp()
    r = None if rst is None else (ctypes.c_double * 3)(*[float(v) for v in rst])
    t = None if tuning is None else ctypes.byref(_tuning_to_c(tuning))
    st = _stream(stream) if stream is not None or _torch_cuda() else None
    _check(_lib.fcc_dct_plan_tuned(ctypes.byref(h), int(n), r, int(prec), int(flags), t, st), "fcc_dct_plan_tuned")
    return Plan(h.value, int(n), int(prec), int(flags))


def fcc_dct_get_tuning(plan):
    c = _Tuning()
    _check(_lib.fcc_dct_get_tuning(plan.handle, ctypes.byref(c)), "fcc_dct_get_tuning")
    return _tuning_from_c(c)


def fcc_dct_autotune(n, rst=None, prec=FCC_PREC_FP32, flags=FCC_REAL_INPUT, reps=5, stream=None):
    """Search the schedule for (n, prec, flags); later plans of that kind use it."""
    r = None if rst is None else (ctypes.c_double * 3)(*[float(v) for v in rst])
    c = _Tuning()
    _check(_lib.fcc_dct_autotune(int(n), r, int(prec), int(flags), int(reps), ctypes.byref(c), _stream(stream)),
           "fcc_dct_autotune")
    return _tuning_from_c(c)


def _torch_cuda():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def fcc_dct_forward(plan, x, X, stream=None):
    _check(_lib.fcc_dct_forward(plan.handle, _ptr(x), _ptr(X), _stream(stream)), "fcc_dct_forward")


def fcc_dct_forward_static(plan, x, X, stream=None):
    """fcc_dct_forward with scratch in the library's static device array (no allocation; n <= 64)."""
    _check(_lib.fcc_dct_forward_static(plan.handle, _ptr(x), _ptr(X), _stream(stream)), "fcc_dct_forward_static")


def fcc_dct_inverse(plan, X, x, stream=None):
    _check(_lib.fcc_dct_inverse(plan.handle, _ptr(X), _ptr(x), _stream(stream)), "fcc_dct_inverse")


class BatchedCall:
    """The arguments of one fcc_dct_batched call marshalled once, for repeated
    calls (the library replays its recorded graph on every call)."""

    def __init__(self, plans, ins, outs, direction):
        self.cnt = len(plans)
        self.plans = list(plans)  # keep the plans alive
        self.P = (_vp * self.cnt)(*[p.handle for p in plans])
        self.I = (_vp * self.cnt)(*[_ptr(t) for t in ins])
        self.O = (_vp * self.cnt)(*[_ptr(t) for t in outs])
        self.direction = int(direction)

    def __call__(self, stream=None):
        _check(_lib.fcc_dct_batched(self.P, self.cnt, self.I, self.O, self.direction, _stream(stream)),
               "fcc_dct_batched")


def fcc_dct_batched(plans, ins, outs, direction, stream=None):
    BatchedCall(plans, ins, outs, direction)(stream)


def fcc_spectrum_quantise(X, threshold, step, codes=None, Xq=None, kept=None, stream=None):
    """Threshold and quantise a complex64 spectrum on the GPU (block-wise coding).
    X: complex64 tensor; codes: int16 tensor of 2*len(X) (or None); Xq: complex64
    tensor (or None); kept: int64 device tensor of one element (or None).
    Returns the kept tensor (the count is read after synchronisation)."""
    import torch
    if kept is None:
        kept = torch.zeros(1, dtype=torch.int64, device=X.device)
    _check(_lib.fcc_spectrum_quantise(_ptr(X), int(X.numel()), float(threshold), float(step), _ptr(codes), _ptr(Xq),
                                      _ptr(kept), _stream(stream)), "fcc_spectrum_quantise")
    return kept


def fcc_dct_packed_size(plan):
    """Complex values of the plan's forward output (n^3, or the Hermitian-packed count)."""
    c = ctypes.c_longlong(0)
    _check(_lib.fcc_dct_packed_size(plan.handle, ctypes.byref(c)), "fcc_dct_packed_size")
    return int(c.value)


def fcc_fold_unfold_tables(n, rst=None):
    """Host-only unfold tables of the fold+FFT inverse: (pid uint8[n^3], K complex[npat, 24])."""
    import numpy as np
    r = (ctypes.c_double * 3)(*([0.125, 0.0, 0.375] if rst is None else [float(v) for v in rst]))
    pid = np.zeros(n ** 3, dtype=np.uint8)
    K = np.zeros((256, 24), dtype=np.complex128)
    npat = ctypes.c_int(0)
    _check(_lib.fcc_fold_unfold_tables(int(n), r, pid.ctypes.data, K.ctypes.data, ctypes.byref(npat)),
           "fcc_fold_unfold_tables")
    return pid, K[:npat.value].copy()


def fcc_dct_batched_release():
    """Free every graph fcc_dct_batched has recorded."""
    _check(_lib.fcc_dct_batched_release(), "fcc_dct_batched_release")


def _infos(arr, k):
    return [{"name": arr[i].name.decode(), "points": int(arr[i].points), "in_bytes": int(arr[i].in_bytes),
             "out_bytes": int(arr[i].out_bytes)} for i in range(k)]


def fcc_dct_describe_launches(plan, direction):
    """Launch slots of one transform: name, points, algorithmic bytes per point read and written."""
    cnt = ctypes.c_int(0)
    _check(_lib.fcc_dct_describe_launches(plan.handle, int(direction), None, 0, ctypes.byref(cnt)),
           "fcc_dct_describe_launches")
    arr = (_LaunchInfo * max(1, cnt.value))()
    _check(_lib.fcc_dct_describe_launches(plan.handle, int(direction), arr, cnt.value, ctypes.byref(cnt)),
           "fcc_dct_describe_launches")
    return _infos(arr, cnt.value)


def fcc_dct_batched_time_launches(plans, ins, outs, direction, reps=5, stream=None):
    """Average duration (ms) and description of every launch slot of the batched work."""
    c = BatchedCall(plans, ins, outs, direction)
    cnt = ctypes.c_int(0)
    _check(_lib.fcc_dct_batched_time_launches(c.P, c.cnt, c.I, c.O, c.direction, 1, None, None, 0,
                                              ctypes.byref(cnt), _stream(stream)), "fcc_dct_batched_time_launches")
    ms = (ctypes.c_float * cnt.value)()
    arr = (_LaunchInfo * cnt.value)()
    _check(_lib.fcc_dct_batched_time_launches(c.P, c.cnt, c.I, c.O, c.direction, int(reps), ms, arr, cnt.value,
                                              ctypes.byref(cnt), _stream(stream)), "fcc_dct_batched_time_launches")
    out = _infos(arr, cnt.value)
    for i, v in enumerate(out):
        v["ms"] = float(ms[i])
    return out


def fcc_dct_time_launches(plan, x, out, direction, reps=10, stream=None):
    """Average duration (ms) of each kernel launch of one transform, in launch order."""
    cnt = ctypes.c_int(0)
    _check(_lib.fcc_dct_time_launches(plan.handle, _ptr(x), _ptr(out), int(direction), 1, None, 0,
                                      ctypes.byref(cnt), _stream(stream)), "fcc_dct_time_launches")
    ms = (ctypes.c_float * cnt.value)()
    _check(_lib.fcc_dct_time_launches(plan.handle, _ptr(x), _ptr(out), int(direction), int(reps), ms, cnt.value,
                                      ctypes.byref(cnt), _stream(stream)), "fcc_dct_time_launches")
    return [float(v) for v in ms]


def fcc_dct_roundtrip_residual(plan, x, y, stream=None):
    """max|x - y| / max|x| computed in FP64 on the GPU (x, y shaped like the forward input)."""
    r = ctypes.c_double(0.0)
    _check(_lib.fcc_dct_roundtrip_residual(plan.handle, _ptr(x), _ptr(y), ctypes.byref(r), _stream(stream)),
           "fcc_dct_roundtrip_residual")
    return r.value


def fcc_dct_destroy(plan):
    if plan.handle:
        _check(_lib.fcc_dct_destroy(plan.handle), "fcc_dct_destroy")
        plan.handle = None


def fcc_asp_tables(nl):
    """Host copies of the basis-change gather tables for node size nl."""
    t = _LevelTables()
    _check(_lib.fcc_asp_tables(int(nl), ctypes.byref(t)), "fcc_asp_tables")
    rows = 8 * t.m ** 3

    def arr(p, k, dt):
        return np.ctypeslib.as_array(p, shape=(k,)).astype(dt).copy()

    out = {"nl": t.nl, "m": t.m, "nmono": t.nmono, "npoly": t.npoly,
           "mono": arr(t.mono, 3 * t.nmono, np.int64).reshape(-1, 3),
           "poly": arr(t.poly, t.npoly * t.nmono, np.float64).reshape(t.npoly, t.nmono)}
    for side in ("b", "c"):
        rp = arr(getattr(t, side + "_rowptr"), rows + 1, np.int64)
        out[side + "_rowptr"] = rp
        out[side + "_src"] = arr(getattr(t, side + "_src"), int(rp[-1]), np.int64)
        out[side + "_pid"] = arr(getattr(t, side + "_pid"), int(rp[-1]), np.int64)
    out["cube_block"] = arr(t.cube_block, t.m ** 3, np.int64)
    out["kappa_block"] = arr(t.kappa_block, t.nl ** 3, np.int64)
    return out


def fcc_asp_orbit_blocks(nl):
    """Host copies of the orbit-block templates and representatives for node size nl."""
    b = _OrbitBlocks()
    _check(_lib.fcc_asp_orbit_blocks(int(nl), ctypes.byref(b)), "fcc_asp_orbit_blocks")

    def arr(p, k, dt):
        return np.ctypeslib.as_array(p, shape=(k,)).astype(dt).copy() if k else np.zeros(0, dt)

    out = {"nl": b.nl, "m": b.m, "npoly": b.npoly, "nconst": b.nconst,
           "poly": arr(b.poly, 5 * b.npoly, np.float64).reshape(b.npoly, 5),
           "group": arr(b.group, 24 * 9, np.int64).reshape(24, 3, 3), "templ": []}
    for t in range(b.ntempl):
        T = b.templ[t]
        nc = T.nc
        brp = arr(T.b_rowptr, 8 * nc + 1, np.int64)
        crp = arr(T.c_rowptr, 8 * nc + 1, np.int64)
        out["templ"].append({"nc": nc, "w": arr(T.w, nc, np.int64),
                             "b_rowptr": brp, "b_ent": arr(T.b_ent, int(brp[-1]), np.int64),
                             "c_rowptr": crp, "c_ent": arr(T.c_ent, int(crp[-1]), np.int64),
                             "rep": arr(T.rep, T.nrep, np.int64)})
    return out
