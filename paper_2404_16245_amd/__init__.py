"""MI355X (gfx950) nuclear-attraction integrals over contracted solid-harmonic Gaussian orbitals.

Thin ctypes binding of the C ABI in ``include/shgo.h`` (``libshgo.so`` next to this file,
built by ``build.py``). Functions named ``shgo_*`` marshal arguments to the C entry points of
the same name; PyTorch only supplies device memory and the current HIP stream. There is no CPU
fallback: importing the binding on a machine without the built library raises, and every call
that reaches the device needs a GPU.

Method: arXiv:2404.16245 (Gaussian product Eq. 5, shift to the product center Eqs. 7-8,
product rule of solid harmonics supplement Eq. 4, one-center integral Eqs. 11-12).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshgo.so")

SHGO_OK = 0
SHGO_ERR_INVALID_ARG = 1
SHGO_ERR_UNSUPPORTED_L = 2
SHGO_ERR_NOT_FINITE = 3
SHGO_ERR_OUT_OF_MEMORY = 4
SHGO_ERR_DEVICE = 5
SHGO_ERR_INTERNAL = 6
SHGO_LMAX = 7

EXPORTED = ["shgo_create", "shgo_destroy", "shgo_status_string", "shgo_last_error", "shgo_nbf", "shgo_validate",
            "shgo_plan_matrix", "shgo_plan_pairs", "shgo_plan_destroy", "shgo_plan_output_size",
            "shgo_plan_integrals", "shgo_execute", "shgo_execute_graph", "shgo_execute_grad", "shgo_boys",
            "shgo_execute_overlap", "shgo_execute_cartesian", "shgo_eri_blocks", "shgo_eri_output_size",
            "shgo_plan_set_timing", "shgo_plan_phase_ms", "shgo_plan_get_schedule", "shgo_plan_set_schedule",
            "shgo_plan_autotune", "shgo_max_tiles", "shgo_options_default", "shgo_check_call",
            "shgo_nuclear_attraction", "shgo_nuclear_attraction_grad", "shgo_plan_get_info", "shgo_plan_set_precision",
            "shgo_nuclear_attraction_noalloc", "shgo_plan_item_profile"]
SHGO_NUM_CLASSES = 36
SHGO_TUNE_CANDIDATES = 5
SHGO_NUM_PHASES = 2
SHGO_PREC_FP64 = 0
SHGO_PREC_MIXED = 1
SHGO_NOALLOC_SCRATCH_BYTES = 32 << 20


class ShgoError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


class _Basis(ctypes.Structure):
    _fields_ = [("n_shells", ctypes.c_int32), ("center", ctypes.c_void_p), ("l", ctypes.c_void_p),
                ("n_prim", ctypes.c_void_p), ("prim_offset", ctypes.c_void_p), ("exponent", ctypes.c_void_p),
                ("coef", ctypes.c_void_p)]


class _Nuclei(ctypes.Structure):
    _fields_ = [("n_nuclei", ctypes.c_int32), ("position", ctypes.c_void_p), ("charge", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("screen_threshold", ctypes.c_double), ("use_graph", ctypes.c_int32),
                ("autotune_cache", ctypes.c_char_p), ("scratch_limit_bytes", ctypes.c_size_t)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("candidate_pairs", ctypes.c_int64), ("kept_pairs", ctypes.c_int64),
                ("kept_prim_pairs", ctypes.c_int64), ("integrals", ctypes.c_int64), ("output_size", ctypes.c_int64),
                ("nbf", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libshgo.so (torch is imported first so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2404_16245_amd/build.py (no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.shgo_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    lib.shgo_create.restype = ctypes.c_int
    lib.shgo_destroy.argtypes = [vp]
    lib.shgo_destroy.restype = None
    lib.shgo_status_string.argtypes = [ctypes.c_int]
    lib.shgo_status_string.restype = ctypes.c_char_p
    lib.shgo_last_error.argtypes = [vp]
    lib.shgo_last_error.restype = ctypes.c_char_p
    lib.shgo_nbf.argtypes = [ctypes.POINTER(_Basis)]
    lib.shgo_nbf.restype = i64
    lib.shgo_validate.argtypes = [ctypes.POINTER(_Basis), ctypes.POINTER(_Nuclei), dbl, ctypes.c_char_p, ctypes.c_size_t]
    lib.shgo_validate.restype = ctypes.c_int
    lib.shgo_plan_matrix.argtypes = [vp, ctypes.POINTER(_Basis), ctypes.POINTER(_Nuclei), dbl, ctypes.POINTER(vp)]
    lib.shgo_plan_matrix.restype = ctypes.c_int
    lib.shgo_plan_pairs.argtypes = [vp, ctypes.POINTER(_Basis), ctypes.POINTER(_Nuclei), i64, vp, vp, dbl,
                                    ctypes.POINTER(vp)]
    lib.shgo_plan_pairs.restype = ctypes.c_int
    lib.shgo_plan_destroy.argtypes = [vp]
    lib.shgo_plan_destroy.restype = None
    lib.shgo_plan_output_size.argtypes = [vp]
    lib.shgo_plan_output_size.restype = i64
    lib.shgo_plan_integrals.argtypes = [vp]
    lib.shgo_plan_integrals.restype = i64
    lib.shgo_execute.argtypes = [vp, vp, vp]
    lib.shgo_execute.restype = ctypes.c_int
    lib.shgo_execute_graph.argtypes = [vp, vp, vp]
    lib.shgo_execute_graph.restype = ctypes.c_int
    lib.shgo_execute_overlap.argtypes = [vp, vp, vp]
    lib.shgo_execute_overlap.restype = ctypes.c_int
    lib.shgo_execute_cartesian.argtypes = [vp, vp, vp]
    lib.shgo_execute_cartesian.restype = ctypes.c_int
    lib.shgo_eri_blocks.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.shgo_eri_blocks.restype = ctypes.c_int
    lib.shgo_eri_output_size.argtypes = [vp, i64, vp, ctypes.POINTER(i64)]
    lib.shgo_eri_output_size.restype = ctypes.c_int
    lib.shgo_plan_get_schedule.argtypes = [vp, vp, vp]
    lib.shgo_plan_get_schedule.restype = ctypes.c_int
    lib.shgo_plan_set_schedule.argtypes = [vp, vp, vp]
    lib.shgo_plan_set_schedule.restype = ctypes.c_int
    lib.shgo_max_tiles.argtypes = [i32]
    lib.shgo_max_tiles.restype = i32
    lib.shgo_plan_autotune.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.shgo_plan_autotune.restype = ctypes.c_int
    lib.shgo_execute_grad.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.shgo_execute_grad.restype = ctypes.c_int
    lib.shgo_boys.argtypes = [vp, i64, vp, i32, vp, vp]
    lib.shgo_boys.restype = ctypes.c_int
    lib.shgo_plan_set_timing.argtypes = [vp, i32]
    lib.shgo_plan_set_timing.restype = ctypes.c_int
    lib.shgo_plan_phase_ms.argtypes = [vp, vp, vp]
    lib.shgo_plan_phase_ms.restype = ctypes.c_int
    lib.shgo_options_default.argtypes = [ctypes.POINTER(_Options)]
    lib.shgo_options_default.restype = None
    lib.shgo_check_call.argtypes = [ctypes.POINTER(_Basis), ctypes.POINTER(_Nuclei), ctypes.POINTER(_Options),
                                    ctypes.POINTER(_PlanInfo), ctypes.c_char_p, ctypes.c_size_t]
    lib.shgo_check_call.restype = ctypes.c_int
    lib.shgo_nuclear_attraction.argtypes = [vp, ctypes.POINTER(_Basis), ctypes.POINTER(_Nuclei),
                                            ctypes.POINTER(_Options), vp, vp]
    lib.shgo_nuclear_attraction.restype = ctypes.c_int
    lib.shgo_nuclear_attraction_grad.argtypes = [vp, ctypes.POINTER(_Basis), ctypes.POINTER(_Nuclei),
                                                 ctypes.POINTER(_Options), vp, vp, vp, vp]
    lib.shgo_nuclear_attraction_grad.restype = ctypes.c_int
    lib.shgo_nuclear_attraction_noalloc.argtypes = [vp, ctypes.POINTER(_Basis), ctypes.POINTER(_Nuclei),
                                                    ctypes.POINTER(_Options), vp, vp]
    lib.shgo_nuclear_attraction_noalloc.restype = ctypes.c_int
    lib.shgo_plan_item_profile.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
    lib.shgo_plan_item_profile.restype = ctypes.c_int
    lib.shgo_plan_get_info.argtypes = [vp, ctypes.POINTER(_PlanInfo)]
    lib.shgo_plan_get_info.restype = ctypes.c_int
    lib.shgo_plan_set_precision.argtypes = [vp, i32]
    lib.shgo_plan_set_precision.restype = ctypes.c_int
    _lib = lib
    return lib


# ----------------------------------------------------------------------------------------------
# argument marshalling
# ----------------------------------------------------------------------------------------------
class _HostBasis:
    """Keeps contiguous host copies alive while the C call reads them."""

    def __init__(self, basis):
        self.center = np.ascontiguousarray(basis.center, dtype=np.float64).reshape(-1, 3)
        self.l = np.ascontiguousarray(basis.l, dtype=np.int32)
        self.nprim = np.ascontiguousarray(basis.nprim, dtype=np.int32)
        self.prim_off = np.ascontiguousarray(basis.prim_off, dtype=np.int64)
        self.expo = np.ascontiguousarray(basis.expo, dtype=np.float64)
        self.coef = np.ascontiguousarray(basis.coef, dtype=np.float64)
        self.struct = _Basis(int(self.l.shape[0]), self.center.ctypes.data, self.l.ctypes.data,
                             self.nprim.ctypes.data, self.prim_off.ctypes.data, self.expo.ctypes.data,
                             self.coef.ctypes.data)


class _HostNuclei:
    def __init__(self, nuclei):
        self.pos = np.ascontiguousarray(nuclei.pos, dtype=np.float64).reshape(-1, 3)
        self.Z = np.ascontiguousarray(nuclei.Z, dtype=np.float64)
        self.struct = _Nuclei(int(self.Z.shape[0]), self.pos.ctypes.data, self.Z.ctypes.data)


_PRECISIONS = {"fp64": SHGO_PREC_FP64, "mixed": SHGO_PREC_MIXED}


def shgo_options_default():
    o = _Options()
    load_library().shgo_options_default(ctypes.byref(o))
    return o


def options(precision="fp64", screen=0.0, use_graph=False, autotune_cache=None, scratch_limit_bytes=0):
    """A shgo_options struct for the single-call entry points."""
    o = shgo_options_default()
    o.precision = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.screen_threshold = float(screen)
    o.use_graph = 1 if use_graph else 0
    o.autotune_cache = None if autotune_cache is None else os.fsencode(autotune_cache)
    o.scratch_limit_bytes = int(scratch_limit_bytes)
    return o


def shgo_check_call(basis, nuclei, opts=None):
    """(status, message, plan sizes as a dict) of the host-side checks of a single call."""
    hb, hn = _HostBasis(basis), _HostNuclei(nuclei)
    buf = ctypes.create_string_buffer(256)
    info = _PlanInfo()
    st = load_library().shgo_check_call(ctypes.byref(hb.struct), ctypes.byref(hn.struct),
                                        None if opts is None else ctypes.byref(opts), ctypes.byref(info), buf, 256)
    return int(st), buf.value.decode(), {k: int(getattr(info, k)) for k, _ in _PlanInfo._fields_}


def _stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check(lib, ctx, status):
    if status != SHGO_OK:
        msg = lib.shgo_last_error(ctx).decode() if ctx else lib.shgo_status_string(status).decode()
        raise ShgoError(status, msg or lib.shgo_status_string(status).decode())


# ----------------------------------------------------------------------------------------------
# entry points with the C names
# ----------------------------------------------------------------------------------------------
def shgo_create(device=0):
    lib = load_library()
    h = ctypes.c_void_p()
    st = lib.shgo_create(int(device), ctypes.byref(h))
    if st != SHGO_OK:
        raise ShgoError(st, "shgo_create: " + lib.shgo_status_string(st).decode())
    return h


def shgo_destroy(ctx):
    load_library().shgo_destroy(ctx)


def shgo_status_string(status):
    return load_library().shgo_status_string(int(status)).decode()


def shgo_last_error(ctx):
    return load_library().shgo_last_error(ctx).decode()


def shgo_nbf(basis):
    hb = _HostBasis(basis)
    return int(load_library().shgo_nbf(ctypes.byref(hb.struct)))


def shgo_validate(basis, nuclei, screen=0.0):
    """(status, message) of the host-side validation."""
    hb, hn = _HostBasis(basis), _HostNuclei(nuclei)
    buf = ctypes.create_string_buffer(256)
    st = load_library().shgo_validate(ctypes.byref(hb.struct), ctypes.byref(hn.struct), float(screen), buf, 256)
    return int(st), buf.value.decode()


class Plan:
    """A device-resident plan (owns the C plan handle)."""

    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle
        lib = load_library()
        self.output_size = int(lib.shgo_plan_output_size(handle))
        self.integrals = int(lib.shgo_plan_integrals(handle))

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.shgo_plan_destroy(self.handle)
            self.handle = None


def shgo_plan_matrix(ctx, basis, nuclei, screen=0.0):
    lib = load_library()
    hb, hn = _HostBasis(basis), _HostNuclei(nuclei)
    h = ctypes.c_void_p()
    _check(lib, ctx, lib.shgo_plan_matrix(ctx, ctypes.byref(hb.struct), ctypes.byref(hn.struct), float(screen),
                                          ctypes.byref(h)))
    return Plan(ctx, h)


def shgo_plan_pairs(ctx, basis, nuclei, pair_a, pair_b, screen=0.0):
    lib = load_library()
    hb, hn = _HostBasis(basis), _HostNuclei(nuclei)
    pa = np.ascontiguousarray(pair_a, dtype=np.int32)
    pb = np.ascontiguousarray(pair_b, dtype=np.int32)
    if pa.shape != pb.shape:
        raise ValueError("pair_a and pair_b differ in length")
    h = ctypes.c_void_p()
    _check(lib, ctx, lib.shgo_plan_pairs(ctx, ctypes.byref(hb.struct), ctypes.byref(hn.struct), int(pa.shape[0]),
                                         pa.ctypes.data, pb.ctypes.data, float(screen), ctypes.byref(h)))
    return Plan(ctx, h)


def shgo_nuclear_attraction(ctx, basis, nuclei, opts, V, stream=None):
    """The single call: V (float64 device tensor, nbf x nbf) from the host basis and nuclei."""
    lib = load_library()
    hb, hn = _HostBasis(basis), _HostNuclei(nuclei)
    nbf = int(lib.shgo_nbf(ctypes.byref(hb.struct)))  # -1 for an l out of range: the call refuses it
    _check(lib, ctx, lib.shgo_nuclear_attraction(ctx, ctypes.byref(hb.struct), ctypes.byref(hn.struct),
                                                 None if opts is None else ctypes.byref(opts),
                                                 _f64_device(V, "V", max(nbf, 0) ** 2), _stream_handle(stream)))
    return V


def shgo_nuclear_attraction_noalloc(ctx, basis, nuclei, opts, V, stream=None):
    """The allocation-free single call: V (float64 device tensor, nbf x nbf), workspace in the
    library's static scratch array."""
    lib = load_library()
    hb, hn = _HostBasis(basis), _HostNuclei(nuclei)
    nbf = int(lib.shgo_nbf(ctypes.byref(hb.struct)))
    _check(lib, ctx, lib.shgo_nuclear_attraction_noalloc(ctx, ctypes.byref(hb.struct), ctypes.byref(hn.struct),
                                                         None if opts is None else ctypes.byref(opts),
                                                         _f64_device(V, "V", max(nbf, 0) ** 2), _stream_handle(stream)))
    return V


def shgo_nuclear_attraction_grad(ctx, basis, nuclei, opts, D, dE_dnuclei, dE_dcenters, stream=None):
    """The single call of the gradient of E = sum D V (float64 device tensors)."""
    lib = load_library()
    hb, hn = _HostBasis(basis), _HostNuclei(nuclei)
    nbf = max(int(lib.shgo_nbf(ctypes.byref(hb.struct))), 0)
    _check(lib, ctx, lib.shgo_nuclear_attraction_grad(ctx, ctypes.byref(hb.struct), ctypes.byref(hn.struct),
                                                      None if opts is None else ctypes.byref(opts),
                                                      _f64_device(D, "D", nbf * nbf),
                                                      _f64_device(dE_dnuclei, "dE_dnuclei", 3 * int(hn.Z.shape[0])),
                                                      _f64_device(dE_dcenters, "dE_dcenters", 3 * int(hb.l.shape[0])),
                                                      _stream_handle(stream)))


def shgo_plan_get_info(plan):
    info = _PlanInfo()
    lib = load_library()
    _check(lib, plan.ctx, lib.shgo_plan_get_info(plan.handle, ctypes.byref(info)))
    return {k: int(getattr(info, k)) for k, _ in _PlanInfo._fields_}


def shgo_plan_set_precision(plan, precision):
    lib = load_library()
    p = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib, plan.ctx, lib.shgo_plan_set_precision(plan.handle, p))


def shgo_plan_destroy(plan):
    if plan.handle is not None:
        load_library().shgo_plan_destroy(plan.handle)
        plan.handle = None


def shgo_plan_output_size(plan):
    return plan.output_size


def shgo_plan_integrals(plan):
    return plan.integrals


def shgo_execute(plan, out, stream=None):
    """Enqueue the whole evaluation; ``out`` is a float64 CUDA tensor of plan.output_size."""
    lib = load_library()
    if out.dtype.__str__() != "torch.float64" or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 device tensor")
    if out.numel() < plan.output_size:
        raise ValueError("out is smaller than the plan's output")
    _check(lib, plan.ctx, lib.shgo_execute(plan.handle, ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def shgo_execute_graph(plan, out, stream=None):
    """As shgo_execute, through a captured HIP graph (captured on the first call for ``out``)."""
    lib = load_library()
    _check(lib, plan.ctx, lib.shgo_execute_graph(plan.handle, _f64_device(out, "out", plan.output_size),
                                                 _stream_handle(stream)))
    return out


def shgo_execute_cartesian(plan, out, stream=None):
    """Enqueue the plan's V by the Cartesian (McMurchie-Davidson) route into ``out``; l <= 4."""
    lib = load_library()
    _check(lib, plan.ctx, lib.shgo_execute_cartesian(plan.handle, _f64_device(out, "out", plan.output_size),
                                                     _stream_handle(stream)))
    return out


def shgo_execute_overlap(plan, out, stream=None):
    """Enqueue the overlap matrix S of the plan's shells into ``out`` (the layout V has)."""
    lib = load_library()
    _check(lib, plan.ctx, lib.shgo_execute_overlap(plan.handle, _f64_device(out, "out", plan.output_size),
                                                   _stream_handle(stream)))
    return out


def shgo_eri_output_size(basis, quartets):
    """Doubles shgo_eri_blocks writes for the quartets [n, 4] (host only; the library checks the
    indices and the shells' l)."""
    lib = load_library()
    hb = basis if isinstance(basis, _HostBasis) else _HostBasis(basis)
    q = np.ascontiguousarray(quartets, dtype=np.int32).reshape(-1, 4)
    n = ctypes.c_int64()
    _check(lib, None, lib.shgo_eri_output_size(ctypes.byref(hb.struct), int(len(q)), q.ctypes.data, ctypes.byref(n)))
    return n.value


def shgo_max_tiles(class_id):
    """Largest tiles-per-item the LDS accumulator allows for a class (-1 if invalid)."""
    return int(load_library().shgo_max_tiles(int(class_id)))


def shgo_plan_get_schedule(plan):
    """(weight[SHGO_NUM_CLASSES] float32, tiles[SHGO_NUM_CLASSES] int32) of the plan's persistent launch."""
    lib = load_library()
    weight = np.zeros(SHGO_NUM_CLASSES, dtype=np.float32)
    tiles = np.zeros(SHGO_NUM_CLASSES, dtype=np.int32)
    _check(lib, plan.ctx, lib.shgo_plan_get_schedule(plan.handle, weight.ctypes.data, tiles.ctypes.data))
    return weight, tiles


def shgo_plan_set_schedule(plan, weight, tiles):
    lib = load_library()
    weight = np.ascontiguousarray(weight, dtype=np.float32)
    tiles = np.ascontiguousarray(tiles, dtype=np.int32)
    if weight.shape != (SHGO_NUM_CLASSES,) or tiles.shape != (SHGO_NUM_CLASSES,):
        raise ValueError(f"weight and tiles need one entry per class ({SHGO_NUM_CLASSES})")
    _check(lib, plan.ctx, lib.shgo_plan_set_schedule(plan.handle, weight.ctypes.data, tiles.ctypes.data))


def shgo_plan_autotune(plan, out, rounds=5, stream=None):
    """Tune the plan's schedule; returns (ms per candidate [5], index of the candidate refined and
    kept). Synchronizes."""
    lib = load_library()
    ms = np.zeros(SHGO_TUNE_CANDIDATES)
    chosen = np.zeros(1, dtype=np.int32)
    _check(lib, plan.ctx, lib.shgo_plan_autotune(plan.handle, _f64_device(out, "out", plan.output_size),
                                                 int(rounds), _stream_handle(stream), ms.ctypes.data,
                                                 chosen.ctypes.data))
    return ms, int(chosen[0])


def _f64_device(t, name, n):
    if str(t.dtype) != "torch.float64" or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 device tensor")
    if t.numel() < n:
        raise ValueError(f"{name} is too small ({t.numel()} < {n})")
    return ctypes.c_void_p(t.data_ptr())


def shgo_execute_grad(plan, D, dE_dnuclei, dE_dcenters, energy=None, stream=None):
    """Enqueue the adjoint kernel: gradient of E = sum_ij D_ij V_ij for a matrix plan.
    D [nbf, nbf], dE_dnuclei [n_nuclei, 3], dE_dcenters [n_shells, 3], energy [1] or None:
    contiguous float64 device tensors."""
    lib = load_library()
    e = ctypes.c_void_p(0) if energy is None else _f64_device(energy, "energy", 1)
    _check(lib, plan.ctx, lib.shgo_execute_grad(plan.handle, _f64_device(D, "D", 0),
                                                _f64_device(dE_dnuclei, "dE_dnuclei", 0),
                                                _f64_device(dE_dcenters, "dE_dcenters", 0), e,
                                                _stream_handle(stream)))


def shgo_plan_item_profile(plan, out, stream=None):
    """One profiled execution: (items [n] int32 (class << 24 | block), start [n] us, duration [n] us)
    in dispatch order. Synchronizes."""
    lib = load_library()
    n = np.zeros(1, dtype=np.int32)
    _check(lib, plan.ctx, lib.shgo_plan_item_profile(plan.handle, _f64_device(out, "out", plan.output_size), 0, None,
                                                     None, None, n.ctypes.data, _stream_handle(stream)))
    m = int(n[0])
    items = np.zeros(max(m, 1), dtype=np.int32)
    start = np.zeros(max(m, 1))
    dur = np.zeros(max(m, 1))
    _check(lib, plan.ctx, lib.shgo_plan_item_profile(plan.handle, _f64_device(out, "out", plan.output_size), m,
                                                     items.ctypes.data, start.ctypes.data, dur.ctypes.data,
                                                     n.ctypes.data, _stream_handle(stream)))
    return items[:m], start[:m], dur[:m]


def shgo_plan_set_timing(plan, n_slots):
    lib = load_library()
    _check(lib, plan.ctx, lib.shgo_plan_set_timing(plan.handle, int(n_slots)))


def shgo_plan_phase_ms(plan):
    """(ms[SHGO_NUM_PHASES] summed over the recorded executions, number of executions).
    Phase 0: pair build; phase 1: the integral kernel."""
    lib = load_library()
    ms = np.zeros(SHGO_NUM_PHASES)
    cnt = np.zeros(1, dtype=np.int32)
    _check(lib, plan.ctx, lib.shgo_plan_phase_ms(plan.handle, ms.ctypes.data, cnt.ctypes.data))
    return ms, int(cnt[0])


def shgo_boys(ctx, T, mmax, F=None, stream=None):
    """Device Boys function: T float64 CUDA tensor [n] -> F [n, mmax+1]."""
    import torch
    lib = load_library()
    T = T.contiguous()
    if F is None:
        F = torch.empty((T.numel(), mmax + 1), dtype=torch.float64, device=T.device)
    _check(lib, ctx, lib.shgo_boys(ctx, int(T.numel()), ctypes.c_void_p(T.data_ptr()), int(mmax),
                                   ctypes.c_void_p(F.data_ptr()), _stream_handle(stream)))
    return F


# ----------------------------------------------------------------------------------------------
# convenience (still only marshalling)
# ----------------------------------------------------------------------------------------------
_ctx = {}


def context(device=0):
    if device not in _ctx:
        _ctx[device] = shgo_create(device)
    return _ctx[device]


def nuclear_attraction(basis, nuclei, screen=0.0, device=0, precision="fp64", use_graph=False, autotune_cache=None,
                       scratch_limit_bytes=0):
    """Full nbf x nbf nuclear-attraction matrix as a float64 CUDA tensor (shgo_nuclear_attraction)."""
    import torch
    ctx = context(device)
    nbf = shgo_nbf(basis)
    out = torch.empty((nbf, nbf), dtype=torch.float64, device=f"cuda:{device}")
    opts = options(precision, screen, use_graph, autotune_cache, scratch_limit_bytes)
    shgo_nuclear_attraction(ctx, basis, nuclei, opts, out)
    torch.cuda.current_stream().synchronize()
    return out


def nuclear_attraction_pairs(basis, nuclei, pair_a, pair_b, screen=0.0, device=0):
    """Blocks of the listed shell pairs, back to back, as a flat float64 CUDA tensor."""
    import torch
    ctx = context(device)
    plan = shgo_plan_pairs(ctx, basis, nuclei, pair_a, pair_b, screen)
    out = torch.empty(plan.output_size, dtype=torch.float64, device=f"cuda:{device}")
    shgo_execute(plan, out)
    torch.cuda.current_stream().synchronize()
    return out


def nuclear_attraction_grad(basis, nuclei, D, screen=0.0, device=0):
    """(dE/d nuclear positions [n, 3], dE/d shell centers [n_shells, 3], E) for E = sum D V, as
    float64 CUDA tensors."""
    import torch
    ctx = context(device)
    plan = shgo_plan_matrix(ctx, basis, nuclei, screen)
    dev = f"cuda:{device}"
    Dt = torch.as_tensor(D, dtype=torch.float64, device=dev).contiguous()
    dn = torch.empty((nuclei.n, 3), dtype=torch.float64, device=dev)
    dc = torch.empty((basis.n_shells, 3), dtype=torch.float64, device=dev)
    e = torch.empty(1, dtype=torch.float64, device=dev)
    shgo_execute_grad(plan, Dt, dn, dc, e)
    torch.cuda.current_stream().synchronize()
    return dn, dc, e


def _no_nuclei():
    class _N:
        pos = np.zeros((0, 3))
        Z = np.zeros(0)
        n = 0
    return _N()


def nuclear_attraction_cartesian(basis, nuclei, screen=0.0, device=0):
    """V by the Cartesian route (shgo_execute_cartesian), full nbf x nbf float64 CUDA tensor."""
    import torch
    plan = shgo_plan_matrix(context(device), basis, nuclei, screen)
    nbf = shgo_nbf(basis)
    out = torch.empty((nbf, nbf), dtype=torch.float64, device=f"cuda:{device}")
    shgo_execute_cartesian(plan, out)
    torch.cuda.current_stream().synchronize()
    return out


def nuclear_attraction_cartesian_pairs(basis, nuclei, pair_a, pair_b, screen=0.0, device=0):
    """Blocks of the listed shell pairs by the Cartesian route, as a flat float64 CUDA tensor."""
    import torch
    plan = shgo_plan_pairs(context(device), basis, nuclei, pair_a, pair_b, screen)
    out = torch.empty(plan.output_size, dtype=torch.float64, device=f"cuda:{device}")
    shgo_execute_cartesian(plan, out)
    torch.cuda.current_stream().synchronize()
    return out


def eri_blocks(basis, quartets, device=0, stream=None):
    """Two-electron blocks (ab|cd) of the quartets [n, 4] of shell indices (shells up to l = 2), as a
    flat float64 CUDA tensor: each block (2la+1)(2lb+1)(2lc+1)(2ld+1) row-major, in quartet order."""
    import torch
    lib = load_library()
    ctx = context(device)
    q = np.ascontiguousarray(quartets, dtype=np.int32).reshape(-1, 4)
    hb = _HostBasis(basis)
    size = shgo_eri_output_size(hb, q)
    out = torch.empty(max(size, 1), dtype=torch.float64, device=f"cuda:{device}")
    _check(lib, ctx, lib.shgo_eri_blocks(ctx, ctypes.byref(hb.struct), int(len(q)), q.ctypes.data,
                                         out.data_ptr(), _stream_handle(stream)))
    return out[:size]


def overlap(basis, device=0):
    """Full nbf x nbf overlap matrix S of the basis as a float64 CUDA tensor."""
    import torch
    plan = shgo_plan_matrix(context(device), basis, _no_nuclei(), 0.0)
    nbf = shgo_nbf(basis)
    out = torch.empty((nbf, nbf), dtype=torch.float64, device=f"cuda:{device}")
    shgo_execute_overlap(plan, out)
    torch.cuda.current_stream().synchronize()
    return out


def overlap_pairs(basis, pair_a, pair_b, device=0):
    """Overlap blocks of the listed shell pairs, back to back, as a flat float64 CUDA tensor."""
    import torch
    plan = shgo_plan_pairs(context(device), basis, _no_nuclei(), pair_a, pair_b, 0.0)
    out = torch.empty(plan.output_size, dtype=torch.float64, device=f"cuda:{device}")
    shgo_execute_overlap(plan, out)
    torch.cuda.current_stream().synchronize()
    return out


def _autograd_function():
    import torch

    class NuclearAttractionFn(torch.autograd.Function):
        """V(centers, nuclear positions) with a backward through the adjoint kernel.

        forward(centers [n_shells, 3], positions [n_nuclei, 3], basis, charges, screen) -> V [nbf, nbf];
        the basis supplies l, exponents and contraction coefficients (its centers are ignored in
        favour of ``centers``). backward(dL/dV) runs shgo_execute_grad with D = dL/dV on the plan
        built in forward, so Boys values are recomputed, not stored."""

        @staticmethod
        def forward(ctx, centers, positions, basis, charges, screen=0.0):
            from . import synth
            dev = centers.device
            b = synth.Basis(centers.detach().cpu().numpy().astype(np.float64), basis.l, basis.nprim,
                            basis.prim_off, basis.expo, basis.coef)
            n = synth.Nuclei(positions.detach().cpu().numpy().astype(np.float64), np.asarray(charges, np.float64))
            sctx = context(dev.index or 0)
            plan = shgo_plan_matrix(sctx, b, n, screen)
            nbf = b.nbf()
            V = torch.empty((nbf, nbf), dtype=torch.float64, device=dev)
            shgo_execute(plan, V)
            ctx.plan = plan
            ctx.shapes = (b.n_shells, n.n)
            return V

        @staticmethod
        def backward(ctx, grad_V):
            n_shells, n_nuc = ctx.shapes
            dev = grad_V.device
            dn = torch.empty((n_nuc, 3), dtype=torch.float64, device=dev)
            dc = torch.empty((n_shells, 3), dtype=torch.float64, device=dev)
            shgo_execute_grad(ctx.plan, grad_V.to(torch.float64).contiguous(), dn, dc)
            return dc, dn, None, None, None

    return NuclearAttractionFn


def __getattr__(name):
    if name == "NuclearAttractionFn":
        fn = _autograd_function()
        globals()["NuclearAttractionFn"] = fn
        return fn
    raise AttributeError(name)
