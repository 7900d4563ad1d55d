"""Python binding of libpc.so: exact angular pair counting on AMD MI355X.

Argument marshalling only -- every step runs in the HIP library.  Functions
carry the C names of include/pc.h.  Catalogues are (ra_deg, dec_deg) pairs of
float64 arrays: torch CUDA tensors are passed as device pointers, numpy arrays
(or CPU tensors) as host pointers.  Counts come back as numpy uint64 arrays of
n_edges + 1 entries [underflow, bins..., overflow].
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpc.so")

PC_OK, PC_ERR_INVALID, PC_ERR_NOMEM, PC_ERR_DEVICE, PC_ERR_BUSY, PC_ERR_CANCELLED = range(6)
PC_MIXED, PC_FP64_PLAIN = 0, 1
PC_NO_PRUNE = 0x100
PC_MATRIX_CORES = 0x200
PC_TUNED = 0x400


class PcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpc error {code}: {msg}")
        self.code = code


class pc_catalog(ctypes.Structure):
    _fields_ = [("ra_deg", ctypes.c_void_p), ("dec_deg", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("on_device", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class pc_job(ctypes.Structure):
    _fields_ = [("A", ctypes.POINTER(pc_catalog)), ("B", ctypes.POINTER(pc_catalog)),
                ("theta_edges_deg", ctypes.c_void_p), ("n_edges", ctypes.c_int32),
                ("auto_flag", ctypes.c_int32), ("row_begin", ctypes.c_int64),
                ("row_end", ctypes.c_int64), ("counts", ctypes.c_void_p)]


class pc_shear_catalog(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("e1", ctypes.c_void_p), ("e2", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("on_device", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class pc_grid(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


_lib = None

_i32, _i64, _u64, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
_PCAT = ctypes.POINTER(pc_catalog)

_SIGNATURES = {
    "pc_aperture_mass": ([ctypes.POINTER(pc_shear_catalog), ctypes.POINTER(pc_grid), ctypes.c_double, ctypes.c_double,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p],
                         ctypes.c_int),
    "pc_debug_ap_filter": ([_vp, _i64, _vp], ctypes.c_int),
    "pc_debug_ap_points_per_lane": ([_i32], ctypes.c_int),
    "pc_debug_last_aperture": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64),
                                ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "pc_debug_admission_plan": ([_vp, _vp, _vp, _i32, _u64, _u64, _u64, _i32, ctypes.c_char_p, _vp],
                                ctypes.c_int),
    "pc_debug_last_rechecks": ([ctypes.POINTER(_u64)], ctypes.c_int),
    "pc_debug_last_paths": ([_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64)], ctypes.c_int),
    "pc_count": ([_PCAT, _PCAT, _vp, _i32, _i32, _vp, _vp], ctypes.c_int),
    "pc_count_ex": ([_PCAT, _PCAT, _vp, _i32, _i32, _i32, _i64, _i64, _vp, _vp], ctypes.c_int),
    "pc_count_batch": ([ctypes.POINTER(pc_job), _i32, _i32, _vp], ctypes.c_int),
    "pc_count_batch_static": ([ctypes.POINTER(pc_job), _i32, _i32, _vp], ctypes.c_int),
    "pc_wtheta": ([_vp, _vp, _vp, _i32, _i64, _i64, _vp], ctypes.c_int),
    "pc_bin_edges": ([_i32, ctypes.c_double, ctypes.c_double, _i32, ctypes.c_double, _i32, _vp,
                      ctypes.POINTER(_i32)], ctypes.c_int),
    "pc_last_error": ([], ctypes.c_char_p),
    "pc_version": ([], ctypes.c_char_p),
    "pc_catalog_upload": ([_PCAT, _vp, ctypes.POINTER(_u64)], ctypes.c_int),
    "pc_catalog_release": ([_u64], ctypes.c_int),
    "pc_count_h": ([_u64, _u64, _vp, _i32, _i32, _i32, _i64, _i64, _vp, _vp], ctypes.c_int),
    "pc_unit_vectors": ([_PCAT, _vp, _vp, _vp], ctypes.c_int),
    "pc_chord2_edges": ([_vp, _i32, _vp], ctypes.c_int),
    "pc_guard_band": ([_vp, _i32, _vp, _vp], ctypes.c_int),
    "pc_estimator": ([_i32, _vp, _vp, _vp, _i32, _i64, _i64, _vp], ctypes.c_int),
    "pc_autotune": ([_vp, _i32, _i32, ctypes.c_char_p, _vp, ctypes.c_char_p, _i32], ctypes.c_int),
    "pc_autotune_load": ([ctypes.c_char_p], ctypes.c_int),
    "pc_debug_lut32": ([_vp, _i32, _vp, _vp, _i64], ctypes.c_int),
    "pc_debug_set_timing": ([_i32], ctypes.c_int),
    "pc_debug_set_flush_every": ([_u64], ctypes.c_int),
    "pc_debug_set_compact_table": ([_i32], ctypes.c_int),
    "pc_debug_fail_allocations": ([_i32], ctypes.c_int),
    "pc_debug_set_tile": ([_i32], ctypes.c_int),
    "pc_debug_server_hold": ([_vp, _i32], ctypes.c_int),
    "pc_debug_request_parts": ([_i64, _i64, _i32, _i32, ctypes.c_double, _i32, _vp, _vp, ctypes.POINTER(_i32)],
                               ctypes.c_int),
    "pc_debug_last_launch": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "pc_debug_last_pruning": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "pc_debug_guard_band_gram": ([_vp, _i32, _vp, _vp], ctypes.c_int),
    "pc_debug_fused_band": ([_vp, _i32, _i32, _vp, _vp], ctypes.c_int),
    "pc_server_create": ([ctypes.c_char_p, ctypes.POINTER(_vp)], ctypes.c_int),
    "pc_server_set_random": ([_vp, _i32, _PCAT], ctypes.c_int),
    "pc_server_submit": ([_vp, _PCAT, _i32, _vp, _i32, ctypes.POINTER(_u64)], ctypes.c_int),
    "pc_server_poll": ([_vp, _u64, ctypes.POINTER(_i32), _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "pc_server_cancel": ([_vp, _u64, ctypes.POINTER(_i32)], ctypes.c_int),
    "pc_server_drain": ([_vp], ctypes.c_int),
    "pc_server_stats": ([_vp], ctypes.c_char_p),
    "pc_server_destroy": ([_vp], ctypes.c_int),
}


def _torch_runtime_first():
    """PyTorch ships its own HIP runtime beside the system one libpc.so links.
    Both can drive the GPU in one process, but only when PyTorch's starts
    first (the other order leaves PyTorch without a device), so initialise it
    before loading the library whenever PyTorch and a GPU are present."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def lib():
    """The loaded libpc.so.  Raises ImportError when it has not been built:
    there is no fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1208_3658_amd.build` "
                              "(or __graft_entry__.build()); there is no CPU fallback")
        _torch_runtime_first()
        L = ctypes.CDLL(LIB_PATH)
        for name, (argt, rest) in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = argt
            f.restype = rest
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PC_OK:
        raise PcError(rc, lib().pc_last_error().decode())


def pc_last_error() -> str:
    return lib().pc_last_error().decode()


def pc_version() -> str:
    return lib().pc_version().decode()


# ---------------------------------------------------------------- marshalling

def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class Catalog:
    """Holds a pc_catalog and keeps its arrays alive."""

    def __init__(self, ra, dec):
        if _is_torch(ra):
            if ra.dtype != dec.dtype or str(ra.dtype) != "torch.float64":
                raise TypeError("catalogue tensors must be float64")
            if ra.device != dec.device:
                raise ValueError("ra and dec on different devices")
            if ra.is_cuda:
                ra, dec = ra.contiguous(), dec.contiguous()
                self.keep = (ra, dec)
                self.c = pc_catalog(ra.data_ptr(), dec.data_ptr(), ra.numel(), 1, 0)
                if ra.numel() != dec.numel():
                    raise ValueError("ra and dec differ in length")
                return
            ra, dec = ra.numpy(), dec.numpy()
        ra = np.ascontiguousarray(ra, dtype=np.float64)
        dec = np.ascontiguousarray(dec, dtype=np.float64)
        if ra.shape != dec.shape or ra.ndim != 1:
            raise ValueError("ra and dec must be 1-D arrays of equal length")
        self.keep = (ra, dec)
        self.c = pc_catalog(ra.ctypes.data, dec.ctypes.data, ra.size, 0, 0)

    @property
    def n(self) -> int:
        return int(self.c.n)

    def ref(self):
        return ctypes.byref(self.c)


def as_catalog(x) -> Catalog:
    if isinstance(x, Catalog):
        return x
    ra, dec = x
    return Catalog(ra, dec)


def _edges(theta):
    t = np.ascontiguousarray(theta, dtype=np.float64)
    return t, t.ctypes.data


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


# --------------------------------------------------------------------- API

def pc_count(A, theta_edges, B=None, auto: bool = True, stream=None) -> np.ndarray:
    """Pair counts [under, bins, over] (uint64, len(theta_edges)+1)."""
    return pc_count_ex(A, theta_edges, B=B, auto=auto, mode=PC_MIXED, stream=stream)


def pc_count_ex(A, theta_edges, B=None, auto: bool = True, mode: int = PC_MIXED,
                rows=(0, -1), stream=None) -> np.ndarray:
    a = as_catalog(A)
    b = None if auto else as_catalog(B)
    t, tp = _edges(theta_edges)
    out = np.zeros(t.size + 1, dtype=np.uint64)
    _check(lib().pc_count_ex(a.ref(), None if b is None else b.ref(), tp, t.size, 1 if auto else 0,
                             int(mode), int(rows[0]), int(rows[1]), out.ctypes.data, _stream(stream)))
    return out


def _job_array(jobs, keep):
    cats = {}

    def cat(x):
        key = id(x)
        if key not in cats:
            cats[key] = as_catalog(x)
        return cats[key]

    arr = (pc_job * len(jobs))()
    outs = []
    for q, j in enumerate(jobs):
        a = cat(j["A"])
        auto = bool(j.get("auto", True))
        b = None if auto else cat(j["B"])
        t, tp = _edges(j["edges"])
        out = np.zeros(t.size + 1, dtype=np.uint64)
        r0, r1 = j.get("rows", (0, -1))
        keep += [a, b, t, out]
        arr[q] = pc_job(ctypes.pointer(a.c), None if b is None else ctypes.pointer(b.c), tp, t.size,
                        1 if auto else 0, int(r0), int(r1), out.ctypes.data)
        outs.append(out)
    return arr, outs


def pc_autotune(jobs, mode: int = PC_MIXED, cache_path=None, stream=None):
    """Time the batch under each candidate launch configuration, keep the
    fastest for batches of this shape (used with PC_TUNED) and add it to
    cache_path if given.  Returns (counts per job, chosen configuration)."""
    keep = []
    arr, outs = _job_array(jobs, keep)
    buf = ctypes.create_string_buffer(1024)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().pc_autotune(arr, len(jobs), int(mode), path, _stream(stream), buf, len(buf)))
    return outs, json.loads(buf.value.decode())


def pc_autotune_load(cache_path) -> None:
    _check(lib().pc_autotune_load(os.fsencode(cache_path)))


def pc_count_batch(jobs, mode: int = PC_MIXED, stream=None):
    """jobs: list of dicts {A, B (cross only), edges, auto, rows}.  Returns a
    list of count arrays, one per job, from one launch."""
    keep = []
    cats = {}

    def cat(x):
        key = id(x)
        if key not in cats:
            cats[key] = as_catalog(x)
        return cats[key]

    arr = (pc_job * len(jobs))()
    outs = []
    for q, j in enumerate(jobs):
        a = cat(j["A"])
        auto = bool(j.get("auto", True))
        b = None if auto else cat(j["B"])
        t, tp = _edges(j["edges"])
        out = np.zeros(t.size + 1, dtype=np.uint64)
        r0, r1 = j.get("rows", (0, -1))
        keep += [a, b, t, out]
        arr[q] = pc_job(ctypes.pointer(a.c), None if b is None else ctypes.pointer(b.c), tp, t.size,
                        1 if auto else 0, int(r0), int(r1), out.ctypes.data)
        outs.append(out)
    _check(lib().pc_count_batch(arr, len(jobs), int(mode), _stream(stream)))
    return outs


PC_STATIC_SCRATCH_BYTES = 256 * 1024 * 1024


def pc_count_batch_static(jobs, mode: int = PC_MIXED, stream=None):
    """pc_count_batch in the library's fixed device work area of
    PC_STATIC_SCRATCH_BYTES (no device allocation by the library; calls on
    one GPU share that area).  Same jobs, same counts."""
    keep = []
    arr, outs = _job_array(jobs, keep)
    _check(lib().pc_count_batch_static(arr, len(jobs), int(mode), _stream(stream)))
    return outs


PC_BINS_EVEN, PC_BINS_LN, PC_BINS_LOG10 = 0, 1, 2


def pc_bin_edges(preset: int, lo_deg: float, hi_deg: float, n_bins: int = 0, width: float = 0.0) -> np.ndarray:
    """Theta edges (degrees) from the paper's binning presets: limits lo, hi
    and evenly spaced, natural-log or log10 bins, given as a number of bins
    or as a width in the preset's scale (include/pc.h)."""
    n = _i32(0)
    _check(lib().pc_bin_edges(int(preset), float(lo_deg), float(hi_deg), int(n_bins), float(width), 0, None,
                              ctypes.byref(n)))
    e = np.empty(n.value, dtype=np.float64)
    _check(lib().pc_bin_edges(int(preset), float(lo_deg), float(hi_deg), int(n_bins), float(width), e.size,
                              e.ctypes.data, ctypes.byref(n)))
    return e


def pc_wtheta(DD, DR, RR, nD: int, nR: int) -> np.ndarray:
    """Landy-Szalay w(theta) from in-range bin counts (pass counts[1:-1])."""
    DD = np.ascontiguousarray(DD, dtype=np.uint64)
    DR = np.ascontiguousarray(DR, dtype=np.uint64)
    RR = np.ascontiguousarray(RR, dtype=np.uint64)
    if not (DD.size == DR.size == RR.size):
        raise ValueError("DD, DR, RR differ in length")
    w = np.empty(DD.size, dtype=np.float64)
    _check(lib().pc_wtheta(DD.ctypes.data, DR.ctypes.data, RR.ctypes.data, DD.size, int(nD), int(nR),
                           w.ctypes.data))
    return w


PC_EST_LANDY_SZALAY, PC_EST_NATURAL, PC_EST_DAVIS_PEEBLES, PC_EST_HAMILTON = 0, 1, 2, 3


def pc_estimator(kind: int, DD, DR, RR, nD: int, nR: int) -> np.ndarray:
    """w(theta) by estimator `kind` (PC_EST_*) from in-range bin counts; DR
    (natural) or RR (Davis-Peebles) may be None."""
    arrs = [None if x is None else np.ascontiguousarray(x, dtype=np.uint64) for x in (DD, DR, RR)]
    n = arrs[0].size
    if any(a is not None and a.size != n for a in arrs):
        raise ValueError("DD, DR, RR differ in length")
    w = np.empty(n, dtype=np.float64)
    ptrs = [None if a is None else a.ctypes.data for a in arrs]
    _check(lib().pc_estimator(int(kind), ptrs[0], ptrs[1], ptrs[2], n, int(nD), int(nR), w.ctypes.data))
    return w


def pc_catalog_upload(A, stream=None) -> int:
    a = as_catalog(A)
    h = _u64(0)
    _check(lib().pc_catalog_upload(a.ref(), _stream(stream), ctypes.byref(h)))
    return int(h.value)


def pc_catalog_release(handle: int):
    _check(lib().pc_catalog_release(int(handle)))


def pc_count_h(hA: int, theta_edges, hB: int = 0, auto: bool = True, mode: int = PC_MIXED,
               rows=(0, -1), stream=None) -> np.ndarray:
    t, tp = _edges(theta_edges)
    out = np.zeros(t.size + 1, dtype=np.uint64)
    _check(lib().pc_count_h(int(hA), int(hB), tp, t.size, 1 if auto else 0, int(mode), int(rows[0]),
                            int(rows[1]), out.ctypes.data, _stream(stream)))
    return out


def pc_unit_vectors(A, stream=None):
    a = as_catalog(A)
    x64 = np.empty((a.n, 3), dtype=np.float64)
    x32 = np.empty((a.n, 3), dtype=np.float32)
    _check(lib().pc_unit_vectors(a.ref(), x64.ctypes.data, x32.ctypes.data, _stream(stream)))
    return x64, x32


def pc_chord2_edges(theta_edges) -> np.ndarray:
    t, tp = _edges(theta_edges)
    e = np.empty(t.size, dtype=np.float64)
    _check(lib().pc_chord2_edges(tp, t.size, e.ctypes.data))
    return e


def pc_guard_band(theta_edges, gram: bool = False):
    """Per-edge binary32 guard band (lo, hi); gram=True: the matrix-core
    path's band (tile-centred chords)."""
    t, tp = _edges(theta_edges)
    lo = np.empty(t.size, dtype=np.float32)
    hi = np.empty(t.size, dtype=np.float32)
    f = lib().pc_debug_guard_band_gram if gram else lib().pc_guard_band
    _check(f(tp, t.size, lo.ctypes.data, hi.ctypes.data))
    return lo, hi


def pc_debug_fused_band(theta_edges, gram: bool = False):
    """Per-edge thresholds (h, w) of the vector few-edge paths' fused
    differences d = h - c; gram=True: tile-centred Gram chords."""
    t, tp = _edges(theta_edges)
    h = np.empty(t.size, dtype=np.float32)
    w = np.empty(t.size, dtype=np.float32)
    _check(lib().pc_debug_fused_band(tp, t.size, 1 if gram else 0, h.ctypes.data, w.ctypes.data))
    return h, w


def pc_debug_lut32(theta_edges):
    t, tp = _edges(theta_edges)
    f = lib().pc_debug_lut32
    info = np.zeros(8, dtype=np.int64)
    _check(f(tp, t.size, info.ctypes.data, None, 0))
    ent = np.zeros((int(info[0]), 4), dtype=np.uint32)
    _check(f(tp, t.size, info.ctypes.data, ent.ctypes.data, int(info[0])))
    keys = ["n_cells", "shift", "clamp_lo", "clamp_hi", "row_bytes", "cols", "multi", "_"]
    return dict(zip(keys, (int(v) for v in info))), ent


def pc_debug_set_timing(on: bool):
    _check(lib().pc_debug_set_timing(1 if on else 0))


def pc_debug_set_flush_every(items: int):
    """items > 0: flush the counting kernel's LDS histograms at least every
    `items` work items on this thread (testing); 0: default."""
    _check(lib().pc_debug_set_flush_every(int(items)))


def pc_debug_set_compact_table(mode: int):
    """Cell table form of this thread's later mixed counting launches: 0 the
    8-byte form when it raises the waves per CU (default), 1 whenever built,
    -1 never (testing)."""
    _check(lib().pc_debug_set_compact_table(int(mode)))


def pc_debug_set_tile(tile: int):
    """Tile size (128 or 256 points) of this thread's later counting launches
    that have no explicit launch parameters; 0 restores the default."""
    _check(lib().pc_debug_set_tile(int(tile)))


def pc_debug_fail_allocations(n: int):
    """The calling thread's next n device allocations in the library fail as
    out of memory (testing); 0 turns it off."""
    _check(lib().pc_debug_fail_allocations(int(n)))


def pc_debug_last_launch() -> dict:
    ms = ctypes.c_double(0)
    items = _u64(0)
    grid = _i32(0)
    lds = ctypes.c_uint32(0)
    _check(lib().pc_debug_last_launch(ctypes.byref(ms), ctypes.byref(items), ctypes.byref(grid), ctypes.byref(lds)))
    return {"kernel_ms": ms.value, "items": int(items.value), "grid": int(grid.value), "lds_bytes": int(lds.value)}


def pc_debug_last_pruning() -> dict:
    vals = [_u64(0) for _ in range(7)]
    _check(lib().pc_debug_last_pruning(*(ctypes.byref(v) for v in vals)))
    keys = ("survivors", "pairs_computed", "pairs_total", "mfma_items", "few_items", "gram_items", "split_items")
    return {k: int(v.value) for k, v in zip(keys, vals)}


def pc_debug_last_paths() -> dict:
    """Pairs of the calling thread's last counting launch by the path that
    binned them: by_edges[m] (m = 1..3 edges compared one by one, 0 = cell
    table), gram (Gram-form chords), mfma (matrix-core chords)."""
    by = np.zeros(4, dtype=np.uint64)
    g, m = _u64(0), _u64(0)
    _check(lib().pc_debug_last_paths(by.ctypes.data, ctypes.byref(g), ctypes.byref(m)))
    return {"by_edges": [int(x) for x in by], "gram": int(g.value), "mfma": int(m.value)}


def pc_debug_last_rechecks() -> int:
    """Pairs of the calling thread's last counting launch that were re-checked
    in binary64 (binary32 chord inside an edge's guard band)."""
    v = _u64(0)
    _check(lib().pc_debug_last_rechecks(ctypes.byref(v)))
    return int(v.value)


# ------------------------------------------------------------ aperture mass

def pc_aperture_mass(cat, grid, theta_max: float, n_gal: float, out=None, stream=None) -> dict:
    """Aperture mass (Eq. 3), SNR (Eq. 5) and aperture occupancy on a grid
    (include/pc_aperture.h).  cat = (x, y, e1, e2): float64 torch CUDA
    tensors (device catalogue) or arrays (host).  grid = (x0, y0, dx, dy, nx,
    ny): point (ix, iy) at (x0 + ix*dx, y0 + iy*dy), index iy*nx + ix.
    out = None: returns numpy arrays {map, snr, n_in}; otherwise a dict of
    contiguous torch CUDA tensors map (float64), snr (float64 or None) and
    n_in (int32 or None) of nx*ny entries, written on the device."""
    x, y, e1, e2 = cat
    if _is_torch(x) and x.is_cuda:
        arrs = [a.contiguous() for a in (x, y, e1, e2)]
        if any(str(a.dtype) != "torch.float64" or not a.is_cuda for a in arrs):
            raise TypeError("shear catalogue tensors must be float64 CUDA tensors")
        on_dev = 1
        ptrs = [a.data_ptr() for a in arrs]
    else:
        arrs = [np.ascontiguousarray(a.numpy() if _is_torch(a) else a, dtype=np.float64) for a in (x, y, e1, e2)]
        on_dev = 0
        ptrs = [a.ctypes.data for a in arrs]
    n = arrs[0].numel() if on_dev else arrs[0].size
    for a in arrs[1:]:
        if (a.numel() if on_dev else a.size) != n:
            raise ValueError("x, y, e1 and e2 differ in length")
    c = pc_shear_catalog(*ptrs, n, on_dev, 0)
    x0, y0, dx, dy, nx, ny = grid
    g = pc_grid(float(x0), float(y0), float(dx), float(dy), int(nx), int(ny))
    m = int(nx) * int(ny)
    if out is None:
        alloc = m if 0 <= m < 2 ** 31 else 1  # sizes out of range are the library's to reject
        res = {"map": np.empty(alloc), "snr": np.empty(alloc), "n_in": np.empty(alloc, dtype=np.uint32)}
        _check(lib().pc_aperture_mass(ctypes.byref(c), ctypes.byref(g), float(theta_max), float(n_gal),
                                      res["map"].ctypes.data, res["snr"].ctypes.data, res["n_in"].ctypes.data, 0,
                                      _stream(stream)))
        return res
    ptr = lambda k: out[k].data_ptr() if out.get(k) is not None else None
    for k, dt, sz in (("map", "torch.float64", 8), ("snr", "torch.float64", 8), ("n_in", "torch.int32", 4)):
        t = out.get(k)
        if t is not None and (str(t.dtype) != dt or not t.is_cuda or not t.is_contiguous() or t.numel() != m):
            raise TypeError(f"out[{k!r}] must be a contiguous {dt} CUDA tensor of {m} entries")
    _check(lib().pc_aperture_mass(ctypes.byref(c), ctypes.byref(g), float(theta_max), float(n_gal), ptr("map"),
                                  ptr("snr"), ptr("n_in"), 1, _stream(stream)))
    return out


def pc_debug_ap_filter(x) -> np.ndarray:
    """Eq. 4's Q(x) as the map kernel evaluates it (its table and binary32
    steps), computed on the host."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    q = np.empty(x.size, dtype=np.float64)
    _check(lib().pc_debug_ap_filter(x.ctypes.data, x.size, q.ctypes.data))
    return q


def pc_debug_ap_points_per_lane(points: int):
    """Force 1 or 2 grid points per lane along each axis in this thread's
    aperture-mass calls (0: the call's own choice)."""
    _check(lib().pc_debug_ap_points_per_lane(int(points)))


def pc_debug_last_aperture() -> dict:
    ms = ctypes.c_double(0)
    tested = ctypes.c_uint64(0)
    inside = ctypes.c_uint64(0)
    cell = ctypes.c_double(0)
    _check(lib().pc_debug_last_aperture(ctypes.byref(ms), ctypes.byref(tested), ctypes.byref(inside),
                                        ctypes.byref(cell)))
    return {"kernel_ms": ms.value, "pairs_tested": int(tested.value), "pairs_in": int(inside.value),
            "cell_side": cell.value}


def pc_debug_request_parts(n_points: int, n_random: int, n_edges: int, count_rr: bool = True,
                           slice_pairs: float = 5e11):
    """The server's plan for one request (host only): a list of parts
    {"rows": (a, b), "rr_rows": (c, d), "need_bytes": B}."""
    n = _i32(0)
    _check(lib().pc_debug_request_parts(int(n_points), int(n_random), int(n_edges), 1 if count_rr else 0,
                                        float(slice_pairs), 0, None, None, ctypes.byref(n)))
    rows = np.zeros((max(n.value, 1), 4), dtype=np.int64)
    need = np.zeros(max(n.value, 1), dtype=np.uint64)
    _check(lib().pc_debug_request_parts(int(n_points), int(n_random), int(n_edges), 1 if count_rr else 0,
                                        float(slice_pairs), n.value, rows.ctypes.data, need.ctypes.data,
                                        ctypes.byref(n)))
    return [{"rows": (int(r[0]), int(r[1])), "rr_rows": (int(r[2]), int(r[3])), "need_bytes": int(b)}
            for r, b in zip(rows[: n.value], need[: n.value])]


ADMIT, NEVER_FITS, EXPIRED, WAIT = range(4)


def pc_debug_admission_plan(need_bytes, pairs, age_s, free_bytes: int, total_bytes: int,
                            reserved_bytes: int = 0, inflight: int = 0, config: dict | None = None):
    """The server's admission decision for a described queue (front first):
    int32 array of ADMIT, NEVER_FITS, EXPIRED or WAIT.  No device involved."""
    need = np.ascontiguousarray(need_bytes, dtype=np.uint64)
    prs = np.ascontiguousarray(pairs, dtype=np.float64)
    age = np.ascontiguousarray(age_s, dtype=np.float64)
    if not (need.ndim == prs.ndim == age.ndim == 1 and need.size == prs.size == age.size):
        raise ValueError("need_bytes, pairs and age_s must be 1-D arrays of one length")
    out = np.full(max(need.size, 1), -1, dtype=np.int32)
    cfg = None if config is None else json.dumps(config).encode()
    _check(lib().pc_debug_admission_plan(need.ctypes.data, prs.ctypes.data, age.ctypes.data, need.size,
                                         int(free_bytes), int(total_bytes), int(reserved_bytes), int(inflight),
                                         cfg, out.ctypes.data))
    return out[: need.size]


# ------------------------------------------------------------------ serving

class Server:
    """w(theta) request server (pc_server_*)."""

    def __init__(self, config: dict | None = None):
        self._h = _vp()
        cfg = None if config is None else json.dumps(config).encode()
        _check(lib().pc_server_create(cfg, ctypes.byref(self._h)))
        self._keep = {}

    def set_random(self, patch_id: int, R):
        r = as_catalog(R)
        _check(lib().pc_server_set_random(self._h, int(patch_id), r.ref()))

    def submit(self, D, patch_id: int, theta_edges) -> int:
        d = as_catalog(D)
        t, tp = _edges(theta_edges)
        jid = _u64(0)
        _check(lib().pc_server_submit(self._h, d.ref(), int(patch_id), tp, t.size, ctypes.byref(jid)))
        self._keep[int(jid.value)] = t.size
        return int(jid.value)

    def poll(self, job_id: int):
        """None while running; else dict with DD, DR, RR, w, latency_s."""
        ne = self._keep[job_id]
        DD = np.zeros(ne + 1, dtype=np.uint64)
        DR = np.zeros(ne + 1, dtype=np.uint64)
        RR = np.zeros(ne + 1, dtype=np.uint64)
        w = np.zeros(max(ne - 1, 1), dtype=np.float64)
        lat = ctypes.c_double(0.0)
        done = _i32(0)
        rc = lib().pc_server_poll(self._h, int(job_id), ctypes.byref(done), DD.ctypes.data, DR.ctypes.data,
                                  RR.ctypes.data, w.ctypes.data, ctypes.byref(lat))
        if done.value == 0:
            return None
        del self._keep[job_id]
        _check(rc)
        return {"DD": DD, "DR": DR, "RR": RR, "w": w[: ne - 1], "latency_s": lat.value}

    def cancel(self, job_id: int) -> bool:
        """True when the request will report PC_ERR_CANCELLED from poll; False
        when it had already finished (its answer stays pollable)."""
        c = _i32(0)
        _check(lib().pc_server_cancel(self._h, int(job_id), ctypes.byref(c)))
        return bool(c.value)

    def drain(self):
        _check(lib().pc_server_drain(self._h))

    def hold(self, on: bool):
        """Debug gate (pc_debug_server_hold): while on, admitted batches wait
        before their launch."""
        _check(lib().pc_debug_server_hold(self._h, 1 if on else 0))

    def stats(self) -> dict:
        return json.loads(lib().pc_server_stats(self._h).decode())

    def close(self):
        if self._h:
            _check(lib().pc_server_destroy(self._h))
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
