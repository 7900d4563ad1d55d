"""CPU oracle for exact angular pair counting -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The product library never imports, links or calls it.  See
pc_oracle.c for the definition it implements and the readings it takes.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)
_up = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def lib():
    """The oracle library: oracle/libpc_oracle.so (rebuilt when a source is
    newer), or the build named by PC_ORACLE_LIB (variant builds in tests)."""
    global _lib
    if _lib is None:
        path = os.environ.get("PC_ORACLE_LIB")
        if not path:
            path = LIB
            srcs = [os.path.join(os.path.dirname(LIB), f) for f in ("pc_oracle.c", "ap_oracle.c")]
            if not os.path.exists(LIB) or any(os.path.getmtime(f) > os.path.getmtime(LIB) for f in srcs):
                build()
        L = ctypes.CDLL(path)
        L.oracle_sincosd.argtypes = [ctypes.c_double, _dp, _dp]
        L.oracle_sincosd.restype = None
        L.oracle_unit_vectors.argtypes = [_i64, _dp, _dp, _dp]
        L.oracle_unit_vectors.restype = None
        L.oracle_chord2_edges.argtypes = [_i32, _dp, _dp]
        L.oracle_chord2_edges.restype = None
        L.oracle_count_xyz.argtypes = [_i64, _dp, _i64, _dp, _i32, _i32, _dp, _i64, _i64, _up]
        L.oracle_count_xyz.restype = None
        L.oracle_count.argtypes = [_i64, _dp, _dp, _i64, _dp, _dp, _i32, _i32, _dp, _i64, _i64, _up]
        L.oracle_count.restype = ctypes.c_int
        L.oracle_wtheta.argtypes = [_up, _up, _up, _i32, _i64, _i64, _dp]
        L.oracle_wtheta.restype = None
        L.oracle_estimator.argtypes = [_i32, _up, _up, _up, _i32, _i64, _i64, _dp]
        L.oracle_estimator.restype = None
        L.oracle_q_nfw.argtypes = [ctypes.c_double]
        L.oracle_q_nfw.restype = ctypes.c_double
        L.oracle_aperture_points.argtypes = [_i64, _dp, _dp, _dp, _dp, _i64, _dp, _dp, ctypes.c_double,
                                             ctypes.c_double, _dp, _dp, _u32p, _dp]
        L.oracle_aperture_points.restype = None
        L.oracle_aperture_grid.argtypes = [_i64, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, _i32, _i32, ctypes.c_double,
                                           ctypes.c_double, _dp, _dp, _u32p, _dp]
        L.oracle_aperture_grid.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _u(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(_up)


def sincosd(x: float):
    s = ctypes.c_double()
    c = ctypes.c_double()
    lib().oracle_sincosd(float(x), ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def unit_vectors(ra, dec) -> np.ndarray:
    ra, pr = _d(ra)
    dec, pd = _d(dec)
    out = np.empty((ra.size, 3), dtype=np.float64)
    lib().oracle_unit_vectors(ra.size, pr, pd, out.ctypes.data_as(_dp))
    return out


def chord2_edges(theta_deg) -> np.ndarray:
    t, pt = _d(theta_deg)
    out = np.empty(t.size, dtype=np.float64)
    lib().oracle_chord2_edges(t.size, pt, out.ctypes.data_as(_dp))
    return out


def count_xyz(xyzA, e, xyzB=None, auto=True, rows=None) -> np.ndarray:
    xa, pa = _d(xyzA)
    nA = xa.size // 3
    if auto:
        xb, pb, nB = None, None, 0
    else:
        xb, pb = _d(xyzB)
        nB = xb.size // 3
    e, pe = _d(e)
    r0, r1 = (0, nA) if rows is None else rows
    out = np.zeros(e.size + 1, dtype=np.uint64)
    lib().oracle_count_xyz(nA, pa, nB, pb, 1 if auto else 0, e.size, pe, r0, r1,
                           out.ctypes.data_as(_up))
    return out


def count(A, theta_edges, B=None, auto=True, rows=None) -> np.ndarray:
    """Pair counts [under, bin 0..B-1, over] for catalogue A = (ra, dec) (auto
    pairs i<j) or A x B (cross).  rows = (r0, r1) restricts i to [r0, r1)."""
    ra, pra = _d(A[0])
    da, pda = _d(A[1])
    if auto:
        rb = db = None
        prb = pdb = None
        nB = 0
    else:
        rb, prb = _d(B[0])
        db, pdb = _d(B[1])
        nB = rb.size
    t, pt = _d(theta_edges)
    r0, r1 = (0, ra.size) if rows is None else rows
    out = np.zeros(t.size + 1, dtype=np.uint64)
    rc = lib().oracle_count(ra.size, pra, pda, nB, prb, pdb, 1 if auto else 0, t.size, pt,
                            int(r0), int(r1), out.ctypes.data_as(_up))
    if rc != 0:
        raise MemoryError("oracle_count: out of memory")
    return out


def wtheta(DD, DR, RR, nD: int, nR: int) -> np.ndarray:
    DD, p1 = _u(DD)
    DR, p2 = _u(DR)
    RR, p3 = _u(RR)
    out = np.empty(DD.size, dtype=np.float64)
    lib().oracle_wtheta(p1, p2, p3, DD.size, int(nD), int(nR), out.ctypes.data_as(_dp))
    return out


def estimator(kind: int, DD, DR, RR, nD: int, nR: int) -> np.ndarray:
    """kind 0 Landy-Szalay, 1 natural, 2 Davis-Peebles, 3 Hamilton (DR or RR
    may be None where the estimator does not use it)."""
    DD, p1 = _u(DD)
    p2 = _u(DR)[1] if DR is not None else None
    p3 = _u(RR)[1] if RR is not None else None
    out = np.empty(DD.size, dtype=np.float64)
    lib().oracle_estimator(int(kind), p1, p2, p3, DD.size, int(nD), int(nR), out.ctypes.data_as(_dp))
    return out


def q_nfw(x: float) -> float:
    """Eq. 4 filter at x = theta / theta_max."""
    return lib().oracle_q_nfw(float(x))


def _ap_out(m):
    out = {"map": np.empty(m), "snr": np.empty(m), "n_in": np.empty(m, dtype=np.uint32),
           "sums": np.empty((m, 3))}
    ptrs = (out["map"].ctypes.data_as(_dp), out["snr"].ctypes.data_as(_dp),
            out["n_in"].ctypes.data_as(_u32p), out["sums"].ctypes.data_as(_dp))
    return out, ptrs


def _ap_unpack(out):
    s = out.pop("sums")
    out["s1"], out["s2"], out["qe_abs"] = s[:, 0].copy(), s[:, 1].copy(), s[:, 2].copy()
    return out


def aperture_points(cat, px, py, theta_max: float, n_gal: float) -> dict:
    """Aperture mass (Eq. 3) and SNR (Eq. 5) at the points (px, py) for the
    shear catalogue cat = (x, y, e1, e2).  Returns map, snr, n_in and the raw
    sums s1 = sum Q eps_t, s2 = sum Q^2 |eps|^2, qe_abs = sum Q |eps|."""
    (x, p0), (y, p1), (e1, p2), (e2, p3) = (_d(a) for a in cat)
    px, pp = _d(px)
    py, pq = _d(py)
    out, ptrs = _ap_out(px.size)
    lib().oracle_aperture_points(x.size, p0, p1, p2, p3, px.size, pp, pq, float(theta_max), float(n_gal), *ptrs)
    return _ap_unpack(out)


def aperture_grid(cat, grid, theta_max: float, n_gal: float) -> dict:
    """The same on grid = (x0, y0, dx, dy, nx, ny): point (ix, iy) at
    (x0 + ix*dx, y0 + iy*dy), flattened row-major (index iy*nx + ix)."""
    (x, p0), (y, p1), (e1, p2), (e2, p3) = (_d(a) for a in cat)
    x0, y0, dx, dy, nx, ny = grid
    out, ptrs = _ap_out(int(nx) * int(ny))
    rc = lib().oracle_aperture_grid(x.size, p0, p1, p2, p3, float(x0), float(y0), float(dx), float(dy),
                                    int(nx), int(ny), float(theta_max), float(n_gal), *ptrs)
    if rc != 0:
        raise MemoryError("oracle_aperture_grid: out of memory")
    return _ap_unpack(out)


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    """Number of OpenMP threads the oracle's counting loops use from now on."""
    lib().oracle_set_num_threads(int(n))
