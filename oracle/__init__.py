"""CPU oracle for the docking hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library in
``paper_2303_06150_amd``) never imports it, and the two share no code.

The arithmetic lives in ``oracle.cpp`` (plain single-threaded C++, templated on
float / double, compiled with ``-ffp-contract=off`` and no fast-math); this
module only marshals numpy arrays through ctypes.  See ``oracle.cpp`` for the
steps and the passages of the paper they follow.

Parity status of each entry point:
  dock_ligand, scan, place, score, topk -- pinned by the tests in
      tests/test_oracle_pins.py (closed-form grids, voxel-shift invariance,
      rigid-distance invariants, brute-force clash sets, exhaustive one-torsion
      search, a textbook sort);
  pose_grad -- pinned by central finite differences of pose_map and by the
      closed form on a linear grid;
  pose_map  -- pinned by rigid-distance invariants and by reduction to the
      rigid moves at zero torsion.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# Plain, unvectorised build: no fast-math, no contraction of a*b+c into fma.
CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-mfma"]


def build() -> str:
    cmd = ["g++", *CXXFLAGS, "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double),
                ("inv_spacing", ctypes.c_double), ("out_value", ctypes.c_double),
                ("values", ctypes.c_void_p)]


class _Lig(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("K", ctypes.c_int), ("xyz", ctypes.c_void_p),
                ("ref", ctypes.c_void_p), ("ta", ctypes.c_void_p), ("tb", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("inv_len", ctypes.c_void_p)]


class _Dock(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int), ("A", ctypes.c_int), ("T", ctypes.c_int), ("S", ctypes.c_int),
                ("restarts", ctypes.c_void_p), ("angles", ctypes.c_void_p),
                ("trans_step", ctypes.c_double), ("clash2", ctypes.c_double),
                ("center", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_score.restype = ctypes.c_double
        lib.oracle_pose_grad.restype = ctypes.c_double
        lib.oracle_refine.restype = ctypes.c_double
        lib.oracle_move_grad.restype = ctypes.c_double
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class _Keep:
    """Holds the numpy buffers a ctypes struct points into."""

    def __init__(self):
        self.bufs = []

    def __call__(self, a, dt):
        a = np.ascontiguousarray(a, dt)
        self.bufs.append(a)
        return a


def _grid(pocket, keep):
    g = keep(pocket.grid, np.float32)
    nz, ny, nx = g.shape
    s = _Grid(nx, ny, nz, (ctypes.c_double * 3)(*[float(v) for v in pocket.origin]),
              float(pocket.spacing), float(pocket.inv_spacing), float(pocket.out_value), _p(g))
    return s


def _lig(lig, keep, fp64=False):
    xyz = keep(lig["xyz64"] if fp64 else lig["xyz"], np.float64)
    ref = keep(lig["ref64"] if fp64 else lig["ref"], np.float64)
    ta = keep(lig["tors_a"], np.int32)
    tb = keep(lig["tors_b"], np.int32)
    mk = keep(lig["frag_mask"], np.uint32)
    il = keep(lig["inv_len64"] if fp64 else lig["inv_len"], np.float64)
    return _Lig(int(lig["N"]), int(lig["K"]), _p(xyz), _p(ref), _p(ta), _p(tb), _p(mk), _p(il))


def _dock(restarts, angles, T, S, trans_step, clash2, center, keep):
    rs = keep(restarts, np.float64)
    an = keep(angles, np.float64)
    ce = keep(center, np.float64)
    return _Dock(int(rs.shape[0]), int(an.shape[0]), int(T), int(S), _p(rs), _p(an),
                 float(trans_step), float(clash2), _p(ce))


def dock_ligand(lig, pocket, restarts, angles, T, S, trans_step, clash2, bits=32, fp64_input=False,
                want_poses=True, want_trace=True, want_scan_scores=False):
    """Dock one ligand over every row of ``restarts``.

    Returns dict(final [R], poses [R,N,3], pivots [R,3], trace [R,S,6+K] int16,
    scan_scores [R,S,6+K])."""
    lib = _load()
    keep = _Keep()
    g = _grid(pocket, keep)
    L = _lig(lig, keep, fp64_input)
    D = _dock(restarts, angles, T, S, trans_step, clash2, pocket.center, keep)
    R, N, K = D.R, L.N, L.K
    final = np.zeros(R)
    poses = np.zeros((R, N, 3)) if want_poses else None
    pivots = np.zeros((R, 3)) if want_poses else None
    trace = np.zeros((R, S, 6 + K), np.int16) if want_trace else None
    ss = np.zeros((R, S, 6 + K)) if want_scan_scores else None
    lib.oracle_dock_ligand(ctypes.c_int(bits), ctypes.byref(g), ctypes.byref(L), ctypes.byref(D),
                           _p(final), _p(poses), _p(pivots), _p(trace), _p(ss))
    return dict(final=final, poses=poses, pivots=pivots, trace=trace, scan_scores=ss)


def place(lig, row, center, bits=32, fp64_input=False):
    lib = _load()
    keep = _Keep()
    L = _lig(lig, keep, fp64_input)
    row = keep(row, np.float64)
    c = keep(center, np.float64)
    xyz = np.zeros((L.N, 3))
    P = np.zeros(3)
    lib.oracle_place(ctypes.c_int(bits), ctypes.byref(L), _p(row), _p(c), _p(xyz), _p(P))
    return xyz, P


def scan(lig, pocket, angles, T, trans_step, clash2, kind, which, xyz, P, bits=32, fp64_input=False):
    """One scan (kind 0 rotation, 1 translation, 2 torsion) from pose (xyz, P).

    Returns (j*, xyz_out, P_out, sample_scores, sample_ok, best)."""
    lib = _load()
    keep = _Keep()
    g = _grid(pocket, keep)
    L = _lig(lig, keep, fp64_input)
    D = _dock(np.zeros((1, 12)), angles, T, 1, trans_step, clash2, pocket.center, keep)
    xi = keep(xyz, np.float64)
    Pi = keep(P, np.float64)
    xo = np.zeros_like(xi)
    Po = np.zeros(3)
    n = T if kind == 1 else D.A
    sc = np.zeros(n)
    ok = np.zeros(n, np.int32)
    best = ctypes.c_double(0)
    j = lib.oracle_scan(ctypes.c_int(bits), ctypes.byref(g), ctypes.byref(L), ctypes.byref(D),
                        ctypes.c_int(kind), ctypes.c_int(which), _p(xi), _p(Pi), _p(xo), _p(Po),
                        _p(sc), _p(ok), ctypes.byref(best))
    return j, xo, Po, sc, ok.astype(bool), best.value


def score(pocket, xyz, interp, bits=32, per_atom=False, grad=False):
    """Sum of nearest (interp=0) or trilinear (interp=1) values over atoms."""
    lib = _load()
    keep = _Keep()
    g = _grid(pocket, keep)
    x = keep(np.asarray(xyz).reshape(-1, 3), np.float64)
    N = x.shape[0]
    pa = np.zeros(N) if per_atom else None
    gr = np.zeros((N, 3)) if grad else None
    s = lib.oracle_score(ctypes.c_int(bits), ctypes.byref(g), ctypes.c_int(interp), ctypes.c_int(N),
                         _p(x), _p(pa), _p(gr))
    out = [s]
    if per_atom:
        out.append(pa)
    if grad:
        out.append(gr)
    return s if len(out) == 1 else tuple(out)


def pose_grad(lig, pocket, xyz, P):
    """FP64 trilinear score and d(score)/d(t, omega, theta) at zero."""
    lib = _load()
    keep = _Keep()
    g = _grid(pocket, keep)
    L = _lig(lig, keep, True)
    x = keep(np.asarray(xyz).reshape(-1, 3), np.float64)
    Pp = keep(P, np.float64)
    gr = np.zeros(6 + L.K)
    s = lib.oracle_pose_grad(ctypes.byref(g), ctypes.byref(L), _p(x), _p(Pp), _p(gr))
    return s, gr


def pose_map(lig, xyz, P, q):
    """FP64 pose of local parameters q = (t, omega, theta) applied at (xyz, P)."""
    lib = _load()
    keep = _Keep()
    L = _lig(lig, keep, True)
    x = keep(np.asarray(xyz).reshape(-1, 3), np.float64)
    Pp = keep(P, np.float64)
    qq = keep(q, np.float64)
    out = np.zeros_like(x)
    lib.oracle_pose_map(ctypes.byref(L), _p(x), _p(Pp), _p(qq), _p(out))
    return out


REFINE_DEFAULTS = dict(steps=50, eta_t=1e-2, eta_w=1e-3, eta_th=1e-3, clip_t=0.1, clip_w=0.05, clip_th=0.1)


def refine(lig, pocket, xyz, P, bits=32, fp64_input=False, clash2=None, **kw):
    """Refine one pose; returns (best_score, best_xyz [N,3], accepted_steps)."""
    lib = _load()
    keep = _Keep()
    g = _grid(pocket, keep)
    L = _lig(lig, keep, fp64_input)
    x = keep(np.asarray(xyz).reshape(-1, 3), np.float64)
    L.xyz = _p(x)
    Pp = keep(P, np.float64)
    prm = dict(REFINE_DEFAULTS, **kw)
    arr = keep(np.array([prm["steps"], prm["eta_t"], prm["eta_w"], prm["eta_th"], prm["clip_t"], prm["clip_w"],
                         prm["clip_th"], CLASH2 if clash2 is None else clash2], np.float64), np.float64)
    out = np.zeros_like(x)
    acc = ctypes.c_int(0)
    s = lib.oracle_refine(ctypes.c_int(bits), ctypes.byref(g), ctypes.byref(L), _p(Pp), _p(arr), _p(out),
                          ctypes.byref(acc))
    return s, out, acc.value


def apply_move(lig, xyz, P, q, bits=64, fp64_input=True):
    """The refinement's local move q = (t, omega, theta) applied at (xyz, P)."""
    lib = _load()
    keep = _Keep()
    L = _lig(lig, keep, fp64_input)
    x = keep(np.asarray(xyz).reshape(-1, 3), np.float64)
    Pp = keep(P, np.float64)
    qq = keep(q, np.float64)
    out = np.zeros_like(x)
    Po = np.zeros(3)
    lib.oracle_apply_move(ctypes.c_int(bits), ctypes.byref(L), _p(x), _p(Pp), _p(qq), _p(out), _p(Po))
    return out, Po


def move_grad(lig, pocket, xyz, P, bits=64, fp64_input=True):
    lib = _load()
    keep = _Keep()
    g = _grid(pocket, keep)
    L = _lig(lig, keep, fp64_input)
    x = keep(np.asarray(xyz).reshape(-1, 3), np.float64)
    Pp = keep(P, np.float64)
    gr = np.zeros(6 + L.K)
    s = lib.oracle_move_grad(ctypes.c_int(bits), ctypes.byref(g), ctypes.byref(L), _p(x), _p(Pp), _p(gr))
    return s, gr


def move_clash_free(lig, xyz, bits=64, fp64_input=True, clash2=None):
    lib = _load()
    keep = _Keep()
    L = _lig(lig, keep, fp64_input)
    x = keep(np.asarray(xyz).reshape(-1, 3), np.float64)
    return bool(lib.oracle_move_clash_free(ctypes.c_int(bits), ctypes.byref(L), _p(x),
                                           ctypes.c_double(CLASH2 if clash2 is None else clash2)))


def topk(scores, k):
    lib = _load()
    s = np.ascontiguousarray(scores, np.float64)
    out = np.zeros(min(k, len(s)), np.int32)
    lib.oracle_topk(ctypes.c_int(len(s)), _p(s), ctypes.c_int(k), _p(out))
    return out


def rank(scores, group_size, top_m):
    """Global ranking of a library (Sec. 2: rank the chemical library by the
    docked ligands' scores): each ligand's value is the best of its group_size
    consecutive scores (first member on equal values); ligands by value
    descending, equal values by lower ligand id.  Returns (ids, values, members)
    of the first top_m."""
    s = np.asarray(scores, np.float64).reshape(-1, group_size)
    member = np.argmax(s, axis=1)
    best = s[np.arange(len(s)), member]
    order = np.lexsort((np.arange(len(best)), -best))[:top_m]
    return order.astype(np.int32), best[order], member[order].astype(np.int32)


def trans_step(T: int, halfwidth: float = 2.0) -> float:
    """delta = 2W/T as the FP32 value both sides receive."""
    return float(np.float32(2.0 * halfwidth / T))


CLASH2 = float(np.float32(4.84))   # (2.2 A)^2 as an FP32 value
