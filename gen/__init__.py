"""Seeded synthetic inputs for the docking hot path (pocket grid, ligands,
restart table, angle table).

This package only *builds inputs*; it holds none of the docking method's
arithmetic.  The GPU library and the CPU oracle both consume what it returns,
and neither of them is imported here.  The heavy lifting is in ``gen.cpp``
(compiled with g++ into ``libgen.so``); this file marshals numpy arrays.

Workload recipes (sizes, distributions) stand in for the paper's unpublished
ligand library: mixed ligands whose cost follows atom and rotamer counts
(Sec. 3 and the mixed-dataset experiment of Sec. 5.3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.cpp")
_LIB = os.path.join(_HERE, "libgen.so")
_lib = None


def build() -> str:
    """Compile gen.cpp into libgen.so (host code only)."""
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-ffp-contract=off",
           _SRC, "-o", _LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------- pocket
@dataclass
class Pocket:
    grid: np.ndarray          # float32 [nz, ny, nx], x fastest
    origin: np.ndarray        # float32 [3], position of node (0,0,0)
    spacing: float            # float32 value, Angstrom
    center: np.ndarray        # float32 [3]
    out_value: float = 0.0

    @property
    def n(self):
        return self.grid.shape[::-1]   # (nx, ny, nz)

    @property
    def inv_spacing(self) -> float:
        return float(np.float32(1.0) / np.float32(self.spacing))


DEFAULT_CENTER = (10.0, -4.0, 6.5)


def pocket(n: int, spacing: float, n_gauss: int, n_shell: int, seed: int = 0,
           center=DEFAULT_CENTER) -> Pocket:
    lib = _load()
    grid = np.empty((n, n, n), np.float32)
    origin = np.empty(3, np.float32)
    c = np.asarray(center, np.float64)
    rc = lib.gen_pocket(ctypes.c_int(n), ctypes.c_double(spacing), ctypes.c_int(n_gauss),
                        ctypes.c_int(n_shell), ctypes.c_uint64(seed), _p(c), _p(grid), _p(origin))
    if rc != 0:
        raise ValueError("gen_pocket failed")
    return Pocket(grid, origin, float(np.float32(spacing)), c.astype(np.float32))


# -------------------------------------------------------------------- ligands
@dataclass
class Ligands:
    ids: np.ndarray            # int64 [n] item ids
    n_atoms: np.ndarray        # int32 [n]
    n_tors: np.ndarray         # int32 [n] realised rotatable bonds
    atom_offset: np.ndarray    # int32 [n+1]
    tors_offset: np.ndarray    # int32 [n+1]
    x: np.ndarray              # float32 [total_atoms] input conformation
    y: np.ndarray
    z: np.ndarray
    xyz64: np.ndarray          # float64 [total_atoms, 3] (pre-rounding geometry)
    parent: np.ndarray         # int32 [total_atoms], local ids, -1 = root
    frag_mask: np.ndarray      # uint32 [total_atoms], bit k = moves with bond k
    tors_atoms: np.ndarray     # int32 [2*total_tors] (a_k, b_k) local ids
    inv_bond_len: np.ndarray   # float32 [total_tors], FP64 1/|x_b-x_a| of the FP32 input
    inv_bond_len64: np.ndarray
    ref_point: np.ndarray      # float32 [3n], FP64 centroid of the FP32 input, rounded
    ref_point64: np.ndarray

    @property
    def n(self) -> int:
        return int(self.n_atoms.shape[0])

    def ligand(self, i: int) -> dict:
        """Per-ligand view (local ids), for tests and the oracle."""
        a0, a1 = int(self.atom_offset[i]), int(self.atom_offset[i + 1])
        t0, t1 = int(self.tors_offset[i]), int(self.tors_offset[i + 1])
        return dict(
            N=a1 - a0, K=t1 - t0,
            xyz=np.stack([self.x[a0:a1], self.y[a0:a1], self.z[a0:a1]], 1).astype(np.float64),
            xyz64=self.xyz64[a0:a1],
            parent=self.parent[a0:a1], frag_mask=self.frag_mask[a0:a1],
            tors_a=self.tors_atoms[2 * t0:2 * t1:2], tors_b=self.tors_atoms[2 * t0 + 1:2 * t1:2],
            inv_len=self.inv_bond_len[t0:t1].astype(np.float64),
            inv_len64=self.inv_bond_len64[t0:t1],
            ref=self.ref_point[3 * i:3 * i + 3].astype(np.float64),
            ref64=self.ref_point64[3 * i:3 * i + 3],
        )

    def subset(self, idx) -> "Ligands":
        idx = np.asarray(idx, np.int64)
        parts = [self.ligand_arrays(int(i)) for i in idx]
        return _assemble(self.ids[idx], parts)

    def ligand_arrays(self, i):
        a0, a1 = int(self.atom_offset[i]), int(self.atom_offset[i + 1])
        t0, t1 = int(self.tors_offset[i]), int(self.tors_offset[i + 1])
        return dict(x=self.x[a0:a1], y=self.y[a0:a1], z=self.z[a0:a1], xyz64=self.xyz64[a0:a1],
                    parent=self.parent[a0:a1], frag_mask=self.frag_mask[a0:a1],
                    tors_atoms=self.tors_atoms[2 * t0:2 * t1],
                    inv_bond_len=self.inv_bond_len[t0:t1], inv_bond_len64=self.inv_bond_len64[t0:t1],
                    ref_point=self.ref_point[3 * i:3 * i + 3], ref_point64=self.ref_point64[3 * i:3 * i + 3])


def _assemble(ids, parts) -> Ligands:
    n_atoms = np.array([len(p["x"]) for p in parts], np.int32)
    n_tors = np.array([len(p["inv_bond_len"]) for p in parts], np.int32)
    ao = np.zeros(len(parts) + 1, np.int32); ao[1:] = np.cumsum(n_atoms)
    to = np.zeros(len(parts) + 1, np.int32); to[1:] = np.cumsum(n_tors)
    cat = lambda k, dt: (np.concatenate([p[k] for p in parts]).astype(dt) if parts else np.zeros(0, dt))
    xyz64 = np.concatenate([p["xyz64"] for p in parts]) if parts else np.zeros((0, 3))
    return Ligands(np.asarray(ids, np.int64), n_atoms, n_tors, ao, to,
                   cat("x", np.float32), cat("y", np.float32), cat("z", np.float32), xyz64,
                   cat("parent", np.int32), cat("frag_mask", np.uint32), cat("tors_atoms", np.int32),
                   cat("inv_bond_len", np.float32), cat("inv_bond_len64", np.float64),
                   cat("ref_point", np.float32), cat("ref_point64", np.float64))


def ligand_sizes(ids, seed: int, mode: int, nlo: int, nhi: int, klo: int, khi: int,
                 median: float = 38.0):
    lib = _load()
    ids = np.ascontiguousarray(ids, np.int64)
    n = np.empty(len(ids), np.int32)
    k = np.empty(len(ids), np.int32)
    lib.gen_ligand_sizes(ctypes.c_int(len(ids)), _p(ids), ctypes.c_uint64(seed), ctypes.c_int(mode),
                         ctypes.c_int(nlo), ctypes.c_int(nhi), ctypes.c_int(klo), ctypes.c_int(khi),
                         ctypes.c_double(median), _p(n), _p(k))
    return n, k


def ligands_from_sizes(ids, seed: int, n_req, k_req) -> Ligands:
    lib = _load()
    ids = np.ascontiguousarray(ids, np.int64)
    n_req = np.ascontiguousarray(n_req, np.int32)
    k_req = np.ascontiguousarray(k_req, np.int32)
    cnt = len(ids)
    ao64 = np.zeros(cnt + 1, np.int64); ao64[1:] = np.cumsum(n_req)
    bo64 = np.zeros(cnt + 1, np.int64); bo64[1:] = np.cumsum(k_req)
    TA, TB = int(ao64[-1]), int(bo64[-1])
    xyz64 = np.empty((TA, 3), np.float64)
    parent = np.empty(TA, np.int32)
    mask = np.empty(TA, np.uint32)
    ta = np.zeros(max(TB, 1), np.int32)
    tb = np.zeros(max(TB, 1), np.int32)
    kout = np.empty(cnt, np.int32)

    def run(lo, hi):
        # offsets are absolute, so every chunk writes into the shared output arrays
        return lib.gen_ligands(ctypes.c_int(hi - lo), _p(ids[lo:hi]), ctypes.c_uint64(seed), _p(n_req[lo:hi]),
                               _p(k_req[lo:hi]), _p(ao64[lo:hi]), _p(bo64[lo:hi]), _p(xyz64), _p(parent), _p(mask),
                               _p(ta), _p(tb), _p(kout[lo:hi]))

    nthreads = max(1, min(16, os.cpu_count() or 1, cnt // 256))
    bounds = np.linspace(0, cnt, nthreads + 1).astype(int)
    with ThreadPoolExecutor(nthreads) as ex:
        rcs = list(ex.map(lambda b: run(b[0], b[1]), zip(bounds[:-1], bounds[1:])))
    if any(rc != 0 for rc in rcs):
        raise RuntimeError(f"gen_ligands failed ({rcs})")
    # compact bonds to the realised counts
    keep = np.zeros(max(TB, 1), bool)
    for_idx = np.repeat(np.arange(cnt), k_req)
    pos_in = np.arange(TB) - bo64[:-1][for_idx] if TB else np.zeros(0, np.int64)
    keep[:TB] = pos_in < kout[for_idx] if TB else keep[:0]
    ta_c, tb_c = ta[:TB][keep[:TB]], tb[:TB][keep[:TB]]
    tors_atoms = np.empty(2 * len(ta_c), np.int32)
    tors_atoms[0::2] = ta_c
    tors_atoms[1::2] = tb_c
    x32 = xyz64.astype(np.float32)
    ao = ao64.astype(np.int32)
    to = np.zeros(cnt + 1, np.int32); to[1:] = np.cumsum(kout)
    # Derived inputs.  FP32 side: pivot = FP64 centroid of the FP32 conformation, and
    # 1/bond length in FP64 from the FP32 conformation, both rounded to FP32.  FP64 side:
    # the same quantities of the FP64 conformation (used by FP64 invariants and FD checks).
    lig_of_atom = np.repeat(np.arange(cnt), n_req)
    lig_of_bond = np.repeat(np.arange(cnt), kout)
    abs_a = ao64[:-1][lig_of_bond] + ta_c
    abs_b = ao64[:-1][lig_of_bond] + tb_c

    def centroid_and_inv(xf):
        sums = np.zeros((cnt, 3))
        np.add.at(sums, lig_of_atom, xf)
        d = xf[abs_b] - xf[abs_a]
        inv = 1.0 / np.sqrt((d * d).sum(1)) if len(d) else np.zeros(0)
        return sums / n_req[:, None], inv

    ref_f, inv_f = centroid_and_inv(x32.astype(np.float64))
    ref64, inv64 = centroid_and_inv(xyz64)
    return Ligands(ids, n_req.copy(), kout, ao, to,
                   np.ascontiguousarray(x32[:, 0]), np.ascontiguousarray(x32[:, 1]),
                   np.ascontiguousarray(x32[:, 2]), xyz64, parent, mask, tors_atoms,
                   inv_f.astype(np.float32), inv64, ref_f.astype(np.float32).reshape(-1), ref64.reshape(-1))


def replica_ligand(N: int, seed: int = 0) -> Ligands:
    """The one ligand of N atoms (round(0.18 N) rotatable bonds) that the
    batch-size experiment replicates (the paper replicates three ligands of 17,
    53 and 99 atoms); its generator item id is 9_000_000 + N."""
    return ligands_from_sizes(np.array([9_000_000 + N]), seed, np.array([N]), np.array([int(round(0.18 * N))]))


def replicas(L1: Ligands, count: int) -> Ligands:
    """count copies of the single ligand of L1, as one batch."""
    N, K = int(L1.n_atoms[0]), int(L1.n_tors[0])
    tile = lambda a: np.tile(np.asarray(a), count)
    ao = np.arange(count + 1, dtype=np.int32) * N
    to = np.arange(count + 1, dtype=np.int32) * K
    return Ligands(np.full(count, L1.ids[0]), np.full(count, N, np.int32), np.full(count, K, np.int32), ao, to,
                   tile(L1.x), tile(L1.y), tile(L1.z), np.tile(L1.xyz64, (count, 1)), tile(L1.parent),
                   tile(L1.frag_mask), tile(L1.tors_atoms), tile(L1.inv_bond_len), tile(L1.inv_bond_len64),
                   tile(L1.ref_point), tile(L1.ref_point64))


# ------------------------------------------------------------------- tables
def restarts(R: int, seed: int = 0, radius: float = 2.0):
    """[R,12] restart table: row-major rotation then offset; row 0 identity."""
    lib = _load()
    o64 = np.empty((R, 12), np.float64)
    o32 = np.empty((R, 12), np.float32)
    lib.gen_restarts(ctypes.c_int(R), ctypes.c_uint64(seed), ctypes.c_double(radius), _p(o64), _p(o32))
    return o32, o64


def angles(A: int):
    """[A,2] (cos, sin) of 2*pi*j/A, FP32 and FP64."""
    lib = _load()
    o64 = np.empty((A, 2), np.float64)
    o32 = np.empty((A, 2), np.float32)
    lib.gen_angles(ctypes.c_int(A), _p(o64), _p(o32))
    return o32, o64


def uniform(count: int, dim: int, seed: int, stream: int, scale: float):
    lib = _load()
    out = np.empty((count, dim), np.float64)
    lib.gen_uniform(ctypes.c_int64(count), ctypes.c_int(dim), ctypes.c_uint64(seed),
                    ctypes.c_uint64(stream), ctypes.c_double(scale), _p(out))
    return out


# ------------------------------------------------------------------ workloads
@dataclass
class Workload:
    name: str
    n_ligands: int
    size_mode: int             # 0 uniform ranges, 1 lognormal
    nlo: int
    nhi: int
    klo: int
    khi: int
    grid_n: int
    spacing: float
    n_gauss: int
    n_shell: int
    restarts: int
    angle_samples: int
    sweeps: int
    top_k: int
    seed: int = 0
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    # 64 ligands, atoms U[20,40], bonds U[2,6]; 32^3 @ 0.5 A, 40 Gaussians, 300 shell atoms
    "tiny": Workload("tiny", 64, 0, 20, 40, 2, 6, 32, 0.5, 40, 300, 32, 64, 2, 32),
    # 10k ligands, 48 atoms, 8 bonds; 96^3 @ 0.375 A, 200 Gaussians, 2000 shell atoms
    "uniform": Workload("uniform", 10_000, 0, 48, 48, 8, 8, 96, 0.375, 200, 2000, 256, 256, 3, 10),
    # 100k ligands, lognormal atoms (median 38, [12,120]), bonds round(0.18N+N(0,2)) in [0,24]
    "mixed": Workload("mixed", 100_000, 1, 12, 120, 0, 24, 96, 0.375, 200, 2000, 256, 256, 3, 10),
    # 1M ligands, atoms up to 160, bonds up to 32; 128^3 @ 0.375 A
    "screen": Workload("screen", 1_000_000, 1, 12, 160, 0, 32, 128, 0.375, 200, 2000, 256, 256, 3, 8),
}


def workload_ligands(w: Workload, ids=None) -> Ligands:
    if ids is None:
        ids = np.arange(w.n_ligands, dtype=np.int64)
    n, k = ligand_sizes(ids, w.seed, w.size_mode, w.nlo, w.nhi, w.klo, w.khi)
    return ligands_from_sizes(ids, w.seed, n, k)


def workload_pocket(w: Workload) -> Pocket:
    return pocket(w.grid_n, w.spacing, w.n_gauss, w.n_shell, w.seed)
