"""Thin Python binding of the docking library's C ABI (include/lg.h).

Argument marshalling only: every step of the docking path runs in the HIP
kernels of ``liblg.so``.  PyTorch provides device memory and streams.  If the
library cannot be loaded this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblg.so")

LG_OK = 0
LG_ERR_INVALID_ARG = -1
LG_ERR_LIMIT = -2
LG_ERR_OUT_OF_MEMORY = -3
LG_ERR_DEVICE = -4
LG_ERR_UNSUPPORTED = -5
LG_NEAREST, LG_TRILINEAR = 0, 1
LG_PLAIN, LG_BUCKETED = 0, 1
LG_MAX_ATOMS, LG_MAX_TORSIONS, LG_MAX_SAMPLES = 256, 32, 1024

EXPORTS = ("lg_load_pocket", "lg_free_pocket", "lg_dock_batch", "lg_dock_sites", "lg_dock_stream", "lg_score",
           "lg_refine", "lg_rank", "lg_rank_static", "lg_autotune", "lg_valu_probe",
           "lg_set_tuning", "lg_get_tuning", "lg_bucket_stats", "lg_bucket_size", "lg_atom_clusters", "lg_rotamer_clusters",
           "lg_last_error", "lg_version")


class LgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lg status {status}: {msg}")
        self.status = status


c_int32, c_float, c_void_p = ctypes.c_int32, ctypes.c_float, ctypes.c_void_p


class lg_pocket_desc(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("spacing", c_float),
                ("inv_spacing", c_float), ("origin", c_float * 3), ("center", c_float * 3),
                ("out_value", c_float)]


class lg_ligands(ctypes.Structure):
    _fields_ = [("n", c_int32), ("total_atoms", c_int32), ("total_torsions", c_int32),
                ("atom_offset", c_void_p), ("tors_offset", c_void_p), ("x", c_void_p), ("y", c_void_p),
                ("z", c_void_p), ("frag_mask", c_void_p), ("tors_atoms", c_void_p),
                ("inv_bond_len", c_void_p), ("ref_point", c_void_p), ("atom_offset_host", c_void_p),
                ("tors_offset_host", c_void_p), ("tors_atoms_host", c_void_p)]


class lg_dock_params(ctypes.Structure):
    _fields_ = [("restarts", c_int32), ("angle_samples", c_int32), ("trans_samples", c_int32),
                ("sweeps", c_int32), ("top_k", c_int32), ("mode", c_int32), ("trans_step", c_float),
                ("clash_dist2", c_float), ("restart_table", c_void_p), ("angle_table", c_void_p)]


class lg_dock_out(ctypes.Structure):
    _fields_ = [("score", c_void_p), ("restart_id", c_void_p), ("x", c_void_p), ("y", c_void_p),
                ("z", c_void_p), ("all_scores", c_void_p), ("trace", c_void_p), ("trace_kmax", c_int32),
                ("pivot", c_void_p)]


class lg_host_ligands(ctypes.Structure):
    _fields_ = [("n", c_int32), ("total_atoms", c_int32), ("total_torsions", c_int32),
                ("atom_offset", c_void_p), ("tors_offset", c_void_p), ("x", c_void_p), ("y", c_void_p),
                ("z", c_void_p), ("frag_mask", c_void_p), ("tors_atoms", c_void_p),
                ("inv_bond_len", c_void_p), ("ref_point", c_void_p)]


class lg_host_out(ctypes.Structure):
    _fields_ = [("score", c_void_p), ("restart_id", c_void_p), ("x", c_void_p), ("y", c_void_p),
                ("z", c_void_p), ("pivot", c_void_p), ("chunk_done", c_void_p)]


class lg_refine_params(ctypes.Structure):
    _fields_ = [("steps", c_int32), ("eta_t", c_float), ("eta_w", c_float), ("eta_th", c_float),
                ("clip_t", c_float), ("clip_w", c_float), ("clip_th", c_float), ("clash_dist2", c_float),
                ("poses_per_ligand", c_int32)]


class lg_tuning(ctypes.Structure):
    _fields_ = [("n_atom_clusters", c_int32), ("atom_bounds", c_int32 * 16), ("n_rot_clusters", c_int32),
                ("rot_bounds", c_int32 * 32), ("waves_per_block", c_int32 * 4), ("restart_chunk", c_int32),
                ("grid_scale", c_int32), ("plain_waves_per_block", c_int32), ("use_graph", c_int32),
                ("lazy_clash", c_int32)]


class lg_bucket_stat(ctypes.Structure):
    _fields_ = [("bucket", c_int32), ("atom_bound", c_int32), ("rot_bound", c_int32), ("slots", c_int32),
                ("samples_per_lane", c_int32), ("waves_per_block", c_int32), ("vgprs", c_int32),
                ("lds_bytes", c_int32), ("blocks_per_cu", c_int32), ("blocks", c_int32), ("ligands", c_int32),
                ("ms", c_float), ("span_ms", c_float)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblg.so (building it first if it is absent).  Raises on failure."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.lg_load_pocket.argtypes = [P(lg_pocket_desc), c_void_p, c_int32, c_void_p, P(c_void_p)]
    lib.lg_free_pocket.argtypes = [c_void_p]
    lib.lg_dock_batch.argtypes = [c_void_p, P(lg_ligands), P(lg_dock_params), P(lg_dock_out), c_void_p]
    lib.lg_dock_sites.argtypes = [P(c_void_p), c_int32, P(lg_ligands), P(lg_dock_params), P(lg_dock_out), c_int32,
                                  c_void_p]
    lib.lg_dock_stream.argtypes = [c_void_p, P(lg_host_ligands), P(lg_dock_params), c_int32, P(lg_host_out),
                                   c_void_p]
    lib.lg_score.argtypes = [c_void_p, P(lg_ligands), c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                             c_void_p, c_void_p]
    lib.lg_refine.argtypes = [c_void_p, P(lg_ligands), P(lg_refine_params), c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p]
    lib.lg_rank.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.lg_rank_static.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.lg_autotune.argtypes = [c_void_p, P(lg_ligands), P(lg_dock_params), c_int32, P(lg_tuning),
                                P(c_float), c_void_p]
    lib.lg_valu_probe.argtypes = [c_void_p, c_int32, c_int32, P(ctypes.c_double), c_void_p]
    lib.lg_set_tuning.argtypes = [c_void_p, P(lg_tuning)]
    lib.lg_get_tuning.argtypes = [c_void_p, P(lg_tuning)]
    lib.lg_bucket_stats.argtypes = [c_void_p, P(lg_bucket_stat), c_int32]
    lib.lg_bucket_stats.restype = c_int32
    lib.lg_bucket_size.argtypes = [ctypes.c_int64] * 4
    lib.lg_bucket_size.restype = ctypes.c_int64
    lib.lg_atom_clusters.argtypes = [c_int32, c_int32, c_int32, P(c_int32)]
    lib.lg_rotamer_clusters.argtypes = [c_int32, c_int32, P(c_int32)]
    lib.lg_last_error.restype = ctypes.c_char_p
    for name in ("lg_load_pocket", "lg_free_pocket", "lg_dock_batch", "lg_dock_sites", "lg_dock_stream", "lg_score",
                 "lg_refine", "lg_rank", "lg_rank_static", "lg_autotune", "lg_valu_probe", "lg_set_tuning",
                 "lg_get_tuning"):
        getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def _check(status):
    if status != LG_OK:
        raise LgError(status, _lib.lg_last_error().decode())


# ----------------------------------------------------------------- host-only calls
def lg_bucket_size(blocks_per_unit: int, units: int, threads_per_block: int, wave_size: int) -> int:
    return int(load_library().lg_bucket_size(blocks_per_unit, units, threads_per_block, wave_size))


def lg_atom_clusters(n_clusters: int, wave_size: int, max_atoms: int):
    b = (c_int32 * max(n_clusters, 1))()
    n = load_library().lg_atom_clusters(n_clusters, wave_size, max_atoms, b)
    return [b[i] for i in range(n)]


def lg_rotamer_clusters(n_clusters: int, max_rot: int):
    b = (c_int32 * max(n_clusters, 1))()
    n = load_library().lg_rotamer_clusters(n_clusters, max_rot, b)
    return [b[i] for i in range(n)]


def lg_version() -> int:
    return int(load_library().lg_version())


def lg_last_error() -> str:
    return load_library().lg_last_error().decode()


# ----------------------------------------------------------------- device data
def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class DeviceLigands:
    """A batch of ligands (or poses) in device memory, as lg_ligands expects."""
    n: int
    atom_offset: object
    tors_offset: object
    x: object
    y: object
    z: object
    frag_mask: object
    tors_atoms: object
    inv_bond_len: object
    ref_point: object
    atom_offset_host: np.ndarray
    tors_offset_host: np.ndarray
    tors_atoms_host: np.ndarray | None = None
    host_checks: bool = True   # pass the host copies (checked on the host, no read-back)

    @property
    def total_atoms(self) -> int:
        return int(self.atom_offset_host[-1])

    @property
    def total_torsions(self) -> int:
        return int(self.tors_offset_host[-1])

    def struct(self) -> lg_ligands:
        host = self.host_checks
        tah = self.tors_atoms_host if host else None
        return lg_ligands(self.n, self.total_atoms, self.total_torsions, _ptr(self.atom_offset),
                          _ptr(self.tors_offset), _ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.frag_mask),
                          _ptr(self.tors_atoms), _ptr(self.inv_bond_len), _ptr(self.ref_point),
                          self.atom_offset_host.ctypes.data_as(c_void_p) if host else None,
                          self.tors_offset_host.ctypes.data_as(c_void_p) if host else None,
                          tah.ctypes.data_as(c_void_p) if tah is not None else None)


def device_ligands(atom_offset, tors_offset, x, y, z, frag_mask, tors_atoms, inv_bond_len, ref_point,
                   device="cuda") -> DeviceLigands:
    """Copy host arrays (numpy) of a ligand batch to device memory."""
    torch = _torch()

    def dev(a, dt):
        a = np.ascontiguousarray(a, dt)
        if a.size == 0:
            a = np.zeros(1, dt)
        return torch.from_numpy(a.view(np.int32) if dt == np.uint32 else a).to(device)

    ao = np.ascontiguousarray(atom_offset, np.int32)
    to = np.ascontiguousarray(tors_offset, np.int32)
    ta = np.ascontiguousarray(tors_atoms, np.int32).reshape(-1)
    return DeviceLigands(len(ao) - 1, dev(ao, np.int32), dev(to, np.int32), dev(x, np.float32), dev(y, np.float32),
                         dev(z, np.float32), dev(frag_mask, np.uint32), dev(ta, np.int32),
                         dev(inv_bond_len, np.float32), dev(ref_point, np.float32), ao, to, ta)


# ----------------------------------------------------------------- pocket handle
class Pocket:
    """lg_load_pocket / lg_free_pocket around a library-owned grid copy."""

    def __init__(self, grid, origin, spacing, center, out_value=0.0, inv_spacing=None, stream=None):
        torch = _torch()
        lib = load_library()
        g = grid if isinstance(grid, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(grid, np.float32))
        g = g.contiguous()
        nz, ny, nx = g.shape
        inv = float(np.float32(1.0) / np.float32(spacing)) if inv_spacing is None else inv_spacing
        self.desc = lg_pocket_desc(nx, ny, nz, float(spacing), inv, (c_float * 3)(*map(float, origin)),
                                   (c_float * 3)(*map(float, center)), float(out_value))
        handle = c_void_p()
        on_dev = 1 if g.is_cuda else 0
        _check(lib.lg_load_pocket(ctypes.byref(self.desc), c_void_p(g.data_ptr()), on_dev,
                                  _stream_handle(stream), ctypes.byref(handle)))
        self.handle = handle
        self.shape = (nx, ny, nz)

    def free(self):
        if getattr(self, "handle", None) and self.handle.value:
            _check(_lib.lg_free_pocket(self.handle))
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def set_tuning(self, tuning: lg_tuning):
        _check(_lib.lg_set_tuning(self.handle, ctypes.byref(tuning)))

    def bucket_stats(self) -> list:
        """lg_bucket_stats of the last bucketed call, as dicts."""
        cap = 512
        buf = (lg_bucket_stat * cap)()
        n = _lib.lg_bucket_stats(self.handle, buf, cap)
        if n < 0:
            _check(n)
        return [{f: getattr(buf[i], f) for f, _ in lg_bucket_stat._fields_} for i in range(min(n, cap))]

    def get_tuning(self) -> lg_tuning:
        t = lg_tuning()
        _check(_lib.lg_get_tuning(self.handle, ctypes.byref(t)))
        return t


def lg_dock_batch(pocket: Pocket, ligs: DeviceLigands, restart_table, angle_table, *, sweeps: int, top_k: int,
                  trans_samples: int, trans_step: float, clash_dist2: float, mode: int = LG_BUCKETED,
                  out: dict | None = None, want_all_scores=False, trace_kmax: int | None = None, stream=None):
    """Dock a batch.  Returns a dict of device tensors: score [n,k], restart_id [n,k],
    x/y/z [k*total_atoms], pivot [n,k,3], and all_scores [n,R] / trace [n,R,S,6+kmax]
    when asked."""
    torch = _torch()
    R, A = int(restart_table.shape[0]), int(angle_table.shape[0])
    n, TA, dev = ligs.n, ligs.total_atoms, ligs.x.device
    if out is None:
        out = dict(score=torch.empty((n, top_k), dtype=torch.float32, device=dev),
                   restart_id=torch.empty((n, top_k), dtype=torch.int32, device=dev),
                   x=torch.empty(top_k * TA, dtype=torch.float32, device=dev),
                   y=torch.empty(top_k * TA, dtype=torch.float32, device=dev),
                   z=torch.empty(top_k * TA, dtype=torch.float32, device=dev),
                   pivot=torch.empty((n, top_k, 3), dtype=torch.float32, device=dev))
        if want_all_scores:
            out["all_scores"] = torch.empty((n, R), dtype=torch.float32, device=dev)
        if trace_kmax is not None:
            out["trace"] = torch.full((n, R, sweeps, 6 + trace_kmax), -1, dtype=torch.int16, device=dev)
    params = lg_dock_params(R, A, int(trans_samples), int(sweeps), int(top_k), int(mode), float(trans_step),
                            float(clash_dist2), _ptr(restart_table), _ptr(angle_table))
    o = lg_dock_out(_ptr(out["score"]), _ptr(out["restart_id"]), _ptr(out["x"]), _ptr(out["y"]), _ptr(out["z"]),
                    _ptr(out.get("all_scores")), _ptr(out.get("trace")),
                    int(trace_kmax) if out.get("trace") is not None else 0, _ptr(out.get("pivot")))
    L = ligs.struct()
    _check(_lib.lg_dock_batch(pocket.handle, ctypes.byref(L), ctypes.byref(params), ctypes.byref(o),
                              _stream_handle(stream)))
    return out


def lg_dock_sites(pockets, ligs: DeviceLigands, restart_table, angle_table, *, sweeps: int, top_k: int,
                  trans_samples: int, trans_step: float, clash_dist2: float, site_major: bool = True,
                  want_all_scores=False, stream=None):
    """Dock a batch into every site of `pockets` (same grid dimensions and
    spacing) in one call.  Returns one dict per site, as lg_dock_batch."""
    torch = _torch()
    R, A = int(restart_table.shape[0]), int(angle_table.shape[0])
    n, TA, dev = ligs.n, ligs.total_atoms, ligs.x.device
    outs = []
    for _ in pockets:
        o = dict(score=torch.empty((n, top_k), dtype=torch.float32, device=dev),
                 restart_id=torch.empty((n, top_k), dtype=torch.int32, device=dev),
                 x=torch.empty(top_k * TA, dtype=torch.float32, device=dev),
                 y=torch.empty(top_k * TA, dtype=torch.float32, device=dev),
                 z=torch.empty(top_k * TA, dtype=torch.float32, device=dev),
                 pivot=torch.empty((n, top_k, 3), dtype=torch.float32, device=dev))
        if want_all_scores:
            o["all_scores"] = torch.empty((n, R), dtype=torch.float32, device=dev)
        outs.append(o)
    params = lg_dock_params(R, A, int(trans_samples), int(sweeps), int(top_k), LG_BUCKETED, float(trans_step),
                            float(clash_dist2), _ptr(restart_table), _ptr(angle_table))
    O = (lg_dock_out * len(pockets))(*[
        lg_dock_out(_ptr(o["score"]), _ptr(o["restart_id"]), _ptr(o["x"]), _ptr(o["y"]), _ptr(o["z"]),
                    _ptr(o.get("all_scores")), None, 0, _ptr(o["pivot"])) for o in outs])
    H = (c_void_p * len(pockets))(*[p.handle.value for p in pockets])
    L = ligs.struct()
    _check(_lib.lg_dock_sites(H, len(pockets), ctypes.byref(L), ctypes.byref(params), O, int(bool(site_major)),
                              _stream_handle(stream)))
    return outs


def lg_dock_stream(pocket: Pocket, atom_offset, tors_offset, x, y, z, frag_mask, tors_atoms, inv_bond_len,
                   ref_point, restart_table, angle_table, *, sweeps: int, top_k: int, trans_samples: int,
                   trans_step: float, clash_dist2: float, chunk: int, want_pivot: bool = True, out=None,
                   chunk_done=None, stream=None):
    """Dock a library held in host memory (numpy arrays), streamed through the
    device in chunks.  Returns numpy arrays: score [n,k], restart_id [n,k],
    x/y/z [k*total_atoms], pivot [n,k,3] (if asked).  `out` may supply those
    arrays (e.g. memory-mapped files); `chunk_done` (int32 [ceil(n/chunk)]) is
    the resume manifest: chunks marked non-zero are skipped, the others marked
    once their outputs are written."""
    arrs = [np.ascontiguousarray(atom_offset, np.int32), np.ascontiguousarray(tors_offset, np.int32),
            np.ascontiguousarray(x, np.float32), np.ascontiguousarray(y, np.float32),
            np.ascontiguousarray(z, np.float32), np.ascontiguousarray(frag_mask, np.uint32),
            np.ascontiguousarray(tors_atoms, np.int32).reshape(-1), np.ascontiguousarray(inv_bond_len, np.float32),
            np.ascontiguousarray(ref_point, np.float32).reshape(-1)]
    n = len(arrs[0]) - 1
    ta, tt = int(arrs[0][-1]), int(arrs[1][-1])
    ptr = [a.ctypes.data_as(c_void_p) for a in arrs]
    H = lg_host_ligands(n, ta, tt, *ptr)
    R, A = int(restart_table.shape[0]), int(angle_table.shape[0])
    params = lg_dock_params(R, A, int(trans_samples), int(sweeps), int(top_k), LG_BUCKETED, float(trans_step),
                            float(clash_dist2), _ptr(restart_table), _ptr(angle_table))
    if out is None:
        out = dict(score=np.empty((n, top_k), np.float32), restart_id=np.empty((n, top_k), np.int32),
                   x=np.empty(top_k * ta, np.float32), y=np.empty(top_k * ta, np.float32),
                   z=np.empty(top_k * ta, np.float32))
        if want_pivot:
            out["pivot"] = np.empty((n, top_k, 3), np.float32)
    shapes = dict(score=((n, top_k), np.float32), restart_id=((n, top_k), np.int32), x=((top_k * ta,), np.float32),
                  y=((top_k * ta,), np.float32), z=((top_k * ta,), np.float32), pivot=((n, top_k, 3), np.float32))
    for k_, a in out.items():
        if k_ in shapes and (a.shape != shapes[k_][0] or a.dtype != shapes[k_][1] or not a.flags.c_contiguous):
            raise ValueError(f"out[{k_!r}] must be a C-contiguous {np.dtype(shapes[k_][1])} array of shape "
                             f"{shapes[k_][0]}")
    if chunk_done is not None:
        nch = -(-n // int(chunk)) if n else 0
        if chunk_done.shape != (nch,) or chunk_done.dtype != np.int32 or not chunk_done.flags.c_contiguous:
            raise ValueError(f"chunk_done must be a C-contiguous int32 array of shape ({nch},)")
    ptrs = [out[k_].ctypes.data_as(c_void_p) if k_ in out else None
            for k_ in ("score", "restart_id", "x", "y", "z", "pivot")]
    O = lg_host_out(*ptrs, chunk_done.ctypes.data_as(c_void_p) if chunk_done is not None else None)
    _check(_lib.lg_dock_stream(pocket.handle, ctypes.byref(H), ctypes.byref(params), int(chunk), ctypes.byref(O),
                               _stream_handle(stream)))
    return out


def lg_autotune(pocket: Pocket, ligs: DeviceLigands, restart_table, angle_table, *, sweeps: int, top_k: int,
                trans_samples: int, trans_step: float, clash_dist2: float, passes: int = 1, stream=None):
    """Search the bucketed path's tuning on a sample batch; the handle keeps the
    best.  Returns (lg_tuning, best_ms)."""
    R, A = int(restart_table.shape[0]), int(angle_table.shape[0])
    params = lg_dock_params(R, A, int(trans_samples), int(sweeps), int(top_k), LG_BUCKETED, float(trans_step),
                            float(clash_dist2), _ptr(restart_table), _ptr(angle_table))
    t = lg_tuning()
    ms = c_float(0.0)
    L = ligs.struct()
    _check(_lib.lg_autotune(pocket.handle, ctypes.byref(L), ctypes.byref(params), int(passes), ctypes.byref(t),
                            ctypes.byref(ms), _stream_handle(stream)))
    return t, float(ms.value)


def lg_score(pocket: Pocket, poses: DeviceLigands, interp: int = LG_TRILINEAR, grad: bool = False,
             top_m: int = 0, moves=None, stream=None):
    """Score poses (optionally moved by local parameters `moves`, a device tensor of
    6n + total_torsions floats); returns dict(score [n], grad [6n + total_torsions]
    or None, top_idx, top_score)."""
    torch = _torch()
    dev = poses.x.device
    n = poses.n
    res = dict(score=torch.empty(max(n, 1), dtype=torch.float32, device=dev)[:n])
    res["grad"] = torch.empty(max(6 * n + poses.total_torsions, 1), dtype=torch.float32, device=dev) if grad else None
    res["top_idx"] = torch.empty(max(top_m, 1), dtype=torch.int32, device=dev)[:top_m] if top_m else None
    res["top_score"] = torch.empty(max(top_m, 1), dtype=torch.float32, device=dev)[:top_m] if top_m else None
    L = poses.struct()
    _check(_lib.lg_score(pocket.handle, ctypes.byref(L), int(interp), _ptr(moves), _ptr(res["score"]),
                         _ptr(res["grad"]), int(top_m), _ptr(res["top_idx"]), _ptr(res["top_score"]),
                         _stream_handle(stream)))
    return res


def lg_refine(pocket: Pocket, poses: DeviceLigands, params: lg_refine_params, stream=None):
    """Refine poses; with params.poses_per_ligand = k > 1 the coordinates hold k poses
    per ligand (lg_dock_out layout) and ref_point one pivot per pose.  Returns
    dict(x, y, z [k*total_atoms], score [n*k])."""
    torch = _torch()
    dev = poses.x.device
    k = max(int(params.poses_per_ligand), 1)
    TA = k * poses.total_atoms
    out = dict(x=torch.empty(TA, dtype=torch.float32, device=dev), y=torch.empty(TA, dtype=torch.float32, device=dev),
               z=torch.empty(TA, dtype=torch.float32, device=dev),
               score=torch.empty(max(poses.n * k, 1), dtype=torch.float32, device=dev)[:poses.n * k])
    L = poses.struct()
    _check(_lib.lg_refine(pocket.handle, ctypes.byref(L), ctypes.byref(params), _ptr(out["x"]), _ptr(out["y"]),
                          _ptr(out["z"]), _ptr(out["score"]), _stream_handle(stream)))
    return out


def refine_params(steps=50, eta_t=1e-2, eta_w=1e-3, eta_th=1e-3, clip_t=0.1, clip_w=0.05, clip_th=0.1,
                  clash_dist2=4.84, poses_per_ligand=1) -> lg_refine_params:
    return lg_refine_params(int(steps), eta_t, eta_w, eta_th, clip_t, clip_w, clip_th, clash_dist2,
                            int(poses_per_ligand))


VALU_PROBE_KINDS = ("v_fma_f32", "v_add_f32", "v_add_u32", "v_med3_f32", "v_mad_i32_i24", "v_fma_f32+v_add_u32",
                    "scan index mix")


def lg_valu_probe(pocket: Pocket, kind: int = 0, iters: int = 200000, stream=None) -> float:
    """Sustained lane-operations per second of one non-packed VALU operation
    (VALU_PROBE_KINDS[kind]) on the pocket's device."""
    r = ctypes.c_double(0.0)
    _check(_lib.lg_valu_probe(pocket.handle, int(kind), int(iters), ctypes.byref(r), _stream_handle(stream)))
    return float(r.value)


def lg_rank(pocket: Pocket, score, group_size: int, top_m: int, stream=None):
    """Rank ligands by the best of their group_size consecutive scores.  Returns
    dict(top_idx [top_m] ligand ids, top_score [top_m], top_member [top_m])."""
    torch = _torch()
    dev = score.device
    ng = int(score.numel()) // int(group_size)
    res = {k: torch.empty(max(top_m, 1), dtype=dt, device=dev)[:top_m]
           for k, dt in (("top_idx", torch.int32), ("top_score", torch.float32), ("top_member", torch.int32))}
    _check(_lib.lg_rank(pocket.handle, _ptr(score), ng, int(group_size), int(top_m), _ptr(res["top_idx"]),
                        _ptr(res["top_score"]), _ptr(res["top_member"]), _stream_handle(stream)))
    return res


LG_RANK_STATIC_MAX_GROUPS, LG_RANK_STATIC_MAX_TOP = 1 << 20, 4096


def lg_rank_static(score, group_size: int, top_m: int, top_idx, top_score, top_member=None, stream=None) -> None:
    """lg_rank without a pocket and without any allocation (the library's fixed
    device scratch): the caller passes the output tensors (top_idx int32
    [top_m], top_score float32 [top_m], top_member int32 [top_m] or None), all
    on the current device."""
    ng = int(score.numel()) // int(group_size)
    _check(_lib.lg_rank_static(_ptr(score), ng, int(group_size), int(top_m), _ptr(top_idx), _ptr(top_score),
                               _ptr(top_member), _stream_handle(stream)))


def docked_poses(ligs: DeviceLigands, out: dict) -> DeviceLigands:
    """The kept poses of an lg_dock_batch result as refinement input: the ligands'
    topology with the output coordinates and pivots (k poses per ligand)."""
    return DeviceLigands(ligs.n, ligs.atom_offset, ligs.tors_offset, out["x"], out["y"], out["z"], ligs.frag_mask,
                         ligs.tors_atoms, ligs.inv_bond_len, out["pivot"].reshape(-1), ligs.atom_offset_host,
                         ligs.tors_offset_host, ligs.tors_atoms_host, ligs.host_checks)
