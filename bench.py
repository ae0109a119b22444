#!/usr/bin/env python3
"""Benchmark: ligands docked per second at 256 restarts on one MI355X.

Workload (default): the mixed library -- 100,000 ligands, atoms lognormal
(median 38, clipped to [12, 120]), rotatable bonds round(0.18 N + N(0, 2))
clipped to [0, 24]; 96^3 pocket grid at 0.375 A; 256 restarts, 256 angle and
256 translation samples, 3 sweeps, top-10 per ligand.  Synthetic, seeded inputs
(the paper's ligand library is not public), resident in device memory before
the timed region.

A step is one lg_dock_batch call over the whole library in the bucketed
persistent mode (device-side bucketing, one persistent launch per size bucket,
replayed as one HIP graph, per-ligand top-k).  The plain method (one launch
per ligand, largest-class kernel) is timed on a prefix of the same library and
reported beside it, with the single-bucket ablation.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 vector peak of the MI355X, 157.3 TFLOP/s, counted in lane-operations (an
# FMA is one): 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz.  gfx950 issues a wave64
# v_fma_f32 / v_add_f32 / v_mul_f32 with VGPR operands in two cycles (32 lanes per
# cycle per SIMD); integer shift-adds, three-way adds, med3 and float-to-int
# conversions take four.
PEAK_LANE_OPS = 256 * 4 * 32 * 2.4e9
VALU_PROBE_MIX = 6   # lg_valu_probe kind: the nearest-node index sequence of a scan sample

# VALU instructions per lane, per unit of work, in the inner loops of the docking
# scans, counted in the gfx950 assembly of dock_bucket_kernel<1, 4> (four samples
# per lane, loop control included), for the variants a scan takes when every
# sample's node is inside the grid (the usual case): a loop pass of the rotation
# scan handles two atoms x four samples in 91 (the lane's four quarter-turn
# samples share one 2-D rotation), of the staged translation scan one atom x four
# samples in 25 (node values read from LDS; the group gathers that stage them are
# not counted), of the torsion scan two moving atoms x two samples in 132 (the
# per-atom set-up of the clash-pair loop included, the pair tests themselves
# not); each torsion sample's rotation matrix takes 13.  Placement and the final
# trilinear score are counted from the op script (15 and 45 per atom and restart).
ISA_ROT = 91 / 8         # per (rotation sample, atom)
ISA_TRANS = 25 / 4       # per (translation sample, atom)
ISA_TORS = 132 / 4       # per (torsion sample, moving atom)
ISA_TMAT = 13            # per torsion sample
OPS_PLACE = 15           # per atom per restart: placement
OPS_TRI = 45             # per atom per restart: trilinear final score
# The plain method's count: op-script constants per (sample, atom) of a rotation,
# translation and torsion scan with its nearest lookup, and a pair test of every
# (moving, static) atom pair for every torsion sample.
PLAIN_ROT, PLAIN_TRANS, PLAIN_TORS, PLAIN_PAIR = 32, 23, 37, 8


# Refinement, per pose and step (the op script of one step): per atom the trilinear
# value with gradient, its score / force / torque sums and the rigid part of the
# move; per (bond, moving atom) the bond torque and the torsion move; per bond its
# axis, step, matrix and step polynomial; per atom pair whose rigid pieces differ
# the clash test.  The moved pose's score is not counted: it is the value column
# of the next step's gradient pass.  A rejected step leaves the pose, so its
# gradient need not be recomputed; it is still counted here, which makes the
# fraction an upper bound (about 31 % of the steps are rejected on the mixed
# library).
OPS_REF_ATOM = 63 + 19 + 18
OPS_REF_BOND_ATOM = 15 + 15
OPS_REF_BOND = 45
OPS_REF_PAIR = 7


def refine_ops_per_step(L):
    """Lane-ops of one refinement step of one pose, per ligand of L."""
    ops = np.zeros(L.n)
    for i in range(L.n):
        a0, a1 = L.atom_offset[i], L.atom_offset[i + 1]
        m = L.frag_mask[a0:a1]
        N, K = a1 - a0, int(L.n_tors[i])
        moving = sum(int(((m >> k) & 1).sum()) for k in range(K))
        _, cnt = np.unique(m, return_counts=True)
        pairs = N * (N - 1) // 2 - int((cnt * (cnt - 1) // 2).sum())
        ops[i] = N * OPS_REF_ATOM + moving * OPS_REF_BOND_ATOM + K * OPS_REF_BOND + pairs * OPS_REF_PAIR
    return ops


def _per_ligand(n_atoms, frag_sizes_per_lig, fn):
    out = np.zeros(len(n_atoms))
    for i, (N, F) in enumerate(zip(n_atoms, frag_sizes_per_lig)):
        out[i] = fn(float(N), np.asarray(F, np.float64) - 1.0)   # moving atoms of each torsion, axis atom excluded
    return out


def isa_ops(n_atoms, frag_sizes_per_lig, R, A, T, S):
    """VALU lane-ops of docking each ligand: every sample of every scan at the
    inner loops' per-unit instruction counts (a lower bound of what the kernel
    issues: per-scan work and the tests of pairs that can clash are left out)."""
    return _per_ligand(n_atoms, frag_sizes_per_lig, lambda N, mv: R * (
        S * (3 * A * N * ISA_ROT + 3 * T * N * ISA_TRANS + A * mv.sum() * ISA_TORS + len(mv) * A * ISA_TMAT)
        + N * (OPS_PLACE + OPS_TRI)))


def plain_method_ops(n_atoms, frag_sizes_per_lig, R, A, T, S):
    """Lane-ops of the plain method per ligand: op-script constants and a clash
    test of every (moving, static) pair for every torsion sample."""
    return _per_ligand(n_atoms, frag_sizes_per_lig, lambda N, mv: R * (
        S * (3 * A * N * PLAIN_ROT + 3 * T * N * PLAIN_TRANS
             + A * (mv.sum() * PLAIN_TORS + (mv * (N - mv - 2)).sum() * PLAIN_PAIR))
        + N * (OPS_PLACE + OPS_TRI)))


def lookups(n_atoms, frag_sizes_per_lig, R, A, T, S):
    """Grid values read per ligand: one nearest-node value per (sample, moved
    atom) of every scan, the current pose's atoms at each rotation and torsion
    scan, eight per atom for the final trilinear score."""
    return _per_ligand(n_atoms, frag_sizes_per_lig, lambda N, mv: R * (
        S * (3 * A * N + 3 * T * N + A * mv.sum() + 3 * N + mv.sum()) + 8 * N))


def frag_sizes(L):
    out = []
    for i in range(L.n):
        a0, a1 = L.atom_offset[i], L.atom_offset[i + 1]
        m = L.frag_mask[a0:a1]
        K = int(L.n_tors[i])
        out.append([int(((m >> k) & 1).sum()) for k in range(K)])
    return out


def bucket_of(n_atoms, n_tors, tuning):
    na, nr = tuning.n_atom_clusters, tuning.n_rot_clusters
    ab = list(tuning.atom_bounds[:na])
    ab[-1] = 256
    rb = list(tuning.rot_bounds[:nr])
    ca = np.full(len(n_atoms), na - 1)
    for c in range(na - 1, -1, -1):
        ca = np.where(n_atoms <= ab[c], c, ca)
    cr = np.full(len(n_tors), nr - 1)
    for c in range(nr - 1, -1, -1):
        cr = np.where(n_tors <= rb[c], c, cr)
    return ca * nr + cr


# Tuning of the bucketed path on the mixed workload: size classes of at most 64,
# 128, 192 and 256 atoms, one bond class, two restarts per work item, two
# wavefronts per block for the one-slot kernel and four for the others.  The
# library's search (--autotune-ligands) lands within run-to-run noise of it.
DEFAULT_TUNING = {"atom_bounds": [64, 128, 192, 256], "rot_bounds": [32], "restart_chunk": 2, "grid_scale": 1,
                  "waves_per_block": [2, 4, 4, 4], "lazy_clash": 0}


def kernel_tag(stat):
    return f"dock_bucket_{stat['slots']}_{stat['samples_per_lane']}"


def tuning_key(t):
    """The tuning fields that shape the bucket launches, as one string."""
    return (f"atoms {list(t.atom_bounds[:t.n_atom_clusters])} bonds {list(t.rot_bounds[:t.n_rot_clusters])} "
            f"chunk {t.restart_chunk} scale {t.grid_scale} waves {list(t.waves_per_block)} lazy {t.lazy_clash}")


DOCK_SOURCES = ("dock.hip", "lg_internal.h", "lg_device.h")
REFINE_SOURCES = ("refine.hip", "lg_internal.h", "lg_device.h")


def read_profile_value(name, field, tune_key, sources=DOCK_SOURCES):
    """A figure of a committed rocprofv3 counter summary under profiles/, if it was
    taken on the current source of its kernels and the same tuning (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash(sources) or kv.get("tuning") != tune_key:
        return None
    try:
        return float(kv[field])
    except (KeyError, ValueError):
        return None


def source_hash(sources=DOCK_SOURCES):
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_2303_06150_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def experiment_bucket_size(lg, torch, pocket, rt, at, kw, log, sizes=(17, 53, 99),
                           multiples=(1, 2, 3, 4, 5, 6, 9, 12, 24), min_ligands=2000):
    """The bucket-size experiment of Sec. 5 (Fig. 2) on synthetic replicas: one
    ligand of 17, 53 or 99 atoms replicated, docked in batches of l ligands;
    throughput against l at multiples of a third of l_fill.  l_fill = resident
    wavefronts x restart chunk / R is the batch that fills the chip once (one
    wavefront per work item of chunk restarts), the MI355X form of Eq. 1 for this
    mapping."""
    import gen
    t = pocket.get_tuning()
    rows = []
    for N in sizes:
        L1 = gen.replica_ligand(N)
        K = int(L1.n_tors[0])
        dev = lambda L: lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                                          L.inv_bond_len, L.ref_point)
        lg.lg_dock_batch(pocket, dev(gen.replicas(L1, 64)), rt, at, mode=lg.LG_BUCKETED, **kw)
        torch.cuda.synchronize()
        st = pocket.bucket_stats()
        waves = max(b["blocks"] * b["waves_per_block"] for b in st)
        R = int(rt.shape[0])
        l_fill = max(1, waves * t.restart_chunk // R)
        for m in multiples:
            l = max(1, l_fill * m // 3)
            dl = dev(gen.replicas(L1, l))
            out = lg.lg_dock_batch(pocket, dl, rt, at, mode=lg.LG_BUCKETED, **kw)
            torch.cuda.synchronize()
            reps = max(1, -(-max(min_ligands, 4 * l) // l))
            t0 = time.perf_counter()
            for _ in range(reps):
                out = lg.lg_dock_batch(pocket, dl, rt, at, mode=lg.LG_BUCKETED, out=out, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rows.append(dict(atoms=N, bonds=K, l_fill=l_fill, ligands_per_batch=l, thirds_of_fill=m,
                             value=round(l * reps / dt, 1), unit="ligands/s"))
            log(f"bucket size: {N} atoms, l = {l} ({m}/3 of {l_fill}): {l * reps / dt:.1f} ligands/s")
    return dict(experiment="bucket_size", restart_chunk=t.restart_chunk, rows=rows)


def experiment_clusters(lg, torch, pocket, dl, rt, at, kw, n, log):
    """The cluster experiment of Sec. 5 (Fig. 4): throughput of the mixed library
    for atom clusters x rotamer clusters, against one cluster of each."""
    base = pocket.get_tuning()
    rows = []
    for na_bounds in ([256], [64, 256], [64, 128, 192, 256]):
        for nr in (1, 2, 4, 8, 23):
            t = lg.lg_tuning.from_buffer_copy(base)
            t.n_atom_clusters = len(na_bounds)
            for c, b in enumerate(na_bounds):
                t.atom_bounds[c] = b
            rb = lg.lg_rotamer_clusters(nr, 24)
            t.n_rot_clusters = len(rb)
            for c, b in enumerate(rb):
                t.rot_bounds[c] = b
            pocket.set_tuning(t)
            out = lg.lg_dock_batch(pocket, dl, rt, at, mode=lg.LG_BUCKETED, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                out = lg.lg_dock_batch(pocket, dl, rt, at, mode=lg.LG_BUCKETED, out=out, **kw)
            torch.cuda.synchronize()
            v = 2 * n / (time.perf_counter() - t0)
            rows.append(dict(atom_clusters=len(na_bounds), rotamer_clusters=len(rb), value=round(v, 1),
                             unit="ligands/s"))
            log(f"clusters: {len(na_bounds)} x {len(rb)}: {v:.1f} ligands/s")
    pocket.set_tuning(base)
    one = rows[0]["value"]
    for r in rows:
        r["speedup_vs_one_cluster"] = round(r["value"] / one, 3)
    return dict(experiment="clusters", ligands=n, rows=rows)


def experiment_sites(lg, torch, w, pocket, L, rt, at, kw, n_sites, n_lig, log):
    """Sec. 5.2 docks every ligand into twelve docking sites of one target: a
    prefix of the library docked into n_sites synthetic sites of the workload's
    grid size, in one call (site by site, or interleaved per ligand) against one
    single-site call per site.  Site 0 is the workload's pocket."""
    import gen
    t = pocket.get_tuning()
    pockets = [pocket]
    for s in range(1, n_sites):
        c = (10.0 + 6.0 * np.cos(s), -4.0 + 6.0 * np.sin(s), 6.5 + 0.5 * s)
        pk = gen.pocket(w.grid_n, w.spacing, w.n_gauss, w.n_shell, w.seed + 1000 + s, center=c)
        p = lg.Pocket(torch.from_numpy(pk.grid).cuda(), pk.origin, pk.spacing, pk.center, pk.out_value,
                      inv_spacing=pk.inv_spacing)
        p.set_tuning(t)
        pockets.append(p)
    Ls = L.subset(np.arange(n_lig))
    dl = lg.device_ligands(Ls.atom_offset, Ls.tors_offset, Ls.x, Ls.y, Ls.z, Ls.frag_mask, Ls.tors_atoms,
                           Ls.inv_bond_len, Ls.ref_point)
    rows = []
    results = {}

    def timed(label, fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            res = fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 2
        results[label] = res
        rows.append(dict(mode=label, seconds=round(dt, 3), value=round(n_lig * n_sites / dt, 1),
                         unit="ligand-site dockings/s"))
        log(f"sites: {label}: {n_lig * n_sites / dt:.1f} ligand-site dockings/s")

    outs = [None] * n_sites

    def sequential():
        for s, p in enumerate(pockets):
            outs[s] = lg.lg_dock_batch(p, dl, rt, at, mode=lg.LG_BUCKETED, out=outs[s], **kw)
        return list(outs)

    timed("one call per site", sequential)
    timed("one call, site by site", lambda: lg.lg_dock_sites(pockets, dl, rt, at, site_major=True, **kw))
    timed("one call, interleaved", lambda: lg.lg_dock_sites(pockets, dl, rt, at, site_major=False, **kw))
    ref = results["one call per site"]
    same = all(torch.equal(o[k], r[k]) for label in ("one call, site by site", "one call, interleaved")
               for o, r in zip(results[label], ref) for k in ("score", "restart_id", "x", "pivot"))
    base = rows[0]["value"]
    for r in rows:
        r["speedup_vs_one_call_per_site"] = round(r["value"] / base, 3)
    for p in pockets[1:]:
        p.free()
    return dict(experiment="sites", sites=n_sites, ligands=n_lig, grid=w.grid_n, results_bitwise_equal=same,
                rows=rows)


def experiment_screen(lg, torch, w, pocket, L, dl, rt, at, kw, chunk, log):
    """A whole screen of the library on one GPU (the large mixed screen: dock
    every ligand, refine its kept poses, rank the library): the library stays in
    host memory and is docked through lg_dock_stream; the kept poses go to the
    device for refinement; lg_rank gives the global top 1000.  Wall-clock times
    of each stage, transfers included."""
    k = kw["top_k"]
    host = (L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms, L.inv_bond_len, L.ref_point)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = lg.lg_dock_stream(pocket, *host, rt, at, chunk=chunk, **kw)
    t1 = time.perf_counter()
    log(f"screen: {L.n} ligands docked from host memory in {t1 - t0:.2f} s")
    dev_out = {c: torch.from_numpy(out[c]).cuda() for c in ("x", "y", "z", "pivot")}
    poses = lg.docked_poses(dl, dev_out)
    prm = lg.refine_params(clash_dist2=kw["clash_dist2"], poses_per_ligand=k)
    rf = lg.lg_refine(pocket, poses, prm)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"screen: {L.n * k} kept poses refined in {t2 - t1:.2f} s (copy to the device included)")
    rk = lg.lg_rank(pocket, rf["score"], k, min(1000, L.n))
    top = rk["top_idx"].cpu().numpy()
    top_s = rk["top_score"].cpu().numpy()
    t3 = time.perf_counter()
    gain = float((rf["score"].reshape(L.n, k).cpu() - torch.from_numpy(out["score"])).double().mean())
    return dict(experiment="screen", ligands=L.n, poses=L.n * k, chunk=chunk,
                dock_s=round(t1 - t0, 3), dock_value=round(L.n / (t1 - t0), 1),
                refine_s=round(t2 - t1, 3), refine_value=round(L.n * k / (t2 - t1), 1),
                rank_ms=round((t3 - t2) * 1e3, 3), total_s=round(t3 - t0, 3),
                value=round(L.n / (t3 - t0), 1), unit="ligands/s end to end", mean_refine_gain=round(gain, 4),
                top5=[[int(i), float(v)] for i, v in zip(top[:5], top_s[:5])])


def cpu_baseline(w, sample_ids, procs):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    chunks = [c for c in np.array_split(np.asarray(sample_ids), procs) if len(c)]
    t0 = time.perf_counter()
    with ctx.Pool(len(chunks)) as pool:
        done = pool.map(_oracle_chunk, [(w.name, [int(i) for i in c]) for c in chunks])
    wall = time.perf_counter() - t0
    return sum(done), wall, len(chunks)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_chunk(arg):
    name, ids = arg
    sys.path.insert(0, ROOT)
    import gen
    import oracle
    w = gen.WORKLOADS[name]
    pk = gen.workload_pocket(w)
    L = gen.workload_ligands(w, np.array(ids, np.int64))
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    for i in range(L.n):
        oracle.dock_ligand(L.ligand(i), pk, r32.astype(np.float64), a32.astype(np.float64), w.angle_samples,
                           w.sweeps, oracle.trans_step(w.angle_samples), oracle.CLASH2, bits=32,
                           want_poses=False, want_trace=False)
    return L.n


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixed")
    ap.add_argument("--ligands", type=int, default=None, help="use the first n ligands of the workload")
    ap.add_argument("--plain-ligands", type=int, default=2000)
    ap.add_argument("--ablation-ligands", type=int, default=20000)
    ap.add_argument("--stream-chunk", type=int, default=25000,
                    help="side run: the library docked from host memory in chunks of this many ligands (0: skip)")
    ap.add_argument("--autotune-ligands", type=int, default=0,
                    help="tune the bucketed path on this many ligands before timing instead of using "
                         "--tuning (0: no search); a small sample favours fewer buckets, whose second launch "
                         "it cannot fill")
    ap.add_argument("--tuning", default=json.dumps(DEFAULT_TUNING),
                    help="JSON object of tuning fields (atom_bounds, rot_bounds, restart_chunk, grid_scale, "
                         "waves_per_block, lazy_clash); the default is the best of a sweep on the mixed "
                         "workload, the tuning the committed counter summaries were taken on")
    ap.add_argument("--refine-ligands", type=int, default=20000,
                    help="side run: refine the top --refine-poses poses of this many ligands (0: skip)")
    ap.add_argument("--refine-poses", type=int, default=64)
    ap.add_argument("--refine-steps", type=int, default=50)
    ap.add_argument("--cpu-sample", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side-runs", action="store_true", help="skip the plain and ablation runs")
    ap.add_argument("--sites", type=int, default=12, help="docking sites of the sites experiment")
    ap.add_argument("--sites-ligands", type=int, default=10000, help="library prefix of the sites experiment")
    ap.add_argument("--experiment", choices=("bucket-size", "clusters", "sites", "screen"), default=None,
                    help="run one of the paper's experiments on synthetic inputs instead of the benchmark "
                         "(prints its own JSON line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark docks on one GPU; --gpus {args.gpus} is not supported "
              "(ligands shard across GPUs with no exchange but the final ranking).", file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    from paper_2303_06150_amd import lg

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    w = gen.WORKLOADS[args.workload]
    n = w.n_ligands if args.ligands is None else min(args.ligands, w.n_ligands)
    t0 = time.perf_counter()
    L = gen.workload_ligands(w, np.arange(n, dtype=np.int64))
    pk = gen.workload_pocket(w)
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    log(f"inputs: {n} ligands, {int(L.atom_offset[-1])} atoms, {int(L.tors_offset[-1])} bonds "
        f"({time.perf_counter() - t0:.1f}s)")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lg.load_library()
    pocket = lg.Pocket(torch.from_numpy(pk.grid).to(dev), pk.origin, pk.spacing, pk.center, pk.out_value,
                       inv_spacing=pk.inv_spacing)
    dl = lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                           L.inv_bond_len, L.ref_point)
    rt = torch.from_numpy(r32).to(dev)
    at = torch.from_numpy(a32).to(dev)
    T = w.angle_samples
    step = float(np.float32(4.0 / T))
    clash2 = float(np.float32(4.84))
    kw = dict(sweeps=w.sweeps, top_k=w.top_k, trans_samples=T, trans_step=step, clash_dist2=clash2)

    def dock(ligs, mode, out=None):
        return lg.lg_dock_batch(pocket, ligs, rt, at, mode=mode, out=out, **kw)

    if args.experiment == "bucket-size":
        print(json.dumps(experiment_bucket_size(lg, torch, pocket, rt, at, kw, log)), flush=True)
        pocket.free()
        return
    if args.experiment == "clusters":
        print(json.dumps(experiment_clusters(lg, torch, pocket, dl, rt, at, kw, n, log)), flush=True)
        pocket.free()
        return

    # ---- autotuning on a prefix of the library (reported, not timed)
    tune = None
    if args.tuning and args.autotune_ligands <= 0:
        spec = json.loads(args.tuning)
        t = pocket.get_tuning()
        t.n_atom_clusters = len(spec["atom_bounds"])
        for c, b in enumerate(spec["atom_bounds"]):
            t.atom_bounds[c] = b
        t.n_rot_clusters = len(spec["rot_bounds"])
        for c, b in enumerate(spec["rot_bounds"]):
            t.rot_bounds[c] = b
        for c, v in enumerate(spec["waves_per_block"]):
            t.waves_per_block[c] = v
        t.restart_chunk, t.grid_scale, t.lazy_clash = spec["restart_chunk"], spec["grid_scale"], spec["lazy_clash"]
        pocket.set_tuning(t)
        tune = dict(given=spec)
        log(f"tuning given: {tuning_key(t)}")
    elif args.autotune_ligands > 0:
        nt = min(args.autotune_ligands, n)
        Lt = L.subset(np.arange(nt))
        dlt = lg.device_ligands(Lt.atom_offset, Lt.tors_offset, Lt.x, Lt.y, Lt.z, Lt.frag_mask, Lt.tors_atoms,
                                Lt.inv_bond_len, Lt.ref_point)
        t0 = time.perf_counter()
        tt, tms = lg.lg_autotune(pocket, dlt, rt, at, **kw)
        tune = dict(ligands=nt, seconds=round(time.perf_counter() - t0, 2), sample_ms=round(tms, 3),
                    restart_chunk=tt.restart_chunk, grid_scale=tt.grid_scale,
                    waves_per_block=list(tt.waves_per_block), lazy_clash=tt.lazy_clash,
                    atom_bounds=list(tt.atom_bounds[:tt.n_atom_clusters]),
                    rot_bounds=list(tt.rot_bounds[:tt.n_rot_clusters]))
        log(f"autotune on {nt} ligands: {tune}")
        log("  as --tuning: " + json.dumps({k: tune[k] for k in ("atom_bounds", "rot_bounds", "restart_chunk",
                                                                 "grid_scale", "waves_per_block", "lazy_clash")}))
        del dlt
    if args.experiment == "screen":
        print(json.dumps(experiment_screen(lg, torch, w, pocket, L, dl, rt, at, kw, max(args.stream_chunk, 1000),
                                           log)), flush=True)
        pocket.free()
        return
    if args.experiment == "sites":
        print(json.dumps(experiment_sites(lg, torch, w, pocket, L, rt, at, kw, args.sites,
                                          min(args.sites_ligands, n), log)), flush=True)
        pocket.free()
        return

    # ---- bucketed persistent path: the timed steps
    out = None
    for s in range(args.warmup):
        out = dock(dl, lg.LG_BUCKETED, out)
        torch.cuda.synchronize()
        log(f"warmup step {s} done")
    bucket_ms = {}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        out = dock(dl, lg.LG_BUCKETED, out)
        log(f"step {s} enqueued")
    torch.cuda.synchronize()
    log("timed steps done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / max(args.steps, 1)
    value = n * args.steps / elapsed

    # ---- per-kernel durations: a few more steps launched directly on the stream
    # (no graph), the bucket launches one after another exactly as in the graph
    # replays, with HIP events recorded on that stream between them
    tuning = pocket.get_tuning()
    eager = lg.lg_tuning.from_buffer_copy(tuning)
    eager.use_graph = 0
    pocket.set_tuning(eager)
    timing_steps = max(1, min(3, args.steps))
    stats = []
    direct_ms = []
    for s in range(timing_steps):
        out = dock(dl, lg.LG_BUCKETED, out)
        torch.cuda.synchronize()
        stats = pocket.bucket_stats()
        for b in stats:
            bucket_ms.setdefault(b["bucket"], []).append(b["ms"])
        direct_ms.append(stats[0]["span_ms"] if stats else 0.0)
    pocket.set_tuning(tuning)
    log(f"timing steps (events between bucket launches) done: bucket launches {np.mean(direct_ms):.1f} ms "
        f"per step against {ms_per_step:.1f} ms per graph-replayed step")

    # ---- roofline of the dominant kernel: the bucket launch that takes the most time
    bid = bucket_of(L.n_atoms, L.n_tors, tuning)
    fs = frag_sizes(L)
    ops = isa_ops(L.n_atoms, fs, w.restarts, w.angle_samples, T, w.sweeps)
    plain_ops = plain_method_ops(L.n_atoms, fs, w.restarts, w.angle_samples, T, w.sweeps)
    looks = lookups(L.n_atoms, fs, w.restarts, w.angle_samples, T, w.sweeps)
    busy = [b for b in stats if b["ligands"] > 0]
    dom = max(busy, key=lambda b: float(np.mean(bucket_ms[b["bucket"]])))
    dom_ms = float(np.mean(bucket_ms[dom["bucket"]]))
    sel = bid == dom["bucket"]
    dom_ops, dom_plain, dom_looks = float(ops[sel].sum()), float(plain_ops[sel].sum()), float(looks[sel].sum())
    kernel = f"dock_bucket_kernel<{dom['slots']},{dom['samples_per_lane']}>"
    tune_key = tuning_key(tuning)
    # HBM bytes and VALU issue of the dominant launch, from the committed rocprofv3
    # counter summaries, when they were taken on this kernel source and tuning
    traffic = read_profile_value(f"{kernel_tag(dom)}_{args.workload}_traffic.txt", "hbm_bytes_per_dispatch",
                                 tune_key)
    valu_busy = read_profile_value(f"{kernel_tag(dom)}_{args.workload}_valu.txt", "valu_busy", tune_key)
    valu_issue = read_profile_value(f"{kernel_tag(dom)}_{args.workload}_valu.txt", "valu_issue_per_simd_cycle",
                                    tune_key)
    l2_hit = read_profile_value(f"{kernel_tag(dom)}_{args.workload}_valu.txt", "l2_hit", tune_key)
    achieved = dom_ops / (dom_ms * 1e-3)
    # the sustained rate of the scans' index arithmetic on this device, beside the peak
    valu_meas = lg.lg_valu_probe(pocket, VALU_PROBE_MIX, 2000)
    roofline = dict(bound="alu", achieved=round(achieved / 1e12, 3), peak=round(PEAK_LANE_OPS / 1e12, 3),
                    unit="TOP/s", frac=round(achieved / PEAK_LANE_OPS, 4), traffic=traffic, kernel=kernel,
                    kernel_ms=round(dom_ms, 3), ligands_in_launch=int(dom["ligands"]),
                    ops_per_launch=dom_ops,
                    ops_basis="VALU lane-ops of the scans' inner loops, every sample of every scan (gfx950 "
                              "assembly count per unit; pair tests and per-scan work not counted)",
                    valu_busy=valu_busy,
                    # every VALU instruction the counters saw, against gfx950's issue limit of one
                    # wave64 VALU instruction per SIMD per two cycles (the 78.6 T lane-op peak)
                    valu_issue_frac=round(2.0 * valu_issue, 4) if valu_issue is not None else None,
                    l2_hit=l2_hit,   # TCC hits / (hits + misses) of the launch: the grid stays L2-resident
                    gather_bw=round(4.0 * dom_looks / (dom_ms * 1e-3) / 1e9, 1), gather_unit="GB/s",
                    measured_valu_peak=round(valu_meas / 1e12, 3),
                    plain_method=dict(ops_per_launch=dom_plain,
                                      rate=round(dom_plain / (dom_ms * 1e-3) / 1e12, 3),
                                      ratio_to_peak=round(dom_plain / (dom_ms * 1e-3) / PEAK_LANE_OPS, 3),
                                      basis="lane-ops the plain method would issue: op-script constants "
                                            "32/23/37 per rotation/translation/torsion sample and atom, a "
                                            "pair test (8) of every moving and static atom for every "
                                            "torsion sample; a ratio above 1 is the speed-up of exact pair "
                                            "pruning, not a hardware fraction"))
    total_ops = float(ops.sum())

    # ---- side runs: plain per-ligand launches, single-bucket ablation
    side = {}
    if not args.no_side_runs:
        npl = min(args.plain_ligands, n)
        Lp = L.subset(np.arange(npl))
        dlp = lg.device_ligands(Lp.atom_offset, Lp.tors_offset, Lp.x, Lp.y, Lp.z, Lp.frag_mask, Lp.tors_atoms,
                                Lp.inv_bond_len, Lp.ref_point)
        Lw = L.subset(np.arange(min(8, n)))
        dock(lg.device_ligands(Lw.atom_offset, Lw.tors_offset, Lw.x, Lw.y, Lw.z, Lw.frag_mask, Lw.tors_atoms,
                               Lw.inv_bond_len, Lw.ref_point), lg.LG_PLAIN)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        dock(dlp, lg.LG_PLAIN)
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - tp
        ob = dock(dlp, lg.LG_BUCKETED)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        dock(dlp, lg.LG_BUCKETED, ob)
        torch.cuda.synchronize()
        buck_small_s = time.perf_counter() - tb
        side["plain"] = dict(ligands=npl, value=round(npl / plain_s, 2), unit="ligands/s")
        side["bucketed_same_prefix"] = dict(ligands=npl, value=round(npl / buck_small_s, 2), unit="ligands/s")
        log(f"plain: {npl / plain_s:.1f} ligands/s on {npl} ligands; bucketed on the same: {npl / buck_small_s:.1f}")
        # ablation: one bucket for every ligand (the 1x1-cluster baseline), largest-class kernel
        nab = min(args.ablation_ligands, n)
        La = L.subset(np.arange(nab))
        dla = lg.device_ligands(La.atom_offset, La.tors_offset, La.x, La.y, La.z, La.frag_mask, La.tors_atoms,
                                La.inv_bond_len, La.ref_point)
        one = lg.lg_tuning.from_buffer_copy(tuning)
        one.n_atom_clusters = 1
        one.atom_bounds[0] = 256
        one.n_rot_clusters = 1
        one.rot_bounds[0] = 32
        pocket.set_tuning(one)
        oa = dock(dla, lg.LG_BUCKETED)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        dock(dla, lg.LG_BUCKETED, oa)
        torch.cuda.synchronize()
        abl_s = time.perf_counter() - ta
        pocket.set_tuning(tuning)
        ob = dock(dla, lg.LG_BUCKETED)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        dock(dla, lg.LG_BUCKETED, ob)
        torch.cuda.synchronize()
        buck_ab_s = time.perf_counter() - tb
        side["one_bucket_ablation"] = dict(ligands=nab, value=round(nab / abl_s, 2), unit="ligands/s",
                                           bucketed_same_ligands=round(nab / buck_ab_s, 2))
        log(f"one-bucket ablation: {nab / abl_s:.1f} ligands/s vs bucketed {nab / buck_ab_s:.1f} on {nab}")

        # end to end: the library in host memory, streamed through the device in chunks
        # (copies in and out included, overlapped with docking)
        if args.stream_chunk > 0:
            host = (L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms, L.inv_bond_len,
                    L.ref_point)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            lg.lg_dock_stream(pocket, *host, rt, at, chunk=args.stream_chunk, **kw)
            torch.cuda.synchronize()
            stream_s = time.perf_counter() - ts
            side["end_to_end"] = dict(ligands=n, chunk=args.stream_chunk, value=round(n / stream_s, 2),
                                      unit="ligands/s", seconds=round(stream_s, 3),
                                      note="host-resident library, pinned staging, transfers included")
            log(f"end to end from host memory: {n / stream_s:.1f} ligands/s (chunks of {args.stream_chunk})")

        # refinement of the kept poses (k per ligand, about their docking pivots) and the
        # global ranking of the ligands by their best refined pose
        nrf = min(args.refine_ligands, n)
        if nrf > 0:
            kp = args.refine_poses
            Lr = L.subset(np.arange(nrf))
            dlr = lg.device_ligands(Lr.atom_offset, Lr.tors_offset, Lr.x, Lr.y, Lr.z, Lr.frag_mask, Lr.tors_atoms,
                                    Lr.inv_bond_len, Lr.ref_point)
            od = lg.lg_dock_batch(pocket, dlr, rt, at, mode=lg.LG_BUCKETED, **dict(kw, top_k=kp))
            poses = lg.docked_poses(dlr, od)
            prm = lg.refine_params(steps=args.refine_steps, clash_dist2=clash2, poses_per_ligand=kp)
            lg.lg_refine(pocket, poses, prm)
            torch.cuda.synchronize()
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            rf = lg.lg_refine(pocket, poses, prm)
            e1.record()
            rk = lg.lg_rank(pocket, rf["score"], kp, min(1000, nrf))
            e2.record()
            torch.cuda.synchronize()
            rms = e0.elapsed_time(e1)
            gain = (rf["score"].reshape(nrf, kp) - od["score"]).double()
            rops = float(refine_ops_per_step(Lr).sum()) * kp * args.refine_steps
            rach = rops / (rms * 1e-3)
            side["refine"] = dict(ligands=nrf, poses=nrf * kp, steps=args.refine_steps, ms=round(rms, 3),
                                  value=round(nrf * kp / (rms * 1e-3), 1), unit="poses/s",
                                  mean_score_gain=round(float(gain.mean()), 4),
                                  rank_top_m=min(1000, nrf), rank_ms=round(e1.elapsed_time(e2), 3),
                                  roofline=dict(bound="alu", achieved=round(rach / 1e12, 3),
                                                peak=round(PEAK_LANE_OPS / 1e12, 3), unit="TOP/s",
                                                frac=round(rach / PEAK_LANE_OPS, 4), kernel="refine_kernel<s>",
                                                algorithmic_ops=rops,
                                                measured_valu_peak=round(
                                                    lg.lg_valu_probe(pocket, VALU_PROBE_MIX, 2000) / 1e12, 3)))
            # the refinement kernels' VALU issue from the committed counter summary
            # (time-weighted over the size classes), against the dual-rate limit
            rvi = read_profile_value("refine_mixed20k_counters.md", "valu_issue_per_simd_cycle", "refine",
                                     REFINE_SOURCES)
            side["refine"]["roofline"]["valu_issue_frac"] = round(2.0 * rvi, 4) if rvi is not None else None
            if not args.no_cpu_baseline:
                import oracle
                hx, hy, hz = (od[c].cpu().numpy() for c in ("x", "y", "z"))
                hp = od["pivot"].cpu().numpy()
                tc0 = time.perf_counter()
                done = 0
                for i in range(16):
                    lig = Lr.ligand(i)
                    a0, N = int(Lr.atom_offset[i]), int(Lr.n_atoms[i])
                    for q in range(8):
                        b = kp * a0 + q * N
                        pose = np.stack([hx[b:b + N], hy[b:b + N], hz[b:b + N]], 1).astype(np.float64)
                        oracle.refine(lig, pk, pose, hp[i, q].astype(np.float64), bits=32)
                        done += 1
                tcs = time.perf_counter() - tc0
                side["refine"]["cpu_baseline"] = dict(value=round(done / tcs, 2), unit="poses/s", cores=1,
                                                      kind="oracle",
                                                      sample=f"{done} poses (8 kept poses of each of the first 16 "
                                                             f"ligands), {args.refine_steps} steps, FP32 oracle, "
                                                             f"one process")
                log(f"refine cpu baseline: {done / tcs:.1f} poses/s on one core")
            log(f"refine: {nrf * kp} poses x {args.refine_steps} steps in {rms:.1f} ms "
                f"({nrf * kp / (rms * 1e-3):.0f} poses/s); ranking {e1.elapsed_time(e2):.3f} ms")
            del od, poses, rf, rk

    if args.copy_calibration:
        # an elementwise kernel that reads 1 GiB and writes 1 GiB (a device-to-device
        # copy_ would go to the DMA engines and not show up as a kernel)
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()

    # ---- CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        procs = max(1, min(16, os.cpu_count() or 1))
        sample = np.linspace(0, w.n_ligands - 1, args.cpu_sample).astype(np.int64)
        done, wall, used = cpu_baseline(w, sample, procs)
        cpu = dict(value=round(done / wall, 3), unit="ligands/s", cores=used, kind="oracle",
                   sample=f"{done} ligands of the {args.workload} workload (ids spread evenly over "
                          f"{w.n_ligands}), every restart ({w.restarts}), FP32 oracle, one process per core")
        log(f"cpu baseline: {done / wall:.2f} ligands/s on {used} processes")
        # one core, measured (not divided out): 4 ligands spread over the library
        one = np.linspace(0, w.n_ligands - 1, 4).astype(np.int64)
        d1, wall1, _ = cpu_baseline(w, one, 1)
        cpu["one_core"] = dict(value=round(d1 / wall1, 3), unit="ligands/s",
                               sample=f"{d1} ligands (ids spread evenly), every restart, one process")
        cpu["cpu_model"] = cpu_model()
        log(f"cpu baseline, one core: {d1 / wall1:.3f} ligands/s ({cpu['cpu_model']})")

    buckets = [dict(bucket=b["bucket"], atoms_le=b["atom_bound"], slots=b["slots"], vgprs=b["vgprs"],
                    lds_bytes=b["lds_bytes"], blocks_per_cu=b["blocks_per_cu"], waves_in_flight=b["blocks"] * b["waves_per_block"],
                    ligands=b["ligands"], ms=round(float(np.mean(bucket_ms.get(b["bucket"], [b["ms"]]))), 3))
               for b in stats]
    rec = dict(
        metric="ligands docked/sec at 256 restarts (bucketed vs plain, 1 MI355X)",
        value=round(value, 2), unit="ligands/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms_per_step, 3), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32", data="synthetic",
        config=dict(workload=f"{args.workload}: {n} ligands, atoms {w.nlo}-{w.nhi}"
                             f"{' (lognormal median 38)' if w.size_mode == 1 else ''}, "
                             f"bonds {w.klo}-{w.khi}, {w.grid_n}^3 grid @ {w.spacing} A, R={w.restarts}, "
                             f"A=T={w.angle_samples}, S={w.sweeps}, top-{w.top_k}",
                    ligands=n, restarts=w.restarts, angle_samples=w.angle_samples, sweeps=w.sweeps,
                    top_k=w.top_k, mode="bucketed persistent, one HIP graph"),
        roofline=roofline, cpu_baseline=cpu, autotune=tune,
        isa_ops_rate_whole_step=round(total_ops / (ms_per_step * 1e-3) / 1e12, 3),
        direct_launch_ms_per_step=round(float(np.mean(direct_ms)), 3),
        speedup_vs_plain=(round(side["bucketed_same_prefix"]["value"] / side["plain"]["value"], 2)
                          if "plain" in side else None),
        buckets=buckets, **side)
    print(json.dumps(rec), flush=True)
    pocket.free()


if __name__ == "__main__":
    main()
