"""GPU parity of the docking path against the CPU oracle (same seeded inputs).

The bar: selected sample indices identical, final scores and poses bitwise
identical (FP32, quantised grid), top-k identical; plain and bucketed launches
bitwise identical; runs deterministic; batch order irrelevant.
"""
import numpy as np
import pytest

import gen
import oracle
from gpu_common import compare_ligand, dock_gpu, dock_oracle, device_pocket, pose_of, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lgmod():
    import torch
    from paper_2303_06150_amd import lg
    assert torch.cuda.is_available()
    lg.load_library()
    return lg


def test_tiny_workload_plain_and_bucketed(lgmod, tiny):
    lg = lgmod
    w, pk, L = tiny["w"], tiny["pocket"], tiny["ligs"]
    say("tiny: 64 ligands, R=32 A=64 S=2")
    pocket = device_pocket(pk)
    kw = dict(T=w.angle_samples, S=w.sweeps, top_k=w.top_k)
    plain = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], mode=lg.LG_PLAIN, **kw)
    buck = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], mode=lg.LG_BUCKETED, **kw)
    for key in plain:
        np.testing.assert_array_equal(plain[key], buck[key], err_msg=f"plain vs bucketed: {key}")
    rows = np.arange(w.restarts)
    for i in range(L.n):
        ref = dock_oracle(pk, L, i, tiny["r32"], tiny["a32"], T=w.angle_samples, S=w.sweeps)
        compare_ligand(buck, L, i, ref, rows, w.top_k, w.restarts, "tiny")
    pocket.free()


def ragged_ligands():
    N = [1, 2, 3, 20, 63, 64, 65, 127, 128, 129, 200, 255, 256, 40]
    K = [0, 0, 0, 5, 12, 1, 20, 32, 8, 31, 16, 32, 32, 0]
    ids = np.arange(100, 100 + len(N))
    return gen.ligands_from_sizes(ids, 11, np.array(N), np.array(K))


@pytest.mark.parametrize("A,T", [(48, 40), (130, 64), (256, 256), (512, 128)])
def test_ragged_sizes_and_sample_counts(lgmod, tiny, A, T):
    lg = lgmod
    pk = gen.pocket(48, 0.5, 60, 400, 3)
    L = ragged_ligands()
    assert L.n_tors.max() == 32 and L.n_atoms.max() == 256
    r32, _ = gen.restarts(5, 5)
    a32, _ = gen.angles(A)
    say(f"ragged: N up to 256, K up to 32, A={A} T={T}")
    pocket = device_pocket(pk, on_device=False)
    kw = dict(T=T, S=1, top_k=3)
    buck = dock_gpu(pocket, L, r32, a32, mode=lg.LG_BUCKETED, **kw)
    plain = dock_gpu(pocket, L, r32, a32, mode=lg.LG_PLAIN, **kw)
    for key in plain:
        np.testing.assert_array_equal(plain[key], buck[key], err_msg=f"plain vs bucketed: {key}")
    t = pocket.get_tuning()
    z = lg.lg_tuning.from_buffer_copy(t)
    z.lazy_clash = 1
    pocket.set_tuning(z)
    lazy = dock_gpu(pocket, L, r32, a32, mode=lg.LG_BUCKETED, **kw)
    pocket.set_tuning(t)
    for key in plain:
        np.testing.assert_array_equal(lazy[key], buck[key], err_msg=f"winner-only clash test: {key}")
    for i in range(L.n):
        ref = dock_oracle(pk, L, i, r32, a32, T=T, S=1)
        compare_ligand(buck, L, i, ref, np.arange(5), 3, 5, f"ragged A={A}")
    pocket.free()


def test_refine_ragged_sizes(lgmod, tiny):
    """Refinement of ligands of 1 to 256 atoms and 0 to 32 bonds (every kernel
    size class, two poses per wavefront for the small ones at k = 2): each kept
    pose refined bit for bit as the FP32 oracle refines it."""
    lg = lgmod
    import torch
    w, pk = tiny["w"], tiny["pocket"]
    L = ragged_ligands()
    pocket = device_pocket(pk)
    rt = torch.from_numpy(tiny["r32"]).cuda()
    at = torch.from_numpy(tiny["a32"]).cuda()
    dl = lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                           L.inv_bond_len, L.ref_point)
    for k in (1, 2):
        say(f"refine ragged: N up to 256, K up to 32, k = {k}")
        out = lg.lg_dock_batch(pocket, dl, rt, at, sweeps=1, top_k=k, trans_samples=w.angle_samples,
                               trans_step=oracle.trans_step(w.angle_samples), clash_dist2=oracle.CLASH2)
        res = lg.lg_refine(pocket, lg.docked_poses(dl, out),
                           lg.refine_params(steps=20, clash_dist2=oracle.CLASH2, poses_per_ligand=k))
        torch.cuda.synchronize()
        h = {key: v.cpu().numpy() for key, v in out.items()}
        r = {key: v.cpu().numpy() for key, v in res.items()}
        for i in range(L.n):
            lig = L.ligand(i)
            for q in range(k):
                pose = pose_of(h, L, i, q, k).astype(np.float64)
                sc, best, _ = oracle.refine(lig, pk, pose, h["pivot"][i, q].astype(np.float64), bits=32, steps=20)
                np.testing.assert_array_equal(pose_of(r, L, i, q, k).astype(np.float64), best,
                                              err_msg=f"k={k}: ligand {i} (N={L.n_atoms[i]}, K={L.n_tors[i]}) pose {q}")
                assert r["score"][i * k + q] == sc, (k, i, q)
    pocket.free()


def test_full_size_mixed_sampled(lgmod):
    """Mixed workload at full per-ligand size (96^3 grid, R=256, A=T=256, S=3, top-10) in
    the bucketed launch; sampled restarts checked against the oracle one by one."""
    lg = lgmod
    w = gen.WORKLOADS["mixed"]
    ids = np.arange(0, w.n_ligands, 50)          # 2000 ligands spread over the 100k set
    L = gen.workload_ligands(w, ids)
    pk = gen.workload_pocket(w)
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    say(f"mixed slice: {L.n} ligands, {L.atom_offset[-1]} atoms")
    pocket = device_pocket(pk)
    out = dock_gpu(pocket, L, r32, a32, T=w.angle_samples, S=w.sweeps, top_k=w.top_k, mode=lg.LG_BUCKETED)
    rng = np.random.default_rng(0)
    picks = rng.choice(L.n, 6, replace=False)
    for i in picks:
        rows = np.sort(rng.choice(w.restarts, 3, replace=False))
        ref = dock_oracle(pk, L, int(i), r32, a32, T=w.angle_samples, S=w.sweeps, rows=rows)
        compare_ligand(out, L, int(i), ref, rows, w.top_k, w.restarts, "mixed")
        say(f"  ligand {i} (N={L.n_atoms[i]}, K={L.n_tors[i]}) restarts {rows.tolist()} ok")
    # one ligand with every restart: the top-10 selection and its poses
    i = int(np.argmin(np.abs(L.n_atoms - 30)))
    ref = dock_oracle(pk, L, i, r32, a32, T=w.angle_samples, S=w.sweeps)
    compare_ligand(out, L, i, ref, np.arange(w.restarts), w.top_k, w.restarts, "mixed all restarts")
    pocket.free()


def test_determinism_and_batch_order(lgmod, tiny):
    lg = lgmod
    w, pk, L = tiny["w"], tiny["pocket"], tiny["ligs"]
    pocket = device_pocket(pk)
    kw = dict(T=w.angle_samples, S=w.sweeps, top_k=4, mode=lg.LG_BUCKETED)
    a = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], **kw)
    b = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], **kw)
    for key in a:
        np.testing.assert_array_equal(a[key], b[key])
    # launched directly (no graph, events between the bucket launches): same bits
    t = pocket.get_tuning()
    e = lg.lg_tuning.from_buffer_copy(t)
    e.use_graph = 0
    pocket.set_tuning(e)
    d = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], **kw)
    stats = pocket.bucket_stats()
    pocket.set_tuning(t)
    for key in a:
        np.testing.assert_array_equal(a[key], d[key])
    assert sum(b["ligands"] for b in stats) == L.n
    assert all(b["ms"] >= 0 for b in stats)
    # launches one after another: the span covers their sum
    assert all(b["span_ms"] >= b["ms"] - 1e-3 for b in stats)
    assert stats[0]["span_ms"] >= sum(b["ms"] for b in stats) - 1e-2
    # every instance is sized for the batch's largest ligand (at most 40 atoms here)
    assert all(b["slots"] == 1 for b in stats)
    # other tunings (one bucket, rotamer clusters, chunking): same bits
    o = lg.lg_tuning.from_buffer_copy(t)
    o.n_atom_clusters, o.n_rot_clusters, o.restart_chunk = 2, 3, 3
    o.atom_bounds[0], o.atom_bounds[1] = 30, 256
    o.rot_bounds[0], o.rot_bounds[1], o.rot_bounds[2] = 2, 4, 32
    o.waves_per_block[0], o.grid_scale = 1, 2
    pocket.set_tuning(o)
    f = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], **kw)
    pocket.set_tuning(t)
    for key in a:
        np.testing.assert_array_equal(a[key], f[key])
    # clash test of the winner only (no pruned pair list): same bits
    z = lg.lg_tuning.from_buffer_copy(t)
    z.lazy_clash = 1
    pocket.set_tuning(z)
    g = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], **kw)
    pocket.set_tuning(t)
    for key in a:
        np.testing.assert_array_equal(a[key], g[key])
    perm = np.random.default_rng(1).permutation(L.n)
    Lp = L.subset(perm)
    c = dock_gpu(pocket, Lp, tiny["r32"], tiny["a32"], **kw)
    np.testing.assert_array_equal(c["all_scores"], a["all_scores"][perm])
    np.testing.assert_array_equal(c["restart_id"], a["restart_id"][perm])
    np.testing.assert_array_equal(c["trace"][..., :12], a["trace"][perm][..., :12])
    pocket.free()


def test_score_and_gradient(lgmod, tiny):
    lg = lgmod
    import torch
    pk, L = tiny["pocket"], tiny["ligs"]
    pocket = device_pocket(pk)
    rng = np.random.default_rng(3)
    # poses: input conformations moved into the pocket with random offsets
    shift = pk.center + rng.uniform(-3, 3, size=(L.n, 3)).astype(np.float32)
    lig_of = np.repeat(np.arange(L.n), L.n_atoms)
    cen = np.stack([L.ref_point[0::3], L.ref_point[1::3], L.ref_point[2::3]], 1)
    xs = (L.x - cen[lig_of, 0] + shift[lig_of, 0]).astype(np.float32)
    ys = (L.y - cen[lig_of, 1] + shift[lig_of, 1]).astype(np.float32)
    zs = (L.z - cen[lig_of, 2] + shift[lig_of, 2]).astype(np.float32)
    refp = shift.reshape(-1).astype(np.float32)
    dl = lg.device_ligands(L.atom_offset, L.tors_offset, xs, ys, zs, L.frag_mask, L.tors_atoms,
                           L.inv_bond_len, refp)
    near = lg.lg_score(pocket, dl, lg.LG_NEAREST)["score"].cpu().numpy()
    tri = lg.lg_score(pocket, dl, lg.LG_TRILINEAR, grad=True, top_m=10)
    torch.cuda.synchronize()
    ts, tg = tri["score"].cpu().numpy(), tri["grad"].cpu().numpy()
    worst = 0.0
    for i in range(L.n):
        a0, a1 = L.atom_offset[i], L.atom_offset[i + 1]
        xyz = np.stack([xs[a0:a1], ys[a0:a1], zs[a0:a1]], 1).astype(np.float64)
        assert near[i] == oracle.score(pk, xyz, 0, 32)
        assert ts[i] == oracle.score(pk, xyz, 1, 32)
        lig = L.ligand(i)
        _, g64 = oracle.pose_grad(lig, pk, xyz, shift[i].astype(np.float64))
        K = int(L.n_tors[i])
        g = tg[6 * i + L.tors_offset[i]: 6 * i + L.tors_offset[i] + 6 + K]
        scale = max(np.abs(g64).max(), 1e-3)
        worst = max(worst, np.abs(g - g64).max() / scale)
    assert worst < 1e-4, worst
    order = np.lexsort((np.arange(L.n), -ts.astype(np.float64)))[:10]
    np.testing.assert_array_equal(tri["top_idx"].cpu().numpy(), order)
    np.testing.assert_array_equal(tri["top_score"].cpu().numpy(), ts[order])
    pocket.free()


def test_device_validation_errors(lgmod, tiny):
    lg = lgmod
    import torch
    pk, L = tiny["pocket"], tiny["ligs"]
    pocket = device_pocket(pk)
    r = torch.from_numpy(tiny["r32"]).cuda()
    a = torch.from_numpy(tiny["a32"]).cuda()
    for fault in ("out of range", "same atom twice"):
        bad = L.tors_atoms.copy()
        bad[1] = 999 if fault == "out of range" else bad[0]
        dl = lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, bad, L.inv_bond_len,
                               L.ref_point)
        # checked on the host (host copies given), then by the device check kernel
        for host in (True, False):
            dl.host_checks = host
            with pytest.raises(lg.LgError) as e:
                lg.lg_dock_batch(pocket, dl, r, a, sweeps=1, top_k=1, trans_samples=64, trans_step=0.0625,
                                 clash_dist2=oracle.CLASH2)
            assert e.value.status == lg.LG_ERR_INVALID_ARG, (fault, host)
    with pytest.raises(lg.LgError) as e:
        lg.lg_dock_batch(pocket, device_ligands_ok(lg, L), r, a, sweeps=1, top_k=33, trans_samples=64,
                         trans_step=0.0625, clash_dist2=oracle.CLASH2)
    assert e.value.status == lg.LG_ERR_INVALID_ARG
    pocket.free()


def device_ligands_ok(lg, L):
    return lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                             L.inv_bond_len, L.ref_point)


def refine_against_oracle(lg, pocket, pk, L, out, k):
    """lg_refine on every ligand's top-k docked poses; best pose and score must
    equal the FP32 oracle's refinement bitwise.  Returns how many poses moved."""
    import torch
    parts, idx = [], []
    for i in range(L.n):
        for q in range(k):
            a0, a1 = L.atom_offset[i], L.atom_offset[i + 1]
            base = k * a0 + q * (a1 - a0)
            xyz = np.stack([out["x"][base:base + a1 - a0], out["y"][base:base + a1 - a0],
                            out["z"][base:base + a1 - a0]], 1)
            parts.append(xyz)
            idx.append(i)
    Lp = L.subset(np.array(idx))
    xyz_all = np.concatenate(parts)
    # pivot = FP32 centroid of the pose
    cen = np.stack([p.astype(np.float64).mean(0) for p in parts]).astype(np.float32)
    dl = lg.device_ligands(Lp.atom_offset, Lp.tors_offset, xyz_all[:, 0], xyz_all[:, 1], xyz_all[:, 2],
                           Lp.frag_mask, Lp.tors_atoms, Lp.inv_bond_len, cen.reshape(-1))
    prm = lg.refine_params(clash_dist2=oracle.CLASH2)
    res = lg.lg_refine(pocket, dl, prm)
    torch.cuda.synchronize()
    rx, ry, rz, rs = (res[c].cpu().numpy() for c in ("x", "y", "z", "score"))
    moved = 0
    for j in range(Lp.n):
        lig = Lp.ligand(j)
        a0, a1 = Lp.atom_offset[j], Lp.atom_offset[j + 1]
        s, best, acc = oracle.refine(lig, pk, parts[j].astype(np.float64), cen[j].astype(np.float64), bits=32)
        got = np.stack([rx[a0:a1], ry[a0:a1], rz[a0:a1]], 1).astype(np.float64)
        np.testing.assert_array_equal(got, best, err_msg=f"refined pose {j}")
        assert rs[j] == s, (j, rs[j], s)
        moved += not np.array_equal(best, parts[j].astype(np.float64))
    return moved, Lp.n


def test_refine_matches_oracle(lgmod, tiny):
    """lg_refine on docked poses: best pose and score bitwise equal to the FP32
    oracle's refinement (same step script, same step polynomial, sums in atom
    order)."""
    lg = lgmod
    w, pk, L = tiny["w"], tiny["pocket"], tiny["ligs"]
    pocket = device_pocket(pk)
    k = 2
    out = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], T=w.angle_samples, S=w.sweeps, top_k=k, mode=lg.LG_BUCKETED,
                   trace=False, all_scores=False)
    moved, n = refine_against_oracle(lg, pocket, pk, L, out, k)
    assert moved > n // 2
    pocket.free()


def reversed_bonds(L):
    """The same ligands with their rotatable bonds listed in reverse (children
    before parents): frag_mask bits, bond atoms and lengths permuted alike."""
    parts = []
    for i in range(L.n):
        a = L.ligand_arrays(i)
        K = len(a["inv_bond_len"])
        m = np.asarray(a["frag_mask"], np.uint32)
        rm = np.zeros_like(m)
        for k in range(K):
            rm |= ((m >> np.uint32(k)) & np.uint32(1)) << np.uint32(K - 1 - k)
        a = dict(a, frag_mask=rm, tors_atoms=np.asarray(a["tors_atoms"]).reshape(-1, 2)[::-1].reshape(-1).copy(),
                 inv_bond_len=np.asarray(a["inv_bond_len"])[::-1].copy(),
                 inv_bond_len64=np.asarray(a["inv_bond_len64"])[::-1].copy())
        parts.append(a)
    return gen._assemble(L.ids, parts)


def test_bonds_in_any_order(lgmod, tiny):
    """Bonds listed children first: a torsion then moves the axes of bonds
    applied after it, so refinement must take its sequential path (matrices
    cannot be built up front).  Docking and refinement still match the oracle
    bitwise."""
    lg = lgmod
    w, pk = tiny["w"], tiny["pocket"]
    L = reversed_bonds(tiny["ligs"].subset(np.arange(24)))
    assert (L.n_tors >= 2).sum() >= 12
    pocket = device_pocket(pk)
    k = 2
    out = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], T=w.angle_samples, S=w.sweeps, top_k=k, mode=lg.LG_BUCKETED,
                   trace=True, all_scores=True)
    rows = np.arange(w.restarts)
    for i in range(0, L.n, 3):
        ref = dock_oracle(pk, L, i, tiny["r32"], tiny["a32"], T=w.angle_samples, S=w.sweeps)
        compare_ligand(out, L, i, ref, rows, k, w.restarts, "reversed bonds")
    moved, n = refine_against_oracle(lg, pocket, pk, L, out, k)
    assert moved > n // 2
    pocket.free()


def test_dock_refine_rank_pipeline(lgmod, tiny):
    """Dock (top-k with pivots) -> refine every kept pose in place (k poses per
    ligand, pivots from docking) -> rank ligands by their best refined pose, all
    against the oracle on the same inputs."""
    lg = lgmod
    import torch
    w, pk, L = tiny["w"], tiny["pocket"], tiny["ligs"]
    pocket = device_pocket(pk)
    k = 3
    dl = lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                           L.inv_bond_len, L.ref_point)
    rt = torch.from_numpy(tiny["r32"]).cuda()
    at = torch.from_numpy(tiny["a32"]).cuda()
    out = lg.lg_dock_batch(pocket, dl, rt, at, sweeps=w.sweeps, top_k=k, trans_samples=w.angle_samples,
                           trans_step=oracle.trans_step(w.angle_samples), clash_dist2=oracle.CLASH2)
    res = lg.lg_refine(pocket, lg.docked_poses(dl, out), lg.refine_params(clash_dist2=oracle.CLASH2, poses_per_ligand=k))
    top_m = 20
    rk = lg.lg_rank(pocket, res["score"], k, top_m)
    torch.cuda.synchronize()
    h = {key: v.cpu().numpy() for key, v in out.items()}
    r = {key: v.cpu().numpy() for key, v in res.items()}
    ref_scores = np.zeros((L.n, k))
    for i in range(L.n):
        ref = dock_oracle(pk, L, i, tiny["r32"], tiny["a32"], T=w.angle_samples, S=w.sweeps)
        idx = oracle.topk(ref["final"], k)
        lig = L.ligand(i)
        for q in range(k):
            P = ref["pivots"][idx[q]]
            np.testing.assert_array_equal(h["pivot"][i, q].astype(np.float64), P, err_msg=f"pivot {i},{q}")
            s, best, _ = oracle.refine(lig, pk, ref["poses"][idx[q]], P, bits=32)
            got = pose_of(r, L, i, q, k).astype(np.float64)
            np.testing.assert_array_equal(got, best, err_msg=f"refined pose of ligand {i} rank {q}")
            assert r["score"][i * k + q] == s
            ref_scores[i, q] = s
    ids, vals, members = oracle.rank(ref_scores.reshape(-1), k, top_m)
    np.testing.assert_array_equal(rk["top_idx"].cpu().numpy(), ids)
    np.testing.assert_array_equal(rk["top_score"].cpu().numpy().astype(np.float64), vals)
    np.testing.assert_array_equal(rk["top_member"].cpu().numpy(), members)
    # ranking a single score per ligand through lg_score's top_m agrees with lg_rank
    one = lg.lg_rank(pocket, res["score"], 1, 10)
    ids1, vals1, _ = oracle.rank(ref_scores.reshape(-1), 1, 10)
    np.testing.assert_array_equal(one["top_idx"].cpu().numpy(), ids1)
    pocket.free()



def test_refine_two_poses_per_wavefront(lgmod, tiny):
    """Ligands of at most 32 atoms with k >= 2 poses are refined two poses per
    wavefront (both halves of a wavefront run one ligand's control flow): with
    k = 2 and k = 5 (a wavefront with one pose), bonds listed parents first
    (matrices built up front) and children first (sequential torsions), and
    ligands on both sides of 32 atoms, every refined pose and score equals the
    FP32 oracle's bitwise; k = 1 takes the one-pose kernel and agrees too."""
    lg = lgmod
    import torch
    w, pk = tiny["w"], tiny["pocket"]
    base = tiny["ligs"].subset(np.arange(20))
    assert (base.n_atoms <= 32).sum() >= 5 and (base.n_atoms > 32).sum() >= 5
    pocket = device_pocket(pk)
    rt = torch.from_numpy(tiny["r32"]).cuda()
    at = torch.from_numpy(tiny["a32"]).cuda()
    for label, L in (("parents first", base), ("children first", reversed_bonds(base))):
        dl = lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                               L.inv_bond_len, L.ref_point)
        for k in (1, 2, 5):
            say(f"refine pairs: {label}, k = {k}")
            out = lg.lg_dock_batch(pocket, dl, rt, at, sweeps=w.sweeps, top_k=k, trans_samples=w.angle_samples,
                                   trans_step=oracle.trans_step(w.angle_samples), clash_dist2=oracle.CLASH2)
            res = lg.lg_refine(pocket, lg.docked_poses(dl, out),
                               lg.refine_params(clash_dist2=oracle.CLASH2, poses_per_ligand=k))
            torch.cuda.synchronize()
            h = {key: v.cpu().numpy() for key, v in out.items()}
            r = {key: v.cpu().numpy() for key, v in res.items()}
            moved = 0
            for i in range(L.n):
                lig = L.ligand(i)
                for q in range(k):
                    pose = pose_of(h, L, i, q, k).astype(np.float64)
                    sc, best, _ = oracle.refine(lig, pk, pose, h["pivot"][i, q].astype(np.float64), bits=32)
                    np.testing.assert_array_equal(pose_of(r, L, i, q, k).astype(np.float64), best,
                                                  err_msg=f"{label}, k={k}: ligand {i} (N={L.n_atoms[i]}) pose {q}")
                    assert r["score"][i * k + q] == sc, (label, k, i, q)
                    moved += not np.array_equal(best, pose)
            assert moved > L.n * k // 2
    pocket.free()


def test_autotune_keeps_results(lgmod):
    """The autotuner returns a valid tuning that the handle keeps, and docking
    under it gives the same bits as under the default tuning."""
    lg = lgmod
    import torch
    w = gen.WORKLOADS["mixed"]
    L = gen.workload_ligands(w, np.arange(600, dtype=np.int64))
    pk = gen.workload_pocket(w)
    r32, _ = gen.restarts(64, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    pocket = device_pocket(pk)
    kw = dict(T=w.angle_samples, S=1, top_k=4, mode=lg.LG_BUCKETED, trace=False)
    say("autotune: 600 mixed ligands, R=64, S=1")
    before = dock_gpu(pocket, L, r32, a32, **kw)
    dl = lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                           L.inv_bond_len, L.ref_point)
    t, ms = lg.lg_autotune(pocket, dl, torch.from_numpy(r32).cuda(), torch.from_numpy(a32).cuda(), sweeps=1,
                           top_k=4, trans_samples=w.angle_samples, trans_step=oracle.trans_step(w.angle_samples),
                           clash_dist2=oracle.CLASH2)
    kept = pocket.get_tuning()
    assert bytes(kept) == bytes(t) and ms > 0
    assert kept.use_graph == 1
    after = dock_gpu(pocket, L, r32, a32, **kw)
    for key in before:
        np.testing.assert_array_equal(before[key], after[key], err_msg=f"tuned vs default: {key}")
    say(f"autotune: {ms:.2f} ms, chunk {t.restart_chunk}, grid x{t.grid_scale}, "
        f"waves/block {list(t.waves_per_block)}, lazy clash {t.lazy_clash}, "
        f"{t.n_atom_clusters} x {t.n_rot_clusters} clusters")
    pocket.free()


def test_degenerate_cases(lgmod, tiny):
    """An empty batch through every call; A = T = 1 (only the identity sample)
    and S = 0 (no sweeps): the kept poses are the placements, bitwise as in the
    oracle."""
    lg = lgmod
    import torch
    w, pk, L = tiny["w"], tiny["pocket"], tiny["ligs"]
    pocket = device_pocket(pk)
    empty = L.subset(np.array([], np.int64))
    de = lg.device_ligands(empty.atom_offset, empty.tors_offset, empty.x, empty.y, empty.z, empty.frag_mask,
                           empty.tors_atoms, empty.inv_bond_len, empty.ref_point)
    rt = torch.from_numpy(tiny["r32"]).cuda()
    at = torch.from_numpy(tiny["a32"]).cuda()
    out = lg.lg_dock_batch(pocket, de, rt, at, sweeps=1, top_k=2, trans_samples=64, trans_step=0.0625,
                           clash_dist2=oracle.CLASH2)
    assert out["score"].numel() == 0 and out["x"].numel() == 0
    assert lg.lg_refine(pocket, de, lg.refine_params())["score"].numel() == 0
    assert lg.lg_score(pocket, de, lg.LG_TRILINEAR, grad=True)["score"].numel() == 0
    assert lg.lg_rank(pocket, torch.empty(0, device="cuda"), 4, 0)["top_idx"].numel() == 0

    sub = L.subset(np.arange(6))
    one = np.array([[1.0, 0.0]], np.float32)
    for A, S in ((1, 2), (64, 0)):
        a32 = one if A == 1 else tiny["a32"]
        say(f"degenerate: A = T = {A}, S = {S}")
        got = dock_gpu(pocket, sub, tiny["r32"], a32, T=A, S=S, top_k=4, mode=lg.LG_BUCKETED, trace=S > 0)
        for i in range(sub.n):
            ref = dock_oracle(pk, sub, i, tiny["r32"], a32, T=A, S=S)
            compare_ligand(got, sub, i, ref, np.arange(w.restarts), 4, w.restarts, f"A={A} S={S}")
            for r in range(w.restarts):
                start, P0 = oracle.place(sub.ligand(i), tiny["r32"][r].astype(np.float64),
                                         pk.center.astype(np.float64), bits=32)
                np.testing.assert_array_equal(ref["poses"][r], start)
    # refinement with no steps returns every pose unchanged with its trilinear
    # score (one and two poses per wavefront)
    dl = lg.device_ligands(sub.atom_offset, sub.tors_offset, sub.x, sub.y, sub.z, sub.frag_mask, sub.tors_atoms,
                           sub.inv_bond_len, sub.ref_point)
    for k in (1, 2):
        out = lg.lg_dock_batch(pocket, dl, rt, at, sweeps=w.sweeps, top_k=k, trans_samples=w.angle_samples,
                               trans_step=oracle.trans_step(w.angle_samples), clash_dist2=oracle.CLASH2)
        poses = lg.docked_poses(dl, out)
        res = lg.lg_refine(pocket, poses, lg.refine_params(steps=0, clash_dist2=oracle.CLASH2, poses_per_ligand=k))
        torch.cuda.synchronize()
        h = {key: v.cpu().numpy() for key, v in out.items()}
        r = {key: v.cpu().numpy() for key, v in res.items()}
        for c in ("x", "y", "z"):
            np.testing.assert_array_equal(r[c], h[c], err_msg=f"steps = 0, k = {k}: {c}")
        for i in range(sub.n):
            for q in range(k):
                pose = pose_of(h, sub, i, q, k).astype(np.float64)
                sc, best, acc = oracle.refine(sub.ligand(i), pk, pose, h["pivot"][i, q].astype(np.float64), bits=32,
                                              steps=0)
                np.testing.assert_array_equal(best, pose)
                assert r["score"][i * k + q] == sc and acc == 0
    pocket.free()


def test_bench_configuration_full_library(lgmod):
    """The benchmark's own configuration: the whole 100k mixed library in
    bench.py's tuning, docked through the graph replay.  Sampled restarts
    and one ligand's full top-10 against the oracle; at full size, properties
    that hold for every ligand: top-k sorted (equal scores: lower restart),
    kept scores equal to those restarts' final scores, every kept pose keeps
    its bond lengths and its rigid root piece about the pivot."""
    lg = lgmod
    import torch
    w = gen.WORKLOADS["mixed"]
    L = gen.workload_ligands(w)
    pk = gen.workload_pocket(w)
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    pocket = device_pocket(pk)
    rt, at = torch.from_numpy(r32).cuda(), torch.from_numpy(a32).cuda()
    T = w.angle_samples
    kw = dict(sweeps=w.sweeps, top_k=w.top_k, trans_samples=T, trans_step=oracle.trans_step(T),
              clash_dist2=oracle.CLASH2)
    import bench
    spec = bench.DEFAULT_TUNING
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
    say(f"bench configuration: {L.n} ligands, {bench.tuning_key(pocket.get_tuning())}")
    dl = lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                           L.inv_bond_len, L.ref_point)
    out = lg.lg_dock_batch(pocket, dl, rt, at, want_all_scores=True, **kw)
    out = lg.lg_dock_batch(pocket, dl, rt, at, want_all_scores=True, out=out, **kw)   # graph replay
    torch.cuda.synchronize()
    h = {key: v.cpu().numpy() for key, v in out.items()}
    pocket.free()
    k = w.top_k
    # properties over the whole library
    sc, rid, alls = h["score"], h["restart_id"], h["all_scores"]
    assert np.all(np.isfinite(alls))
    assert np.all((sc[:, :-1] > sc[:, 1:]) | ((sc[:, :-1] == sc[:, 1:]) & (rid[:, :-1] < rid[:, 1:])))
    np.testing.assert_array_equal(np.take_along_axis(alls, rid.astype(np.int64), 1), sc)
    assert np.all(sc[:, 0] == alls.max(1))
    N = L.n_atoms.astype(np.int64)
    base = k * L.atom_offset[:-1].astype(np.int64)
    lig_of_atom = np.repeat(np.arange(L.n), N)
    local = np.arange(L.atom_offset[-1]) - L.atom_offset[:-1][lig_of_atom]
    for q in (0, k - 1):
        idx = base[lig_of_atom] + q * N[lig_of_atom] + local
        xyz = np.stack([h["x"][idx], h["y"][idx], h["z"][idx]], 1).astype(np.float64)
        has_parent = L.parent >= 0
        child = np.nonzero(has_parent)[0]
        par = L.atom_offset[:-1][lig_of_atom[child]] + L.parent[child]
        blen = np.linalg.norm(xyz[child] - xyz[par], axis=1)
        # FP32 rigid moves keep lengths to ~1e-5 A; a corrupted pose is off by far more
        assert np.max(np.abs(blen - 1.5)) < 2e-3, f"rank {q}: bond lengths off by {np.max(np.abs(blen - 1.5))}"
        root = L.frag_mask == 0
        piv = h["pivot"][lig_of_atom, q].astype(np.float64)
        d_now = np.linalg.norm(xyz - piv, axis=1)
        ref_piv = L.ref_point.reshape(-1, 3)[lig_of_atom].astype(np.float64)
        x0 = np.stack([L.x, L.y, L.z], 1).astype(np.float64)
        d0 = np.linalg.norm(x0 - ref_piv, axis=1)
        assert np.max(np.abs(d_now[root] - d0[root])) < 2e-3
    say("bench configuration: properties hold for every ligand")
    # sampled restarts and one full ligand against the oracle
    rng = np.random.default_rng(3)
    for i in rng.choice(L.n, 8, replace=False):
        rows = np.sort(rng.choice(w.restarts, 3, replace=False))
        ref = dock_oracle(pk, L, int(i), r32, a32, T=T, S=w.sweeps, rows=rows)
        compare_ligand(h, L, int(i), ref, rows, k, w.restarts, "bench configuration")
    i = int(rng.integers(L.n))
    ref = dock_oracle(pk, L, i, r32, a32, T=T, S=w.sweeps)
    compare_ligand(h, L, i, ref, np.arange(w.restarts), k, w.restarts, "bench configuration, all restarts")


def test_valu_probe_is_below_the_derived_peak(lgmod, tiny):
    """The probe's sustained rates (the roofline's measured context) are
    positive and never above the FP32 vector peak, 256 CUs x 4 SIMDs x 32 lanes
    x 2.4 GHz; the single-operation kinds (an SGPR operand each, issued at one
    wave64 instruction per four cycles) stay below half of it."""
    lg = lgmod
    pocket = device_pocket(tiny["pocket"])
    peak = 256 * 4 * 32 * 2.4e9
    for kind, name in enumerate(lg.VALU_PROBE_KINDS):
        r = lg.lg_valu_probe(pocket, kind, 20000 if kind < 6 else 2000)
        say(f"valu probe {name}: {r / 1e12:.2f} T lane-op/s")
        assert 0.25 * peak < r < (0.51 if kind < 6 else 1.0) * peak, (name, r)
    with pytest.raises(lg.LgError):
        lg.lg_valu_probe(pocket, 9, 10)
    pocket.free()
