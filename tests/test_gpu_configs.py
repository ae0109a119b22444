"""GPU parity on the remaining workload shapes: the uniform workload at full
size (10 000 ligands of 48 atoms and 8 rotatable bonds, 96^3 grid, R = A = T =
256, S = 3, top-10) and the replicated ligands of the batch-size experiment
(17 / 53 / 99 atoms, Sec. 5.2), plus the paper-experiment harnesses of bench.py
run end to end on small sizes."""
import numpy as np
import pytest

import gen
from gpu_common import compare_ligand, device_ligands, device_pocket, dock_gpu, dock_oracle, pose_of, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lgmod():
    import torch
    from paper_2303_06150_amd import lg
    assert torch.cuda.is_available()
    lg.load_library()
    return lg


def test_uniform_workload_sampled(lgmod):
    lg = lgmod
    w = gen.WORKLOADS["uniform"]
    L = gen.workload_ligands(w)
    assert L.n == 10000 and (L.n_atoms == 48).all() and (L.n_tors == 8).all()
    pk = gen.workload_pocket(w)
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    say(f"uniform: {L.n} ligands x 48 atoms, R={w.restarts} A=T={w.angle_samples} S={w.sweeps}")
    pocket = device_pocket(pk)
    out = dock_gpu(pocket, L, r32, a32, T=w.angle_samples, S=w.sweeps, top_k=w.top_k, mode=lg.LG_BUCKETED)
    rng = np.random.default_rng(1)
    for i in rng.choice(L.n, 6, replace=False):
        rows = np.sort(rng.choice(w.restarts, 3, replace=False))
        ref = dock_oracle(pk, L, int(i), r32, a32, T=w.angle_samples, S=w.sweeps, rows=rows)
        compare_ligand(out, L, int(i), ref, rows, w.top_k, w.restarts, "uniform")
        say(f"  ligand {i} restarts {rows.tolist()} ok")
    i = L.n - 1                                   # the last ligand: every restart, its top-10 and poses
    ref = dock_oracle(pk, L, i, r32, a32, T=w.angle_samples, S=w.sweeps)
    compare_ligand(out, L, i, ref, np.arange(w.restarts), w.top_k, w.restarts, "uniform all restarts")
    pocket.free()


@pytest.mark.parametrize("N", [17, 53, 99])
def test_bucket_size_replicas_match_oracle(lgmod, N):
    """Every replica in a batch of the batch-size experiment gets the oracle's
    top-10 of the single ligand: ids, scores, poses and pivots."""
    lg = lgmod
    w = gen.WORKLOADS["mixed"]
    pk = gen.workload_pocket(w)
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    L1 = gen.replica_ligand(N)
    count = 200
    L = gen.replicas(L1, count)
    say(f"replicas: {count} x {N} atoms, {int(L1.n_tors[0])} bonds")
    pocket = device_pocket(pk)
    out = dock_gpu(pocket, L, r32, a32, T=w.angle_samples, S=w.sweeps, top_k=w.top_k, mode=lg.LG_BUCKETED,
                   trace=False, all_scores=False)
    ref = dock_oracle(pk, L1, 0, r32, a32, T=w.angle_samples, S=w.sweeps)
    import oracle
    idx = oracle.topk(ref["final"], w.top_k)
    for i in range(count):
        np.testing.assert_array_equal(out["restart_id"][i], idx, err_msg=f"replica {i}")
        np.testing.assert_array_equal(out["score"][i].astype(np.float64), ref["final"][idx])
        np.testing.assert_array_equal(out["pivot"][i].astype(np.float64), ref["pivots"][idx])
        for q in range(w.top_k):
            np.testing.assert_array_equal(pose_of(out, L, i, q, w.top_k).astype(np.float64), ref["poses"][idx[q]])
    pocket.free()


def test_experiment_harnesses_run(lgmod):
    """bench.py's batch-size and cluster experiments run on small sizes and report
    what the paper's figures plot."""
    import torch
    import bench
    import oracle
    lg = lgmod
    w = gen.WORKLOADS["mixed"]
    pk = gen.workload_pocket(w)
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    pocket = device_pocket(pk)
    rt, at = torch.from_numpy(r32).cuda(), torch.from_numpy(a32).cuda()
    T = w.angle_samples
    kw = dict(sweeps=w.sweeps, top_k=w.top_k, trans_samples=T, trans_step=oracle.trans_step(T),
              clash_dist2=oracle.CLASH2)
    res = bench.experiment_bucket_size(lg, torch, pocket, rt, at, kw, say, sizes=(17, 53), multiples=(1, 3, 6),
                                       min_ligands=200)
    assert len(res["rows"]) == 6 and all(r["value"] > 0 and r["l_fill"] >= 1 for r in res["rows"])
    assert [r["ligands_per_batch"] for r in res["rows"][:3]] == [max(1, res["rows"][0]["l_fill"] * m // 3)
                                                                 for m in (1, 3, 6)]
    L = gen.workload_ligands(w, np.arange(1500))
    res = bench.experiment_clusters(lg, torch, pocket, device_ligands(L), rt, at, kw, L.n, say)
    assert len(res["rows"]) == 15 and res["rows"][0]["speedup_vs_one_cluster"] == 1.0
    assert {(r["atom_clusters"], r["rotamer_clusters"]) for r in res["rows"]} >= {(1, 1), (2, 2), (4, 8)}
    pocket.free()
