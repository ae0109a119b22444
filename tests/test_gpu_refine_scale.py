"""Refinement at full size: the mixed library's first 20,000 ligands, the top 64
poses of each from docking (96^3 grid, R = 256, A = T = 256, S = 3), 50 steps of
the clipped ascent on the trilinear grid about each pose's docking pivot.

Checked against the oracle on seeded samples: refined poses and scores bit for
bit (FP32); the adjoint against central differences of the FP64 oracle (h =
1e-4) on 1,000 poses at zero moves and 100 poses at random non-zero moves,
skipping parameters whose +-h evaluations cross a voxel face (the trilinear
score is only C0 there); the global ranking against the definition applied to
the refined scores."""
import numpy as np
import pytest

import gen
import oracle
from gpu_common import device_pocket, pose_of, say

pytestmark = pytest.mark.gpu

N_LIG, K_POSES = 20_000, 64


@pytest.fixture(scope="module")
def refined():
    import torch
    from paper_2303_06150_amd import lg
    lg.load_library()
    w = gen.WORKLOADS["mixed"]
    L = gen.workload_ligands(w, np.arange(N_LIG, dtype=np.int64))
    pk = gen.workload_pocket(w)
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    pocket = device_pocket(pk)
    dl = lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                           L.inv_bond_len, L.ref_point)
    T = w.angle_samples
    say(f"refine scale: docking {N_LIG} mixed ligands, top-{K_POSES}")
    out = lg.lg_dock_batch(pocket, dl, torch.from_numpy(r32).cuda(), torch.from_numpy(a32).cuda(),
                           sweeps=w.sweeps, top_k=K_POSES, trans_samples=T, trans_step=oracle.trans_step(T),
                           clash_dist2=oracle.CLASH2)
    say("refine scale: refining every kept pose")
    res = lg.lg_refine(pocket, lg.docked_poses(dl, out),
                       lg.refine_params(clash_dist2=oracle.CLASH2, poses_per_ligand=K_POSES))
    rk = lg.lg_rank(pocket, res["score"], K_POSES, 1000)
    torch.cuda.synchronize()
    d = dict(pk=pk, L=L, pocket=pocket, dl=dl,
             dock={k: v.cpu().numpy() for k, v in out.items()},
             ref={k: v.cpu().numpy() for k, v in res.items()},
             rank={k: v.cpu().numpy() for k, v in rk.items()})
    yield d
    pocket.free()


def sample_poses(n, seed):
    rng = np.random.default_rng(seed)
    flat = rng.choice(N_LIG * K_POSES, size=n, replace=False)
    return [(int(f) // K_POSES, int(f) % K_POSES) for f in np.sort(flat)]


def test_refined_poses_match_oracle(refined):
    L, pk, dock, ref = refined["L"], refined["pk"], refined["dock"], refined["ref"]
    for i, q in sample_poses(300, 41):
        pose = pose_of(dock, L, i, q, K_POSES).astype(np.float64)
        P = dock["pivot"][i, q].astype(np.float64)
        s, best, _ = oracle.refine(L.ligand(i), pk, pose, P, bits=32)
        np.testing.assert_array_equal(pose_of(ref, L, i, q, K_POSES).astype(np.float64), best,
                                      err_msg=f"refined pose of ligand {i} rank {q}")
        assert ref["score"][i * K_POSES + q] == s, (i, q)
    # refinement never loses score
    assert np.all(ref["score"].reshape(N_LIG, K_POSES) >= dock["score"])


def test_global_ranking(refined):
    ids, vals, members = oracle.rank(refined["ref"]["score"], K_POSES, 1000)
    rk = refined["rank"]
    np.testing.assert_array_equal(rk["top_idx"], ids)
    np.testing.assert_array_equal(rk["top_score"].astype(np.float64), vals)
    np.testing.assert_array_equal(rk["top_member"], members)


def _fd_errors(pocket, L, pk, dock, picks, q_of, h=1e-4):
    """Library gradient at the moves q_of(j) vs central differences of the FP64 oracle."""
    import torch
    from paper_2303_06150_amd import lg
    lig_ids = np.array([i for i, _ in picks])
    Lp = L.subset(lig_ids)
    xyz = np.concatenate([pose_of(dock, L, i, q, K_POSES) for i, q in picks])
    piv = np.stack([dock["pivot"][i, q] for i, q in picks]).astype(np.float32)
    dl = lg.device_ligands(Lp.atom_offset, Lp.tors_offset, xyz[:, 0], xyz[:, 1], xyz[:, 2], Lp.frag_mask,
                           Lp.tors_atoms, Lp.inv_bond_len, piv.reshape(-1))
    size = 6 * Lp.n + int(Lp.tors_offset[-1])
    qall = np.zeros(size, np.float32)
    for j in range(Lp.n):
        off = 6 * j + int(Lp.tors_offset[j])
        qall[off:off + 6 + int(Lp.n_tors[j])] = q_of(j, int(Lp.n_tors[j]))
    res = lg.lg_score(pocket, dl, lg.LG_TRILINEAR, grad=True, moves=torch.from_numpy(qall).cuda())
    torch.cuda.synchronize()
    g_all, s_all = res["grad"].cpu().numpy(), res["score"].cpu().numpy()
    errs, skipped, total = [], 0, 0
    for j in range(Lp.n):
        lig = Lp.ligand(j)
        a0, a1 = int(Lp.atom_offset[j]), int(Lp.atom_offset[j + 1])
        x0 = xyz[a0:a1].astype(np.float64)
        lig["xyz64"] = x0
        lig["inv_len64"] = lig["inv_len"]
        K = int(Lp.n_tors[j])
        off = 6 * j + int(Lp.tors_offset[j])
        qj = qall[off:off + 6 + K].astype(np.float64)
        P = piv[j].astype(np.float64)
        moved, _ = oracle.apply_move(lig, x0, P, qj)
        assert s_all[j] == pytest.approx(oracle.score(pk, moved, 1, 64), rel=1e-4, abs=1e-3)
        fd = np.zeros(6 + K)
        kink = np.zeros(6 + K, bool)
        for c in range(6 + K):
            e = np.zeros(6 + K)
            e[c] = h
            xp, _ = oracle.apply_move(lig, x0, P, qj + e)
            xm, _ = oracle.apply_move(lig, x0, P, qj - e)
            kink[c] = np.any(np.floor((xp - pk.origin) / pk.spacing) != np.floor((xm - pk.origin) / pk.spacing))
            fd[c] = (oracle.score(pk, xp, 1, 64) - oracle.score(pk, xm, 1, 64)) / (2 * h)
        g = g_all[off:off + 6 + K]
        floor = max(1e-2 * np.abs(fd).max(), 1e-6)
        for c in range(6 + K):
            total += 1
            if kink[c]:
                skipped += 1
                continue
            errs.append(abs(g[c] - fd[c]) / max(abs(fd[c]), floor))
    return np.array(errs), skipped, total


def test_adjoint_vs_finite_differences_at_zero(refined):
    picks = sample_poses(1000, 4)
    errs, skipped, total = _fd_errors(refined["pocket"], refined["L"], refined["pk"], refined["dock"], picks,
                                      lambda j, K: np.zeros(6 + K, np.float32))
    say(f"FD at zero: {len(errs)} parameters checked, {skipped}/{total} skipped at voxel faces "
        f"({100.0 * skipped / total:.1f} %), max rel err {errs.max():.2e}")
    assert errs.max() <= 1e-3
    assert skipped < 0.25 * total


def test_adjoint_vs_finite_differences_at_nonzero_moves(refined):
    rng = np.random.default_rng(44)
    picks = sample_poses(100, 45)

    def q_of(j, K):
        return np.concatenate([rng.normal(scale=0.2, size=3), rng.normal(scale=0.3, size=3),
                               rng.uniform(-0.5, 0.5, size=K)]).astype(np.float32)

    errs, skipped, total = _fd_errors(refined["pocket"], refined["L"], refined["pk"], refined["dock"], picks, q_of)
    say(f"FD at non-zero moves: {len(errs)} parameters checked, {skipped}/{total} skipped, "
        f"max rel err {errs.max():.2e}")
    assert errs.max() <= 1e-3
    assert skipped < 0.25 * total
