"""Shared helpers of the GPU parity tests: marshal generator outputs to the C ABI
and run the oracle on the same inputs."""
import sys

import numpy as np

import gen
import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_ligands(L: gen.Ligands):
    from paper_2303_06150_amd import lg
    return lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                             L.inv_bond_len, L.ref_point)


def device_pocket(pk: gen.Pocket, on_device=True):
    import torch
    from paper_2303_06150_amd import lg
    g = torch.from_numpy(pk.grid)
    if on_device:
        g = g.cuda()
    return lg.Pocket(g, pk.origin, pk.spacing, pk.center, pk.out_value, inv_spacing=pk.inv_spacing)


def dock_gpu(pocket, L, r32, a32, *, T, S, top_k, mode, trace=True, all_scores=True, trans_step=None):
    import torch
    from paper_2303_06150_amd import lg
    dl = device_ligands(L)
    rt = torch.from_numpy(np.ascontiguousarray(r32, np.float32)).cuda()
    at = torch.from_numpy(np.ascontiguousarray(a32, np.float32)).cuda()
    kmax = int(L.n_tors.max()) if L.n else 0
    out = lg.lg_dock_batch(pocket, dl, rt, at, sweeps=S, top_k=top_k, trans_samples=T,
                           trans_step=oracle.trans_step(T) if trans_step is None else trans_step,
                           clash_dist2=oracle.CLASH2, mode=mode, want_all_scores=all_scores,
                           trace_kmax=kmax if trace else None)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def dock_oracle(pk, L, i, r32, a32, *, T, S, rows=None):
    lig = L.ligand(i)
    rt = r32.astype(np.float64)
    if rows is not None:
        rt = rt[rows]
    return oracle.dock_ligand(lig, pk, rt, a32.astype(np.float64), T, S, oracle.trans_step(T), oracle.CLASH2,
                              bits=32)


def pose_of(out, L, i, q, k):
    """Rank-q pose of ligand i from the dock outputs ([N,3])."""
    a0, a1 = int(L.atom_offset[i]), int(L.atom_offset[i + 1])
    N = a1 - a0
    base = k * a0 + q * N
    return np.stack([out["x"][base:base + N], out["y"][base:base + N], out["z"][base:base + N]], 1)


def compare_ligand(out, L, i, ref, rows, top_k, R, label=""):
    """Compare GPU outputs of ligand i with the oracle on restart rows `rows`."""
    K = int(L.n_tors[i])
    gs = out["all_scores"][i][rows].astype(np.float64)
    bad = np.nonzero(gs != ref["final"])[0]
    assert len(bad) == 0, f"{label} ligand {i}: final scores differ at restarts {np.asarray(rows)[bad][:8]}: " \
                          f"gpu {gs[bad][:4]} oracle {ref['final'][bad][:4]}"
    if "trace" in out and ref["trace"] is not None:
        gt = out["trace"][i][rows][:, :, :6 + K]
        mism = np.argwhere(gt != ref["trace"])
        assert len(mism) == 0, f"{label} ligand {i}: trace differs at (restart,sweep,scan) {mism[:5].tolist()}"
    if len(rows) == R:
        idx = oracle.topk(ref["final"], top_k)
        np.testing.assert_array_equal(out["restart_id"][i], idx, err_msg=f"{label} ligand {i} top-k ids")
        np.testing.assert_array_equal(out["score"][i].astype(np.float64), ref["final"][idx])
        for q in range(top_k):
            np.testing.assert_array_equal(pose_of(out, L, i, q, top_k).astype(np.float64), ref["poses"][idx[q]],
                                          err_msg=f"{label} ligand {i} rank {q} pose")
            if "pivot" in out:
                np.testing.assert_array_equal(out["pivot"][i, q].astype(np.float64), ref["pivots"][idx[q]],
                                              err_msg=f"{label} ligand {i} rank {q} pivot")
