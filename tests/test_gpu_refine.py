"""Moved-pose scoring and its adjoint on the GPU against the FP64 oracle:
scores of moved poses, gradients against central finite differences of the
oracle's FP64 local move (h = 1e-4, voxel-face kinks skipped), and the
torch.autograd.Function wrapper."""
import numpy as np
import pytest

import oracle
from gpu_common import device_pocket, dock_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def docked(tiny):
    import torch
    from paper_2303_06150_amd import lg
    lg.load_library()
    w, pk, L = tiny["w"], tiny["pocket"], tiny["ligs"]
    pocket = device_pocket(pk)
    out = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], T=w.angle_samples, S=w.sweeps, top_k=1,
                   mode=lg.LG_BUCKETED, trace=False, all_scores=False)
    xyz = np.stack([out["x"], out["y"], out["z"]], 1)
    cen = np.stack([xyz[L.atom_offset[i]:L.atom_offset[i + 1]].astype(np.float64).mean(0)
                    for i in range(L.n)]).astype(np.float32)
    dl = lg.device_ligands(L.atom_offset, L.tors_offset, xyz[:, 0], xyz[:, 1], xyz[:, 2], L.frag_mask,
                           L.tors_atoms, L.inv_bond_len, cen.reshape(-1))
    yield dict(pocket=pocket, dl=dl, xyz=xyz, cen=cen, L=L, pk=pk)
    pocket.free()


def lig64(L, i, xyz):
    """Oracle view of pose i with FP64 copies of its FP32 data."""
    lig = L.ligand(i)
    a0, a1 = L.atom_offset[i], L.atom_offset[i + 1]
    lig["xyz64"] = xyz[a0:a1].astype(np.float64)
    lig["inv_len64"] = lig["inv_len"]
    return lig


def test_moved_scores_and_gradients_vs_finite_differences(docked):
    import torch
    from paper_2303_06150_amd import lg
    from paper_2303_06150_amd.autograd import move_layout
    L, pk, dl, xyz, cen = docked["L"], docked["pk"], docked["dl"], docked["xyz"], docked["cen"]
    rng = np.random.default_rng(11)
    idx_t, idx_w, idx_th, pob, size = move_layout(dl)
    q = np.zeros(size, np.float32)
    q[idx_t.cpu().numpy()] = rng.normal(scale=0.3, size=len(idx_t))
    q[idx_w.cpu().numpy()] = rng.normal(scale=0.3, size=len(idx_w))
    q[idx_th.cpu().numpy()] = rng.normal(scale=0.6, size=len(idx_th))
    res = lg.lg_score(docked["pocket"], dl, lg.LG_TRILINEAR, grad=True, moves=torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    s_gpu, g_gpu = res["score"].cpu().numpy(), res["grad"].cpu().numpy()
    h = 1e-4
    errs, skipped, total = [], 0, 0
    for i in range(L.n):
        lig = lig64(L, i, xyz)
        a0, a1 = L.atom_offset[i], L.atom_offset[i + 1]
        K = int(L.n_tors[i])
        off = 6 * i + L.tors_offset[i]
        qi = q[off:off + 6 + K].astype(np.float64)
        P = cen[i].astype(np.float64)
        moved, _ = oracle.apply_move(lig, xyz[a0:a1].astype(np.float64), P, qi)
        assert s_gpu[i] == pytest.approx(oracle.score(pk, moved, 1, 64), rel=1e-4, abs=1e-3)
        fd = np.zeros(6 + K)
        kink = np.zeros(6 + K, bool)
        for c in range(6 + K):
            e = np.zeros(6 + K)
            e[c] = h
            xp, _ = oracle.apply_move(lig, xyz[a0:a1].astype(np.float64), P, qi + e)
            xm, _ = oracle.apply_move(lig, xyz[a0:a1].astype(np.float64), P, qi - e)
            kink[c] = np.any(np.floor((xp - pk.origin) / pk.spacing) != np.floor((xm - pk.origin) / pk.spacing))
            fd[c] = (oracle.score(pk, xp, 1, 64) - oracle.score(pk, xm, 1, 64)) / (2 * h)
        g = g_gpu[off:off + 6 + K]
        scale = max(np.abs(fd).max() * 1e-2, 1e-6)
        for c in range(6 + K):
            total += 1
            if kink[c]:
                skipped += 1
                continue
            errs.append(abs(g[c] - fd[c]) / max(abs(fd[c]), scale))
    print(f"FD check: {len(errs)} parameters, {skipped} skipped at kinks, max rel err {max(errs):.2e}")
    assert max(errs) <= 1e-3
    assert skipped < 0.5 * total


def test_autograd_function_matches_library_gradient(docked):
    import torch
    from paper_2303_06150_amd import lg
    from paper_2303_06150_amd.autograd import RefineScore, move_layout
    dl, n = docked["dl"], docked["dl"].n
    rng = np.random.default_rng(12)
    t = torch.tensor(rng.normal(scale=0.2, size=(n, 3)), dtype=torch.float32, device="cuda", requires_grad=True)
    w = torch.tensor(rng.normal(scale=0.2, size=(n, 3)), dtype=torch.float32, device="cuda", requires_grad=True)
    th = torch.tensor(rng.normal(scale=0.3, size=dl.total_torsions), dtype=torch.float32, device="cuda",
                      requires_grad=True)
    s = RefineScore.apply(t, w, th, docked["pocket"], dl)
    weights = torch.linspace(0.5, 1.5, n, device="cuda")
    (s * weights).sum().backward()
    idx_t, idx_w, idx_th, pob, size = move_layout(dl)
    q = torch.zeros(size, device="cuda")
    q[idx_t] = t.detach().reshape(-1)
    q[idx_w] = w.detach().reshape(-1)
    q[idx_th] = th.detach()
    res = lg.lg_score(docked["pocket"], dl, lg.LG_TRILINEAR, grad=True, moves=q)
    torch.cuda.synchronize()
    torch.testing.assert_close(s, res["score"])
    torch.testing.assert_close(t.grad, res["grad"][idx_t].reshape(n, 3) * weights[:, None])
    torch.testing.assert_close(w.grad, res["grad"][idx_w].reshape(n, 3) * weights[:, None])
    torch.testing.assert_close(th.grad, res["grad"][idx_th] * weights[pob])
    # at zero moves the moved-pose path equals plain scoring of the poses
    z = lg.lg_score(docked["pocket"], dl, lg.LG_TRILINEAR, grad=True, moves=torch.zeros(size, device="cuda"))
    p0 = lg.lg_score(docked["pocket"], dl, lg.LG_TRILINEAR, grad=True)
    torch.cuda.synchronize()
    torch.testing.assert_close(z["score"], p0["score"], rtol=0, atol=0)
    torch.testing.assert_close(z["grad"], p0["grad"], rtol=2e-5, atol=2e-5)
