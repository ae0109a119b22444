"""Docking and refinement at the edge of the pocket box, with a far value other
than zero, against the oracle.

The tiny workload's box is moved so that the docking site sits 2 A inside its
low-x face and the value outside the box is -0.75 (a multiple of 2^-10, so the
scan sums stay exact).  Placements, rotations, translations and torsions then
carry many atoms out of the box (nearest node clamped to the border, far
value), and refinement moves atoms across the edge of the trilinear range (far
value, zero gradient).  Every ligand's docking trace, scores, top-k poses and
pivots, and the refinement of its kept poses with one and with two poses per
wavefront, must equal the FP32 oracle's bitwise; so must the scores of poses
placed across the low-x and the high-z faces, with their adjoint checked
against the FP64 oracle.
"""
import dataclasses

import numpy as np
import pytest

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


@pytest.fixture(scope="module")
def border(tiny):
    pk = tiny["pocket"]
    origin = pk.origin.copy()
    origin[0] = np.float32(pk.center[0] - 2.0)
    return dataclasses.replace(pk, origin=origin, out_value=-0.75)


def test_dock_at_the_box_edge_with_far_value(lgmod, tiny, border):
    lg = lgmod
    w, L, pk = tiny["w"], tiny["ligs"], border
    # the border is really crossed: at placement (restart 0, no rotation) some
    # atoms of most ligands lie outside the box
    out_x = [(L.x[L.atom_offset[i]:L.atom_offset[i + 1]] - L.ref_point[3 * i] + pk.center[0] < pk.origin[0]).any()
             for i in range(L.n)]
    assert np.mean(out_x) > 0.5
    pocket = device_pocket(pk)
    kw = dict(T=w.angle_samples, S=w.sweeps, top_k=w.top_k)
    for mode in (lg.LG_BUCKETED, lg.LG_PLAIN):
        say(f"box edge, far value -0.75: mode {mode}")
        out = dock_gpu(pocket, L, tiny["r32"], tiny["a32"], mode=mode, **kw)
        rows = np.arange(w.restarts)
        for i in range(L.n):
            ref = dock_oracle(pk, L, i, tiny["r32"], tiny["a32"], T=w.angle_samples, S=w.sweeps)
            compare_ligand(out, L, i, ref, rows, w.top_k, w.restarts, f"box edge mode {mode}")
    pocket.free()


@pytest.mark.parametrize("k", [1, 2])
def test_refine_at_the_box_edge_with_far_value(lgmod, tiny, border, k):
    """k = 1: one pose per wavefront; k = 2: two poses per wavefront for the
    ligands of at most 32 atoms."""
    lg = lgmod
    import torch
    w, L, pk = tiny["w"], tiny["ligs"], border
    pocket = device_pocket(pk)
    rt = torch.from_numpy(tiny["r32"]).cuda()
    at = torch.from_numpy(tiny["a32"]).cuda()
    dl = lg.device_ligands(L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms,
                           L.inv_bond_len, L.ref_point)
    out = lg.lg_dock_batch(pocket, dl, rt, at, sweeps=w.sweeps, top_k=k, trans_samples=w.angle_samples,
                           trans_step=oracle.trans_step(w.angle_samples), clash_dist2=oracle.CLASH2)
    res = lg.lg_refine(pocket, lg.docked_poses(dl, out),
                       lg.refine_params(clash_dist2=oracle.CLASH2, poses_per_ligand=k))
    torch.cuda.synchronize()
    h = {key: v.cpu().numpy() for key, v in out.items()}
    r = {key: v.cpu().numpy() for key, v in res.items()}
    moved = outside = 0
    for i in range(L.n):
        lig = L.ligand(i)
        for q in range(k):
            pose = pose_of(h, L, i, q, k).astype(np.float64)
            sc, best, _ = oracle.refine(lig, pk, pose, h["pivot"][i, q].astype(np.float64), bits=32)
            np.testing.assert_array_equal(pose_of(r, L, i, q, k).astype(np.float64), best,
                                          err_msg=f"k={k}: ligand {i} (N={L.n_atoms[i]}) pose {q}")
            assert r["score"][i * k + q] == sc, (k, i, q)
            moved += not np.array_equal(best, pose)
            outside += bool((best[:, 0] < pk.origin[0]).any())
    say(f"refined at the box edge (k = {k}): {moved} poses moved, {outside} with atoms outside the box")
    assert moved > L.n * k // 2
    assert outside > 0
    pocket.free()


def test_score_and_adjoint_across_the_box_faces(lgmod, tiny, border):
    """lg_score on poses that straddle the low-x face (the moved box) or the
    high-z face: nearest and trilinear scores equal the FP32 oracle's bitwise
    (atoms outside take the far value), the adjoint at zero moves the FP64
    oracle's to 1e-4 of its largest component (zero gradient outside the
    trilinear range)."""
    lg = lgmod
    import torch
    pk, L = border, tiny["ligs"]
    pocket = device_pocket(pk)
    rng = np.random.default_rng(11)
    hi_z = pk.origin[2] + (pk.grid.shape[0] - 1) * pk.spacing
    shift = np.repeat(pk.center[None].astype(np.float64), L.n, 0)
    low = np.arange(L.n) % 2 == 0
    shift[low, 0] = pk.origin[0] + rng.uniform(-2, 2, size=low.sum())
    shift[~low, 2] = hi_z + rng.uniform(-2, 2, size=(~low).sum())
    shift = shift.astype(np.float32)
    lig_of = np.repeat(np.arange(L.n), L.n_atoms)
    cen = np.stack([L.ref_point[0::3], L.ref_point[1::3], L.ref_point[2::3]], 1)
    xs = (L.x - cen[lig_of, 0] + shift[lig_of, 0]).astype(np.float32)
    ys = (L.y - cen[lig_of, 1] + shift[lig_of, 1]).astype(np.float32)
    zs = (L.z - cen[lig_of, 2] + shift[lig_of, 2]).astype(np.float32)
    outside = (xs < pk.origin[0]) | (zs > hi_z)
    inside = ~outside
    per_lig_out = np.bincount(lig_of, weights=outside, minlength=L.n)
    per_lig_in = np.bincount(lig_of, weights=inside, minlength=L.n)
    assert ((per_lig_out > 0) & (per_lig_in > 0)).mean() > 0.5   # most poses straddle a face
    dl = lg.device_ligands(L.atom_offset, L.tors_offset, xs, ys, zs, L.frag_mask, L.tors_atoms,
                           L.inv_bond_len, shift.reshape(-1))
    say("lg_score across the box faces, far value -0.75")
    near = lg.lg_score(pocket, dl, lg.LG_NEAREST)["score"].cpu().numpy()
    tri = lg.lg_score(pocket, dl, lg.LG_TRILINEAR, grad=True)
    torch.cuda.synchronize()
    ts, tg = tri["score"].cpu().numpy(), tri["grad"].cpu().numpy()
    worst = 0.0
    for i in range(L.n):
        a0, a1 = L.atom_offset[i], L.atom_offset[i + 1]
        xyz = np.stack([xs[a0:a1], ys[a0:a1], zs[a0:a1]], 1).astype(np.float64)
        assert near[i] == oracle.score(pk, xyz, 0, 32), i
        assert ts[i] == oracle.score(pk, xyz, 1, 32), i
        _, g64 = oracle.pose_grad(L.ligand(i), pk, xyz, shift[i].astype(np.float64))
        K = int(L.n_tors[i])
        g = tg[6 * i + L.tors_offset[i]: 6 * i + L.tors_offset[i] + 6 + K]
        worst = max(worst, np.abs(g - g64).max() / max(np.abs(g64).max(), 1e-3))
    assert worst < 1e-4, worst
    pocket.free()
