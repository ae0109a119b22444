"""Pins of the oracle's local refinement: the local move against the independent
FP64 pose map (Rodrigues, normalised axes), its gradient against the
finite-difference-pinned adjoint, its clash rule against brute force over atoms
three or more bonds apart, and closed forms of the ascent on constant and
linear grids."""
import numpy as np
import pytest

import oracle
from conftest import topo_distances
from test_oracle_pins import make_pocket


def docked_poses(tiny, n_lig=6, rows=3):
    pk = tiny["pocket"]
    out = []
    for i in range(n_lig):
        lig = tiny["ligs"].ligand(i)
        d = oracle.dock_ligand(lig, pk, tiny["r64"][:rows], tiny["a64"], 64, 1, oracle.trans_step(64),
                               oracle.CLASH2, bits=64, fp64_input=True)
        for r in range(rows):
            xyz = d["poses"][r]
            out.append((lig, xyz, xyz.mean(0)))
    return out


def test_apply_move_matches_rodrigues_pose_map(tiny):
    rng = np.random.default_rng(7)
    for lig, xyz, P in docked_poses(tiny, 4, 2):
        K = lig["K"]
        for _ in range(5):
            q = np.concatenate([rng.normal(size=3), rng.normal(size=3) * 0.7, rng.normal(size=K) * 1.3])
            moved, Pm = oracle.apply_move(lig, xyz, P, q)
            np.testing.assert_allclose(moved, oracle.pose_map(lig, xyz, P, q), atol=1e-11)
            np.testing.assert_allclose(Pm, P + q[:3], atol=1e-14)


def test_move_grad_matches_pinned_adjoint(tiny):
    pk = tiny["pocket"]
    for lig, xyz, P in docked_poses(tiny, 5, 2):
        s1, g1 = oracle.move_grad(lig, pk, xyz, P)
        s0, g0 = oracle.pose_grad(lig, pk, xyz, P)
        assert s1 == pytest.approx(s0, abs=1e-12)
        np.testing.assert_allclose(g1, g0, atol=1e-10)


def test_clash_rule_matches_brute_force(tiny):
    rng = np.random.default_rng(8)
    seen = {True: 0, False: 0}
    for lig, xyz, P in docked_poses(tiny, 8, 1):
        D = topo_distances(lig["parent"])
        far = D >= 3
        for _ in range(12):
            q = np.concatenate([np.zeros(6), rng.uniform(-np.pi, np.pi, size=lig["K"])])
            moved, _ = oracle.apply_move(lig, xyz, P, q)
            d2 = ((moved[:, None] - moved[None]) ** 2).sum(-1)
            brute = not np.any(d2[far] < oracle.CLASH2)
            margin = np.min(np.abs(d2[far] - oracle.CLASH2))
            if margin < 1e-9:
                continue
            rule = oracle.move_clash_free(lig, moved)
            assert rule == brute
            seen[rule] += 1
    assert seen[True] > 5 and seen[False] > 5


def test_refine_invariants(tiny):
    pk = tiny["pocket"]
    improved = 0
    for lig, xyz, P in docked_poses(tiny, 6, 2):
        s_in = oracle.score(pk, xyz, 1, 64)
        s, out, acc = oracle.refine(lig, pk, xyz, P, bits=64, fp64_input=True)
        assert s >= s_in
        assert s == pytest.approx(oracle.score(pk, out, 1, 64), abs=1e-9)
        assert oracle.move_clash_free(lig, out)
        same = lig["frag_mask"][:, None] == lig["frag_mask"][None, :]
        d0 = np.linalg.norm(xyz[:, None] - xyz[None], axis=-1)
        d1 = np.linalg.norm(out[:, None] - out[None], axis=-1)
        np.testing.assert_allclose(d1[same], d0[same], atol=1e-9)
        for c, p in enumerate(lig["parent"]):
            if p >= 0:
                assert abs(d1[c, p] - 1.5) < 1e-9
        improved += s > s_in
        # FP32 refinement obeys the same invariants within FP32 rounding
        s32, out32, _ = oracle.refine(lig, pk, xyz, P, bits=32)
        assert s32 >= oracle.score(pk, xyz, 1, 32) - 1e-6
        assert oracle.move_clash_free(lig, out32, bits=32, fp64_input=False)
    assert improved >= 6


def single_atom():
    z = np.zeros(1)
    return dict(N=1, K=0, xyz=np.zeros((1, 3)), xyz64=np.zeros((1, 3)), parent=np.array([-1], np.int32),
                frag_mask=np.zeros(1, np.uint32), tors_a=np.zeros(0, np.int32), tors_b=np.zeros(0, np.int32),
                inv_len=z[:0], inv_len64=z[:0], ref=z.repeat(3), ref64=z.repeat(3))


@pytest.mark.parametrize("alpha,expect_step", [(0.25, 0.01 * 0.25 / 0.5), (40.0, 0.1)])
def test_refine_single_atom_on_linear_grid(alpha, expect_step):
    """One atom, pivot on the atom: no torque; every step moves +x by
    min(eta_t * alpha / h, clip_t); 50 accepted steps."""
    n = 64
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    pk = make_pocket((alpha * ix).astype(np.float32), origin=(-8.0, -8.0, -8.0), h=0.5)
    lig = single_atom()
    x0 = np.array([[-3.1, 0.2, 0.3]])
    s, out, acc = oracle.refine(lig, pk, x0, x0[0], bits=64, fp64_input=True)
    assert acc == 50
    np.testing.assert_allclose(out[0], x0[0] + [50 * expect_step, 0, 0], atol=1e-9)
    assert s == pytest.approx(alpha * (out[0, 0] + 8.0) / 0.5, abs=1e-9)


def test_refine_constant_grid_keeps_pose(tiny):
    pk = make_pocket(np.full((40, 40, 40), 1.25, np.float32), origin=(-10.0, -10.0, -10.0), h=0.5)
    lig = tiny["ligs"].ligand(3)
    xyz = lig["xyz64"] - lig["xyz64"].mean(0)
    s, out, acc = oracle.refine(lig, pk, xyz, np.zeros(3), bits=64, fp64_input=True)
    np.testing.assert_array_equal(out, xyz)
    assert s == pytest.approx(1.25 * lig["N"])
