"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks the oracle against an independent statement of the same fact:
closed forms on constant / linear / single-voxel grids, voxel-shift invariance,
rotations rebuilt with scipy's Rotation (a different parametrisation than the
oracle's fma matrix script), a brute-force all-pairs clash rule by bond
distance, exhaustive search over torsion angles, numpy's lexsort, and central
finite differences.  A dropped term, a wrong sign or axis, a transposed
matrix or an off-by-one voxel rule fails at least one of them.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import gen
import oracle
from conftest import topo_distances

CL2 = oracle.CLASH2


# ---------------------------------------------------------------- helpers (independent)
def np_nearest_index(pocket, xyz):
    """Nearest grid node by the plain definition round((x - o)/h), FP64."""
    n = np.array(pocket.grid.shape[::-1])
    f = (np.asarray(xyz) - pocket.origin.astype(np.float64)) / np.float64(pocket.spacing) + 0.5
    inside = np.all((f >= 0) & (f < n), axis=1)
    return np.floor(f).astype(np.int64), inside


def np_nearest_score(pocket, xyz):
    idx, inside = np_nearest_index(pocket, xyz)
    vals = np.full(len(idx), pocket.out_value, np.float64)
    ii = idx[inside]
    vals[inside] = pocket.grid[ii[:, 2], ii[:, 1], ii[:, 0]]
    return vals.sum()


def np_trilinear(pocket, xyz):
    """Textbook trilinear interpolation: sum of 8 corner values x product weights."""
    n = np.array(pocket.grid.shape[::-1])
    f = (np.asarray(xyz) - pocket.origin.astype(np.float64)) / np.float64(pocket.spacing)
    out = np.full(len(f), pocket.out_value, np.float64)
    for a, fa in enumerate(f):
        if not np.all((fa >= 0) & (fa < n - 1)):
            continue
        i = np.floor(fa).astype(int)
        w = fa - i
        s = 0.0
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    wt = (w[0] if dx else 1 - w[0]) * (w[1] if dy else 1 - w[1]) * (w[2] if dz else 1 - w[2])
                    s += wt * pocket.grid[i[2] + dz, i[1] + dy, i[0] + dx]
        out[a] = s
    return out


def make_pocket(grid, origin=(0.0, 0.0, 0.0), h=0.5, center=None):
    grid = np.ascontiguousarray(grid, np.float32)
    n = grid.shape[0]
    origin = np.asarray(origin, np.float32)
    if center is None:
        center = origin + np.float32((n - 1) * h / 2)
    return gen.Pocket(grid, origin, float(np.float32(h)), np.asarray(center, np.float32))


def lab_rotation(e, theta):
    v = np.zeros(3)
    v[e] = theta
    return Rotation.from_rotvec(v)


def scan_setup(tiny, i, row=3):
    lig = tiny["ligs"].ligand(i)
    xyz, P = oracle.place(lig, tiny["r64"][row], tiny["pocket"].center.astype(np.float64), bits=64, fp64_input=True)
    return lig, xyz, P


# ---------------------------------------------------------------- grids and lookups
def test_constant_grid_scores():
    g = np.full((16, 16, 16), 0.75, np.float32)
    pk = make_pocket(g, origin=(-4.0, -4.0, -4.0), h=0.5)
    rng = np.random.default_rng(1)
    xyz = rng.uniform(-3.0, 3.0, size=(37, 3))
    for bits in (32, 64):
        assert oracle.score(pk, xyz, 0, bits) == pytest.approx(37 * 0.75, abs=0)
        assert oracle.score(pk, xyz, 1, bits) == pytest.approx(37 * 0.75, rel=1e-6)
    # atoms outside the box contribute the far-field value (0)
    # nearest rule: f = (x - o)/h + 1/2 must lie in [0, n): x=-4.25 -> f=0 (in), x=-4.26 -> f<0 (out,
    # although truncation toward zero would give node 0), z=3.7 -> f=15.9 (in), z=3.76 -> f=16.02 (out)
    edge_in = np.array([[-4.25, 0, 0], [0, 0, 3.7]])
    edge_out = np.array([[50.0, 0, 0], [0, -50.0, 0], [-4.26, 0, 0], [0, 0, 3.76]])
    for bits in (32, 64):
        assert oracle.score(pk, edge_in, 0, bits) == 1.5
        assert oracle.score(pk, edge_out, 0, bits) == 0.0
    # trilinear needs the whole cell: f = (x - o)/h in [0, n-1)
    assert oracle.score(pk, np.array([[0, 0, 3.49]]), 1, 64) == pytest.approx(0.75)
    assert oracle.score(pk, np.array([[0, 0, 3.5]]), 1, 64) == 0.0


def test_single_voxel_counts_atoms_rounding_to_it():
    g = np.zeros((12, 12, 12), np.float32)
    g[5, 7, 3] = 1.0
    pk = make_pocket(g, origin=(1.0, 2.0, 3.0), h=0.5)
    rng = np.random.default_rng(2)
    node = np.array([1.0 + 3 * 0.5, 2.0 + 7 * 0.5, 3.0 + 5 * 0.5])
    xyz = node + rng.uniform(-0.6, 0.6, size=(400, 3))
    idx, inside = np_nearest_index(pk, xyz)
    # keep atoms clear of rounding boundaries (independent rule is FP64 math)
    frac = ((xyz - pk.origin) / 0.5 + 0.5) % 1.0
    ok = np.all((frac > 1e-4) & (frac < 1 - 1e-4), axis=1)
    xyz = xyz[ok]
    expect = np.sum(np.all(np_nearest_index(pk, xyz)[0] == [3, 7, 5], axis=1))
    assert expect > 20
    for bits in (32, 64):
        assert oracle.score(pk, xyz, 0, bits) == expect


@pytest.mark.parametrize("coef", [(0.25, 0.0, 0.0), (0.0, -0.5, 0.0), (0.125, 0.375, -0.25)])
def test_linear_grid_closed_forms(coef):
    n = 20
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    a, b, c = coef
    g = (a * ix + b * iy + c * iz).astype(np.float32)
    pk = make_pocket(g, origin=(-2.0, 1.0, 0.5), h=0.5)
    rng = np.random.default_rng(3)
    xyz = pk.origin + rng.uniform(0.3, (n - 1.3) * 0.5, size=(25, 3))
    f = (xyz - pk.origin) / 0.5
    # trilinear of a linear function is the function itself; its gradient is (a, b, c)/h
    s, per, grad = oracle.score(pk, xyz, 1, 64, per_atom=True, grad=True)
    np.testing.assert_allclose(per, a * f[:, 0] + b * f[:, 1] + c * f[:, 2], atol=1e-12)
    np.testing.assert_allclose(grad, np.tile(np.array(coef) / 0.5, (25, 1)), atol=1e-12)
    # nearest of a linear function = the function at the rounded node
    idx, inside = np_nearest_index(pk, xyz)
    assert inside.all()
    s0, per0 = oracle.score(pk, xyz, 0, 64, per_atom=True)
    np.testing.assert_allclose(per0, a * idx[:, 0] + b * idx[:, 1] + c * idx[:, 2], atol=1e-12)


def test_trilinear_matches_textbook_and_edges(tiny):
    pk = tiny["pocket"]
    rng = np.random.default_rng(4)
    n = pk.grid.shape[0]
    xyz = pk.origin + rng.uniform(-1.0, (n + 0.5) * pk.spacing, size=(300, 3))
    s, per = oracle.score(pk, xyz, 1, 64, per_atom=True)
    np.testing.assert_allclose(per, np_trilinear(pk, xyz), atol=1e-12)
    # FP32 mode within FP32 rounding of the same quantity
    s32, per32 = oracle.score(pk, xyz, 1, 32, per_atom=True)
    np.testing.assert_allclose(per32, per, atol=2e-4)


def test_voxel_shift_invariance(tiny):
    """Shift a pose by whole voxels and the grid array by as many nodes."""
    pk = tiny["pocket"]
    v = np.array([2, -1, 3])
    g = pk.grid
    n = g.shape[0]
    g2 = np.zeros_like(g)
    src = [slice(max(0, -s), n - max(0, s)) for s in v[::-1]]
    dst = [slice(max(0, s), n - max(0, -s)) for s in v[::-1]]
    g2[tuple(dst)] = g[tuple(src)]
    pk2 = gen.Pocket(g2, pk.origin, pk.spacing, pk.center)
    lig = tiny["ligs"].ligand(5)
    out = oracle.dock_ligand(lig, pk, tiny["r64"][:4], tiny["a64"], 64, 1, oracle.trans_step(64), CL2,
                             bits=64, fp64_input=True)
    for pose in out["poses"]:
        shifted = pose + v * pk.spacing
        assert oracle.score(pk2, shifted, 0, 64) == oracle.score(pk, pose, 0, 64)
        assert oracle.score(pk2, shifted, 1, 64) == pytest.approx(oracle.score(pk, pose, 1, 64), abs=1e-12)
        assert oracle.score(pk, pose, 0, 64) == np_nearest_score(pk, pose)


# ---------------------------------------------------------------- placement and moves
def test_placement_matches_matrix_product(tiny):
    lig = tiny["ligs"].ligand(3)
    c = tiny["pocket"].center.astype(np.float64)
    for r in (0, 1, 7):
        row = tiny["r64"][r]
        xyz, P = oracle.place(lig, row, c, bits=64, fp64_input=True)
        M, t = row[:9].reshape(3, 3), row[9:]
        expect = (lig["xyz64"] - lig["ref64"]) @ M.T + c + t
        np.testing.assert_allclose(xyz, expect, atol=1e-12)
        np.testing.assert_allclose(P, c + t, atol=1e-15)


@pytest.mark.parametrize("e", [0, 1, 2])
def test_rotation_scan_against_scipy(tiny, e):
    pk = tiny["pocket"]
    A = 64
    moved = 0
    for i in range(6):
        lig, xyz, P = scan_setup(tiny, i, row=1 + i)
        j, xo, Po, sc, ok, best = oracle.scan(lig, pk, tiny["a64"], A, oracle.trans_step(A), CL2, 0, e,
                                              xyz, P, bits=64, fp64_input=True)
        expect_scores = []
        for jj in range(A):
            rot = lab_rotation(e, 2 * np.pi * jj / A)
            expect_scores.append(np_nearest_score(pk, rot.apply(xyz - P) + P))
        expect_scores = np.array(expect_scores)
        np.testing.assert_array_equal(sc, expect_scores)
        assert ok.all()
        assert j == int(np.argmax(expect_scores))           # first index of the maximum
        np.testing.assert_allclose(xo, lab_rotation(e, 2 * np.pi * j / A).apply(xyz - P) + P, atol=1e-12)
        np.testing.assert_array_equal(Po, P)
        moved += j != 0
    assert moved >= 3


@pytest.mark.parametrize("e", [0, 1, 2])
def test_translation_scan_closed_form(tiny, e):
    pk = tiny["pocket"]
    T = 64
    delta = oracle.trans_step(T)
    for i in range(4):
        lig, xyz, P = scan_setup(tiny, i, row=2 + i)
        j, xo, Po, sc, ok, best = oracle.scan(lig, pk, tiny["a64"], T, delta, CL2, 1, e, xyz, P,
                                              bits=64, fp64_input=True)
        offs = delta * np.array([m if m < T // 2 else m - T for m in range(T)], np.float64)
        expect = [np_nearest_score(pk, xyz + np.eye(3)[e] * d) for d in offs]
        np.testing.assert_array_equal(sc, expect)
        assert j == int(np.argmax(expect))
        np.testing.assert_allclose(xo, xyz + np.eye(3)[e] * offs[j], atol=1e-12)
        np.testing.assert_allclose(Po, P + np.eye(3)[e] * offs[j], atol=1e-12)


def brute_clash_free(xyz, D, clash2):
    """All pairs three or more bonds apart at least sqrt(clash2) apart."""
    d2 = ((xyz[:, None, :] - xyz[None, :, :]) ** 2).sum(-1)
    far = D >= 3
    return not np.any(d2[far] < clash2), np.min(np.abs(d2[far] - clash2)) if far.any() else 1.0


def torsion_pose(lig, xyz, k, theta):
    a, b = int(lig["tors_a"][k]), int(lig["tors_b"][k])
    u = xyz[b] - xyz[a]
    u = u / np.linalg.norm(u)
    rot = Rotation.from_rotvec(theta * u)
    out = xyz.copy()
    mv = ((lig["frag_mask"] >> k) & 1).astype(bool)
    mv[b] = False
    out[mv] = rot.apply(xyz[mv] - xyz[a]) + xyz[a]
    return out


def test_torsion_scan_against_brute_force(tiny):
    pk = tiny["pocket"]
    A = 64
    n_clash = 0
    n_checked = 0
    for i in range(12):
        lig, xyz, P = scan_setup(tiny, i, row=4 + i)
        D = topo_distances(lig["parent"])
        for k in range(lig["K"]):
            j, xo, Po, sc, ok, best = oracle.scan(lig, pk, tiny["a64"], A, oracle.trans_step(A), CL2, 2, k,
                                                  xyz, P, bits=64, fp64_input=True)
            scores, oks = [], []
            for jj in range(A):
                cand = torsion_pose(lig, xyz, k, 2 * np.pi * jj / A)
                scores.append(np_nearest_score(pk, cand))
                free, margin = brute_clash_free(cand, D, CL2)
                oks.append(True if jj == 0 else free)
                if jj and margin < 1e-9:
                    pytest.skip("sample within 1e-9 of the clash threshold")
            np.testing.assert_array_equal(sc, scores)
            np.testing.assert_array_equal(ok, oks)
            masked = np.where(oks, scores, -np.inf)
            assert j == int(np.argmax(masked))
            np.testing.assert_allclose(xo, torsion_pose(lig, xyz, k, 2 * np.pi * j / A), atol=1e-12)
            n_clash += int((~np.array(oks)).sum())
            n_checked += A
    assert n_checked > 1000
    assert n_clash > 0, "no clashing sample seen: the clash pin would be vacuous"


def test_greedy_two_torsions_not_above_exhaustive():
    """K=2, A=16: the greedy two-scan result is one of the A^2 joint choices."""
    pk = gen.workload_pocket(gen.WORKLOADS["tiny"])
    ids = np.arange(40)
    n, k = gen.ligand_sizes(ids, 7, 0, 14, 24, 2, 2)
    L = gen.ligands_from_sizes(ids, 7, n, k)
    A = 16
    a32, a64 = gen.angles(A)
    r32, r64 = gen.restarts(4, 7)
    done = 0
    for i in range(L.n):
        lig = L.ligand(i)
        if lig["K"] != 2:
            continue
        D = topo_distances(lig["parent"])
        xyz, P = oracle.place(lig, r64[1], pk.center.astype(np.float64), bits=64, fp64_input=True)
        j0, x1, P1, *_ = oracle.scan(lig, pk, a64, A, 0.0625, CL2, 2, 0, xyz, P, bits=64, fp64_input=True)
        j1, x2, P2, sc, ok, best = oracle.scan(lig, pk, a64, A, 0.0625, CL2, 2, 1, x1, P1, bits=64, fp64_input=True)
        greedy = np_nearest_score(pk, x2)
        assert greedy == best
        top = -np.inf
        for a in range(A):
            p1 = torsion_pose(lig, xyz, 0, 2 * np.pi * a / A)
            for b in range(A):
                p2 = torsion_pose(lig, p1, 1, 2 * np.pi * b / A)
                if brute_clash_free(p2, D, CL2)[0]:
                    top = max(top, np_nearest_score(pk, p2))
        assert greedy <= top
        done += 1
    assert done >= 5


def test_rigid_and_bond_invariants_fp64(tiny):
    pk = tiny["pocket"]
    for i in range(8):
        lig = tiny["ligs"].ligand(i)
        out = oracle.dock_ligand(lig, pk, tiny["r64"][:3], tiny["a64"], 64, 2, oracle.trans_step(64), CL2,
                                 bits=64, fp64_input=True)
        mask = lig["frag_mask"]
        same = mask[:, None] == mask[None, :]
        bonds = [(c, p) for c, p in enumerate(lig["parent"]) if p >= 0]
        root = mask == 0
        for r in range(3):
            start, P0 = oracle.place(lig, tiny["r64"][r], pk.center.astype(np.float64), bits=64, fp64_input=True)
            d0 = np.linalg.norm(start[:, None] - start[None], axis=-1)
            d1 = np.linalg.norm(out["poses"][r][:, None] - out["poses"][r][None], axis=-1)
            np.testing.assert_allclose(d1[same], d0[same], atol=1e-9)
            for c, p in bonds:
                assert abs(d1[c, p] - 1.5) < 1e-9
            assert not np.allclose(d1, d0)   # the torsions did move something
            # the pivot rides with the rigid root piece: rotations turn about it,
            # translations carry it along
            np.testing.assert_allclose(np.linalg.norm(out["poses"][r][root] - out["pivots"][r], axis=1),
                                       np.linalg.norm(start[root] - P0, axis=1), atol=1e-9)


def test_fp32_invariants_and_axis_bond_exact(tiny):
    pk = tiny["pocket"]
    lig = tiny["ligs"].ligand(9)
    out = oracle.dock_ligand(lig, pk, tiny["r32"].astype(np.float64)[:4], tiny["a32"].astype(np.float64), 64, 2,
                             oracle.trans_step(64), CL2, bits=32)
    mask = lig["frag_mask"]
    same = mask[:, None] == mask[None, :]
    for r in range(4):
        start, _ = oracle.place(lig, tiny["r32"][r].astype(np.float64), pk.center.astype(np.float64), bits=32)
        d0 = np.linalg.norm(start[:, None] - start[None], axis=-1)
        d1 = np.linalg.norm(out["poses"][r][:, None] - out["poses"][r][None], axis=-1)
        np.testing.assert_allclose(d1[same], d0[same], atol=1e-4)
        for c, p in enumerate(lig["parent"]):
            if p >= 0:
                assert abs(d1[c, p] - d0[c, p]) < 1e-4


def test_dock_monotone_and_final_score(tiny):
    pk = tiny["pocket"]
    for bits in (32, 64):
        for i in range(4):
            lig = tiny["ligs"].ligand(i)
            rt = tiny["r64"] if bits == 64 else tiny["r32"].astype(np.float64)
            at = tiny["a64"] if bits == 64 else tiny["a32"].astype(np.float64)
            out = oracle.dock_ligand(lig, pk, rt[:6], at, 64, 2, oracle.trans_step(64), CL2, bits=bits,
                                     fp64_input=(bits == 64), want_scan_scores=True)
            for r in range(6):
                ss = out["scan_scores"][r].reshape(-1)
                start, _ = oracle.place(lig, rt[r], pk.center.astype(np.float64), bits=bits, fp64_input=(bits == 64))
                assert ss[0] >= oracle.score(pk, start, 0, bits)
                assert np.all(np.diff(ss) >= 0)
                assert ss[-1] == oracle.score(pk, out["poses"][r], 0, bits)
                tri = np_trilinear(pk, out["poses"][r]).sum()
                assert out["final"][r] == pytest.approx(tri, rel=1e-5 if bits == 32 else 1e-12, abs=1e-4)


def test_degenerate_scans(tiny):
    """A=1 and T=1 leave the placed pose unchanged; K=0 gives rigid scans only."""
    pk = tiny["pocket"]
    lig = tiny["ligs"].ligand(2)
    one = np.array([[1.0, 0.0]])
    out = oracle.dock_ligand(lig, pk, tiny["r64"][:3], one, 1, 2, 0.0, CL2, bits=64, fp64_input=True)
    for r in range(3):
        start, _ = oracle.place(lig, tiny["r64"][r], pk.center.astype(np.float64), bits=64, fp64_input=True)
        np.testing.assert_array_equal(out["poses"][r], start)
        assert np.all(out["trace"][r] == 0)
    rigid = dict(lig)
    rigid["K"] = 0
    rigid["tors_a"] = rigid["tors_a"][:0]
    rigid["tors_b"] = rigid["tors_b"][:0]
    rigid["inv_len"] = rigid["inv_len"][:0]
    rigid["inv_len64"] = rigid["inv_len64"][:0]
    rigid["frag_mask"] = np.zeros_like(rigid["frag_mask"])
    out = oracle.dock_ligand(rigid, pk, tiny["r64"][:2], tiny["a64"], 64, 2, oracle.trans_step(64), CL2,
                             bits=64, fp64_input=True)
    assert out["trace"].shape == (2, 2, 6)
    start, _ = oracle.place(rigid, tiny["r64"][1], pk.center.astype(np.float64), bits=64, fp64_input=True)
    d0 = np.linalg.norm(start[:, None] - start[None], axis=-1)
    d1 = np.linalg.norm(out["poses"][1][:, None] - out["poses"][1][None], axis=-1)
    np.testing.assert_allclose(d1, d0, atol=1e-9)


def test_topk_is_a_sort():
    rng = np.random.default_rng(5)
    s = np.round(rng.normal(size=300) * 4) / 4      # many exact ties
    for k in (1, 10, 64, 300):
        idx = oracle.topk(s, k)
        expect = np.lexsort((np.arange(len(s)), -s))[:k]
        np.testing.assert_array_equal(idx, expect)


def test_rank_is_a_grouped_selection():
    rng = np.random.default_rng(6)
    for g in (1, 3, 8):
        s = np.round(rng.normal(size=(97, g)) * 3) / 4       # ties within and across ligands
        ids, vals, members = oracle.rank(s.reshape(-1), g, 40)
        left = list(range(97))
        for q in range(40):
            # brute force: scan every remaining ligand and member, strict > keeps the first
            bi, bm, bv = -1, -1, -np.inf
            for i in left:
                for m in range(g):
                    if s[i, m] > bv:
                        bi, bm, bv = i, m, s[i, m]
            assert (ids[q], members[q], vals[q]) == (bi, bm, bv)
            left.remove(bi)


# ---------------------------------------------------------------- adjoint
def _fd_check(lig, pk, xyz, P, h=1e-4):
    s, g = oracle.pose_grad(lig, pk, xyz, P)
    n = 6 + lig["K"]
    fd = np.zeros(n)
    kink = np.zeros(n, bool)
    for q in range(n):
        e = np.zeros(n)
        e[q] = h
        xp = oracle.pose_map(lig, xyz, P, e)
        xm = oracle.pose_map(lig, xyz, P, -e)
        fp, fm = (xp - pk.origin) / pk.spacing, (xm - pk.origin) / pk.spacing
        kink[q] = np.any(np.floor(fp) != np.floor(fm))
        fd[q] = (oracle.score(pk, xp, 1, 64) - oracle.score(pk, xm, 1, 64)) / (2 * h)
    return g, fd, kink


def test_pose_grad_matches_central_differences(tiny):
    pk = tiny["pocket"]
    errs, skipped, total = [], 0, 0
    for i in range(10):
        lig = tiny["ligs"].ligand(i)
        out = oracle.dock_ligand(lig, pk, tiny["r64"][:3], tiny["a64"], 64, 1, oracle.trans_step(64), CL2,
                                 bits=64, fp64_input=True)
        for r in range(3):
            xyz = out["poses"][r]
            P = xyz.mean(0)
            g, fd, kink = _fd_check(lig, pk, xyz, P)
            scale = max(np.abs(fd).max() * 1e-2, 1e-12)
            for q in range(len(g)):
                total += 1
                if kink[q]:
                    skipped += 1
                    continue
                errs.append(abs(g[q] - fd[q]) / max(abs(fd[q]), scale))
    assert max(errs) <= 1e-3
    assert skipped < 0.5 * total


def test_pose_grad_linear_grid_closed_form(tiny):
    n = 40
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    al, be, ga = 0.25, -0.125, 0.5
    g = (al * ix + be * iy + ga * iz).astype(np.float32)
    pk = make_pocket(g, origin=(-10.0, -10.0, -10.0), h=0.5)
    lig = tiny["ligs"].ligand(4)
    xyz = lig["xyz64"] - lig["xyz64"].mean(0)
    P = np.array([0.3, -0.2, 0.1])
    s, grad = oracle.pose_grad(lig, pk, xyz, P)
    gv = np.array([al, be, ga]) / 0.5
    N = lig["N"]
    np.testing.assert_allclose(grad[:3], N * gv, atol=1e-9)
    np.testing.assert_allclose(grad[3:6], np.cross(xyz - P, gv).sum(0), atol=1e-9)
    for k in range(lig["K"]):
        a, b = lig["tors_a"][k], lig["tors_b"][k]
        u = (xyz[b] - xyz[a]) / np.linalg.norm(xyz[b] - xyz[a])
        mv = ((lig["frag_mask"] >> k) & 1).astype(bool)
        np.testing.assert_allclose(grad[6 + k], u @ np.cross(xyz[mv] - xyz[a], gv).sum(0), atol=1e-9)
    # constant grid: no force, no torque
    pk0 = make_pocket(np.full((n, n, n), 2.0, np.float32), origin=(-10.0, -10.0, -10.0), h=0.5)
    s0, g0 = oracle.pose_grad(lig, pk0, xyz, P)
    assert s0 == pytest.approx(2.0 * N)
    np.testing.assert_allclose(g0, 0, atol=1e-12)


def test_pose_map_reduces_to_rigid_moves(tiny):
    lig = tiny["ligs"].ligand(6)
    xyz = lig["xyz64"]
    P = xyz.mean(0)
    K = lig["K"]
    q = np.zeros(6 + K)
    q[:3] = [0.5, -1.0, 2.0]
    np.testing.assert_allclose(oracle.pose_map(lig, xyz, P, q), xyz + q[:3], atol=1e-14)
    q[:3] = 0
    q[3:6] = [0.3, -0.2, 0.4]
    rot = Rotation.from_rotvec(q[3:6])
    np.testing.assert_allclose(oracle.pose_map(lig, xyz, P, q), rot.apply(xyz - P) + P, atol=1e-12)
    q[3:6] = 0
    q[6 + K - 1] = 0.7
    np.testing.assert_allclose(oracle.pose_map(lig, xyz, P, q), torsion_pose(lig, xyz, K - 1, 0.7), atol=1e-12)
