"""Properties of the seeded input generators (shared by the oracle and the GPU path)."""
import numpy as np

import gen
from conftest import topo_distances


def test_same_seed_same_bytes_and_item_streams():
    w = gen.WORKLOADS["mixed"]
    a = gen.workload_ligands(w, np.arange(50))
    b = gen.workload_ligands(w, np.arange(50))
    for f in ("x", "y", "z", "frag_mask", "tors_atoms", "inv_bond_len", "ref_point"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    # ligand 37 does not depend on the batch it sits in
    c = gen.workload_ligands(w, np.array([37, 3]))
    la, lc = a.ligand(37), c.ligand(0)
    np.testing.assert_array_equal(la["xyz"], lc["xyz"])
    np.testing.assert_array_equal(la["frag_mask"], lc["frag_mask"])
    p1 = gen.pocket(24, 0.5, 10, 50, 3)
    p2 = gen.pocket(24, 0.5, 10, 50, 3)
    np.testing.assert_array_equal(p1.grid, p2.grid)


def test_ligand_geometry_rules():
    w = gen.WORKLOADS["tiny"]
    L = gen.workload_ligands(w)
    for i in range(L.n):
        lig = L.ligand(i)
        x = lig["xyz64"]
        par = lig["parent"]
        N = lig["N"]
        assert par[0] == -1 and np.all(par[1:] < np.arange(1, N))      # preorder: parent before child
        for c in range(1, N):
            assert abs(np.linalg.norm(x[c] - x[par[c]]) - 1.5) < 1e-12
        # every bond angle at an atom is at least 100 degrees
        nbrs = [[] for _ in range(N)]
        for c in range(1, N):
            nbrs[c].append(par[c]); nbrs[par[c]].append(c)
        for a in range(N):
            for p in range(len(nbrs[a])):
                for q in range(p + 1, len(nbrs[a])):
                    u = x[nbrs[a][p]] - x[a]; v = x[nbrs[a][q]] - x[a]
                    ang = np.degrees(np.arccos(u @ v / np.linalg.norm(u) / np.linalg.norm(v)))
                    assert ang >= 100 - 1e-6
        # the input is clash-free: atoms 3+ bonds apart are at least 2.4 A apart
        D = topo_distances(par)
        d = np.linalg.norm(x[:, None] - x[None], axis=-1)
        assert np.all(d[D >= 3] >= 2.4 - 1e-9)
        # rotatable bonds: (parent, child), both of degree >= 2, ordered by child; fragments are
        # the child's subtree, a contiguous preorder range
        deg = np.array([len(n) for n in nbrs])
        b = lig["tors_b"]
        assert np.all(np.diff(b) > 0)
        for k in range(lig["K"]):
            assert lig["tors_a"][k] == par[b[k]]
            assert deg[b[k]] >= 2 and deg[par[b[k]]] >= 2
            mv = np.nonzero((lig["frag_mask"] >> k) & 1)[0]
            assert mv[0] == b[k] and np.all(np.diff(mv) == 1)
            sub = {b[k]}
            for c in range(b[k] + 1, N):
                if par[c] in sub:
                    sub.add(c)
            assert set(mv.tolist()) == sub


def test_size_distributions():
    w = gen.WORKLOADS["mixed"]
    n, k = gen.ligand_sizes(np.arange(20000), 0, 1, 12, 120, 0, 24)
    assert n.min() >= 12 and n.max() <= 120 and k.min() >= 0 and k.max() <= 24
    assert abs(np.median(n) - 38) <= 1
    assert 39 < n.mean() < 43
    t = gen.WORKLOADS["tiny"]
    n, k = gen.ligand_sizes(np.arange(2000), 0, 0, t.nlo, t.nhi, t.klo, t.khi)
    assert n.min() == 20 and n.max() == 40 and k.min() == 2 and k.max() == 6


def test_pocket_quantised_and_placed():
    p = gen.pocket(32, 0.5, 40, 300, 0)
    q = p.grid.astype(np.float64) * 1024
    assert np.all(q == np.round(q))
    assert p.grid.min() >= -63 and p.grid.max() <= 63
    np.testing.assert_allclose(p.origin, p.center - 15.5 * 0.5)
    assert p.grid.min() < -4.5            # the shell penalty is present
    assert p.grid[16, 16, 16] > 0         # the centre is attractive


def test_tables():
    a32, a64 = gen.angles(256)
    assert tuple(a32[0]) == (1.0, 0.0) and tuple(a32[64]) == (0.0, 1.0) and tuple(a32[128]) == (-1.0, 0.0)
    np.testing.assert_allclose(a64[:, 0], np.cos(2 * np.pi * np.arange(256) / 256), atol=1e-15)
    r32, r64 = gen.restarts(64)
    assert np.all(r64[0] == [1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0])
    for r in r64:
        M = r[:9].reshape(3, 3)
        np.testing.assert_allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(M) - 1) < 1e-12
        assert np.linalg.norm(r[9:]) <= 2.0


def test_angle_table_turn_symmetries():
    """The generated (cos, sin) table is exactly symmetric under quarter and half
    turns at every A that is a multiple of 4: sample j + A/4 holds (-s_j, c_j),
    j + A/2 holds (-c_j, -s_j), j + 3A/4 holds (s_j, -c_j).  The docking kernel
    checks this at start and then rotates once per four samples."""
    for A in (4, 64, 128, 256, 512, 1024):
        a, _ = gen.angles(A)
        c, s = a[:, 0], a[:, 1]
        q = A // 4
        j = np.arange(q)
        assert np.array_equal(c[j + q], -s[j]) and np.array_equal(s[j + q], c[j]), A
        assert np.array_equal(c[j + 2 * q], -c[j]) and np.array_equal(s[j + 2 * q], -s[j]), A
        assert np.array_equal(c[j + 3 * q], s[j]) and np.array_equal(s[j + 3 * q], -c[j]), A
        assert c[0] == 1.0 and s[0] == 0.0
