import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def tiny():
    """The tiny workload: 64 ligands, 32^3 grid, R=32, A=64, S=2."""
    import gen
    w = gen.WORKLOADS["tiny"]
    pocket = gen.workload_pocket(w)
    ligs = gen.workload_ligands(w)
    r32, r64 = gen.restarts(w.restarts, w.seed)
    a32, a64 = gen.angles(w.angle_samples)
    return dict(w=w, pocket=pocket, ligs=ligs, r32=r32, r64=r64, a32=a32, a64=a64)


def topo_distances(parent):
    """All-pairs bond counts of a tree given its parent array (BFS, numpy)."""
    N = len(parent)
    adj = [[] for _ in range(N)]
    for i, p in enumerate(parent):
        if p >= 0:
            adj[i].append(int(p))
            adj[int(p)].append(i)
    D = np.full((N, N), -1, np.int64)
    for s in range(N):
        D[s, s] = 0
        frontier = [s]
        while frontier:
            nxt = []
            for u in frontier:
                for v in adj[u]:
                    if D[s, v] < 0:
                        D[s, v] = D[s, u] + 1
                        nxt.append(v)
            frontier = nxt
    return D
