"""The global ranking kernels (radix select of the top m keys, bitonic sort) against
the oracle's ranking, which is pinned to a brute-force selection loop: sizes from
one ligand to 200 000, group sizes 1 to 64, m from 1 to a full sort, both sort paths
(m <= 4096 in one block, larger m through global merge steps), heavy exact ties,
-0 / +0, all-equal values."""
import numpy as np
import pytest

import oracle
from gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lgpocket():
    import torch
    import gen
    from paper_2303_06150_amd import lg
    assert torch.cuda.is_available()
    lg.load_library()
    pk = gen.pocket(8, 0.5, 4, 8, 0)
    p = lg.Pocket(torch.from_numpy(pk.grid).cuda(), pk.origin, pk.spacing, pk.center, pk.out_value)
    yield lg, p
    p.free()


def scores(n, group, kind, rng):
    if kind == "ties":       # few distinct values: many exact ties within and across groups
        s = rng.integers(-20, 20, size=n * group).astype(np.float32) / 8
    elif kind == "zeros":    # -0 and +0 only
        s = np.where(rng.random(n * group) < 0.5, np.float32(-0.0), np.float32(0.0)).astype(np.float32)
    elif kind == "equal":
        s = np.full(n * group, 1.25, np.float32)
    else:
        s = (rng.normal(size=n * group) * 30).astype(np.float32)
    return s


CASES = [
    (1, 1, 1, "normal"), (2, 3, 2, "ties"), (1000, 1, 1000, "ties"), (1000, 10, 7, "normal"),
    (5000, 4, 4096, "ties"), (5000, 4, 4097, "normal"), (20000, 64, 1000, "ties"),
    (70000, 1, 70000, "ties"), (200000, 2, 9000, "normal"), (3000, 5, 3000, "zeros"), (4500, 1, 4500, "equal"),
]


@pytest.mark.parametrize("n,group,m,kind", CASES)
def test_rank_matches_oracle(lgpocket, n, group, m, kind):
    import torch
    lg, pocket = lgpocket
    rng = np.random.default_rng(n + 7 * group + m)
    s = scores(n, group, kind, rng)
    say(f"rank: n={n} group={group} m={m} {kind}")
    rk = lg.lg_rank(pocket, torch.from_numpy(s).cuda(), group, m)
    torch.cuda.synchronize()
    ids, vals, members = oracle.rank(s.astype(np.float64), group, m)
    np.testing.assert_array_equal(rk["top_idx"].cpu().numpy(), ids)
    np.testing.assert_array_equal(rk["top_score"].cpu().numpy().astype(np.float64), vals)
    np.testing.assert_array_equal(rk["top_member"].cpu().numpy(), members)


def test_rank_back_to_back_calls_share_no_state(lgpocket):
    """A second, smaller call on the same handle starts from a clean selection."""
    import torch
    lg, pocket = lgpocket
    rng = np.random.default_rng(3)
    big = scores(50000, 2, "ties", rng)
    small = scores(300, 1, "normal", rng)
    lg.lg_rank(pocket, torch.from_numpy(big).cuda(), 2, 5000)
    rk = lg.lg_rank(pocket, torch.from_numpy(small).cuda(), 1, 17)
    torch.cuda.synchronize()
    ids, vals, _ = oracle.rank(small.astype(np.float64), 1, 17)
    np.testing.assert_array_equal(rk["top_idx"].cpu().numpy(), ids)
    np.testing.assert_array_equal(rk["top_score"].cpu().numpy().astype(np.float64), vals)
