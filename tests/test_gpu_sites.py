"""Several docking sites in one call (a docking site: Sec. 2; twelve sites of
one target: Sec. 5.2).  Each site's results must equal a single-site bucketed
batch on that site bitwise, in both work orders, and the oracle on that site.
"""
import dataclasses

import numpy as np
import pytest

import gen
import oracle
from gpu_common import compare_ligand, device_ligands, device_pocket, dock_gpu, dock_oracle, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lgmod():
    import torch
    from paper_2303_06150_amd import lg
    assert torch.cuda.is_available()
    lg.load_library()
    return lg


def sites(n, count, seed):
    """`count` pockets of one grid size and spacing, with their own fields,
    centres (so origins) and far values."""
    out = []
    for s in range(count):
        c = (10.0 - 7.5 * s, -4.0 + 3.25 * s, 6.5 + 1.5 * s)
        pk = gen.pocket(n, 0.5, 40 + 10 * s, 300, seed + s, center=c)
        out.append(dataclasses.replace(pk, out_value=float(np.float32(0.25 * s))))
    return out


def dock_sites(lg, pockets, L, r32, a32, *, T, S, top_k, site_major):
    import torch
    rt = torch.from_numpy(np.ascontiguousarray(r32, np.float32)).cuda()
    at = torch.from_numpy(np.ascontiguousarray(a32, np.float32)).cuda()
    outs = lg.lg_dock_sites(pockets, device_ligands(L), rt, at, sweeps=S, top_k=top_k, trans_samples=T,
                            trans_step=oracle.trans_step(T), clash_dist2=oracle.CLASH2, site_major=site_major,
                            want_all_scores=True)
    torch.cuda.synchronize()
    return [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]


def check_against_single_site(lg, pks, pockets, L, r32, a32, *, T, S, top_k, label):
    single = [dock_gpu(p, L, r32, a32, T=T, S=S, top_k=top_k, mode=lg.LG_BUCKETED, trace=False) for p in pockets]
    for order in (True, False):
        say(f"{label}: {len(pockets)} sites, {'site by site' if order else 'interleaved'}")
        got = dock_sites(lg, pockets, L, r32, a32, T=T, S=S, top_k=top_k, site_major=order)
        for s, (g, ref) in enumerate(zip(got, single)):
            for key in g:
                np.testing.assert_array_equal(g[key], ref[key], err_msg=f"{label} site {s} order {order}: {key}")
    # the sites really differ: a site's results are not another's
    assert not np.array_equal(single[0]["all_scores"], single[1]["all_scores"])
    return single


def test_tiny_three_sites(lgmod, tiny):
    lg = lgmod
    w, L = tiny["w"], tiny["ligs"]
    pks = sites(32, 3, 21)
    pockets = [device_pocket(p) for p in pks]
    single = check_against_single_site(lg, pks, pockets, L, tiny["r32"], tiny["a32"], T=w.angle_samples,
                                       S=w.sweeps, top_k=w.top_k, label="tiny")
    rows = np.arange(w.restarts)
    for s in (1, 2):
        for i in range(0, L.n, 9):
            ref = dock_oracle(pks[s], L, i, tiny["r32"], tiny["a32"], T=w.angle_samples, S=w.sweeps)
            compare_ligand(single[s], L, i, ref, rows, w.top_k, w.restarts, f"tiny site {s}")
    for p in pockets:
        p.free()


def test_ragged_two_sites_full_samples(lgmod):
    """Every kernel instance (1..4 atom slots, K up to 32) at A=T=256."""
    lg = lgmod
    N = [3, 20, 63, 64, 65, 127, 128, 129, 200, 256]
    K = [0, 5, 12, 1, 20, 32, 8, 31, 16, 32]
    L = gen.ligands_from_sizes(np.arange(500, 500 + len(N)), 17, np.array(N), np.array(K))
    pks = sites(48, 2, 41)
    pockets = [device_pocket(p) for p in pks]
    r32, _ = gen.restarts(6, 9)
    a32, _ = gen.angles(256)
    single = check_against_single_site(lg, pks, pockets, L, r32, a32, T=256, S=1, top_k=2, label="ragged")
    for i in (0, 4, 9):
        ref = dock_oracle(pks[1], L, i, r32, a32, T=256, S=1)
        compare_ligand(single[1], L, i, ref, np.arange(6), 2, 6, "ragged site 1")
    for p in pockets:
        p.free()


def test_sites_validation_and_handle_reuse(lgmod, tiny):
    lg = lgmod
    w, L = tiny["w"], tiny["ligs"]
    pks = sites(32, 2, 5)
    pockets = [device_pocket(p) for p in pks]
    other = device_pocket(gen.pocket(40, 0.5, 40, 300, 7))
    with pytest.raises(lg.LgError, match="dimensions and spacing"):
        dock_sites(lg, [pockets[0], other], L, tiny["r32"], tiny["a32"], T=w.angle_samples, S=w.sweeps,
                   top_k=w.top_k, site_major=True)
    kw = dict(T=w.angle_samples, S=w.sweeps, top_k=w.top_k)
    before = dock_gpu(pockets[0], L, tiny["r32"], tiny["a32"], mode=lg.LG_BUCKETED, trace=False, **kw)
    dock_sites(lg, pockets, L, tiny["r32"], tiny["a32"], site_major=False, **kw)
    after = dock_gpu(pockets[0], L, tiny["r32"], tiny["a32"], mode=lg.LG_BUCKETED, trace=False, **kw)
    for key in before:
        np.testing.assert_array_equal(before[key], after[key], err_msg=f"single-site batch after sites: {key}")
    assert len(pockets[0].bucket_stats()) > 0
    for p in pockets + [other]:
        p.free()


def test_sites_single_site_and_empty_batch(lgmod, tiny):
    """One site is lg_dock_batch; an empty batch docks nothing and succeeds."""
    lg = lgmod
    w, L = tiny["w"], tiny["ligs"]
    pks = sites(32, 1, 9)
    pockets = [device_pocket(p) for p in pks]
    kw = dict(T=w.angle_samples, S=w.sweeps, top_k=w.top_k)
    ref = dock_gpu(pockets[0], L, tiny["r32"], tiny["a32"], mode=lg.LG_BUCKETED, trace=False, **kw)
    got = dock_sites(lg, pockets, L, tiny["r32"], tiny["a32"], site_major=True, **kw)[0]
    for key in ref:
        np.testing.assert_array_equal(got[key], ref[key], err_msg=key)
    E = L.subset(np.arange(0))
    assert E.n == 0
    out = dock_sites(lg, pockets, E, tiny["r32"], tiny["a32"], site_major=False, **kw)
    assert out[0]["score"].shape == (0, w.top_k)
    for p in pockets:
        p.free()


def test_sites_full_size_sampled(lgmod):
    """Three sites at the mixed workload's full per-ligand size (96^3 grid at
    0.375 A, R = A = T = 256, S = 3, top-10), 400 ligands spread over the
    library: every site equals its single-site batch bitwise, and sampled
    restarts of each site match the oracle on that site."""
    lg = lgmod
    import torch
    w = gen.WORKLOADS["mixed"]
    L = gen.workload_ligands(w, np.arange(0, w.n_ligands, 250))
    pks = []
    for s in range(3):
        c = (10.0 + 6.0 * np.cos(s), -4.0 + 6.0 * np.sin(s), 6.5 + 0.5 * s)
        pks.append(gen.pocket(w.grid_n, w.spacing, w.n_gauss, w.n_shell, w.seed + 1000 + s, center=c))
    pockets = [device_pocket(p) for p in pks]
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    kw = dict(T=w.angle_samples, S=w.sweeps, top_k=w.top_k)
    say(f"sites at full size: {L.n} ligands, 3 sites of {w.grid_n}^3")
    got = dock_sites(lg, pockets, L, r32, a32, site_major=True, **kw)
    rng = np.random.default_rng(3)
    for s, p in enumerate(pockets):
        ref = dock_gpu(p, L, r32, a32, mode=lg.LG_BUCKETED, trace=False, **kw)
        for key in ref:
            np.testing.assert_array_equal(got[s][key], ref[key], err_msg=f"site {s}: {key}")
        for i in rng.choice(L.n, 2, replace=False):
            rows = np.sort(rng.choice(w.restarts, 3, replace=False))
            o = dock_oracle(pks[s], L, int(i), r32, a32, T=w.angle_samples, S=w.sweeps, rows=rows)
            compare_ligand(got[s], L, int(i), o, rows, w.top_k, w.restarts, f"site {s}")
            say(f"  site {s} ligand {i} (N={L.n_atoms[i]}) restarts {rows.tolist()} ok")
    for p in pockets:
        p.free()
