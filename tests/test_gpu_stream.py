"""lg_dock_stream: a host-resident library streamed through the device in
chunks (pinned staging, copy-in / dock / copy-out overlapped, two buffer
slots) gives exactly what lg_dock_batch gives on the whole library."""
import numpy as np
import pytest

import gen
import oracle
from gpu_common import device_pocket, say

pytestmark = pytest.mark.gpu


def host_args(L):
    return (L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, L.tors_atoms, L.inv_bond_len, L.ref_point)


@pytest.mark.parametrize("n,chunk", [(3000, 700), (3000, 5000), (7, 1)])
def test_stream_equals_batch(n, chunk):
    import torch
    from paper_2303_06150_amd import lg
    lg.load_library()
    w = gen.WORKLOADS["mixed"]
    L = gen.workload_ligands(w, np.arange(n, dtype=np.int64))
    pk = gen.workload_pocket(w)
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    pocket = device_pocket(pk)
    rt, at = torch.from_numpy(r32).cuda(), torch.from_numpy(a32).cuda()
    T = w.angle_samples
    kw = dict(sweeps=w.sweeps, top_k=w.top_k, trans_samples=T, trans_step=oracle.trans_step(T),
              clash_dist2=oracle.CLASH2)
    say(f"stream: {n} mixed ligands in chunks of {chunk}")
    dl = lg.device_ligands(*host_args(L))
    ref = lg.lg_dock_batch(pocket, dl, rt, at, **kw)
    torch.cuda.synchronize()
    got = lg.lg_dock_stream(pocket, *host_args(L), rt, at, chunk=chunk, **kw)
    for key in ("score", "restart_id", "x", "y", "z", "pivot"):
        np.testing.assert_array_equal(got[key], ref[key].cpu().numpy(), err_msg=key)
    pocket.free()


def test_stream_rejects_bad_host_input():
    import torch
    from paper_2303_06150_amd import lg
    lg.load_library()
    w = gen.WORKLOADS["tiny"]
    L = gen.workload_ligands(w, np.arange(4, dtype=np.int64))
    pk = gen.workload_pocket(w)
    pocket = device_pocket(pk)
    r32, _ = gen.restarts(8, 0)
    a32, _ = gen.angles(16)
    bad = L.tors_atoms.copy()
    bad[1] = 999
    args = list(host_args(L))
    args[6] = bad
    with pytest.raises(lg.LgError) as e:
        lg.lg_dock_stream(pocket, *args, torch.from_numpy(r32).cuda(), torch.from_numpy(a32).cuda(), sweeps=1,
                          top_k=2, trans_samples=16, trans_step=0.25, clash_dist2=oracle.CLASH2, chunk=2)
    assert e.value.status == lg.LG_ERR_INVALID_ARG
    pocket.free()
