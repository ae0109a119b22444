"""Boundary behaviour of the C ABI on the device: limits rejected before any
launch, the host-validated path enqueueing without waiting on the stream, and
host-side rejection of malformed bonds in the streamed pipeline."""
import numpy as np
import pytest

import gen
import oracle
from gpu_common import device_ligands, device_pocket, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lgmod():
    import torch
    from paper_2303_06150_amd import lg
    assert torch.cuda.is_available()
    lg.load_library()
    return lg


def test_work_item_limit_and_chunk_cap(lgmod, tiny):
    """n * ceil(R / restart_chunk) >= 2^30 work items is LG_ERR_LIMIT before any
    allocation or launch; restart_chunk above LG_MAX_RESTARTS is rejected."""
    lg = lgmod
    import torch
    pocket = device_pocket(tiny["pocket"])
    t = pocket.get_tuning()
    big = lg.lg_tuning.from_buffer_copy(t)
    big.restart_chunk = 65537
    with pytest.raises(lg.LgError) as e:
        pocket.set_tuning(big)
    assert e.value.status == lg.LG_ERR_INVALID_ARG
    one = lg.lg_tuning.from_buffer_copy(t)
    one.restart_chunk = 1
    pocket.set_tuning(one)
    n, R = 16384, 65536                        # 2^14 ligands x 2^16 chunks of one restart = 2^30 items
    ao = np.arange(n + 1, dtype=np.int32)      # one atom per ligand, no bonds
    dl = lg.device_ligands(ao, np.zeros(n + 1, np.int32), np.zeros(n), np.zeros(n), np.zeros(n),
                           np.zeros(n, np.uint32), np.zeros(0, np.int32), np.zeros(0, np.float32),
                           np.zeros(3 * n, np.float32))
    rt = torch.zeros((R, 12), dtype=torch.float32, device="cuda")
    at = torch.from_numpy(tiny["a32"]).cuda()
    with pytest.raises(lg.LgError) as e:
        lg.lg_dock_batch(pocket, dl, rt, at, sweeps=1, top_k=1, trans_samples=64, trans_step=0.0625,
                         clash_dist2=oracle.CLASH2, mode=lg.LG_BUCKETED)
    assert e.value.status == lg.LG_ERR_LIMIT and "2^30" in lg.lg_last_error()
    pocket.set_tuning(t)
    pocket.free()


def test_host_validated_call_does_not_wait(lgmod):
    """With host copies of offsets and bonds, lg_dock_batch returns while its
    work is still running, and gives the same bits as the device-checked call."""
    lg = lgmod
    import torch
    w = gen.WORKLOADS["mixed"]
    L = gen.workload_ligands(w, np.arange(8000))
    pk = gen.workload_pocket(w)
    r32, _ = gen.restarts(w.restarts, w.seed)
    a32, _ = gen.angles(w.angle_samples)
    pocket = device_pocket(pk)
    dl = device_ligands(L)
    rt, at = torch.from_numpy(r32).cuda(), torch.from_numpy(a32).cuda()
    kw = dict(sweeps=w.sweeps, top_k=w.top_k, trans_samples=w.angle_samples,
              trans_step=oracle.trans_step(w.angle_samples), clash_dist2=oracle.CLASH2, mode=lg.LG_BUCKETED)
    out = lg.lg_dock_batch(pocket, dl, rt, at, **kw)          # workspace and graph set up
    torch.cuda.synchronize()
    say(f"host-validated call: {L.n} mixed ligands, R = {w.restarts}")
    out = lg.lg_dock_batch(pocket, dl, rt, at, out=out, **kw)
    busy = not torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    assert busy, "the call waited for its own work"
    got = {k: v.cpu().numpy() for k, v in out.items()}
    dl.host_checks = False
    ref = lg.lg_dock_batch(pocket, dl, rt, at, **kw)
    torch.cuda.synchronize()
    for k in got:
        np.testing.assert_array_equal(got[k], ref[k].cpu().numpy(), err_msg=k)
    pocket.free()


def test_stream_rejects_a_bond_with_one_atom_twice(lgmod, tiny):
    lg = lgmod
    import torch
    L = tiny["ligs"]
    pocket = device_pocket(tiny["pocket"])
    ta = L.tors_atoms.copy()
    ta[3] = ta[2]
    with pytest.raises(lg.LgError) as e:
        lg.lg_dock_stream(pocket, L.atom_offset, L.tors_offset, L.x, L.y, L.z, L.frag_mask, ta, L.inv_bond_len,
                          L.ref_point, torch.from_numpy(tiny["r32"]).cuda(), torch.from_numpy(tiny["a32"]).cuda(),
                          sweeps=1, top_k=2, trans_samples=64, trans_step=oracle.trans_step(64),
                          clash_dist2=oracle.CLASH2, chunk=16)
    assert e.value.status == lg.LG_ERR_INVALID_ARG and "distinct" in lg.lg_last_error()
    pocket.free()
