"""Host logic of bench.py (no GPU): the committed counter summaries it reads,
the roofline's work counts on hand-built ligands, and the bucket assignment."""
import os
import types

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def tuning_obj(spec):
    t = types.SimpleNamespace(**spec)
    t.n_atom_clusters = len(spec["atom_bounds"])
    t.n_rot_clusters = len(spec["rot_bounds"])
    return t


def parse(path):
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


@pytest.mark.parametrize("name,fields", [
    ("dock_bucket_1_4_mixed_traffic.txt", ("fetch_bytes_per_dispatch", "write_bytes_per_dispatch",
                                           "hbm_bytes_per_dispatch")),
    ("dock_bucket_1_4_mixed_valu.txt", ("valu_busy", "valu_issue_per_simd_cycle", "td_busy", "ta_busy", "l2_hit")),
    ("refine_mixed20k_counters.md", ("valu_issue_per_simd_cycle",)),
])
def test_committed_counter_summaries(name, fields, tmp_path, monkeypatch):
    """Each summary names its commands, the kernel source and tuning it was taken
    on, and positive figures; the bench uses it only for that source and tuning."""
    path = os.path.join(ROOT, "profiles", name)
    text = open(path).read()
    assert "rocprofv3 --pmc" in text and "bench.py" in text
    kv = parse(path)
    assert len(kv["source_sha256"]) == 16
    for f in fields:
        assert float(kv[f]) > 0, f
    assert float(kv.get("hbm_bytes_per_dispatch", 1)) == pytest.approx(
        float(kv.get("fetch_bytes_per_dispatch", 0.5)) + float(kv.get("write_bytes_per_dispatch", 0.5)), rel=1e-5)
    # read through bench's own reader in a copy of the tree whose source hash matches
    monkeypatch.setattr(bench, "source_hash", lambda *a: kv["source_sha256"])
    key = kv["tuning"]
    assert bench.read_profile_value(name, fields[0], key) == pytest.approx(float(kv[fields[0]]))
    assert bench.read_profile_value(name, fields[0], key + " other") is None
    monkeypatch.setattr(bench, "source_hash", lambda *a: "0" * 16)
    assert bench.read_profile_value(name, fields[0], key) is None
    assert bench.read_profile_value("no_such_summary.txt", fields[0], key) is None


def test_default_tuning_key_and_limits():
    t = tuning_obj(bench.DEFAULT_TUNING)
    assert bench.tuning_key(t) == "atoms [64, 128, 192, 256] bonds [32] chunk 2 scale 1 waves [2, 4, 4, 4] lazy 0"
    assert all(w in (1, 2, 4) for w in t.waves_per_block) and len(t.waves_per_block) == 4
    assert sorted(t.atom_bounds) == t.atom_bounds and t.atom_bounds[-1] <= 256
    assert 1 <= t.restart_chunk and 1 <= t.grid_scale <= 64 and t.lazy_clash in (0, 1)


def test_work_counts_on_hand_built_ligands():
    """Counts per ligand: no torsion leaves only rigid scans, placement and the
    final score; each moving atom adds A torsion samples; the plain count adds the
    pair tests of every (moving, static) pair, which the kernel's count leaves out."""
    R, A, T, S = 4, 8, 6, 2
    n = np.array([10, 10, 10])
    frags = [[], [3], [3, 5]]          # fragment sizes (axis atom b included)
    isa = bench.isa_ops(n, frags, R, A, T, S)
    plain = bench.plain_method_ops(n, frags, R, A, T, S)
    looks = bench.lookups(n, frags, R, A, T, S)
    rigid = R * (S * (3 * A * 10 * bench.ISA_ROT + 3 * T * 10 * bench.ISA_TRANS) + 10 * (bench.OPS_PLACE + bench.OPS_TRI))
    assert isa[0] == pytest.approx(rigid)
    per_moving = R * S * A * bench.ISA_TORS
    per_bond = R * S * A * bench.ISA_TMAT
    assert isa[1] - isa[0] == pytest.approx(2 * per_moving + per_bond)
    assert isa[2] - isa[1] == pytest.approx(4 * per_moving + per_bond)
    # plain: 2 moving atoms against 10 - 2 - 2 static ones (the axis atoms excluded)
    pair_terms = R * S * A * bench.PLAIN_PAIR * np.array([0, 2 * 6, 2 * 6 + 4 * 4])
    tors_terms = R * S * A * bench.PLAIN_TORS * np.array([0, 2, 6])
    base = R * (S * (3 * A * 10 * bench.PLAIN_ROT + 3 * T * 10 * bench.PLAIN_TRANS) + 10 * (bench.OPS_PLACE + bench.OPS_TRI))
    np.testing.assert_allclose(plain, base + tors_terms + pair_terms)
    # lookups: every sample of every scan, the current pose at rotation and torsion
    # scans, eight per atom for the trilinear score
    np.testing.assert_allclose(looks, R * (S * (3 * A * 10 + 3 * T * 10 + A * np.array([0, 2, 6]) + 30
                                               + np.array([0, 2, 6])) + 80))


def test_bucket_of_follows_the_bounds():
    t = tuning_obj({"atom_bounds": [64, 128, 192, 256], "rot_bounds": [4, 32], "restart_chunk": 2, "grid_scale": 1,
                    "waves_per_block": [2, 4, 4, 4], "lazy_clash": 0})
    atoms = np.array([1, 64, 65, 128, 129, 192, 193, 256])
    tors = np.array([0, 4, 5, 32, 0, 4, 5, 32])
    np.testing.assert_array_equal(bench.bucket_of(atoms, tors, t), [0, 0, 3, 3, 4, 4, 7, 7])
    # the last bound takes every larger ligand
    t1 = tuning_obj({"atom_bounds": [64], "rot_bounds": [32], "restart_chunk": 2, "grid_scale": 1,
                     "waves_per_block": [2, 4, 4, 4], "lazy_clash": 0})
    np.testing.assert_array_equal(bench.bucket_of(np.array([10, 200]), np.array([3, 30]), t1), [0, 0])
