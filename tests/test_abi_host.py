"""The C-ABI library loads on the host and exports every declared symbol; the
host-only calls (Eq. 1, cluster boundaries) and argument checks work without a GPU."""
import ctypes
import os
import re


from paper_2303_06150_amd import lg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lg_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = lg.load_library()
    names = declared_symbols()
    assert {"lg_load_pocket", "lg_dock_batch", "lg_score", "lg_refine"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(lg.EXPORTS) == set(names)


def test_eq1_reproduces_table1():
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "table1_eq1.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for impl, atoms, regs, active in rows:
        active = int(active)
        b, rem = divmod(active, 108)
        assert rem == 0                      # a whole number of resident blocks per SM
        assert lg.lg_bucket_size(b, 108, 32, 32) == active
    # Eq. 2 (SYCL form) with wgs = b*t resident work items per CU is the same number
    assert lg.lg_bucket_size(16, 108, 64, 64) == 1728
    # MI355X form: 256 CUs, wavefront 64, four wavefronts per block
    assert lg.lg_bucket_size(8, 256, 256, 64) == 8192
    assert lg.lg_bucket_size(-1, 1, 1, 1) == -1


def test_cluster_boundaries():
    # Sec. 3: three atom clusters at warp-size multiples -> up to 32, up to 64, the rest
    assert lg.lg_atom_clusters(3, 32, 120) == [32, 64, 120]
    assert lg.lg_atom_clusters(3, 64, 160) == [64, 128, 160]
    assert lg.lg_atom_clusters(6, 64, 120) == [64, 120]          # no empty clusters
    assert lg.lg_atom_clusters(1, 64, 256) == [256]
    r = lg.lg_rotamer_clusters(4, 24)
    assert r[-1] == 24 and all(b > a for a, b in zip(r, r[1:]))
    widths = [r[0] + 1] + [b - a for a, b in zip(r, r[1:])]
    assert widths == sorted(widths)                              # finer at low counts
    assert lg.lg_rotamer_clusters(23, 20)[-1] == 20


def test_argument_checks_need_no_device():
    lib = lg.load_library()
    assert lib.lg_dock_batch(None, None, None, None, None) == lg.LG_ERR_INVALID_ARG
    assert "NULL" in lg.lg_last_error()
    assert lib.lg_score(None, None, 0, None, None, None, 0, None, None, None) == lg.LG_ERR_INVALID_ARG
    assert lib.lg_refine(None, None, None, None, None, None, None, None) != lg.LG_OK
    assert lib.lg_rank(None, None, 0, 1, 0, None, None, None, None) == lg.LG_ERR_INVALID_ARG
    assert lib.lg_autotune(None, None, None, 1, None, None, None) == lg.LG_ERR_INVALID_ARG
    assert lib.lg_dock_stream(None, None, None, 1, None, None) == lg.LG_ERR_INVALID_ARG
    assert lib.lg_dock_sites(None, 1, None, None, None, 1, None) == lg.LG_ERR_INVALID_ARG
    assert [f for f, _ in lg.lg_host_out._fields_][-1] == "chunk_done"
    handles = (ctypes.c_void_p * 1)()
    params = lg.lg_dock_params()
    outs = (lg.lg_dock_out * 1)()
    assert lib.lg_dock_sites(handles, 0, None, ctypes.byref(params), outs, 1, None) == lg.LG_ERR_INVALID_ARG
    assert "n_sites" in lg.lg_last_error()
    assert lib.lg_dock_sites(handles, 1, None, ctypes.byref(params), outs, 1, None) == lg.LG_ERR_INVALID_ARG
    assert "pocket 0 is NULL" in lg.lg_last_error()
    assert lib.lg_set_tuning(None, None) == lg.LG_ERR_INVALID_ARG
    assert lib.lg_valu_probe(None, 0, 1, None, None) == lg.LG_ERR_INVALID_ARG
    assert lib.lg_free_pocket(None) == lg.LG_OK
    desc = lg.lg_pocket_desc(1, 32, 32, 0.5, 2.0, (ctypes.c_float * 3)(), (ctypes.c_float * 3)(), 0.0)
    h = ctypes.c_void_p()
    g = (ctypes.c_float * 4)()
    assert lib.lg_load_pocket(ctypes.byref(desc), g, 0, None, ctypes.byref(h)) == lg.LG_ERR_LIMIT
    assert lib.lg_load_pocket(None, g, 0, None, ctypes.byref(h)) == lg.LG_ERR_INVALID_ARG
    assert lg.lg_version() >= 1
