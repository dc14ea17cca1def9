"""Host-side checks of the C ABI: the library builds, loads without a GPU, and exports
every entry point that include/qdw.h declares."""
import os
import re
import subprocess

import pytest

from paper_2202_07388_amd import qdw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qdw.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*([A-Za-z_][A-Za-z_0-9]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(qdw.LIB_PATH):
        from paper_2202_07388_amd import build
        build.build(verbose=False)
    return qdw.load()


def test_header_declares_the_four_named_calls():
    names = declared_functions()
    for n in ("dw_apply", "dw_dag_apply", "cgne_solve", "sap_gcr_solve", "qdw_norm2", "nn_forward", "nn_train_step"):
        assert n in names, n


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", qdw.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(lib, n)


def test_errors_are_reported_without_gpu(lib):
    import ctypes
    rc = lib.dw_apply(None, None, None, 0, None)
    assert rc == -1
    assert b"null" in lib.qdw_last_error()
    assert lib.qdw_field_bytes(None, 0) == 0


def test_format_eps_match_paper_table():
    """Machine epsilons used for the reset threshold are the paper's Table 1 values."""
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden",
                                                 "table1_format_limits.txt"))
            if l.strip() and not l.startswith("#")]
    table = {r[0]: float(r[-1]) for r in rows}
    for name, key in (("binary64", "f64"), ("binary32", "f32"), ("binary16", "f16"),
                      ("bfloat16", "bf16")):
        assert abs(qdw.EPS[key] - table[name]) <= 0.05 * table[name]


def test_batched_and_tuning_entry_points_reject_bad_arguments_without_gpu(lib):
    import ctypes
    assert lib.dw_apply_multi(None, None, None, 1, 0, None) == -1
    assert b"null" in lib.qdw_last_error()
    assert lib.qdw_autotune(None, 0, 1, None, 0, None, 0, None) == -1
    assert lib.qdw_autotune_workspace_bytes(None, 0, 1) == 0
    prm = qdw.SapGcrParams(1e-10, 100, 16, 5, 4, (ctypes.c_int * 4)(4, 4, 4, 4), 2, 1, None)
    assert lib.qdw_sap_gcr_batched_workspace_bytes(None, 1, ctypes.byref(prm)) == 0
    infos = (qdw.Info * 1)()
    rc = lib.sap_gcr_solve_batched(None, None, None, 1, ctypes.byref(prm), None, 0, infos,
                                   None, None)
    assert rc == -1
    # the learned preconditioner is not offered in batched form
    prm.precond = qdw.PRECOND["nn"]
    assert lib.qdw_sap_gcr_batched_workspace_bytes(None, 1, ctypes.byref(prm)) == 0


def test_adaptive_sap_rejects_bad_arguments_without_gpu(lib):
    import ctypes
    bs = (ctypes.c_int * 4)(4, 4, 4, 4)
    rc = lib.sap_adaptive_apply(None, None, None, 20, 20, 0.9, 0.0, ctypes.byref(bs), 2, None, 0,
                                None, None, None)
    assert rc == -1 and b"null" in lib.qdw_last_error()


def test_cascade_workspace_without_gpu(lib):
    import ctypes
    prm = qdw.CgneParams(1e-10, 100, 99, -1.0, 1, 1, 1.0)  # inner ignored by the cascade
    assert lib.qdw_cgne_workspace_bytes(None, ctypes.byref(prm)) == 0
    prm.cascade = 0
    assert lib.qdw_cgne_workspace_bytes(None, ctypes.byref(prm)) == 0


def test_schur_entry_points_reject_null_without_gpu(lib):
    assert lib.dw_schur_apply(None, None, None, 0, None) == -1
    assert lib.dw_schur_dag_apply(None, None, None, 0, None) == -1


def test_full_link_control_rejects_null_without_gpu(lib):
    assert lib.qdw_full_links_bytes(None) == 0
    assert lib.qdw_set_full_links(None, None, 0, None) == -1
    assert b"qdw_set_full_links" in lib.qdw_last_error()
    assert lib.dw_apply_full_links(None, None, None, 0, None) == -1
    assert b"dw_apply_full_links" in lib.qdw_last_error()


def test_sap_eo_rejects_bad_arguments_without_gpu(lib):
    import ctypes
    bs = (ctypes.c_int * 4)(4, 4, 4, 4)
    rc = lib.sap_eo_apply(None, None, None, 5, 4, ctypes.byref(bs), 2, None, 0, None)
    assert rc == -1 and b"sap_eo_apply" in lib.qdw_last_error()


def test_bench_refuses_several_gpus():
    """One GPU only: --gpus above 1 exits with a message, before touching a device."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_record_is_consistent_and_current():
    """The HBM byte count bench.py reports as roofline.traffic: its parts add up, the read
    bytes are FETCH_SIZE scaled by the calibration factor, and it was taken on the current
    FP64 D kernel sources in the shape the benchmark times (re-profile after changing them:
    otherwise the benchmark reports no traffic)."""
    import json
    import sys
    sys.path.insert(0, ROOT)
    import bench
    t = json.load(open(bench.TRAFFIC_FILE))
    assert t["read_bytes"] + t["write_bytes"] == t["bytes_per_launch"]
    assert t["fetch_scale"] == 2.0
    assert list(t["shape"]) == list(bench.PINNED_SHAPES["f64"])
    if t["kernel_hash"] != bench.kernel_hash():
        # taken on other kernel sources: the benchmark must not report it
        assert bench.measured_traffic(bench.PINNED_SHAPES["f64"]) is None
        return
    assert bench.measured_traffic(bench.PINNED_SHAPES["f64"]) == t["bytes_per_launch"]
    # at least the compulsory stored bytes (1040 per site read: spinor 192, four links of
    # 12 reals and a determinant double, the 54-real clover; one spinor written)
    assert t["read_bytes"] >= 1040 * 2 ** 21 and t["write_bytes"] >= 192 * 2 ** 21


def test_operator_memory_comes_from_the_caller(lib):
    """qdw_create takes its device and host blocks from the caller: the size query works
    without a GPU, scales with the volume (about 4.1 kB per site), rejects bad lattices, and
    create refuses missing or short blocks before touching the device."""
    import ctypes
    small = qdw.Lattice(4, 4, 4, 4, -1)
    big = qdw.Lattice(8, 8, 8, 8, -1)
    ns, nb = lib.qdw_op_device_bytes(ctypes.byref(small)), lib.qdw_op_device_bytes(ctypes.byref(big))
    assert 0 < ns < nb
    # per site: links 4 x (104 + 56 + 32 + 32) B, clover blocks and inverses 2 x (576 + 288
    # + 144 + 144) B, the compact clover 432 + 224 + 112 + 112 B; the rest is a fixed
    # reduction scratch
    assert (nb - ns) == (8 ** 4 - 4 ** 4) * (4 * 224 + 2 * 1152 + 880)
    assert lib.qdw_op_device_bytes(ctypes.byref(qdw.Lattice(4, 4, 4, 3, -1))) == 0
    assert lib.qdw_op_host_bytes() >= 8 * 1024
    h = ctypes.c_void_p()
    rc = lib.qdw_create(ctypes.byref(small), None, None, 0.1, 1.5, None, 0, None, 0, None,
                        ctypes.byref(h))
    assert rc == -1 and b"null" in lib.qdw_last_error()
    fake = ctypes.c_void_p(0x1000)
    rc = lib.qdw_create(ctypes.byref(small), fake, fake, 0.1, 1.5, fake, ns - 1, fake,
                        lib.qdw_op_host_bytes(), None, ctypes.byref(h))
    assert rc == -6 and b"qdw_op_device_bytes" in lib.qdw_last_error()
