"""The C ABI on the CPU: the library loads, exports every symbol include/dmlmc.h declares,
and rejects invalid arguments with DMLMC_EINVAL before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "dmlmc.h")) as f:
        text = f.read()
    decl = r"^(?:dmlmc_status|void|const char\s*\*)\s*(dmlmc_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_header_matches_binding():
    from paper_2211_15383_amd import dmlmc
    assert sorted(dmlmc.EXPORTED) == _declared()


def test_library_exports_all_symbols():
    from paper_2211_15383_amd import dmlmc
    lib = dmlmc.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.dmlmc_version().startswith(b"dmlmc")


def test_invalid_arguments_without_device():
    from paper_2211_15383_amd import dmlmc
    lib = dmlmc.load()
    h = C.c_void_p()
    assert lib.dmlmc_create(None, 0, None) == dmlmc.EINVAL
    assert lib.dmlmc_create(C.byref(h), -1, None) == dmlmc.EINVAL
    assert b"device" in lib.dmlmc_last_error(None)
    assert lib.dmlmc_build_hierarchy(None, None, None, None) == dmlmc.EINVAL
    assert lib.dmlmc_solve_multi_rhs(None, None, 1, None, None, None, 1, 1, 0, 1e-10, 10, None) == dmlmc.EINVAL
    assert lib.dmlmc_deflate_project_noalloc(None, None, None, None, 1) == dmlmc.EINVAL
    assert lib.dmlmc_level_info(None, 1, None, None, None) == dmlmc.EINVAL
    assert lib.dmlmc_deflation_info(None, None, None, None) == dmlmc.EINVAL
    assert lib.dmlmc_set_deflation(None, None) == dmlmc.EINVAL
    ld = C.c_int64(-1)
    assert lib.dmlmc_work_stride(None, 1, C.byref(ld)) == dmlmc.EINVAL and ld.value == -1
    assert lib.dmlmc_apply(None, None, dmlmc.OP_D, 1, None, None, 1, dmlmc.MIXED, 0) == dmlmc.EINVAL
    assert lib.dmlmc_apply_strided(None, None, dmlmc.OP_D, 1, None, 0, None, 0, 1, dmlmc.MIXED, 0) == dmlmc.EINVAL
    assert lib.dmlmc_coarsest_direct(None, None, None, 3) == dmlmc.EINVAL
    # destroy/free accept NULL
    lib.dmlmc_destroy(None)
    lib.dmlmc_free_hierarchy(None)
    lib.dmlmc_free_deflation(None)


def test_no_device_is_an_error_not_a_crash():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2211_15383_amd import dmlmc
    lib = dmlmc.load()
    h = C.c_void_p()
    assert lib.dmlmc_create(C.byref(h), 0, None) == dmlmc.EHIP


def test_bench_refuses_several_gpus():
    """The benchmark measures one GPU's share; asking for more exits with a message."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_recorded_traffic_lookup():
    """The benchmark reports HBM traffic only from a committed counter summary taken on the
    current source of the kernel and the same launch mix (algorithmic bytes within 0.5 %)."""
    import importlib.util
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        spec.loader.exec_module(b)
    finally:
        sys.argv = argv
    text = open(os.path.join(root, "profiles", "hbm_traffic_coarse16_gs_mfma_mgmlmc1024.md")).read()
    m = re.search(r"traffic: class=coarse_gs source_sha256=(\S+) bytes_per_launch=(\S+) "
                  r"algorithmic_bytes_per_launch=(\S+)", text)
    assert m, "the summary has no traffic line"
    assert m.group(1) == b.source_digest("coarse_gs"), "counters were taken on another source of the kernel"
    alg = float(m.group(3))
    got, src = b.recorded_traffic("coarse_gs", alg)
    assert got == float(m.group(2)) and src.startswith("hbm_traffic_")
    assert b.recorded_traffic("coarse_gs", alg * 1.02) == (None, None)
    # every class the benchmark can rank as dominant names the source its digest is taken of
    for cls in b.HBM_CLASSES:
        assert os.path.isfile(os.path.join(root, "paper_2211_15383_amd", "csrc", b.CLASS_SOURCE[cls])), cls
        assert b.recorded_traffic(cls, 1.0) == (None, None)


def test_kernel_variant_calls_reject_bad_arguments():
    """The launch-variant calls validate their handles before any device work."""
    from paper_2211_15383_amd import dmlmc
    lib = dmlmc.load()
    v = C.c_int32()
    assert lib.dmlmc_set_kernel_variant(None, 1, 0, 1) == dmlmc.EINVAL
    assert lib.dmlmc_get_kernel_variant(None, 1, 0, C.byref(v)) == dmlmc.EINVAL
    assert lib.dmlmc_tune_kernels(None, None, 32, 10, None, None, None, None) == dmlmc.EINVAL
