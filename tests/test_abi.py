"""The C ABI library loads on the host and exports every declared symbol.

No GPU is needed: only host-side entry points are called.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "agn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(agn_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for f in ["agn_psd_spectrum", "agn_lc_iterate", "agn_lc_generate", "agn_lc_generate_batch",
              "agn_ctx_create", "agn_ctx_destroy", "agn_last_error", "agn_workspace_size"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_1909_06374_amd as agn
    if not os.path.exists(agn.LIB_PATH):
        pytest.skip("libagn.so not built")
    lib = ctypes.CDLL(agn.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_host_side_entry_points():
    import paper_1909_06374_amd as agn
    if not os.path.exists(agn.LIB_PATH):
        pytest.skip("libagn.so not built")
    for n, ok in [(2, True), (6, True), (1024, True), (3 * 2**25, True), (2**27, True), (2**28, False),
                  (0, False), (10, False), (7, False), (-4, False)]:
        assert agn.agn_supported_n(n) == ok, n
    assert agn.agn_workspace_size(1024, agn.AGN_FP64) > 1024 * 8 * 3
    assert agn.agn_batch_workspace_size([1024, 96], agn.AGN_FP32) > agn.agn_workspace_size(1024, agn.AGN_FP32)
    with pytest.raises(agn.AgnError) as e:
        agn.agn_workspace_size(1000, agn.AGN_FP32)
    assert e.value.code == agn.AGN_EUNSUPPORTED_N
    with pytest.raises(agn.AgnError):
        agn.agn_workspace_size(1024, 7)
    assert "precision" in agn.lib().agn_last_error().decode()


def test_no_gpu_means_loud_failure():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import paper_1909_06374_amd as agn
    if not os.path.exists(agn.LIB_PATH):
        pytest.skip("libagn.so not built")
    with pytest.raises(agn.AgnError):
        agn.Context(0)
