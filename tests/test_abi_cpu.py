"""The C-ABI library loads and exports every symbol include/trbl.h declares (no GPU calls)."""
import ctypes

import paper_1902_02064_amd as trbl


def test_library_exports_header_symbols():
    lib = trbl.load()
    names = trbl.header_symbols()
    assert "trbl_apply" in names and "trbl_solve" in names and "trbl_tbme_grad" in names
    for n in names:
        assert hasattr(lib, n), n


def test_last_error_without_gpu_call():
    lib = trbl.load()
    assert isinstance(lib.trbl_last_error(), bytes)
    # argument errors are caught on the host before any device work
    rc = lib.trbl_model_dim(None, None)
    assert rc == -1
    assert b"NULL" in lib.trbl_last_error()
