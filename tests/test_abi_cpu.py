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


def test_random_tbme_matches_the_workload_generator():
    """trbl_random_tbme (host only) draws the interaction of the workloads byte for byte: the
    same elements in the same order and the same doubles, for the sd, pf and Sn-region spaces
    at seeds 1-3."""
    import struct

    from workloads import PF_ORBITS, SD_ORBITS, SNSB_ORBITS, random_tbme
    for orbits in (SD_ORBITS, PF_ORBITS, SNSB_ORBITS):
        for seed in (1, 2, 3):
            lib_t = trbl.random_tbme(orbits, seed, 1.0)
            ref = random_tbme(orbits, seed, 1.0)
            assert len(lib_t) == len(ref)
            for a, b in zip(lib_t, ref):
                assert a[:6] == b[:6]
                assert struct.pack("<d", a[6]) == struct.pack("<d", b[6])
    assert len(trbl.random_tbme(SD_ORBITS, 1)) == 158  # 30 pp + 30 nn + 98 pn
    assert len(trbl.random_tbme(PF_ORBITS, 1)) == 94 + 94 + 330
    # sigma scales every draw
    s2 = trbl.random_tbme(SD_ORBITS, 2, 2.5)
    s1 = trbl.random_tbme(SD_ORBITS, 2, 1.0)
    assert all(x[6] == 2.5 * y[6] for x, y in zip(s2, s1))


def test_random_tbme_errors():
    lib = trbl.load()
    arr = (trbl.Orbit * 1)(trbl.Orbit(0, 3, 7))
    n = ctypes.c_int64()
    assert lib.trbl_random_tbme(arr, 1, 1, 1.0, None, 0, ctypes.byref(n)) == 0 and n.value > 0
    out = (trbl.Tbme * 1)()
    assert lib.trbl_random_tbme(arr, 1, 1, 1.0, out, 1, ctypes.byref(n)) == -1  # buffer too small
    bad = (trbl.Orbit * 1)(trbl.Orbit(0, 3, 6))  # even 2j
    assert lib.trbl_random_tbme(bad, 1, 1, 1.0, None, 0, ctypes.byref(n)) == -1
