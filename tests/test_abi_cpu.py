"""CPU-side checks of the C ABI: the library loads, exports every declared symbol, and
rejects malformed input on the host before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2406_18655_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols(header="qlsd.h"):
    with open(os.path.join(ROOT, "include", header)) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(qlsd_[a-z_0-9]+)\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2406_18655_amd import build
        build.build()
    return binding.lib()


def test_every_declared_symbol_is_exported(lib):
    decl = _declared_symbols()
    assert set(decl) == set(binding.EXPORTS)
    serve = [x for x in _declared_symbols("qlsd_serve.h") if x.startswith("qlsd_server")]
    assert set(serve) == set(binding.SERVE_EXPORTS)
    net = [x for x in _declared_symbols("qlsd_net.h") if x.startswith(("qlsd_net", "qlsd_decoder_set_net"))]
    assert set(net) == set(binding.NET_EXPORTS)
    smp = [x for x in _declared_symbols("qlsd_sample.h") if x != "qlsd_last_error"]
    assert set(smp) == set(binding.SAMPLE_EXPORTS)
    win = _declared_symbols("qlsd_window.h")
    assert set(win) == set(binding.WINDOW_EXPORTS)
    for name in decl + serve + net + smp + win:
        assert hasattr(lib, name), name


def test_code_create_rejects_bad_csr(lib):
    h = ctypes.c_void_p()
    rp = np.array([0, 2, 4], dtype=np.int32)
    bad_cols = np.array([1, 0, 0, 1], dtype=np.int32)  # row 0 not sorted
    st = lib.qlsd_code_create(2, 2, 4, rp.ctypes.data, bad_cols.ctypes.data, ctypes.byref(h))
    assert st == -1 and b"sorted" in lib.qlsd_last_error()
    out_of_range = np.array([0, 5, 0, 1], dtype=np.int32)
    st = lib.qlsd_code_create(2, 2, 4, rp.ctypes.data, out_of_range.ctypes.data, ctypes.byref(h))
    assert st == -1
    st = lib.qlsd_code_create(0, 2, 0, rp.ctypes.data, None, ctypes.byref(h))
    assert st == -1
    bad_ptr = np.array([0, 3, 4], dtype=np.int32)
    st = lib.qlsd_code_create(2, 2, 3, bad_ptr.ctypes.data, bad_cols.ctypes.data, ctypes.byref(h))
    assert st == -1


def test_null_handles_are_rejected(lib):
    assert lib.qlsd_decode(None, None, 0, None, None, None) == -1
    assert lib.qlsd_sync(None) == -1
    assert lib.qlsd_decoder_set_lsd_capacity(None, 64) == -1
    assert lib.qlsd_decoder_set_lsd_schedule(None, 0) == -1
    assert lib.qlsd_last_error() != b""
    lib.qlsd_decoder_destroy(None)
    lib.qlsd_code_destroy(None)


def test_info_layout_matches_header():
    assert binding.INFO_DTYPE.itemsize == 12
    assert ctypes.sizeof(binding.QlsdParams) == 24  # six 4-byte fields of qlsd_params
    assert binding.COMPLETION_DTYPE.itemsize == 40
    import oracle.learned as ol
    with open(os.path.join(ROOT, "include", "qlsd_net.h")) as f:
        assert f"#define QLSD_NET_PARAMS {ol.N_PARAMS}" in f.read()
    assert binding.NET_PARAMS == ol.N_PARAMS


def test_server_host_side_validation(lib):
    L = binding._serve_lib()
    h = ctypes.c_void_p()
    assert L.qlsd_server_create(1 << 20, ctypes.byref(h)) == 0
    cid, lanes = ctypes.c_int32(), ctypes.c_int32()
    params = binding.QlsdParams(30, 0.625, 0, 0, 0)
    # no code handle: refused before any device work
    assert L.qlsd_server_add_code(h, None, ctypes.byref(params), None, 16, 1, ctypes.byref(cid),
                                  ctypes.byref(lanes)) == -1
    assert L.qlsd_server_submit_many(h, 0, 1, None, None, None, None) == -1
    L.qlsd_server_destroy(h)


def test_binding_rejects_strided_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        binding._ptr(torch.zeros((4, 3), dtype=torch.uint8).t())
    assert binding._ptr(torch.zeros((4, 3), dtype=torch.uint8)) is not None


def test_generated_syndromes_are_row_major():
    from paper_2406_18655_amd.workloads import bivariate_bicycle, sample
    e, s = sample(bivariate_bicycle(), 64, seed=1)
    assert e.flags["C_CONTIGUOUS"] and s.flags["C_CONTIGUOUS"]


def test_binding_rejects_mis_shaped_tensors():
    """The C ABI trusts buffer sizes; the binding must refuse tensors that do not match the
    decoder's (m, n) before any pointer reaches it (checked here without a GPU: the shape check
    runs first, so a CPU tensor of the right shape fails on the device check instead)."""
    import torch
    from paper_2406_18655_amd import binding

    class FakeCode:
        m, n = 4, 7

    class FakeDecoder(binding.Decoder):
        def __init__(self):
            self.code = FakeCode()
            self.max_batch = 8

    d = FakeDecoder()
    s = torch.zeros((3, 4), dtype=torch.uint8)
    with pytest.raises(ValueError, match="shape"):
        d.decode_into(torch.zeros((3, 5), dtype=torch.uint8), torch.zeros((3, 7), dtype=torch.uint8))
    with pytest.raises(ValueError, match="CUDA"):
        d.decode_into(s, torch.zeros((3, 7), dtype=torch.uint8))
    with pytest.raises(ValueError):
        d.lsd_into(s, torch.zeros((3, 7), dtype=torch.float64), torch.zeros((3, 7), dtype=torch.uint8))
    with pytest.raises(ValueError):
        d.bp_into(s, torch.zeros((3, 6), dtype=torch.float32))
