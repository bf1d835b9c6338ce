"""The C-ABI library: it loads, exports every function include/vc.h declares, and its
host-only entry points behave. No compute call is made here (no GPU needed)."""

import ctypes
import os
import re

import pytest

import paper_2204_10402_amd as vc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "vc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vc_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return vc.load_library()


def test_header_matches_binding():
    assert declared_functions() == sorted(vc.EXPORTS)


def test_every_declared_symbol_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_and_version(lib):
    assert vc.version().count(".") == 2
    for code, word in ((vc.OK, "ok"), (vc.ERR_INVALID_GRAPH, "graph"), (vc.ERR_BUDGET, "budget"),
                       (vc.ERR_DEVICE, "device"), (vc.ERR_INTERNAL, "internal"),
                       (vc.ERR_NO_MEMORY, "memory"), (vc.ERR_INVALID_ARG, "argument")):
        assert word in lib.vc_strerror(code).decode().lower()
    assert lib.vc_last_error(None).decode() == ""


def test_null_arguments(lib):
    assert lib.vc_create(None, 0, None) == vc.ERR_INVALID_ARG
    assert lib.vc_destroy(None) == vc.OK
    assert lib.vc_mvc(None, None, None, None, None, None) == vc.ERR_INVALID_ARG


def test_struct_layouts_match_header():
    # sizes implied by include/vc.h on LP64
    from paper_2204_10402_amd import _binding as b
    assert ctypes.sizeof(b._Graph) == 24
    assert ctypes.sizeof(b._Options) == 48
    assert ctypes.sizeof(b._Stats) == 7 * 8 + 10 * 4 + 3 * 8 + 10 * 8 + 3 * 8 + 2 * 4
    assert ctypes.sizeof(b._Batch) == 8 + 4 * 8
    assert ctypes.sizeof(b._ServerOptions) == 4 + 4 + 8 + 4 + 3 * 4
    assert ctypes.sizeof(b._Served) == 8 + 6 * 4 + 8 + 3 * 8


def test_no_gpu_means_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    assert lib.vc_create(ctypes.byref(ctx), 0, None) == vc.ERR_DEVICE
    assert not ctx.value


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2204_10402_amd import _binding as b
    saved = b._lib
    b._lib = None
    try:
        with pytest.raises(ImportError):
            b.load_library(str(tmp_path / "missing.so"))
    finally:
        b._lib = saved


def test_product_package_does_not_use_oracle():
    pkg = os.path.join(ROOT, "paper_2204_10402_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "vc_oracle" not in text and "liboracle" not in text, f


def test_pack_batch_layout():
    """The packed batch is each graph's own CSR, one after another."""
    import graphs as G
    from paper_2204_10402_amd import _binding as b
    gs = [G.path(3), G.empty(0), G.cycle(4)]
    n, nnz, rp, ci = b.pack_batch(gs)
    assert n.tolist() == [3, 0, 4] and nnz.tolist() == [4, 0, 8]
    assert rp.tolist() == [0, 1, 3, 4, 0, 0, 2, 4, 6, 8]
    assert ci.tolist() == [1, 0, 2, 1, 1, 3, 0, 2, 1, 3, 0, 2]
    assert b._offsets(n).tolist() == [0, 3, 3, 7]


def test_null_arguments_of_the_workspace_forms(lib):
    size = ctypes.c_size_t()
    assert lib.vc_abort(None) == vc.ERR_INVALID_ARG
    assert lib.vc_workspace_bytes(None, 10, 20, 0, None, ctypes.byref(size)) == vc.ERR_INVALID_ARG
    assert lib.vc_batch_workspace_bytes(None, None, 0, None, ctypes.byref(size)) == \
        vc.ERR_INVALID_ARG
    assert lib.vc_mvc_device_ws(None, None, None, None, 0, None, None, None) == vc.ERR_INVALID_ARG
    assert lib.vc_pvc_device_ws(None, None, 1, None, None, 0, None, None, None, None) == \
        vc.ERR_INVALID_ARG
    assert lib.vc_mvc_batch_device_ws(None, None, None, None, 0, None, None, None, None,
                                      None) == vc.ERR_INVALID_ARG
    assert lib.vc_pvc_batch_device_ws(None, None, None, None, None, 0, None, None, None, None,
                                      None, None) == vc.ERR_INVALID_ARG


def _fake_device(t):
    """A CPU tensor that reports itself as a GPU tensor, to reach the binding's later checks
    without a GPU (the library is never called with it)."""
    import torch

    class FakeCuda(torch.Tensor):
        @property
        def is_cuda(self):
            return True

    return t.as_subclass(FakeCuda)


def test_binding_rejects_bad_output_tensors():
    """Device outputs the library writes through must be GPU tensors of the right dtype,
    contiguous and long enough; anything else raises before the library sees a pointer."""
    import torch
    from paper_2204_10402_amd import _binding as b
    assert b._device_out(None, "cover", 5, "uint8") is None
    with pytest.raises(TypeError):
        b._device_out(torch.zeros(5, dtype=torch.uint8), "cover", 5, "uint8")  # CPU tensor
    with pytest.raises(TypeError):
        b._device_out(_fake_device(torch.zeros(5, dtype=torch.int32)), "cover", 5, "uint8")
    with pytest.raises(TypeError):
        b._device_out(_fake_device(torch.zeros(10, dtype=torch.uint8)[::2]), "cover", 5, "uint8")
    with pytest.raises(ValueError):
        b._device_out(_fake_device(torch.zeros(4, dtype=torch.uint8)), "cover", 5, "uint8")
    with pytest.raises(TypeError):
        b._device_out(_fake_device(torch.zeros(5, dtype=torch.uint8)), "deg", 5, "int32")
    t = _fake_device(torch.zeros(5, dtype=torch.int32))
    assert b._device_out(t, "deg", 5, "int32") == t.data_ptr()
    with pytest.raises(TypeError):
        b._workspace(torch.zeros(1024, dtype=torch.uint8))  # CPU tensor
    with pytest.raises(TypeError):
        b._workspace(_fake_device(torch.zeros(256, dtype=torch.int32)))
