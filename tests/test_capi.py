"""CPU-side checks of the C ABI: the library loads and exports every declared symbol."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:lw_status|void|const char\*)\s+(lw_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("lw_create", "lw_set_directions", "lw_set_frequencies", "lw_accumulate",
                 "lw_read_spectra", "lw_reset"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import ctypes

    import torch  # noqa: F401  (the binding loads the library after torch)

    from paper_1003_1140_amd import lw

    if not os.path.exists(lw.LIB_PATH):
        pytest.fail("liblw.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(lw.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(lw.EXPORTED) == set(declared_symbols())


def test_binding_refuses_to_run_without_library(monkeypatch, tmp_path):
    from paper_1003_1140_amd import lw

    monkeypatch.setattr(lw, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(lw, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        lw.load_library()


def test_binding_refuses_host_index_lists():
    """Index lists reach the kernels as device pointers: a host tensor, a numpy array or an
    int32 tensor is refused before any library call."""
    import numpy as np
    import torch

    from paper_1003_1140_amd.lw import _checked_indices

    for bad in (torch.arange(3, dtype=torch.int64), np.arange(3, dtype=np.int64), [0, 1, 2],
                torch.arange(3, dtype=torch.int32)):
        with pytest.raises(TypeError):
            _checked_indices(bad)
