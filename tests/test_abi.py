"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every entry point declared in include/cvo.h, and reports errors cleanly."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "cvo.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(cvo_\w+)\(", src, re.M)))


def test_header_declares_the_abi():
    names = declared()
    for n in ("cvo_create", "cvo_destroy", "cvo_set_stream", "cvo_eval", "cvo_register", "cvo_submit",
              "cvo_poll", "cvo_trace", "cvo_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1904_02266_amd import _binding
    L = _binding.load()
    for n in declared():
        assert hasattr(L, n), n
    assert set(declared()) == set(_binding.EXPORTED)


def test_strerror_and_null_handling():
    from paper_1904_02266_amd import _binding
    L = _binding.load()
    assert L.cvo_strerror(-1) == b"invalid argument"
    assert L.cvo_strerror(-4).startswith(b"no pair")
    assert L.cvo_destroy(None) == -1
    assert L.cvo_eval(None, None, None, None, None, None, None, None) == -1
    assert L.cvo_poll(None, 1, 0, None, None) == -1


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_1904_02266_amd import Context, CvoError
    with pytest.raises(CvoError):
        Context(0)
