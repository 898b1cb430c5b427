"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every entry point declared in include/cvo.h, and reports errors cleanly."""
import ctypes
import os
import re

import numpy as np
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


def _P(A, t):
    return t * (A[1] + t * (A[2] + t * (A[3] + t * A[4])))


def test_quartic_step_host_rule_matches_oracle():
    # The library's step rule for the quartic model (Newton's method on P'
    # inside the brackets cut at the roots of P'') against the oracle's
    # (plain bisection of P' inside the same kind of brackets), on random
    # coefficient sets of mixed signs and scales, A1 >= 0 as along a gradient.
    import oracle
    from paper_1904_02266_amd import quartic_step
    rng = np.random.default_rng(5)
    agree = none_both = 0
    for _ in range(4000):
        sc = 10.0 ** rng.uniform(-3, 3, size=4)
        A = np.concatenate([[1.0], rng.normal(size=4) * sc])
        A[1] = abs(A[1])
        if rng.random() < 0.1:
            A[4] = 0.0
        t_lib = quartic_step(A)
        t_or = oracle.quartic_step(A)
        if t_or is None:
            assert t_lib is None, A
            none_both += 1
            continue
        assert t_lib is not None, A
        if abs(t_lib - t_or) > 1e-9 * t_or:
            # two maxima of (numerically) equal height: the values must agree
            assert abs(_P(A, t_lib) - _P(A, t_or)) <= 1e-12 * max(abs(_P(A, t_or)), 1e-300), A
        agree += 1
    assert agree > 1000 and none_both > 100


@pytest.mark.parametrize("A,t", [
    ([0, 1.0, -1.0, 0.0, 0.0], 0.5),
    ([0, 1.0, 0.0, -1.0, 0.0], 3 ** -0.5),
    ([0, 1.0, 1.0, 1.0, 1.0], None),
    ([0, 1.0, 0.0, 0.0, 0.0], None),
    ([0, 0.0, 0.0, 0.0, 0.0], None),
])
def test_quartic_step_host_rule_special_cases(A, t):
    from paper_1904_02266_amd import quartic_step
    got = quartic_step(A)
    if t is None:
        assert got is None
    else:
        assert abs(got - t) < 1e-14


def test_quartic_step_bounded_host_rule_matches_oracle():
    # the trusted interval (0, tmax]: only local maxima at t <= tmax count,
    # in the library's rule and in the oracle's alike
    import oracle
    from paper_1904_02266_amd import quartic_step
    rng = np.random.default_rng(11)
    cut = 0
    for _ in range(3000):
        sc = 10.0 ** rng.uniform(-3, 3, size=4)
        A = np.concatenate([[1.0], rng.normal(size=4) * sc])
        A[1] = abs(A[1])
        t_free = oracle.quartic_step(A)
        tmax = 10.0 ** rng.uniform(-4, 2)
        a, b = quartic_step(A, tmax=tmax), oracle.quartic_step(A, tmax=tmax)
        assert (a is None) == (b is None), (A, tmax)
        if a is not None:
            assert a <= tmax and b <= tmax
            if abs(a - b) > 1e-9 * b:
                assert abs(_P(A, a) - _P(A, b)) <= 1e-12 * max(abs(_P(A, b)), 1e-300), A
        if t_free is not None and t_free > tmax:
            cut += 1
    assert cut > 100
    # P = t - t^2 has its maximum at 0.5
    assert quartic_step([0, 1.0, -1.0, 0, 0], tmax=0.4) is None
    assert abs(quartic_step([0, 1.0, -1.0, 0, 0], tmax=0.6) - 0.5) < 1e-14
    assert abs(quartic_step([0, 1.0, -1.0, 0, 0], tmax=float("inf")) - 0.5) < 1e-14
