"""Host-side checks of the C ABI (no GPU needed): exports, host plan, errors."""
import ctypes
import os
import re
from math import comb

import numpy as np
import pytest

import oracle as O

S = pytest.importorskip("paper_2410_19844_amd")

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "sos.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(sos_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_header_function():
    names = header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(S._lib, name), name
    assert set(S.EXPORTS) == set(names)


def test_binding_flag_values_match_the_header():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    flags = dict(re.findall(r"SOS_(FLAG_\w+)\s*=\s*(\d+)", text))
    assert len(flags) >= 9
    for name, value in flags.items():
        assert getattr(S, name) == int(value), name
    assert len(set(flags.values())) == len(flags)  # distinct bits


@pytest.mark.parametrize("n,d", [(1, 1), (1, 7), (2, 2), (3, 2), (4, 3), (6, 3), (6, 4), (16, 1), (2, 7)])
def test_exponents_match_oracle(n, d):
    pl = S.Plan(n, d, 3, "fp32", device="cpu")
    assert pl.N == comb(n + d, d) and pl.M == comb(n + 2 * d, 2 * d)
    assert np.array_equal(pl.exponents(0), O.monomials(n, d))
    assert np.array_equal(pl.exponents(1), O.monomials(n, 2 * d))


@pytest.mark.parametrize("n,d", [(17, 2), (20, 3), (40, 2)])
def test_exponents_match_oracle_many_variables(n, d):
    pl = S.Plan(n, d, 3, "fp32", device="cpu")
    assert pl.N == comb(n + d, d) and pl.M == comb(n + 2 * d, 2 * d)
    assert np.array_equal(pl.exponents(0), O.monomials(n, d))
    if n <= 20:
        assert np.array_equal(pl.exponents(1), O.monomials(n, 2 * d))


def test_quartic_hundred_variable_sizes():
    """The paper's largest workload, quartic forms in 100 variables (Section
    1.2: l = 5,050, m = 4,421,275), is (n, d) = (99, 2) in the degree-<=d basis."""
    pl = S.Plan(99, 2, 5050, "bf16x3", device="cpu")
    assert (pl.N, pl.M) == (5050, 4421275)


@pytest.mark.parametrize("n,d", [(10, 5), (12, 6)])
def test_large_basis_matches_oracle(n, d):
    pl = S.Plan(n, d, 7, "bf16x3", device="cpu")
    assert np.array_equal(pl.exponents(0), O.monomials(n, d))


def _plan_rc(n, d, k, prec):
    h = ctypes.c_void_p()
    rc = S._lib.sos_plan(n, d, k, prec, ctypes.byref(h))
    if rc == 0:
        S._lib.sos_plan_destroy(h)
    return rc


def test_plan_argument_errors():
    assert _plan_rc(3, 2, 5, 0) == 0
    assert _plan_rc(0, 2, 5, 0) == -1          # n < 1
    assert _plan_rc(3, 0, 5, 0) == -1          # d < 1
    assert _plan_rc(3, 2, 0, 0) == -1          # rank < 1
    assert _plan_rc(3, 2, 5, 9) == -1          # unknown precision
    assert _plan_rc(3, 8, 5, 0) == -2          # 2d = 16 > 15
    assert b"2d <= 15" in S._lib.sos_last_error()
    assert _plan_rc(17, 1, 5, 0) == 0          # n > 16: variable-list ranking
    assert _plan_rc(17, 5, 5, 0) == -2         # n > 16 needs 2d <= 8
    assert b"2d <= 8" in S._lib.sos_last_error()
    assert _plan_rc(256, 1, 5, 0) == -2        # n > 255
    assert b"n <= 255" in S._lib.sos_last_error()
    assert _plan_rc(16, 7, 5, 0) == -2         # N*N >= 2^31
    assert b"2^31" in S._lib.sos_last_error()


def test_unbound_plan_rejects_device_calls():
    h = S.sos_plan(3, 2, 5, "fp64")
    z = ctypes.c_void_p(0)
    rc = S._lib.sos_loss_grad(h, z, z, z, z, z, 0, z)
    assert rc == -1 and b"not bound" in S._lib.sos_last_error()
    S._lib.sos_plan_destroy(h)


def test_bind_checks_alignment_and_size():
    h = S.sos_plan(3, 2, 5, "fp64")
    ws, st = ctypes.c_size_t(), ctypes.c_size_t()
    S._lib.sos_plan_query(h, None, None, ctypes.byref(ws), ctypes.byref(st))
    assert S._lib.sos_plan_bind(h, ctypes.c_void_p(256 * 7 + 8), ws.value, None) == -1
    assert S._lib.sos_plan_bind(h, ctypes.c_void_p(256 * 7), ws.value - 1, None) == -3
    S._lib.sos_plan_destroy(h)


def test_adam_argument_errors():
    h = S.sos_plan(3, 2, 5, "fp64")
    S._lib.sos_plan_destroy(h)
    bad = S.Adam(lr=-1.0)
    z = ctypes.c_void_p(0)
    h2 = S.sos_plan(3, 2, 5, "fp64")
    # unbound check happens first; the Adam check is exercised on the GPU tests
    assert S._lib.sos_step(h2, z, z, 1, z, ctypes.byref(bad.c()), z, 0, z) == -1
    S._lib.sos_plan_destroy(h2)


def test_noalloc_argument_errors():
    """sos_loss_grad_noalloc checks its arguments before touching a GPU."""
    z = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every check below fails first
    assert S._lib.sos_loss_grad_noalloc(z, fake, fake, fake, z, z, 0, z) == -1
    h = S.sos_plan(3, 2, 5, "fp32")
    assert S._lib.sos_loss_grad_noalloc(h, z, fake, fake, z, z, 0, z) == -1
    assert S._lib.sos_loss_grad_noalloc(h, fake, fake, fake, z, z, 64, z) == -1
    assert b"flags" in S._lib.sos_last_error()
    S._lib.sos_plan_destroy(h)
    # (10, 5) at full rank needs ~213 MiB of workspace, above the static 64 MiB
    big = S.sos_plan(10, 5, 3003, "bf16x3")
    ws = ctypes.c_size_t()
    S._lib.sos_plan_query(big, None, None, ctypes.byref(ws), None)
    assert ws.value > 64 << 20
    assert S._lib.sos_loss_grad_noalloc(big, fake, fake, fake, z, z, 0, z) == -2
    assert b"static" in S._lib.sos_last_error()
    S._lib.sos_plan_destroy(big)
