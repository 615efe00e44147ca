"""Host-side checks of the C-ABI library (no GPU needed).

The built library loads, exports every function that include/ci.h
declares, and its host-only bank maker reproduces the oracle's
counter-based generator bit for bit.
"""
import os
import re

import numpy as np
import pytest

from oracle import mf_oracle as O
from paper_1006_4644_amd import ci

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ci.LIB_PATH):
        from paper_1006_4644_amd import build
        build.build()
    return ci.load()


def _declared():
    src = open(os.path.join(ROOT, "include", "ci.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ci_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_function(lib):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib.dll, n), n
    assert sorted(ci.EXPORTED_SYMBOLS) == names


def test_version(lib):
    assert "gfx950" in lib.version()


@pytest.mark.parametrize("kind,lo,hi,seed,n", [
    (ci.BANK_LOGUNIFORM, 1.0, 10.0, 4646, 3000),
    (ci.BANK_UNIFORM, 1.0, 3.0, 1, 257),
    (ci.BANK_LOGUNIFORM, 1.0, 50.0, 2**63 + 5, 100),
    (ci.BANK_GRID, 1.0, 3.0, 0, 10),
    (ci.BANK_GRID, 2.0, 2.0, 0, 1),
    (ci.BANK_GRID, 1.0, 30.0, 0, 1000),
])
def test_make_bank_matches_oracle_bit_exact(lib, kind, lo, hi, seed, n):
    got = lib.make_bank(kind, lo, hi, seed, n)
    ref = O.make_bank(kind, lo, hi, seed, n)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("kind,lo,hi", [(ci.BANK_UNIFORM, 0.0, 1.0),
                                        (ci.BANK_UNIFORM, 3.0, 1.0),
                                        (7, 1.0, 2.0)])
def test_make_bank_rejects_bad_specs(lib, kind, lo, hi):
    with pytest.raises(ci.CiError) as ei:
        lib.make_bank(kind, lo, hi, 0, 4)
    assert ei.value.code == ci.EINVAL
    assert lib.dll.ci_last_error(None)


def test_make_bank_empty(lib):
    assert lib.make_bank(ci.BANK_UNIFORM, 1.0, 2.0, 0, 0).shape == (0, 2)


def test_struct_layouts():
    # ci_trigger is 32 bytes, ci_tparams 96 bytes (documented in ci.h)
    assert ci.TRIGGER_DTYPE.itemsize == 32
    assert ci.TPARAMS_DTYPE.itemsize == 96
