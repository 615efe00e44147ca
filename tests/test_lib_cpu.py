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


@pytest.mark.parametrize("fs,f_low,lo,hi", [(4096.0, 20.0, 1.0, 30.0),
                                            (4096.0, 10.0, 1.0, 50.0)])
def test_length_classes_match_oracle(lib, fs, f_low, lo, hi):
    """Class of every template equals the oracle's rule (shortest segment
    covering the 2PN chirp duration), including the clamp to the last."""
    from paper_1006_4644_amd import synth
    bank = synth.draw_masses(3000, lo, hi, "loguniform", 4647)
    classes = synth.CLASS_LENGTHS
    got = lib.length_classes(bank, fs, f_low, classes)
    want = [classes.index(O.length_class(m1, m2, f_low, fs, classes)) for m1, m2 in bank]
    assert got.tolist() == want
    # m1 < m2 order does not matter
    assert np.array_equal(lib.length_classes(bank[:, ::-1], fs, f_low, classes), got)


def test_length_classes_reject_bad_input(lib):
    bank = np.array([[1.4, 1.4]])
    for classes in ([], [3 << 16], [1 << 18, 1 << 17]):
        with pytest.raises(ci.CiError) as e:
            lib.length_classes(bank, 4096.0, 20.0, classes)
        assert e.value.code == ci.EINVAL
    with pytest.raises(ci.CiError):
        lib.length_classes(np.array([[0.0, 1.4]]), 4096.0, 20.0, [1 << 17])
    assert lib.length_classes(np.zeros((0, 2)), 4096.0, 20.0, [1 << 17]).shape == (0,)


def test_ctypes_structs_match_header(tmp_path):
    """Sizes and field offsets of the binding's ctypes structures equal the C
    compiler's for include/ci.h (compiled with gcc, no GPU)."""
    import ctypes
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    structs = {"ci_tune": ci._Tune, "ci_class_job": ci._ClassJob, "ci_bank_spec": ci._BankSpec,
               "ci_segment_spec": ci._SegSpec, "ci_kernel_time": ci._KernelTime,
               "ci_stream_spec": ci._StreamSpec}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ci.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    dtypes = {"ci_trigger": ci.TRIGGER_DTYPE, "ci_tparams": ci.TPARAMS_DTYPE,
              "ci_tdparams": ci.TDPARAMS_DTYPE}
    for cname, dt in dtypes.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname in dt.names:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {tuple(l.split()[:-1]): int(l.split()[-1]) for l in out.splitlines()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
    for cname, dt in dtypes.items():
        assert got[(cname, "size")] == dt.itemsize, cname
        for fname in dt.names:
            assert got[(cname, fname)] == dt.fields[fname][1], (cname, fname)


def test_tune_cache_roundtrip(tmp_path):
    """The launch-configuration cache: tuned entries are written per device
    key, length and precision, merged into an existing file, and applied
    only to a context of the same device key."""
    from paper_1006_4644_amd import ci

    class Fake:
        def __init__(self, tuned):
            self.t = {}
            self.tuned = tuned
            self.applied = []

        def get_tune(self, l2, p):
            d = dict(tile_c=8, tile_j=4 + 4 * (l2 % 2), p2_per_cu=l2 % 5, batch=16 * l2,
                     streams=1 + p % 2, p2_wave=l2 % 2, tuned=int((l2, p) in self.tuned))
            return d

        def set_tune(self, l2, p, c, j, p2, batch, streams=2, p2_wave=0):
            self.applied.append((l2, p, c, j, p2, batch, streams, p2_wave))

    path = str(tmp_path / "tune.json")
    assert ci.load_tune_cache(Fake(set()), path, "dev") == []
    assert ci.save_tune_cache(Fake({(20, 0), (17, 1)}), path, "devA") == 2
    assert ci.save_tune_cache(Fake({(21, 2)}), path, "devB") == 1
    fa = Fake(set())
    assert sorted(ci.load_tune_cache(fa, path, "devA")) == [(17, 1), (20, 0)]
    assert sorted(fa.applied) == [(17, 1, 8, 8, 2, 272, 2, 1), (20, 0, 8, 4, 0, 320, 1, 0)]
    fb = Fake(set())
    assert ci.load_tune_cache(fb, path, "devB") == [(21, 2)]
    assert ci.load_tune_cache(Fake(set()), path, "other") == []
