"""Template-bank placement (host library, CPU): the metric against the
oracle's, the lattice's range and determinism, and its coverage checked by
the oracle's brute-force match."""

import numpy as np
import pytest

from oracle import bank_oracle as B
from paper_1006_4644_amd import ci, synth


@pytest.fixture(scope="module")
def lib():
    try:
        return ci.load()
    except ci.LibraryMissing:
        pytest.skip("libci.so not built")


@pytest.mark.parametrize("n,fs,fl", [(1 << 16, 4096.0, 20.0), (1 << 17, 8192.0, 30.0)])
@pytest.mark.parametrize("m1,m2", [(1.4, 1.4), (5.0, 2.0), (12.0, 9.0)])
def test_metric_matches_oracle(lib, n, fs, fl, m1, m2):
    psd = synth.make_psd(n, fs)
    g = lib.bank_metric(psd, n, fs, fl, m1, m2)
    go = B.metric(psd, n, fs, fl, m1, m2)
    assert np.max(np.abs(g - go) / np.abs(go)) < 1e-7
    # order of the masses does not matter
    assert np.array_equal(lib.bank_metric(psd, n, fs, fl, m2, m1), g)


def test_lattice_range_and_determinism(lib):
    n, fs, fl = 1 << 16, 4096.0, 40.0
    psd = synth.make_psd(n, fs)
    bank = lib.make_bank_lattice(3.0, 8.0, 0.97, psd, n, fs, fl)
    assert len(bank) > 20
    assert np.all(bank[:, 0] >= bank[:, 1])
    assert np.all(bank >= 3.0) and np.all(bank <= 8.0)
    assert np.array_equal(lib.make_bank_lattice(3.0, 8.0, 0.97, psd, n, fs, fl), bank)
    # a looser match needs fewer templates, a tighter one more
    assert len(lib.make_bank_lattice(3.0, 8.0, 0.95, psd, n, fs, fl)) < len(bank)
    assert len(lib.make_bank_lattice(3.0, 8.0, 0.98, psd, n, fs, fl)) > len(bank)


def test_lattice_arguments(lib):
    n, fs, fl = 1 << 16, 4096.0, 40.0
    psd = synth.make_psd(n, fs)
    for args in ((8.0, 3.0, 0.97), (0.0, 3.0, 0.97), (3.0, 8.0, 1.0), (3.0, 8.0, 0.4)):
        with pytest.raises(ci.CiError) as e:
            lib.make_bank_lattice(*args, psd, n, fs, fl)
        assert e.value.code == ci.EINVAL
    with pytest.raises(ci.CiError) as e:
        lib.bank_metric(psd, n, fs, fl, -1.0, 2.0)
    assert e.value.code == ci.EINVAL


def test_lattice_coverage_by_brute_force_match(lib):
    """Random points of the range: the best continuous-time match over the
    bank (oracle, FP64) reaches the requested minimum."""
    n, fs, fl, mm = 1 << 16, 4096.0, 40.0, 0.97
    psd = synth.make_psd(n, fs)
    bank = lib.make_bank_lattice(3.0, 8.0, mm, psd, n, fs, fl)
    tb = np.array([B.chirp_times(a, b, fl) for a, b in bank])
    rng = np.random.default_rng(2024)
    worst = 1.0
    for _ in range(16):
        a, b = rng.uniform(3.0, 8.0, 2)
        m1, m2 = max(a, b), min(a, b)
        g = lib.bank_metric(psd, n, fs, fl, m1, m2)
        d = tb - np.array(B.chirp_times(m1, m2, fl))
        near = np.argsort(np.einsum("ij,jk,ik->i", d, g, d))[:6]
        best = max(B.match(psd, n, fs, fl, (m1, m2), tuple(bank[k])) for k in near)
        worst = min(worst, best)
    print(f"{len(bank)} templates, worst best-match {worst:.4f}")
    assert worst >= mm
