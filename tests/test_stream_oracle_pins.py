"""Pins of the stream oracle (CPU only): the windowed periodogram's exact
values for a sinusoid and its Parseval total, an unbiased PSD estimate on
coloured Gaussian noise of known spectrum, the tiling of the valid regions,
and an injection found once, at its global sample, in a long stream."""
import math

import numpy as np
import pytest

from oracle import mf_oracle as O
from oracle import stream_oracle as SO
from paper_1006_4644_amd import synth


def test_hann_periodogram_of_a_sinusoid():
    # A cos(2 pi k0 j / n): X_k0 = dt A n / 4, X_{k0 +- 1} = -dt A n / 8, so
    # P_k0 = A^2 T / 3 and the three bins carry the variance A^2 / 2
    n, fs, A, k0 = 4096, 1024.0, 3.0, 300
    T = n / fs
    x = A * np.cos(2 * np.pi * k0 * np.arange(n) / n)
    X = np.fft.rfft(SO.hann(n) * x) / fs
    assert abs(X[k0] - A * n / 4 / fs) < 1e-12 * A * n / fs
    assert abs(X[k0 + 1] + A * n / 8 / fs) < 1e-12 * A * n / fs
    S = SO.psd_estimate(x, fs, 10.0, 0)              # h = 0: the periodogram
    assert abs(S[k0] - A * A * T / 3) < 1e-10 * A * A * T
    assert abs(np.sum(S) / T - A * A / 2) < 1e-10 * A * A
    # smoothing over h bins averages: the 3-bin total spreads, conserved
    S5 = SO.psd_estimate(x, fs, 10.0, 5)
    assert abs(S5[k0] - (A * A * T / 3) * 1.5 / 11) < 1e-10 * A * A * T


def _coloured_stream(total, fs, fl, seed):
    """A time series of `total` samples whose spectrum is the synthetic
    noise of the matched-filter tests (one-sided PSD synth.make_psd)."""
    xt = synth.make_noise(total, fs, fl, synth.make_psd(total, fs), seed)
    return np.fft.irfft(xt, total) * fs


def test_psd_estimate_unbiased_on_coloured_noise():
    n, fs, fl, h = 1 << 15, 4096.0, 20.0, 16
    x = _coloured_stream(8 * n, fs, fl, 3)
    psd = synth.make_psd(n, fs)
    kl = int(math.ceil(fl * n / fs))
    ratios = []
    for s in range(4):
        S = SO.psd_estimate(x[s * n:(s + 1) * n], fs, fl, h)
        ratios.append(S[kl + 2 * h:n // 2 - 1] / psd[kl + 2 * h:n // 2 - 1])
        assert np.all(S[:kl] == 0) and S[n // 2] == 0
    r = np.concatenate(ratios)
    assert abs(np.mean(r) - 1) < 0.01
    # per-bin scatter of a (2h+1)-bin average of unit-mean exponential
    # variables whose neighbours correlate as the Hann window makes them
    # (complex correlation -2/3 at lag 1 and 1/6 at lag 2, so the powers
    # correlate by 4/9 and 1/36); the moving average leaves ~2000 independent
    # values in the four segments, so the scatter is known to ~2 %
    want = math.sqrt((1 + 2 * 4 / 9 + 2 / 36) / (2 * h + 1))
    assert abs(np.std(r) - want) < 0.06 * want
    # without the neighbour correlation the scatter would be 28 % lower
    assert np.std(r) > 1.2 / math.sqrt(2 * h + 1)


@pytest.mark.parametrize("segs", [1, 2, 5])
def test_valid_regions_tile_the_stream(segs):
    n = 1 << 16
    total = n + (segs - 1) * n // 2
    assert SO.segment_count(total, n) == segs
    assert SO.segment_count(total + n // 2 - 1, n) == segs
    cover = np.zeros(total, int)
    for s in range(segs):
        cover[s * n // 2 + n // 4:s * n // 2 + 3 * n // 4] += 1
    assert np.all(cover[n // 4:total - n // 4] == 1)
    assert np.all(cover[:n // 4] == 0) and np.all(cover[total - n // 4:] == 0)


def test_stream_finds_injection_once_at_its_sample():
    """A loud short chirp in a long noisy stream is found in exactly one
    segment (the one whose valid region holds it), at its global sample,
    with the PSD estimated from the data."""
    n, fs, fl, h = 1 << 16, 4096.0, 30.0, 16
    segs = 5
    total = n + (segs - 1) * n // 2
    m1, m2, snr, j0 = 8.0, 6.0, 25.0, 3 * n // 2 + 5000
    psd_t = synth.make_psd(total, fs)
    xt = synth.make_noise(total, fs, fl, psd_t, 11)
    hinj = O.spa_htilde(total, fs, fl, m1, m2, tc=j0 / fs, phic=0.4)
    _, _, _, kl, kh = O.band(m1, m2, total, fs, fl)
    xt = xt + hinj * (snr / math.sqrt(O.sigma2(hinj, psd_t, fs / total, kl, kh)))
    x = np.fft.irfft(xt, total) * fs
    assert O.tau_2pn(fl, m1, m2) < n / 4 / fs
    bank = np.array([[m1, m2], [3.0, 2.0], [12.0, 10.0]])
    out, psds, specs = SO.stream_search(x, n, fs, fl, bank, 8.0, 4096, h)
    assert len(out) == segs
    hits = [(s, w, v) for s, m in enumerate(out) for w, v in m.items() if v[2] > 15.0 ** 2]
    assert len(hits) == 1
    s, w, (t, j, r2) = hits[0]
    assert t == 0 and abs(j - j0) <= 1
    assert s * n // 2 + n // 4 <= j < s * n // 2 + 3 * n // 4
    assert w == j // 4096
    assert abs(math.sqrt(r2) - snr) < 0.15 * snr


def test_psd_average_covers_the_last_k_segments():
    """The K-segment PSD average (Welch's average over time) of the stream
    search, pinned by white noise whose power steps by a factor of 4 from
    one half-segment block to the next.  For white noise of variance
    sigma^2 c_j^2 the Hann periodogram is unbiased for the window-weighted
    mean power: E P_k = (2 sigma^2 / fs) sum_j w_j^2 c_j^2 / sum_j w_j^2,
    and the Hann window puts half of sum w^2 on each half of a segment, so
    segment s (blocks s and s + 1) estimates (2 sigma^2 / fs) (c_s^2 +
    c_{s+1}^2) / 2.  The PSD used for segment s must then be the mean of
    those over segments max(0, s - K + 1) .. s: fewer at the stream start,
    and never a later segment.  A window off by one segment, or a division
    by K at the start, moves the figure by 25 % or more."""
    n, fs, fl, h, K, segs = 1 << 16, 4096.0, 20.0, 8, 3, 6
    half = n // 2
    sigma = 1.5
    rng = np.random.default_rng(2024)
    blocks = segs + 1
    c2 = 4.0 ** np.arange(blocks)
    x = rng.standard_normal(blocks * half) * sigma * np.repeat(np.sqrt(c2), half)
    bank = np.array([[3.0, 2.0]])
    _, psds, _ = SO.stream_search(x, n, fs, fl, bank, 1e3, 4096, h, avg=K)
    assert len(psds) == segs
    kl = int(math.ceil(fl * n / fs))
    white = 2.0 * sigma ** 2 / fs
    own = (c2[:-1] + c2[1:]) / 2.0                      # segment s: blocks s, s + 1
    for s in range(segs):
        want = np.mean(own[max(0, s - K + 1):s + 1])
        got = np.mean(psds[s][kl + h:half - 1 - h]) / white
        assert abs(got / want - 1.0) < 0.04, (s, got, want)
        # the alternatives a mistake in the window would give are far off
        for alt in (np.mean(own[max(0, s - K):s + 1]),
                    np.mean(own[max(0, s - K + 2):s + 1]),
                    np.sum(own[max(0, s - K + 1):s + 1]) / K,
                    np.mean(own[max(0, s - K + 1):min(s + 2, segs)])):
            if abs(alt / want - 1.0) > 1e-9:
                assert abs(got / alt - 1.0) > 0.15, (s, got, alt)
    # K = 1 is each segment's own estimate
    _, own_psds, _ = SO.stream_search(x[:n + half], n, fs, fl, bank, 1e3, 4096, h)
    for s in range(2):
        got = np.mean(own_psds[s][kl + h:half - 1 - h]) / white
        assert abs(got / own[s] - 1.0) < 0.04, (s, got, own[s])
