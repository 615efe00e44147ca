"""Plain FP64 CPU oracle of continuous stream processing: overlap-save
segments of a long strain series, each Fourier transformed, its noise power
spectral density estimated from the segment itself, and searched over the
part of the segment that a circular correlation leaves valid.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
of the GPU build and the CPU-baseline leg of the benchmark may import or run
this module.  The GPU library never calls it and shares no code with it.

What it follows (Bosi, "cuInspiral", arXiv:1006.4644): the per-chunk loop
of "Matched filtering" (for each input data chunk, the loop over the bank),
applied to consecutive chunks of a continuous stream with the 50 % overlap
that the online-analysis table implies, and the search of each chunk.

Readings (the paper describes neither the chunking nor a PSD estimate; each
is also what the GPU path implements):

* Segments of n samples with stride n/2: segment s covers the global samples
  [s n/2, s n/2 + n).  Its valid lags are j in [n/4, 3n/4) (global
  s n/2 + j); consecutive valid regions tile [n/4, (S+1) n/2 - n/4 ... )
  without gaps or overlaps.  Chirps up to n/4 samples long are filtered
  without wrap-around there.
* Segment spectrum (no window): x~_k = dt sum_j x_j e^{-2 pi i jk/n},
  k = 0..n/2.
* PSD estimate: the Hann-windowed periodogram of the segment,
  w_j = sin^2(pi j / n), X_k = dt sum_j w_j x_j e^{-2 pi i jk/n},
  P_k = 2 |X_k|^2 / (T W2) with W2 = (1/n) sum w_j^2 = 3/8 (so E P_k = S_k
  for a slowly varying one-sided PSD S), smoothed over the in-band bins
  [k - h, k + h] intersected with [k_low, n/2 - 1] (Daniell's average);
  S_k = 0 outside [k_low, n/2 - 1]; optionally the mean of that estimate
  over the segment and the K - 1 before it (Welch's average over time).
* Search of each segment: the frequency-domain path of mf_oracle with that
  spectrum and PSD over [n/4, 3n/4), merged across templates per window;
  windows of W samples align globally, and each lies inside one segment's
  valid region, because W divides n/4 (a window of n/2 would span two
  segments and be reported twice).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import mf_oracle as O

__all__ = ["segment_count", "segment_spectrum", "hann", "psd_estimate",
           "stream_search"]


def segment_count(total: int, n: int) -> int:
    """Complete segments of stride n/2 in a stream of `total` samples."""
    return 0 if total < n else (total - n) // (n // 2) + 1


def segment_spectrum(xs, fs: float):
    """x~_k = dt sum_j x_j e^{-2 pi i jk/n}, k = 0..n/2 (complex128)."""
    return np.fft.rfft(np.asarray(xs, dtype=np.float64)) / fs


def hann(n: int):
    j = np.arange(n, dtype=np.float64)
    return np.sin(np.pi * j / n) ** 2


def psd_estimate(xs, fs: float, f_low: float, h: int):
    """Smoothed Hann periodogram of one segment (float64 [n/2 + 1])."""
    n = len(xs)
    T = n / fs
    X = np.fft.rfft(hann(n) * np.asarray(xs, dtype=np.float64)) / fs
    P = 2.0 * np.abs(X) ** 2 / (T * 0.375)
    kl, kh = int(math.ceil(f_low * T)), n // 2 - 1
    S = np.zeros(n // 2 + 1)
    for k in range(kl, kh + 1):
        a, b = max(k - h, kl), min(k + h, kh)
        S[k] = np.mean(P[a:b + 1])
    return S


def stream_search(x, n: int, fs: float, f_low: float, bank, thr: float,
                  window: int, h: int, avg: int = 1):
    """Search every complete segment of the stream `x` (float64), with the
    PSD of segment s the mean of the estimates of segments
    max(0, s - avg + 1) .. s.  Returns (per-segment list of
    {w_global: (tmpl, j_global, rho2)}, per-segment PSDs used, per-segment
    spectra)."""
    # windows must not straddle two segments' valid regions, which start
    # at n/4 past a multiple of n/2: W divides n/4
    if window < 1 or (n // 4) % window != 0:
        raise ValueError(f"window {window} must divide n/4 = {n // 4}")
    stride = n // 2
    out, psds, specs, own = [], [], [], []
    for s in range(segment_count(len(x), n)):
        xs = x[s * stride:s * stride + n]
        xt = segment_spectrum(xs, fs)
        own.append(psd_estimate(xs, fs, f_low, h))
        S = np.mean(own[max(0, s - avg + 1):s + 1], axis=0)
        res = O.search(xt, S, n, fs, f_low, bank, thr, window, j_lo=n // 4,
                       j_hi=3 * n // 4)
        shift_w = (s * stride) // window
        out.append({w + shift_w: (t, j + s * stride, r2)
                    for w, (t, j, r2) in res["merged"].items()})
        psds.append(S)
        specs.append(xt)
    return out, psds, specs
