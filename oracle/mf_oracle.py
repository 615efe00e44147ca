"""Plain FP64 CPU oracle for batched matched filtering of compact-binary chirps.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
of the GPU build and the CPU-baseline leg of the benchmark may import or run
this module.  The GPU library never calls it and shares no code with it.

What it computes (Bosi, "cuInspiral", arXiv:1006.4644):

* the per-template pipeline of the "Matched filtering" section: generate and
  normalise the template, correlate it with the data through the coloured-
  noise inner product of eq. (matchedfilter), combine the two quadratures,
  keep the maxima above a threshold, and finally reduce the candidates of all
  templates to local maxima;
* the template mismatch of eq. (mismatch) ("Numerical accuracy" section).

Everything is written as the plain definition, in float64, with no blocking,
fusion or reordering.  The only library primitive is numpy's FFT, used as
the unnormalised inverse DFT.  Conventions the paper leaves open are fixed
as follows (the full list of readings lives with the design notes):

* one-sided spectra on f_k = k df, df = fs/n; x~_k = dt * sum_j x_j e^{-2 pi i jk/n};
* inner product <a, b> = 4 Re sum_k df a~_k b~_k* / S_k over the search band
  k_low <= k <= k_high (the paper's eq. (matchedfilter) made one-sided);
* template: restricted (Newtonian-amplitude) stationary-phase chirp with the
  2PN phase of Blanchet, Damour, Iyer, Will & Wiseman (1995), in the form used
  by Cutler & Flanagan (1994) and by FINDCHIRP (Allen et al., PRD 85, 122006):
      h~(f) = A f^{-7/6} exp(-i Psi(f)),
      Psi(f) = 2 pi f t_c - phi_c - pi/4 + 3/(128 eta v^5) [1 + (3715/756 +
               55 eta/9) v^2 - 16 pi v^3 + (15293365/508032 + 27145 eta/504 +
               3085 eta^2/72) v^4],   v = (pi M f)^{1/3};
* band: k_low = ceil(f_low T), k_high = min(floor(f_isco T), n/2 - 1) with
  the Schwarzschild ISCO f_isco = 1 / (6^{3/2} pi M);
* normalisation: the template is scaled so each quadrature has unit norm,
  so in Gaussian noise rho^2 = |z|^2 / sigma^2 is chi^2 with two degrees of
  freedom (mean 2);
* quadrature combination: the complex output z_j of one positive-frequency
  inverse DFT carries both quadratures, |z_j| / sigma = sqrt(c_+^2 + c_x^2);
* threshold: strict ">" (the pipeline's "c(t) > lambda");
* local maxima: aligned windows of W samples, argmax per window, ties to the
  smallest index; across templates, max per window, ties to the smaller
  template id;
* chi-squared veto (the test the Conclusions plan, ref. Chi2): p contiguous
  bands of equal sigma^2 share, chi2 = p sum_l |z_l - z/p|^2.

Every function below is pinned by tests that do not re-type its formula:
brute-force DFT, Parseval, the stationary-phase identity against an
independently written 2PN time-to-coalescence, the f^{-7/6} amplitude law,
the white-noise closed form of sigma^2, noise-free recovery of injections,
chi^2_2 statistics in noise, and brute force on tiny planted series; the
veto by its sum rule, its closed form for an exactly matching signal and
its chi^2_{2p-2} statistics in noise.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "T_SUN", "band", "spa_phase", "spa_htilde", "tau_2pn", "inner",
    "sigma2", "corr_spectrum", "idft", "snr_series", "peak",
    "window_triggers", "merge_windows", "mismatch", "splitmix64",
    "uniform01", "make_bank", "length_class", "search",
    "BANK_GRID", "BANK_UNIFORM", "BANK_LOGUNIFORM",
]

# G M_sun / c^3 in seconds (IAU nominal solar mass parameter / c^3).
T_SUN = 4.925490947641267e-6


def band(m1: float, m2: float, n: int, fs: float, f_low: float):
    """Search band of one template on an n-sample grid.

    Returns (M_seconds, eta, f_isco, k_low, k_high).  k_high < k_low means
    the chirp ends below f_low and the template is empty.
    """
    M = (m1 + m2) * T_SUN
    eta = m1 * m2 / ((m1 + m2) * (m1 + m2))
    T = n / fs
    f_isco = 1.0 / (6.0 * math.sqrt(6.0) * math.pi * M)
    k_low = int(math.ceil(f_low * T))
    k_high = min(int(math.floor(f_isco * T)), n // 2 - 1)
    return M, eta, f_isco, k_low, k_high


def spa_phase(f, m1: float, m2: float, tc: float = 0.0, phic: float = 0.0):
    """Stationary-phase Psi(f) of the restricted 2PN chirp (radians, float64)."""
    f = np.asarray(f, dtype=np.float64)
    M = (m1 + m2) * T_SUN
    eta = m1 * m2 / ((m1 + m2) * (m1 + m2))
    v = np.cbrt(math.pi * M * f)
    pn = (1.0
          + (3715.0 / 756.0 + 55.0 * eta / 9.0) * v ** 2
          - 16.0 * math.pi * v ** 3
          + (15293365.0 / 508032.0 + 27145.0 * eta / 504.0
             + 3085.0 * eta * eta / 72.0) * v ** 4)
    return (2.0 * math.pi * f * tc - phic - math.pi / 4.0
            + 3.0 / (128.0 * eta * v ** 5) * pn)


def spa_htilde(n: int, fs: float, f_low: float, m1: float, m2: float,
               tc: float = 0.0, phic: float = 0.0, amp: float = 1.0):
    """Frequency-domain template h~_k, k = 0..n/2 (complex128).

    h~_k = amp f_k^{-7/6} exp(-i Psi(f_k)) inside [k_low, k_high], else 0.
    """
    _, _, _, kl, kh = band(m1, m2, n, fs, f_low)
    out = np.zeros(n // 2 + 1, dtype=np.complex128)
    if kh < kl:
        return out
    k = np.arange(kl, kh + 1, dtype=np.float64)
    f = k * (fs / n)
    psi = spa_phase(f, m1, m2, tc, phic)
    out[kl:kh + 1] = amp * f ** (-7.0 / 6.0) * np.exp(-1j * psi)
    return out


def tau_2pn(f, m1: float, m2: float):
    """2PN time to coalescence from frequency f (seconds).

    tau = 5M/(256 eta) v^-8 [1 + (743/252 + 11 eta/3) v^2 - (32 pi/5) v^3
          + (3058673/508032 + 5429 eta/504 + 617 eta^2/72) v^4].
    Written independently of spa_phase; the stationary-phase relation
    dPsi/df = 2 pi (t_c - tau(f)) ties the two together.
    """
    f = np.asarray(f, dtype=np.float64)
    M = (m1 + m2) * T_SUN
    eta = m1 * m2 / ((m1 + m2) * (m1 + m2))
    v = np.cbrt(math.pi * M * f)
    return (5.0 * M / (256.0 * eta) / v ** 8
            * (1.0 + (743.0 / 252.0 + 11.0 * eta / 3.0) * v ** 2
               - 32.0 * math.pi / 5.0 * v ** 3
               + (3058673.0 / 508032.0 + 5429.0 * eta / 504.0
                  + 617.0 * eta * eta / 72.0) * v ** 4))


def inner(a, b, psd, df: float, k_lo: int, k_hi: int) -> float:
    """<a, b> = 4 Re sum_{k_lo..k_hi} df a_k conj(b_k) / S_k (eq. matchedfilter
    at zero lag, one-sided)."""
    sl = slice(k_lo, k_hi + 1)
    return float(4.0 * df * np.real(np.sum(a[sl] * np.conj(b[sl]) / psd[sl])))


def sigma2(htilde, psd, df: float, k_lo: int, k_hi: int) -> float:
    """Template norm sigma^2 = <h, h> = 4 df sum |h_k|^2 / S_k."""
    if k_hi < k_lo:
        return 0.0
    sl = slice(k_lo, k_hi + 1)
    return float(4.0 * df * np.sum(np.abs(htilde[sl]) ** 2 / psd[sl]))


def corr_spectrum(xtilde, htilde, psd, n: int, df: float, k_lo: int,
                  k_hi: int):
    """Z_k = 4 df x~_k conj(h~_k) / S_k on [k_lo, k_hi], 0 for every other k
    in [0, n) (the integrand of eq. matchedfilter on the positive half)."""
    Z = np.zeros(n, dtype=np.complex128)
    if k_hi < k_lo:
        return Z
    sl = slice(k_lo, k_hi + 1)
    Z[sl] = 4.0 * df * xtilde[sl] * np.conj(htilde[sl]) / psd[sl]
    return Z


def idft(Z):
    """Unnormalised inverse DFT z_j = sum_k Z_k exp(+2 pi i jk/n)."""
    Z = np.asarray(Z, dtype=np.complex128)
    return np.fft.ifft(Z) * Z.shape[-1]


def snr_series(xtilde, psd, n: int, fs: float, f_low: float, m1: float,
               m2: float):
    """Complex SNR series of one template: (z / sigma  (complex128, n), sigma^2).

    Steps 1-3 of the per-template loop: generate the chirp, normalise it,
    correlate it with the data for both quadratures at every lag.  An empty
    template (k_high < k_low) gives an all-zero series and sigma^2 = 0.
    """
    df = fs / n
    _, _, _, kl, kh = band(m1, m2, n, fs, f_low)
    h = spa_htilde(n, fs, f_low, m1, m2)
    s2 = sigma2(h, psd, df, kl, kh)
    if s2 <= 0.0:
        return np.zeros(n, dtype=np.complex128), 0.0
    z = idft(corr_spectrum(xtilde, h, psd, n, df, kl, kh))
    return z / math.sqrt(s2), s2


def peak(rho2) -> int:
    """Index of the largest rho^2; ties go to the smallest index."""
    return int(np.argmax(rho2))


def window_triggers(rho2, window: int, thr2: float, j_lo: int = 0,
                    j_hi: int | None = None):
    """Step 4 of the per-template loop: for each aligned window [wW, (w+1)W)
    restricted to [j_lo, j_hi), the window argmax m_w (ties to the smallest
    index) is a trigger when rho2[m_w] > thr2.  Returns [(w, m_w, rho2)]."""
    n = len(rho2)
    if j_hi is None:
        j_hi = n
    out = []
    n_win = (n + window - 1) // window
    for w in range(n_win):
        a = max(w * window, j_lo)
        b = min((w + 1) * window, j_hi, n)
        if a >= b:
            continue
        m = a + int(np.argmax(rho2[a:b]))
        if rho2[m] > thr2:
            out.append((w, m, float(rho2[m])))
    return out


def merge_windows(per_template):
    """Final reduction across templates: per window keep the largest rho^2,
    ties to the smaller template id.  ``per_template`` maps template id to
    its [(w, j, rho2)] list; returns {w: (tmpl, j, rho2)}."""
    best = {}
    for t in sorted(per_template):
        for (w, j, r2) in per_template[t]:
            cur = best.get(w)
            if cur is None or r2 > cur[2]:
                best[w] = (t, j, r2)
    return best


def mismatch(a, b, psd, df: float, k_lo: int, k_hi: int) -> float:
    """Eq. (mismatch): 1 - <a, b> / <a, a>."""
    return 1.0 - inner(a, b, psd, df, k_lo, k_hi) / inner(a, a, psd, df,
                                                           k_lo, k_hi)


# --- bank generation ---------------------------------------------------------
# Counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): draw i is
# mix(seed + (i + 1) * 0x9E3779B97F4A7C15), a uniform double is the top 53
# bits times 2^-53.  The library's bank maker implements the same published
# generator on its own.

BANK_GRID, BANK_UNIFORM, BANK_LOGUNIFORM = 0, 1, 2
_M64 = (1 << 64) - 1


def splitmix64(i: int, seed: int) -> int:
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def uniform01(i: int, seed: int) -> float:
    return (splitmix64(i, seed) >> 11) * (1.0 / 9007199254740992.0)


def make_bank(kind: int, m_min: float, m_max: float, seed: int, n: int):
    """(n, 2) float64 bank of (m1, m2), canonical m1 >= m2.

    GRID: g = ceil(sqrt(n)) masses evenly spaced on [m_min, m_max]; template
    t takes (m[t // g], m[t % g]).  UNIFORM / LOGUNIFORM: m1, m2 drawn from
    draws 2t and 2t+1 of the counter-based generator.
    """
    out = np.empty((n, 2), dtype=np.float64)
    if kind == BANK_GRID:
        g = math.isqrt(n)
        if g * g < n:
            g += 1
        for t in range(n):
            ms = []
            for i in (t // g, t % g):
                ms.append(m_min if g == 1 else
                          m_min + (m_max - m_min) * i / (g - 1))
            out[t] = (max(ms), min(ms))
        return out
    for t in range(n):
        ms = []
        for d in (2 * t, 2 * t + 1):
            u = uniform01(d, seed)
            if kind == BANK_UNIFORM:
                ms.append(m_min + u * (m_max - m_min))
            elif kind == BANK_LOGUNIFORM:
                ms.append(m_min * math.exp(u * math.log(m_max / m_min)))
            else:
                raise ValueError("unknown bank kind")
        out[t] = (max(ms), min(ms))
    return out


def length_class(m1: float, m2: float, f_low: float, fs: float,
                 classes=(1 << 17, 1 << 18, 1 << 19, 1 << 20)) -> int:
    """Smallest segment length n_c whose duration n_c/fs covers the chirp's
    2PN duration from f_low; the largest class when none does."""
    tau = float(tau_2pn(f_low, m1, m2))
    for nc in classes:
        if tau <= nc / fs:
            return nc
    return classes[-1]


def chisq_edges(m1: float, m2: float, n: int, fs: float, f_low: float, psd,
                bands: int):
    """Bin edges e_0 .. e_p of the chi-squared veto's frequency bands.

    The planned chi-squared test of the Conclusions (their ref. Chi2; the
    time-frequency discriminator of B. Allen, PRD 71, 062001 (2005)) splits
    the template band [k_low, k_high] into p contiguous bands carrying equal
    shares of sigma^2.  Reading: with the inclusive running sum
    c_k = sum_{k_low <= k' <= k} |h~_k'|^2 / S_k', edge e_l (0 < l < p) is the
    first bin with c_k >= (l / p) c_{k_high}; e_0 = k_low, e_p = k_high + 1;
    band l is [e_l, e_{l+1}).
    """
    df = fs / n
    _, _, _, kl, kh = band(m1, m2, n, fs, f_low)
    if kh < kl:
        return None
    h = spa_htilde(n, fs, f_low, m1, m2)
    c = np.cumsum(np.abs(h[kl:kh + 1]) ** 2 / psd[kl:kh + 1])
    edges = [kl]
    for l in range(1, bands):
        edges.append(kl + int(np.searchsorted(c, (l / bands) * c[-1], side="left")))
    edges.append(kh + 1)
    return edges


def chisq(xtilde, psd, n: int, fs: float, f_low: float, m1: float, m2: float,
          j: int, bands: int):
    """Chi-squared veto value at sample j: p sum_l |z_l(j) - z(j)/p|^2, where
    z_l is the SNR series (same normalisation as snr_series) of the
    correlation restricted to band l, so that z = sum_l z_l.  Returns
    (chi2, z(j), [z_l(j)]); None for an empty template.  In Gaussian noise
    chi2 has 2p - 2 degrees of freedom (each quadrature of z has unit
    variance); for a signal exactly matching the template it vanishes up to
    the discreteness of the band edges."""
    df = fs / n
    _, _, _, kl, kh = band(m1, m2, n, fs, f_low)
    edges = chisq_edges(m1, m2, n, fs, f_low, psd, bands)
    if edges is None:
        return None
    h = spa_htilde(n, fs, f_low, m1, m2)
    s = math.sqrt(sigma2(h, psd, df, kl, kh))
    k = np.arange(n, dtype=np.int64)
    ph = np.exp(2j * np.pi * ((k * j) % n) / n)
    Z = corr_spectrum(xtilde, h, psd, n, df, kl, kh) / s
    zl = [complex(np.sum(Z[edges[l]:edges[l + 1]] * ph[edges[l]:edges[l + 1]]))
          for l in range(bands)]
    z = sum(zl)
    chi2 = bands * sum(abs(v - z / bands) ** 2 for v in zl)
    return chi2, z, zl


def search(xtilde, psd, n: int, fs: float, f_low: float, bank, thr: float,
           window: int, j_lo: int = 0, j_hi: int | None = None,
           keep_series: bool = False):
    """The whole per-chunk pipeline over a bank.

    Returns a dict with, per template t: 'peaks'[t] = (j*, rho2*, z*/sigma)
    ((-1, 0, 0) for an empty template), 'triggers'[t] = [(w, j, rho2)],
    'sigma2'[t]; the cross-template 'merged' windows; and, when asked, the
    complex SNR 'series'.
    """
    thr2 = thr * thr
    peaks, trig, s2s, series = [], {}, [], []
    for t, (m1, m2) in enumerate(np.asarray(bank, dtype=np.float64)):
        zs, s2 = snr_series(xtilde, psd, n, fs, f_low, float(m1), float(m2))
        s2s.append(s2)
        if s2 <= 0.0:
            peaks.append((-1, 0.0, 0j))
            trig[t] = []
            if keep_series:
                series.append(zs)
            continue
        r2 = zs.real ** 2 + zs.imag ** 2
        j = peak(r2) if j_lo == 0 and j_hi is None else \
            j_lo + peak(r2[j_lo:j_hi])
        peaks.append((j, float(r2[j]), complex(zs[j])))
        trig[t] = window_triggers(r2, window, thr2, j_lo, j_hi)
        if keep_series:
            series.append(zs)
    out = {"peaks": peaks, "triggers": trig, "sigma2": s2s,
           "merged": merge_windows(trig)}
    if keep_series:
        out["series"] = series
    return out
