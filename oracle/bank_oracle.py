"""Plain FP64 CPU oracle of template-bank geometry: chirp-time coordinates,
the parameter-space metric of the stationary-phase chirp, and the match
between two templates maximised over time and phase.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
of the GPU build and the CPU-baseline leg of the benchmark may import or run
this module.  The GPU library never calls it and shares no code with it.

What it follows (Bosi, "cuInspiral", arXiv:1006.4644): the template bank of
"Matched filtering", whose points are placed so that neighbouring templates
lose at most a tolerable fraction of SNR (the paper's footnote: 2-5 %
mismatch), with the mismatch of eq. (mismatch) read as one minus the match.

Readings (the paper gives no placement method):

* Coordinates: the chirp times at f_0 = f_low (Sathyaprakash 1994),
      tau_0 = 5 / (256 pi f0 eta) (pi M f0)^{-5/3},
      tau_3 = 1 / (8 f0 eta) (pi M f0)^{-2/3},
  in which the metric of the low-order chirp is nearly constant.
* Match: M(a, b) = max over t_c and phi_c of <h_a, h_b> / (|h_a| |h_b|) with
  the one-sided inner product of the search, over the band of both.
* Metric (Owen, PRD 53, 6749 (1996)): for a phase change dPsi(f) the match is
  1 - (1/2) Var_J[dPsi] to second order, Var_J the variance under the
  weight w(f) = f^{-7/3}/S(f) on the template's band, after maximising over
  phi_c (removes the mean) and t_c (projects out 2 pi f).  With
  psi_a = dPsi/dtheta_a (theta = (tau_0, tau_3), by central differences of
  the 2PN phase) and C the J-covariance of (2 pi f, psi_0, psi_3):
      gamma_ab = (1/2) (C_ab - C_at C_bt / C_tt),
  so 1 - M ~ gamma_ab dtheta^a dtheta^b.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import mf_oracle as O

__all__ = ["chirp_times", "masses_from_chirp_times", "spa_phase_m_eta",
           "metric", "match"]


def chirp_times(m1: float, m2: float, f0: float):
    M = (m1 + m2) * O.T_SUN
    eta = m1 * m2 / (m1 + m2) ** 2
    x = math.pi * M * f0
    return (5.0 / (256.0 * math.pi * f0 * eta) * x ** (-5.0 / 3.0),
            1.0 / (8.0 * f0 * eta) * x ** (-2.0 / 3.0))


def _M_eta(tau0: float, tau3: float, f0: float):
    """(M seconds, eta) from the chirp times (eta may exceed 1/4)."""
    x = 5.0 * tau3 / (32.0 * math.pi * tau0)          # pi M f0
    M = x / (math.pi * f0)
    eta = 1.0 / (8.0 * f0 * tau3) * x ** (-2.0 / 3.0)
    return M, eta


def masses_from_chirp_times(tau0: float, tau3: float, f0: float):
    """(m1, m2) in solar masses, m1 >= m2; None when eta > 1/4 (beyond the
    rounding of an equal-mass point)."""
    M, eta = _M_eta(tau0, tau3, f0)
    if eta > 0.25 * (1.0 + 1e-12):
        return None
    eta = min(eta, 0.25)
    mt = M / O.T_SUN
    d = math.sqrt(max(0.0, 1.0 - 4.0 * eta))
    return 0.5 * mt * (1.0 + d), 0.5 * mt * (1.0 - d)


def spa_phase_m_eta(f, M: float, eta: float):
    """The 2PN stationary-phase Psi(f) (t_c = phi_c = 0) from (M, eta)."""
    f = np.asarray(f, dtype=np.float64)
    v = np.cbrt(math.pi * M * f)
    pn = (1.0 + (3715.0 / 756.0 + 55.0 * eta / 9.0) * v ** 2 - 16.0 * math.pi * v ** 3
          + (15293365.0 / 508032.0 + 27145.0 * eta / 504.0
             + 3085.0 * eta * eta / 72.0) * v ** 4)
    return -math.pi / 4.0 + 3.0 / (128.0 * eta * v ** 5) * pn


def metric(psd, n: int, fs: float, f_low: float, m1: float, m2: float,
           k_high: int | None = None):
    """gamma (2 x 2, float64) in (tau_0, tau_3) at the template (m1, m2), on
    its band [k_low, k_high] (k_high: the template's own by default)."""
    df = fs / n
    M, eta, _, kl, kh = O.band(m1, m2, n, fs, f_low)
    if k_high is not None:
        kh = k_high
    k = np.arange(kl, kh + 1)
    f = k * df
    w = f ** (-7.0 / 3.0) / psd[kl:kh + 1]
    w = w / np.sum(w)
    t0, t3 = chirp_times(m1, m2, f_low)
    cols = [2.0 * math.pi * f]
    for a, th in enumerate((t0, t3)):
        h = 1e-6 * th
        lo = [t0, t3]
        hi = [t0, t3]
        lo[a] -= h
        hi[a] += h
        cols.append((spa_phase_m_eta(f, *_M_eta(hi[0], hi[1], f_low))
                     - spa_phase_m_eta(f, *_M_eta(lo[0], lo[1], f_low))) / (2 * h))
    P = np.array(cols)
    mean = P @ w
    C = (P * w) @ P.T - np.outer(mean, mean)
    g = 0.5 * (C[1:, 1:] - np.outer(C[1:, 0], C[1:, 0]) / C[0, 0])
    return g


def match(psd, n: int, fs: float, f_low: float, a, b, continuous: bool = True,
          band=None):
    """Match of templates a = (m1, m2) and b, maximised over phase and time;
    each template keeps its own band (norm over it, overlap over the common
    part), or, with band = (k_lo, k_hi), both are cut to that band (the
    fixed band the metric assumes).  Time: the best circular lag of
    the sampled correlation, then (continuous=True) the exact correlation
    sum maximised over real lags within one sample of it by golden-section
    search, the continuous-time match the metric approximates."""
    df = fs / n
    ha = O.spa_htilde(n, fs, f_low, *a)
    hb = O.spa_htilde(n, fs, f_low, *b)
    _, _, _, kl, kha = O.band(*a, n, fs, f_low)
    _, _, _, _, khb = O.band(*b, n, fs, f_low)
    if band is not None:
        kl, kha = band
        khb = kha
        ha = O.spa_htilde(n, fs, 0.5 * f_low, *a)   # not cut at f_low ...
        hb = O.spa_htilde(n, fs, 0.5 * f_low, *b)   # ... nor, below, at the ISCO
        _, _, _, _, ea = O.band(*a, n, fs, f_low)
        _, _, _, _, eb = O.band(*b, n, fs, f_low)
        if min(ea, eb) < kha:
            raise ValueError("band reaches beyond a template's ISCO")
    sa = O.sigma2(ha, psd, df, kl, kha)
    sb = O.sigma2(hb, psd, df, kl, khb)
    Z = np.zeros(n, dtype=np.complex128)
    kh = min(kha, khb)
    Z[kl:kh + 1] = 4.0 * df * ha[kl:kh + 1] * np.conj(hb[kl:kh + 1]) / psd[kl:kh + 1]
    z = O.idft(Z)
    j = int(np.argmax(np.abs(z)))
    best = float(np.abs(z[j]))
    if continuous:
        k = np.arange(kl, kh + 1, dtype=np.float64)
        Zb = Z[kl:kh + 1]

        def corr(t):
            return float(np.abs(np.sum(Zb * np.exp(2j * np.pi * k * t / n))))
        lo, hi = j - 1.0, j + 1.0
        g = (math.sqrt(5.0) - 1.0) / 2.0
        x1, x2 = hi - g * (hi - lo), lo + g * (hi - lo)
        f1, f2 = corr(x1), corr(x2)
        for _ in range(60):
            if f1 < f2:
                lo, x1, f1 = x1, x2, f2
                x2 = lo + g * (hi - lo)
                f2 = corr(x2)
            else:
                hi, x2, f2 = x2, x1, f1
                x1 = hi - g * (hi - lo)
                f1 = corr(x1)
        best = max(best, f1, f2)
    return best / math.sqrt(sa * sb)
