"""Plain FP64 CPU oracle of the paper's own template form: a time-domain
chirp in two polarizations, each Fourier transformed and normalised on its
own, correlated with the data, taken back to the time domain by two real
inverse transforms and combined in quadrature.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
of the GPU build and the CPU-baseline leg of the benchmark may import or run
this module.  The GPU library never calls it and shares no code with it.

What it follows (Bosi, "cuInspiral", arXiv:1006.4644):

* "Template generation": the two polarizations h_+, h_x of a chirp with a
  phase of post-Newtonian order 2.5 and a Newtonian (0PN) amplitude,
  generated in the time domain, then FFT transformed and normalised;
* "Matched filtering", steps 1-3 of the per-template loop: the correlators
  c_+ = <x, theta_+>, c_x = <x, theta_x> for every lag, combined as
  c = sqrt(c_+^2 + c_x^2) (the paper's device_complex_mf, two
  device_cufft_C2R and device_madd2 calls).

Readings where the paper gives no formula (each is also what the GPU path
implements):

* Phase: TaylorT2 at 2.5PN.  Energy balance dE/dt = -F with the published
  2PN binding energy and 2.5PN flux (Blanchet, Damour, Iyer, Will &
  Wiseman, PRL 74, 3515 (1995); Blanchet, CQG 13, 619 (1996) for the v^5
  flux term) gives dt/dv = (5M/(32 eta)) v^-9 r(v), with r(v) the ratio
  E'(v)/E'_N(v) over F(v)/F_N(v) expanded to O(v^5).  Integrating term by
  term with t_c = 0 and phi_c = 0:
      t(v)   = -(5M/(256 eta)) v^-8 [1 + sum_k tau_k v^k],  tau_k = 8 r_k/(8-k),
      phi(v) = -(1/(32 eta)) [v^-5 (1 + sum_{k<5} p_k v^k) + p_5 ln v],
               p_k = 5 r_k/(5-k) (k < 5),  p_5 = -5 r_5,
  phi the orbital phase; the gravitational-wave phase is 2 phi.  The series
  coefficients are computed here from E and F, not typed in.
* The chirp runs from v_low = (pi M f_low)^{1/3} to the Schwarzschild ISCO
  v_isco = 6^{-1/2} (dt/dv stays positive there for every eta in (0, 1/4],
  checked by the pins).  Sample m >= 1 before coalescence sits at time
  t = -m/fs and index j = n - m (the template's coalescence is sample 0 of
  the circular grid, as for the frequency-domain template with t_c = 0);
  v at that time solves t(v) = -m/fs.  Samples exist for
  m_lo = ceil(-t(v_isco) fs) <= m <= m_hi = min(floor(-t(v_low) fs), n - 1);
  a chirp longer than the segment keeps its last n - 1 samples.
* Amplitude: h_+ = v^2 cos(2 phi), h_x = v^2 sin(2 phi) (0PN, face-on, up
  to a constant that cancels in the normalisation).
* Spectra: H~_k = dt sum_j h_j e^{-2 pi i jk/n} for k = 0..n/2.
* Band of the statistic: k_low = ceil(f_low T) <= k <= n/2 - 1 (the chirp
  carries its own upper cut-off in time).
* Normalisation: each polarization to unit norm, sigma_+^2 = <h_+, h_+>,
  sigma_x^2 = <h_x, h_x> (the paper's <theta, theta> = 1/2 per polarization
  scaled by sqrt 2, as in the frequency-domain form), so in Gaussian noise
  c_+ and c_x are each unit-variance normal.
* c_+(t_j) = 4 Re sum_band df x~_k conj(H~+_k) e^{2 pi i jk/n} / S_k / sigma_+
  (likewise c_x); rho^2 = c_+^2 + c_x^2.  The complex value c_+ + i c_x is
  what plays the role of z/sigma in the search.
"""
from __future__ import annotations

import math

import numpy as np

from oracle.mf_oracle import T_SUN, idft, peak, window_triggers, merge_windows

__all__ = ["balance_series", "t2_coefficients", "t2_time", "t2_dtdv",
           "t2_phase", "td_layout", "td_chirp", "td_spectra", "td_series",
           "td_search"]


def balance_series(eta: float):
    """r_0..r_5 of dt/dv = (5M/(32 eta)) v^-9 r(v): the ratio of
    E'(v)/E'_N = 1 + e_2 v^2 + e_4 v^4 and F/F_N = 1 + f_2 v^2 + f_3 v^3 +
    f_4 v^4 + f_5 v^5, expanded by plain power-series division."""
    # binding energy E = -(1/2) M eta v^2 [1 - (3/4 + eta/12) v^2
    #                    - (27/8 - 19 eta/8 + eta^2/24) v^4]; d/dv of
    # v^2 (1 + a v^2 + b v^4) is 2 v (1 + 2 a v^2 + 3 b v^4)
    e2 = -2.0 * (3.0 / 4.0 + eta / 12.0)
    e4 = -3.0 * (27.0 / 8.0 - 19.0 * eta / 8.0 + eta * eta / 24.0)
    # flux F = (32/5) eta^2 v^10 [1 + f2 v^2 + ... + f5 v^5]
    f2 = -(1247.0 / 336.0 + 35.0 * eta / 12.0)
    f3 = 4.0 * math.pi
    f4 = -44711.0 / 9072.0 + 9271.0 * eta / 504.0 + 65.0 * eta * eta / 18.0
    f5 = -(8191.0 / 672.0 + 583.0 * eta / 24.0) * math.pi
    num = [1.0, 0.0, e2, 0.0, e4, 0.0]
    den = [1.0, 0.0, f2, f3, f4, f5]
    r = [0.0] * 6
    for k in range(6):
        r[k] = num[k] - sum(r[i] * den[k - i] for i in range(k))
    return r


def t2_coefficients(eta: float):
    """(tau_0..tau_5, p_0..p_5) of the TaylorT2 time and orbital phase."""
    r = balance_series(eta)
    tau = [8.0 * r[k] / (8.0 - k) for k in range(6)]
    p = [5.0 * r[k] / (5.0 - k) for k in range(5)] + [-5.0 * r[5]]
    return tau, p


def _mass(m1, m2):
    M = (m1 + m2) * T_SUN
    eta = m1 * m2 / ((m1 + m2) * (m1 + m2))
    return M, eta


def t2_time(v, m1, m2):
    """t(v) in seconds (t_c = 0)."""
    M, eta = _mass(m1, m2)
    tau, _ = t2_coefficients(eta)
    v = np.asarray(v, dtype=np.float64)
    s = sum(tau[k] * v ** k for k in range(6))
    return -(5.0 * M / (256.0 * eta)) * v ** -8.0 * s


def t2_dtdv(v, m1, m2):
    M, eta = _mass(m1, m2)
    r = balance_series(eta)
    v = np.asarray(v, dtype=np.float64)
    return (5.0 * M / (32.0 * eta)) * v ** -9.0 * sum(r[k] * v ** k for k in range(6))


def t2_phase(v, m1, m2):
    """Orbital phase phi(v) in radians (phi_c = 0)."""
    _, eta = _mass(m1, m2)
    _, p = t2_coefficients(eta)
    v = np.asarray(v, dtype=np.float64)
    s = sum(p[k] * v ** k for k in range(5))
    return -(1.0 / (32.0 * eta)) * (v ** -5.0 * s + p[5] * np.log(v))


def td_layout(n: int, fs: float, f_low: float, m1: float, m2: float):
    """(v_low, v_end, m_lo, m_hi): velocity range and the samples before
    coalescence that carry the chirp; m_lo > m_hi for an empty template."""
    M, _ = _mass(m1, m2)
    v_low = (math.pi * M * f_low) ** (1.0 / 3.0)
    v_end = 1.0 / math.sqrt(6.0)
    if v_low >= v_end:
        return v_low, v_end, 1, 0
    m_lo = int(math.ceil(-float(t2_time(v_end, m1, m2)) * fs))
    m_hi = min(int(math.floor(-float(t2_time(v_low, m1, m2)) * fs)), n - 1)
    return v_low, v_end, max(m_lo, 1), m_hi


def _solve_v(t, m1, m2, v_low, v_end):
    """v with t2_time(v) = t, by Newton's method from the Newtonian guess,
    kept inside [v_low, v_end], iterated until it stops moving."""
    M, eta = _mass(m1, m2)
    v = (256.0 * eta * (-t) / (5.0 * M)) ** (-1.0 / 8.0)
    v = np.clip(v, v_low, v_end)
    for _ in range(100):
        dv = (t2_time(v, m1, m2) - t) / t2_dtdv(v, m1, m2)
        v_new = np.clip(v - dv, v_low, v_end)
        done = np.max(np.abs(v_new - v) / v) < 1e-15
        v = v_new
        if done:
            break
    else:
        raise RuntimeError("Newton iteration for v(t) did not converge")
    return v


def td_chirp(n: int, fs: float, f_low: float, m1: float, m2: float):
    """(h_plus, h_cross): float64 [n] time-domain polarizations, coalescence
    at sample 0 of the circular grid (the chirp at j = n - m)."""
    hp = np.zeros(n)
    hc = np.zeros(n)
    v_low, v_end, m_lo, m_hi = td_layout(n, fs, f_low, m1, m2)
    if m_lo > m_hi:
        return hp, hc
    m = np.arange(m_lo, m_hi + 1, dtype=np.float64)
    v = _solve_v(-m / fs, m1, m2, v_low, v_end)
    phi = t2_phase(v, m1, m2)
    j = (n - np.arange(m_lo, m_hi + 1)) % n
    hp[j] = v * v * np.cos(2.0 * phi)
    hc[j] = v * v * np.sin(2.0 * phi)
    return hp, hc


def td_spectra(n: int, fs: float, f_low: float, m1: float, m2: float):
    """(H+, Hx): complex128 [n/2 + 1], H~_k = dt sum_j h_j e^{-2 pi i jk/n}."""
    hp, hc = td_chirp(n, fs, f_low, m1, m2)
    dt = 1.0 / fs
    return dt * np.fft.rfft(hp), dt * np.fft.rfft(hc)


def _band(n, fs, f_low):
    return int(math.ceil(f_low * n / fs)), n // 2 - 1


def td_series(xtilde, psd, n: int, fs: float, f_low: float, m1: float,
              m2: float):
    """(c_+ + i c_x  complex128 [n], sigma_+^2, sigma_x^2) for one template;
    an empty template gives zeros."""
    df = fs / n
    kl, kh = _band(n, fs, f_low)
    Hp, Hc = td_spectra(n, fs, f_low, m1, m2)
    out = []
    sig = []
    for H in (Hp, Hc):
        s2 = float(4.0 * df * np.sum(np.abs(H[kl:kh + 1]) ** 2 / psd[kl:kh + 1]))
        sig.append(s2)
        if s2 <= 0.0:
            out.append(np.zeros(n))
            continue
        Z = np.zeros(n, dtype=np.complex128)
        Z[kl:kh + 1] = 4.0 * df * xtilde[kl:kh + 1] * np.conj(H[kl:kh + 1]) / psd[kl:kh + 1]
        out.append(np.real(idft(Z)) / math.sqrt(s2))
    return out[0] + 1j * out[1], sig[0], sig[1]


def td_search(xtilde, psd, n: int, fs: float, f_low: float, bank, thr: float,
              window: int, j_lo: int = 0, j_hi: int | None = None):
    """The per-chunk pipeline with the two-polarization template: per
    template the peak (j*, rho2*, c_+ + i c_x) or (-1, 0, 0) when empty,
    the window triggers, and the merged windows."""
    thr2 = thr * thr
    peaks, trig = [], {}
    for t, (m1, m2) in enumerate(np.asarray(bank, dtype=np.float64)):
        z, sp, sc = td_series(xtilde, psd, n, fs, f_low, float(m1), float(m2))
        if sp <= 0.0 or sc <= 0.0:
            peaks.append((-1, 0.0, 0j))
            trig[t] = []
            continue
        r2 = z.real ** 2 + z.imag ** 2
        lo, hi = j_lo, (n if j_hi is None else j_hi)
        j = lo + peak(r2[lo:hi])
        peaks.append((j, float(r2[j]), complex(z[j])))
        trig[t] = window_triggers(r2, window, thr2, j_lo, j_hi)
    return {"peaks": peaks, "triggers": trig, "merged": merge_windows(trig)}
