"""Pins of the two-polarization time-domain oracle (CPU only).

Each pin ties the oracle to something other than its own formulas: the
already pinned 2PN time to coalescence, the published TaylorF2 and TaylorT2
coefficients, identities between amplitude, phase and time along the
generated chirp, the stationary-phase spectrum of the same chirp, a real
inverse FFT (the paper's C2R), noise-free injections and Gaussian noise.
"""
import math

import numpy as np
import pytest

from oracle import mf_oracle as O
from oracle import td_oracle as T
from paper_1006_4644_amd import synth

V_ISCO = 1.0 / math.sqrt(6.0)


@pytest.mark.parametrize("m1,m2", [(1.4, 1.4), (10.0, 1.0), (30.0, 7.0)])
def test_t2_time_extends_the_2pn_duration(m1, m2):
    # without its v^5 term, -t(v) is the (independently pinned) 2PN duration
    M = (m1 + m2) * O.T_SUN
    eta = m1 * m2 / (m1 + m2) ** 2
    tau, _ = T.t2_coefficients(eta)
    v = np.linspace(0.05, 0.35, 13)
    f = v ** 3 / (math.pi * M)
    t5 = (5 * M / (256 * eta)) * v ** -8.0 * tau[5] * v ** 5
    assert np.max(np.abs((-T.t2_time(v, m1, m2) - t5) / O.tau_2pn(f, m1, m2) - 1)) < 1e-12
    # published TaylorT2 2.5PN time coefficient
    assert abs(tau[5] + (7729 / 252 - 13 * eta / 3) * math.pi) < 1e-12


@pytest.mark.parametrize("eta", [0.03, 0.12, 0.2222, 0.25])
def test_t2_phase_reproduces_taylorf2(eta):
    # Psi(f) = 2 pi f t(v) - 2 phi(v): its coefficients (8 p_k - 5 tau_k)/3
    # are the published TaylorF2 ones, and the 2.5PN log term 8 p_5/3 equals
    # 3 psi_5 of the TaylorF2 term psi_5 (1 + 3 ln v).
    tau, p = T.t2_coefficients(eta)
    psi = [1.0, 0.0, 3715 / 756 + 55 * eta / 9, -16 * math.pi,
           15293365 / 508032 + 27145 * eta / 504 + 3085 * eta ** 2 / 72]
    for k in (0, 2, 3, 4):
        assert abs((8 * p[k] - 5 * tau[k]) / 3 - psi[k]) < 1e-12 * max(1, abs(psi[k]))
    assert abs(tau[1]) < 1e-15 and abs(p[1]) < 1e-15
    psi5 = (38645 / 756 - 65 * eta / 9) * math.pi
    assert abs(8 * p[5] / 3 - 3 * psi5) < 1e-10 * abs(psi5)


def test_t2_time_monotone_up_to_isco():
    # dt/dv > 0 on (0, v_isco] for every mass ratio: one chirp, no turning point
    v = np.linspace(1e-3, V_ISCO, 4001)
    for eta in np.linspace(0.005, 0.25, 50):
        r = T.balance_series(float(eta))
        assert np.min(sum(r[k] * v ** k for k in range(6))) > 0.1
    assert np.all(np.diff(T.t2_time(v, 1.4, 1.4)) > 0)


@pytest.mark.parametrize("m1,m2", [(1.4, 1.4), (6.0, 2.0), (20.0, 15.0)])
def test_td_chirp_amplitude_phase_and_time_agree(m1, m2):
    """Along the generated chirp: the amplitude |u| = v^2 and the phase of
    u = h_+ + i h_x satisfy d(arg u)/dt = 2 v^3 / M = 2 |u|^{3/2} / M (the
    orbital-frequency relation), the first sample is the first at or above
    f_low and the last is the last at or below the ISCO."""
    n, fs, fl = 1 << 17, 4096.0, 20.0
    M = (m1 + m2) * O.T_SUN
    hp, hc = T.td_chirp(n, fs, fl, m1, m2)
    u = hp + 1j * hc
    v_low, v_end, m_lo, m_hi = T.td_layout(n, fs, fl, m1, m2)
    j = np.arange(n - m_hi, n - m_lo + 1)
    assert np.all(u[j] != 0) and np.count_nonzero(u) == len(j)
    amp = np.abs(u[j])
    dphi = np.angle(u[j[1:]] / u[j[:-1]]) * fs        # per-sample phase steps
    vm = np.sqrt(0.5 * (amp[1:] + amp[:-1]))           # mid-step v from |u|
    want = 2 * vm ** 3 / M
    sel = want / fs < 0.5                              # resolved phase steps
    rel = np.abs(dphi[sel] / want[sel] - 1)
    assert np.max(rel) < 2e-3 and np.median(rel) < 1e-5
    # chirp start and end
    t_first = -(n - j[0]) / fs
    if m_hi < n - 1:
        assert T.t2_time(v_low, m1, m2) <= t_first < T.t2_time(v_low, m1, m2) + 1 / fs
    assert np.sqrt(amp[-1]) <= V_ISCO + 1e-15
    assert float(T.t2_time(V_ISCO, m1, m2)) > -(n - j[-1]) / fs - 1 / fs


@pytest.mark.parametrize("m1,m2,floor", [(1.4, 1.4, 0.99), (5.0, 3.0, 0.99),
                                         (10.0, 1.2, 0.97)])
def test_td_spectrum_matches_25pn_stationary_phase(m1, m2, floor):
    """The FFT of the time-domain chirp against the TaylorF2 stationary-phase
    chirp with the published 2.5PN term: near-unit match at zero lag (the
    time axis, the signs and the v^5 flux term all enter)."""
    n, fs, fl = 1 << 18, 4096.0, 20.0
    psd = synth.make_psd(n, fs)
    df = fs / n
    Hp, _ = T.td_spectra(n, fs, fl, m1, m2)
    M, eta, _, kl, kh = O.band(m1, m2, n, fs, fl)
    k = np.arange(kl, kh + 1)
    f = k * df
    v = np.cbrt(math.pi * M * f)
    psi = O.spa_phase(f, m1, m2) + 3 / (128 * eta) * (
        38645 / 756 - 65 * eta / 9) * math.pi * (1 + 3 * np.log(v))
    h = np.zeros(n // 2 + 1, complex)
    h[kl:kh + 1] = f ** (-7 / 6) * np.exp(-1j * psi)
    Z = np.zeros(n, complex)
    Z[kl:kh + 1] = Hp[kl:kh + 1] * np.conj(h[kl:kh + 1]) / psd[kl:kh + 1]
    zz = np.fft.ifft(Z) * n
    na = np.sum(np.abs(Hp[kl:kh + 1]) ** 2 / psd[kl:kh + 1])
    nb = np.sum(np.abs(h[kl:kh + 1]) ** 2 / psd[kl:kh + 1])
    j = int(np.argmax(np.abs(zz)))
    assert j == 0
    assert np.abs(zz[0]) / np.sqrt(na * nb) > floor


def _inject(n, fs, fl, m1, m2, rho, j0, psd, noise_seed=None):
    """Data holding h_+ of (m1, m2) shifted to coalesce at sample j0 and
    scaled to optimal SNR rho in the band [k_low, n/2 - 1]."""
    df = fs / n
    hp, _ = T.td_chirp(n, fs, fl, m1, m2)
    H = np.fft.rfft(np.roll(hp, j0)) / fs
    kl, kh = int(math.ceil(fl * n / fs)), n // 2 - 1
    H[:kl] = 0
    H[kh + 1:] = 0
    s = math.sqrt(4 * df * np.sum(np.abs(H[kl:kh + 1]) ** 2 / psd[kl:kh + 1]))
    x = H * (rho / s)
    if noise_seed is not None:
        x = x + synth.make_noise(n, fs, fl, psd, noise_seed)
    return x


def test_td_series_equals_two_real_inverse_transforms():
    """c_+ and c_x are the paper's two C2R outputs: numpy's real inverse FFT
    of the one-sided correlator spectra gives the same series."""
    n, fs, fl = 1 << 14, 4096.0, 20.0
    psd = synth.make_psd(n, fs)
    df = fs / n
    x = _inject(n, fs, fl, 3.0, 2.0, 9.0, 4000, psd, noise_seed=5)
    z, sp, sc = T.td_series(x, psd, n, fs, fl, 3.0, 2.0)
    Hp, Hc = T.td_spectra(n, fs, fl, 3.0, 2.0)
    kl = int(math.ceil(fl * n / fs))
    for H, s2, c in ((Hp, sp, z.real), (Hc, sc, z.imag)):
        Zh = np.zeros(n // 2 + 1, complex)
        Zh[kl:n // 2] = 4 * df * x[kl:n // 2] * np.conj(H[kl:n // 2]) / psd[kl:n // 2]
        c2r = np.fft.irfft(Zh, n) * (n / 2) / math.sqrt(s2)
        assert np.max(np.abs(c2r - c)) < 1e-11 * np.max(np.abs(c))


@pytest.mark.parametrize("j0", [1000, 9000, 16000])
def test_td_noise_free_injection_recovered(j0):
    n, fs, fl = 1 << 14, 4096.0, 20.0
    psd = synth.make_psd(n, fs)
    rho = 10.0
    x = _inject(n, fs, fl, 3.0, 2.0, rho, j0, psd)
    z, _, _ = T.td_series(x, psd, n, fs, fl, 3.0, 2.0)
    r2 = z.real ** 2 + z.imag ** 2
    assert O.peak(r2) == j0
    # c_+ at the injection is the optimal SNR exactly; c_x there is the
    # zero-lag overlap of the two polarizations, which are in quadrature
    assert abs(z[j0].real - rho) < 1e-9 * rho
    assert abs(z[j0].imag) < 0.02 * rho
    # shifting the injection shifts the series
    z2, _, _ = T.td_series(_inject(n, fs, fl, 3.0, 2.0, rho, j0 + 37, psd), psd, n,
                           fs, fl, 3.0, 2.0)
    assert np.max(np.abs(np.roll(z, 37) - z2)) < 1e-9 * rho


def test_td_noise_statistics():
    """Gaussian noise: c_+ and c_x are each unit-variance normal."""
    from scipy import stats
    n, fs, fl = 1 << 14, 4096.0, 20.0
    psd = synth.make_psd(n, fs)
    cp, cx = [], []
    for seed in (41, 42, 43):
        x = synth.make_noise(n, fs, fl, psd, seed)
        z, _, _ = T.td_series(x, psd, n, fs, fl, 4.0, 1.5)
        cp.append(z.real[::97])
        cx.append(z.imag[::97])
    for c in (np.concatenate(cp), np.concatenate(cx)):
        assert stats.kstest(c, "norm").pvalue > 1e-3
        assert abs(np.var(c) - 1) < 0.15


def test_td_empty_and_long_templates():
    n, fs, fl = 1 << 14, 4096.0, 20.0
    # ISCO below f_low: no samples
    _, _, m_lo, m_hi = T.td_layout(n, fs, fl, 150.0, 150.0)
    assert m_lo > m_hi
    hp, hc = T.td_chirp(n, fs, fl, 150.0, 150.0)
    assert not np.any(hp) and not np.any(hc)
    psd = synth.make_psd(n, fs)
    z, sp, sc = T.td_series(np.zeros(n // 2 + 1, complex), psd, n, fs, fl, 150.0, 150.0)
    assert sp == 0.0 and sc == 0.0 and not np.any(z)
    # a chirp longer than the segment keeps the last n - 1 samples
    _, _, m_lo, m_hi = T.td_layout(n, fs, fl, 1.0, 1.0)
    assert m_hi == n - 1
    hp, _ = T.td_chirp(n, fs, fl, 1.0, 1.0)
    assert hp[0] == 0.0 and np.count_nonzero(hp) == n - m_lo
