"""Seeded synthetic inputs for the matched-filter workloads.

This module produces the *inputs* of a search (a detector PSD, a Gaussian
noise spectrum, a template bank's mass draws and the random parameters of
injections).  It holds none of the search's arithmetic: no chirp model, no
inner product, no transform.  Both the GPU library's tests and the CPU
oracle's tests draw their inputs from here, so the two sides see identical
numbers.

Conventions (one-sided spectra on the positive-frequency grid
f_k = k * fs / n, k = 0 .. n/2):

* PSD model: S(f) = 1e-46 * [(150/f)^4 + 2 + 2 (f/150)^2] Hz^-1, evaluated
  exactly at f_k (no bin averaging).  S(0) is undefined; bin 0 receives the
  value of bin 1 and is never used by the search (it lies below f_low).
* Noise: n~_k = sqrt(T S_k / 4) (g1 + i g2) with g ~ N(0, 1) for
  k_low <= k <= n/2 - 1 and 0 elsewhere, so E|n~_k|^2 = T S_k / 2, the
  one-sided normalisation under which the inner product
  <a, b> = 4 Re sum_k df a~_k b~_k* / S_k gives unit-variance quadratures.
* All random draws use numpy's PCG64 ``default_rng`` with the documented
  per-workload seeds.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "psd_model", "make_psd", "k_low_of",
    "make_noise", "draw_masses", "InjectionSpec", "draw_injections",
    "CLASS_LENGTHS", "class_noise_seed",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic search configuration (sizes follow the paper's
    2^18..2^21-sample segments at 4 kHz; see the online-analysis table)."""
    name: str
    n: int                 # samples per segment (power of two)
    fs: float              # sample rate, Hz
    f_low: float           # lower cutoff, Hz
    n_templates: int
    m_min: float           # solar masses
    m_max: float
    dist: str              # "uniform" | "loguniform"
    snr_threshold: float   # lambda
    window: int            # trigger window W (samples)
    n_inj: int             # injections
    inj_snr: tuple
    noise_seed: int
    bank_seed: int
    inj_seed: int


WORKLOADS = {
    # tiny plain case: one 16 s segment, one 1.4+1.4 injection at SNR 10
    "tiny-2^16": Workload("tiny-2^16", 1 << 16, 4096.0, 20.0, 8, 1.0, 3.0,
                          "uniform", 6.0, 4096, 1, (10.0,),
                          1006 + 100, 4644 + 1, 20100625 + 1),
    # headline FP32 case: 256 s segment, 1024 templates, five injections
    "fp32-2^20": Workload("fp32-2^20", 1 << 20, 4096.0, 20.0, 1024, 1.0, 10.0,
                          "loguniform", 6.0, 4096, 5,
                          (8.0, 11.0, 14.0, 17.0, 20.0),
                          1006 + 200, 4644 + 2, 20100625 + 2),
    # uneven-length batch: 16384 templates in length classes 2^17..2^20
    "batched-classes": Workload("batched-classes", 1 << 20, 4096.0, 20.0,
                                16384, 1.0, 30.0, "loguniform", 6.0, 4096, 0,
                                (), 1006 + 300, 4644 + 3, 20100625 + 3),
    # precision comparison: 65536 templates at 2^20
    "precision-2^20": Workload("precision-2^20", 1 << 20, 4096.0, 20.0, 65536,
                               1.0, 10.0, "loguniform", 6.0, 4096, 5,
                               (8.0, 11.0, 14.0, 17.0, 20.0),
                               1006 + 400, 4644 + 4, 20100625 + 4),
    # third-generation-shaped bank: 2^21 samples from 10 Hz, 1M templates
    "3g-2^21": Workload("3g-2^21", 1 << 21, 4096.0, 10.0, 1 << 20, 1.0, 50.0,
                        "loguniform", 6.0, 4096, 5,
                        (8.0, 11.0, 14.0, 17.0, 20.0),
                        1006 + 500, 4644 + 5, 20100625 + 5),
}


# Segment lengths of the length classes (chirps of up to 32, 64, 128 and
# 256 s at 4096 Hz).
CLASS_LENGTHS = (1 << 17, 1 << 18, 1 << 19, 1 << 20)


def class_noise_seed(wl: Workload, c: int) -> int:
    """Noise seed of class c's segment: the workload's seed plus c."""
    return wl.noise_seed + c


def psd_model(f):
    """Analytic one-sided PSD S(f) in Hz^-1 (the workloads' noise model)."""
    f = np.asarray(f, dtype=np.float64)
    x = f / 150.0
    return 1e-46 * ((1.0 / x) ** 4 + 2.0 + 2.0 * x * x)


def make_psd(n: int, fs: float) -> np.ndarray:
    """S_k at f_k = k fs/n for k = 0..n/2 (float64, length n/2+1)."""
    k = np.arange(n // 2 + 1, dtype=np.float64)
    f = k * (fs / n)
    out = np.empty(n // 2 + 1, dtype=np.float64)
    out[1:] = psd_model(f[1:])
    out[0] = out[1]
    return out


def k_low_of(n: int, fs: float, f_low: float) -> int:
    """First bin at or above f_low: ceil(f_low * T) with T = n/fs."""
    return int(math.ceil(f_low * (n / fs)))


def make_noise(n: int, fs: float, f_low: float, psd: np.ndarray,
               seed: int) -> np.ndarray:
    """Band-limited stationary Gaussian noise spectrum (complex128, n/2+1).

    n~_k = sqrt(T S_k / 4) (g1 + i g2) for k_low <= k <= n/2-1, else 0.
    """
    rng = np.random.default_rng(seed)
    T = n / fs
    kl = k_low_of(n, fs, f_low)
    out = np.zeros(n // 2 + 1, dtype=np.complex128)
    m = n // 2 - kl
    g = rng.standard_normal((m, 2))
    amp = np.sqrt(T * psd[kl:n // 2] / 4.0)
    out[kl:n // 2] = amp * (g[:, 0] + 1j * g[:, 1])
    return out


def draw_masses(count: int, m_min: float, m_max: float, dist: str,
                seed: int) -> np.ndarray:
    """(count, 2) float64 array of (m1, m2) in solar masses, m1 >= m2.

    m1 and m2 are drawn independently (uniform or log-uniform on
    [m_min, m_max]) and then swapped so that m1 >= m2.
    """
    rng = np.random.default_rng(seed)
    u = rng.random((count, 2))
    if dist == "uniform":
        m = m_min + u * (m_max - m_min)
    elif dist == "loguniform":
        m = m_min * np.exp(u * math.log(m_max / m_min))
    else:
        raise ValueError(f"unknown mass distribution {dist!r}")
    return np.stack([m.max(axis=1), m.min(axis=1)], axis=1)


@dataclasses.dataclass(frozen=True)
class InjectionSpec:
    m1: float
    m2: float
    snr: float      # target optimal SNR
    j0: int         # coalescence sample (t_c = j0 / fs)
    phi: float      # coalescence phase, radians
    tmpl: int       # bank index whose masses were used (-1: fixed masses)


def draw_injections(wl: Workload, bank: np.ndarray) -> list:
    """Injection parameters: masses of seeded bank entries, j0 = floor((i+1)
    n/6), phases uniform in [0, 2 pi), SNRs from the workload's list.  The
    single-injection tiny case uses 1.4+1.4 at j0 = n/2."""
    rng = np.random.default_rng(wl.inj_seed)
    out = []
    if wl.n_inj == 1:
        phi = float(rng.random() * 2.0 * math.pi)
        out.append(InjectionSpec(1.4, 1.4, wl.inj_snr[0], wl.n // 2, phi, -1))
        return out
    idx = rng.choice(len(bank), size=wl.n_inj, replace=False)
    for i in range(wl.n_inj):
        phi = float(rng.random() * 2.0 * math.pi)
        j0 = ((i + 1) * wl.n) // (wl.n_inj + 1)
        t = int(idx[i])
        out.append(InjectionSpec(float(bank[t, 0]), float(bank[t, 1]),
                                 float(wl.inj_snr[i]), j0, phi, t))
    return out
