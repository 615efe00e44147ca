"""Shared test-case construction and GPU-vs-oracle comparison helpers.

Inputs come from the seeded generator (noise, PSD, masses, injection
parameters); injected chirps are made with the oracle's template generator
on the test side, so both the GPU library and the oracle see the same
complex64 data spectrum.  Nothing here calls the GPU library except through
its Python binding.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import mf_oracle as O
from paper_1006_4644_amd import synth

# Tolerances stated for the FP32 path: SNR relative error <= 1e-5.
TOL_FP32 = 1e-5


def make_case(n, fs, f_low, bank, injections, noise_seed):
    """(xtilde complex64, psd float64, xtilde upcast complex128)."""
    psd = synth.make_psd(n, fs)
    x = synth.make_noise(n, fs, f_low, psd, noise_seed) if noise_seed is not None \
        else np.zeros(n // 2 + 1, dtype=np.complex128)
    for inj in injections:
        h = O.spa_htilde(n, fs, f_low, inj.m1, inj.m2, tc=inj.j0 / fs,
                         phic=inj.phi)
        _, _, _, kl, kh = O.band(inj.m1, inj.m2, n, fs, f_low)
        s = math.sqrt(O.sigma2(h, psd, fs / n, kl, kh))
        x = x + h * (inj.snr / s)
    x64 = x.astype(np.complex64)
    return x64, psd, x64.astype(np.complex128)


def workload_case(name, n_templates=None, extra_exact=True):
    """Inputs of a named workload: (wl, bank, injections, x64, psd, x128)."""
    wl = synth.WORKLOADS[name]
    nt = wl.n_templates if n_templates is None else n_templates
    bank = synth.draw_masses(nt, wl.m_min, wl.m_max, wl.dist, wl.bank_seed)
    injs = synth.draw_injections(wl, bank)
    if extra_exact and wl.n_inj == 1:
        bank = np.vstack([bank, [[injs[0].m1, injs[0].m2]]])
    x64, psd, x128 = make_case(wl.n, wl.fs, wl.f_low, bank, injs, wl.noise_seed)
    return wl, bank, injs, x64, psd, x128


def oracle_series(x128, psd, n, fs, f_low, m1, m2):
    zs, s2 = O.snr_series(x128, psd, n, fs, f_low, m1, m2)
    return zs, s2


def series_error(z_gpu, z_orc):
    """e_series = max_j |rho_gpu - rho_orc| / max_j rho_orc."""
    rg = np.abs(z_gpu.astype(np.complex128))
    ro = np.abs(z_orc)
    return float(np.max(np.abs(rg - ro)) / max(np.max(ro), 1e-300))


def check_peak(gp, zo, tol=TOL_FP32, j_lo=0, j_hi=None):
    """GPU peak record vs the oracle series: index exact unless the oracle's
    own rho^2 at the GPU index ties the oracle maximum within tolerance;
    rho within tol of the oracle's rho at that index, z within 2 tol rho."""
    r2 = np.abs(zo) ** 2
    n = len(r2)
    j_hi = n if j_hi is None else j_hi
    jo = j_lo + int(np.argmax(r2[j_lo:j_hi]))
    jg = int(gp["index"])
    rmax = math.sqrt(r2[jo])
    drho = tol * rmax
    tie = 2 * rmax * drho + drho * drho
    assert j_lo <= jg < j_hi
    assert jg == jo or abs(r2[jg] - r2[jo]) <= tie, (jg, jo, r2[jg], r2[jo])
    rho_o = math.sqrt(r2[jg])
    assert abs(math.sqrt(gp["rho2"]) - rho_o) <= tol * rho_o
    zg = complex(gp["re"], gp["im"])
    assert abs(zg - zo[jg]) <= 2 * tol * rho_o, (zg, zo[jg])
    return jg == jo


def check_triggers(gtr, zo, window, thr, tol=TOL_FP32, j_lo=0, j_hi=None):
    """One template's GPU triggers vs its oracle series.

    Each trigger's rho is held to tol relative to the oracle's rho at that
    sample (and z to 2 tol rho, both quadratures), not to the series
    maximum.  Windows whose oracle maximum is within tol (relative) of the
    threshold may go either way; inside a window the index must match
    unless the oracle's values at the two indices tie within tol of the
    window maximum.  Returns the number of exempted decisions."""
    r2 = np.abs(zo) ** 2
    n = len(r2)
    j_hi = n if j_hi is None else j_hi
    thr2 = thr * thr
    # e_rel = |rho_gpu - rho_orc| / rho_orc at each trigger: every bound
    # below is tol times the oracle's own rho at the sample concerned
    dthr = tol * thr
    band = 2 * thr * dthr + dthr * dthr
    expect = {w: (j, v) for (w, j, v) in O.window_triggers(r2, window, thr2,
                                                          j_lo, j_hi)}
    got = {int(t["window"]): t for t in gtr}
    exempt = 0
    n_win = (n + window - 1) // window
    for w in range(n_win):
        a, b = max(w * window, j_lo), min((w + 1) * window, j_hi, n)
        if a >= b:
            assert w not in got
            continue
        wmax = float(np.max(r2[a:b]))
        near = abs(wmax - thr2) <= band
        if w in expect and not near:
            assert w in got, (w, expect[w])
        if w not in expect and not near:
            assert w not in got, (w, got.get(w))
        if w in got:
            t = got[w]
            jg = int(t["index"])
            assert a <= jg < b and int(t["window"]) == w
            jo = a + int(np.argmax(r2[a:b]))
            dw = tol * math.sqrt(wmax)
            tie = 2 * math.sqrt(wmax) * dw + dw * dw
            assert jg == jo or abs(r2[jg] - r2[jo]) <= tie, (w, jg, jo)
            exempt += int(jg != jo) + int(near)
            rho_o = math.sqrt(r2[jg])
            assert abs(math.sqrt(t["rho2"]) - rho_o) <= tol * rho_o, \
                (w, jg, float(t["rho2"]), r2[jg])
            assert abs(complex(t["re"], t["im"]) - zo[jg]) <= 2 * tol * rho_o, \
                (w, jg, complex(t["re"], t["im"]), zo[jg])
        elif near:
            exempt += 1
    return exempt
