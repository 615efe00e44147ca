"""GPU-vs-oracle parity of the chi-squared veto (needs an MI355X).

The veto is the signal-consistency test the paper's Conclusions plan after
the matched filter (their ref. [Chi2], B. Allen, PRD 71, 062001 (2005)):
chi2 = p sum_l |z_l - z/p|^2 over p bands of equal sigma^2 share.

Tolerance, derived from the arithmetic: every bin's term Z_k e^{2 pi i jk/n}
carries an FP32 rounding of its amplitude and phase (relative error below
~3e-7, independent across bins) and the accumulation is FP64, so each band
value z_l is off by |dz_l| <~ 1e-6 (1 + |z|) (the noise part of a band has
variance 2/p, a signal part scales with |z|).  With d_l = z_l - z/p,
|d chi2| <= 2 p sqrt(chi2) max_l |dz_l| (Cauchy-Schwarz), so the test bar is
|chi2_gpu - chi2_oracle| <= 2e-5 p sqrt(chi2) (1 + |z|) + 1e-9, ten times
that estimate.
"""
import math

import numpy as np
import pytest

from oracle import mf_oracle as O
from paper_1006_4644_amd import ci, synth
from tests import mfcase as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sync():
    import torch
    torch.cuda.synchronize()


def _rows(tmpl, index):
    """ci_trigger rows (m, 4) int64 on the device for given (tmpl, index)."""
    a = np.zeros(len(tmpl), dtype=ci.TRIGGER_DTYPE)
    a["tmpl"] = tmpl
    a["index"] = index
    a["window"] = -1
    return _dev(a.view("<i8").reshape(-1, 4))


def _tol(chi2, z, bands):
    return 2e-5 * bands * math.sqrt(max(chi2, 0.0)) * (1.0 + abs(z)) + 1e-9


def _check(gpu, x128, psd, wl, bank, tmpl, index, bands, label):
    worst = 0.0
    for c, t, j in zip(gpu, tmpl, index):
        m1, m2 = bank[int(t)]
        chi2, z, _ = O.chisq(x128, psd, wl.n, wl.fs, wl.f_low, m1, m2, int(j), bands)
        err = abs(c - chi2)
        tol = _tol(chi2, z, bands)
        assert err <= tol, (label, int(t), int(j), bands, c, chi2, tol)
        worst = max(worst, err / tol)
    print(f"{label}: {len(tmpl)} values, bands {bands}, worst error / bar {worst:.3f}")


@pytest.fixture(scope="module")
def tiny(ctx):
    wl, bank, injs, x64, psd, x128 = C.workload_case("tiny-2^16")
    seg = ctx.segment(_dev(x64), _dev(psd), wl.n, wl.fs, wl.f_low)
    params = ctx.gen_templates(seg, bank)
    return dict(wl=wl, bank=bank, injs=injs, psd=psd, x128=x128, seg=seg,
                params=params)


def test_chisq_at_triggers_and_peaks_tiny(ctx, tiny):
    wl, bank = tiny["wl"], tiny["bank"]
    peaks, trig, cnt = ctx.find_triggers(tiny["seg"], tiny["params"],
                                         wl.snr_threshold, wl.window, cap=4096)
    _sync()
    count = int(cnt.cpu()[0])
    assert 0 < count <= 4096
    T = ci.triggers_to_numpy(trig, count)
    chi = ctx.chisq(tiny["seg"], tiny["params"], trig, count, bands=16)
    _sync()
    _check(chi.cpu().numpy(), tiny["x128"], tiny["psd"], wl, bank, T["tmpl"],
           T["index"], 16, "tiny triggers")
    P = ci.triggers_to_numpy(peaks)
    for bands in (2, 7, 64):
        chi = ctx.chisq(tiny["seg"], tiny["params"], peaks, bands=bands)
        _sync()
        _check(chi.cpu().numpy(), tiny["x128"], tiny["psd"], wl, bank, P["tmpl"],
               P["index"], bands, "tiny peaks")


def test_chisq_invalid_entries_and_arguments(ctx, tiny):
    wl = tiny["wl"]
    bank = np.vstack([tiny["bank"][:2], [[150.0, 150.0]]])
    params = ctx.gen_templates(tiny["seg"], bank)
    rows = _rows([0, -1, 3, 1, 1, 2, 0], [5, 5, 5, -1, wl.n, 100, 0])
    chi = ctx.chisq(tiny["seg"], params, rows, bands=8)
    _sync()
    c = chi.cpu().numpy()
    # tmpl -1, tmpl >= n, index -1, index >= n_seg and the empty template
    assert np.all(np.isnan(c[1:6])), c
    assert np.all(np.isfinite(c[[0, 6]])) and np.all(c[[0, 6]] >= 0)
    for bands in (1, 65, 0):
        with pytest.raises(ci.CiError) as ei:
            ctx.chisq(tiny["seg"], params, rows, bands=bands)
        assert ei.value.code == ci.EINVAL
    # no triggers: nothing to do, success
    out = ctx.chisq(tiny["seg"], params, rows, n_trig=0, bands=8)
    assert out.shape[0] == 0


def test_chisq_matching_noise_free_signal(ctx):
    """Noise-free data holding one template's chirp: at the coalescence
    sample chi2 = p rho^2 sum_l (s_l - 1/p)^2 (s_l the bands' sigma^2
    shares), tiny; the GPU agrees with the oracle's value."""
    n, fs, fl = 1 << 17, 4096.0, 20.0
    m1, m2, rho, j0 = 1.7, 1.3, 12.0, 40000
    inj = synth.InjectionSpec(m1, m2, rho, j0, 0.3, 0)
    bank = np.array([[m1, m2], [1.9, 1.1]])
    x64, psd, x128 = C.make_case(n, fs, fl, bank, [inj], None)
    seg = ctx.segment(_dev(x64), _dev(psd), n, fs, fl)
    params = ctx.gen_templates(seg, bank)
    bands = 16
    chi = ctx.chisq(seg, params, _rows([0, 1], [j0, j0]), bands=bands)
    _sync()
    c = chi.cpu().numpy()
    chi2, z, _ = O.chisq(x128, psd, n, fs, fl, m1, m2, j0, bands)
    assert abs(abs(z) - rho) < 1e-3 * rho
    assert abs(c[0] - chi2) <= _tol(chi2, z, bands), (c[0], chi2)
    assert c[0] < 0.05 * (2 * bands - 2)
    # the other template sees the chirp through a mismatch: its chi2 is large
    chi2b, zb, _ = O.chisq(x128, psd, n, fs, fl, 1.9, 1.1, j0, bands)
    assert abs(c[1] - chi2b) <= _tol(chi2b, zb, bands), (c[1], chi2b)
    seg.close()


def test_chisq_noise_statistics_on_gpu(ctx):
    """Gaussian noise, 256 templates each at four random samples: the GPU
    values follow chi^2 with 2p - 2 degrees of freedom.  (Samples of one
    template share that template's realised in-band noise power, which
    fluctuates by ~10 %, so the sample mean wanders more than for
    independent draws; the KS bar is loose for that reason.)"""
    from scipy import stats
    n, fs, fl, bands = 1 << 18, 4096.0, 20.0, 8
    bank = synth.draw_masses(256, 1.0, 10.0, "loguniform", 4242)
    x64, psd, x128 = C.make_case(n, fs, fl, bank, [], 9191)
    seg = ctx.segment(_dev(x64), _dev(psd), n, fs, fl)
    params = ctx.gen_templates(seg, bank)
    rng = np.random.default_rng(5150)
    tm = np.repeat(np.arange(len(bank)), 4)
    idx = rng.integers(0, n, len(tm))
    chi = ctx.chisq(seg, params, _rows(tm, idx), bands=bands)
    _sync()
    c = chi.cpu().numpy()
    dof = 2 * bands - 2
    assert np.all(np.isfinite(c))
    p = stats.kstest(c, stats.chi2(dof).cdf).pvalue
    print(f"noise chi2: mean {c.mean():.2f} (dof {dof}), KS p {p:.3f}")
    assert p > 1e-3
    # a few against the oracle
    _check(c[:4], x128, psd, type("W", (), dict(n=n, fs=fs, f_low=fl)), bank,
           tm[:4], idx[:4], bands, "noise samples")
    seg.close()


def test_chisq_full_size_merged_triggers(ctx):
    """The 2^20-sample, 1024-template workload: chi2 of the merged trigger
    list (one per window over the bank), every injection's window plus a
    seeded sample of the others against the oracle; each injection's own
    template at its peak is consistent with noise."""
    wl, bank, injs, x64, psd, x128 = C.workload_case("fp32-2^20")
    seg = ctx.segment(_dev(x64), _dev(psd), wl.n, wl.fs, wl.f_low)
    params = ctx.gen_templates(seg, bank)
    peaks, mtrig, mcnt = ctx.find_triggers(seg, params, wl.snr_threshold,
                                           wl.window, cap=1 << 16, merge=True)
    _sync()
    count = int(mcnt.cpu()[0])
    M = ci.triggers_to_numpy(mtrig, count)
    bands = 16
    chi = ctx.chisq(seg, params, mtrig, count, bands=bands).cpu().numpy()
    assert np.all(np.isfinite(chi))
    inj_w = {inj.j0 // wl.window for inj in injs}
    rng = np.random.default_rng(2718)
    pick = [i for i in range(count) if int(M["window"][i]) in inj_w]
    rest = [i for i in range(count) if i not in pick]
    pick += rng.choice(rest, min(8, len(rest)), replace=False).tolist()
    pick = sorted(pick)
    _check(chi[pick], x128, psd, wl, bank, M["tmpl"][pick], M["index"][pick],
           bands, "fp32-2^20 merged")
    P = ci.triggers_to_numpy(peaks)
    tm = np.array([inj.tmpl for inj in injs])
    cp = ctx.chisq(seg, params, peaks, bands=bands).cpu().numpy()
    assert np.all(cp[tm] < 4 * (2 * bands - 2)), cp[tm]
    _check(cp[tm], x128, psd, wl, bank, tm, P["index"][tm], bands,
           "fp32-2^20 injection peaks")
    seg.close()
