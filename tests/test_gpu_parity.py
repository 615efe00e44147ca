"""GPU-vs-oracle parity of the HIP search path (needs an MI355X).

Every GPU call goes through the C ABI (ctypes binding).  The oracle sees the
same complex64 data spectrum, upcast to complex128, and the same float64 PSD.
Bar for the FP32 path: SNR relative error <= 1e-5 (series error relative to
the series maximum, and at every reported peak and trigger); peak and
trigger indices exact except where the oracle's own values tie within that
tolerance, and windows whose maximum lies within tolerance of the threshold
may go either way.
"""

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


def _segment(ctx, x64, psd, n, fs, f_low):
    return ctx.segment(_dev(x64), _dev(psd), n, fs, f_low)


def _sync():
    import torch
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def tiny(ctx):
    wl, bank, injs, x64, psd, x128 = C.workload_case("tiny-2^16")
    seg = _segment(ctx, x64, psd, wl.n, wl.fs, wl.f_low)
    params = ctx.gen_templates(seg, bank)
    zo = [C.oracle_series(x128, psd, wl.n, wl.fs, wl.f_low, m1, m2)[0]
          for m1, m2 in bank]
    return dict(wl=wl, bank=bank, injs=injs, x64=x64, psd=psd, x128=x128,
                seg=seg, params=params, zo=zo, ctx=ctx)


def test_gen_templates_params_and_htilde(ctx, tiny):
    wl, bank, psd = tiny["wl"], tiny["bank"], tiny["psd"]
    params, ht = ctx.gen_templates(tiny["seg"], bank, htilde=True)
    _sync()
    P = ci.params_to_numpy(params)
    H = ht.cpu().numpy().astype(np.complex128)
    df = wl.fs / wl.n
    for i, (m1, m2) in enumerate(bank):
        _, _, _, kl, kh = O.band(m1, m2, wl.n, wl.fs, wl.f_low)
        assert (P["k_low"][i], P["k_high"][i]) == (kl, kh)
        h = O.spa_htilde(wl.n, wl.fs, wl.f_low, m1, m2)
        s2 = O.sigma2(h, psd, df, kl, kh)
        assert abs(P["sigma2"][i] / s2 - 1) < 1e-12
        assert np.max(np.abs(H[i] - h)) <= 2e-6 * np.max(np.abs(h))
        # eq. (mismatch) between the GPU and the FP64 template: first order
        # in the FP32 amplitude rounding (the paper reports < 3e-4) ...
        assert abs(O.mismatch(h, H[i], psd, df, kl, kh)) < 1e-7
        # ... while the normalised overlap is second order
        ov = O.inner(h, H[i], psd, df, kl, kh) / np.sqrt(
            O.inner(h, h, psd, df, kl, kh) * O.inner(H[i], H[i], psd, df, kl, kh))
        assert 1 - ov < 1e-12


def test_series_tiny_matches_oracle(ctx, tiny):
    z = ctx.matched_filter(tiny["seg"], tiny["params"])
    _sync()
    zg = z.cpu().numpy()
    for i, zo in enumerate(tiny["zo"]):
        e = C.series_error(zg[i], zo)
        assert e <= C.TOL_FP32, (i, e)
    # the exact injection template recovers the injection (noise-perturbed)
    inj = tiny["injs"][0]
    zi = zg[-1]
    j = int(np.argmax(np.abs(zi)))
    assert abs(j - inj.j0) <= 2
    assert abs(abs(zi[j]) - inj.snr) < 3.0


def test_triggers_tiny_match_oracle(ctx, tiny):
    wl = tiny["wl"]
    peaks, trig, cnt = ctx.find_triggers(tiny["seg"], tiny["params"],
                                         wl.snr_threshold, wl.window, cap=4096)
    _sync()
    count = int(cnt.cpu()[0])
    P = ci.triggers_to_numpy(peaks)
    T = ci.triggers_to_numpy(trig, min(count, 4096))
    assert count == len(T)
    # ordered by (template, window)
    keys = [(int(t["tmpl"]), int(t["window"])) for t in T]
    assert keys == sorted(keys)
    for i, zo in enumerate(tiny["zo"]):
        assert int(P[i]["tmpl"]) == i
        C.check_peak(P[i], zo)
        C.check_triggers(T[T["tmpl"] == i], zo, wl.window, wl.snr_threshold)
    # merged: per window, the largest rho^2 over templates
    peaks2, trig2, cnt2 = ctx.find_triggers(tiny["seg"], tiny["params"],
                                            wl.snr_threshold, wl.window,
                                            cap=4096, merge=True)
    _sync()
    M = ci.triggers_to_numpy(trig2, int(cnt2.cpu()[0]))
    assert [int(m["window"]) for m in M] == sorted(set(int(t["window"]) for t in T))
    for m in M:
        same = T[T["window"] == m["window"]]
        best = same[np.argmax(same["rho2"])]
        assert m["rho2"] == best["rho2"] and m["tmpl"] == best["tmpl"]
    assert np.array_equal(ci.triggers_to_numpy(peaks2), P)


@pytest.mark.parametrize("log2n", [16, 17, 18, 19, 20, 21])
def test_series_every_length(ctx, log2n):
    n, fs, fl = 1 << log2n, 4096.0, 20.0
    bank = synth.draw_masses(2, 1.0, 12.0, "loguniform", 900 + log2n)
    inj = synth.InjectionSpec(float(bank[0, 0]), float(bank[0, 1]), 12.0,
                              n // 3 + 17, 0.77, 0)
    x64, psd, x128 = C.make_case(n, fs, fl, bank, [inj], 1000 + log2n)
    seg = _segment(ctx, x64, psd, n, fs, fl)
    params = ctx.gen_templates(seg, bank)
    z = ctx.matched_filter(seg, params)
    peaks, _, _ = ctx.find_triggers(seg, params, 6.0, 4096, cap=16)
    _sync()
    zg = z.cpu().numpy()
    P = ci.triggers_to_numpy(peaks)
    for i, (m1, m2) in enumerate(bank):
        zo, _ = C.oracle_series(x128, psd, n, fs, fl, m1, m2)
        assert C.series_error(zg[i], zo) <= C.TOL_FP32
        C.check_peak(P[i], zo)
    assert abs(int(P[0]["index"]) - inj.j0) <= 2


def test_ragged_batches_are_deterministic(ctx):
    n, fs, fl = 1 << 17, 4096.0, 20.0
    bank = synth.draw_masses(11, 1.0, 8.0, "loguniform", 77)
    injs = [synth.InjectionSpec(float(bank[3, 0]), float(bank[3, 1]), 15.0,
                                40000, 2.0, 3)]
    x64, psd, x128 = C.make_case(n, fs, fl, bank, injs, 78)
    seg = _segment(ctx, x64, psd, n, fs, fl)
    params = ctx.gen_templates(seg, bank)
    outs = []
    for b in (4, 4, 0, 1):
        ctx.set_batch(b)
        p, t, c = ctx.find_triggers(seg, params, 5.0, 4096, cap=1024)
        _sync()
        outs.append((p.cpu().numpy().copy(), t.cpu().numpy()[:int(c.cpu()[0])].copy()))
    ctx.set_batch(0)
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    P = ci.triggers_to_numpy(torch_t(outs[0][0]))
    T = ci.triggers_to_numpy(torch_t(outs[0][1]))
    for i, (m1, m2) in enumerate(bank):
        zo, _ = C.oracle_series(x128, psd, n, fs, fl, m1, m2)
        C.check_peak(P[i], zo)
        C.check_triggers(T[T["tmpl"] == i], zo, 4096, 5.0)


def torch_t(a):
    import torch
    return torch.from_numpy(a)


def test_search_range_and_odd_window(ctx, tiny):
    wl = tiny["wl"]
    j_lo, j_hi, W = 1234, 60001, 3000
    peaks, trig, cnt = ctx.find_triggers(tiny["seg"], tiny["params"], 4.0, W,
                                         j_lo=j_lo, j_hi=j_hi, cap=4096)
    _sync()
    P = ci.triggers_to_numpy(peaks)
    T = ci.triggers_to_numpy(trig, int(cnt.cpu()[0]))
    for i, zo in enumerate(tiny["zo"]):
        C.check_peak(P[i], zo, j_lo=j_lo, j_hi=j_hi)
        C.check_triggers(T[T["tmpl"] == i], zo, W, 4.0, j_lo=j_lo, j_hi=j_hi)


def test_empty_template_and_cap_overflow(ctx, tiny):
    wl = tiny["wl"]
    bank = np.vstack([tiny["bank"][:3], [[150.0, 150.0]]])
    params = ctx.gen_templates(tiny["seg"], bank)
    full_p, full_t, full_c = ctx.find_triggers(tiny["seg"], params, 2.0, 1024,
                                               cap=100000)
    p5, t5, c5 = ctx.find_triggers(tiny["seg"], params, 2.0, 1024, cap=5)
    _sync()
    total = int(full_c.cpu()[0])
    assert total > 5 and int(c5.cpu()[0]) == total
    F = ci.triggers_to_numpy(full_t, total)
    assert np.array_equal(ci.triggers_to_numpy(t5, 5), F[:5])
    P = ci.triggers_to_numpy(full_p)
    assert int(P[3]["index"]) == -1 and float(P[3]["rho2"]) == 0.0
    assert not np.any(F["tmpl"] == 3)
    assert ci.params_to_numpy(params)["flags"][3] == ci.TMPL_EMPTY
    # the documented overflow behaviour: the call succeeds (it is
    # asynchronous), *d_count holds the true total and the list its first
    # `cap` entries in the stated order, (template, window) unmerged ...
    assert list(zip(F["tmpl"], F["window"])) == sorted(zip(F["tmpl"], F["window"]))
    # ... and by window when merged
    mp, mt, mc = ctx.find_triggers(tiny["seg"], params, 2.0, 1024, cap=100000, merge=True)
    sp, st, sc = ctx.find_triggers(tiny["seg"], params, 2.0, 1024, cap=3, merge=True)
    _sync()
    mtot = int(mc.cpu()[0])
    assert mtot > 3 and int(sc.cpu()[0]) == mtot
    M = ci.triggers_to_numpy(mt, mtot)
    assert list(M["window"]) == sorted(M["window"]) and len(set(M["window"])) == mtot
    assert np.array_equal(ci.triggers_to_numpy(st, 3), M[:3])


@pytest.mark.parametrize("prec", [ci.FP32, ci.SPLIT_BF16])
def test_degenerate_searches(ctx, tiny, prec):
    """Edge cases of the search, against the oracle: no templates; a zero
    threshold (every window's maximum is a trigger); windows of one sample
    (nwin = n) and of the whole series; a one-sample search range at the
    end of the series; all-zero data (every sample ties at rho^2 = 0: the
    peak is sample 0 and, the threshold being strict, nothing triggers)."""
    import torch
    wl, n = tiny["wl"], tiny["wl"].n
    tol = C.TOL_FP32 if prec == ci.FP32 else 1e-3
    seg, params, zo = tiny["seg"], tiny["params"], tiny["zo"]
    nt = len(zo)
    # no templates: nothing is written but the count
    cnt0 = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    ctx.find_triggers(seg, params, 6.0, 4096, n=0, count=cnt0, precision=prec)
    _sync()
    assert int(cnt0.cpu()[0]) == 0
    cases = [dict(thr=0.0, W=4096), dict(thr=3.5, W=1), dict(thr=3.0, W=n),
             dict(thr=0.0, W=1000, j_lo=n - 1, j_hi=n)]
    for cs in cases:
        jl, jh = cs.get("j_lo", 0), cs.get("j_hi", 0)
        cap = nt * ((n + cs["W"] - 1) // cs["W"])
        peaks, trig, cnt = ctx.find_triggers(seg, params, cs["thr"], cs["W"], j_lo=jl, j_hi=jh,
                                             cap=cap, precision=prec)
        _sync()
        P = ci.triggers_to_numpy(peaks)
        T = ci.triggers_to_numpy(trig, int(cnt.cpu()[0]))
        for i in range(nt):
            C.check_peak(P[i], zo[i], tol=tol, j_lo=jl, j_hi=jh or None)
            C.check_triggers(T[T["tmpl"] == i], zo[i], cs["W"], cs["thr"], tol=tol, j_lo=jl,
                             j_hi=jh or None)
        if cs["thr"] == 0.0:
            # every window of the range has a trigger (the data has no zeros)
            nw = len({j // cs["W"] for j in range(jl, jh or n)})
            assert int(cnt.cpu()[0]) == nt * nw
    # all-zero data
    zero = np.zeros(n // 2 + 1, dtype=np.complex64)
    zseg = _segment(ctx, zero, tiny["psd"], n, wl.fs, wl.f_low)
    zpar = ctx.gen_templates(zseg, tiny["bank"])
    peaks, trig, cnt = ctx.find_triggers(zseg, zpar, 0.0, 4096, cap=64, precision=prec)
    _sync()
    P = ci.triggers_to_numpy(peaks)
    assert int(cnt.cpu()[0]) == 0
    assert np.all(P["index"] == 0) and np.all(P["rho2"] == 0.0)
    zseg.close()


def test_argument_errors(ctx, tiny):
    with pytest.raises(ci.CiError) as ei:
        ctx.find_triggers(tiny["seg"], tiny["params"], 6.0, 0)
    assert ei.value.code == ci.EINVAL
    with pytest.raises(ci.CiError) as ei:
        ctx.find_triggers(tiny["seg"], tiny["params"], 6.0, 4096, j_lo=10, j_hi=5)
    assert ei.value.code == ci.EINVAL
    with pytest.raises(ci.CiError) as ei:
        ctx.matched_filter(tiny["seg"], tiny["params"], precision=7)
    assert ei.value.code == ci.EINVAL
    import torch
    bad = torch.zeros(2**15 + 1, dtype=torch.complex64, device="cuda")
    badp = torch.ones(2**15 + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(ci.CiError) as ei:
        ctx.segment(bad, badp, 2**16, 4096.0, 3000.0)
    assert ei.value.code == ci.EINVAL


def test_segment_outlives_its_context(gpu_lib, tiny):
    """A segment still alive when its context is destroyed is detached: it
    can only be destroyed, other calls reject it, and nothing the library
    does afterwards sees a stale device error."""
    wl = tiny["wl"]
    x = _dev(tiny["x64"])
    p = _dev(tiny["psd"])
    a = gpu_lib.context(0)
    sa = a.segment(x, p, wl.n, wl.fs, wl.f_low)
    a.close()
    b = gpu_lib.context(0)
    with pytest.raises(ci.CiError) as ei:
        b.gen_templates(sa, tiny["bank"])
    assert ei.value.code == ci.EINVAL
    with pytest.raises(ci.CiError) as ei:
        b.segment_update(sa, x, p)
    assert ei.value.code == ci.EINVAL
    sa.close()
    sb = b.segment(x, p, wl.n, wl.fs, wl.f_low)
    params = b.gen_templates(sb, tiny["bank"])
    z = b.matched_filter(sb, params)
    _sync()
    assert np.array_equal(z.cpu().numpy()[0],
                          tiny["ctx"].matched_filter(tiny["seg"], tiny["params"])
                          .cpu().numpy()[0])
    sb.close()
    b.close()


def test_full_size_fp32_workload_sampled(ctx):
    """The 2^20-sample, 1024-template, five-injection workload in the
    benchmark's launch configuration; the oracle checks a sample of
    templates (every injection's template plus seeded random ones)."""
    wl, bank, injs, x64, psd, x128 = C.workload_case("fp32-2^20")
    seg = _segment(ctx, x64, psd, wl.n, wl.fs, wl.f_low)
    params = ctx.gen_templates(seg, bank)
    peaks, trig, cnt = ctx.find_triggers(seg, params, wl.snr_threshold,
                                         wl.window, cap=1 << 20)
    _, mtrig, mcnt = ctx.find_triggers(seg, params, wl.snr_threshold,
                                       wl.window, cap=1 << 20, merge=True)
    _sync()
    P = ci.triggers_to_numpy(peaks)
    count = int(cnt.cpu()[0])
    T = ci.triggers_to_numpy(trig, count)
    M = ci.triggers_to_numpy(mtrig, int(mcnt.cpu()[0]))
    # the declared sample: 64 seeded random templates, every injection's
    # template, and the winner of every injection's window in the merged list
    win = {int(m["window"]): int(m["tmpl"]) for m in M}
    winners = {win[inj.j0 // wl.window] for inj in injs if inj.j0 // wl.window in win}
    rng = np.random.default_rng(12345)
    sample = sorted(set([i.tmpl for i in injs]) | winners |
                    set(rng.choice(len(bank), 64, replace=False).tolist()))
    assert all(inj.j0 // wl.window in win for inj in injs)
    for i in sample:
        zo, _ = C.oracle_series(x128, psd, wl.n, wl.fs, wl.f_low, *bank[i])
        C.check_peak(P[i], zo)
        C.check_triggers(T[T["tmpl"] == i], zo, wl.window, wl.snr_threshold)
    # every injection is found by its own template at its coalescence sample
    for inj in injs:
        assert abs(int(P[inj.tmpl]["index"]) - inj.j0) <= 2
    # merged list: per window the best of the per-template triggers
    assert sorted(set(T["window"].tolist())) == M["window"].tolist()
    for m in M:
        same = T[T["window"] == m["window"]]
        best = same[np.lexsort((same["tmpl"], -same["rho2"]))][0]
        assert (m["tmpl"], m["index"], m["rho2"]) == (best["tmpl"], best["index"],
                                                      best["rho2"])


@pytest.mark.parametrize("tc,tj", [(4, 4), (4, 8), (8, 4), (8, 8)])
@pytest.mark.parametrize("log2n", [16, 20, 21])
def test_tile_shapes(ctx, tc, tj, log2n):
    """Every pass-1 / pass-2 tile shape, with the batches in order on one
    stream or alternating over two, gives the oracle's series and peaks,
    bit-identical to the default configuration's."""
    n, fs, fl = 1 << log2n, 4096.0, 20.0
    bank = synth.draw_masses(3, 1.0, 20.0, "loguniform", 31 * tc + tj + log2n)
    inj = synth.InjectionSpec(float(bank[1, 0]), float(bank[1, 1]), 9.0,
                              n // 5 + 3, 1.1, 1)
    x64, psd, x128 = C.make_case(n, fs, fl, bank, [inj], 2000 + log2n)
    seg = _segment(ctx, x64, psd, n, fs, fl)
    params = ctx.gen_templates(seg, bank)
    z0 = ctx.matched_filter(seg, params)
    p0, t0, c0 = ctx.find_triggers(seg, params, 5.5, 4096, cap=256)
    ctx.set_tune(log2n, ci.FP32, tc, tj, 1 + (tc + tj) % 3, 2,
                 streams=1 + (tc // 4 + tj // 4 + log2n) % 2)
    try:
        z = ctx.matched_filter(seg, params)
        peaks, trig, cnt = ctx.find_triggers(seg, params, 5.5, 4096, cap=256)
        _sync()
    finally:
        ctx.set_tune(log2n, ci.FP32)
    assert np.array_equal(z.cpu().numpy(), z0.cpu().numpy())
    assert np.array_equal(peaks.cpu().numpy(), p0.cpu().numpy())
    assert int(cnt.cpu()[0]) == int(c0.cpu()[0])
    k = min(int(c0.cpu()[0]), 256)
    assert np.array_equal(trig.cpu().numpy()[:k], t0.cpu().numpy()[:k])
    zg = z.cpu().numpy()
    P = ci.triggers_to_numpy(peaks)
    T = ci.triggers_to_numpy(trig, int(cnt.cpu()[0]))
    for i, (m1, m2) in enumerate(bank):
        zo, _ = C.oracle_series(x128, psd, n, fs, fl, m1, m2)
        assert C.series_error(zg[i], zo) <= C.TOL_FP32
        C.check_peak(P[i], zo)
        C.check_triggers(T[T["tmpl"] == i], zo, 4096, 5.5)
    seg.close()


@pytest.mark.parametrize("tj", [4, 8])
@pytest.mark.parametrize("log2n", [17, 18, 19, 20, 21])
def test_second_pass_wave_columns(ctx, tj, log2n):
    """The FP32 second pass with wave-owned columns after its first stage
    (p2_wave) gives the default second pass's peaks and trigger lists bit
    for bit (merged and unmerged, full and restricted search ranges), and
    the oracle's peaks."""
    n, fs, fl = 1 << log2n, 4096.0, 20.0
    bank = synth.draw_masses(6, 1.0, 20.0, "loguniform", 77 + 3 * tj + log2n)
    inj = synth.InjectionSpec(float(bank[2, 0]), float(bank[2, 1]), 12.0,
                              n // 3 + 11, 0.7, 2)
    x64, psd, x128 = C.make_case(n, fs, fl, bank, [inj], 3000 + log2n)
    seg = _segment(ctx, x64, psd, n, fs, fl)
    params = ctx.gen_templates(seg, bank)
    cases = [dict(merge=False), dict(merge=True),
             dict(merge=False, j_lo=n // 7 + 5, j_hi=n - n // 5 - 3)]
    cap = 4096

    def run():
        out = []
        for kw in cases:
            p, t, c = ctx.find_triggers(seg, params, 4.0, 2048, cap=cap, **kw)
            out.append((p, t, c))
        _sync()
        return [(p.cpu().numpy().copy(), t.cpu().numpy()[:min(int(c.cpu()[0]), cap)].copy(),
                 int(c.cpu()[0])) for p, t, c in out]

    ctx.set_tune(log2n, ci.FP32, 8, tj, 0, 0, streams=1)
    try:
        ref = run()
        ctx.set_tune(log2n, ci.FP32, 8, tj, 0, 0, streams=1, p2_wave=1)
        got = run()
        assert ctx.get_tune(log2n, ci.FP32)["p2_wave"] == 1
    finally:
        ctx.set_tune(log2n, ci.FP32)
    for (p0, t0, c0), (p1, t1, c1) in zip(ref, got):
        assert c0 == c1 and c0 > 0
        assert np.array_equal(p0, p1)
        assert np.array_equal(t0, t1)
    P = got[0][0].view(ci.TRIGGER_DTYPE).reshape(-1)
    for i, (m1, m2) in enumerate(bank):
        zo, _ = C.oracle_series(x128, psd, n, fs, fl, m1, m2)
        C.check_peak(P[i], zo)
    seg.close()


# --------------------------------------------------------------------------
# split-precision path: radix-16 stages on the matrix cores (bar: 1e-3)
# --------------------------------------------------------------------------

TOL_SPLIT = 1e-3


@pytest.mark.parametrize("prec", [ci.SPLIT_BF16, ci.SPLIT_FP16])
@pytest.mark.parametrize("log2n", [16, 17, 18, 19, 20, 21])
def test_split_precision_series(ctx, prec, log2n):
    n, fs, fl = 1 << log2n, 4096.0, 20.0
    bank = synth.draw_masses(2, 1.0, 12.0, "loguniform", 700 + log2n)
    inj = synth.InjectionSpec(float(bank[0, 0]), float(bank[0, 1]), 14.0,
                              n // 3 + 5, 2.2, 0)
    x64, psd, x128 = C.make_case(n, fs, fl, bank, [inj], 3000 + log2n)
    seg = _segment(ctx, x64, psd, n, fs, fl)
    params = ctx.gen_templates(seg, bank)
    z = ctx.matched_filter(seg, params, precision=prec)
    peaks, trig, cnt = ctx.find_triggers(seg, params, 6.0, 4096, cap=256,
                                         precision=prec)
    _sync()
    zg = z.cpu().numpy()
    P = ci.triggers_to_numpy(peaks)
    T = ci.triggers_to_numpy(trig, int(cnt.cpu()[0]))
    for i, (m1, m2) in enumerate(bank):
        zo, _ = C.oracle_series(x128, psd, n, fs, fl, m1, m2)
        e = C.series_error(zg[i], zo)
        print(f"precision {prec} n 2^{log2n} template {i}: series error {e:.2e}")
        assert e <= TOL_SPLIT, e
        C.check_peak(P[i], zo, tol=TOL_SPLIT)
        C.check_triggers(T[T["tmpl"] == i], zo, 4096, 6.0, tol=TOL_SPLIT)
    assert abs(int(P[0]["index"]) - inj.j0) <= 2
    seg.close()


@pytest.mark.parametrize("prec", [ci.SPLIT_BF16, ci.SPLIT_FP16])
@pytest.mark.parametrize("snr", [5.0e3, 5.0e4])
@pytest.mark.parametrize("log2n", [16, 20])
def test_split_precision_loud_signal(ctx, prec, snr, log2n):
    """A loud chirp (optimal SNR 5e3 or 5e4, far above the 2^9 limit of
    the FP16 operands' fixed 2^6 pre-scale in the last matrix-core stages):
    the matrix-core instances whose inputs exceed the limit take their own
    power-of-two scale, so the series, the peak and the triggers stay at
    the split bar (relative to the series maximum and to each trigger's
    own rho) on both split paths."""
    n, fs, fl = 1 << log2n, 4096.0, 20.0
    bank = synth.draw_masses(2, 1.0, 8.0, "loguniform", 900 + log2n)
    inj = synth.InjectionSpec(float(bank[0, 0]), float(bank[0, 1]), snr,
                              n // 4 + 17, 0.9, 0)
    x64, psd, x128 = C.make_case(n, fs, fl, bank, [inj], 3100 + log2n)
    seg = _segment(ctx, x64, psd, n, fs, fl)
    params = ctx.gen_templates(seg, bank)
    z = ctx.matched_filter(seg, params, precision=prec)
    thr = 0.01 * snr
    peaks, trig, cnt = ctx.find_triggers(seg, params, thr, 4096, cap=4096, precision=prec)
    _sync()
    zg = z.cpu().numpy()
    assert np.all(np.isfinite(zg))
    P = ci.triggers_to_numpy(peaks)
    T = ci.triggers_to_numpy(trig, int(cnt.cpu()[0]))
    for i, (m1, m2) in enumerate(bank):
        zo, _ = C.oracle_series(x128, psd, n, fs, fl, m1, m2)
        e = C.series_error(zg[i], zo)
        print(f"precision {prec} snr {snr:g} n 2^{log2n} template {i}: series error {e:.2e}, "
              f"max rho {np.max(np.abs(zo)):.4g}")
        assert e <= TOL_SPLIT, e
        C.check_peak(P[i], zo, tol=TOL_SPLIT)
        C.check_triggers(T[T["tmpl"] == i], zo, 4096, thr, tol=TOL_SPLIT)
    assert int(P[0]["index"]) == inj.j0
    assert abs(np.sqrt(P[0]["rho2"]) / snr - 1) < 0.01
    seg.close()


@pytest.mark.parametrize("prec", [ci.SPLIT_BF16, ci.SPLIT_FP16])
def test_split_precision_full_size_sampled(ctx, prec):
    """The 2^20 x 1024-template workload on the matrix-core path; errors
    per injection against the FP64 oracle stay below 1e-3."""
    wl, bank, injs, x64, psd, x128 = C.workload_case("fp32-2^20")
    seg = _segment(ctx, x64, psd, wl.n, wl.fs, wl.f_low)
    params = ctx.gen_templates(seg, bank)
    peaks, trig, cnt = ctx.find_triggers(seg, params, wl.snr_threshold,
                                         wl.window, cap=1 << 20, precision=prec)
    _sync()
    P = ci.triggers_to_numpy(peaks)
    T = ci.triggers_to_numpy(trig, int(cnt.cpu()[0]))
    for inj in injs:
        i = inj.tmpl
        zo, _ = C.oracle_series(x128, psd, wl.n, wl.fs, wl.f_low, *bank[i])
        C.check_peak(P[i], zo, tol=TOL_SPLIT)
        C.check_triggers(T[T["tmpl"] == i], zo, wl.window, wl.snr_threshold,
                         tol=TOL_SPLIT)
        rho_o = np.abs(zo[int(P[i]["index"])])
        err = abs(np.sqrt(P[i]["rho2"]) - rho_o) / rho_o
        print(f"precision {prec} injection snr {inj.snr}: peak rho error {err:.2e}")
        assert err <= TOL_SPLIT


@pytest.mark.parametrize("name", ["precision-2^20", "3g-2^21"])
def test_large_banks_sampled(ctx, name):
    """The 65536-template bank at 2^20 and the 1 048 576-template bank at 2^21
    (from 10 Hz), FP32 and split-BF16 in their default launch
    configurations: every injection's template, the winners of the
    injections' windows and 64 seeded random ones against the oracle (FP32
    bar for FP32, 1e-3 for split-BF16), merged lists consistent between
    the paths."""
    wl, bank, injs, x64, psd, x128 = C.workload_case(name)
    seg = _segment(ctx, x64, psd, wl.n, wl.fs, wl.f_low)
    params = ctx.gen_templates(seg, bank)
    res = {}
    for prec in (ci.FP32, ci.SPLIT_BF16):
        peaks, trig, cnt = ctx.find_triggers(seg, params, wl.snr_threshold, wl.window,
                                             cap=1 << 16, merge=True, precision=prec)
        _sync()
        res[prec] = (ci.triggers_to_numpy(peaks).copy(),
                     ci.triggers_to_numpy(trig, min(int(cnt.cpu()[0]), 1 << 16)).copy())
    # the declared sample: 64 seeded random templates, every injection's
    # template, and each path's winner of every injection's window; a
    # winner's merged record is checked against the oracle at its sample
    rng = np.random.default_rng(777)
    inj_w = {inj.j0 // wl.window for inj in injs}
    wrec = {}
    for prec in (ci.FP32, ci.SPLIT_BF16):
        for m in res[prec][1]:
            if int(m["window"]) in inj_w:
                wrec.setdefault(int(m["tmpl"]), []).append((prec, m))
    assert sum(len(v) for v in wrec.values()) == 2 * len(inj_w)
    sample = sorted(set(i.tmpl for i in injs) | set(wrec) |
                    set(rng.choice(len(bank), 64, replace=False).tolist()))
    for i in sample:
        zo, _ = C.oracle_series(x128, psd, wl.n, wl.fs, wl.f_low, *bank[i])
        C.check_peak(res[ci.FP32][0][i], zo)
        C.check_peak(res[ci.SPLIT_BF16][0][i], zo, tol=TOL_SPLIT)
        for prec, m in wrec.get(i, []):
            tol = C.TOL_FP32 if prec == ci.FP32 else TOL_SPLIT
            ro = abs(zo[int(m["index"])])
            assert abs(np.sqrt(float(m["rho2"])) - ro) <= tol * ro, (prec, i, m)
            # the winner's value is the window maximum of its own series
            w = int(m["window"])
            wmax = np.max(np.abs(zo[w * wl.window:(w + 1) * wl.window]))
            assert ro >= wmax * (1 - 2 * tol), (prec, i, ro, wmax)
    # (an injection's own template need not peak at its coalescence sample:
    # in the 65536-template bank the SNR-8 injection's template responds more
    # strongly to the SNR-17 injection of nearly the same chirp mass; the
    # oracle comparison above is the check)
    # the merged windows of the two paths: the same windows, and where the
    # winning template differs the two values tie within the split bar
    M32, M16 = res[ci.FP32][1], res[ci.SPLIT_BF16][1]
    print(f"{name}: {len(bank)} templates, {len(M32)} merged windows")
    w32 = {int(m["window"]): m for m in M32}
    for m in M16:
        w = int(m["window"])
        if w in w32:
            a, b = float(w32[w]["rho2"]), float(m["rho2"])
            assert abs(np.sqrt(a) - np.sqrt(b)) <= 2 * TOL_SPLIT * np.sqrt(a)
        else:
            assert float(m["rho2"]) <= wl.snr_threshold ** 2 * (1 + 4 * TOL_SPLIT)
    for w, m in w32.items():
        if w not in {int(x["window"]) for x in M16}:
            assert float(m["rho2"]) <= wl.snr_threshold ** 2 * (1 + 4 * TOL_SPLIT)
    seg.close()


@pytest.mark.parametrize("prec", [ci.SPLIT_BF16, ci.SPLIT_FP16])
def test_split_range_window_merge_and_overflow(ctx, tiny, prec):
    """The matrix-core second pass's own post-pass: a search range, an odd
    window, the merged list and a capacity overflow, against the oracle at
    the split bar, and the merged list against its per-template list."""
    j_lo, j_hi, W = 1234, 60001, 3000
    peaks, trig, cnt = ctx.find_triggers(tiny["seg"], tiny["params"], 4.0, W, j_lo=j_lo,
                                         j_hi=j_hi, cap=4096, precision=prec)
    _, mtrig, mcnt = ctx.find_triggers(tiny["seg"], tiny["params"], 4.0, W, j_lo=j_lo,
                                       j_hi=j_hi, cap=4096, merge=True, precision=prec)
    _, t3, c3 = ctx.find_triggers(tiny["seg"], tiny["params"], 4.0, W, j_lo=j_lo,
                                  j_hi=j_hi, cap=3, precision=prec)
    _sync()
    P = ci.triggers_to_numpy(peaks)
    total = int(cnt.cpu()[0])
    T = ci.triggers_to_numpy(trig, total)
    for i, zo in enumerate(tiny["zo"]):
        C.check_peak(P[i], zo, tol=TOL_SPLIT, j_lo=j_lo, j_hi=j_hi)
        C.check_triggers(T[T["tmpl"] == i], zo, W, 4.0, tol=TOL_SPLIT, j_lo=j_lo, j_hi=j_hi)
    assert np.all((T["index"] >= j_lo) & (T["index"] < j_hi))
    M = ci.triggers_to_numpy(mtrig, int(mcnt.cpu()[0]))
    assert sorted(set(T["window"].tolist())) == M["window"].tolist()
    for m in M:
        same = T[T["window"] == m["window"]]
        best = same[np.lexsort((same["tmpl"], -same["rho2"]))][0]
        assert (m["tmpl"], m["index"], m["rho2"]) == (best["tmpl"], best["index"], best["rho2"])
    assert total > 3 and int(c3.cpu()[0]) == total
    assert np.array_equal(ci.triggers_to_numpy(t3, 3), T[:3])


def test_segment_update_equals_fresh_segment(ctx):
    """ci_segment_update with new data and PSD gives bit for bit what a
    segment created from that data gives (parameters and search)."""
    n, fs, fl = 1 << 17, 4096.0, 20.0
    bank = synth.draw_masses(5, 1.0, 8.0, "loguniform", 31)
    psd_a = synth.make_psd(n, fs)
    psd_b = psd_a * (1.0 + 0.3 * np.sin(np.arange(n // 2 + 1) / 500.0) ** 2)
    xa = synth.make_noise(n, fs, fl, psd_a, 41).astype(np.complex64)
    xb = synth.make_noise(n, fs, fl, psd_b, 42).astype(np.complex64)
    seg = _segment(ctx, xa, psd_a, n, fs, fl)
    ctx.segment_update(seg, _dev(xb), _dev(psd_b))
    fresh = _segment(ctx, xb, psd_b, n, fs, fl)
    pu, pf = ctx.gen_templates(seg, bank), ctx.gen_templates(fresh, bank)
    ru = ctx.find_triggers(seg, pu, 4.0, 4096, cap=4096)
    rf = ctx.find_triggers(fresh, pf, 4.0, 4096, cap=4096)
    _sync()
    assert np.array_equal(pu.cpu().numpy(), pf.cpu().numpy())
    assert np.array_equal(ru[0].cpu().numpy(), rf[0].cpu().numpy())
    cu, cf = int(ru[2].cpu()[0]), int(rf[2].cpu()[0])
    assert cu == cf
    assert np.array_equal(ru[1].cpu().numpy()[:cu], rf[1].cpu().numpy()[:cf])
    # and against the oracle on the new data
    P = ci.triggers_to_numpy(ru[0])
    for i, (m1, m2) in enumerate(bank):
        zo, _ = C.oracle_series(xb.astype(np.complex128), psd_b, n, fs, fl, m1, m2)
        C.check_peak(P[i], zo)
    seg.close()
    fresh.close()
