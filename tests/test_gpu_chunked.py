"""A large bank searched in resumable chunks (needs an MI355X): the device
merge of per-chunk window lists, and a run interrupted after some chunks and
resumed from its checkpoint, both equal one search over the whole bank bit
for bit (peaks with bank-wide template ids, merged list, count)."""
import numpy as np
import pytest

from paper_1006_4644_amd import ci, synth
from tests import mfcase as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case(gpu_lib):
    import torch
    ctx = gpu_lib.context(0)
    n, fs, fl = 1 << 16, 4096.0, 20.0
    bank = synth.draw_masses(70, 1.0, 12.0, "loguniform", 1212)
    # a duplicate in a later chunk: every window ties between the two, and
    # the earlier template must keep it, as in one search over the bank
    bank[41] = bank[5]
    inj = synth.InjectionSpec(float(bank[23, 0]), float(bank[23, 1]), 15.0, n // 2 + 7, 0.3, 23)
    x64, psd, _ = C.make_case(n, fs, fl, bank, [inj], 1313)
    seg = ctx.segment(torch.from_numpy(x64).cuda(), torch.from_numpy(psd).cuda(), n, fs, fl)
    yield dict(ctx=ctx, seg=seg, bank=bank, n=n)
    seg.close()
    ctx.close()


def _ref(c, thr, W, prec):
    import torch
    params = c["ctx"].gen_templates(c["seg"], c["bank"])
    nwin = (c["n"] + W - 1) // W
    p, t, k = c["ctx"].find_triggers(c["seg"], params, thr, W, cap=nwin, merge=True,
                                     precision=prec)
    torch.cuda.synchronize()
    kk = int(k.cpu()[0])
    return p.cpu().numpy(), t.cpu().numpy()[:kk], kk


def _host(res):
    import torch
    p, m, k = res
    torch.cuda.synchronize()
    kk = int(k.cpu()[0])
    return p.cpu().numpy(), m.cpu().numpy()[:kk], kk


@pytest.mark.parametrize("prec", [ci.FP32, ci.SPLIT_BF16])
def test_chunked_equals_one_search(case, prec):
    thr, W = 3.5, 2048
    rp, rt, rk = _ref(case, thr, W, prec)
    assert rk > 10
    T = rt.view(ci.TRIGGER_DTYPE).reshape(-1)
    assert not np.any(T["tmpl"] == 41)          # the duplicate never wins a tie
    for chunk in (16, 70, 128):
        gp, gt, gk = _host(case["ctx"].search_bank_chunked(case["seg"], case["bank"], thr, W,
                                                           chunk, precision=prec))
        assert gk == rk
        assert np.array_equal(gp, rp)
        assert np.array_equal(gt, rt)


def test_chunked_resume_after_failure(case, tmp_path):
    thr, W = 3.5, 2048
    rp, rt, rk = _ref(case, thr, W, ci.FP32)
    ck = str(tmp_path / "bank.ckpt.npz")
    with pytest.raises(ci.ChunkFailure):
        case["ctx"].search_bank_chunked(case["seg"], case["bank"], thr, W, 16, checkpoint=ck,
                                        fail_after=2)
    with np.load(ck) as z:
        assert int(z["cursor"]) == 32
    gp, gt, gk = _host(case["ctx"].search_bank_chunked(case["seg"], case["bank"], thr, W, 16,
                                                       checkpoint=ck))
    assert gk == rk and np.array_equal(gp, rp) and np.array_equal(gt, rt)
    # a finished checkpoint: nothing left to do, the same results
    gp2, gt2, gk2 = _host(case["ctx"].search_bank_chunked(case["seg"], case["bank"], thr, W, 16,
                                                          checkpoint=ck))
    assert gk2 == rk and np.array_equal(gp2, rp) and np.array_equal(gt2, rt)
    # another search cannot resume from it
    with pytest.raises(ValueError):
        case["ctx"].search_bank_chunked(case["seg"], case["bank"], thr + 1.0, W, 16,
                                        checkpoint=ck)


def _list(rng, nwin, frac, tmpl_hi):
    """A per-window list (one entry on a random subset of windows, window
    order) as (m, 4) int64 rows."""
    w = np.flatnonzero(rng.random(nwin) < frac)
    a = np.zeros(len(w), dtype=ci.TRIGGER_DTYPE)
    a["window"] = w
    a["index"] = w * 100 + rng.integers(0, 100, len(w))
    a["tmpl"] = rng.integers(0, tmpl_hi, len(w))
    a["rho2"] = rng.choice([9.0, 16.0, 25.0, 36.0], len(w)).astype(np.float32)
    a["re"] = rng.standard_normal(len(w)).astype(np.float32)
    a["im"] = rng.standard_normal(len(w)).astype(np.float32)
    return a


def _expected(a, b, off, nwin):
    """Per window: the larger rho2, a's entry on equal values; b's ids shifted."""
    rec = {}
    for e in a:
        rec[int(e["window"])] = e.copy()
    for e in b:
        e = e.copy()
        e["tmpl"] += off
        w = int(e["window"])
        if w not in rec or e["rho2"] > rec[w]["rho2"]:
            rec[w] = e
    out = np.array([rec[w] for w in sorted(rec) if w < nwin], dtype=ci.TRIGGER_DTYPE)
    return out


def _dev(a, rows=None):
    import torch
    rows = len(a) if rows is None else rows
    buf = np.zeros(max(rows, 1), dtype=ci.TRIGGER_DTYPE)
    buf[:len(a)] = a
    return torch.from_numpy(buf.view(np.int64).reshape(-1, 4).copy()).cuda()


def _cnt(k):
    import torch
    return torch.tensor([k], dtype=torch.int64).cuda()


def test_merge_lists(gpu_lib):
    import torch
    ctx = gpu_lib.context(0)
    rng = np.random.default_rng(4242)
    try:
        for nwin, fa, fb, off in ((1, 1.0, 1.0, 7), (300, 0.4, 0.5, 1000), (5000, 0.1, 0.9, 3),
                                  (257, 0.0, 0.3, 0), (257, 0.3, 0.0, 5)):
            a, b = _list(rng, nwin, fa, 50), _list(rng, nwin, fb, 50)
            exp = _expected(a, b, off, nwin)
            out, cnt = ctx.merge_triggers(_dev(a), _cnt(len(a)), _dev(b), _cnt(len(b)), nwin,
                                          tmpl_offset_b=off)
            torch.cuda.synchronize()
            k = int(cnt.cpu()[0])
            assert k == len(exp)
            got = out.cpu().numpy().view(ci.TRIGGER_DTYPE).reshape(-1)[:k]
            assert np.array_equal(got.view(np.int64), exp.view(np.int64)), nwin
        # only the first min(count, cap) entries of an input are read, only
        # cap entries are written while the count reports every window, and
        # the output may be the first list itself
        nwin = 400
        a, b = _list(rng, nwin, 0.5, 20), _list(rng, nwin, 0.5, 20)
        da = _dev(a, rows=nwin)
        ca = _cnt(len(a))
        cut = len(b) // 2
        exp = _expected(a, b[:cut], 11, nwin)
        db = _dev(b)[:cut]
        out, cnt = ctx.merge_triggers(da, ca, db, _cnt(len(b)), nwin, tmpl_offset_b=11,
                                      out=da, count=ca)
        torch.cuda.synchronize()
        assert out.data_ptr() == da.data_ptr() and int(ca.cpu()[0]) == len(exp)
        got = da.cpu().numpy().view(ci.TRIGGER_DTYPE).reshape(-1)[:len(exp)]
        assert np.array_equal(got.view(np.int64), exp.view(np.int64))
        small = torch.zeros((5, 4), dtype=torch.int64, device="cuda")
        sc = _cnt(0)
        ctx.merge_triggers(_dev(a), _cnt(len(a)), _dev(b), _cnt(len(b)), nwin, out=small,
                           count=sc)
        torch.cuda.synchronize()
        full = _expected(a, b, 0, nwin)
        assert int(sc.cpu()[0]) == len(full)
        got = small.cpu().numpy().view(ci.TRIGGER_DTYPE).reshape(-1)
        assert np.array_equal(got.view(np.int64), full[:5].view(np.int64))
        with pytest.raises(ci.CiError):
            ctx.merge_triggers(_dev(a), _cnt(len(a)), _dev(b), _cnt(len(b)), 0)
    finally:
        ctx.close()
