"""The search without allocation (ci_find_triggers_noalloc, the library's
fixed per-GPU scratch) against the ordinary search (ci_find_triggers, the
context's workspaces), through the C ABI: three calls in a row, each on a
smaller input than the one before (2^21, where the scratch holds one
template per batch and FP32 and the split paths factor the length
differently, then 2^20 and 2^17), each equal to the ordinary search bit for
bit (the same kernels and arithmetic; only the batch size and the schedule
differ, and no launch configuration changes the results)."""
import numpy as np
import pytest

from paper_1006_4644_amd import ci, synth

pytestmark = pytest.mark.gpu


def _case(ctx, n, count, seed):
    import torch
    fs, fl = 4096.0, 20.0
    psd = synth.make_psd(n, fs)
    x = synth.make_noise(n, fs, fl, psd, seed).astype(np.complex64)
    seg = ctx.segment(torch.from_numpy(x).cuda(), torch.from_numpy(psd).cuda(), n, fs, fl)
    params = ctx.gen_templates(seg, synth.draw_masses(count, 1.0, 10.0, "loguniform", seed))
    return seg, params


def _outputs(count, cap):
    import torch
    return (torch.full((count, 4), -7, dtype=torch.int64, device="cuda"),
            torch.full((cap, 4), -7, dtype=torch.int64, device="cuda"),
            torch.full((1,), -7, dtype=torch.int64, device="cuda"))


@pytest.mark.parametrize("prec", [ci.FP32, ci.SPLIT_BF16, ci.SPLIT_FP16])
def test_noalloc_matches_find_triggers(gpu_lib, prec):
    import torch
    ctx = gpu_lib.context(0)
    cap = 1 << 14
    # (samples, templates, window, merge); each call smaller than the last
    cases = [(1 << 21, 3, 4096, True), (1 << 20, 9, 4096, True), (1 << 17, 5, 1024, False)]
    for i, (n, count, W, merge) in enumerate(cases):
        seg, params = _case(ctx, n, count, 4100 + i)
        thr = 4.0
        ref = ctx.find_triggers(seg, params, thr, W, cap=cap, merge=merge, precision=prec)
        torch.cuda.synchronize()
        rp, rt, rc = (t.cpu().numpy().copy() for t in ref)
        out = _outputs(count, cap)
        ctx.find_triggers_noalloc(seg, params, thr, W, *out, merge=merge, precision=prec)
        torch.cuda.synchronize()
        p, t, c = (v.cpu().numpy() for v in out)
        k = min(int(rc[0]), cap)
        print(f"precision {prec}, n = 2^{n.bit_length() - 1}, {count} templates: "
              f"{int(rc[0])} triggers")
        assert int(rc[0]) > 0
        assert int(c[0]) == int(rc[0])
        assert np.array_equal(p, rp)
        assert np.array_equal(t[:k], rt[:k])
        seg.close()
    ctx.close()


def test_noalloc_rejects_what_does_not_fit(gpu_lib):
    """Window 1 at 2^20: 2^20 windows of trigger bookkeeping for one
    template exceed the scratch; the call fails before enqueuing work."""
    ctx = gpu_lib.context(0)
    seg, params = _case(ctx, 1 << 20, 2, 4200)
    out = _outputs(2, 16)
    with pytest.raises(ci.CiError) as e:
        ctx.find_triggers_noalloc(seg, params, 6.0, 1, *out)
    assert e.value.code == ci.EINVAL and "scratch" in str(e.value)
    seg.close()
    ctx.close()
