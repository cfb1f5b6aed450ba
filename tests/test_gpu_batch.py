"""Batched persistent launch: many 2-D pairs of mixed size, window, step and
border in one launch (plus separate launches for pairs without a compiled
variant), captured in a hipGraph and replayed.

Every pair is compared with the CPU oracle (bit-exact for integer input,
|dc| <= 2^-24 for float input); integer batches must equal single-pair
launches bit for bit; graph replays (with eager work in between), repeated
launches and alternating plans must equal the eager result every time.
"""
import numpy as np
import pytest

import oracle
from gpu_util import F32_TOL, say, to_dev
from workloads import batched_pairs, random_pair

pytestmark = pytest.mark.gpu


def _mixed_pairs(dtype, seed=0):
    rng = np.random.default_rng(seed)
    pairs = []
    specs = [((37, 300), 5, 1, "clip"), ((130, 517), 7, 1, "fill"), ((64, 256), 9, 1, "valid"),
             ((90, 1001), 15, 1, "clip"), ((33, 65), 3, (2, 1), "clip"), ((200, 128), 7, 1, "clip"),
             ((51, 77), 4, 1, "clip"),      # even window: separate launch
             ((40, 90), 11, 1, "fill"),     # width without a batch variant
             ((300, 640), 7, (1, 2), "fill")]
    for i, (shape, k, step, border) in enumerate(specs):
        x, y = random_pair(shape, dtype, seed=seed * 100 + i)
        pairs.append(dict(x=x, y=y, window=k, step=step, border=border))
    return pairs


def _run_batch(pairs, accum="default", params=None):
    import torch
    import paper_1807_06507_amd as swc
    dev_pairs = [dict(x=to_dev(p["x"]), y=to_dev(p["y"]), window=p["window"], step=p["step"],
                      border=p["border"]) for p in pairs]
    plan = swc.BatchPlan(dev_pairs, accum=accum, params=params, return_flags=True)
    plan.launch()
    torch.cuda.synchronize()
    outs = [o.cpu().numpy() for o in plan.outputs]
    fls = [f.cpu().numpy() for f in plan.flags]
    return plan, dev_pairs, outs, fls


def _check_pair(p, c, fl):
    o32, o64, ofl = oracle.corr(p["x"], p["y"], p["window"], p["step"], p["border"])
    assert np.array_equal(fl, ofl)
    ok = ofl == 0
    assert np.all(c[~ok] == np.float32(-2.0))
    if p["x"].dtype.kind == "u":
        assert np.array_equal(c[ok].view(np.uint32), o32[ok].view(np.uint32))
        return 0.0
    d = float(np.max(np.abs(c[ok].astype(np.float64) - o64[ok]))) if ok.any() else 0.0
    assert d <= F32_TOL, d
    return d


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_batch_matches_oracle(dtype):
    pairs = _mixed_pairs(dtype, seed=1)
    plan, _, outs, fls = _run_batch(pairs)
    say(f"[batch] {dtype}: {len(pairs)} pairs, {plan.items} work items")
    for p, c, fl in zip(pairs, outs, fls):
        _check_pair(p, c, fl)


@pytest.mark.parametrize("dtype", ["u16", "u8"])
def test_batch_equals_single_launches_integer(dtype):
    import torch
    import paper_1807_06507_amd as swc
    pairs = _mixed_pairs(dtype, seed=2)
    _, dev_pairs, outs, fls = _run_batch(pairs)
    for p, dp, c, fl in zip(pairs, dev_pairs, outs, fls):
        c1, f1 = swc.corr(dp["x"], dp["y"], p["window"], p["step"], p["border"],
                          return_flags=True)
        torch.cuda.synchronize()
        assert np.array_equal(f1.cpu().numpy(), fl)
        assert np.array_equal(c1.cpu().numpy().view(np.uint32), c.view(np.uint32))


@pytest.mark.parametrize("params", [(4, 8, 1), (4, 24, 2), (4, 64, 4)])
def test_batch_launch_params(params):
    pairs = _mixed_pairs("f32", seed=3)
    _, _, outs, fls = _run_batch(pairs, params=params)
    for p, c, fl in zip(pairs, outs, fls):
        _check_pair(p, c, fl)


def test_batch_graph_replays():
    """Capture one batched launch in a graph, replay it several times with
    eager work and synchronisations in between; every replay must equal the
    eager result (inputs are refreshed before each replay)."""
    import torch
    import paper_1807_06507_amd as swc
    pairs = _mixed_pairs("f32", seed=4)
    plan, dev_pairs, outs, fls = _run_batch(pairs)
    g = plan.capture_graph()
    torch.cuda.synchronize()
    for rep in range(4):
        for o in plan.outputs:
            o.fill_(123.0)
        for f in plan.flags:
            f.fill_(255)
        # unrelated eager work on the same device
        t = torch.randn(1 << 20, device="cuda")
        (t * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        for c, fl, o, f in zip(outs, fls, plan.outputs, plan.flags):
            assert np.array_equal(o.cpu().numpy().view(np.uint32), c.view(np.uint32)), rep
            assert np.array_equal(f.cpu().numpy(), fl), rep


def test_batch_relaunch_and_interleaved_plans():
    """The persistent waves take work items from the plan's device counters,
    which every launch leaves at zero: two plans launched alternately on one
    stream, each several times back to back without synchronisation, must
    give their first results every time."""
    import torch
    import paper_1807_06507_amd as swc
    pa = _mixed_pairs("u16", seed=7)
    pb = _mixed_pairs("u16", seed=8)[:5]
    plan_a, _, outs_a, fls_a = _run_batch(pa)
    plan_b, _, outs_b, fls_b = _run_batch(pb)
    for rep in range(3):
        for o in plan_a.outputs + plan_b.outputs:
            o.fill_(7.0)
        for _ in range(3):
            plan_a.launch()
            plan_b.launch()
        torch.cuda.synchronize()
        for outs, fls, plan in ((outs_a, fls_a, plan_a), (outs_b, fls_b, plan_b)):
            for c, fl, o, f in zip(outs, fls, plan.outputs, plan.flags):
                assert np.array_equal(o.cpu().numpy().view(np.uint32), c.view(np.uint32)), rep
                assert np.array_equal(f.cpu().numpy(), fl), rep
    for p, c, fl in zip(pa, outs_a, fls_a):
        _check_pair(p, c, fl)


def test_batch_config_scaled():
    """The batched configuration's generator and window mix (64 pairs, k from
    {5, 7, 9, 15}, CLIP) at 1/8 of each side: every pair against the oracle."""
    import torch
    pairs = [dict(x=x, y=y, window=k, step=1, border="clip")
             for x, y, k in batched_pairs(64, seed=1, scale=0.125)]
    _, _, outs, fls = _run_batch(pairs)
    dmax = 0.0
    for p, c, fl in zip(pairs, outs, fls):
        dmax = max(dmax, _check_pair(p, c, fl))
    say(f"[batch] scaled c3: max|dc| = {dmax:.3e}")


def test_batch_config_full_sampled():
    """The batched configuration at full size (64 pairs, 229.7 Mpx, k from
    {5, 7, 9, 15}, CLIP) in the launch configuration the benchmark times:
    2000 sampled outputs of every pair plus its first row, one by one
    against the oracle."""
    import torch
    import paper_1807_06507_amd as swc
    pairs = batched_pairs(64, seed=1)
    dev = [dict(x=to_dev(x), y=to_dev(y), window=k, step=1, border="clip") for x, y, k in pairs]
    plan = swc.BatchPlan(dev, return_flags=True)
    plan.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    dmax = 0.0
    for (x, y, k), o, f in zip(pairs, plan.outputs, plan.flags):
        c, fl = o.cpu().numpy(), f.cpu().numpy()
        idx = np.unique(np.concatenate([rng.integers(0, x.size, 2000), np.arange(x.shape[1])]))
        o32, o64, ofl = oracle.corr(x, y, (k, k), 1, "clip", indices=idx)
        cs, fs = c.ravel()[idx], fl.ravel()[idx]
        assert np.array_equal(fs, ofl)
        ok = ofl == 0
        assert np.all(cs[~ok] == np.float32(-2.0))
        if ok.any():
            dmax = max(dmax, float(np.max(np.abs(cs[ok].astype(np.float64) - o64[ok]))))
    assert dmax <= F32_TOL, dmax
    say(f"[batch] full c3 (sampled): max|dc| = {dmax:.3e}, items {plan.items}")
    plan.close()
