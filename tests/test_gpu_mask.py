"""GPU parity of the application step (cloud mask and detection filter)
against the oracle's definition on the oracle's map: bit-exact masks.
Cases: paper-shaped u16 data with a cloud region, with and without the flag
map, ragged and misaligned lengths, detections outside the map."""
import numpy as np
import pytest

import oracle
from gpu_util import say, to_dev
from workloads import paper_shaped_u16

pytestmark = pytest.mark.gpu


def _map(shape, seed):
    import torch
    import paper_1807_06507_amd as swc
    x, y = paper_shaped_u16(shape, seed=seed)
    c, fl = swc.corr(to_dev(x), to_dev(y), (7, 7), 1, "fill", return_flags=True)
    torch.cuda.synchronize()
    o32, _, ofl = oracle.corr(x, y, (7, 7), 1, "fill")
    assert np.array_equal(c.cpu().numpy().view(np.uint32), o32.view(np.uint32))
    return c, fl, o32, ofl


@pytest.mark.parametrize("tau", [0.0, 0.5, 0.8])
def test_cloud_mask_matches_definition(tau):
    import torch
    import paper_1807_06507_amd as swc
    c, fl, o32, ofl = _map((600, 800), seed=7)
    want = oracle.cloud_mask(o32, ofl, tau)
    say(f"[mask] tau={tau} cloud fraction {want.mean():.3f}")
    got = swc.cloud_mask(c, fl, tau).cpu().numpy()
    assert np.array_equal(got, want)
    got2 = swc.cloud_mask(c, None, tau).cpu().numpy()        # validity from the invalid value
    assert np.array_equal(got2, want)
    # ragged and misaligned: a flat view starting one element in
    cf, ff = c.reshape(-1)[1:], fl.reshape(-1)[1:]
    n = cf.numel() - 3
    got3 = swc.cloud_mask(cf[:n], ff[:n], tau)
    torch.cuda.synchronize()
    assert np.array_equal(got3.cpu().numpy(), want.reshape(-1)[1:1 + n])


def test_filter_detections():
    import torch
    import paper_1807_06507_amd as swc
    c, fl, o32, ofl = _map((600, 800), seed=8)
    mask = oracle.cloud_mask(o32, ofl, 0.6).reshape(-1)
    rng = np.random.default_rng(3)
    idx = rng.integers(-50, c.numel() + 50, size=5003).astype(np.int64)
    want = np.where((idx < 0) | (idx >= c.numel()), 2,
                    1 - mask[np.clip(idx, 0, c.numel() - 1)]).astype(np.uint8)
    got = swc.filter_detections(c, to_dev(idx), fl, 0.6).cpu().numpy()
    assert np.array_equal(got, want)
    assert set(np.unique(got)) <= {0, 1, 2}
    torch.cuda.synchronize()


def test_mask_empty_inputs():
    import torch
    import paper_1807_06507_amd as swc
    c = torch.empty((0,), dtype=torch.float32, device="cuda")
    assert swc.cloud_mask(c).numel() == 0
    k = swc.filter_detections(torch.zeros(10, device="cuda"),
                              torch.empty((0,), dtype=torch.int64, device="cuda"))
    assert k.numel() == 0
