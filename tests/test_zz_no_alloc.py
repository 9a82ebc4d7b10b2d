"""st_bounding_boxes_noalloc (the allocation-free entry point) against
st_bounding_boxes through the C ABI: two calls in a row, the second with a
smaller input, device and host outputs, bit for bit; and the size limit."""
import numpy as np
import pytest

from gpu_helpers import fields, tracker, workload

pytestmark = pytest.mark.gpu


def test_bounding_boxes_noalloc_matches_bounding_boxes():
    import torch
    import paper_2603_26691_amd as pkg
    from paper_2603_26691_amd import _native as N
    w = workload("tg32", P=50_000, noise=0.1)
    t = tracker(w, "fp32_local")
    x, up, d = w.particles()
    t.inject(x, up, d)
    Udev, _ = fields(w, "fp32_local")
    for _ in range(3):
        t.step(Udev, w.dt)
    # first call: every particle in 1000 partitions of 50; second call: a
    # smaller input, 37 partitions of 211 ids from id 1234 (the last ones
    # partly empty), so stale bounds of the first call would show
    for id0, per_part, nparts in [(0, 50, 1000), (1234, 211, 37)]:
        want = t.bounding_boxes(id0, per_part, nparts).cpu().numpy()
        got_dev = t.bounding_boxes_noalloc(id0, per_part, nparts).cpu().numpy()
        got_host = t.bounding_boxes_noalloc(id0, per_part, nparts, out=np.empty((nparts, 6)))
        assert np.array_equal(got_dev, want), (id0, per_part, nparts)
        assert np.array_equal(got_host, want), (id0, per_part, nparts)
        assert np.isfinite(want[: (w.P - id0) // per_part]).all()
    with pytest.raises(N.STError) as e:
        t.bounding_boxes_noalloc(0, 1, N.NOALLOC_MAX_PARTS + 1,
                                 out=torch.empty((N.NOALLOC_MAX_PARTS + 1, 6),
                                                 dtype=torch.float64, device="cuda"))
    assert e.value.status == N.ST_ERR_INVALID
    assert "exceeds the maximum" in str(e.value)
    t.close()
