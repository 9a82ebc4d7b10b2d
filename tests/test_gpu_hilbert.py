"""Hilbert-segment placement, injection and partition bounding boxes on the
GPU (paper Sec. 2.2) against the FP64 oracle, through the C ABI.

Placement is integer work plus one rounding per coordinate done the same way
on both sides, so positions must be bit-exact; bounding boxes are minima and
maxima of the positions st_get_particles returns, so they must be bit-exact
against the oracle's boxes of those positions.
"""
import math

import numpy as np
import pytest

from gpu_helpers import fields, oracle_mesh, state, tracker, workload
from oracle.oracle import load as load_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return load_oracle()


def _tracker(n=(32, 32, 32), L=(0.1, 0.1, 0.1), capacity=200000, form="fp64"):
    w = workload("tg32", n=n, L=L, P=capacity)
    return tracker(w, form, capacity=capacity), w


@pytest.mark.parametrize("order,nseg,per_seg", [(1, 3, 5), (3, 37, 50), (5, 1000, 7),
                                                (7, 4096, 25)])
def test_positions_match_oracle(orc, order, nseg, per_seg):
    import torch
    t, w = _tracker(L=(0.1, 0.06, 0.05))
    rng = np.random.default_rng(order)
    u = rng.random((nseg * per_seg, 3))
    want = orc.hilbert_positions(order, nseg, 0, nseg, per_seg, w.L, u)
    got = t.hilbert_positions(order, nseg, 0, nseg, per_seg, torch.from_numpy(u).cuda())
    assert np.array_equal(got.cpu().numpy(), want), "device placement bit-exact"
    got_h = t.hilbert_positions(order, nseg, 0, nseg, per_seg, u)
    assert np.array_equal(got_h, want), "host placement bit-exact"
    # a range of segments alone gives the same particles
    a, b = nseg // 3, nseg // 3 + max(1, nseg // 4)
    part = t.hilbert_positions(order, nseg, a, b, per_seg, u[a * per_seg:b * per_seg])
    assert np.array_equal(part, want[a * per_seg:b * per_seg])
    t.close()


def test_positions_reject_bad_arguments():
    import paper_2603_26691_amd._native as N
    t, _ = _tracker()
    u = np.zeros((64, 3))
    for args in [(0, 1, 0, 1, 8), (11, 1, 0, 1, 8), (1, 9, 0, 1, 8), (2, 4, 3, 2, 2),
                 (2, 4, 0, 5, 2), (2, 4, 0, 1, 0)]:
        with pytest.raises(N.STError):
            t.hilbert_positions(*args, u[:max(0, (args[3] - args[2]) * args[4])])
    # an empty range is no error
    assert t.hilbert_positions(2, 4, 1, 1, 5, u[:0]).shape == (0, 3)
    t.close()


@pytest.mark.parametrize("form", ["fp64", "fp32_local"])
def test_inject_hilbert(orc, form):
    import torch
    t, w = _tracker(form=form)
    order, nseg, per_seg = 5, 64, 300
    rng = np.random.default_rng(5)
    n = nseg * per_seg
    u = rng.random((n, 3))
    up = rng.normal(0, 0.2, (n, 3))
    d = np.exp(rng.normal(math.log(20e-6), 0.4, n))
    # two calls: host arrays for the first segments, device arrays for the rest
    t.inject_hilbert(order, nseg, 0, 20, per_seg, u[:20 * per_seg], up[:20 * per_seg],
                     d[:20 * per_seg])
    t.inject_hilbert(order, nseg, 20, nseg, per_seg, *(torch.from_numpy(a[20 * per_seg:]).cuda()
                                                       for a in (u, up, d)))
    assert t.count() == n
    s = state(t)
    want = orc.hilbert_positions(order, nseg, 0, nseg, per_seg, w.L, u)
    assert np.array_equal(s["id"], np.arange(n)), "ids follow the segments in order"
    # positions come back through the chunk-local offsets of the store
    tol = 1e-15 * max(w.L) if form == "fp64" else 1e-6 * w.h.max()
    assert np.abs(s["x"] - want).max() <= tol
    cells = orc.cells(oracle_mesh(w), want)
    q = want / w.h
    near = (np.abs(q - np.round(q)) < 1e-6).any(axis=1)
    assert np.array_equal(s["cell"][~near], cells[~near]), "cells bit-exact away from faces"
    vtol = 0.0 if form == "fp64" else 1e-6
    assert np.abs(s["up"] - up).max() <= vtol
    t.close()


@pytest.mark.parametrize("form", ["fp64", "fp32_local", "fp32"])
def test_bounding_boxes_match_oracle(orc, form):
    import torch
    t, w = _tracker(form=form)
    order, nseg, per_seg = 4, 40, 500
    rng = np.random.default_rng(6)
    n = nseg * per_seg
    t.inject_hilbert(order, nseg, 0, nseg, per_seg, rng.random((n, 3)), np.zeros((n, 3)),
                     np.exp(rng.normal(math.log(20e-6), 0.4, n)))
    Udev, _ = fields(w, form)
    for _ in range(3):
        t.step(Udev, 2e-3)    # long steps: particles mix between partitions
    s = state(t)
    for id0, per_part, nparts in [(0, per_seg, nseg), (7, 333, 70), (0, n, 1), (0, 1, 50)]:
        got = t.bounding_boxes(id0, per_part, nparts).cpu().numpy()
        want = orc.bounding_boxes(s["x"], s["id"], id0, per_part, nparts)
        assert np.array_equal(got, want), (form, id0, per_part, nparts)
    t.close()


def test_hilbert_partitions_are_compact(orc):
    # the purpose of the Hilbert initialisation: compact partitions with small
    # bounding boxes; compare with the same particles partitioned at random
    t, w = _tracker()
    order, nseg, per_seg = 5, 64, 500
    rng = np.random.default_rng(7)
    n = nseg * per_seg
    t.inject_hilbert(order, nseg, 0, nseg, per_seg, rng.random((n, 3)), np.zeros((n, 3)),
                     np.full(n, 20e-6))
    box = t.bounding_boxes(0, per_seg, nseg).cpu().numpy()
    vol = np.prod(box[:, 3:] - box[:, :3], axis=1)
    dom = np.prod(w.L)
    # a segment holds 1/64 of the voxels: its box is a few times that volume
    assert vol.mean() < 0.1 * dom, vol.mean() / dom
    s = state(t)
    perm = rng.permutation(n)
    rbox = orc.bounding_boxes(s["x"], perm, 0, per_seg, nseg)
    rvol = np.prod(rbox[:, 3:] - rbox[:, :3], axis=1)
    assert rvol.mean() > 0.8 * dom
    t.close()
