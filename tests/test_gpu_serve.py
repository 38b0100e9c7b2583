"""Serving runtime on the GPU: frames of mixed shapes submitted while others
are in flight must come back bit-identical to the oracle's map of the same
frame (each pool frame's oracle map is computed once), with slots
overlapping on the device and the admission budget respected.  The pool
holds the four shapes of the served workload (640x480 Dmax 64, 1436x992
Dmax 145, 1920x1080 Dmax 256, 2872x1984 Dmax 290) and three smaller ones,
one of them odd-sized."""

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2212_00488_amd import Stereo
from paper_2212_00488_amd.serve import Server, replay
from paper_2212_00488_amd.synth import make_pair

pytestmark = pytest.mark.gpu

SHAPES = [(160, 120, 16), (320, 240, 32), (641, 479, 64), (640, 480, 64), (1436, 992, 145),
          (1920, 1080, 256), (2872, 1984, 290)]


@pytest.fixture(scope="module")
def pool():
    frames, ref = {}, {}
    for k, (W, H, dmax) in enumerate(SHAPES):
        print(f"[serve pool] oracle maps of {W}x{H} Dmax={dmax}", flush=True)
        frames[k] = [make_pair(W, H, dmax, segments=6, seed=10000 + 10 * k + j) for j in range(2)]
        for j, p in enumerate(frames[k]):
            ref[(k, j)] = oracle.disparity(p.left, p.right, dmax)["out"]
    sys.stdout.flush()
    return frames, ref


def make_stream(n, seed, rate):
    rng = np.random.default_rng(seed)
    kinds = rng.integers(0, len(SHAPES), size=n)
    which = rng.integers(0, 2, size=n)
    if rate is None:
        arrivals = np.zeros(n)
    else:
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return kinds, which, arrivals


def run_stream(pool, n, seed, rate, slots, budget=0, pinned=False, max_batch=8, kinds_from=None):
    frames, ref = pool
    kinds, which, arrivals = make_stream(n, seed, rate)
    if kinds_from is not None:
        kinds = np.asarray(kinds_from)[kinds % len(kinds_from)]
    srv = Server(0, slots=slots, mem_budget=budget, max_batch=max_batch)
    try:
        fr = [(frames[k][j].left, frames[k][j].right) for k, j in zip(kinds, which)]
        dm = [SHAPES[k][2] for k in kinds]
        outs = None
        if pinned:  # page-locked outputs take the maps by DMA, without staging
            outs = [torch.empty(f[0].shape[:2], dtype=torch.int16).pin_memory().numpy() for f in fr]
        rep, outs = replay(srv, fr, arrivals, dm, outs=outs)
    finally:
        srv.close()
    for i, (k, j) in enumerate(zip(kinds, which)):
        assert np.array_equal(outs[i], ref[(k, j)]), (i, SHAPES[k])
    return rep, kinds


def volume(k):
    W, H, dmax = SHAPES[k]
    return ((W + 1) // 2) * ((H + 1) // 2) * ((dmax + 1) // 2) * 4


def test_burst_of_mixed_frames_matches_alone(pool):
    rep, kinds = run_stream(pool, 48, seed=600, rate=None, slots=4)
    res = rep.results
    # the slots really ran frames concurrently
    overlaps = 0
    for a in res:
        for b in res:
            if a["tag"] < b["tag"] and a["t_admit_ms"] < b["t_done_ms"] and b["t_admit_ms"] < a["t_done_ms"]:
                overlaps += 1
    assert overlaps > 0
    assert len({r["slot"] for r in res}) == 4
    assert np.all(rep.latency_ms > 0)


def test_poisson_stream_single_slot_matches_alone(pool):
    rep, _ = run_stream(pool, 24, seed=601, rate=400.0, slots=1, max_batch=1)
    assert {r["slot"] for r in rep.results} == {0}
    # one slot: frames run one after the other in submission order
    res = sorted(rep.results, key=lambda r: r["t_admit_ms"])
    assert [r["tag"] for r in res] == sorted(r["tag"] for r in res)


def test_admission_budget_bounds_frames_in_flight(pool):
    budget = volume(4) + volume(0)  # a paper-sized frame and one small frame
    rep, kinds = run_stream(pool, 40, seed=602, rate=None, slots=4, budget=budget)
    res = rep.results
    for r in res:
        t = r["t_admit_ms"]
        live = [q for q in res if q["t_admit_ms"] <= t < q["t_done_ms"]]
        total = sum(volume(kinds[q["tag"]]) for q in live)
        assert total <= budget or len(live) == 1, (t, total, budget)


def test_page_locked_outputs_match_alone(pool):
    rep, _ = run_stream(pool, 32, seed=603, rate=None, slots=4, pinned=True)
    assert len({r["slot"] for r in rep.results}) > 1


def test_served_maps_equal_stereo_disparity(pool):
    """The same frames computed alone by stereo_disparity equal the oracle
    too: alone and in the mix give one result."""
    frames, ref = pool
    ctx = Stereo(0)
    try:
        for k, (W, H, dmax) in enumerate(SHAPES):
            p = frames[k][0]
            out = ctx.disparity(torch.from_numpy(p.left).cuda(), torch.from_numpy(p.right).cuda(),
                                dmax)
            assert np.array_equal(out.cpu().numpy(), ref[(k, 0)]), SHAPES[k]
    finally:
        ctx.close()


def test_same_shape_frames_are_batched(pool):
    """A burst of frames of two shapes on two slots: pending frames of the
    head's shape join its launch (1, 2, 4 or 8 frames), every map still
    equals the oracle's, and the frames of one launch share shape, slot and
    admission time."""
    rep, kinds = run_stream(pool, 40, seed=604, rate=None, slots=2, kinds_from=[1, 4])
    res = rep.results
    sizes = {r["batch"] for r in res}
    assert sizes <= {1, 2, 4, 8} and max(sizes) > 1, sizes
    launches = {}
    for r in res:
        launches.setdefault((r["slot"], r["t_admit_ms"]), []).append(r)
    for group in launches.values():
        assert len(group) == group[0]["batch"]
        assert len({SHAPES[kinds[r["tag"]]] for r in group}) == 1


def test_budget_holds_with_batches(pool):
    """Batches count every frame against the budget: at most two paper-sized
    frames in flight, whatever the batching."""
    budget = 2 * volume(4)
    rep, kinds = run_stream(pool, 24, seed=605, rate=None, slots=4, budget=budget,
                            kinds_from=[4])
    res = rep.results
    assert max(r["batch"] for r in res) <= 2
    for r in res:
        t = r["t_admit_ms"]
        live = [q for q in res if q["t_admit_ms"] <= t < q["t_done_ms"]]
        assert sum(volume(kinds[q["tag"]]) for q in live) <= budget
