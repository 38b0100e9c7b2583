"""stereo_disparity_noalloc (fixed per-device scratch, no allocation by the
library) against stereo_disparity, through the C interface (needs an MI355X).

Both entry points run the same kernels over the same integer arithmetic, so
maps must be identical.  The fixed array keeps the previous call's contents:
calls of different shapes in a row check that each call re-initialises what
must start at zero."""

import ctypes
import sys

import numpy as np
import pytest

from paper_2212_00488_amd.synth import make_pair, workload_pairs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sm():
    import paper_2212_00488_amd as sm
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sm.lib()
    return sm


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def call_noalloc(sm, ctx, lt, rt, dmax, out, params=None):
    """The C entry point itself (ctypes), on the current stream."""
    H, W, _ = lt.shape
    rc = sm.lib().stereo_disparity_noalloc(
        ctx._h, lt.data_ptr(), rt.data_ptr(), W, H, dmax,
        ctypes.byref(params) if params is not None else None, out.data_ptr(),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc


def test_noalloc_matches_stereo_disparity_on_calls_in_a_row(sm):
    ctx = sm.Stereo(0)
    big = workload_pairs("paper_1436x992_d145")[0]
    small = workload_pairs("small_320x240_d32")[0]
    cases = [("paper 1436x992 Dmax 145", big, 145), ("small 320x240 Dmax 32", small, 32),
             ("paper 1436x992 Dmax 145 again", big, 145)]
    outs = []
    # two (then three) calls in a row, the second on a smaller input, each into
    # a preallocated map; the fixed array holds the previous call's planes
    for label, pair, dmax in cases:
        say(f"[noalloc] {label}")
        lt, rt = dev(pair.left), dev(pair.right)
        out = torch.full(lt.shape[:2], -7, dtype=torch.int16, device="cuda")
        rc = call_noalloc(sm, ctx, lt, rt, dmax, out)
        assert rc == 0, ctx.last_error()
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
    for (label, pair, dmax), got in zip(cases, outs):
        ref = ctx.disparity(dev(pair.left), dev(pair.right), dmax)
        torch.cuda.synchronize()
        exp = ref.cpu().numpy()
        bad = int((got != exp).sum())
        assert bad == 0, f"{label}: {bad} of {exp.size} pixels differ from stereo_disparity"
    ctx.close()


def test_noalloc_makes_no_device_allocation_and_refuses_oversize(sm):
    ctx = sm.Stereo(0)
    pair = make_pair(640, 480, 64, segments=6, seed=41)
    lt, rt = dev(pair.left), dev(pair.right)
    out = torch.empty((480, 640), dtype=torch.int16, device="cuda")
    torch.cuda.synchronize()
    say("[noalloc] 640x480 Dmax 64, free device memory before and after")
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        assert call_noalloc(sm, ctx, lt, rt, 64, out) == 0, ctx.last_error()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    # the cached-plan path makes a plan of about 13 MB for this shape
    ref = ctx.disparity(lt, rt, 64)
    torch.cuda.synchronize()
    free2, _ = torch.cuda.mem_get_info()
    assert free0 - free1 < 4 << 20, (free0, free1)
    assert free1 - free2 >= 8 << 20, (free1, free2)
    assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy())
    # a shape whose planes exceed the fixed array is refused before any launch
    say("[noalloc] 2872x1984 Dmax 290 refused")
    big_l = torch.zeros((1984, 2872, 3), dtype=torch.uint8, device="cuda")
    big_o = torch.zeros((1984, 2872), dtype=torch.int16, device="cuda")
    rc = call_noalloc(sm, ctx, big_l, big_l, 290, big_o)
    assert rc == sm.EINVAL and "fixed array" in ctx.last_error()
    # flags that need allocations are refused
    p = sm.default_params(flags=sm.F_KEEP_INTERMEDIATES)
    assert call_noalloc(sm, ctx, lt, rt, 64, out, p) == sm.EINVAL
    # the context still works after the refusals
    assert call_noalloc(sm, ctx, lt, rt, 64, out) == 0, ctx.last_error()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy())
    ctx.close()


def test_noalloc_under_graph_capture(sm):
    """The caller this entry point is for: code under graph capture.  The call
    is captured in a HIP graph and replayed three times; between replays an
    eager no-allocation call of another shape overwrites the fixed array, and
    each replay (which re-initialises it) still gives stereo_disparity's map."""
    ctx = sm.Stereo(0)
    pair = make_pair(320, 240, 32, segments=6, seed=43)
    other = make_pair(200, 120, 48, segments=4, seed=44)
    lt, rt = dev(pair.left), dev(pair.right)
    ol, orr = dev(other.left), dev(other.right)
    out = torch.empty((240, 320), dtype=torch.int16, device="cuda")
    oout = torch.empty((120, 200), dtype=torch.int16, device="cuda")
    ref = ctx.disparity(lt, rt, 32).cpu().numpy()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("[noalloc] capture 320x240 Dmax 32")
    with torch.cuda.graph(g, stream=s):
        rc = call_noalloc(sm, ctx, lt, rt, 32, out)
    assert rc == 0, ctx.last_error()
    for k in range(3):
        out.fill_(-7)
        assert call_noalloc(sm, ctx, ol, orr, 48, oout) == 0, ctx.last_error()
        torch.cuda.synchronize()
        say(f"[noalloc] replay {k}")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), k
    del g
    torch.cuda.synchronize()
    ctx.close()
