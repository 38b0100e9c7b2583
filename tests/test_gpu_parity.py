"""Parity of the HIP path with the CPU oracle, element by element, through the
C interface (needs an MI355X).

Every comparison is exact: the path is integer arithmetic end to end (the
cost tables are built from exp() on the host by each side independently and
compared too)."""

import sys

import numpy as np
import pytest

import oracle
from paper_2212_00488_amd.synth import (extremes_pair, make_pair, textured_shift_pair,
                                        workload_pairs)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HALF_KEYS = ("half_l", "half_r", "census_l", "census_r", "arms_l", "arms_r", "disp_l", "disp_r",
             "gcp", "median", "filled")
MIN_KEYS = (("mincost_l", "min_l"), ("mincost_r", "min_r"))


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


@pytest.fixture(scope="module")
def ctx(sm):
    c = sm.Stereo(0)
    yield c
    c.close()


def keep_params(sm, **kw):
    return sm.default_params(flags=sm.F_KEEP_INTERMEDIATES, **kw)


def oracle_params(p):
    return oracle.Params(lambda_ad=float(np.float32(p.lambda_ad)),
                         lambda_mc=float(np.float32(p.lambda_mc)), cost_scale=p.cost_scale,
                         color_delta=p.color_delta, arm_x=p.arm_x, arm_y=p.arm_y,
                         fill_T=p.fill_T, arm_x_r=p.arm_x_r, fill_mode=p.fill_mode,
                         full_res=bool(p.flags & 4))


def run_gpu(ctx, left, right, dmax, params):
    lt = torch.from_numpy(np.ascontiguousarray(left)).cuda()
    rt = torch.from_numpy(np.ascontiguousarray(right)).cuda()
    out = ctx.disparity(lt, rt, dmax, params)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def assert_same(name, got, exp):
    if not np.array_equal(got, exp):
        diff = np.argwhere(got != exp)
        i = tuple(diff[0])
        raise AssertionError(f"{name}: {len(diff)} of {exp.size} differ; first at {i}: "
                             f"gpu {got[i]} oracle {exp[i]}")


def full_parity(sm, ctx, left, right, dmax, params=None, label=""):
    p = params if params is not None else keep_params(sm)
    say(f"[parity] {label} {left.shape[1]}x{left.shape[0]} Dmax={dmax}")
    got = run_gpu(ctx, left, right, dmax, p)
    exp = oracle.disparity(left, right, dmax, oracle_params(p))
    for k in HALF_KEYS:
        assert_same(k, ctx.intermediate(k), exp[k])
    for gk, ok in MIN_KEYS:
        assert_same(gk, ctx.intermediate(gk), exp[ok])
    assert_same("out", got, exp["out"])
    return exp


def test_cost_tables_match_oracle(sm, ctx):
    pair = make_pair(32, 16, 8, segments=2, seed=1)
    run_gpu(ctx, pair.left, pair.right, 8, keep_params(sm))
    lut = ctx.intermediate("lut")
    ad, mc = oracle.lut(oracle.Params())
    assert np.array_equal(lut[:256], ad) and np.array_equal(lut[256:], mc)


def test_small_workload_all_intermediates(sm, ctx):
    """320x240, Dmax 32 (16 at half resolution): every plane bit-exact."""
    pair = workload_pairs("small_320x240_d32")[0]
    full_parity(sm, ctx, pair.left, pair.right, 32, label="small")


@pytest.mark.parametrize("d", [0, 1, 7, 15])
def test_per_disparity_planes(sm, ctx, d):
    """C^L, C^R (Eq. 3-6), CA_x (Eq. 7) and CA (Eq. 8) planes at one d."""
    pair = workload_pairs("small_320x240_d32")[0]
    p = keep_params(sm)
    run_gpu(ctx, pair.left, pair.right, 32, p)
    q = oracle_params(p)
    hl = oracle.downscale(oracle.gray(pair.left))
    hr = oracle.downscale(oracle.gray(pair.right))
    cl, cr = oracle.census(hl), oracle.census(hr)
    al, ar = oracle.arms(hl, q), oracle.arms(hr, q)
    ad, mc = oracle.lut(q)
    cmax = int(ad[255]) + int(mc[6])
    cL = oracle.cost_left(hl, hr, cl, cr, d, q)
    cR = oracle.cost_right_from_left(cL, d, cmax)
    assert_same("cost_l", ctx.intermediate("cost_l_d", d), cL)
    assert_same("cax_l", ctx.intermediate("cax_l_d", d), oracle.agg_x(cL, al))
    assert_same("ca_l", ctx.intermediate("ca_l_d", d), oracle.agg_y(oracle.agg_x(cL, al), al))
    assert_same("cost_r", ctx.intermediate("cost_r_d", d), cR)
    assert_same("cax_r", ctx.intermediate("cax_r_d", d), oracle.agg_x(cR, ar))
    assert_same("ca_r", ctx.intermediate("ca_r_d", d), oracle.agg_y(oracle.agg_x(cR, ar), ar))


@pytest.mark.parametrize("d", [0, 3, 12])
def test_extreme_brightness_differences(sm, ctx, d):
    """Black and white squares: half-res differences of exactly -255 and +255
    (both ends of the LUT_AD index, Eq. 4) occur at every d; the cost and
    window-sum planes and the whole map stay bit-exact."""
    left, right = extremes_pair(240, 160, block=8, seed=21)
    p = keep_params(sm)
    got = run_gpu(ctx, left, right, 32, p)
    q = oracle_params(p)
    hl = oracle.downscale(oracle.gray(left))
    hr = oracle.downscale(oracle.gray(right))
    assert (hl.astype(int)[:, d:] - hr.astype(int)[:, : hl.shape[1] - d] == 255).any()
    assert (hl.astype(int)[:, d:] - hr.astype(int)[:, : hl.shape[1] - d] == -255).any()
    cl, cr = oracle.census(hl), oracle.census(hr)
    al, ar = oracle.arms(hl, q), oracle.arms(hr, q)
    ad, mc = oracle.lut(q)
    cL = oracle.cost_left(hl, hr, cl, cr, d, q)
    cR = oracle.cost_right_from_left(cL, d, int(ad[255]) + int(mc[6]))
    assert_same("cost_l", ctx.intermediate("cost_l_d", d), cL)
    assert_same("cost_r", ctx.intermediate("cost_r_d", d), cR)
    assert_same("ca_l", ctx.intermediate("ca_l_d", d), oracle.agg_y(oracle.agg_x(cL, al), al))
    assert_same("ca_r", ctx.intermediate("ca_r_d", d), oracle.agg_y(oracle.agg_x(cR, ar), ar))
    exp = oracle.disparity(left, right, 32, q)
    assert_same("out", got, exp["out"])


@pytest.mark.parametrize("W,H,dmax,seed", [
    (37, 23, 10, 1), (3, 2, 1, 2), (2, 2, 2, 3), (131, 7, 20, 4), (65, 33, 64, 5),
    (129, 130, 40, 6), (1501, 12, 100, 7), (300, 200, 299, 8)])
def test_odd_and_ragged_sizes(sm, ctx, W, H, dmax, seed):
    """Odd widths/heights, strips with a ragged tail, D close to X, tiny images."""
    pair = make_pair(W, H, dmax, segments=3, seed=seed)
    full_parity(sm, ctx, pair.left, pair.right, dmax, label="ragged")


def test_tall_image_uses_row_bands(sm, ctx):
    """Y = 700 half-res rows exceeds one LDS plane: two row bands with halos."""
    pair = make_pair(200, 1400, 64, segments=5, seed=9)
    full_parity(sm, ctx, pair.left, pair.right, 64, label="bands")


@pytest.mark.parametrize("kw", [
    dict(arm_x=40, arm_y=5), dict(arm_x=0, arm_y=0), dict(arm_x=63, arm_y=12, color_delta=30),
    dict(fill_T=0, cost_scale=512, lambda_ad=0.5, lambda_mc=1.0),
    dict(color_delta=0), dict(arm_x=100, arm_y=20, cost_scale=64)])
def test_parameter_variants(sm, ctx, kw):
    pair = make_pair(150, 90, 30, segments=4, seed=10)
    full_parity(sm, ctx, pair.left, pair.right, 30, keep_params(sm, **kw), label=str(kw))


@pytest.mark.parametrize("W,H,dmax,full", [
    (8192, 40, 512, False),   # widest half-res row (4096 columns, 64 strips) and largest D (256)
    (40, 8192, 32, False),    # tallest: 4096 half-res rows in eight or more row bands
    (4096, 16, 64, True),     # widest full-resolution row
])
def test_maximum_sides(sm, ctx, W, H, dmax, full):
    """The largest sides the library accepts (STEREO_MAX_SIDE, or half of it
    at full resolution) and the largest Dmax, bit-exact against the oracle."""
    pair = make_pair(W, H, dmax, segments=6, seed=14)
    flags = sm.F_KEEP_INTERMEDIATES | (sm.F_FULL_RES if full else 0)
    p = sm.default_params(flags=flags, arm_x=41 if full else 21, arm_y=61 if full else 31)
    full_parity(sm, ctx, pair.left, pair.right, dmax, p, label=f"max {W}x{H}")


def test_largest_arms(sm, ctx):
    """Both arms at their cap of 127 (three 128-column sub-passes of the row
    pass; cost scale small enough for the 2^24 window-sum bound)."""
    pair = make_pair(600, 600, 30, segments=4, seed=15)
    p = keep_params(sm, arm_x=127, arm_y=127, cost_scale=128)
    full_parity(sm, ctx, pair.left, pair.right, 30, p, label="arms 127")


def test_paper_sized_workload_bit_exact(sm, ctx):
    """1436x992, Dmax 145 (718x496, D = 73 at half resolution), the shape the
    paper times; the launch configuration the benchmark uses."""
    pair = workload_pairs("paper_1436x992_d145")[0]
    full_parity(sm, ctx, pair.left, pair.right, 145, label="paper")


def test_largest_served_shape_bit_exact(sm, ctx):
    """2872x1984, Dmax 290 (1436x992, D = 145 at half resolution: three row
    bands, an 8-bit d field), the largest shape of the served workload."""
    pair = make_pair(2872, 1984, 290, segments=40, textureless=0.1, seed=10030)
    full_parity(sm, ctx, pair.left, pair.right, 290, label="served 2872x1984")


def test_batched_workload_bit_exact(sm, ctx):
    """8 x 1920x1080, Dmax 256 in one batched launch sequence; every pair's
    output equals the oracle's."""
    pairs = workload_pairs("batch8_1920x1080_d256")
    say("[parity] batch of 8 1920x1080 Dmax=256")
    lefts = [torch.from_numpy(p.left).cuda() for p in pairs]
    rights = [torch.from_numpy(p.right).cuda() for p in pairs]
    outs = ctx.disparity_batch(lefts, rights, 256, keep_params(sm))
    torch.cuda.synchronize()
    for i, p in enumerate(pairs):
        exp = oracle.disparity(p.left, p.right, 256)
        assert_same(f"pair {i}", outs[i].cpu().numpy(), exp["out"])
        if i == 0:
            for k in ("disp_l", "disp_r", "gcp", "filled"):
                assert_same(k, ctx.intermediate(k), exp[k])


@pytest.mark.parametrize("k", [0, 5])
def test_constant_shift_pair(sm, ctx, k):
    """R(x) = L(x + 2k) on noise: the minimum aggregate is 0 in the interior and
    the output equals 2k there (property at any size)."""
    W, H = 1436, 992
    left, right = textured_shift_pair(W, H, 2 * k, seed=40 + k)
    got = run_gpu(ctx, left, right, 145, keep_params(sm))
    X = W // 2
    lo, hi = k + 26, X - k - 26
    assert np.all(ctx.intermediate("mincost_l")[:, lo:hi] == 0)
    dl = ctx.intermediate("disp_l")
    assert np.all(dl[:, lo:hi] <= k) and np.mean(dl[:, lo:hi] == k) > 0.99
    assert np.mean(got[4:-4, 2 * lo + 4:2 * hi - 4] == 2 * k) > 0.98


def test_deterministic_and_batch_equals_single(sm, ctx):
    pairs = [make_pair(320, 240, 32, segments=6, seed=s) for s in (50, 51, 52)]
    lefts = [torch.from_numpy(p.left).cuda() for p in pairs]
    rights = [torch.from_numpy(p.right).cuda() for p in pairs]
    single = [ctx.disparity(l, r, 32).cpu().numpy() for l, r in zip(lefts, rights)]
    for _ in range(10):
        outs = ctx.disparity_batch(lefts, rights, 32)
        torch.cuda.synchronize()
        for a, b in zip(outs, single):
            assert np.array_equal(a.cpu().numpy(), b)
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s2):
        o2 = ctx.disparity(lefts[0], rights[0], 32, stream=s2)
    s2.synchronize()
    assert np.array_equal(o2.cpu().numpy(), single[0])


def test_ten_runs_bit_identical_at_paper_size(sm, ctx):
    """1436x992, Dmax 145: ten frames in flight on two streams at once, then
    ten one after another on the launch stream, all give the bits of the first
    frame (a race or an order-dependent reduction would show as a mismatch;
    the first frame itself is checked against the oracle elsewhere)."""
    say("case: 20 frames of 1436x992 Dmax 145, two streams then one")
    pair = workload_pairs("paper_1436x992_d145")[0]
    lt = torch.from_numpy(pair.left).cuda()
    rt = torch.from_numpy(pair.right).cuda()
    ref = ctx.disparity(lt, rt, 145).cpu().numpy()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty(ref.shape, dtype=torch.int16, device="cuda") for _ in range(10)]
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        ctx.disparity(lt, rt, 145, out=o, stream=streams[i % 2])
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), ref), ("two streams", i)
    for i in range(10):
        assert np.array_equal(ctx.disparity(lt, rt, 145).cpu().numpy(), ref), ("serial", i)


def test_frames_in_flight_on_two_streams(sm, ctx):
    # frames issued round-robin on two streams (each with its own plan), many in
    # flight at once as in the throughput measurement: every map equals the
    # one-stream map of its pair
    say("case: 12 frames of 3 pairs (640x480, Dmax 64) on two streams")
    pairs = [make_pair(640, 480, 64, segments=6, seed=s) for s in (70, 71, 72)]
    lefts = [torch.from_numpy(p.left).cuda() for p in pairs]
    rights = [torch.from_numpy(p.right).cuda() for p in pairs]
    single = [ctx.disparity(l, r, 64).cpu().numpy() for l, r in zip(lefts, rights)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    outs = []
    for i in range(12):
        p = (i // 2 + i) % 3
        outs.append((p, ctx.disparity(lefts[p], rights[p], 64, stream=streams[i % 2])))
    torch.cuda.synchronize()
    for p, o in outs:
        assert np.array_equal(o.cpu().numpy(), single[p])


def test_errors_leave_context_usable(sm, ctx):
    pair = make_pair(64, 32, 16, segments=2, seed=60)
    lt = torch.from_numpy(pair.left).cuda()
    rt = torch.from_numpy(pair.right).cuda()
    with pytest.raises(sm.StereoError) as e:
        ctx.disparity(lt, rt, 65)             # Dmax > W
    assert e.value.code == -1 and "Dmax" in ctx.last_error()
    bad = sm.default_params()
    bad.size = 12
    with pytest.raises(sm.StereoError):
        ctx.disparity(lt, rt, 16, bad)
    for kw in (dict(arm_x=128), dict(lambda_ad=0.0), dict(cost_scale=2048)):
        with pytest.raises(sm.StereoError):
            ctx.disparity(lt, rt, 16, sm.default_params(**kw))
    # 201 x 255 x 1936 > 2^24, the aggregate field of the keys for D = 145
    # (8 bits of d); with D = 8 (3 bits) the same caps are valid
    wide = torch.zeros((32, 300, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(sm.StereoError) as e:
        ctx.disparity(wide, wide, 290, sm.default_params(arm_x=100, arm_y=127))
    assert "2^24" in ctx.last_error()
    ctx.disparity(wide, wide, 16, sm.default_params(arm_x=100, arm_y=127))
    L = sm.lib()
    assert L.stereo_disparity(ctx._h, None, rt.data_ptr(), 64, 32, 16, None,
                              lt.data_ptr(), None) == -1
    assert L.stereo_disparity(None, None, None, 64, 32, 16, None, None, None) == -1
    got = ctx.disparity(lt, rt, 16)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.disparity(pair.left, pair.right, 16)["out"])


def test_captured_plan_is_not_evicted(sm):
    """Under a memory cap, a plan a captured graph launches into is kept: a
    later call of another shape that would need its memory fails with
    STEREO_ENOMEM instead, and the graph's replays stay correct."""
    import re
    a = make_pair(320, 240, 32, segments=3, seed=62)
    b = make_pair(480, 320, 48, segments=3, seed=63)
    la, ra = torch.from_numpy(a.left).cuda(), torch.from_numpy(a.right).cuda()
    lb, rb = torch.from_numpy(b.left).cuda(), torch.from_numpy(b.right).cuda()

    def need(left, right, dmax):  # bytes of a plan, from the cap's error text
        c = sm.Stereo(0, mem_cap=1)
        with pytest.raises(sm.StereoError):
            c.disparity(left, right, dmax)
        n = int(re.search(r"needs (\d+) bytes", c.last_error()).group(1))
        c.close()
        return n

    na, nb = need(la, ra, 32), need(lb, rb, 48)
    c = sm.Stereo(0, mem_cap=na + nb - 1)
    s = torch.cuda.Stream()
    ref = oracle.disparity(a.left, a.right, 32)["out"]
    out = torch.empty((240, 320), dtype=torch.int16, device="cuda")
    with torch.cuda.stream(s):
        c.disparity(la, ra, 32, out=out, stream=s)      # the plan exists before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        c.disparity(la, ra, 32, out=out, stream=s)
    with torch.cuda.stream(s):
        with pytest.raises(sm.StereoError) as e:
            c.disparity(lb, rb, 48, stream=s)           # would evict the captured plan
    assert e.value.code == -2
    for _ in range(2):
        out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref)
    del g
    c.close()


def test_new_shape_under_capture_is_refused(sm, ctx):
    """A first call of a shape needs an allocation, which a capturing stream
    cannot make: the call fails cleanly and the context stays usable."""
    p = make_pair(112, 80, 16, segments=2, seed=64)
    lt, rt = torch.from_numpy(p.left).cuda(), torch.from_numpy(p.right).cuda()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(g, stream=s):
        try:
            ctx.disparity(lt, rt, 16, stream=s)
        except sm.StereoError as e:
            err = e
    assert err is not None and err.code == -1 and "capture" in ctx.last_error()
    del g
    got = ctx.disparity(lt, rt, 16)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.disparity(p.left, p.right, 16)["out"])


def test_memory_cap(sm):
    c = sm.Stereo(0, mem_cap=1 << 16)
    pair = make_pair(320, 240, 32, segments=2, seed=61)
    lt = torch.from_numpy(pair.left).cuda()
    rt = torch.from_numpy(pair.right).cuda()
    with pytest.raises(sm.StereoError) as e:
        c.disparity(lt, rt, 32)
    assert e.value.code == -2
    c.close()


# ------------------------------------------------ variants (Sec. III-E, Sec. V)

@pytest.mark.parametrize("kw", [
    dict(fill_mode=1), dict(fill_mode=2), dict(arm_x_r=7), dict(arm_x=9, arm_x_r=40),
    dict(arm_x_r=0, fill_mode=1),
])
def test_variants_bit_exact(sm, ctx, kw):
    pair = make_pair(150, 90, 30, segments=4, seed=11)
    full_parity(sm, ctx, pair.left, pair.right, 30, keep_params(sm, **kw), label=str(kw))


@pytest.mark.parametrize("W,H,dmax,kw", [
    (160, 120, 32, dict(arm_x=41, arm_y=61)),            # the paper's full-size caps
    (97, 53, 20, dict(arm_x=41, arm_y=61, fill_mode=2)),
    (640, 480, 64, dict(arm_x=41, arm_y=61)),
    (301, 77, 145, dict(arm_x=41, arm_y=61, cost_scale=512, arm_x_r=30)),  # 8-bit d field
])
def test_full_resolution_mode_bit_exact(sm, ctx, W, H, dmax, kw):
    pair = make_pair(W, H, dmax, segments=5, seed=12)
    p = sm.default_params(flags=sm.F_KEEP_INTERMEDIATES | sm.F_FULL_RES, **kw)
    full_parity(sm, ctx, pair.left, pair.right, dmax, p, label=f"full {W}x{H} {kw}")


def test_variant_parameter_checks(sm, ctx):
    pair = make_pair(64, 48, 16, segments=3, seed=13)
    lt = torch.from_numpy(pair.left).cuda()
    rt = torch.from_numpy(pair.right).cuda()
    for kw in (dict(fill_mode=3), dict(arm_x_r=-2), dict(arm_x_r=128),
               # 83 x 123 x 1936 exceeds 2^24 with an 8-bit d field
               dict(flags=sm.F_FULL_RES, arm_x=41, arm_y=61)):
        with pytest.raises(sm.StereoError) as e:
            dmax = 145 if "flags" in kw else 16
            big = torch.zeros((64, 160, 3), dtype=torch.uint8, device="cuda")
            if "flags" in kw:
                ctx.disparity(big, big, dmax, sm.default_params(**kw))
            else:
                ctx.disparity(lt, rt, 16, sm.default_params(**kw))
        assert e.value.code == -1, kw
    # still usable
    ctx.disparity(lt, rt, 16)


# ------------------------------------------------- captured graphs, autotune

def test_graph_replays_match_eager(sm, ctx):
    """A batched call captured in a HIP graph, replayed ten times with other
    eager work and synchronisations between, gives the eager maps each time."""
    pairs = [make_pair(96, 64, 24, segments=3, seed=70 + i) for i in range(3)]
    lefts = [torch.from_numpy(p.left).cuda() for p in pairs]
    rights = [torch.from_numpy(p.right).cuda() for p in pairs]
    outs = [torch.empty((64, 96), dtype=torch.int16, device="cuda") for _ in pairs]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ref = [o.cpu().numpy() for o in ctx.disparity_batch(lefts, rights, 24)]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ctx.disparity_batch(lefts, rights, 24, outs=outs)
    other = make_pair(80, 40, 16, segments=2, seed=79)
    assert np.array_equal(ref[0], oracle.disparity(pairs[0].left, pairs[0].right, 24)["out"])
    for k in range(10):
        for o in outs:
            o.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(3):
            assert np.array_equal(outs[i].cpu().numpy(), ref[i]), (k, i)
        ctx.disparity(torch.from_numpy(other.left).cuda(), torch.from_numpy(other.right).cuda(), 16)
        torch.cuda.synchronize()


def test_autotune_keeps_results(sm, ctx):
    pairs = [make_pair(300, 200, 48, segments=4, seed=80 + i) for i in range(2)]
    lefts = [torch.from_numpy(p.left).cuda() for p in pairs]
    rights = [torch.from_numpy(p.right).cuda() for p in pairs]
    chosen, cands = ctx.autotune(lefts, rights, 48)
    assert chosen in cands and len(cands) >= 2 and all(v > 0 for v in cands.values())
    outs = ctx.disparity_batch(lefts, rights, 48)
    torch.cuda.synchronize()
    for i in range(2):
        exp = oracle.disparity(pairs[i].left, pairs[i].right, 48)["out"]
        assert np.array_equal(outs[i].cpu().numpy(), exp)
