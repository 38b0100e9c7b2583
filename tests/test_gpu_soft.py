"""GPU parity of the soft-argmin head against the FP64 oracle (oracle/soft.py).

Tolerances follow from the kernel's arithmetic: costs enter the aggregate in
fixed point with 2^-19 resolution (k = 18 for the default arms), so the mean
cost is within 2^-19 of the exact one and a logit (mean / tau) within
2e-5; the rest is float32 (relative 1e-6 per operation).  d_hat is compared
to 1e-3 absolute, the loss to 1e-4 relative and every gradient to 1e-3
relative to its largest magnitude (and in norm).
"""

import numpy as np
import pytest
import torch

from oracle import soft as osoft
from paper_2212_00488_amd import Stereo
from paper_2212_00488_amd.binding import soft_default_params
from paper_2212_00488_amd.soft import l1_loss, soft_disparity
from paper_2212_00488_amd.synth import make_pair

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = Stereo(0)
    yield c
    c.close()


def float_pairs(n, W, H, dmax, seed, noise=0.0):
    """n synthetic pairs as float32 [0,1] images (plus GT and mask); noise
    adds small uniform jitter so that no two intensities tie exactly."""
    rng = np.random.default_rng(seed)
    L, R, G, M = [], [], [], []
    for i in range(n):
        p = make_pair(W, H, dmax, segments=4, seed=seed + i)
        l = p.left.astype(np.float32) / np.float32(255.0)
        r = p.right.astype(np.float32) / np.float32(255.0)
        if noise:
            l = np.clip(l + rng.uniform(-noise, noise, l.shape).astype(np.float32), 0, 1)
            r = np.clip(r + rng.uniform(-noise, noise, r.shape).astype(np.float32), 0, 1)
        L.append(l.astype(np.float32))
        R.append(r.astype(np.float32))
        G.append(p.gt)
        M.append(p.nonocc)
    return np.stack(L), np.stack(R), np.stack(G), np.stack(M)


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return t.to(dtype) if dtype is not None else t


def sp_from(p: osoft.SoftParams, slab=0):
    return soft_default_params(tau=p.tau, color_delta=p.color_delta, arm_x=p.arm_x,
                               arm_y=p.arm_y, slab=slab)


def run_gpu(ctx, L, R, G, M, dmax, p, lam=None, slab=0):
    lam = lam if lam is not None else (p.lambda_ad, p.lambda_census)
    left = to_dev(L).requires_grad_(True)
    right = to_dev(R).requires_grad_(True)
    lambdas = torch.tensor(lam, dtype=torch.float32, device=DEV, requires_grad=True)
    d_hat = soft_disparity(ctx, left, right, lambdas, dmax, sp_from(p, slab))
    loss = l1_loss(ctx, d_hat, to_dev(G.astype(np.int16)), to_dev(M.astype(np.uint8)))
    loss.backward()
    torch.cuda.synchronize()
    return (d_hat.detach().cpu().numpy(), float(loss.detach().cpu()[0]),
            left.grad.cpu().numpy(), right.grad.cpu().numpy(), lambdas.grad.cpu().numpy())


def oracle_dhat(L, R, dmax, p):
    out = []
    for i in range(len(L)):
        r = osoft.forward(torch.tensor(L[i], dtype=torch.float64),
                          torch.tensor(R[i], dtype=torch.float64), dmax,
                          torch.tensor(p.lambda_ad, dtype=torch.float64),
                          torch.tensor(p.lambda_census, dtype=torch.float64), p)
        out.append(r["d_hat"].numpy())
    return np.stack(out)


def assert_grad_close(g, r, name, rel=1e-3, floor=1e-2, rel_elem=5e-3):
    """Max error within rel of the largest reference magnitude, the norm of
    the error within rel of the reference's norm, and every entry whose
    reference magnitude is at least floor x the largest within rel_elem of
    itself (the per-entry check sees errors on smaller entries that the
    first two hide)."""
    scale = float(np.abs(r).max())
    assert scale > 0, name
    err = float(np.abs(g - r).max())
    assert err <= rel * scale, f"{name}: max err {err:.3e} vs {rel} x {scale:.3e}"
    nerr = float(np.linalg.norm((g - r).ravel()) / np.linalg.norm(r.ravel()))
    assert nerr <= rel, f"{name}: norm rel err {nerr:.3e}"
    big = np.abs(r) >= floor * scale
    eel = float((np.abs(g - r)[big] / np.abs(r)[big]).max())
    print(f"[grad] {name}: max err {err / scale:.2e} of max, worst entry above "
          f"{floor:g} x max {eel:.2e} relative ({int(big.sum())} entries)", flush=True)
    assert eel <= rel_elem, f"{name}: entry rel err {eel:.3e} above {floor} x max"


@pytest.mark.parametrize("case", [
    dict(W=64, H=48, dmax=32, n=2, seed=500),          # the FD configuration (D = 16)
    # the same with the adjoint in slabs of 3 and of 5 disparities (6 and 4
    # slabs, the last ones short): slab offsets and per-slab lambda partials
    dict(W=64, H=48, dmax=32, n=2, seed=500, slab=3),
    dict(W=64, H=48, dmax=32, n=2, seed=500, slab=5),
    dict(W=67, H=41, dmax=20, n=1, seed=510),          # odd sizes, ragged strip and band
    dict(W=67, H=41, dmax=20, n=1, seed=510, slab=4),
    dict(W=150, H=30, dmax=40, n=3, seed=520),         # three strips
])
def test_forward_loss_and_gradients_match_oracle(ctx, case):
    W, H, dmax, n, seed = case["W"], case["H"], case["dmax"], case["n"], case["seed"]
    L, R, G, M = float_pairs(n, W, H, dmax, seed, noise=0.002)
    p = osoft.SoftParams()
    print(f"[soft] {W}x{H} Dmax={dmax} n={n} slab={case.get('slab', 0)}", flush=True)
    d_hat, loss, gl, gr, glam = run_gpu(ctx, L, R, G, M, dmax, p, slab=case.get("slab", 0))
    ref = oracle_dhat(L, R, dmax, p)
    assert np.all(np.isfinite(d_hat))
    assert float(np.abs(d_hat - ref).max()) <= 1e-3
    rloss, rgl, rgr, rglam = osoft.loss_and_grads(list(L), list(R), list(G), list(M), dmax, p)
    assert abs(loss - rloss) <= 1e-4 * abs(rloss)
    assert_grad_close(gl, rgl, "g_left")
    assert_grad_close(gr, rgr, "g_right")
    for k in range(2):
        assert abs(glam[k] - rglam[k]) <= 1e-3 * abs(rglam[k]), (k, glam, rglam)


def test_arm_and_temperature_variants_match_oracle(ctx):
    L, R, G, M = float_pairs(1, 70, 36, 24, 530, noise=0.002)
    for p in (osoft.SoftParams(tau=0.3, arm_x=5, arm_y=4, color_delta=30),
              osoft.SoftParams(tau=0.05, arm_x=31, arm_y=63),
              osoft.SoftParams(arm_x=0, arm_y=0)):
        d_hat, loss, gl, gr, glam = run_gpu(ctx, L, R, G, M, 24, p)
        ref = oracle_dhat(L, R, 24, p)
        assert float(np.abs(d_hat - ref).max()) <= 1e-3, p
        rloss, rgl, rgr, rglam = osoft.loss_and_grads(list(L), list(R), list(G), list(M), 24, p)
        assert_grad_close(gl, rgl, f"g_left {p}")
        assert_grad_close(gr, rgr, f"g_right {p}")
        for k in range(2):
            assert abs(glam[k] - rglam[k]) <= 1e-3 * abs(rglam[k]) + 1e-9, (p, k, glam, rglam)


def test_lambda_gradient_matches_gpu_central_differences(ctx):
    """Central differences of the GPU forward itself for both lambdas, a
    coarse check of the adjoint on the kernels alone (the 1e-3 checks above
    compare against the FP64 reference gradient, itself pinned by float64
    central differences).  The differenced function is a fixed random linear
    functional of d_hat (the L1 loss has kinks a finite step crosses), summed
    in float64 on the host; its gradient comes from the adjoint with g_dhat =
    the weights.  The float32 forward with fixed-point costs carries about
    1e-5 of noise per d_hat, about 4e-4 in the functional, so a step of 1e-2
    lambda leaves about 1% of noise and truncation: tolerance 1.5e-2 (the
    check against the FP64 reference gradient above is the 1e-3 one)."""
    L, R, G, M = float_pairs(2, 64, 48, 32, 540, noise=0.002)
    p = osoft.SoftParams()
    w = np.random.default_rng(541).standard_normal((2, 24, 32)).astype(np.float32)
    left, right = to_dev(L), to_dev(R)
    lam = torch.tensor([p.lambda_ad, p.lambda_census], dtype=torch.float32, device=DEV,
                       requires_grad=True)
    d = soft_disparity(ctx, left, right, lam, 32, sp_from(p))
    (d * to_dev(w)).sum().backward()
    glam = lam.grad.cpu().numpy()
    base = np.array([p.lambda_ad, p.lambda_census])

    def f(lv):
        with torch.no_grad():
            lt = torch.tensor(lv, dtype=torch.float32, device=DEV)
            dh = soft_disparity(ctx, left, right, lt, 32, sp_from(p)).cpu().numpy()
        return float(np.sum(dh.astype(np.float64) * w))

    for k in range(2):
        e = np.zeros(2)
        e[k] = 1e-2 * base[k]
        fd = (f(base + e) - f(base - e)) / (2 * e[k])
        assert abs(fd - glam[k]) <= 1.5e-2 * abs(glam[k]) + 1e-6, (k, fd, glam[k])


def test_backward_is_deterministic_and_batch_matches_single(ctx):
    L, R, G, M = float_pairs(3, 96, 40, 30, 550, noise=0.002)
    p = osoft.SoftParams()
    a = run_gpu(ctx, L, R, G, M, 30, p)
    for rep in range(9):  # ten runs in all, the same bits each time
        b = run_gpu(ctx, L, R, G, M, 30, p)
        for u, v in zip(a, b):
            assert np.array_equal(np.asarray(u), np.asarray(v)), rep
    # pair 1 alone: same d_hat (chunk sums may group differently) and, with the
    # loss of one pair instead of the mean of three, 3x the image gradients
    s = run_gpu(ctx, L[1:2], R[1:2], G[1:2], M[1:2], 30, p)
    assert float(np.abs(s[0][0] - a[0][1]).max()) <= 1e-5
    assert_grad_close(s[2][0], 3.0 * a[2][1], "single vs batch g_left", rel=1e-4)


def launch_step(ctx, L, R, G, M, dmax, p):
    """Forward + loss + backward enqueued on the current stream, no wait."""
    left = to_dev(L).requires_grad_(True)
    right = to_dev(R).requires_grad_(True)
    lambdas = torch.tensor((p.lambda_ad, p.lambda_census), dtype=torch.float32, device=DEV,
                           requires_grad=True)
    d_hat = soft_disparity(ctx, left, right, lambdas, dmax, sp_from(p))
    loss = l1_loss(ctx, d_hat, to_dev(G.astype(np.int16)), to_dev(M.astype(np.uint8)))
    loss.backward()
    return d_hat, loss, left, right, lambdas


def test_ten_training_steps_bit_identical_at_paper_size(ctx):
    """4 x 1436x992, Dmax = 145: ten forward + loss + backward steps (the
    saved-weights path) give the same d_hat, loss and gradients bit for bit."""
    L, R, G, M = float_pairs(4, 1436, 992, 145, 400)
    p = osoft.SoftParams()
    first = None
    for rep in range(10):
        d_hat, loss, left, right, lam = launch_step(ctx, L, R, G, M, 145, p)
        torch.cuda.synchronize()
        got = (d_hat.detach().cpu().numpy(), loss.detach().cpu().numpy(),
               left.grad.cpu().numpy(), right.grad.cpu().numpy(), lam.grad.cpu().numpy())
        if first is None:
            first = got
            continue
        for u, v in zip(got, first):
            assert np.array_equal(u, v), rep


def test_two_streams_equal_serial_runs(ctx):
    """Forward + backward of two batches in flight on two streams at once
    (each stream has its own plan and loss scratch) equal the same runs made
    one after the other, bit for bit."""
    A = float_pairs(2, 96, 40, 30, 560, noise=0.002)
    B = float_pairs(1, 80, 48, 24, 570, noise=0.002)
    p = osoft.SoftParams()
    serial = [run_gpu(ctx, *A, 30, p), run_gpu(ctx, *B, 24, p)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(2):
        torch.cuda.synchronize()
        live = []
        for i, (case, dmax) in enumerate(((A, 30), (B, 24))):
            with torch.cuda.stream(streams[i]):
                live.append(launch_step(ctx, *case, dmax, p))
        torch.cuda.synchronize()
        for i, (d_hat, loss, left, right, lam) in enumerate(live):
            got = (d_hat.detach().cpu().numpy(), float(loss.detach().cpu()[0]),
                   left.grad.cpu().numpy(), right.grad.cpu().numpy(), lam.grad.cpu().numpy())
            for u, v in zip(got, serial[i]):
                assert np.array_equal(np.asarray(u), np.asarray(v)), (rep, i)


def test_paper_size_batch_rows_match_oracle(ctx):
    """4 x 1436x992, Dmax = 145 (the differentiable configuration): d_hat of
    a band of rows against the oracle run on a crop of rows wide enough that
    the band's features, windows and borders are those of the full image."""
    W, H, dmax = 1436, 992, 145
    L, R, G, M = float_pairs(4, W, H, dmax, 400)
    p = osoft.SoftParams()
    lambdas = torch.tensor([p.lambda_ad, p.lambda_census], dtype=torch.float32, device=DEV,
                           requires_grad=True)
    left = to_dev(L).requires_grad_(True)
    right = to_dev(R).requires_grad_(True)
    d_hat = soft_disparity(ctx, left, right, lambdas, dmax, sp_from(p))
    loss = l1_loss(ctx, d_hat, to_dev(G.astype(np.int16)), to_dev(M.astype(np.uint8)))
    loss.backward()
    torch.cuda.synchronize()
    dh = d_hat.detach().cpu().numpy()
    assert np.all(np.isfinite(dh)) and dh.min() >= 0 and dh.max() <= 72
    assert np.all(np.isfinite(left.grad.cpu().numpy()))
    assert np.all(np.isfinite(right.grad.cpu().numpy()))
    assert np.all(np.isfinite(lambdas.grad.cpu().numpy()))
    y0, y1 = 240, 256                    # half-res rows checked (band boundary at 248)
    ya, yb = y0 - 36, y1 + 36            # crop in half-res rows
    for i in (0, 3):
        Lc = L[i, 2 * ya:2 * yb]
        Rc = R[i, 2 * ya:2 * yb]
        ref = oracle_dhat(Lc[None], Rc[None], dmax, p)[0]
        got = dh[i, y0:y1]
        assert float(np.abs(got - ref[y0 - ya:y1 - ya]).max()) <= 1e-3


def test_feature_reuse_in_interleaved_backwards(ctx):
    """The autograd backward reuses the forward's features and weights when
    the plan still holds them: forward A, forward B (other tensors, same
    shape, same plan, whose weights replace A's), then the backward of A must
    recompute A's features and aggregate and give A's gradients, as must B's
    backward after it (A's backward recomputed the slabs over B's weights).
    The reference runs took the saved-weights path, these the recomputing
    one: equal to float rounding."""
    p = osoft.SoftParams()
    A = float_pairs(1, 96, 40, 30, 570, noise=0.002)
    B = float_pairs(1, 96, 40, 30, 571, noise=0.002)
    ref_a = run_gpu(ctx, *A, 30, p)
    ref_b = run_gpu(ctx, *B, 30, p)
    outs = []
    for L, R, G, M in (A, B):
        left = to_dev(L).requires_grad_(True)
        right = to_dev(R).requires_grad_(True)
        lam = torch.tensor((p.lambda_ad, p.lambda_census), dtype=torch.float32, device=DEV,
                           requires_grad=True)
        d = soft_disparity(ctx, left, right, lam, 30, sp_from(p))
        loss = l1_loss(ctx, d, to_dev(G.astype(np.int16)), to_dev(M.astype(np.uint8)))
        outs.append((loss, left, right, lam))
    for (loss, left, right, lam), ref, nm in zip(outs, (ref_a, ref_b), "AB"):
        loss.backward()
        torch.cuda.synchronize()
        assert_grad_close(left.grad.cpu().numpy(), ref[2], f"{nm} g_left", rel=1e-5,
                          rel_elem=1e-4)
        assert_grad_close(right.grad.cpu().numpy(), ref[3], f"{nm} g_right", rel=1e-5,
                          rel_elem=1e-4)
        g = lam.grad.cpu().numpy()
        assert np.all(np.abs(g - ref[4]) <= 1e-5 * np.abs(ref[4])), (nm, g, ref[4])


def soft_grads(ctx, left, right, lam, dmax, p, g_dhat, fwd_flags, bwd_flags, slab=0):
    """Forward then backward through the C ABI with the given flags."""
    fp = sp_from(p, slab)
    fp.flags = fwd_flags
    d_hat, lse2 = ctx.soft_forward(left, right, lam, dmax, fp)
    bp = sp_from(p, slab)
    bp.flags = bwd_flags
    gl, gr, glam = ctx.soft_backward(left, right, lam, dmax, d_hat, lse2, g_dhat, bp)
    torch.cuda.synchronize()
    return d_hat.cpu().numpy(), gl.cpu().numpy(), gr.cpu().numpy(), glam.cpu().numpy()


def test_saved_weights_path_matches_recompute(ctx):
    """The backward that forms dL/dCA from the forward's saved weights
    (k_soft_tcolw) equals the one that recomputes the aggregate per slab
    (k_soft_agg, k_soft_tcol) to float rounding, on the FD configuration and
    on odd sizes with three strips; with the slab smaller than D the forward
    cannot save the weights and both calls take the recomputing path, bit
    for bit."""
    from paper_2212_00488_amd.binding import SOFT_F_REUSE_FEATURES, SOFT_F_SAVE_WEIGHTS
    p = osoft.SoftParams()
    for (n, W, H, dmax, seed) in ((2, 64, 48, 32, 580), (3, 150, 30, 40, 581), (1, 67, 41, 20, 582)):
        L, R, G, M = float_pairs(n, W, H, dmax, seed, noise=0.002)
        left, right = to_dev(L), to_dev(R)
        lam = torch.tensor((p.lambda_ad, p.lambda_census), dtype=torch.float32, device=DEV)
        X, Y = (W + 1) // 2, (H + 1) // 2
        g = to_dev(np.random.default_rng(seed).standard_normal((n, Y, X)).astype(np.float32))
        print(f"[soft] saved weights vs recompute {W}x{H} Dmax={dmax} n={n}", flush=True)
        rec = soft_grads(ctx, left, right, lam, dmax, p, g, 0, SOFT_F_REUSE_FEATURES)
        sav = soft_grads(ctx, left, right, lam, dmax, p, g, SOFT_F_SAVE_WEIGHTS,
                         SOFT_F_REUSE_FEATURES)
        assert np.array_equal(rec[0], sav[0])
        assert_grad_close(sav[1], rec[1], "saved g_left", rel=1e-5, rel_elem=1e-4)
        assert_grad_close(sav[2], rec[2], "saved g_right", rel=1e-5, rel_elem=1e-4)
        assert np.all(np.abs(sav[3] - rec[3]) <= 1e-5 * np.abs(rec[3])), (sav[3], rec[3])
        # slabs of 3: nothing saved, the same recomputing path both times
        a = soft_grads(ctx, left, right, lam, dmax, p, g, 0, SOFT_F_REUSE_FEATURES, slab=3)
        b = soft_grads(ctx, left, right, lam, dmax, p, g, SOFT_F_SAVE_WEIGHTS,
                       SOFT_F_REUSE_FEATURES, slab=3)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


def test_saved_weights_dropped_by_a_later_forward(ctx):
    """A forward that saves weights, then new data written into the same
    tensors and a forward without saving: the backward (same pointers,
    REUSE_FEATURES) must not take the first forward's weights; its gradients
    are those of the new data."""
    from paper_2212_00488_amd.binding import SOFT_F_REUSE_FEATURES, SOFT_F_SAVE_WEIGHTS
    p = osoft.SoftParams()
    A = float_pairs(1, 96, 40, 30, 590, noise=0.002)
    B = float_pairs(1, 96, 40, 30, 591, noise=0.002)
    lam = torch.tensor((p.lambda_ad, p.lambda_census), dtype=torch.float32, device=DEV)
    g = to_dev(np.random.default_rng(592).standard_normal((1, 20, 48)).astype(np.float32))
    lb, rb = to_dev(B[0]), to_dev(B[1])
    ref = soft_grads(ctx, lb, rb, lam, 30, p, g, 0, 0)
    left, right = to_dev(A[0]), to_dev(A[1])
    fp = sp_from(p)
    fp.flags = SOFT_F_SAVE_WEIGHTS
    ctx.soft_forward(left, right, lam, 30, fp)
    left.copy_(lb)
    right.copy_(rb)
    got = soft_grads(ctx, left, right, lam, 30, p, g, 0, SOFT_F_REUSE_FEATURES)
    for u, v in zip(got, ref):
        assert np.array_equal(u, v)
