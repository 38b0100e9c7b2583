"""Pins of the FP64 soft-argmin head oracle (no GPU).

The head's forward is checked against a pixel-by-pixel brute force of the
same definitions (cross-region cell lists, math.exp), against closed forms
and limits (tau -> 0 gives the hard argmin, huge lambdas give a uniform
distribution, a constant-shift pair has zero cost at its shift), and its
autograd gradients against central finite differences in float64.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from oracle import brute
from oracle import soft
from paper_2212_00488_amd.synth import make_pair, textured_shift_pair

F64 = torch.float64


def rand_pair(rng, H, W):
    return (rng.random((H, W, 3), dtype=np.float32), rng.random((H, W, 3), dtype=np.float32))


def test_quantize_round_trip_and_clamp():
    u = np.arange(256, dtype=np.float32)
    assert np.array_equal(soft.quantize(u / np.float32(255.0)), np.arange(256, dtype=np.uint8))
    assert soft.quantize(np.array([-0.3, 1.7], np.float32)).tolist() == [0, 255]
    # ties round up: inputs whose float32 product 255 v is exactly k + 1/2
    k = np.arange(255, dtype=np.float32)
    v = ((k + np.float32(0.5)) / np.float32(255.0)).astype(np.float32)
    tie = (np.float32(255.0) * v) == k + np.float32(0.5)
    assert tie.sum() > 10
    assert np.array_equal(soft.quantize(v[tie]), (k[tie] + 1).astype(np.uint8))


def test_gray_and_downscale_closed_forms():
    c = torch.full((7, 9, 3), 0.37, dtype=F64)
    g = soft.gray_f(c)
    assert torch.allclose(g, torch.full((7, 9), 0.37, dtype=F64), atol=1e-15)
    h = soft.downscale_f(g)
    assert h.shape == (4, 5)
    assert torch.allclose(h, torch.full((4, 5), 0.37, dtype=F64), atol=1e-15)
    # a single bright full-res pixel at (2,2) spreads 1/9 to half-res (1,1) only
    g2 = torch.zeros((7, 9), dtype=F64)
    g2[2, 2] = 9.0
    h2 = soft.downscale_f(g2)
    expect = torch.zeros((4, 5), dtype=F64)
    expect[1, 1] = 1.0
    assert torch.equal(h2, expect)


def test_forward_matches_pixel_brute_force():
    rng = np.random.default_rng(7)
    H, W, dmax = 10, 13, 6
    left, right = rand_pair(rng, H, W)
    p = soft.SoftParams(arm_x=3, arm_y=2, color_delta=60)
    feats = soft.features(left, right, p)
    out = soft.forward(torch.tensor(left, dtype=F64), torch.tensor(right, dtype=F64), dmax,
                       torch.tensor(p.lambda_ad, dtype=F64),
                       torch.tensor(p.lambda_census, dtype=F64), p, feats)
    cl, cr, arms = feats
    hl = brute.soft_half(left.astype(np.float64).tolist())
    hr = brute.soft_half(right.astype(np.float64).tolist())
    assert np.allclose(out["half_l"].numpy(), np.array(hl), atol=1e-14)
    a = arms.tolist()
    ref = brute.soft_d_hat(hl, hr, cl.tolist(), cr.tolist(), a, (dmax + 1) // 2,
                           p.lambda_ad, p.lambda_census, p.tau)
    assert np.allclose(out["d_hat"].numpy(), np.array(ref), atol=1e-12, rtol=0)
    # the support size is the number of cells of the cross region
    Y, X = out["size"].shape
    for y in range(Y):
        for x in range(X):
            assert out["size"][y, x] == len(brute.cross_region(a, x, y))
    # arms are non-trivial in this case (so the windows are exercised)
    assert arms.max() > 0


def test_cost_values_and_invalid_columns():
    rng = np.random.default_rng(3)
    left, right = rand_pair(rng, 6, 10)
    p = soft.SoftParams()
    cl, cr, arms = soft.features(left, right, p)
    hl = soft.downscale_f(soft.gray_f(torch.tensor(left, dtype=F64)))
    hr = soft.downscale_f(soft.gray_f(torch.tensor(right, dtype=F64)))
    C = soft.cost_volume(hl, hr, cl, cr, 4, p.lambda_ad, p.lambda_census)
    for d in range(4):
        for y in range(3):
            for x in range(5):
                if x < d:
                    assert float(C[d, y, x]) == 2.0
                else:
                    ad = 255.0 * abs(float(hl[y, x]) - float(hr[y, x - d]))
                    h = bin(int(cl[y, x]) ^ int(cr[y, x - d])).count("1")
                    want = 2.0 - math.exp(-ad / p.lambda_ad) - math.exp(-h / p.lambda_census)
                    assert abs(float(C[d, y, x]) - want) < 1e-14
                    assert 0.0 <= float(C[d, y, x]) < 2.0


def test_tau_to_zero_is_hard_argmin():
    rng = np.random.default_rng(11)
    left, right = rand_pair(rng, 16, 20)
    p = soft.SoftParams(tau=1e-4)
    feats = soft.features(left, right, p)
    out = soft.forward(torch.tensor(left, dtype=F64), torch.tensor(right, dtype=F64), 10,
                       torch.tensor(p.lambda_ad, dtype=F64),
                       torch.tensor(p.lambda_census, dtype=F64), p, feats)
    mean = (out["agg"] / out["size"]).numpy()
    best = np.argmin(mean, axis=0)
    srt = np.sort(mean, axis=0)
    clear = (srt[1] - srt[0]) > 0.01
    assert clear.sum() > 0.5 * clear.size
    assert np.all(np.abs(out["d_hat"].numpy()[clear] - best[clear]) < 1e-9)


def test_huge_lambdas_give_uniform_distribution():
    rng = np.random.default_rng(5)
    left, right = rand_pair(rng, 12, 120)
    p = soft.SoftParams(lambda_ad=1e15, lambda_census=1e15)
    D = 4
    feats = soft.features(left, right, p)
    out = soft.forward(torch.tensor(left, dtype=F64), torch.tensor(right, dtype=F64), 2 * D,
                       torch.tensor(p.lambda_ad, dtype=F64),
                       torch.tensor(p.lambda_census, dtype=F64), p, feats)
    # columns whose whole support is valid for every d have mean cost 0 for all d
    m = feats[2][..., 0].astype(int)
    X = out["d_hat"].shape[1]
    cols = np.arange(X)[None, :]
    ok = (cols - p.arm_x) >= D  # support starts at x - m >= x - arm_x >= D - 1
    assert ok.any()
    assert np.allclose(out["d_hat"].numpy()[np.broadcast_to(ok, m.shape)], (D - 1) / 2.0,
                       atol=1e-9)


def test_constant_shift_pair_has_zero_cost_at_the_shift():
    k = 3
    lu8, ru8 = textured_shift_pair(96, 40, 2 * k, seed=4)
    left = lu8.astype(np.float32) / np.float32(255.0)
    right = ru8.astype(np.float32) / np.float32(255.0)
    p = soft.SoftParams(tau=0.01)
    feats = soft.features(left, right, p)
    out = soft.forward(torch.tensor(left, dtype=F64), torch.tensor(right, dtype=F64), 16,
                       torch.tensor(p.lambda_ad, dtype=F64),
                       torch.tensor(p.lambda_census, dtype=F64), p, feats)
    mean = (out["agg"] / out["size"]).numpy()
    Y, X = mean.shape[1:]
    arms = feats[2].astype(int)
    # pixels whose cross region stays where the shifted copy is exact
    # (columns >= k + 2 after the census reach, rows away from the clamp)
    clean = np.zeros((Y, X), bool)
    for y in range(2, Y - 2):
        for x in range(k + 3, X - 2):
            cells = brute.cross_region(arms.tolist(), x, y)
            clean[y, x] = all(k + 3 <= cx < X - 2 and 2 <= cy < Y - 2 for cx, cy in cells)
    assert clean.sum() > 100
    assert np.all(mean[k][clean] == 0.0)
    dh = out["d_hat"].numpy()[clean]
    assert np.mean(np.abs(dh - k) < 1e-3) > 0.95


def test_l1_loss_hand_example():
    d_hat = torch.tensor([[1.0, 2.5], [0.0, 3.0]], dtype=F64)
    gt = np.zeros((4, 4), np.int16)
    gt[0, 0], gt[0, 2], gt[2, 0], gt[2, 2] = 2, 4, 9, 5
    nonocc = np.ones((4, 4), bool)
    nonocc[2, 0] = False
    # |2-2| + |5-4| + |6-5| over 3 pixels
    assert abs(float(soft.l1_loss(d_hat, gt, nonocc)) - 2.0 / 3.0) < 1e-15


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_central_differences(seed):
    """Autograd of the FP64 forward against central finite differences, for
    both lambdas and sampled intensities of both images of both pairs."""
    rng = np.random.default_rng(100 + seed)
    H, W, dmax, n = 12, 18, 8, 2
    lefts, rights, gts, nonoccs = [], [], [], []
    for i in range(n):
        l, r = rand_pair(rng, H, W)
        lefts.append(l)
        rights.append(r)
        gts.append(rng.integers(0, dmax, size=(H, W)).astype(np.int16))
        nonoccs.append(rng.random((H, W)) < 0.8)
    p = soft.SoftParams(tau=0.3, color_delta=40, arm_x=4, arm_y=3)
    loss, gl, gr, glam = soft.loss_and_grads(lefts, rights, gts, nonoccs, dmax, p)
    feats = [soft.features(lefts[i], rights[i], p) for i in range(n)]
    h = 1e-6

    def fd_lambda(name):
        pp = soft.SoftParams(**{**p.__dict__, name: getattr(p, name) + h})
        pm = soft.SoftParams(**{**p.__dict__, name: getattr(p, name) - h})
        return (soft.loss_value(lefts, rights, gts, nonoccs, dmax, pp, feats) -
                soft.loss_value(lefts, rights, gts, nonoccs, dmax, pm, feats)) / (2 * h)

    for idx, name in enumerate(("lambda_ad", "lambda_census")):
        fd = fd_lambda(name)
        assert abs(fd - glam[idx]) <= 1e-6 * abs(fd) + 2e-9, (name, fd, glam[idx])

    checked = 0
    for _ in range(12):
        i = int(rng.integers(n))
        y, x, c = int(rng.integers(H)), int(rng.integers(W)), int(rng.integers(3))
        for imgs, g in ((lefts, gl), (rights, gr)):
            plus = [a.astype(np.float64) for a in imgs]
            minus = [a.astype(np.float64) for a in imgs]
            plus[i][y, x, c] += h
            minus[i][y, x, c] -= h
            if imgs is lefts:
                lp = soft.loss_value(plus, rights, gts, nonoccs, dmax, p, feats)
                lm = soft.loss_value(minus, rights, gts, nonoccs, dmax, p, feats)
            else:
                lp = soft.loss_value(lefts, plus, gts, nonoccs, dmax, p, feats)
                lm = soft.loss_value(lefts, minus, gts, nonoccs, dmax, p, feats)
            fd = (lp - lm) / (2 * h)
            # h = 1e-6 leaves about 1e-16 / h of rounding in the difference
            assert abs(fd - g[i, y, x, c]) <= 1e-6 * abs(fd) + 2e-9, (i, y, x, c, fd,
                                                                       g[i, y, x, c])
            checked += abs(fd) > 1e-6
    assert checked > 4  # most sampled intensities do move the loss


def test_features_match_integer_path():
    """The frozen features are the integer path's, on the quantised images."""
    pair = make_pair(40, 30, 12, segments=3, seed=9)
    left = pair.left.astype(np.float32) / np.float32(255.0)
    right = pair.right.astype(np.float32) / np.float32(255.0)
    cl, cr, al = soft.features(left, right, soft.SoftParams())
    ref = oracle.disparity(pair.left, pair.right, 12)
    assert np.array_equal(cl, ref["census_l"])
    assert np.array_equal(cr, ref["census_r"])
    assert np.array_equal(al, ref["arms_l"])
