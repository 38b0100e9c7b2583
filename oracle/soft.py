"""Plain FP64 statement of the differentiable soft-argmin head.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  Nothing here is shared
with the GPU library.

The head keeps the paper's matching cost and cross-based aggregation
(Eq. 3-5, 7-8) in floating point, so that the disparity is a smooth
function of the image intensities and of the two cost weights; the census
strings and the cross arms (Sec. III-B, III-C) are integer features, frozen
(not differentiated).  Readings taken where the paper has no such head:

* input: RGB float in [0, 1] per pair; gray = (77 R + 150 G + 29 B) / 256,
  the same weights as the integer path, unrounded; half image = the mean of
  the 3x3 block at (2x, 2y), borders clamped (Eq. 2, K = 2), unrounded;
* frozen features: each channel is quantised to q = floor(255 v + 1/2)
  (clamped to 0..255) in float32 arithmetic, and the integer path's gray,
  downscale, census and arms are taken of q;
* cost (the robust combination of Eq. 3-5 on the 0..255 brightness scale):
  C = (1 - exp(-AD / lambda_AD)) + (1 - exp(-H / lambda_census)) with
  AD = 255 |L(x,y) - R(x-d,y)|, H the census Hamming distance; C = 2 where
  x - d < 0; d in [0, D-1], D = ceil(Dmax / 2);
* aggregation: CA = sum of C over the cross region of the left pixel
  (Eq. 7 then Eq. 8), divided by the region's pixel count |S(x,y)|;
* soft-argmin: p_d = softmax over d of -CA_mean / tau, d_hat = sum d p_d
  (half-resolution units);
* loss: the mean over pixels with a non-occluded full-resolution ground
  truth at (2x, 2y) of |2 d_hat - GT(2x, 2y)|.

Gradients come from torch's autograd over these float64 CPU operations; the
tests pin them with central finite differences.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

import oracle

F64 = torch.float64


@dataclass
class SoftParams:
    lambda_ad: float = 10.0
    lambda_census: float = 30.0
    tau: float = 0.1
    color_delta: int = 13
    arm_x: int = 21
    arm_y: int = 31


def quantize(rgb: np.ndarray) -> np.ndarray:
    """q = floor(255 v + 1/2) clamped to 0..255, each step in float32."""
    v = np.asarray(rgb, dtype=np.float32)
    t = np.float32(255.0) * v
    t = t + np.float32(0.5)
    return np.clip(np.floor(t), 0, 255).astype(np.uint8)


def features(left: np.ndarray, right: np.ndarray, p: SoftParams):
    """Frozen integer features of one float pair: census of both half images
    and the arms of the left one, as [Y][X] and [Y][X][4] (m, n, M, N)."""
    ip = oracle.Params(color_delta=p.color_delta, arm_x=p.arm_x, arm_y=p.arm_y)
    hl = oracle.downscale(oracle.gray(quantize(left)))
    hr = oracle.downscale(oracle.gray(quantize(right)))
    return oracle.census(hl), oracle.census(hr), oracle.arms(hl, ip)


def gray_f(rgb: torch.Tensor) -> torch.Tensor:
    return (77.0 * rgb[..., 0] + 150.0 * rgb[..., 1] + 29.0 * rgb[..., 2]) / 256.0


def downscale_f(g: torch.Tensor) -> torch.Tensor:
    """Mean of the 3x3 block centred on (2x, 2y), borders clamped."""
    H, W = g.shape
    X, Y = (W + 1) // 2, (H + 1) // 2
    out = torch.zeros((Y, X), dtype=g.dtype)
    ys = torch.arange(Y) * 2
    xs = torch.arange(X) * 2
    for j in (-1, 0, 1):
        rows = torch.clamp(ys + j, 0, H - 1)
        for i in (-1, 0, 1):
            cols = torch.clamp(xs + i, 0, W - 1)
            out = out + g[rows][:, cols]
    return out / 9.0


def popcount6(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.int64)
    return sum((v >> k) & 1 for k in range(6))


def cost_volume(hl, hr, cl, cr, D, lam_ad, lam_census):
    """C[d][y][x] of the left base (Eq. 3-5 in the head's robust form)."""
    Y, X = hl.shape
    vols = []
    for d in range(D):
        c = torch.full((Y, X), 2.0, dtype=F64)
        if d < X:
            ad = 255.0 * torch.abs(hl[:, d:] - hr[:, :X - d])
            ham = torch.from_numpy(popcount6(cl[:, d:] ^ cr[:, :X - d])).to(F64)
            valid = (1.0 - torch.exp(-ad / lam_ad)) + (1.0 - torch.exp(-ham / lam_census))
            c = torch.cat([c[:, :d], valid], dim=1)
        vols.append(c)
    return torch.stack(vols)


def agg_x(v: torch.Tensor, m: np.ndarray, n: np.ndarray, cap: int) -> torch.Tensor:
    """Eq. 7: sum over t in [-m(x,y), n(x,y)] of v[..., y, x + t]."""
    X = v.shape[-1]
    mt, nt = torch.from_numpy(m.astype(np.int64)), torch.from_numpy(n.astype(np.int64))
    out = torch.zeros_like(v)
    for t in range(-cap, cap + 1):
        inside = (t >= -mt) & (t <= nt)
        if not bool(inside.any()):
            continue
        shifted = torch.zeros_like(v)
        if t >= 0:
            shifted[..., :X - t] = v[..., t:]
        else:
            shifted[..., -t:] = v[..., :X + t]
        out = out + torch.where(inside, shifted, torch.zeros_like(shifted))
    return out


def agg_y(v: torch.Tensor, M: np.ndarray, N: np.ndarray, cap: int) -> torch.Tensor:
    """Eq. 8: sum over s in [-M(x,y), N(x,y)] of v[..., y + s, x]."""
    Y = v.shape[-2]
    Mt, Nt = torch.from_numpy(M.astype(np.int64)), torch.from_numpy(N.astype(np.int64))
    out = torch.zeros_like(v)
    for s in range(-cap, cap + 1):
        inside = (s >= -Mt) & (s <= Nt)
        if not bool(inside.any()):
            continue
        shifted = torch.zeros_like(v)
        if s >= 0:
            shifted[..., :Y - s, :] = v[..., s:, :]
        else:
            shifted[..., -s:, :] = v[..., :Y + s, :]
        out = out + torch.where(inside, shifted, torch.zeros_like(shifted))
    return out


def forward(left, right, dmax: int, lam_ad, lam_census, p: SoftParams, feats=None):
    """d_hat [Y][X] (float64 tensor) of one pair.

    left, right: float64 tensors [H][W][3] (may require grad); lam_ad and
    lam_census: float64 scalar tensors (may require grad); feats: the frozen
    features of the pair (computed from the float32 values when None).
    Returns a dict with d_hat and the intermediates (half images, cost
    volume, aggregate, support size, probabilities).
    """
    if feats is None:
        feats = features(left.detach().to(torch.float32).numpy(),
                         right.detach().to(torch.float32).numpy(), p)
    cl, cr, arms = feats
    m, n, M, N = (arms[..., k] for k in range(4))
    D = (dmax + 1) // 2
    hl = downscale_f(gray_f(left))
    hr = downscale_f(gray_f(right))
    C = cost_volume(hl, hr, cl, cr, D, lam_ad, lam_census)
    CA = agg_y(agg_x(C, m, n, p.arm_x), M, N, p.arm_y)
    size = agg_y(agg_x(torch.ones(hl.shape, dtype=F64), m, n, p.arm_x), M, N, p.arm_y)
    mean = CA / size
    prob = torch.softmax(-mean / p.tau, dim=0)
    dv = torch.arange(D, dtype=F64).view(D, 1, 1)
    d_hat = (dv * prob).sum(dim=0)
    return {"d_hat": d_hat, "half_l": hl, "half_r": hr, "cost": C, "agg": CA,
            "size": size, "prob": prob}


def l1_loss(d_hat: torch.Tensor, gt: np.ndarray, nonocc: np.ndarray) -> torch.Tensor:
    """Mean of |2 d_hat(x,y) - GT(2x,2y)| over non-occluded (2x, 2y)."""
    g = torch.from_numpy(np.asarray(gt)[::2, ::2].astype(np.float64))
    mask = torch.from_numpy(np.asarray(nonocc)[::2, ::2].astype(bool))
    diff = torch.abs(2.0 * d_hat - g)
    return diff[mask].sum() / max(int(mask.sum()), 1)


def loss_and_grads(lefts, rights, gts, nonoccs, dmax: int, p: SoftParams):
    """Mean over the batch of the per-pair L1 losses, and its gradient with
    respect to both images of every pair and the two cost weights.

    lefts, rights: float32 arrays [n][H][W][3].  Returns (loss, g_left,
    g_right, g_lambda) as float64 numpy values, g_lambda = (d/d lambda_AD,
    d/d lambda_census).
    """
    lam_ad = torch.tensor(p.lambda_ad, dtype=F64, requires_grad=True)
    lam_c = torch.tensor(p.lambda_census, dtype=F64, requires_grad=True)
    ls = [torch.tensor(np.asarray(l, np.float64), requires_grad=True) for l in lefts]
    rs = [torch.tensor(np.asarray(r, np.float64), requires_grad=True) for r in rights]
    total = 0.0
    for i in range(len(ls)):
        feats = features(np.asarray(lefts[i], np.float32), np.asarray(rights[i], np.float32), p)
        out = forward(ls[i], rs[i], dmax, lam_ad, lam_c, p, feats)
        total = total + l1_loss(out["d_hat"], gts[i], nonoccs[i])
    loss = total / len(ls)
    loss.backward()
    return (float(loss.detach()), np.stack([l.grad.numpy() for l in ls]),
            np.stack([r.grad.numpy() for r in rs]),
            np.array([float(lam_ad.grad), float(lam_c.grad)]))


def loss_value(lefts, rights, gts, nonoccs, dmax: int, p: SoftParams, feats=None) -> float:
    """The batch loss alone (no autograd), for finite differences; feats may
    hold the frozen features per pair so that a perturbation that would flip
    a quantised value does not change them."""
    total = 0.0
    with torch.no_grad():
        for i in range(len(lefts)):
            f = feats[i] if feats is not None else None
            out = forward(torch.as_tensor(np.asarray(lefts[i], np.float64)),
                          torch.as_tensor(np.asarray(rights[i], np.float64)), dmax,
                          torch.tensor(p.lambda_ad, dtype=F64),
                          torch.tensor(p.lambda_census, dtype=F64), p, f)
            total += float(l1_loss(out["d_hat"], gts[i], nonoccs[i]))
    return total / len(lefts)
