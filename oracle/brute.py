"""Pure-Python brute force of the stereo path, for tiny inputs only.

TEST INFRASTRUCTURE ONLY.  A second, deliberately naive statement of each
step, used to pin the C oracle.  It differs in form from the C code where
that can expose a slip:

* the cost tables come from ``math.exp``;
* arms are the largest k such that *every* pixel up to k passes the test;
* the right-based cost is computed directly from R(x) and L(x+d), not
  through the identity of Eq. 6;
* the aggregate is a sum over the explicit set of pixels of the cross
  region (each row segment of the vertical arm), not two passes;
* the winner-take-all is ``min`` over (cost, d) tuples.
"""

from __future__ import annotations

import math
from fractions import Fraction

CENSUS_PATTERN = ((-1, -1), (1, -1), (-2, 0), (2, 0), (-1, 1), (1, 1))


def clamp(v, lo, hi):
    return max(lo, min(hi, v))


def tables(lambda_ad, lambda_mc, S):
    ad = [math.floor(S * (1.0 - math.exp(-(a / 255.0) / lambda_ad)) + 0.5) for a in range(256)]
    mc = [math.floor(S * (1.0 - math.exp(-h / lambda_mc)) + 0.5) for h in range(7)]
    return ad, mc


def gray(rgb):
    return [[(77 * int(p[0]) + 150 * int(p[1]) + 29 * int(p[2]) + 128) // 256 for p in row]
            for row in rgb]


def downscale(g):
    H, W = len(g), len(g[0])
    X, Y = (W + 1) // 2, (H + 1) // 2
    out = [[0] * X for _ in range(Y)]
    for y in range(Y):
        for x in range(X):
            vals = [g[clamp(2 * y + j, 0, H - 1)][clamp(2 * x + i, 0, W - 1)]
                    for j in (-1, 0, 1) for i in (-1, 0, 1)]
            q, r = divmod(sum(vals), 9)          # mean, rounded half up
            out[y][x] = q + (1 if 2 * r >= 9 else 0)
    return out


def census(h):
    Y, X = len(h), len(h[0])
    out = [[0] * X for _ in range(Y)]
    for y in range(Y):
        for x in range(X):
            bits = 0
            for k, (dx, dy) in enumerate(CENSUS_PATTERN):
                if h[clamp(y + dy, 0, Y - 1)][clamp(x + dx, 0, X - 1)] < h[y][x]:
                    bits += 2 ** k
            out[y][x] = bits
    return out


def arm_len(h, x, y, ddx, ddy, cap, delta):
    Y, X = len(h), len(h[0])
    best = 0
    for k in range(cap + 1):
        cells = [(x + ddx * t, y + ddy * t) for t in range(1, k + 1)]
        if all(0 <= cx < X and 0 <= cy < Y and abs(h[cy][cx] - h[y][x]) < delta
               for cx, cy in cells):
            best = k
    return best


def arms(h, delta, ax, ay):
    Y, X = len(h), len(h[0])
    return [[(arm_len(h, x, y, -1, 0, ax, delta), arm_len(h, x, y, 1, 0, ax, delta),
              arm_len(h, x, y, 0, -1, ay, delta), arm_len(h, x, y, 0, 1, ay, delta))
             for x in range(X)] for y in range(Y)]


def popcount(v):
    return bin(v).count("1")


def pixel_cost(b, cb, o, co, tad, tmc):
    return tad[abs(b - o)] + tmc[popcount(cb ^ co)]


def cost_l(hl, hr, cl, cr, x, y, d, tad, tmc):
    if x - d < 0:
        return tad[255] + tmc[6]
    return pixel_cost(hl[y][x], cl[y][x], hr[y][x - d], cr[y][x - d], tad, tmc)


def cost_r(hl, hr, cl, cr, x, y, d, tad, tmc):
    X = len(hl[0])
    if x + d >= X:
        return tad[255] + tmc[6]
    return pixel_cost(hr[y][x], cr[y][x], hl[y][x + d], cl[y][x + d], tad, tmc)


def cross_region(a, x, y):
    """Pixels of the cross region of (x, y): each row of the vertical arm,
    spanned by that row's own horizontal arms."""
    m, n, M, N = a[y][x][0], a[y][x][1], a[y][x][2], a[y][x][3]
    cells = []
    for s in range(-M, N + 1):
        r = a[y + s][x]
        cells.extend((x + t, y + s) for t in range(-r[0], r[1] + 1))
    return cells


def aggregate(costfn, a, x, y, d):
    return sum(costfn(cx, cy, d) for cx, cy in cross_region(a, x, y))


def wta(hl, hr, cl, cr, al, ar, D, tad, tmc):
    Y, X = len(hl), len(hl[0])
    fl = lambda x, y, d: cost_l(hl, hr, cl, cr, x, y, d, tad, tmc)
    fr = lambda x, y, d: cost_r(hl, hr, cl, cr, x, y, d, tad, tmc)
    dl = [[0] * X for _ in range(Y)]
    dr = [[0] * X for _ in range(Y)]
    ml = [[0] * X for _ in range(Y)]
    mr = [[0] * X for _ in range(Y)]
    for y in range(Y):
        for x in range(X):
            bl = min((aggregate(fl, al, x, y, d), d) for d in range(D))
            br = min((aggregate(fr, ar, x, y, d), d) for d in range(D))
            ml[y][x], dl[y][x] = bl
            mr[y][x], dr[y][x] = br
    return dl, dr, ml, mr


def crosscheck(dl, dr):
    Y, X = len(dl), len(dl[0])
    return [[1 if (x - dl[y][x] >= 0 and dr[y][x - dl[y][x]] == dl[y][x]) else 0
             for x in range(X)] for y in range(Y)]


def median(d):
    Y, X = len(d), len(d[0])
    return [[sorted(d[clamp(y + j, 0, Y - 1)][clamp(x + i, 0, X - 1)]
                    for j in (-1, 0, 1) for i in (-1, 0, 1))[4]
             for x in range(X)] for y in range(Y)]


def fill(med, gcp, hl, T, mode=0):
    """mode 0: the bilateral rule; 1: the GCP nearer in distance (ties to
    the right); 2: the smaller disparity of the two."""
    Y, X = len(med), len(med[0])
    out = [[0] * X for _ in range(Y)]
    for y in range(Y):
        gx = [x for x in range(X) if gcp[y][x]]
        for x in range(X):
            if gcp[y][x]:
                out[y][x] = med[y][x]
                continue
            left = [g for g in gx if g < x]
            right = [g for g in gx if g > x]
            if left and right:
                xl, xr = left[-1], right[0]
                i, j = x - xl, xr - x
                a, b = med[y][xl], med[y][xr]
                if mode == 1:
                    out[y][x] = min((i, 1, a), (j, 0, b))[2]  # equal distance: right
                elif mode == 2:
                    out[y][x] = min(a, b)
                elif abs(a - b) <= T:
                    # a + i (b - a) / (i + j), rounded half up, in exact rationals
                    out[y][x] = math.floor(Fraction(a) + Fraction(i * (b - a), i + j)
                                           + Fraction(1, 2))
                else:
                    out[y][x] = a if abs(hl[y][xl] - hl[y][x]) < abs(hl[y][xr] - hl[y][x]) else b
            elif left:
                out[y][x] = med[y][left[-1]]
            elif right:
                out[y][x] = med[y][right[0]]
            else:
                out[y][x] = 0
    return out


def upscale(dp, gfull, T):
    H, W = len(gfull), len(gfull[0])
    Y, X = len(dp), len(dp[0])
    u = [[0] * W for _ in range(Y)]
    for y in range(Y):
        for xo in range(W):
            x = xo // 2
            if xo % 2 == 0 or x + 1 >= X:
                u[y][xo] = 2 * dp[y][x]
                continue
            a, b = dp[y][x], dp[y][x + 1]
            if abs(a - b) <= T:
                u[y][xo] = a + b
            else:
                g = gfull[2 * y]
                u[y][xo] = 2 * a if abs(g[xo - 1] - g[xo]) < abs(g[xo + 1] - g[xo]) else 2 * b
    out = [[0] * W for _ in range(H)]
    for yo in range(H):
        y = yo // 2
        for xo in range(W):
            if yo % 2 == 0 or y + 1 >= Y:
                out[yo][xo] = u[y][xo]
            else:
                out[yo][xo] = (u[y][xo] + u[y + 1][xo] + 1) // 2
    return out


def disparity(left, right, dmax, lambda_ad, lambda_mc, S, delta, ax, ay, T, ax_r=None,
              fill_mode=0, full_res=False):
    """Whole path on nested lists; returns a dict of every intermediate.
    ax_r: horizontal cap of the right image (None: ax); full_res: the method
    on the original images, whole range, no upscale."""
    tad, tmc = tables(lambda_ad, lambda_mc, S)
    gl, gr = gray(left), gray(right)
    if full_res:
        hl, hr = [row[:] for row in gl], [row[:] for row in gr]
    else:
        hl, hr = downscale(gl), downscale(gr)
    cl, cr = census(hl), census(hr)
    al, ar = arms(hl, delta, ax, ay), arms(hr, delta, ax if ax_r is None else ax_r, ay)
    D = dmax if full_res else (dmax + 1) // 2
    dl, dr, ml, mr = wta(hl, hr, cl, cr, al, ar, D, tad, tmc)
    g = crosscheck(dl, dr)
    md = median(dl)
    fl = fill(md, g, hl, T, fill_mode)
    out = [row[:] for row in fl] if full_res else upscale(fl, gl, T)
    return dict(tables=(tad, tmc), gray_l=gl, half_l=hl, half_r=hr, census_l=cl, census_r=cr,
                arms_l=al, arms_r=ar, disp_l=dl, disp_r=dr, min_l=ml, min_r=mr, gcp=g,
                median=md, filled=fl, out=out)


# ---------------------------------------------------------------- soft head
# The differentiable head's forward, pixel by pixel: float half images from
# explicit 3x3 block lists, the cost from math.exp, the aggregate as a mean
# over the explicit cross-region cell list, and the soft-argmin with the
# largest logit subtracted before math.exp.

def soft_half(rgb):
    """Float half image of float RGB rows (gray weights 77/150/29 over 256)."""
    H, W = len(rgb), len(rgb[0])
    g = [[(77.0 * p[0] + 150.0 * p[1] + 29.0 * p[2]) / 256.0 for p in row] for row in rgb]
    X, Y = (W + 1) // 2, (H + 1) // 2
    return [[sum(g[clamp(2 * y + j, 0, H - 1)][clamp(2 * x + i, 0, W - 1)]
                 for j in (-1, 0, 1) for i in (-1, 0, 1)) / 9.0
             for x in range(X)] for y in range(Y)]


def soft_cost(hl, hr, cl, cr, x, y, d, lam_ad, lam_c):
    if x - d < 0:
        return 2.0
    ad = 255.0 * abs(hl[y][x] - hr[y][x - d])
    h = popcount(cl[y][x] ^ cr[y][x - d])
    return (1.0 - math.exp(-ad / lam_ad)) + (1.0 - math.exp(-h / lam_c))


def soft_d_hat(hl, hr, cl, cr, a, D, lam_ad, lam_c, tau):
    Y, X = len(hl), len(hl[0])
    out = [[0.0] * X for _ in range(Y)]
    for y in range(Y):
        for x in range(X):
            cells = cross_region(a, x, y)
            means = [sum(soft_cost(hl, hr, cl, cr, cx, cy, d, lam_ad, lam_c)
                         for cx, cy in cells) / len(cells) for d in range(D)]
            logits = [-v / tau for v in means]
            top = max(logits)
            w = [math.exp(z - top) for z in logits]
            out[y][x] = sum(d * wd for d, wd in enumerate(w)) / sum(w)
    return out
