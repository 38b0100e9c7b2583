/*
 * CPU oracle for the stereo-matching path of Chang & Maruyama,
 * "Real-Time High-Quality Stereo Matching System on a GPU" (arXiv 2212.00488).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or constant with the GPU library.
 *
 * Every quantity is computed from its definition: region sums are explicit
 * loops over the cross arms (no prefix sums), the winner-take-all is a full
 * scan over d, the median sorts nine values.  Floating point appears only in
 * the two cost tables, which are built in double precision from exp().
 *
 * Readings of points the paper leaves open (each listed in the design notes):
 *   gray      G = (77 R + 150 G + 29 B + 128) >> 8            (Sec. III, step 1)
 *   downscale round-half-up mean of the 3x3 block at (2x, 2y), clamped
 *             borders, X = ceil(W/2), Y = ceil(H/2)              (Eq. 2, Step1)
 *   census    6 neighbours (-1,-1) (+1,-1) (-2,0) (+2,0) (-1,+1) (+1,+1),
 *             bit k = [neighbour < centre], clamped borders       (Sec. III-B)
 *   costs     fixed point: S(1 - exp(-(a/255)/lambda_AD)) and
 *             S(1 - exp(-h/lambda_MC)), rounded half up           (Eq. 3-5)
 *             C = C_max = LUT_AD[255] + LUT_MC[6] where x - d < 0
 *   arms      per side, capped at arm_x / arm_y and at the border, strict
 *             |I(x+t) - I(x)| < delta against the centre          (Sec. III-C)
 *   WTA       smallest d among the minima                          (Eq. 9, Step5)
 *   median    3x3, clamped borders, 5th of 9                       (Sec. III step 7)
 *   fill      linear interpolation toward the right GCP, rounded half up with
 *             floor division; ties of the colour test go right   (Sec. III-E, Eq. 11)
 *   upscale   x2 disparity; odd columns by the bilateral rule on full-res
 *             gray; odd rows the rounded-up mean                  (Step8)
 * Variants of Sec. III-E and Sec. V:
 *   fill mode 1: the GCP closer in distance (the right one at equal
 *             distance); mode 2: the smaller of the two disparities; one
 *             side only: copy it; none: 0                         (Sec. III-E)
 *   arm_x_r   horizontal arm cap of the right image, W_y common    (Sec. V)
 *   full_res  no downscale and no upscale: the method on the original
 *             images over the whole range [0, Dmax-1]            (Sec. V)
 *
 * Parity status of each function is stated in its comment.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
static int absi(int v) { return v < 0 ? -v : v; }

/* floor(a / b) for b > 0; C's '/' truncates toward zero. */
static int floordiv(int a, int b) {
  int q = a / b;
  if ((a % b != 0) && (a < 0)) q -= 1;
  return q;
}

/* ---------------------------------------------------------------- tables */

/* Eq. 4 and Eq. 5 in fixed point with scale S.  AD is taken on brightness
 * normalised to [0,1] (a / 255), the only reading under which lambda_AD = 0.3
 * (Sec. V) does not saturate after two grey levels.  Pinned by bounds of
 * 1 - exp(-t) and by an independent recomputation in the brute-force suite. */
void or_lut(double lambda_ad, double lambda_mc, int S,
            uint16_t lut_ad[256], uint16_t lut_mc[7]) {
  for (int a = 0; a < 256; ++a) {
    double v = (double)S * (1.0 - exp(-((double)a / 255.0) / lambda_ad));
    lut_ad[a] = (uint16_t)floor(v + 0.5);
  }
  for (int h = 0; h <= 6; ++h) {
    double v = (double)S * (1.0 - exp(-(double)h / lambda_mc));
    lut_mc[h] = (uint16_t)floor(v + 0.5);
  }
}

/* ------------------------------------------------------ a1: gray + scale */

/* Sec. III step 1: the input images are gray-scaled.  Pinned: G(c,c,c) = c. */
void or_gray(const uint8_t* rgb, int W, int H, uint8_t* g) {
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const uint8_t* p = rgb + ((size_t)y * W + x) * 3;
      g[(size_t)y * W + x] = (uint8_t)((77 * p[0] + 150 * p[1] + 29 * p[2] + 128) >> 8);
    }
}

/* Eq. 2 with K = 2, m = 1: mean of the 3x3 block centred on (2x, 2y)
 * (Step1: pixels with even coordinates and their 8 neighbours).
 * Pinned: constant image, brute force, shift commutation. */
void or_downscale(const uint8_t* g, int W, int H, uint8_t* h) {
  int X = (W + 1) / 2, Y = (H + 1) / 2;
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      int s = 0;
      for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i)
          s += g[(size_t)clampi(2 * y + j, 0, H - 1) * W + clampi(2 * x + i, 0, W - 1)];
      h[(size_t)y * X + x] = (uint8_t)((s + 4) / 9);
    }
}

/* ---------------------------------------------------- a2: census + arms */

static const int census_dx[6] = {-1, +1, -2, +2, -1, +1};
static const int census_dy[6] = {-1, -1, 0, 0, +1, +1};

/* Sec. III-B: the centre is compared with six neighbours, giving 6 bits.
 * The pattern figure is lost; the reading keeps the three-row window the
 * implementation section caches.  Pinned: hand-made example, flat image,
 * brute force. */
void or_census(const uint8_t* h, int X, int Y, uint8_t* c) {
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      int ctr = h[(size_t)y * X + x], bits = 0;
      for (int k = 0; k < 6; ++k) {
        int v = h[(size_t)clampi(y + census_dy[k], 0, Y - 1) * X + clampi(x + census_dx[k], 0, X - 1)];
        if (v < ctr) bits |= 1 << k;
      }
      c[(size_t)y * X + x] = (uint8_t)bits;
    }
}

/* Sec. III-C: m, n (M, N) count the contiguous pixels left/right (up/down)
 * whose brightness differs from the centre by less than delta, at most
 * arm_x (arm_y) per side and never past the border.
 * Output layout [Y][X][4] = m, n, M, N.  Pinned: the verbal example
 * (m = n = 3 for seven similar pixels), edge property, flat image. */
void or_arms(const uint8_t* h, int X, int Y, int delta, int arm_x, int arm_y,
             uint8_t* arms) {
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      int c = h[(size_t)y * X + x];
      int m = 0, n = 0, M = 0, N = 0;
      while (m < arm_x && x - m - 1 >= 0 && absi(h[(size_t)y * X + x - m - 1] - c) < delta) ++m;
      while (n < arm_x && x + n + 1 < X && absi(h[(size_t)y * X + x + n + 1] - c) < delta) ++n;
      while (M < arm_y && y - M - 1 >= 0 && absi(h[(size_t)(y - M - 1) * X + x] - c) < delta) ++M;
      while (N < arm_y && y + N + 1 < Y && absi(h[(size_t)(y + N + 1) * X + x] - c) < delta) ++N;
      uint8_t* a = arms + ((size_t)y * X + x) * 4;
      a[0] = (uint8_t)m; a[1] = (uint8_t)n; a[2] = (uint8_t)M; a[3] = (uint8_t)N;
    }
}

/* ------------------------------------------------------------ a3: costs */

/* Eq. 3-5: C^L(x,y,d) = LUT_AD[|L(x,y) - R(x-d,y)|] + LUT_MC[popcount of the
 * XOR of the two census strings], and C_max where x - d < 0.
 * Pinned: brute force with an independent table. */
void or_cost_left(const uint8_t* hl, const uint8_t* hr, const uint8_t* cl,
                  const uint8_t* cr, int X, int Y, int d,
                  const uint16_t* lut_ad, const uint16_t* lut_mc, uint16_t* out) {
  int cmax = lut_ad[255] + lut_mc[6];
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      size_t i = (size_t)y * X + x;
      if (x - d < 0) { out[i] = (uint16_t)cmax; continue; }
      int ad = absi(hl[i] - hr[i - d]);
      int hx = cl[i] ^ cr[i - d], hd = 0;
      for (int b = 0; b < 6; ++b) hd += (hx >> b) & 1;
      out[i] = (uint16_t)(lut_ad[ad] + lut_mc[hd]);
    }
}

/* Eq. 6: C^R(x,y,d) = C^L(x+d,y,d); C_max where x + d >= X.
 * Pinned: the right-based cost computed directly from R(x) and L(x+d). */
void or_cost_right_from_left(const uint16_t* cost_left, int X, int Y, int d,
                             int cmax, uint16_t* out) {
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x)
      out[(size_t)y * X + x] = (x + d < X) ? cost_left[(size_t)y * X + x + d] : (uint16_t)cmax;
}

/* ------------------------------------------------------ a4/a5: aggregate */

/* Eq. 7: CA_x(x,y) = sum over t in [-m, n] of C(x+t, y). Explicit loop. */
void or_agg_x(const uint16_t* cost, const uint8_t* arms, int X, int Y, uint32_t* cax) {
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      const uint8_t* a = arms + ((size_t)y * X + x) * 4;
      uint32_t s = 0;
      for (int t = -(int)a[0]; t <= (int)a[1]; ++t) s += cost[(size_t)y * X + x + t];
      cax[(size_t)y * X + x] = s;
    }
}

/* Eq. 8: CA(x,y) = sum over s in [-M, N] of CA_x(x, y+s), with the vertical
 * arms of (x,y) and each row's own horizontal arms (already in CA_x). */
void or_agg_y(const uint32_t* cax, const uint8_t* arms, int X, int Y, uint32_t* ca) {
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      const uint8_t* a = arms + ((size_t)y * X + x) * 4;
      uint32_t s = 0;
      for (int t = -(int)a[2]; t <= (int)a[3]; ++t) s += cax[(size_t)(y + t) * X + x];
      ca[(size_t)y * X + x] = s;
    }
}

/* ------------------------------------------------------------- a5: WTA */

/* Eq. 9 read as argmin (Step5 keeps the first d with a strictly smaller
 * aggregate, so the smallest d wins ties).  Both base images.  mincost_* may
 * be NULL.  Uses OpenMP over rows inside each plane (a parallel-for, no
 * reordering of any sum). */
static void agg_plane_omp(const uint16_t* cost, const uint8_t* arms, int X, int Y,
                          uint32_t* cax, uint32_t* ca) {
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      const uint8_t* a = arms + ((size_t)y * X + x) * 4;
      uint32_t s = 0;
      for (int t = -(int)a[0]; t <= (int)a[1]; ++t) s += cost[(size_t)y * X + x + t];
      cax[(size_t)y * X + x] = s;
    }
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      const uint8_t* a = arms + ((size_t)y * X + x) * 4;
      uint32_t s = 0;
      for (int t = -(int)a[2]; t <= (int)a[3]; ++t) s += cax[(size_t)(y + t) * X + x];
      ca[(size_t)y * X + x] = s;
    }
}

int or_wta(const uint8_t* hl, const uint8_t* hr, const uint8_t* cl, const uint8_t* cr,
           const uint8_t* arms_l, const uint8_t* arms_r, int X, int Y, int D,
           const uint16_t* lut_ad, const uint16_t* lut_mc,
           int16_t* disp_l, int16_t* disp_r, uint32_t* mincost_l, uint32_t* mincost_r) {
  size_t n = (size_t)X * Y;
  int cmax = lut_ad[255] + lut_mc[6];
  uint16_t* cL = malloc(n * sizeof(uint16_t));
  uint16_t* cR = malloc(n * sizeof(uint16_t));
  uint32_t* tmp = malloc(n * sizeof(uint32_t));
  uint32_t* caL = malloc(n * sizeof(uint32_t));
  uint32_t* caR = malloc(n * sizeof(uint32_t));
  uint32_t* bestL = malloc(n * sizeof(uint32_t));
  uint32_t* bestR = malloc(n * sizeof(uint32_t));
  if (!cL || !cR || !tmp || !caL || !caR || !bestL || !bestR) {
    free(cL); free(cR); free(tmp); free(caL); free(caR); free(bestL); free(bestR);
    return -2;
  }
  for (size_t i = 0; i < n; ++i) {
    bestL[i] = UINT32_MAX; bestR[i] = UINT32_MAX; disp_l[i] = 0; disp_r[i] = 0;
  }
  for (int d = 0; d < D; ++d) {
    or_cost_left(hl, hr, cl, cr, X, Y, d, lut_ad, lut_mc, cL);
    or_cost_right_from_left(cL, X, Y, d, cmax, cR);
    agg_plane_omp(cL, arms_l, X, Y, tmp, caL);
    agg_plane_omp(cR, arms_r, X, Y, tmp, caR);
    for (size_t i = 0; i < n; ++i) {
      if (caL[i] < bestL[i]) { bestL[i] = caL[i]; disp_l[i] = (int16_t)d; }
      if (caR[i] < bestR[i]) { bestR[i] = caR[i]; disp_r[i] = (int16_t)d; }
    }
  }
  if (mincost_l) memcpy(mincost_l, bestL, n * sizeof(uint32_t));
  if (mincost_r) memcpy(mincost_r, bestR, n * sizeof(uint32_t));
  free(cL); free(cR); free(tmp); free(caL); free(caR); free(bestL); free(bestR);
  return 0;
}

/* ------------------------------------------------------ a6: cross-check */

/* Eq. 10: (x,y) is a ground control point iff, with k = D^L(x,y),
 * x - k >= 0 and D^R(x-k, y) = k.  Pinned: constant-shift pair. */
void or_crosscheck(const int16_t* dl, const int16_t* dr, int X, int Y, uint8_t* gcp) {
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      int k = dl[(size_t)y * X + x];
      gcp[(size_t)y * X + x] = (uint8_t)(x - k >= 0 && dr[(size_t)y * X + x - k] == k);
    }
}

/* ------------------------------------------------ a7: median + bilateral */

/* Sec. III step 7: median filter, read as 3x3 with clamped borders.
 * Pinned: numpy.median of the nine values. */
void or_median(const int16_t* din, int X, int Y, int16_t* out) {
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      int v[9], k = 0;
      for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i)
          v[k++] = din[(size_t)clampi(y + j, 0, Y - 1) * X + clampi(x + i, 0, X - 1)];
      for (int a = 1; a < 9; ++a) {          /* insertion sort */
        int t = v[a], b = a - 1;
        while (b >= 0 && v[b] > t) { v[b + 1] = v[b]; --b; }
        v[b + 1] = t;
      }
      out[(size_t)y * X + x] = (int16_t)v[4];
    }
}

/* Sec. III-E (bilateral estimation).  GCPs keep the median value.  A
 * non-GCP takes the nearest GCPs left (x-i) and right (x+j) in its row; if
 * their median disparities differ by at most T it is interpolated linearly
 * from the left value toward the right one (Eq. 11 with its sign read so
 * that the line reaches D(x+j) at i = i+j), rounded half up; otherwise it
 * copies the side whose brightness is strictly closer, the right one on a
 * tie.  One side only: copy it.  No GCP in the row: 0.
 * Pinned: all-GCP map, linear ramp, step edge, brute force. */
void or_fill(const int16_t* med, const uint8_t* gcp, const uint8_t* hl,
             int X, int Y, int T, int mode, int16_t* out) {
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      size_t r = (size_t)y * X;
      if (gcp[r + x]) { out[r + x] = med[r + x]; continue; }
      int i = 1, j = 1;
      while (x - i >= 0 && !gcp[r + x - i]) ++i;
      while (x + j < X && !gcp[r + x + j]) ++j;
      int hasl = x - i >= 0, hasr = x + j < X, v;
      if (hasl && hasr && mode == 1) {
        v = i < j ? med[r + x - i] : med[r + x + j];
      } else if (hasl && hasr && mode == 2) {
        int dlv = med[r + x - i], drv = med[r + x + j];
        v = dlv < drv ? dlv : drv;
      } else if (hasl && hasr) {
        int dlv = med[r + x - i], drv = med[r + x + j];
        if (absi(dlv - drv) <= T) {
          v = dlv + floordiv(2 * i * (drv - dlv) + (i + j), 2 * (i + j));
        } else {
          int c = hl[r + x];
          v = (absi(hl[r + x - i] - c) < absi(hl[r + x + j] - c)) ? dlv : drv;
        }
      } else if (hasl) {
        v = med[r + x - i];
      } else if (hasr) {
        v = med[r + x + j];
      } else {
        v = 0;
      }
      out[r + x] = (int16_t)v;
    }
}

/* ---------------------------------------------------------- a8: upscale */

/* Step8: back to W x H.  Disparities double.  Along x the bilateral rule is
 * used again: an odd column between half-res neighbours Dl, Dr takes their
 * exact doubled mean Dl + Dr if |Dl - Dr| <= T, else the doubled value of the
 * side whose full-res gray is strictly closer (right on a tie).  Along y the
 * odd rows are the rounded-up mean of the rows above and below.  A last odd
 * column or row with no neighbour copies.  Pinned: constant map, brute force. */
void or_upscale(const int16_t* dp, const uint8_t* gfull, int W, int H, int T, int16_t* out) {
  int X = (W + 1) / 2, Y = (H + 1) / 2;
  int16_t* u = malloc((size_t)W * Y * sizeof(int16_t));
  if (!u) return;
  for (int y = 0; y < Y; ++y) {
    const uint8_t* g = gfull + (size_t)(2 * y) * W;
    for (int xo = 0; xo < W; ++xo) {
      int x = xo / 2, v;
      if ((xo & 1) == 0) {
        v = 2 * dp[(size_t)y * X + x];
      } else if (x + 1 >= X) {
        v = 2 * dp[(size_t)y * X + x];
      } else {
        int dlv = dp[(size_t)y * X + x], drv = dp[(size_t)y * X + x + 1];
        if (absi(dlv - drv) <= T) {
          v = dlv + drv;
        } else {
          int c = g[xo];
          v = (absi(g[xo - 1] - c) < absi(g[xo + 1] - c)) ? 2 * dlv : 2 * drv;
        }
      }
      u[(size_t)y * W + xo] = (int16_t)v;
    }
  }
  for (int yo = 0; yo < H; ++yo) {
    int y = yo / 2;
    for (int xo = 0; xo < W; ++xo) {
      int v;
      if ((yo & 1) == 0 || y + 1 >= Y) v = u[(size_t)y * W + xo];
      else v = (u[(size_t)y * W + xo] + u[(size_t)(y + 1) * W + xo] + 1) >> 1;
      out[(size_t)yo * W + xo] = (int16_t)v;
    }
  }
  free(u);
}

/* ------------------------------------------------------- whole pipeline */

/* Runs every step in the paper's order on one pair of W x H RGB images with
 * maximum full-resolution disparity Dmax (D = ceil(Dmax/2) at half res).
 * Any intermediate pointer may be NULL.  Returns 0, or -1 on bad sizes,
 * -2 on allocation failure. */
int or_disparity(const uint8_t* left_rgb, const uint8_t* right_rgb, int W, int H, int Dmax,
                 double lambda_ad, double lambda_mc, int S, int delta, int arm_x, int arm_y,
                 int T, int arm_x_r, int fill_mode, int full_res, int16_t* out,
                 uint8_t* o_half_l, uint8_t* o_half_r, uint8_t* o_census_l, uint8_t* o_census_r,
                 uint8_t* o_arms_l, uint8_t* o_arms_r, int16_t* o_disp_l, int16_t* o_disp_r,
                 uint32_t* o_min_l, uint32_t* o_min_r, uint8_t* o_gcp, int16_t* o_median,
                 int16_t* o_filled) {
  if (W < 2 || H < 2 || Dmax < 1) return -1;
  /* full resolution: no downscale (K = 1), the whole disparity range, no upscale */
  int X = full_res ? W : (W + 1) / 2, Y = full_res ? H : (H + 1) / 2;
  int D = full_res ? Dmax : (Dmax + 1) / 2;
  size_t nf = (size_t)W * H, nh = (size_t)X * Y;
  uint16_t lut_ad[256], lut_mc[7];
  or_lut(lambda_ad, lambda_mc, S, lut_ad, lut_mc);
  uint8_t* gl = malloc(nf);
  uint8_t* gr = malloc(nf);
  uint8_t* hl = malloc(nh);
  uint8_t* hr = malloc(nh);
  uint8_t* cl = malloc(nh);
  uint8_t* cr = malloc(nh);
  uint8_t* al = malloc(nh * 4);
  uint8_t* ar = malloc(nh * 4);
  int16_t* dl = malloc(nh * 2);
  int16_t* dr = malloc(nh * 2);
  uint8_t* gc = malloc(nh);
  int16_t* md = malloc(nh * 2);
  int16_t* fl = malloc(nh * 2);
  int rc = -2;
  if (!gl || !gr || !hl || !hr || !cl || !cr || !al || !ar || !dl || !dr || !gc || !md || !fl)
    goto done;
  or_gray(left_rgb, W, H, gl);
  or_gray(right_rgb, W, H, gr);
  if (full_res) {
    memcpy(hl, gl, nh);
    memcpy(hr, gr, nh);
  } else {
    or_downscale(gl, W, H, hl);
    or_downscale(gr, W, H, hr);
  }
  or_census(hl, X, Y, cl);
  or_census(hr, X, Y, cr);
  or_arms(hl, X, Y, delta, arm_x, arm_y, al);
  or_arms(hr, X, Y, delta, arm_x_r, arm_y, ar);
  rc = or_wta(hl, hr, cl, cr, al, ar, X, Y, D, lut_ad, lut_mc, dl, dr, o_min_l, o_min_r);
  if (rc) goto done;
  or_crosscheck(dl, dr, X, Y, gc);
  or_median(dl, X, Y, md);
  or_fill(md, gc, hl, X, Y, T, fill_mode, fl);
  if (full_res)
    memcpy(out, fl, nh * 2);
  else
    or_upscale(fl, gl, W, H, T, out);
  if (o_half_l) memcpy(o_half_l, hl, nh);
  if (o_half_r) memcpy(o_half_r, hr, nh);
  if (o_census_l) memcpy(o_census_l, cl, nh);
  if (o_census_r) memcpy(o_census_r, cr, nh);
  if (o_arms_l) memcpy(o_arms_l, al, nh * 4);
  if (o_arms_r) memcpy(o_arms_r, ar, nh * 4);
  if (o_disp_l) memcpy(o_disp_l, dl, nh * 2);
  if (o_disp_r) memcpy(o_disp_r, dr, nh * 2);
  if (o_gcp) memcpy(o_gcp, gc, nh);
  if (o_median) memcpy(o_median, md, nh * 2);
  if (o_filled) memcpy(o_filled, fl, nh * 2);
  rc = 0;
done:
  free(gl); free(gr); free(hl); free(hr); free(cl); free(cr); free(al); free(ar);
  free(dl); free(dr); free(gc); free(md); free(fl);
  return rc;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the OpenMP loops of later calls (benchmark timing only). */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
