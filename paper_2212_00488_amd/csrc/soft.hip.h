// Device kernels of the differentiable soft-argmin head (gfx950, wave64).
//
// The head keeps the cost and the cross-based aggregation of the paper
// (Eq. 3-5, 7-8) in floating point so that the disparity is a smooth
// function of the images and of the two cost weights; the census strings
// and the cross arms (Sec. III-B, III-C) are the integer path's, taken of the
// quantised images and frozen.
//
//   forward   k_soft_prep   RGB float -> float half image, and the uint8 half
//                           image of the quantised RGB (for k_feat)
//             k_feat        census and arms (shared with the integer path),
//                           and the padded pixel planes {float half image, census}
//             k_soft_size   1 / |S(x,y)|, the cross-region pixel count
//             k_soft_agg    cost C = (1 - e^{-255|dI|/lambda_AD}) +
//                           (1 - e^{-H/lambda_census}), CA over the cross
//                           region, and the softmax sums over a d-chunk
//             k_soft_merge  d_hat = sum d e_d / sum e_d, log2 sum e_d
//             (with the weights saved, k_soft_agg also writes every e_d)
//   backward  k_soft_bprep  per-pixel constants of dL/dCA
//             k_soft_agg    (GCA mode) recomputes CA for a slab of d and
//                           writes dL/dCA planes
//             k_soft_tcol   transposed vertical window sums (integer difference
//                           arrays over bands of output rows, LDS atomics)
//             k_soft_tcolw  (weights saved by the forward) the same transpose
//                           with dL/dCA formed from the saved e_d, in place of
//                           k_soft_agg and k_soft_tcol
//             k_soft_tr     transposed horizontal window sums back to dL/dC,
//                           then dC/d(dI), dC/d(lambda) per pixel, summed over
//                           the slab into the half-image gradients
//             k_soft_gright dL/d(right half image) from the strips' partials
//             k_soft_gfull  transposed downscale and gray: dL/d(RGB)
//             k_soft_lam    fixed-order sum of the lambda partials
//   loss      k_l1_*        mean |2 d_hat - GT(2x,2y)| over non-occluded
//                           pixels, per pair, averaged over the batch
//
// Aggregation runs on costs in fixed point (C * 2^k rounded, k chosen per
// plan so that every cross-region sum stays below 2^31): the row and column
// prefix sums then wrap modulo 2^32 and every window difference is the exact
// sum of the rounded costs, whatever the prefix magnitude.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hip.h"

namespace stereo_dev {
// Internal linkage: each source of the library that launches a kernel
// carries its own copy (no relocatable device code).
namespace {

constexpr int kSoftBR = 4;  // output rows per k_soft_tr workgroup (one per wave)

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// ----------------------------------------------------------- k_soft_prep
// One thread per half-res pixel of one image (img = 2 pair + {0 left, 1 right}).
// Float path: gray = (77 R + 150 G + 29 B) / 256, half = mean of the 3x3 block
// at (2x, 2y), borders clamped.  Integer path: each channel quantised to
// floor(255 v + 1/2) in float32 (product and sum rounded separately), clamped
// to 0..255, then the integer gray and (sum + 4) / 9 as in k_prep.
// The workgroup's 64 x 4 half-res pixels cover 9 x 130 full-res pixels
// (rows 2 y0 - 1 .. 2 y0 + 7, columns 2 x0 - 1 .. 2 x0 + 128, clamped): each
// of them is loaded once (coalesced 12-byte loads, all five of a thread
// issued together) and its two grays go to LDS; each half-res pixel then sums
// its block there in the order (row, column).
// grid: (ceil(X/64), ceil(Y/4), 2n), block (64, 4).
constexpr int kPrepTW = 130, kPrepTH = 9, kPrepTN = kPrepTW * kPrepTH;
constexpr int kPrepLoads = (kPrepTN + 255) / 256;

__global__ void __launch_bounds__(256) k_soft_prep(const float* __restrict__ left,
                                                   const float* __restrict__ right, int W, int H,
                                                   int X, int Y, float* __restrict__ half_f,
                                                   uint8_t* __restrict__ half_u8) {
  __shared__ float s_f[kPrepTH][kPrepTW];
  __shared__ int s_i[kPrepTH][kPrepTW];
  const int t = threadIdx.y * 64 + threadIdx.x;
  const int x0 = blockIdx.x * 64, y0 = blockIdx.y * 4, img = blockIdx.z;
  const float* rgb = ((img & 1) ? right : left) + (size_t)(img >> 1) * H * W * 3;
  float pr[kPrepLoads][3];
  int ti[kPrepLoads];
#pragma unroll
  for (int k = 0; k < kPrepLoads; ++k) {
    ti[k] = min(t + 256 * k, kPrepTN - 1);  // past the tile: repeats its last pixel
    const int r = ti[k] / kPrepTW, c = ti[k] - r * kPrepTW;
    const float* p = rgb + ((size_t)clampi(2 * y0 - 1 + r, 0, H - 1) * W +
                            clampi(2 * x0 - 1 + c, 0, W - 1)) * 3;
    pr[k][0] = p[0];
    pr[k][1] = p[1];
    pr[k][2] = p[2];
  }
#pragma unroll
  for (int k = 0; k < kPrepLoads; ++k) {
    const float r = pr[k][0], g = pr[k][1], b = pr[k][2];
    int q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float v = floorf(__fadd_rn(__fmul_rn(255.f, pr[k][c]), 0.5f));
      q[c] = (int)fminf(fmaxf(v, 0.f), 255.f);
    }
    const int row = ti[k] / kPrepTW, col = ti[k] - row * kPrepTW;
    s_f[row][col] = (77.f * r + 150.f * g + 29.f * b) * (1.f / 256.f);
    s_i[row][col] = (77 * q[0] + 150 * q[1] + 29 * q[2] + 128) >> 8;
  }
  __syncthreads();
  const int lx = threadIdx.x, ly = threadIdx.y, x = x0 + lx, y = y0 + ly;
  if (x >= X || y >= Y) return;
  float sf = 0.f;
  int si = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      sf += s_f[2 * ly + j][2 * lx + i];
      si += s_i[2 * ly + j][2 * lx + i];
    }
  }
  const size_t o = (size_t)img * X * Y + (size_t)y * X + x;
  half_f[o] = sf * (1.f / 9.f);
  half_u8[o] = (uint8_t)((si + 4) / 9);
}

// ----------------------------------------------------------- k_soft_size
// 1 / |S(x,y)| for the left image of each pair: |S| = sum over s in
// [-M, N] of (m + n + 1) at (x, y + s) (Eq. 7-8 applied to a unit cost).
// One workgroup = 64 columns x kSizeRows rows.  The row supports m + n + 1
// (at most 63: arm_x <= 31) of the tile rows y0 - arm_y + r, r < 144,
// are summed down each column: wave w loads the rows 9 w .. 9 w + 8 together
// (rows clamped into the image; a window never reaches a clamped row) and
// keeps their running sum, the waves' totals give each wave its offset, and
// the exclusive column prefix P (16 bits: at most 144 x 63) goes to LDS, so
// a window is P[t + N + 1] - P[t - M], t the tile row of y.
// grid: (ceil(X/64), ceil(Y/kSizeRows), n), block (64, kSizeRows).
constexpr int kSizeRows = 16, kSizeMaxArm = 63, kSizeSeg = 9;
static_assert(kSizeRows * kSizeSeg >= kSizeRows + 2 * kSizeMaxArm, "tile rows");

__global__ void __launch_bounds__(64 * kSizeRows) k_soft_size(const uint32_t* __restrict__ arms,
                                                             int X, int Y, int XA, int arm_y,
                                                             float* __restrict__ inv_size) {
  __shared__ uint16_t s_p[kSizeRows * kSizeSeg + 1][64];
  __shared__ uint16_t s_t[kSizeRows][64];
  const int x0 = blockIdx.x * 64, y0 = blockIdx.y * kSizeRows, pair = blockIdx.z;
  const int lx = threadIdx.x, ly = threadIdx.y, x = x0 + lx;  // x < XA: zero padding past X
  const uint32_t* a = arms + (size_t)(2 * pair) * Y * XA;
  const int y = y0 + ly;
  uint32_t c = a[(size_t)min(y, Y - 1) * XA + x];
  uint32_t v[kSizeSeg];
#pragma unroll
  for (int k = 0; k < kSizeSeg; ++k)
    v[k] = a[(size_t)clampi(y0 - arm_y + kSizeSeg * ly + k, 0, Y - 1) * XA + x];
  // the pixel's own arms stay loaded with the tile's (not after the barriers)
  __asm__ volatile("" : "+v"(c));
  uint32_t run = 0, loc[kSizeSeg];
#pragma unroll
  for (int k = 0; k < kSizeSeg; ++k) {
    run += (v[k] & 255u) + ((v[k] >> 8) & 255u) + 1u;
    loc[k] = run;
  }
  s_t[ly][lx] = (uint16_t)run;
  __syncthreads();
  uint32_t off = 0;
#pragma unroll
  for (int l = 0; l < kSizeRows; ++l) off += l < ly ? (uint32_t)s_t[l][lx] : 0u;
#pragma unroll
  for (int k = 0; k < kSizeSeg; ++k) s_p[kSizeSeg * ly + k + 1][lx] = (uint16_t)(off + loc[k]);
  if (ly == 0) s_p[0][lx] = 0;
  __syncthreads();
  if (x >= X || y >= Y) return;
  const int M = (c >> 16) & 255, N = c >> 24, t = ly + arm_y;  // tile row of y
  const int sum = (int)s_p[t + N + 1][lx] - (int)s_p[t - M][lx];
  inv_size[(size_t)pair * X * Y + (size_t)y * X + x] = 1.f / (float)sum;
}

// ------------------------------------------------------------ k_soft_agg
struct SoftArgs {
  const uint2* sp;          // [2n][Y][XS] padded pixel planes
  const uint32_t* arms;     // [2n][Y][XA]
  const float* lam;         // device [2]: lambda_AD, lambda_census
  const float* inv_size;    // [n][Y][X]                    (forward)
  float2* part;             // [n][nchunk][Y][X] {sum e, sum d e}  (forward)
  const float4* pc;         // [n][Y][X] {w, log2 sum e, d_hat, A}  (GCA)
  float* gca;               // [nds][n][Y][X] dL/dCA           (GCA)
  float* wts;               // [D][n][Y][X] e_d, or NULL        (forward)
  int X, Y, XS, pads, XA, arm_x, arm_y;
  int nbands, dlo, dhi, nstrips, ngroups, npair;
  int csize, nchunk;        // d-chunk size; chunks = ceil((dhi - dlo) / csize), the last the remainder
  float fx;                 // fixed-point scale 2^k of the costs
  float zc;                 // 2^-k log2(e) / tau: CA_int * inv_size * zc = mean / tau in log2 units
  uint32_t sp_bytes, arms_bytes;
};

// Inclusive prefix sum of a float over the 64 lanes of a wave (the DPP
// steps of wave_scan_incl, in float).
template <int CTRL, int RMASK>
__device__ __forceinline__ float dpp_add_f(float v) {
  return v + __int_as_float(
                 __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RMASK, 0xf, false));
}
__device__ __forceinline__ float wave_scan_incl_f(float v) {
  v = dpp_add_f<0x111, 0xf>(v);
  v = dpp_add_f<0x112, 0xf>(v);
  v = dpp_add_f<0x114, 0xf>(v);
  v = dpp_add_f<0x118, 0xf>(v);
  v = dpp_add_f<0x142, 0xa>(v);
  v = dpp_add_f<0x143, 0xc>(v);
  return v;
}

// One workgroup = one 64-column strip x one band of rows x one pair x one
// chunk of disparities; 16 waves, the layout of k_match (row pass with a DPP
// wave scan, running column sums into the LDS plane, segment offsets, window
// differences).  The cost of a column c at disparity d:
//   c - d >= 0: C = (2 - exp(-255 |L(c) - R(c-d)| / lambda_AD)) - exp(-H / lambda_census)
//   c - d <  0: C = 2
// taken to fixed point.  Output rows of a thread: o0 + wave + 16 k, k < KMAX.
//   GCA = false: e = 2^{-CA mean / tau (log2 units)}, sums of e and d e per
//                output pixel over the chunk -> part;
//   GCA = true : dL/dCA(x,y,d) = A p_d (d - d_hat), p_d = 2^{-z_d - log2 sum e}
//                -> gca plane of d (slot d - dlo).
// grid: ceil(groups / 8) * 8 * nchunk workgroups (1-D), block 1024.
template <int NS, int KMAX, bool GCA>
__global__ void __launch_bounds__(kThreads) k_soft_agg(SoftArgs a) {
  constexpr int PR = plane_rows(NS);
  __shared__ uint32_t s_row[kWaves][NS * 128];
  __shared__ uint32_t s_seg[kWaves][64];
  __shared__ uint32_t s_plane[(PR + 1) * 64];
  __shared__ float s_ex[8];

  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int X = a.X, Y = a.Y;
  const int wg = blockIdx.x, xcd = wg & (kXcds - 1), j = wg / kXcds;
  int local, chunk;
  chunk_at(j, (a.ngroups + kXcds - 1) / kXcds, (a.dhi - a.dlo) / a.csize, a.nchunk, local, chunk);
  int group = local * kXcds + xcd;
  if (group >= a.ngroups) return;
  const int strip = group % a.nstrips;
  group /= a.nstrips;
  const int band = group % a.nbands;
  const int pair = group / a.nbands;
  const int x0 = strip * kTX;
  const int ob = (Y + a.nbands - 1) / a.nbands;
  const int y0 = band * ob, y1 = min(Y, y0 + ob);
  const int ya = max(0, y0 - a.arm_y), yb = min(Y, y1 + a.arm_y);
  const int nb = yb - ya, o0 = y0 - ya, o1 = y1 - ya;
  const int d0 = a.dlo + chunk * a.csize, d1 = min(a.dhi, d0 + a.csize);
  const int hx = (a.arm_x + 2) & ~1;
  const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(a.sp, a.sp_bytes);
  const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(a.arms, a.arms_bytes);
  const uint32_t img_l = (uint32_t)(2 * pair), img_r = img_l + 1u;
  const uint32_t sprow = (uint32_t)a.XS * 8u, armrow = (uint32_t)a.XA * 4u;
  const float lam_ad = a.lam[0], lam_c = a.lam[1];
  // e^{-255 |dI| / lambda_AD} = 2^{-|dI| k2}
  const float k2 = 255.f * 1.4426950408889634f / lam_ad;
  if (t < 8) s_ex[t] = t < 7 ? fast_exp2(-(float)t * 1.4426950408889634f / lam_c) : 0.f;
  if (t < 64) s_plane[t] = 0u;

  const int c = lane, x = x0 + lane;
  // rows of the band in segments of whole row pairs (the row pass takes its
  // rows in pairs), one per wave in order, the pairs split as evenly as
  // possible: the waves of each SIMD (wave mod 4) then share the rows evenly
  const int nbat = (nb + 1) / 2, bq = nbat / kWaves, br = nbat % kWaves;
  const int r0 = min(nb, 2 * (wave * bq + min(wave, br)));
  const int r1 = min(nb, r0 + 2 * (bq + (wave < br)));

  static_assert(KMAX % 2 == 0, "KMAX must be even");
  uint32_t marm[KMAX / 2];
  float se[GCA ? 1 : KMAX], sde[GCA ? 1 : KMAX], isz[GCA ? 1 : KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int r = o0 + wave + k * kWaves;
    const bool in = x < X && r < o1;
    // no branch around the load (rows past the band read its last row and are
    // masked by a wave-uniform select; columns past X read the zero padding)
    const uint32_t v = a.arms[((size_t)img_l * Y + ya + min(r, o1 - 1)) * a.XA + x] >> 16;
    const uint32_t mn = r < o1 ? v : 0u;
    if (k & 1) marm[k / 2] |= mn << 16;
    else marm[k / 2] = mn;
    if constexpr (!GCA) {
      se[k] = 0.f;
      sde[k] = 0.f;
      // unconditional load at a clamped pixel, then a select (as above)
      const float iv = a.inv_size[((size_t)pair * Y + ya + min(r, o1 - 1)) * X + min(x, X - 1)];
      isz[k] = in ? iv * a.zc : 0.f;
    }
  }
  const int fin_base = (o0 + wave + 1) * 64 + c;
  // byte offset of this lane's first column pair in a padded row
  const uint32_t vb = (uint32_t)(a.pads + x0 - hx + 2 * lane) * 8u;
  const uint32_t vx = (uint32_t)x * 4u;
  const float fx = a.fx;
  __syncthreads();

  auto cost = [&](uint2 l, uint2 r, int col, int d) -> uint32_t {
    const float di = fabsf(__uint_as_float(l.x) - __uint_as_float(r.x));
    const float cf = (2.f - fast_exp2(-di * k2)) - s_ex[__builtin_popcount(l.y ^ r.y)];
    const uint32_t ci = (uint32_t)(cf * fx + 0.5f);
    return col - d >= 0 ? ci : (uint32_t)(2.f * fx + 0.5f);
  };

  for (int d = d0; d < d1; ++d) {
    const uint32_t vo = vb - (uint32_t)(d * 8);
    uint32_t run = 0;
    // rows in batches of two (their scans interleave), the loads of the next
    // batch in flight while this one is processed; a batch running past the
    // segment end loads its last row again and never stores it
    struct RowIn { u32x4 L[NS], R[NS]; uint32_t am; };
    auto load_row = [&](int r, RowIn& in) {
      const uint32_t y = (uint32_t)(ya + r);
      const uint32_t sl = (img_l * (uint32_t)Y + y) * sprow, sr = (img_r * (uint32_t)Y + y) * sprow;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        in.L[s] = __builtin_amdgcn_raw_buffer_load_b128(rs, vb + s * 1024, sl, 0);
        in.R[s] = __builtin_amdgcn_raw_buffer_load_b128(rs, vo + s * 1024, sr, 0);
      }
      in.am = __builtin_amdgcn_raw_buffer_load_b32(ra, vx, (img_l * (uint32_t)Y + y) * armrow, 0);
    };
    auto row_of = [&](int r, int i) { return r + i < r1 ? r + i : r1 - 1; };
    auto load_batch = [&](int r, RowIn (&in)[2]) {
      load_row(row_of(r, 0), in[0]);
      load_row(row_of(r, 1), in[1]);
    };
    auto process_batch = [&](int r, const RowIn (&in)[2]) {
      uint32_t c1v[2][NS], pr[2][NS];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int col = x0 - hx + s * 128 + 2 * lane;
          const uint32_t c0 = cost(make_uint2(in[i].L[s].x, in[i].L[s].y),
                                   make_uint2(in[i].R[s].x, in[i].R[s].y), col, d);
          c1v[i][s] = cost(make_uint2(in[i].L[s].z, in[i].L[s].w),
                           make_uint2(in[i].R[s].z, in[i].R[s].w), col + 1, d);
          pr[i][s] = wave_scan_incl(c0 + c1v[i][s]);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (i > 0 && r + i >= r1) break;
        uint32_t carry = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const uint32_t p = pr[i][s] + carry;
          if (NS > 1) carry = __builtin_amdgcn_readlane(p, 63);
          *reinterpret_cast<u32x2*>(&s_row[wave][s * 128 + 2 * lane]) = u32x2{p - c1v[i][s], p};
        }
        WAVE_LDS_ORDER();
        const int m = in[i].am & 255u, n = (in[i].am >> 8) & 255u;
        run += s_row[wave][lane + hx + n] - s_row[wave][lane + hx - m - 1];
        WAVE_LDS_ORDER();
        s_plane[(r + i + 1) * 64 + lane] = run;
      }
    };
    RowIn in0[2], in1[2];  // two buffer sets, used in turn
    if (r0 < r1) load_batch(r0, in0);
    for (int r = r0; r < r1; r += 4) {
      load_batch(r + 2, in1);  // unconditional: see k_match's row pass
      process_batch(r, in0);
      if (r + 2 >= r1) break;
      load_batch(r + 4, in0);
      process_batch(r + 2, in1);
    }
    s_seg[wave][c] = run;
    __syncthreads();
    uint32_t off = 0;
#pragma unroll
    for (int s = 0; s < kWaves; ++s) {
      const uint32_t v = s_seg[s][c];
      off += s < wave ? v : 0u;
    }
    if (wave > 0) {
#pragma unroll 8
      for (int r = r0; r < r1; ++r) s_plane[(r + 1) * 64 + c] += off;
    }
    __syncthreads();
    const float fd = (float)d;
    // the adjoint's per-pixel constants of 4 output rows at a time, loaded
    // together (unconditionally, at clamped pixels) before they are used
    constexpr int QB = GCA ? 4 : 1;
    float4 qv[QB];
#pragma unroll
    for (int jj = 0; jj < KMAX / 2; ++jj) {
      if constexpr (GCA) {
        if ((2 * jj) % QB == 0) {
#pragma unroll
          for (int u = 0; u < QB; ++u) {
            const int r = min(o0 + wave + (2 * jj + u) * kWaves, o1 - 1);
            qv[u] = a.pc[((size_t)pair * Y + ya + r) * X + min(x, X - 1)];
          }
        }
      }
      uint32_t mj = marm[jj];
      __asm__ volatile("" : "+v"(mj));
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 2 * jj + h;
        const int M = (mj >> (16 * h)) & 255u, N = (mj >> (16 * h + 8)) & 255u;
        const int lo = fin_base - (M + 1) * 64, hi = fin_base + N * 64;
        const uint32_t ca = s_plane[hi + k * kWaves * 64] - s_plane[lo + k * kWaves * 64];
        if constexpr (!GCA) {
          const float e = fast_exp2(-(float)ca * isz[k]);
          se[k] += e;
          sde[k] += fd * e;
          const int r = o0 + wave + k * kWaves;
          if (a.wts && x < X && r < o1)
            a.wts[(size_t)d * a.npair * X * Y + ((size_t)pair * Y + ya + r) * X + x] = e;
        } else {
          const int r = o0 + wave + k * kWaves;
          const float4 q = qv[k % QB];
          const float p = fast_exp2(-(float)ca * q.x - q.y);
          if (x < X && r < o1)
            a.gca[(size_t)(d - a.dlo) * a.npair * X * Y + ((size_t)pair * Y + ya + r) * X + x] =
                q.w * p * (fd - q.z);
        }
      }
    }
    __syncthreads();
  }

  if constexpr (!GCA) {
    if (x < X) {
      float2* out = a.part + (size_t)(pair * a.nchunk + chunk) * X * Y;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        const int r = o0 + wave + k * kWaves;
        if (r < o1) out[(size_t)(ya + r) * X + x] = make_float2(se[k], sde[k]);
      }
    }
  }
}

// ---------------------------------------------------------- k_soft_merge
// Sums the chunk partials in chunk order: d_hat = sum d e / sum e and
// lse2 = log2 sum e.  grid: (ceil(X*Y/256), n), block 256.
__global__ void __launch_bounds__(256) k_soft_merge(const float2* __restrict__ part, int nchunk,
                                                    int npix, float* __restrict__ dhat,
                                                    float* __restrict__ lse2) {
  const int i = blockIdx.x * 256 + threadIdx.x, pair = blockIdx.y;
  if (i >= npix) return;
  const float2* p = part + (size_t)pair * nchunk * npix + i;
  float s = 0.f, sd = 0.f;
  // loads in groups of 8 in flight, sums in chunk order
  for (int c0 = 0; c0 < nchunk; c0 += 8) {
    float2 v[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) v[g] = p[(size_t)min(c0 + g, nchunk - 1) * npix];
#pragma unroll
    for (int g = 0; g < 8; ++g)
      if (c0 + g < nchunk) {
        s += v[g].x;
        sd += v[g].y;
      }
  }
  dhat[(size_t)pair * npix + i] = sd / s;
  lse2[(size_t)pair * npix + i] = __log2f(s);
}

// ---------------------------------------------------------- k_soft_bprep
// Per-pixel constants of the adjoint: w = zc / |S| (log2-unit mean per
// fixed-point aggregate), lse2, d_hat and A = -g_dhat / (tau |S|), so that
// dL/dCA(d) = A p_d (d - d_hat) with p_d = 2^{-CA w - lse2}.
// grid: (ceil(X*Y/256), n), block 256.
__global__ void __launch_bounds__(256) k_soft_bprep(const float* __restrict__ inv_size,
                                                    const float* __restrict__ lse2,
                                                    const float* __restrict__ dhat,
                                                    const float* __restrict__ g_dhat, int npix,
                                                    float zc, float inv_tau,
                                                    float4* __restrict__ pc) {
  const int i = blockIdx.x * 256 + threadIdx.x, pair = blockIdx.y;
  if (i >= npix) return;
  const size_t o = (size_t)pair * npix + i;
  const float is = inv_size[o];
  pc[o] = make_float4(is * zc, lse2[o], dhat[o], -g_dhat[o] * is * inv_tau);
}

// ------------------------------------------------------------ k_soft_tcol
// Transpose of the vertical window sum (Eq. 8) for one disparity over a band
// of kTcolBand output rows of a 64-column strip:
//   CA(x,y) = sum_{s=-M(x,y)}^{N(x,y)} CA_x(x,y+s)  gives
//   dL/dCA_x(x,y') = sum of dL/dCA(x,y) over the y whose window holds y'.
// The band's rows y' in [Y0, Y0 + B) can only be reached from sources y in
// [Y0 - arm_y, Y0 + B + arm_y); each source's window, clipped to the band,
// becomes a difference array (+g at its first row, -g after its last) and a
// prefix down the column gives the sums.  The difference array is integer
// fixed point with a per-column scale 2^k, k = 23 - e where 2^(e-1) <= the
// column's largest |g| < 2^e: each term is below 2^23 and a sum of at most
// 2 arm_y + 1 <= 127 terms below 2^30, so LDS integer atomic adds give exact
// sums in any order (the result does not depend on scheduling) and each
// term is rounded to 2^(e-24), the float resolution of the column's largest
// value.  Thread (wave w, lane l) takes column x0 + l and the source rows
// Y0 - arm_y + w + 4 i, all loads issued together and held in registers.
// grid: (ceil(X/64), ceil(Y/B), nds * n), block 256; B = kTcolBand for
// arm_y <= 31, else kTcolBand / 2 (the sources then still fit 48 per thread).
constexpr int kTcolBand = 128;
constexpr int kTcolSrc = 48;  // source rows per thread at most

__host__ __device__ constexpr int tcol_band(int arm_y) { return arm_y <= 31 ? kTcolBand : kTcolBand / 2; }

__global__ void __launch_bounds__(256) k_soft_tcol(const float* __restrict__ gca,
                                                   const uint32_t* __restrict__ arms, int X,
                                                   int Y, int XA, int arm_y, int npair,
                                                   float* __restrict__ gcax) {
  __shared__ int s_d[kTcolBand + 1][64];
  __shared__ float s_max[4][64];
  __shared__ int s_tot[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int B = tcol_band(arm_y);
  const int x = blockIdx.x * 64 + lane, Y0 = blockIdx.y * B;
  const int dj = blockIdx.z / npair, pair = blockIdx.z - dj * npair;
  const int Y1 = min(Y, Y0 + B);
  const bool xv = x < X;
  const size_t plane = (size_t)X * Y;
  const float* g = gca + ((size_t)dj * npair + pair) * plane;
  const uint32_t* am = arms + (size_t)(2 * pair) * Y * XA;
  const int ys = max(0, Y0 - arm_y), ye = min(Y, Y1 + arm_y);
  // sources y = ys + wave + 4 i < ye; loads at clamped rows, masked after
  float gv[kTcolSrc];
  uint32_t av[kTcolSrc];
#pragma unroll
  for (int i = 0; i < kTcolSrc; ++i) {
    const int y = min(ys + wave + 4 * i, ye - 1);
    gv[i] = xv ? g[(size_t)y * X + x] : 0.f;
    av[i] = am[(size_t)y * XA + min(x, XA - 1)];
  }
  for (int i = threadIdx.x; i < (B + 1) * 64; i += 256) (&s_d[0][0])[i] = 0;
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < kTcolSrc; ++i)
    if (ys + wave + 4 * i < ye) mx = fmaxf(mx, fabsf(gv[i]));
  s_max[wave][lane] = mx;
  __syncthreads();
  const float cmax = fmaxf(fmaxf(s_max[0][lane], s_max[1][lane]), fmaxf(s_max[2][lane], s_max[3][lane]));
  int e = 0;
  (void)frexpf(cmax, &e);
  const float up = cmax > 0.f ? ldexpf(1.f, 23 - e) : 0.f;
#pragma unroll
  for (int i = 0; i < kTcolSrc; ++i) {
    const int y = ys + wave + 4 * i;
    if (y < ye && gv[i] != 0.f) {
      const int q = (int)rintf(gv[i] * up);
      const int M = (int)((av[i] >> 16) & 255u), N = (int)(av[i] >> 24);
      const int lo = max(y - M, Y0), hi = min(y + N, Y1 - 1);
      if (lo <= hi) {
        atomicAdd(&s_d[lo - Y0][lane], q);
        if (hi + 1 < Y1) atomicAdd(&s_d[hi + 1 - Y0][lane], -q);
      }
    }
  }
  __syncthreads();
  // prefix down the column: wave w takes rows w * B/4 .. (w+1) * B/4 - 1,
  // its running sum kept per row, then the totals of the waves above
  const int rpw = B / 4, r0 = wave * rpw;
  int run = 0;
  int loc[kTcolBand / 4];
#pragma unroll
  for (int i = 0; i < kTcolBand / 4; ++i) {
    if (i < rpw) run += s_d[r0 + i][lane];
    loc[i] = run;
  }
  s_tot[wave][lane] = run;
  __syncthreads();
  int off = 0;
#pragma unroll
  for (int w = 0; w < 3; ++w) off += w < wave ? s_tot[w][lane] : 0;
  if (!xv) return;
  const float down = cmax > 0.f ? ldexpf(1.f, e - 23) : 0.f;
  float* out = gcax + ((size_t)dj * npair + pair) * plane + x;
#pragma unroll
  for (int i = 0; i < kTcolBand / 4; ++i) {
    const int y = Y0 + r0 + i;
    if (i < rpw && y < Y1) out[(size_t)y * X] = (float)(loc[i] + off) * down;
  }
}

// ------------------------------------------------------------ k_soft_tcolw
// The transpose of k_soft_tcol with dL/dCA formed on the fly from the
// softmax weights e_d = 2^{-CA(d) w} that the forward saved:
//   dL/dCA(x,y,d) = A p_d (d - d_hat),  p_d = e_d 2^{-lse2}
// (A, lse2 and d_hat from k_soft_bprep's constants), so the backward needs
// neither k_soft_agg's recomputation of CA nor the dL/dCA planes.  A block
// takes a 64-column strip, a band of B output rows (tcol_band) and a range
// of disparities of one pair; thread (wave w, lane l) holds, over the range,
// the constants and vertical arms of column x0 + l at the source rows
// Y0 - arm_y + w + 8 i, and for each disparity builds the band's integer
// difference array exactly as k_soft_tcol does (per-column power-of-two
// scale from the largest |dL/dCA| of the band's sources, LDS integer atomics,
// order-independent sums), then writes dL/dCA_x of the band's rows.
// grid: (ceil(X/64), ceil(Y/B), n * ndg), block 512; disparity group g of
// ndg covers [g D / ndg, (g + 1) D / ndg).
constexpr int kTcwWaves = 16;
constexpr int kTcwSrc = 12;  // source rows per thread: B + 2 arm_y <= 16 * 12
static_assert(tcol_band(31) + 2 * 31 <= kTcwWaves * kTcwSrc &&
                  tcol_band(63) + 2 * 63 <= kTcwWaves * kTcwSrc, "k_soft_tcolw source rows");

__global__ void __launch_bounds__(64 * kTcwWaves) k_soft_tcolw(
    const float* __restrict__ wts, uint32_t wts_bytes, const float4* __restrict__ pc,
    const uint32_t* __restrict__ arms, int X, int Y, int XA, int arm_y, int npair, int D, int ndg,
    float* __restrict__ gcax) {
  __shared__ int s_d[kTcolBand + 1][64];
  __shared__ float s_max[kTcwWaves][64];
  __shared__ int s_tot[kTcwWaves][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int B = tcol_band(arm_y);
  const int x = blockIdx.x * 64 + lane, Y0 = blockIdx.y * B;
  const int pair = blockIdx.z % npair, dg = blockIdx.z / npair;
  const int dlo = dg * D / ndg, dhi = (dg + 1) * D / ndg;
  const int Y1 = min(Y, Y0 + B);
  const bool xv = x < X;
  const int xc = min(x, X - 1);
  const size_t plane = (size_t)X * Y;
  const int ys = max(0, Y0 - arm_y), ye = min(Y, Y1 + arm_y);
  // source row of slot i (wave-uniform), clamped into the sources
  auto src_row = [&](int i) { return min(ys + wave + kTcwWaves * i, ye - 1); };
  // constants of the source rows ys + wave + 8 i (loads at clamped rows; a
  // row outside the sources or a column past X gets A = 0, so it adds nothing)
  float cA[kTcwSrc], cS[kTcwSrc], cD[kTcwSrc];
  uint32_t cMN[kTcwSrc / 2];  // M | N << 8 of two rows, one per 16-bit half
#pragma unroll
  for (int i = 0; i < kTcwSrc; ++i) {
    const int y = src_row(i);
    const float4 q = pc[((size_t)pair * Y + y) * X + xc];
    const uint32_t am = arms[((size_t)(2 * pair) * Y + y) * XA + xc] >> 16;
    cA[i] = xv && ys + wave + kTcwWaves * i < ye ? q.w : 0.f;
    cS[i] = fast_exp2(-q.y);
    cD[i] = q.z;
    if (i & 1) cMN[i / 2] |= am << 16;
    else cMN[i / 2] = am;
  }
  // weight loads: the lane's column in the vector offset, the row and plane
  // (wave-uniform) in the scalar one
  const __amdgpu_buffer_rsrc_t rw = buffer_rsrc(wts, wts_bytes);
  const uint32_t vcol = (uint32_t)xc * 4u;
  const int rpw = B / kTcwWaves, r0 = wave * rpw;
  // the weights of disparity d into w[]; the next disparity's are loaded
  // while this one is processed (past the range: the last one again)
  auto load_w = [&](int d, float (&w)[kTcwSrc]) {
    const uint32_t sp = (uint32_t)(((size_t)min(d, dhi - 1) * npair + pair) * plane * 4);
#pragma unroll
    for (int i = 0; i < kTcwSrc; ++i)
      w[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
          rw, vcol, sp + (uint32_t)src_row(i) * (uint32_t)X * 4u, 0));
  };
  float wn[kTcwSrc];
  if (dlo < dhi) load_w(dlo, wn);
  for (int d = dlo; d < dhi; ++d) {
    const float fd = (float)d;
    float g[kTcwSrc];
#pragma unroll
    for (int i = 0; i < kTcwSrc; ++i) g[i] = wn[i];
    load_w(d + 1, wn);
    float mx = 0.f;
#pragma unroll
    for (int i = 0; i < kTcwSrc; ++i) {
      g[i] = cA[i] * (g[i] * cS[i]) * (fd - cD[i]);
      mx = fmaxf(mx, fabsf(g[i]));
    }
    s_max[wave][lane] = mx;
    for (int i = threadIdx.x; i < (B + 1) * 64; i += 64 * kTcwWaves) (&s_d[0][0])[i] = 0;
    __syncthreads();
    float cmax = 0.f;
#pragma unroll
    for (int w = 0; w < kTcwWaves; ++w) cmax = fmaxf(cmax, s_max[w][lane]);
    int e = 0;
    (void)frexpf(cmax, &e);
    const float up = cmax > 0.f ? ldexpf(1.f, 23 - e) : 0.f;
#pragma unroll
    for (int i = 0; i < kTcwSrc; ++i) {
      const int q = (int)rintf(g[i] * up);
      if (q != 0) {
        const int y = ys + wave + kTcwWaves * i;
        const uint32_t mn = cMN[i / 2] >> (16 * (i & 1));
        const int M = (int)(mn & 255u), N = (int)((mn >> 8) & 255u);
        const int lo = max(y - M, Y0), hi = min(y + N, Y1 - 1);
        if (lo <= hi) {
          atomicAdd(&s_d[lo - Y0][lane], q);
          if (hi + 1 < Y1) atomicAdd(&s_d[hi + 1 - Y0][lane], -q);
        }
      }
    }
    __syncthreads();
    // prefix down the column: wave w takes rows w B/8 .. (w+1) B/8 - 1
    int run = 0;
    int loc[kTcolBand / kTcwWaves];
#pragma unroll
    for (int i = 0; i < kTcolBand / kTcwWaves; ++i) {
      if (i < rpw) run += s_d[r0 + i][lane];
      loc[i] = run;
    }
    s_tot[wave][lane] = run;
    __syncthreads();
    int off = 0;
#pragma unroll
    for (int w = 0; w < kTcwWaves - 1; ++w) off += w < wave ? s_tot[w][lane] : 0;
    if (xv) {
      const float down = cmax > 0.f ? ldexpf(1.f, e - 23) : 0.f;
      float* out = gcax + ((size_t)d * npair + pair) * plane + x;
#pragma unroll
      for (int i = 0; i < kTcolBand / kTcwWaves; ++i) {
        const int y = Y0 + r0 + i;
        if (i < rpw && y < Y1) out[(size_t)y * X] = (float)(loc[i] + off) * down;
      }
    }
  }
}

// ------------------------------------------------------------- k_soft_tr
// Transpose of the horizontal window sum (Eq. 7) over a 64-column strip and
// a band of kSoftBR rows, for every disparity of a slab in turn, then the
// cost derivatives there, summed over the slab into the half-image gradients.
//   CA_x(x,y) = sum_{t=-m}^{n} C(x+t,y) transposes to a difference array
//   along the row (+g at x - m, -g at x + n + 1) and a prefix along it,
//   giving dL/dC from dL/dCA_x (k_soft_tcol's planes).
// Then with dI = L(x,y) - R(x-d,y), a = 255 |dI|, E = e^{-a/lambda_AD}:
//   t = dL/dC * dC/d(dI) = dL/dC * (255 / lambda_AD) E sign(dI)
//   dL/dL(x,y)        += t       dL/dR(x-d,y) -= t
//   dL/dlambda_AD     += dL/dC * (-E a / lambda_AD^2)
//   dL/dlambda_census += dL/dC * (-e^{-H/lambda_census} H / lambda_census^2)
// for x - d >= 0 (the constant cost of x - d < 0 has no derivative).
// The sources of a row are the columns x0 - 32 .. x0 + 95 (every column
// whose horizontal window reaches the strip, arm_x <= 31).  Wave w owns the
// band rows w + 4 i, i < kSoftBR / 4 (one row with bands of 4: 51 VGPRs, 8
// waves per SIMD, and the grid of 5952 workgroups at the paper's size takes
// 2.9 rounds; bands of 16 rows took 120 VGPRs and 1.45 rounds, and ran
// slower than bands of 8, which ran slower than bands of 4): lane l loads
// source columns x0 - 32 + l and x0 + 32 + l of them (coalesced), scatters
// them into the rows' difference arrays, scans the rows and takes the
// derivatives at output column x0 + l, so the disparity loop needs no
// barrier (a wave's LDS
// accesses are served in order).  The difference arrays are integer fixed
// point with a per-row scale (as in k_soft_tcol: terms below 2^23, sums of
// at most 63 terms below 2^29), added with LDS integer atomics, so the
// result does not depend on their order.  The left gradient of a pixel stays
// in a register over the slab and goes to g_half once (written by the first
// slab, added by the others); the right one, at column x - d, goes to the
// wave's LDS row (one writer per entry and
// disparity, disparities in order) and then to this strip's partial row,
// which k_soft_gright sums over the strips.  The horizontal arms and the
// left pixels do not depend on d and are loaded once.
// grid: (strips * bands, n), block 256.
struct TrArgs {
  const float* gcax;        // [nds][n][Y][X] dL/dCA_x
  const uint32_t* arms;     // [2n][Y][XA]
  const uint2* sp;          // [2n][Y][XS] padded pixel planes
  const float* lam;         // device [2]
  float* g_half;            // [2n][Y][X] half-image gradients (left ones written or added here)
  float* gr_part;           // [n][strips][Y][WP] -dL/dR partials of this slab
  float2* lam_part;         // one {d/dlambda_AD, d/dlambda_census} per workgroup
  int X, Y, XS, pads, XA, npair, dlo, dhi, nstrips, nbands, WP;
  int first;                // first slab: the left gradients are written, not added
};

// Inclusive maximum scan over the 64 lanes of a wave of values >= 0 (the
// steps of wave_scan_incl; lanes a shift reaches past the row's start see 0).
__device__ __forceinline__ int wave_max_scan_incl(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return v;
}

// Maximum over the 64 lanes of a wave (row rotations inside rows of 16
// lanes, then row broadcasts; lane 63 ends with the maximum of all).
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false));  // row_ror:8
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false));  // row_ror:4
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false));   // quad_perm 2,3,0,1
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false));   // quad_perm 1,0,3,2
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

constexpr int kTrMaxWP = 64 + 127;  // 64 columns + a slab of up to 128 disparities

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_soft_tr(TrArgs a) {
  constexpr int BR = kSoftBR;
  static_assert(BR % 4 == 0, "whole rows per wave");
  constexpr int RPW = BR / 4;  // rows per wave: r = wave + 4 i
  __shared__ int s_d[BR][64];
  __shared__ float s_gr[BR][kTrMaxWP];
  __shared__ float2 s_red[4];
  __shared__ float s_hc[4][8];  // per wave: the census term of dC/dlambda_census by h
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int strip = blockIdx.x % a.nstrips, band = blockIdx.x / a.nstrips;
  const int pair = blockIdx.y;
  const int X = a.X, Y = a.Y;
  const int x0 = strip * 64, y0 = band * BR;
  const size_t plane = (size_t)X * Y;
  const uint32_t* arm = a.arms + (size_t)(2 * pair) * Y * a.XA;
  const uint2* spl = a.sp + (size_t)(2 * pair) * Y * a.XS + a.pads;
  const uint2* spr = a.sp + (size_t)(2 * pair + 1) * Y * a.XS + a.pads;
  const int x = x0 + lane;
  const bool xin = x < X;
  // per row i and source h: column x0 - 32 + 64 h + lane
  int ys[RPW];
  bool yv[RPW], cv[RPW][2];
  uint32_t mv[RPW][2];
  uint2 pl_[RPW];
  float gl[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int y = y0 + wave + 4 * i;
    yv[i] = y < Y;
    ys[i] = min(y, Y - 1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = x0 - 32 + 64 * h + lane;
      cv[i][h] = yv[i] && col >= 0 && col < X;
      mv[i][h] = arm[(size_t)ys[i] * a.XA + min(max(col, 0), X - 1)];
    }
    pl_[i] = xin ? spl[(size_t)ys[i] * a.XS + x] : make_uint2(0u, 0u);
    gl[i] = 0.f;
    for (int c = lane; c < kTrMaxWP; c += 64) s_gr[wave + 4 * i][c] = 0.f;
  }
  // Each source adds +q at the left end of its window (its position clamped
  // to the strip's first column) and -q after the right end (when that is
  // inside the strip).  Neighbouring sources whose windows end at the same
  // edge form runs of lanes with the same position, which would serialise
  // their atomics on one address.  The runs do not depend on d: per row,
  // source set h and end, 16 bits give the lane before the run's first
  // (bits 0..7, as a ds_bpermute address) and whether it exists (bit 8),
  // whether this lane ends a run of contributing sources (bit 9) and the
  // position (bits 10..15); the left end's in the low half of a word, the
  // right end's in the high half.  Per d and source set one wave scan of the
  // terms serves both ends: each run's sum is the scan at its last lane
  // minus the scan before its first, added (left ends) or subtracted (right
  // ends) by its last lane.
  uint32_t rw[RPW][2];
  auto run_word = [&](int key, bool ends, int pos) -> uint32_t {
    const int kp = __builtin_amdgcn_update_dpp(1000, key, 0x138, 0xf, 0xf, false);  // wave_shr:1
    const int kn = __builtin_amdgcn_update_dpp(1000, key, 0x130, 0xf, 0xf, false);  // wave_shl:1
    const int hs = wave_max_scan_incl(key != kp ? lane : 0);  // first lane of the run
    return (uint32_t)(max(hs - 1, 0) * 4) | (hs > 0 ? 256u : 0u) |
           (ends && key != kn ? 512u : 0u) | (uint32_t)(pos & 63) << 10;
  };
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = x0 - 32 + 64 * h + lane;
      const int lo = col - (int)(mv[i][h] & 255u) - x0;
      const int hi = col + (int)((mv[i][h] >> 8) & 255u) + 1 - x0;
      // the window reaches the strip (lo < 64 for h = 0 and hi > 0 for h = 1
      // always hold with arm_x <= 31)
      const bool part = cv[i][h] && (h == 0 ? hi > 0 : lo < 64);
      const int plo = max(lo, 0);
      const bool phi = part && hi < 64;
      rw[i][h] = run_word(part ? plo : -1 - lane, part, plo) |
                 run_word(phi ? hi : -1 - lane, phi, hi) << 16;
    }
  }
  const float lam_ad = a.lam[0], lam_c = a.lam[1];
  const float k2 = 255.f * 1.4426950408889634f / lam_ad;
  const float kt = 255.f / lam_ad, ka = 1.f / (lam_ad * lam_ad), kc = 1.f / (lam_c * lam_c);
  const float l2c = 1.4426950408889634f / lam_c;
  // -e^{-h/lambda_census} h / lambda_census^2 for h = 0..6, one copy per wave
  // (a wave's LDS accesses are served in order: no barrier)
  if (lane < 7) s_hc[wave][lane] = -fast_exp2(-(float)lane * l2c) * (float)lane * kc;
  WAVE_LDS_ORDER();
  float pa = 0.f, pcs = 0.f;
  // the loads of disparity d + 1 are issued before d is processed (two
  // register sets used in turn; the last disparity is reloaded past the end,
  // so the loads are unconditional and the waits stay exact)
  struct DIn {
    float g[RPW][2];
    uint2 pr[RPW];
  };
  const float* gbase = a.gcax + (size_t)pair * plane;
  const size_t dstride = (size_t)a.npair * plane;
  auto load_d = [&](int d, DIn& in) {
    const float* g = gbase + (size_t)(d - a.dlo) * dstride;
    const bool dv = x - d >= 0;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int cc = min(max(x0 - 32 + 64 * h + lane, 0), X - 1);
        in.g[i][h] = g[ys[i] * X + cc];
      }
      in.pr[i] = spr[ys[i] * a.XS + min(max(x - d, 0), X - 1)];
      if (!(xin && dv)) in.pr[i] = make_uint2(0u, 0u);
    }
  };
  auto process_d = [&](int d, const DIn& in) {
    const bool dv = x - d >= 0;
    // the wave's LDS accesses stay in program order across lanes: the
    // compiler may not move one across these points
    WAVE_LDS_ORDER();
#pragma unroll
    for (int i = 0; i < RPW; ++i) s_d[wave + 4 * i][lane] = 0;
    WAVE_LDS_ORDER();
    float down[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = wave + 4 * i;
      const float g0 = cv[i][0] ? in.g[i][0] : 0.f, g1 = cv[i][1] ? in.g[i][1] : 0.f;
      // the row's scale 2^(23 - e), 2^(e - 1) <= max |g| < 2^e (frexp's e),
      // from the largest magnitude's bits (the bit order of floats >= 0)
      const uint32_t mb = wave_max_u32(max(__float_as_uint(g0) & 0x7fffffffu,
                                           __float_as_uint(g1) & 0x7fffffffu));
      const int be = (int)(mb >> 23);
      const int e = be > 0 ? be - 126 : -117 - (int)__builtin_clz(mb | 1u);
      const float up = mb ? ldexpf(1.f, 23 - e) : 0.f;
      down[i] = mb ? ldexpf(1.f, e - 23) : 0.f;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = (int)rintf((h ? g1 : g0) * up);
        const int P = (int)wave_scan_incl((uint32_t)q);
        const uint32_t w = rw[i][h];
        const int Pl = __builtin_amdgcn_ds_bpermute((int)(w & 255u), P);
        const int Ph = __builtin_amdgcn_ds_bpermute((int)((w >> 16) & 255u), P);
        if (w & (512u << 16)) atomicSub(&s_d[r][w >> 26], P - ((w & (256u << 16)) ? Ph : 0));
        if (w & 512u) atomicAdd(&s_d[r][(w >> 10) & 63u], P - ((w & 256u) ? Pl : 0));
      }
    }
    WAVE_LDS_ORDER();
    // prefix along each row, then the cost derivatives; the right gradient
    // of column x - d sits at s_gr[r][x - d - (x0 - dhi + 1)]
    const int gcol = lane + (a.dhi - 1 - d);
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = wave + 4 * i;
      const float gc = (float)(int)wave_scan_incl((uint32_t)s_d[r][lane]) * down[i];
      if (xin && dv && yv[i]) {
        const float di = __uint_as_float(pl_[i].x) - __uint_as_float(in.pr[i].x);
        const float ad = fabsf(di);
        const float E = fast_exp2(-ad * k2);
        const float sg = di > 0.f ? 1.f : (di < 0.f ? -1.f : 0.f);
        const float tv = gc * kt * E * sg;
        gl[i] += tv;
        s_gr[r][gcol] -= tv;
        pa += gc * (-E * 255.f * ad * ka);
        const int hh = __builtin_popcount(pl_[i].y ^ in.pr[i].y);
        pcs += gc * s_hc[wave][hh];
      }
    }
    WAVE_LDS_ORDER();
  };
  DIn in0, in1;
  load_d(a.dlo, in0);
  for (int d = a.dlo; d < a.dhi; d += 2) {
    load_d(min(d + 1, a.dhi - 1), in1);
    process_d(d, in0);
    if (d + 1 >= a.dhi) break;
    load_d(min(d + 2, a.dhi - 1), in0);
    process_d(d + 1, in1);
  }
  WAVE_LDS_ORDER();
  // left gradients: each pixel has one owner (so the first slab writes every
  // one); slabs run one after another
  float* glp = a.g_half + (size_t)(2 * pair) * plane;
  // right partials of this strip: columns x0 - dhi + 1 .. x0 + 63 - dlo
  const int wd = 64 + (a.dhi - a.dlo) - 1;
  float* gp = a.gr_part + ((size_t)pair * a.nstrips + strip) * Y * a.WP;
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    if (!yv[i]) continue;
    const int y = ys[i], r = wave + 4 * i;
    if (xin) {
      float* g = glp + (size_t)y * X + x;
      *g = a.first ? gl[i] : *g + gl[i];
    }
    for (int c = lane; c < wd; c += 64) gp[(size_t)y * a.WP + c] = s_gr[r][c];
  }
  // fixed-order reduction of the lambda partials over the workgroup
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    pa += __shfl_down(pa, o);
    pcs += __shfl_down(pcs, o);
  }
  if (lane == 0) s_red[wave] = make_float2(pa, pcs);
  __syncthreads();
  if (t == 0) {
    float2 s = s_red[0];
    for (int w = 1; w < 4; ++w) { s.x += s_red[w].x; s.y += s_red[w].y; }
    a.lam_part[(size_t)pair * gridDim.x + blockIdx.x] = s;
  }
}

// --------------------------------------------------------- k_soft_gright
// dL/dR(x,y) over a slab [dlo, dhi): the partials of the strips s whose
// columns x + d (d in the slab) reach, floor((x + dlo) / 64) ..
// floor((x + dhi - 1) / 64), summed in strip order, written to g_half for the
// first slab and added to it for the others.
// grid: (ceil(X/256), Y, n), block 256.
__global__ void __launch_bounds__(256) k_soft_gright(const float* __restrict__ gr_part, int nstrips,
                                                     int WP, int dlo, int dhi, int X, int Y,
                                                     int first, float* __restrict__ g_half) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, pair = blockIdx.z;
  if (x >= X) return;
  const int s0 = (x + dlo) / 64, s1 = min(nstrips - 1, (x + dhi - 1) / 64);
  float acc = 0.f;
  for (int s = s0; s <= s1; ++s) {
    const int c = x - (s * 64 - dhi + 1);  // in 0 .. WP - 1 for the strips reached
    acc += gr_part[(((size_t)pair * nstrips + s) * Y + y) * WP + c];
  }
  float* g = g_half + ((size_t)(2 * pair + 1) * Y + y) * X + x;
  *g = first ? acc : *g + acc;
}

// ---------------------------------------------------------- k_soft_gfull
// dL/d(RGB) from dL/d(half image): a full-res pixel (u, v) receives g/9 from
// every half-res pixel whose clamped 3x3 block holds it, once per block cell
// that lands on it, times the channel's gray weight (77, 150, 29) / 256.
// Along each axis those pixels are among p >> 1 and (p + 1) >> 1 (the latter
// only for odd p inside the image), with weight #{j in -1..1 :
// clamp(2 q + j) = p}: the four loads are unconditional (indices clamped, a
// repeated index gets weight 0).
// grid: (ceil(W/256), H, 2n), block 256.
__device__ __forceinline__ int gfull_weight(int q, int p, int lim) {
  int w = 0;
#pragma unroll
  for (int j = -1; j <= 1; ++j) w += clampi(2 * q + j, 0, lim - 1) == p;
  return w;
}

__global__ void __launch_bounds__(256) k_soft_gfull(const float* __restrict__ g_half, int W, int H,
                                                    int X, int Y, float* __restrict__ g_left,
                                                    float* __restrict__ g_right) {
  const int u = blockIdx.x * 256 + threadIdx.x, v = blockIdx.y, img = blockIdx.z;
  if (u >= W) return;
  const float* gh = g_half + (size_t)img * X * Y;
  const int ya = v >> 1, yb = min((v + 1) >> 1, Y - 1);
  const int xa = u >> 1, xb = min((u + 1) >> 1, X - 1);
  const float g00 = gh[(size_t)ya * X + xa], g01 = gh[(size_t)ya * X + xb];
  const float g10 = gh[(size_t)yb * X + xa], g11 = gh[(size_t)yb * X + xb];
  const float wya = (float)gfull_weight(ya, v, H), wyb = yb != ya ? (float)gfull_weight(yb, v, H) : 0.f;
  const float wxa = (float)gfull_weight(xa, u, W), wxb = xb != xa ? (float)gfull_weight(xb, u, W) : 0.f;
  const float acc = (wya * (wxa * g00 + wxb * g01) + wyb * (wxa * g10 + wxb * g11)) *
                    (1.f / (9.f * 256.f));
  float* out = ((img & 1) ? g_right : g_left) + ((size_t)(img >> 1) * H * W + (size_t)v * W + u) * 3;
  out[0] = 77.f * acc;
  out[1] = 150.f * acc;
  out[2] = 29.f * acc;
}

// ------------------------------------------------------------ k_soft_lam
// Sum of the per-workgroup lambda partials in a fixed order: thread t sums
// entries t + 1024 j into four accumulators (j mod 4), then a tree.
// grid: 1, block 1024.
__global__ void __launch_bounds__(1024) k_soft_lam(const float2* __restrict__ part, int count,
                                                   float* __restrict__ g_lam) {
  __shared__ float2 s[1024];
  const int t = threadIdx.x;
  float2 acc[4] = {};
  int i = t, j = 0;
  for (; i + 3 * 1024 < count; i += 4 * 1024) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float2 v = part[i + u * 1024];
      acc[u].x += v.x;
      acc[u].y += v.y;
    }
  }
  for (; i < count; i += 1024, ++j) {
    const float2 v = part[i];
    acc[j & 3].x += v.x;
    acc[j & 3].y += v.y;
  }
  s[t] = make_float2((acc[0].x + acc[1].x) + (acc[2].x + acc[3].x),
                     (acc[0].y + acc[1].y) + (acc[2].y + acc[3].y));
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) {
      s[t].x += s[t + o].x;
      s[t].y += s[t + o].y;
    }
    __syncthreads();
  }
  if (t == 0) {
    g_lam[0] = s[0].x;
    g_lam[1] = s[0].y;
  }
}

// ----------------------------------------------------------- k_fill_f32
__global__ void k_fill_f32(float* __restrict__ p, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------- k_l1_*
// L = (1/n) sum over pairs of mean over {(x,y): nonocc(2x,2y)} of
// |2 d_hat(x,y) - GT(2x,2y)|; dL/dd_hat = 2 sign(2 d_hat - GT) / (n count)
// there (sign(0) = 0), 0 elsewhere.
// k_l1_partial grid: (nblk, n), block 256; partial sums per block.  Block b
// takes the rows b, b + nblk, ...; each thread four columns of a row at a
// time, their loads issued together (columns past X clamped, then not
// counted); a fixed-order reduction over the block.
__global__ void __launch_bounds__(256) k_l1_partial(const float* __restrict__ dhat,
                                                    const int16_t* __restrict__ gt,
                                                    const uint8_t* __restrict__ nonocc, int W,
                                                    int H, int X, int Y,
                                                    float2* __restrict__ part) {
  __shared__ float2 s[4];
  const int t = threadIdx.x, pair = blockIdx.y;
  const int npix = X * Y;
  float sum = 0.f, cnt = 0.f;
  for (int y = blockIdx.x; y < Y; y += gridDim.x) {
    const size_t fr = (size_t)pair * H * W + (size_t)(2 * y) * W;
    const float* dr = dhat + (size_t)pair * npix + (size_t)y * X;
    for (int x0 = 0; x0 < X; x0 += 4 * 256) {
      float dv[4];
      int gv[4];
      uint32_t mv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int x = min(x0 + t + 256 * k, X - 1);
        dv[k] = dr[x];
        gv[k] = gt[fr + 2 * x];
        mv[k] = nonocc[fr + 2 * x];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool use = x0 + t + 256 * k < X && mv[k] != 0u;
        sum += use ? fabsf(2.f * dv[k] - (float)gv[k]) : 0.f;
        cnt += use ? 1.f : 0.f;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_xor(sum, o, 64);
    cnt += __shfl_xor(cnt, o, 64);
  }
  if ((t & 63) == 0) s[t >> 6] = make_float2(sum, cnt);
  __syncthreads();
  if (t == 0) {
    float2 r = s[0];
    for (int w = 1; w < 4; ++w) {
      r.x += s[w].x;
      r.y += s[w].y;
    }
    part[(size_t)pair * gridDim.x + blockIdx.x] = r;
  }
}

// k_l1_final grid: 1, block 256: loss and the per-pair counts.  Wave w takes
// the pairs w, w + 4, ...: lane b sums the blocks b, b + 64, ... of a pair,
// then a butterfly over the lanes; the per-pair means are summed in pair
// order (a fixed order: the result does not depend on scheduling).
__global__ void __launch_bounds__(256) k_l1_final(const float2* __restrict__ part, int nblk,
                                                  int npair, float* __restrict__ loss,
                                                  float* __restrict__ counts) {
  __shared__ float s_mean[64];  // npair <= 64
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int p = wave; p < npair; p += 4) {
    float s = 0.f, c = 0.f;
#pragma unroll 4
    for (int b = lane; b < nblk; b += 64) {
      const float2 v = part[(size_t)p * nblk + b];
      s += v.x;
      c += v.y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      s += __shfl_xor(s, o, 64);
      c += __shfl_xor(c, o, 64);
    }
    if (lane == 0) {
      counts[p] = c;
      s_mean[p] = s / fmaxf(c, 1.f);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float total = 0.f;
    for (int p = 0; p < npair; ++p) total += s_mean[p];
    *loss = total / (float)npair;
  }
}

// k_l1_grad grid: (ceil(X*Y/256), n), block 256.
__global__ void __launch_bounds__(256) k_l1_grad(const float* __restrict__ dhat,
                                                 const int16_t* __restrict__ gt,
                                                 const uint8_t* __restrict__ nonocc,
                                                 const float* __restrict__ counts,
                                                 const float* __restrict__ gscale, int W, int H,
                                                 int X, int Y, int npair,
                                                 float* __restrict__ g_dhat) {
  const int i = blockIdx.x * 256 + threadIdx.x, pair = blockIdx.y;
  const int npix = X * Y;
  if (i >= npix) return;
  const int y = i / X, x = i - y * X;
  const size_t f = (size_t)pair * H * W + (size_t)(2 * y) * W + 2 * x;
  // all loads issued together, the mask applied after
  const uint8_t m = nonocc[f];
  const float dv = dhat[(size_t)pair * npix + i], gv = (float)gt[f];
  const float cnt = counts[pair], sc = gscale ? *gscale : 1.f;
  const float r = 2.f * dv - gv;
  const float sg = r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f);
  float g = 2.f * sg / (fmaxf(cnt, 1.f) * (float)npair);
  if (gscale) g *= sc;
  g_dhat[(size_t)pair * npix + i] = m ? g : 0.f;
}

}  // namespace
}  // namespace stereo_dev
