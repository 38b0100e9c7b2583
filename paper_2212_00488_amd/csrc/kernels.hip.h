// Device kernels of the stereo path (gfx950, wave64).
//
// Pipeline per pair (Sec. IV, Step1-8), all integer arithmetic:
//   k_prep     RGB -> gray -> 3x3 mean at even coordinates    (Sec. III-A, Eq. 2)
//   k_feat     mini-census + cross arms of both half images    (Sec. III-B, III-C)
//   k_match    cost, x- and y-aggregation and WTA, fused: the  (Eq. 3-9)
//              cost volume never leaves the chip
//   k_wta      combine the d-chunk minima                       (Eq. 9)
//   k_refine   cross-check, 3x3 median and bilateral filling    (Eq. 10, Sec. III-E, Eq. 11)
//   k_upscale  bilateral x / linear y upscale to full res      (Step8)
//   k_gray_full, k_copy_out: the full-resolution mode's ends   (Sec. V)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "common.h"

namespace stereo_dev {
// Internal linkage: each source of the library that launches a kernel
// carries its own copy (no relocatable device code).
namespace {

constexpr int kTX = 64;           // k_match strip width = one wave
constexpr int kWaves = 16;        // k_match workgroup = 16 waves
constexpr int kThreads = kWaves * 64;
constexpr int kKMax = 34;         // most output rows per k_match thread (band <= 544 rows)
constexpr int kLdsBytes = 163840; // LDS per workgroup on gfx950
constexpr int kXcds = 8;          // accelerator complex dies, each with its own L2
constexpr int kXcdQueues = 4;     // workgroup dispatch queues per XCD (position mod 4)

// Position j of an XCD's workgroup sequence -> (local group, d-chunk), for
// nloc groups of nchunk chunks each, nfull of them full-size and, when
// nchunk > nfull, one shorter remainder chunk.  Workgroup j waits in the
// XCD's dispatch queue j % kXcdQueues for a CU of that queue.  The remainder
// chunks take the last positions of one queue, T-1, T-1-4, ... (T = nloc *
// nchunk), so that the workgroups past the first round follow short ones
// there; where that does not fit they simply come last.
__device__ __forceinline__ void chunk_at(int j, int nloc, int nfull, int nchunk, int& local,
                                         int& chunk) {
  const int T = nloc * nchunk;
  if (nchunk == nfull) {
    local = j / nfull;
    chunk = j - local * nfull;
  } else if (kXcdQueues * (nloc - 1) > T - 1) {
    local = j < nloc * nfull ? j / nfull : j - nloc * nfull;
    chunk = j < nloc * nfull ? j - local * nfull : nfull;
  } else {
    const int q = T - 1 - j;  // remainder chunks at q = 0, 4, ..., 4 (nloc - 1)
    if (q % kXcdQueues == 0 && q / kXcdQueues < nloc) {
      local = nloc - 1 - q / kXcdQueues;
      chunk = nfull;
    } else {
      const int i = j - max(0, nloc - (q / kXcdQueues + 1));  // full chunks before j
      local = i / nfull;
      chunk = i - local * nfull;
    }
  }
}
constexpr int kRowBatch = 2;      // k_match rows whose lookups and scans interleave


__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
__device__ __forceinline__ int gray_of(const uint8_t* p) {
  return (77 * p[0] + 150 * p[1] + 29 * p[2] + 128) >> 8;
}

// ---------------------------------------------------------------- k_prep
// One workgroup = 64 x 8 half-res pixels of one image.  The gray values of
// the full-res rows 2 y0 - 1 .. 2 y0 + 15 and columns 2 x0 - 4 .. 2 x0 + 131
// (borders clamped) go to LDS; each thread then forms the rounded-half-up
// mean of the 3x3 block centred on (2x, 2y) for two output rows.  Where the
// tile's columns lie inside the image, rows start 4-byte aligned (W a
// multiple of 4, aligned base) and a thread reads 4 RGB pixels as three
// aligned words; each gray is then one byte-align and one 4-byte dot product.
// Elsewhere each pixel is read bytewise with clamped coordinates.
// grid: (ceil(X/64), ceil(Y/8), 2 * npair), block (64, 4).
constexpr int kPrepRows = 8;

__global__ void __launch_bounds__(256) k_prep(PairPtrs pp, int W, int H, int X, int Y,
                                              uint8_t* __restrict__ half) {
  constexpr int TR = 2 * kPrepRows + 1, TC = 136, TG = TC / 4;  // TG groups of 4 pixels a row
  constexpr uint32_t kGrayW = 77u | 150u << 8 | 29u << 16;      // gray weights per byte
  __shared__ __align__(4) uint8_t g[TR + 1][TC];  // row TR takes the stores of idle items
  const int x0 = blockIdx.x * 64, y0 = blockIdx.y * kPrepRows, img = blockIdx.z;
  const int pair = img >> 1;
  const uint8_t* rgb = (img & 1) ? pp.right[pair] : pp.left[pair];
  const int t = threadIdx.y * 64 + threadIdx.x, cb = 2 * x0 - 4;  // tile column 0
  const bool words = (W & 3) == 0 && (reinterpret_cast<uintptr_t>(rgb) & 3u) == 0 && cb >= 0 &&
                     cb + TC <= W;
  constexpr int NG = (TR * TG + 255) / 256;  // groups of 4 pixels per thread
  if (words) {
    uint32_t w[NG][3];
#pragma unroll
    for (int k = 0; k < NG; ++k) {  // all loads first; groups past the tile repeat its last
      const int gi = min(t + 256 * k, TR * TG - 1), r = gi / TG, c = 4 * (gi - r * TG);
      const uint32_t* q = reinterpret_cast<const uint32_t*>(
          rgb + ((size_t)clampi(2 * y0 - 1 + r, 0, H - 1) * W + cb + c) * 3);
      w[k][0] = q[0];
      w[k][1] = q[1];
      w[k][2] = q[2];
    }
#pragma unroll
    for (int k = 0; k < NG; ++k) {  // no branch, so no load is sunk next to its use
      const int gi = t + 256 * k;
      const int r = gi < TR * TG ? gi / TG : TR, c = gi < TR * TG ? 4 * (gi - r * TG) : 0;
      // pixel i's bytes start at byte 3i of the 12
      const uint32_t p0 = w[k][0], p1 = __builtin_amdgcn_alignbyte(w[k][1], w[k][0], 3),
                     p2 = __builtin_amdgcn_alignbyte(w[k][2], w[k][1], 2),
                     p3 = __builtin_amdgcn_alignbyte(w[k][2], w[k][2], 1);
      const uint32_t g0 = __builtin_amdgcn_udot4(p0 & 0xffffffu, kGrayW, 128u, false) >> 8;
      const uint32_t g1 = __builtin_amdgcn_udot4(p1 & 0xffffffu, kGrayW, 128u, false) >> 8;
      const uint32_t g2 = __builtin_amdgcn_udot4(p2 & 0xffffffu, kGrayW, 128u, false) >> 8;
      const uint32_t g3 = __builtin_amdgcn_udot4(p3 & 0xffffffu, kGrayW, 128u, false) >> 8;
      *reinterpret_cast<uint32_t*>(&g[r][c]) = g0 | g1 << 8 | g2 << 16 | g3 << 24;
    }
  } else {
    constexpr int NP = (TR * TC + 255) / 256;  // pixels per thread
    uint32_t px[NP][3];
#pragma unroll
    for (int k = 0; k < NP; ++k) {  // all loads first, clamped into the image
      const int pi = min(t + 256 * k, TR * TC - 1), r = pi / TC, c = pi - r * TC;
      const uint8_t* q = rgb + ((size_t)clampi(2 * y0 - 1 + r, 0, H - 1) * W +
                                clampi(cb + c, 0, W - 1)) * 3;
      px[k][0] = q[0];
      px[k][1] = q[1];
      px[k][2] = q[2];
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int pi = t + 256 * k;
      const int r = pi < TR * TC ? pi / TC : TR, c = pi < TR * TC ? pi - r * TC : 0;
      g[r][c] = (uint8_t)((77 * px[k][0] + 150 * px[k][1] + 29 * px[k][2] + 128) >> 8);
    }
  }
  __syncthreads();
  const int lx = threadIdx.x, x = x0 + lx;
  if (x >= X) return;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int ly = threadIdx.y + 4 * k, y = y0 + ly;
    if (y >= Y) break;
    int s = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i) s += g[2 * ly + j][2 * lx + 3 + i];
    half[(size_t)img * X * Y + (size_t)y * X + x] = (uint8_t)((s + 4) / 9);
  }
}

// ---------------------------------------------------------------- k_feat
// Packed half-res pixels.  The differentiable head takes {the float half
// image value's bits, census string} (8 bytes).  k_match takes gray in
// bits 0..7 and the census string in bits 8..13 (16 bits), two pixels per
// 32-bit load; that plane is stored twice, the second copy one pixel to the
// right, so that the pair of pixels starting at any column is one aligned
// word of one of the copies (half the bytes per row of the 32-bit form, which
// k_match's row loads are bound by).
constexpr int kFeatRows = 16;    // output rows per k_feat workgroup (one pixel per thread)
constexpr int kMaxArm = 127;

// Columns left of a 64-column strip in k_match's row buffer for a horizontal
// arm cap: arm + 1, rounded up to even (the row pass takes column pairs).
__host__ __device__ constexpr int row_halo(int arm_cap) { return (arm_cap + 2) & ~1; }

// Length of one arm of a pixel of value c: the number of steps t = 1, 2, ...
// along the axis, taken without a break, whose pixel satisfies |I - c| < delta,
// at most lim.  p points at the pixel in an LDS tile and STRIDE is the tile
// distance of one step (negative for the left / upper arm).  Steps are tested
// in chunks of up to 32 into a bitmask of the steps that fail, step t of a
// chunk in bit t-1, built from the farthest step down; the chunk's run is the
// number of trailing zeros.  A test is two VALU ops: v_sad_u16 forms
// |v - c| + 2^31 - delta, whose bit 31 is [|v - c| >= delta], and
// v_alignbit_b32 shifts that bit into the mask.  A chunk's loads are all
// issued before its first test.  The last chunk tests the cap rounded up to a
// multiple of 8 steps (a wave-uniform choice among four unrolled forms): the
// steps past the cap only set bits above it, which lim (<= cap) cuts off, and
// the tile holds kArmPad spare pixels for them.
constexpr int kArmPad = 7;

// Run of passing steps 1..N (N <= 32) from p, bias = 2^31 - delta.
template <int STRIDE, int N>
__device__ __forceinline__ int arm_run(const uint8_t* p, uint32_t c, uint32_t bias) {
  // one byte load per step (merged into wide loads, each byte would take
  // one more VALU op to extract; the compiler barrier keeps them apart)
  uint32_t v[N];
#pragma unroll
  for (int t = 1; t <= N; ++t) {
    v[t - 1] = p[t * STRIDE];
    __asm__ volatile("" ::: "memory");
  }
  // the bits above N - 1 start as failures, so a chunk of fewer than 32
  // steps ends its run at N at most
  uint32_t m = 0xffffffffu;
#pragma unroll
  for (int t = N; t >= 1; --t)
    m = __builtin_amdgcn_alignbit(m, __builtin_amdgcn_sad_u16(v[t - 1], c, bias), 31);
  return m == 0u ? 32 : __builtin_ctz(m);
}

template <int STRIDE>
__device__ __forceinline__ int arm_len(const uint8_t* p, int c, int delta, int cap, int lim) {
  if (delta <= 0 || cap <= 0) return 0;
  const uint32_t bias = 0x80000000u - (uint32_t)delta;
  const uint32_t cu = (uint32_t)c;
  int len = 0;
  bool alive = true;
  for (; cap > 32; cap -= 32, p += 32 * STRIDE) {
    const int run = arm_run<STRIDE, 32>(p, cu, bias);
    len += alive ? run : 0;
    alive = alive && run == 32;
  }
  int run;
  switch ((cap + 7) >> 3) {
    case 1: run = arm_run<STRIDE, 8>(p, cu, bias); break;
    case 2: run = arm_run<STRIDE, 16>(p, cu, bias); break;
    case 3: run = arm_run<STRIDE, 24>(p, cu, bias); break;
    default: run = arm_run<STRIDE, 32>(p, cu, bias); break;
  }
  len += alive ? run : 0;
  return min(len, lim);
}

// One workgroup = 64 columns x kFeatRows rows of one image, one pixel per
// thread.  Two LDS tiles of the half image (borders clamped): rows y0-1 ..
// y0+kFeatRows over the columns reachable by the horizontal arms and the
// census, and rows y0-arm_y .. y0+kFeatRows-1+arm_y over the 64 columns for
// the vertical arms, each with kArmPad spare pixels past the arms.
//   census: 6 neighbours in three rows, bit k = [neighbour < centre]
//   arms  : contiguous pixels with |I - I(centre)| < delta, capped per side
//           and at the image border; packed m | n<<8 | M<<16 | N<<24
// Pixels go to sp ({bits of half_f at the pixel (an unpadded [Y][X] plane per
// image), census}, may be NULL) and to the two copies of pk16 (gray | census
// << 8, may be NULL; the second copy copy16 elements after the first, one
// pixel to the right); pitch XP, column x at pad + x.
// xoff (may be NULL) takes, for k_match's row pass, the byte offsets in a
// wave's row buffer of the row-prefix entries that bound CA_x (Eq. 7) at x:
// 4 (x mod 64 + h - m - 1) in bits 0..15 and 4 (x mod 64 + h + n) in bits
// 16..31, h = row_halo(cap) of the image; pitch XA like arms.
// Two workgroups share a CU only while a wave holds at most 80 SGPRs; the
// waves-per-EU bound keeps the compiler under that (above it the kernel took
// a fifth longer).
// grid: (ceil(X/64), ceil(Y/kFeatRows), 2 * npair), block (64, kFeatRows).
__global__ void __launch_bounds__(64 * kFeatRows) __attribute__((amdgpu_waves_per_eu(8)))
k_feat(const uint8_t* __restrict__ half, int X, int Y, int delta, int arm_x_l, int arm_x_r,
       int arm_y, int XP, int pad, int XA, const float* __restrict__ half_f,
       uint2* __restrict__ sp, uint32_t* __restrict__ arms, uint32_t* __restrict__ xoff,
       uint16_t* __restrict__ pk16, size_t copy16) {
  constexpr int TXW = 64 + 2 * (kMaxArm + kArmPad);
  __shared__ uint8_t tx[kFeatRows + 2][TXW];
  __shared__ uint8_t ty[kFeatRows + 2 * (kMaxArm + kArmPad)][64];
  const int x0 = blockIdx.x * 64, y0 = blockIdx.y * kFeatRows, img = blockIdx.z;
  const uint8_t* h = half + (size_t)img * X * Y;
  // horizontal cap of this image (the two images may differ, Sec. V)
  const int arm_x = (img & 1) ? arm_x_r : arm_x_l;
  // tile margins: the arms plus the spare steps (at least the census's 2)
  const int hx = arm_x + kArmPad, wx = 64 + 2 * hx;
  const int my = arm_y + kArmPad, hy = kFeatRows + 2 * my;
  // Tile loads: the loads of both tiles' first batches are issued before
  // the first store (one load, wait and store after another was bound by
  // memory latency); larger caps take more batches.  Rows and columns past a
  // tile's end are clamped to its last one: such a load and store repeat a
  // valid one with the same value.
  {
    const int r0 = (int)threadIdx.y, r1 = min(r0 + kFeatRows, kFeatRows + 1);
    const uint8_t* s0 = h + (size_t)clampi(y0 - 1 + r0, 0, Y - 1) * X;
    const uint8_t* s1 = h + (size_t)clampi(y0 - 1 + r1, 0, Y - 1) * X;
    const uint8_t* sc = h + clampi(x0 + (int)threadIdx.x, 0, X - 1);
    // tx: rows r0, r1 and columns c0 + lane, c0 + 64 + lane
    auto load_x = [&](int c0, int* cc, uint8_t* v) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        cc[k] = min(c0 + 64 * k + (int)threadIdx.x, wx - 1);
        const int gx = clampi(x0 - hx + cc[k], 0, X - 1);
        v[2 * k] = s0[gx];
        v[2 * k + 1] = s1[gx];
      }
    };
    auto store_x = [&](const int* cc, const uint8_t* v) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        tx[r0][cc[k]] = v[2 * k];
        tx[r1][cc[k]] = v[2 * k + 1];
      }
    };
    // ty: rows (j0 + j) * kFeatRows + r0, j < 8, of column lane
    auto load_y = [&](int j0, int* rr, uint8_t* v) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        rr[j] = min((j0 + j) * kFeatRows + r0, hy - 1);
        v[j] = sc[(size_t)clampi(y0 - my + rr[j], 0, Y - 1) * X];
      }
    };
    auto store_y = [&](const int* rr, const uint8_t* v) {
#pragma unroll
      for (int j = 0; j < 8; ++j) ty[rr[j]][threadIdx.x] = v[j];
    };
    int cc[2], rr[8];
    uint8_t vx[4], vy[8];
    load_x(0, cc, vx);
    load_y(0, rr, vy);
    store_x(cc, vx);
    store_y(rr, vy);
    for (int c0 = 128; c0 < wx; c0 += 128) {
      load_x(c0, cc, vx);
      store_x(cc, vx);
    }
    for (int j0 = 8; j0 * kFeatRows < hy; j0 += 8) {
      load_y(j0, rr, vy);
      store_y(rr, vy);
    }
  }
  __syncthreads();
  const int lx = threadIdx.x, x = x0 + lx, ly = threadIdx.y, y = y0 + ly;
  const bool inside = x < X && y < Y;
  uint32_t p16 = 0;
  if (inside) {
    const uint8_t* row = &tx[ly + 1][hx + lx];   // row[i] = I(x + i, y)
    const int c = row[0];
    int bits = 0;
    bits |= (tx[ly][hx + lx - 1] < c) << 0;
    bits |= (tx[ly][hx + lx + 1] < c) << 1;
    bits |= (row[-2] < c) << 2;
    bits |= (row[2] < c) << 3;
    bits |= (tx[ly + 2][hx + lx - 1] < c) << 4;
    bits |= (tx[ly + 2][hx + lx + 1] < c) << 5;
    const uint8_t* col = &ty[ly + my][lx];       // col[64 i] = I(x, y + i)
    const int m = arm_len<-1>(row, c, delta, arm_x, min(arm_x, x));
    const int n = arm_len<1>(row, c, delta, arm_x, min(arm_x, X - 1 - x));
    const int M = arm_len<-64>(col, c, delta, arm_y, min(arm_y, y));
    const int N = arm_len<64>(col, c, delta, arm_y, min(arm_y, Y - 1 - y));
    if (sp)
      sp[((size_t)img * Y + y) * XP + pad + x] =
          make_uint2(__float_as_uint(half_f[((size_t)img * Y + y) * X + x]), (uint32_t)bits);
    arms[((size_t)img * Y + y) * XA + x] =
        (uint32_t)m | ((uint32_t)n << 8) | ((uint32_t)M << 16) | ((uint32_t)N << 24);
    if (xoff) {
      const uint32_t lh = (uint32_t)(lx + row_halo(arm_x));
      xoff[((size_t)img * Y + y) * XA + x] = 4u * (lh - (uint32_t)m - 1u) | 4u * (lh + (uint32_t)n) << 16;
    }
    p16 = (uint32_t)c | (uint32_t)bits << 8;
  }
  if (pk16) {
    // pairs (x, x + 1) as aligned words: copy 0 from the even columns, copy 1
    // (one column to the right) from the odd ones, the pixel x + 1 from the
    // next lane (one wave is one row of the tile); the copy-1 pair across two
    // workgroups (lane 63 here, lane 0 of the next) is written in halves
    const uint32_t nb = (uint32_t)__shfl_down((int)p16, 1, 64);
    if (inside) {
      uint16_t* q = pk16 + ((size_t)img * Y + y) * XP + pad + x;
      if ((lx & 1) == 0) {
        *reinterpret_cast<uint32_t*>(q) = p16 | nb << 16;
        if (lx == 0) q[copy16 + 1] = (uint16_t)p16;
      } else if (lx != 63) {
        *reinterpret_cast<uint32_t*>(q + copy16 + 1) = p16 | nb << 16;
      } else {
        q[copy16 + 1] = (uint16_t)p16;
      }
    }
  }
}

// ---------------------------------------------------------------- k_match
// Inclusive prefix sum over the 64 lanes of a wave (DPP row shifts inside
// rows of 16 lanes, then row broadcasts across rows).
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
  v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}


// Keeps the compiler from moving LDS accesses of one wave across this point;
// the LDS itself serves the accesses of a wave in issue order.
#define WAVE_LDS_ORDER() __asm__ volatile("" ::: "memory")

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}

// cost table [h'][signed brightness difference + 256], h' = census distance
// h (rows 0..6) or h + 7 for a match outside the other image (rows 7..13, all
// C_max): 14 rows of 511 entries.  The row pitch, 530 entries = 265 words,
// is 9 banks mod 64: entries of rows 1..6 apart land 9, 18, ..., 54 banks
// apart, so lookups of neighbouring pixels (census distances a row or two
// apart, brightness differences a few entries apart) rarely share a bank
// (bank conflicts of the lookups 8.6 M -> 6.8 M cycles per launch against a
// pitch of 257 words, 1 bank mod 64)
constexpr int kTabPitch = 530;
constexpr int kTabRows = 14;
constexpr int kTab = kTabRows * kTabPitch;
constexpr int kOutBias = 7;       // added to h for a match outside the image

// Values the device cost table is built from: the tables of Eq. 4 (AD) and
// Eq. 5 (census) in fixed point, computed on the host in double, and C_max.
struct TabArgs {
  uint16_t ad[256];
  uint16_t mc[7];
  uint16_t cmax;
};

// Set-up of a plan's device state, ordered on the plan's stream (no memset
// node, so it may be captured in a graph): clears nzero words at zero (the
// padding of the pixel and arm planes must read 0; the kernels write the
// image part) and writes the cost table, entry (h', 256 + diff) = LUT_AD[|diff|]
// + LUT_MC[h'] for h' < kOutBias, else C_max; column 0 and the pitch's spare
// columns 0.
// grid: any, block 256.
__global__ void __launch_bounds__(256) k_plan_init(uint32_t* __restrict__ zero, size_t nzero,
                                                   uint16_t* __restrict__ tab, TabArgs t) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nzero; i += stride)
    zero[i] = 0u;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)kTab; i += stride) {
    const int h = (int)i / kTabPitch, col = (int)i - h * kTabPitch;
    const int a = col < 256 ? 256 - col : col - 256;
    // columns 1..511 hold differences -255..255; column 0 (a difference of
    // -256) and the spare columns are never read
    tab[i] = (col == 0 || col > 511) ? (uint16_t)0
                                     : (h < kOutBias ? (uint16_t)(t.ad[a] + t.mc[h]) : t.cmax);
  }
}

// Bytes of k_match's static LDS: the cost table.
constexpr int kMatchTabBytes = ((kTab * 2 + 15) / 16) * 16;

// Bytes of k_match's dynamic LDS block with NS sub-passes and a plane of
// `rows` rows (plane row 0 is the zero row): row buffers, segment totals and
// the plane.
__host__ __device__ constexpr int match_lds_bytes(int ns, int rows) {
  return kWaves * ns * 128 * 4 + kWaves * 64 * 4 + rows * 64 * 4;
}

// LDS rows of the k_match plane for NS sub-passes of 128 row-buffer columns.
__host__ __device__ constexpr int plane_rows(int ns) {
  return (kLdsBytes - kTab * 2 - kWaves * 64 * 4 - kWaves * ns * 128 * 4) / 256 - 2;
}

struct MatchArgs {
  const uint16_t* pk;     // [2][2*npair][Y][XP]  padded: gray | census << 8, two copies
  const uint32_t* arms;   // [2*npair][Y][XA]  zero past column X
  const uint32_t* xoff;   // [2*npair][Y][XA]  row-buffer offsets (k_feat), zero past column X
  const uint16_t* tab;    // [kTabRows][kTabPitch]
  uint32_t* keys;         // [npair][nchunk][2][nk]  (min CA) << dbits | argmin d
  int X, Y, XP, pad, XA, nk, arm_x, arm_x_r, arm_y;
  int dbits;              // key = CA << dbits | d
  int nbands, dlo, dhi;
  int csize, nchunk;      // d-chunk size; chunks = ceil((dhi - dlo) / csize), the last the remainder
  int nstrips, ngroups;   // groups = strips x bands x 2 bases x pairs
  uint32_t pk_bytes, arms_bytes;  // sizes of the pk (both copies) and arms buffers
  uint32_t copy_bytes;    // bytes from the first pk copy to the second
  // debug planes (pair 0, the single disparity dlo; used by the DBG variant)
  uint16_t* dbg_cost;
  uint32_t* dbg_cax;
  uint32_t* dbg_ca;
  int dbg_base;
};

// One workgroup = one 64-column strip x one band of rows x one base image
// x one chunk of disparities; 16 waves.  For each d of the chunk:
//   row pass   : each wave takes rows of the band; every lane evaluates the
//                cost (Eq. 3-5, one lookup in a table indexed by census distance
//                and signed brightness difference) of two adjacent columns of
//                the strip plus arm_x+1 (rounded up to even) columns on either
//                side, an inclusive wave scan gives the row prefix P, and
//                CA_x = P[x+n] - P[x-m-1] (Eq. 7) goes into the LDS plane;
//   column pass: segmented prefix down each column of the plane, in place, then
//                CA = Q[y+N] - Q[y-M-1] (Eq. 8) for the band's output rows and
//                key = min(key, CA << dbits | d): the smallest d wins ties (Step5).
// The right-based cost is evaluated as cost(R(x), L(x+d)), which is C^L(x+d)
// of Eq. 6 term for term.  Sums wrap modulo 2^32; every difference taken is a
// window sum below 2^(32 - dbits) (the parameter check), hence exact and room
// for d in the key's low dbits.  KMAX (<= kKMax) bounds the output rows
// per thread: a band has at most 16 * KMAX output rows.
// grid: ceil(groups / 8) * 8 * nchunk workgroups (1-D), block 1024.
template <int NS, int KMAX, bool DBG>
__global__ void __launch_bounds__(kThreads) k_match(MatchArgs a) {
  constexpr int PR = plane_rows(NS);
  // The cost table is the kernel's static LDS, at LDS address 0, so table
  // addresses fold into the read's offset field.  The rest is one dynamic
  // block carved at constant offsets, sized by the host to the plane rows the
  // plan reads (match_lds_bytes), at most PR + 1: LDS the plan does not need
  // is left to the kernels of other streams (the next frame's), which can
  // then share the CU.
  constexpr int kOffRow = 0;
  constexpr int kOffSeg = kOffRow + kWaves * NS * 128 * 4;
  constexpr int kOffPlane = kOffSeg + kWaves * 64 * 4;
  static_assert(kMatchTabBytes + kOffPlane + (PR + 1) * 64 * 4 <= kLdsBytes, "LDS block");
  __shared__ __align__(16) uint16_t s_tab[kMatchTabBytes / 2];
  extern __shared__ __align__(16) uint8_t s_lds[];
  auto s_row = reinterpret_cast<uint32_t(*)[NS * 128]>(s_lds + kOffRow);
  auto s_seg = reinterpret_cast<uint32_t(*)[64]>(s_lds + kOffSeg);
  uint32_t* s_plane = reinterpret_cast<uint32_t*>(s_lds + kOffPlane);  // row 0 = zeros

  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // uniform: row offsets stay scalar
  const int X = a.X, Y = a.Y;
  // Workgroups are dealt to the 8 XCDs in turn (id mod 8).  All d-chunks of
  // one (strip, band, base, pair) group read the same image rows, so they are
  // given ids of one residue mod 8: the group's rows stay in one XCD's L2;
  // chunk_at orders each XCD's sequence for its dispatch queues.
  const int wg = blockIdx.x, xcd = wg & (kXcds - 1), j = wg / kXcds;
  int local, chunk;
  chunk_at(j, (a.ngroups + kXcds - 1) / kXcds, (a.dhi - a.dlo) / a.csize, a.nchunk, local, chunk);
  int group = local * kXcds + xcd;
  if (group >= a.ngroups) return;  // padding workgroup
  const int strip = group % a.nstrips;
  group /= a.nstrips;
  const int band = group % a.nbands;
  group /= a.nbands;
  const int base = group & 1, pair = group >> 1;
  const int x0 = strip * kTX;
  const int ob = (Y + a.nbands - 1) / a.nbands;
  const int y0 = band * ob, y1 = min(Y, y0 + ob);
  const int ya = max(0, y0 - a.arm_y), yb = min(Y, y1 + a.arm_y);
  const int nb = yb - ya, o0 = y0 - ya, o1 = y1 - ya;
  const int d0 = a.dlo + chunk * a.csize, d1 = min(a.dhi, d0 + a.csize);
  // row buffer starts at column x0 - hx (even); hx covers this base's arms
  const int hx = row_halo(base ? a.arm_x_r : a.arm_x);
  const int sgn = base ? 1 : -1;       // other-image column is x + sgn * d
  const __amdgpu_buffer_rsrc_t rb = buffer_rsrc(a.pk, a.pk_bytes);
  const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(a.xoff, a.arms_bytes);
  const uint32_t img_b = (uint32_t)(2 * pair + base), img_o = (uint32_t)(2 * pair + (base ^ 1));
  const uint32_t pkrow = (uint32_t)a.XP * 2u, armrow = (uint32_t)a.XA * 4u;
  const bool dbg = DBG && pair == 0 && base == a.dbg_base;
  (void)dbg;

  for (int i = t; i < kTab; i += kThreads) s_tab[i] = a.tab[i];
  if (t < 64) s_plane[t] = 0u;

  const int c = lane, x = x0 + lane;
  // rows of the band in segments of whole row pairs (the row pass takes its
  // rows in pairs), one per wave in order, the pairs split as evenly as
  // possible: the waves of each SIMD (wave mod 4) then share the rows evenly
  const int nbat = (nb + 1) / 2, bq = nbat / kWaves, br = nbat % kWaves;
  const int r0 = min(nb, 2 * (wave * bq + min(wave, br)));
  const int r1 = min(nb, r0 + 2 * (bq + (wave < br)));

  // Output rows of this thread: r = o0 + wave + 16 k.  marm[k / 2] packs the
  // vertical arms (M, N) of two such rows, one byte each.  Rows outside the
  // band or columns outside the image get M = N = 0; their keys are never
  // stored.
  static_assert(KMAX % 2 == 0, "KMAX must be even");
  uint32_t key[KMAX], marm[KMAX / 2];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    key[k] = 0xffffffffu;
    const int r = o0 + wave + k * kWaves;
    // no branch around the load (a branch made every load wait for the one
    // before): rows past the band read its last row and are masked by a
    // wave-uniform select; columns past X read the plane's zero padding
    const uint32_t v = a.arms[((size_t)img_b * Y + ya + min(r, o1 - 1)) * a.XA + x] >> 16;
    const uint32_t mn = r < o1 ? v : 0u;
    if (k & 1) marm[k / 2] |= mn << 16;
    else marm[k / 2] = mn;
  }
  // byte offset in the plane of (band row o0 + wave, column c); plane row =
  // band row + 1
  const uint32_t fin_b = (uint32_t)((o0 + wave + 1) * 64 + c) * 4u;
  // the key shift lives in a VGPR, so that shift-and-or with the scalar d
  // is one instruction (one scalar operand per vector instruction)
  uint32_t vdbits = (uint32_t)a.dbits;
  __asm__ volatile("" : "+v"(vdbits));
  // byte selector of v_perm: bytes 0 and 2 of marm (M of two rows) to bytes
  // 1 and 3, zeros to bytes 0 and 2
  uint32_t kpermM = 0x020c000cu;
  __asm__ volatile("" : "+v"(kpermM));
  // byte offset of this lane's first column pair inside a padded pk row
  const uint32_t vb = (uint32_t)(a.pad + x0 - hx + 2 * lane) * 2u;
  __syncthreads();

  const char* tb = reinterpret_cast<const char*>(s_tab) + 512;
  // cost of pixel J of a pair word: entry (h + bias, 256 + diff) at byte
  // offset (h + bias) * 2 * kTabPitch + 2 * diff + 512; the census distance h
  // is the popcount of the xor of the census bytes (one SDWA xor), and the
  // popcount instruction adds the bias
  auto cost = [&](uint32_t b, uint32_t o, uint32_t bias, auto J) -> uint32_t {
    uint32_t hx;
    if constexpr (decltype(J)::value == 0)
      __asm__("v_xor_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_1 "
              "src1_sel:BYTE_1" : "=v"(hx) : "v"(b), "v"(o));
    else
      __asm__("v_xor_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_3 "
              "src1_sel:BYTE_3" : "=v"(hx) : "v"(b), "v"(o));
    constexpr int sh = decltype(J)::value * 16;
    const uint32_t h = __builtin_popcount(hx) + bias;
    const int df = (int)((b >> sh) & 255u) - (int)((o >> sh) & 255u);
    const int e = (int)h * (2 * kTabPitch) + df + df;
    return *reinterpret_cast<const uint16_t*>(tb + e);
  };
  using J0 = std::integral_constant<int, 0>;
  using J1 = std::integral_constant<int, 1>;
  const uint32_t vx = (uint32_t)x * 4u;

  for (int d = d0; d < d1; ++d) {
    // a pair of other-image pixels starting at an odd column is an aligned
    // word of the second copy (the parity of the column is that of d)
    const uint32_t odd = (uint32_t)d & 1u;
    const uint32_t vo = vb + (uint32_t)(sgn * d * 2) + 2u * odd;
    const uint32_t ocopy = odd ? a.copy_bytes : 0u;
    // where the match oc of a column falls outside the other image, its cost
    // is C_max (the x - d < 0 / x + d >= X convention): the lookup takes the
    // table rows kOutBias.., which hold C_max, by a bias on the census distance
    uint32_t bias[NS][2];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int oc = x0 - hx + s * 128 + 2 * lane + j + sgn * d;
        bias[s][j] = (unsigned)oc < (unsigned)X ? 0u : (uint32_t)kOutBias;
      }
    // ---- row pass over this wave's rows r0..r1-1, kRowBatch rows at a time
    // (their lookups and scans interleave), the loads of the next batch in flight.
    // CA_x of a row is added to a running column sum, so the plane receives
    // the column prefix within the wave's segment of rows.
    struct RowIn { uint32_t b[NS], o[NS]; uint32_t am; };
    auto load_row = [&](int r, RowIn& in) {
      const uint32_t y = (uint32_t)(ya + r);
      const uint32_t sb = (img_b * (uint32_t)Y + y) * pkrow;
      const uint32_t so = (img_o * (uint32_t)Y + y) * pkrow + ocopy;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        in.b[s] = __builtin_amdgcn_raw_buffer_load_b32(rb, vb + s * 256, sb, 0);
        in.o[s] = __builtin_amdgcn_raw_buffer_load_b32(rb, vo + s * 256, so, 0);
      }
      in.am = __builtin_amdgcn_raw_buffer_load_b32(ra, vx, (img_b * (uint32_t)Y + y) * armrow, 0);
    };
    // row prefix of one row (cost pairs c0, c1 per lane and sub-pass) into the
    // row buffer, then CA_x of the lane's output column
    auto finish_row = [&](int r, const uint32_t (&c0)[NS], const uint32_t (&c1)[NS],
                          const uint32_t (&p1)[NS], uint32_t am) -> uint32_t {
      const int y = ya + r;
      uint32_t carry = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const uint32_t p = p1[s] + carry;
        if (NS > 1) carry = __builtin_amdgcn_readlane(p, 63);
        *reinterpret_cast<u32x2*>(&s_row[wave][s * 128 + 2 * lane]) = u32x2{p - c1[s], p};
        if (DBG && dbg && d == a.dlo && y >= y0 && y < y1) {
          const int xc = x0 - hx + s * 128 + 2 * lane;
          if (xc >= x0 && xc < x0 + kTX && xc < X) a.dbg_cost[(size_t)y * X + xc] = (uint16_t)c0[s];
          if (xc + 1 >= x0 && xc + 1 < x0 + kTX && xc + 1 < X)
            a.dbg_cost[(size_t)y * X + xc + 1] = (uint16_t)c1[s];
        }
      }
      WAVE_LDS_ORDER();
      // am: byte offsets of entries x + n and x - m - 1 in the row buffer
      const uint8_t* rw = reinterpret_cast<const uint8_t*>(s_row[wave]);
      const uint32_t cax = *reinterpret_cast<const uint32_t*>(rw + (am >> 16)) -
                           *reinterpret_cast<const uint32_t*>(rw + (am & 0xffffu));
      WAVE_LDS_ORDER();
      if (DBG && dbg && d == a.dlo && x < X && y >= y0 && y < y1) a.dbg_cax[(size_t)y * X + x] = cax;
      return cax;
    };
    uint32_t run = 0;
    // Rows go in batches of kRowBatch: their lookups and scans interleave.  A
    // batch running past the segment end loads its last row again in place
    // of the missing ones and never stores them.
    auto row_of = [&](int r, int i) { return r + i < r1 ? r + i : r1 - 1; };
    auto load_batch = [&](int r, RowIn (&in)[kRowBatch]) {
#pragma unroll
      for (int i = 0; i < kRowBatch; ++i) load_row(row_of(r, i), in[i]);
    };
    auto process_batch = [&](int r, const RowIn (&in)[kRowBatch]) {
      uint32_t c0[kRowBatch][NS], c1[kRowBatch][NS], pr[kRowBatch][NS];
#pragma unroll
      for (int i = 0; i < kRowBatch; ++i)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          c0[i][s] = cost(in[i].b[s], in[i].o[s], bias[s][0], J0{});
          c1[i][s] = cost(in[i].b[s], in[i].o[s], bias[s][1], J1{});
        }
#pragma unroll
      for (int i = 0; i < kRowBatch; ++i)
#pragma unroll
        for (int s = 0; s < NS; ++s) pr[i][s] = wave_scan_incl(c0[i][s] + c1[i][s]);
#pragma unroll
      for (int i = 0; i < kRowBatch; ++i) {
        // a row past the segment end (its last row again) is evaluated but
        // neither added nor stored: the plane row belongs to the next segment
        const uint32_t cax = finish_row(r + i, c0[i], c1[i], pr[i], in[i].am);
        if (i == 0 || r + i < r1) {
          run += cax;
          s_plane[(r + i + 1) * 64 + lane] = run;
        }
      }
    };
    // The next batch is loaded unconditionally (past the segment end it
    // reloads the last row): with the loads behind a branch, the waits at the
    // join must hold for the path with them in flight and the path without,
    // and the compiler then waited for the next batch too.
    RowIn in0[kRowBatch], in1[kRowBatch];  // two buffer sets, used in turn
    if (r0 < r1) load_batch(r0, in0);
    for (int r = r0; r < r1; r += 2 * kRowBatch) {
      load_batch(r + kRowBatch, in1);
      process_batch(r, in0);
      if (r + kRowBatch >= r1) break;
      load_batch(r + 2 * kRowBatch, in0);
      process_batch(r + kRowBatch, in1);
    }
    s_seg[wave][c] = run;
    __syncthreads();
    // ---- column pass: add the sum of the segments above to this segment.
    // Each plane entry belongs to one thread; the add is an LDS atomic without
    // return (ds_add_u32), one instruction per row and no read-add-write
    // latency chain.
    uint32_t off = 0;
#pragma unroll
    for (int s = 0; s < kWaves; ++s) {
      const uint32_t v = s_seg[s][c];
      off += s < wave ? v : 0u;
    }
    if (wave > 0) {
#pragma unroll 8
      for (int r = r0; r < r1; ++r)
        __hip_atomic_fetch_add(&s_plane[(r + 1) * 64 + c], off, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    // ---- vertical window and WTA for this wave's output rows
#pragma unroll
    for (int j = 0; j < KMAX / 2; ++j) {
      // byte offsets of plane rows +N and -(M+1) from the output rows 2j and
      // 2j+1: a plane row is 256 bytes, so an offset is an arm byte in bits
      // 8..15 of a 16-bit half: nw holds N of both rows in its halves, mw
      // holds M; each read address is then one SDWA add or subtract.
      // Volatile asm keeps them inside the d loop (hoisted, they would need
      // 32 VGPRs).
      uint32_t nw, mw;
      __asm__ volatile("v_and_b32 %0, 0xff00ff00, %1" : "=v"(nw) : "v"(marm[j]));
      __asm__ volatile("v_perm_b32 %0, 0, %1, %2" : "=v"(mw) : "v"(marm[j]), "v"(kpermM));
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 2 * j + h;
        // rows +N and -(M+1) of output row k (plane row 0 at least: M never
        // reaches above the band); the per-row part k * 4096 bytes becomes
        // the reads' immediate offset
        const uint8_t* row = s_lds + kOffPlane + k * kWaves * 256 + fin_b;
        const uint32_t on = h ? nw >> 16 : nw & 0xffffu, om = h ? mw >> 16 : mw & 0xffffu;
        const uint32_t ca = *reinterpret_cast<const uint32_t*>(row + on) -
                            *reinterpret_cast<const uint32_t*>(row - 256 - om);
        const uint32_t kv = (ca << vdbits) | (uint32_t)d;
        key[k] = kv < key[k] ? kv : key[k];
      }
    }
    __syncthreads();
  }

  int nout = o1 - o0 - wave;  // output rows left for this wave, from row k = 0
  __asm__ volatile("" : "+v"(nout));  // recompute the row tests here
  if (x < X) {
    uint32_t* out = a.keys + ((size_t)(pair * a.nchunk + chunk) * 2 + base) * a.nk;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int r = o0 + wave + k * kWaves;
      if (k * kWaves < nout) {
        out[(size_t)(ya + r) * X + x] = key[k];
        // a debug run covers the single disparity dlo, so the key holds CA
        if (DBG && dbg) a.dbg_ca[(size_t)(ya + r) * X + x] = key[k] >> a.dbits;
      }
    }
  }
}

// ----------------------------------------------------------------- k_wta
// Minimum key over the d-chunks for both bases: D = key & (2^dbits - 1)
// (Eq. 9; the key order makes the smallest d win ties), and the minimum
// aggregate key >> dbits when mincost != NULL.  Four pixels per thread; planes have the
// padded stride nk (a multiple of 64 pixels).
// grid: (ceil(nk / 1024), npair), block 256.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int16_t i16x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_wta(const uint32_t* __restrict__ keys, int nchunk,
                                             int nk, int dbits, int16_t* __restrict__ disp,
                                             uint32_t* __restrict__ mincost) {
  const int i = (blockIdx.x * 256 + threadIdx.x) * 4;
  const int pair = blockIdx.y;
  if (i >= nk) return;
  const uint32_t* kp = keys + (size_t)pair * nchunk * 2 * nk + i;
  // chunks in groups of kWtaGroup, all loads of a group (both bases) in
  // flight together; a group running past the last chunk reloads the last
  // one, which leaves the minimum unchanged
  constexpr int kWtaGroup = 8;
  u32x4 mb[2];
  mb[0] = mb[1] = u32x4{0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu};
  for (int c0 = 0; c0 < nchunk; c0 += kWtaGroup) {
    u32x4 v[kWtaGroup][2];
#pragma unroll
    for (int g = 0; g < kWtaGroup; ++g) {
      const int c = min(c0 + g, nchunk - 1);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        v[g][b] = *reinterpret_cast<const u32x4*>(kp + ((size_t)c * 2 + b) * nk);
    }
#pragma unroll
    for (int g = 0; g < kWtaGroup; ++g)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        mb[b].x = min(mb[b].x, v[g][b].x); mb[b].y = min(mb[b].y, v[g][b].y);
        mb[b].z = min(mb[b].z, v[g][b].z); mb[b].w = min(mb[b].w, v[g][b].w);
      }
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const u32x4 m = mb[b];
    const size_t o = (size_t)(2 * pair + b) * nk + i;
    const uint32_t dm = (1u << dbits) - 1u;
    *reinterpret_cast<i16x4*>(disp + o) =
        i16x4{(int16_t)(m.x & dm), (int16_t)(m.y & dm), (int16_t)(m.z & dm), (int16_t)(m.w & dm)};
    if (mincost)
      *reinterpret_cast<u32x4*>(mincost + o) =
          u32x4{m.x >> dbits, m.y >> dbits, m.z >> dbits, m.w >> dbits};
  }
}

// -------------------------------------------------------------- k_refine
// One workgroup per half-res row.  GCP(x) = [x - k >= 0 and D^R(x - k) = k],
// k = D^L(x) (Eq. 10); M = 3x3 median of D^L (borders clamped); GCPs keep M;
// a non-GCP takes the nearest GCPs left (x-i) and right (x+j): linear
// interpolation from M(x-i) toward M(x+j), rounded half up, when they differ
// by at most T, else the side of strictly closer brightness (the right one on
// a tie) (Sec. III-E).  One side only: copy it; none: 0.  fill_mode 1 and 2
// are the two simpler fills Sec. III-E describes first: the GCP closer in
// distance (the right one at equal distance), or the smaller disparity.
// The rows are staged in LDS, the GCP flags of the row become a bit array
// (one wave ballot per 64 columns), and each non-GCP finds its nearest GCPs
// by bit search in that array.
// grid: (Y, npair), block 256.
__device__ __forceinline__ int floor_div_pos(int n, int d) {  // d > 0
  return n >= 0 ? n / d : -((-n + d - 1) / d);
}

__device__ __forceinline__ int median9(int* v) {
  // 19-comparator median-of-9 selection network (Paeth, Graphics Gems;
  // exhaustively checked on all 0/1 inputs by the test suite's CPU twin)
#define CS(i, j) { int lo = min(v[i], v[j]); int hi = max(v[i], v[j]); v[i] = lo; v[j] = hi; }
  CS(1, 2) CS(4, 5) CS(7, 8) CS(0, 1) CS(3, 4) CS(6, 7) CS(1, 2) CS(4, 5) CS(7, 8)
  CS(0, 3) CS(5, 8) CS(4, 7) CS(3, 6) CS(1, 4) CS(2, 5) CS(4, 7) CS(4, 2) CS(6, 4)
  CS(4, 2)
#undef CS
  return v[4];
}

constexpr int kRefMaxX = 4096;  // widest half-res (or full-res mode) row

__global__ void __launch_bounds__(256) k_refine(const int16_t* __restrict__ disp, int nk,
                                                const uint16_t* __restrict__ pk, int XP, int pad,
                                                int X, int Y, int T, int fill_mode,
                                                uint8_t* __restrict__ gcp_out,
                                                int16_t* __restrict__ med_out,
                                                int16_t* __restrict__ filled) {
  __shared__ int16_t s_d[4][kRefMaxX];          // D^L rows y-1, y, y+1 (clamped), D^R row y
  __shared__ int16_t s_med[kRefMaxX];
  __shared__ uint8_t s_h[kRefMaxX];             // left gray of row y
  __shared__ uint64_t s_gm[kRefMaxX / 64];      // GCP flag of column x in bit x % 64 of word x / 64
  const int y = blockIdx.x, pair = blockIdx.y, t = threadIdx.x;
  const size_t plane = (size_t)X * Y;
  const int16_t* dl = disp + (size_t)(2 * pair) * nk;
  const int16_t* dr = disp + (size_t)(2 * pair + 1) * nk;
  const uint16_t* pkr = pk + ((size_t)(2 * pair) * Y + y) * XP + pad;
  const size_t rm = (size_t)max(y - 1, 0) * X, r0 = (size_t)y * X, rp = (size_t)min(y + 1, Y - 1) * X;
  // stage the rows: four columns per thread and round, all loads of a round
  // issued before its stores (clamped columns load a valid value, not stored)
  for (int xb = 0; xb < X; xb += 1024) {
    int16_t a[4][4];
    uint32_t hp[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int x = min(xb + t + 256 * i, X - 1);
      a[i][0] = dl[rm + x];
      a[i][1] = dl[r0 + x];
      a[i][2] = dl[rp + x];
      a[i][3] = dr[r0 + x];
      hp[i] = pkr[x];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int x = xb + t + 256 * i;
      if (x < X) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s_d[q][x] = a[i][q];
        s_h[x] = (uint8_t)hp[i];
      }
    }
  }
  __syncthreads();
  // cross-check and median; the GCP flags of 64 consecutive columns are one
  // wave's ballot
  for (int xb = 0; xb < X; xb += 256) {
    const int x = xb + t;
    bool g = false;
    if (x < X) {
      const int xm = max(x - 1, 0), xp = min(x + 1, X - 1);
      int v[9] = {s_d[0][xm], s_d[0][x], s_d[0][xp], s_d[1][xm], s_d[1][x],
                  s_d[1][xp], s_d[2][xm], s_d[2][x], s_d[2][xp]};
      const int k = v[4];
      g = x - k >= 0 && s_d[3][x - k] == k;
      const int m = median9(v);
      s_med[x] = (int16_t)m;
      if (gcp_out) gcp_out[(size_t)pair * plane + r0 + x] = (uint8_t)g;
      if (med_out) med_out[(size_t)pair * plane + r0 + x] = (int16_t)m;
    }
    const uint64_t bal = __ballot(g);
    if ((t & 63) == 0) s_gm[x >> 6] = bal;
  }
  __syncthreads();
  // fill: the nearest GCPs left and right from the bit array
  const int nw = (X + 63) >> 6;
  int16_t* fo = filled + (size_t)pair * plane + r0;
  for (int x = t; x < X; x += 256) {
    const int wx = x >> 6, bx = x & 63;
    int v;
    if ((s_gm[wx] >> bx) & 1ull) {
      v = s_med[x];
    } else {
      int w = wx, xl = -1, xr = X;
      uint64_t mk = s_gm[w] & ((1ull << bx) - 1ull);            // columns < x
      while (mk == 0ull && w > 0) mk = s_gm[--w];
      if (mk) xl = w * 64 + 63 - __builtin_clzll(mk);
      w = wx;
      mk = bx == 63 ? 0ull : s_gm[w] & (~0ull << (bx + 1));     // columns > x
      while (mk == 0ull && w + 1 < nw) mk = s_gm[++w];
      if (mk) xr = w * 64 + __builtin_ctzll(mk);
      if (xl >= 0 && xr < X) {
        const int i = x - xl, j = xr - x, dla = s_med[xl], drb = s_med[xr];
        if (fill_mode == 1) {
          v = i < j ? dla : drb;
        } else if (fill_mode == 2) {
          v = min(dla, drb);
        } else if (iabs(dla - drb) <= T) {
          v = dla + floor_div_pos(2 * i * (drb - dla) + (i + j), 2 * (i + j));
        } else {
          const int ch = s_h[x];
          v = iabs(s_h[xl] - ch) < iabs(s_h[xr] - ch) ? dla : drb;
        }
      } else if (xl >= 0) {
        v = s_med[xl];
      } else if (xr < X) {
        v = s_med[xr];
      } else {
        v = 0;
      }
    }
    fo[x] = (int16_t)v;
  }
}

// ------------------------------------------------------------ k_gray_full
// Full-resolution mode (the method on the original images, Sec. V): the
// "half" image is the gray image itself.  grid: (ceil(W/256), H, 2 npair),
// block 256.
__global__ void __launch_bounds__(256) k_gray_full(PairPtrs pp, int W, int H,
                                                   uint8_t* __restrict__ half) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, img = blockIdx.z;
  if (x >= W) return;
  const uint8_t* rgb = (img & 1) ? pp.right[img >> 1] : pp.left[img >> 1];
  half[(size_t)img * W * H + (size_t)y * W + x] = (uint8_t)gray_of(rgb + ((size_t)y * W + x) * 3);
}

// Full-resolution mode: the filled map is the output (no upscale).
// grid: (ceil(W*H/256), npair), block 256.
__global__ void __launch_bounds__(256) k_copy_out(PairPtrs pp, const int16_t* __restrict__ filled,
                                                  int n) {
  const int i = blockIdx.x * 256 + threadIdx.x, pair = blockIdx.y;
  if (i >= n) return;
  pp.out[pair][i] = filled[(size_t)pair * n + i];
}

// ------------------------------------------------------------- k_upscale
// One thread per 2x2 block of full-res output pixels (Step8).  Along x: even
// columns take 2 D+(x); an odd column between D+(x) and D+(x+1) takes their
// sum (the doubled midpoint) when they differ by at most T, else the doubled
// value of the side whose full-res gray is strictly closer (the right one on
// a tie); a last odd column copies.  Along y: odd rows are the rounded-up
// mean of the two neighbouring upscaled rows; a last odd row copies.
// grid: (ceil(X/64), ceil(Y/4), npair), block (64, 4).
// odd column between upscaled values 2*dlv and 2*drv; g0, g1, g2 are the
// full-res grays left of, at and right of it
__device__ __forceinline__ int up_odd(int dlv, int drv, const uint8_t* rgb_row, int xo, int T) {
  if (iabs(dlv - drv) <= T) return dlv + drv;
  const int g0 = gray_of(rgb_row + (xo - 1) * 3), g1 = gray_of(rgb_row + xo * 3),
            g2 = gray_of(rgb_row + (xo + 1) * 3);
  return iabs(g0 - g1) < iabs(g2 - g1) ? 2 * dlv : 2 * drv;
}

__global__ void __launch_bounds__(256) k_upscale(PairPtrs pp, const int16_t* __restrict__ filled,
                                                 int W, int H, int X, int Y, int T) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int pair = blockIdx.z;
  if (x >= X || y >= Y) return;
  const int16_t* f = filled + (size_t)pair * X * Y;
  const uint8_t* rgb = pp.left[pair];
  int16_t* out = pp.out[pair];
  const int xo = 2 * x, yo = 2 * y;
  const bool hasr = x + 1 < X, hasd = y + 1 < Y;
  const int a = f[(size_t)y * X + x], b = hasr ? f[(size_t)y * X + x + 1] : a;
  // upscaled row y at columns 2x and 2x+1
  const int u0 = 2 * a;
  const int u1 = hasr ? up_odd(a, b, rgb + (size_t)yo * W * 3, xo + 1, T) : 2 * a;
  const bool odd_col = xo + 1 < W;
  out[(size_t)yo * W + xo] = (int16_t)u0;
  if (odd_col) out[(size_t)yo * W + xo + 1] = (int16_t)u1;
  if (yo + 1 < H) {
    int v0 = u0, v1 = u1;
    if (hasd) {
      const int c = f[(size_t)(y + 1) * X + x], e = hasr ? f[(size_t)(y + 1) * X + x + 1] : c;
      const int w0 = 2 * c;
      const int w1 = hasr ? up_odd(c, e, rgb + (size_t)(yo + 2) * W * 3, xo + 1, T) : 2 * c;
      v0 = (u0 + w0 + 1) >> 1;
      v1 = (u1 + w1 + 1) >> 1;
    }
    out[(size_t)(yo + 1) * W + xo] = (int16_t)v0;
    if (odd_col) out[(size_t)(yo + 1) * W + xo + 1] = (int16_t)v1;
  }
}

}  // namespace
}  // namespace stereo_dev
