// Host side of the soft-argmin head: plans, launch sequences and the C
// interface declared in include/stereo.h (stereo_soft_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "context.h"
#include "kernels.hip.h"
#include "soft.hip.h"
#include "stereo.h"

using namespace stereo_dev;

namespace stereo_host {

constexpr int kSoftMaxPairs = 64;
constexpr size_t kSlabBudget = size_t(1) << 30;  // dL/dCA + dL/dCA_x planes of a slab

struct SoftPlan {
  int n = 0, W = 0, H = 0, Dmax = 0, X = 0, Y = 0, D = 0;
  stereo_soft_params p{};
  int ns = 1, kmax = 8, nstrips = 0, nbands = 0, rows = 0;
  int csize = 1, nchunk = 0;   // k_soft_agg d-chunk size and forward chunk count
  int XS = 0, pads = 0, XA = 0;
  int fxk = 18;        // fixed-point bits of the costs
  int nds = 1;         // disparities per backward slab
  int nbands_tr = 0;   // k_soft_tr bands of kSoftBR rows
  size_t lam_count = 0;
  size_t bytes = 0;
  void* block = nullptr;
  float* half_f = nullptr;     // [2n][Y][X]
  uint8_t* half_u8 = nullptr;  // [2n][Y][X]
  uint32_t* arms = nullptr;    // [2n][Y][XA]
  uint2* sp = nullptr;         // [2n][Y][XS] padded {half value, census}
  float* inv_size = nullptr;   // [n][Y][X]
  float2* part = nullptr;      // [n][nchunk][Y][X]
  float4* pc = nullptr;        // [n][Y][X]
  float* gca = nullptr;        // [nds][n][Y][X]
  float* gcax = nullptr;       // [nds][n][Y][X] dL/dCA_x
  float* gr_part = nullptr;    // [n][nstrips][Y][WP] right-gradient partials of a slab
  int WP = 0;                  // 64 + nds - 1 columns per partial row
  float* g_half = nullptr;     // [2n][Y][X]
  float2* lam_part = nullptr;  // [lam_count]
  // images of the last feature pass on this plan (STEREO_SOFT_F_REUSE_FEATURES)
  const float* feat_left = nullptr;
  const float* feat_right = nullptr;
  // inputs of the last forward, when it saved its weights e_d in the gca
  // planes (STEREO_SOFT_F_SAVE_WEIGHTS, all D in one slab); any other
  // forward, and a backward that recomputes the slabs, clears wts_valid
  bool wts_valid = false;
  const float* wts_left = nullptr;
  const float* wts_right = nullptr;
  const float* wts_lam = nullptr;
  uint64_t last_use = 0;
  hipStream_t owner = nullptr; // the stream the plan serves (plans are never shared
                               // between streams, so calls on two streams may overlap)
};

void free_soft_plans(std::vector<SoftPlan*>& plans) {
  for (SoftPlan* pl : plans) {
    if (pl->block) (void)hipFree(pl->block);
    delete pl;
  }
  plans.clear();
}

// Plans are shared by calls whose parameters differ in flags only.
bool same_soft(const stereo_soft_params& a, const stereo_soft_params& b) {
  return a.tau == b.tau && a.color_delta == b.color_delta && a.arm_x == b.arm_x &&
         a.arm_y == b.arm_y && a.slab == b.slab;
}

int soft_checks(stereo_ctx* c, int n, int W, int H, int Dmax, const stereo_soft_params* params,
                stereo_soft_params* p) {
  if (n < 1 || n > kSoftMaxPairs) return fail(c, STEREO_EINVAL, "n %d outside 1..%d", n, kSoftMaxPairs);
  if (W < 2 || H < 2 || W > STEREO_MAX_SIDE || H > STEREO_MAX_SIDE)
    return fail(c, STEREO_EINVAL, "image size %dx%d outside 2..%d", W, H, STEREO_MAX_SIDE);
  if (Dmax < 1 || Dmax > W || Dmax > STEREO_MAX_DMAX)
    return fail(c, STEREO_EINVAL, "Dmax %d outside 1..min(W=%d, %d)", Dmax, W, STEREO_MAX_DMAX);
  if (params) {
    if (params->size != sizeof(stereo_soft_params))
      return fail(c, STEREO_EINVAL, "params.size %u != %zu", params->size, sizeof(stereo_soft_params));
    *p = *params;
  } else {
    stereo_soft_default_params(p);
  }
  // exp2 of -mean / tau (log2 units) stays a normal float down to tau = 0.025
  if (!(p->tau >= 0.025f) || !std::isfinite(p->tau))
    return fail(c, STEREO_EINVAL, "tau must be finite and >= 0.025");
  if (p->color_delta < 0 || p->color_delta > 256)
    return fail(c, STEREO_EINVAL, "color_delta %d outside 0..256", p->color_delta);
  if (p->arm_x < 0 || p->arm_x > 31 || p->arm_y < 0 || p->arm_y > 63)
    return fail(c, STEREO_EINVAL, "soft head arm caps: arm_x in 0..31, arm_y in 0..63");
  if (p->slab < 0) return fail(c, STEREO_EINVAL, "slab must be >= 0");
  if (p->flags & ~(STEREO_SOFT_F_REUSE_FEATURES | STEREO_SOFT_F_SAVE_WEIGHTS))
    return fail(c, STEREO_EINVAL, "unknown flags");
  return 0;
}

int make_soft_plan(stereo_ctx* c, int n, int W, int H, int Dmax, const stereo_soft_params& p,
                   hipStream_t s, SoftPlan** out) {
  SoftPlan* pl = new SoftPlan();
  pl->n = n; pl->W = W; pl->H = H; pl->Dmax = Dmax; pl->p = p;
  pl->X = (W + 1) / 2; pl->Y = (H + 1) / 2; pl->D = (Dmax + 1) / 2;
  const int X = pl->X, Y = pl->Y, D = pl->D;
  // fixed point: (2 arm_x + 1)(2 arm_y + 1) costs of at most 2 stay below 2^31
  const double cells = (2.0 * p.arm_x + 1) * (2.0 * p.arm_y + 1);
  pl->fxk = (int)std::floor(std::log2(2147483648.0 / (2.0 * cells + 1.0)));
  pl->fxk = std::min(pl->fxk, 22);
  // k_soft_agg: one row-buffer pass (arm_x <= 31), bands whose output rows
  // fit 16 per thread and whose rows fit the plane
  pl->ns = 1;
  const int pr = plane_rows(1);
  int nb = 1, km = 8;
  for (;; ++nb) {
    const int ob = (Y + nb - 1) / nb;
    const int per = (ob + kWaves - 1) / kWaves;
    if (per > 16) continue;
    km = per <= 8 ? 8 : 16;
    const int rows = nb == 1 ? Y : ob + 2 * p.arm_y;
    const int o0max = nb == 1 ? 0 : p.arm_y;
    if (rows <= pr && o0max + kWaves * km <= pr) break;
  }
  pl->nbands = nb;
  pl->kmax = km;
  pl->rows = nb == 1 ? Y : std::min(Y, (Y + nb - 1) / nb + 2 * p.arm_y);
  pl->nstrips = (X + kTX - 1) / kTX;
  pl->XA = pl->nstrips * kTX;
  // row loads reach x0 - hx - d .. x0 - hx + 127 for every strip x0
  pl->pads = ((128 * pl->ns + D + 2) + 1) & ~1;
  pl->XS = pl->pads + pl->XA + 128 * pl->ns + 2;
  pl->XS = (pl->XS + 1) & ~1;
  const int groups = pl->nstrips * pl->nbands * n;
  pl->csize = best_chunk_size(groups, D, pl->rows, c->num_cu);
  pl->nchunk = (D + pl->csize - 1) / pl->csize;
  const size_t npix = (size_t)X * Y;
  // at most 128 disparities per slab (k_soft_tr's LDS rows of right gradients)
  pl->nds = p.slab > 0 ? std::min(p.slab, D)
                       : (int)std::max<size_t>(1, std::min<size_t>(D, kSlabBudget / (2 * n * npix * 4)));
  pl->nds = std::min(pl->nds, kTrMaxWP - 63);
  pl->WP = 64 + pl->nds - 1;
  pl->nbands_tr = (Y + kSoftBR - 1) / kSoftBR;
  const int nslab = (D + pl->nds - 1) / pl->nds;
  pl->lam_count = (size_t)nslab * n * pl->nstrips * pl->nbands_tr;

  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t nimg = 2 * (size_t)n;
  // k_soft_agg addresses the pixel and arm planes through 32-bit buffer
  // offsets
  if (nimg * Y * pl->XS * 8 >= (size_t(1) << 32) || nimg * Y * pl->XA * 4 >= (size_t(1) << 32)) {
    delete pl;
    return fail(c, STEREO_EINVAL, "%d pairs of %dx%d exceed the 4 GiB pixel or arm planes of the "
                "soft head; pass fewer pairs per call", n, W, H);
  }
  size_t bytes = al(nimg * npix * 4) + al(nimg * npix) +
                 al(nimg * Y * pl->XA * 4) + al(nimg * Y * pl->XS * 8) + al(n * npix * 4) +
                 al((size_t)n * pl->nchunk * npix * 8) + al(n * npix * 16) +
                 2 * al((size_t)pl->nds * n * npix * 4) + al(nimg * npix * 4) +
                 al(pl->lam_count * 8) + al((size_t)n * pl->nstrips * Y * pl->WP * 4);
  if (c->mem_cap && c->used + bytes > c->mem_cap) {
    delete pl;
    return fail(c, STEREO_ENOMEM, "soft plan needs %zu bytes, cap %zu, in use %zu", bytes,
                c->mem_cap, c->used);
  }
  hipError_t e = hipMalloc(&pl->block, bytes);
  if (e != hipSuccess) {
    delete pl;
    (void)hipGetLastError();
    return fail(c, STEREO_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  pl->bytes = bytes;
  char* cur = static_cast<char*>(pl->block);
  pl->half_f = carve<float>(cur, nimg * npix);
  pl->half_u8 = carve<uint8_t>(cur, nimg * npix);
  pl->arms = carve<uint32_t>(cur, nimg * Y * pl->XA);
  pl->sp = carve<uint2>(cur, nimg * Y * pl->XS);
  pl->inv_size = carve<float>(cur, n * npix);
  pl->part = carve<float2>(cur, (size_t)n * pl->nchunk * npix);
  pl->pc = carve<float4>(cur, n * npix);
  pl->gca = carve<float>(cur, (size_t)pl->nds * n * npix);
  pl->gcax = carve<float>(cur, (size_t)pl->nds * n * npix);
  pl->g_half = carve<float>(cur, nimg * npix);
  pl->lam_part = carve<float2>(cur, pl->lam_count);
  pl->gr_part = carve<float>(cur, (size_t)n * pl->nstrips * Y * pl->WP);
  // zero padding of the arm and pixel planes (kernels write the image part),
  // ordered on the plan's stream: no other stream is stalled
  hipLaunchKernelGGL(k_fill_f32, dim3(1024), dim3(256), 0, s, reinterpret_cast<float*>(pl->arms),
                     nimg * Y * pl->XA, 0.f);
  hipLaunchKernelGGL(k_fill_f32, dim3(1024), dim3(256), 0, s, reinterpret_cast<float*>(pl->sp),
                     nimg * Y * pl->XS * 2, 0.f);
  e = hipGetLastError();
  if (e != hipSuccess) {
    (void)hipFree(pl->block);
    delete pl;
    return fail(c, STEREO_EHIP, "soft plan initialisation: %s", hipGetErrorString(e));
  }
  c->used += bytes;
  *out = pl;
  return 0;
}

int get_soft_plan(stereo_ctx* c, int n, int W, int H, int Dmax, const stereo_soft_params& p,
                  hipStream_t s, SoftPlan** out) {
  for (SoftPlan* pl : c->soft_plans)
    if (pl->n == n && pl->W == W && pl->H == H && pl->Dmax == Dmax && pl->owner == s &&
        same_soft(pl->p, p)) {
      pl->last_use = ++c->tick;
      *out = pl;
      return 0;
    }
  SoftPlan* pl = nullptr;
  int rc = make_soft_plan(c, n, W, H, Dmax, p, s, &pl);
  if (rc == STEREO_ENOMEM && !c->soft_plans.empty()) {
    (void)hipDeviceSynchronize();
    for (SoftPlan* q : c->soft_plans) c->used -= q->bytes;
    free_soft_plans(c->soft_plans);
    rc = make_soft_plan(c, n, W, H, Dmax, p, s, &pl);
  }
  if (rc) return rc;
  pl->last_use = ++c->tick;
  pl->owner = s;
  c->soft_plans.push_back(pl);
  *out = pl;
  return 0;
}

// Features shared by forward and backward: float and uint8 half images,
// census and arms (k_feat of the integer path, which also writes the padded
// pixel planes), 1/|S|.
void soft_features(SoftPlan& pl, const float* left, const float* right, hipStream_t s) {
  pl.feat_left = left;
  pl.feat_right = right;
  const int X = pl.X, Y = pl.Y, n2 = 2 * pl.n;
  hipLaunchKernelGGL(k_soft_prep, dim3((X + 63) / 64, (Y + 3) / 4, n2), dim3(64, 4), 0, s, left,
                     right, pl.W, pl.H, X, Y, pl.half_f, pl.half_u8);
  hipLaunchKernelGGL(k_feat, dim3((X + 63) / 64, (Y + kFeatRows - 1) / kFeatRows, n2),
                     dim3(64, kFeatRows), 0, s, pl.half_u8, X, Y, pl.p.color_delta, pl.p.arm_x,
                     pl.p.arm_x, pl.p.arm_y, pl.XS, pl.pads, pl.XA, pl.half_f, pl.sp, pl.arms,
                     nullptr, nullptr, 0);
  hipLaunchKernelGGL(k_soft_size, dim3((X + 63) / 64, (Y + kSizeRows - 1) / kSizeRows, pl.n),
                     dim3(64, kSizeRows), 0, s, pl.arms, X, Y, pl.XA, pl.p.arm_y, pl.inv_size);
}

SoftArgs soft_args(const SoftPlan& pl, const float* lambdas, int dlo, int dhi, int csize) {
  SoftArgs a{};
  a.sp = pl.sp; a.arms = pl.arms; a.lam = lambdas; a.inv_size = pl.inv_size;
  a.part = pl.part; a.pc = pl.pc; a.gca = pl.gca;
  a.X = pl.X; a.Y = pl.Y; a.XS = pl.XS; a.pads = pl.pads; a.XA = pl.XA;
  a.arm_x = pl.p.arm_x; a.arm_y = pl.p.arm_y;
  a.nbands = pl.nbands; a.dlo = dlo; a.dhi = dhi;
  a.csize = std::max(1, std::min(csize, dhi - dlo));
  a.nchunk = (dhi - dlo + a.csize - 1) / a.csize;
  a.nstrips = pl.nstrips; a.ngroups = pl.nstrips * pl.nbands * pl.n; a.npair = pl.n;
  a.fx = std::ldexp(1.0f, pl.fxk);
  a.zc = (float)(std::ldexp(1.0, -pl.fxk) * 1.4426950408889634 / pl.p.tau);
  a.sp_bytes = (uint32_t)((size_t)2 * pl.n * pl.Y * pl.XS * 8);
  a.arms_bytes = (uint32_t)((size_t)2 * pl.n * pl.Y * pl.XA * 4);
  return a;
}

template <bool GCA>
void launch_soft_agg(const SoftPlan& pl, const SoftArgs& a, hipStream_t s) {
  dim3 grid((unsigned)(((a.ngroups + kXcds - 1) / kXcds) * kXcds * a.nchunk));
  if (pl.kmax == 8) hipLaunchKernelGGL((k_soft_agg<1, 8, GCA>), grid, dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL((k_soft_agg<1, 16, GCA>), grid, dim3(kThreads), 0, s, a);
}

int soft_prologue(stereo_ctx* c, int n, int W, int H, int Dmax, const stereo_soft_params* params,
                  hipStream_t s, SoftPlan** pl, uint32_t* flags = nullptr) {
  stereo_soft_params p;
  int rc = soft_checks(c, n, W, H, Dmax, params, &p);
  if (rc) return rc;
  if (flags) *flags = p.flags;
  HIP_TRY(c, hipSetDevice(c->device));
  return get_soft_plan(c, n, W, H, Dmax, p, s, pl);
}

int launch_status(stereo_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, STEREO_EHIP, "kernel launch: %s", hipGetErrorString(e));
  return 0;
}

constexpr int kL1Blocks = 256;  // partial-sum blocks per pair

// L1 scratch of the context for the stream s: partials [kSoftMaxPairs][kL1Blocks],
// counts [kSoftMaxPairs], loss [1]; one block per stream (made on first use),
// so losses on two streams never share partial sums.
int l1_scratch(stereo_ctx* c, hipStream_t s, float2** part, float** counts, float** loss) {
  void* block = nullptr;
  for (const auto& b : c->l1_blocks)
    if (b.first == s) block = b.second;
  if (!block) {
    const size_t bytes = (size_t)kSoftMaxPairs * (kL1Blocks * 8 + 4) + 1024;
    hipError_t e = hipMalloc(&block, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, STEREO_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    c->l1_blocks.emplace_back(s, block);
  }
  char* cur = static_cast<char*>(block);
  *part = carve<float2>(cur, (size_t)kSoftMaxPairs * kL1Blocks);
  *counts = carve<float>(cur, kSoftMaxPairs);
  *loss = carve<float>(cur, 1);
  return 0;
}

int l1_checks(stereo_ctx* c, int n, int W, int H) {
  if (n < 1 || n > kSoftMaxPairs) return fail(c, STEREO_EINVAL, "n %d outside 1..%d", n, kSoftMaxPairs);
  if (W < 2 || H < 2 || W > STEREO_MAX_SIDE || H > STEREO_MAX_SIDE)
    return fail(c, STEREO_EINVAL, "image size %dx%d outside 2..%d", W, H, STEREO_MAX_SIDE);
  HIP_TRY(c, hipSetDevice(c->device));
  return 0;
}

void l1_reduce(int n, int W, int H, const float* d_hat, const int16_t* gt, const uint8_t* nonocc,
               float2* part, float* counts, float* loss, hipStream_t s) {
  const int X = (W + 1) / 2, Y = (H + 1) / 2;
  hipLaunchKernelGGL(k_l1_partial, dim3(kL1Blocks, n), dim3(256), 0, s, d_hat, gt, nonocc, W, H,
                     X, Y, part);
  hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(256), 0, s, part, kL1Blocks, n, loss, counts);
}

}  // namespace stereo_host

using namespace stereo_host;

extern "C" {

void stereo_soft_default_params(stereo_soft_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->size = sizeof(stereo_soft_params);
  p->tau = 0.1f;
  p->color_delta = 13;
  p->arm_x = 21;
  p->arm_y = 31;
  p->slab = 0;
  p->flags = 0;
}

int stereo_soft_forward(stereo_ctx* c, const float* left, const float* right, int n, int W, int H,
                        int Dmax, const float* lambdas, const stereo_soft_params* params,
                        float* d_hat, float* lse2, hipStream_t stream) {
  if (!c) return STEREO_EINVAL;
  c->err.clear();
  if (!left || !right || !lambdas || !d_hat || !lse2) return fail(c, STEREO_EINVAL, "null pointer");
  SoftPlan* pl = nullptr;
  uint32_t flags = 0;
  int rc = soft_prologue(c, n, W, H, Dmax, params, stream, &pl, &flags);
  if (rc) return rc;
  soft_features(*pl, left, right, stream);
  SoftArgs a = soft_args(*pl, lambdas, 0, pl->D, pl->csize);
  // the weights of all D fit the gca planes only when one slab covers D;
  // k_soft_tcolw addresses them through 32-bit buffer offsets
  const size_t wts_bytes = (size_t)pl->D * pl->n * pl->X * pl->Y * 4;
  pl->wts_valid = (flags & STEREO_SOFT_F_SAVE_WEIGHTS) && pl->nds >= pl->D &&
                  wts_bytes < (size_t(1) << 32);
  if (pl->wts_valid) {
    a.wts = pl->gca;
    pl->wts_left = left;
    pl->wts_right = right;
    pl->wts_lam = lambdas;
  }
  launch_soft_agg<false>(*pl, a, stream);
  const int npix = pl->X * pl->Y;
  hipLaunchKernelGGL(k_soft_merge, dim3((npix + 255) / 256, pl->n), dim3(256), 0, stream, pl->part,
                     pl->nchunk, npix, d_hat, lse2);
  return launch_status(c);
}

int stereo_soft_backward(stereo_ctx* c, const float* left, const float* right, int n, int W,
                         int H, int Dmax, const float* lambdas, const stereo_soft_params* params,
                         const float* d_hat, const float* lse2, const float* g_dhat,
                         float* g_left, float* g_right, float* g_lambdas, hipStream_t stream) {
  if (!c) return STEREO_EINVAL;
  c->err.clear();
  if (!left || !right || !lambdas || !d_hat || !lse2 || !g_dhat || !g_left || !g_right ||
      !g_lambdas)
    return fail(c, STEREO_EINVAL, "null pointer");
  SoftPlan* pl = nullptr;
  uint32_t flags = 0;
  int rc = soft_prologue(c, n, W, H, Dmax, params, stream, &pl, &flags);
  if (rc) return rc;
  const int X = pl->X, Y = pl->Y, npix = X * Y;
  const bool reuse = (flags & STEREO_SOFT_F_REUSE_FEATURES) != 0;
  if (!reuse || pl->feat_left != left || pl->feat_right != right)
    soft_features(*pl, left, right, stream);
  // the forward's weights of these inputs are on the plan: dL/dCA comes from
  // them (k_soft_tcolw) instead of a recomputation of the aggregate
  const bool saved = reuse && pl->wts_valid && pl->wts_left == left && pl->wts_right == right &&
                     pl->wts_lam == lambdas;
  const float zc = (float)(std::ldexp(1.0, -pl->fxk) * 1.4426950408889634 / pl->p.tau);
  hipLaunchKernelGGL(k_soft_bprep, dim3((npix + 255) / 256, pl->n), dim3(256), 0, stream,
                     pl->inv_size, lse2, d_hat, g_dhat, npix, zc, 1.f / pl->p.tau, pl->pc);
  const int groups = pl->nstrips * pl->nbands * pl->n;
  const int tb = tcol_band(pl->p.arm_y);
  if (!saved) pl->wts_valid = false;  // the slabs below overwrite the weight planes
  size_t lam_off = 0;
  for (int dlo = 0; dlo < pl->D; dlo += pl->nds) {
    const int dhi = std::min(pl->D, dlo + pl->nds), nds = dhi - dlo;
    if (saved) {
      // one slab holds all D; disparity groups so that the grid fills the
      // CUs about three blocks deep (each group reloads the per-pixel
      // constants: at 4 x 718x496, 4 groups ran faster than 3 or 6)
      const int base = ((X + 63) / 64) * ((Y + tb - 1) / tb) * pl->n;
      const int ndg = std::max(1, std::min(pl->D, (3 * c->num_cu + base - 1) / base));
      hipLaunchKernelGGL(k_soft_tcolw, dim3((X + 63) / 64, (Y + tb - 1) / tb, pl->n * ndg),
                         dim3(64 * kTcwWaves), 0, stream, pl->gca,
                         (uint32_t)((size_t)pl->D * pl->n * npix * 4), pl->pc, pl->arms, X, Y,
                         pl->XA, pl->p.arm_y, pl->n, pl->D, ndg, pl->gcax);
    } else {
      const int cs = best_chunk_size(groups, nds, pl->rows, c->num_cu);
      launch_soft_agg<true>(*pl, soft_args(*pl, lambdas, dlo, dhi, cs), stream);
      hipLaunchKernelGGL(k_soft_tcol, dim3((X + 63) / 64, (Y + tb - 1) / tb, nds * pl->n),
                         dim3(256), 0, stream, pl->gca, pl->arms, X, Y, pl->XA, pl->p.arm_y,
                         pl->n, pl->gcax);
    }
    TrArgs ta{};
    ta.gcax = pl->gcax; ta.arms = pl->arms; ta.sp = pl->sp; ta.lam = lambdas;
    ta.g_half = pl->g_half; ta.gr_part = pl->gr_part;
    ta.lam_part = pl->lam_part + lam_off;
    ta.X = X; ta.Y = Y; ta.XS = pl->XS; ta.pads = pl->pads; ta.XA = pl->XA;
    ta.npair = pl->n; ta.dlo = dlo; ta.dhi = dhi; ta.WP = pl->WP;
    ta.nstrips = pl->nstrips; ta.nbands = pl->nbands_tr;
    ta.first = dlo == 0;  // the first slab writes every half-image gradient
    dim3 tg((unsigned)(pl->nstrips * pl->nbands_tr), (unsigned)pl->n);
    hipLaunchKernelGGL(k_soft_tr, tg, dim3(256), 0, stream, ta);
    lam_off += (size_t)tg.x * tg.y;
    hipLaunchKernelGGL(k_soft_gright, dim3((X + 255) / 256, Y, pl->n), dim3(256), 0, stream,
                       pl->gr_part, pl->nstrips, pl->WP, dlo, dhi, X, Y, (int)(dlo == 0),
                       pl->g_half);
  }
  hipLaunchKernelGGL(k_soft_gfull, dim3((W + 255) / 256, H, 2 * pl->n), dim3(256), 0, stream,
                     pl->g_half, W, H, X, Y, g_left, g_right);
  hipLaunchKernelGGL(k_soft_lam, dim3(1), dim3(1024), 0, stream, pl->lam_part, (int)lam_off,
                     g_lambdas);
  return launch_status(c);
}

int stereo_soft_l1_loss(stereo_ctx* c, const float* d_hat, const int16_t* gt,
                        const uint8_t* nonocc, int n, int W, int H, float* loss,
                        hipStream_t stream) {
  if (!c) return STEREO_EINVAL;
  c->err.clear();
  if (!d_hat || !gt || !nonocc || !loss) return fail(c, STEREO_EINVAL, "null pointer");
  int rc = l1_checks(c, n, W, H);
  if (rc) return rc;
  float2* part;
  float *counts, *scratch_loss;
  rc = l1_scratch(c, stream, &part, &counts, &scratch_loss);
  if (rc) return rc;
  l1_reduce(n, W, H, d_hat, gt, nonocc, part, counts, loss, stream);
  return launch_status(c);
}

int stereo_soft_l1_grad(stereo_ctx* c, const float* d_hat, const int16_t* gt,
                        const uint8_t* nonocc, int n, int W, int H, const float* gscale,
                        float* g_dhat, hipStream_t stream) {
  if (!c) return STEREO_EINVAL;
  c->err.clear();
  if (!d_hat || !gt || !nonocc || !g_dhat) return fail(c, STEREO_EINVAL, "null pointer");
  int rc = l1_checks(c, n, W, H);
  if (rc) return rc;
  float2* part;
  float *counts, *scratch_loss;
  rc = l1_scratch(c, stream, &part, &counts, &scratch_loss);
  if (rc) return rc;
  l1_reduce(n, W, H, d_hat, gt, nonocc, part, counts, scratch_loss, stream);
  const int X = (W + 1) / 2, Y = (H + 1) / 2, npix = X * Y;
  hipLaunchKernelGGL(k_l1_grad, dim3((npix + 255) / 256, n), dim3(256), 0, stream, d_hat, gt,
                     nonocc, counts, gscale, W, H, X, Y, n, g_dhat);
  return launch_status(c);
}

}  // extern "C"
