// Host side of the stereo library: context, per-shape plans, launches and
// the C interface declared in include/stereo.h.
#include "stereo.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "context.h"
#include "kernels.hip.h"
#include "pipeline.h"

using namespace stereo_dev;

// Fixed scratch of stereo_disparity_noalloc: one array per device, allocated
// when the code object is loaded on that device and held until the process
// ends.  Host code never uses its name as an address: the device address of
// each device's copy comes from hipGetSymbolAddress (noalloc_scratch_of).
constexpr size_t kNoallocBytes = size_t(STEREO_NOALLOC_MAX_BYTES);
static __device__ __align__(256) uint8_t scratch[kNoallocBytes];

namespace stereo_host {

// Device address of `scratch` on `device` (the current device), looked up
// once per device; null with *err set when the lookup failed.
void* noalloc_scratch_of(int device, std::string* err) {
  static std::mutex mu;
  static std::vector<void*> addr;
  static std::vector<std::string> why;
  std::lock_guard<std::mutex> lock(mu);
  if ((size_t)device >= addr.size()) {
    addr.resize(device + 1, nullptr);
    why.resize(device + 1);
  }
  if (!addr[device] && why[device].empty()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess && ptr) {
      addr[device] = ptr;
    } else {
      (void)hipGetLastError();
      why[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    }
  }
  *err = why[device];
  return addr[device];
}

// Cost tables of Eq. 4 and Eq. 5 in fixed point: S(1 - exp(-t)) rounded half
// up, with t = (a / 255) / lambda_AD for brightness difference a and
// t = h / lambda_MC for census Hamming distance h.
void build_tables(const stereo_params& p, uint16_t ad[256], uint16_t mc[7]) {
  const double S = p.cost_scale, lad = p.lambda_ad, lmc = p.lambda_mc;
  for (int a = 0; a < 256; ++a) ad[a] = (uint16_t)std::floor(S * (1.0 - std::exp(-(a / 255.0) / lad)) + 0.5);
  for (int h = 0; h < 7; ++h) mc[h] = (uint16_t)std::floor(S * (1.0 - std::exp(-h / lmc)) + 0.5);
}


bool same_params(const stereo_params& a, const stereo_params& b) {
  return a.lambda_ad == b.lambda_ad && a.lambda_mc == b.lambda_mc && a.cost_scale == b.cost_scale &&
         a.color_delta == b.color_delta && a.arm_x == b.arm_x && a.arm_y == b.arm_y &&
         a.fill_T == b.fill_T && a.arm_x_r == b.arm_x_r && a.fill_mode == b.fill_mode &&
         (a.flags & STEREO_F_FULL_RES) == (b.flags & STEREO_F_FULL_RES);
}

bool full_res(const stereo_params& p) { return (p.flags & STEREO_F_FULL_RES) != 0; }

// Bits of the disparity field of the winner-take-all keys: enough for D - 1.
int key_dbits(int D) {
  int b = 1;
  while ((1 << b) < D) ++b;
  return b;
}

}  // namespace stereo_host

namespace stereo_host {

// Checks p for a search range of D disparities (D >= 1); resolves arm_x_r.
int check_params(stereo_ctx* c, stereo_params& p, int D) {
  if (p.size != sizeof(stereo_params))
    return fail(c, STEREO_EINVAL, "params.size %u != %zu", p.size, sizeof(stereo_params));
  if (!(p.lambda_ad > 0.f) || !std::isfinite(p.lambda_ad) || !(p.lambda_mc > 0.f) ||
      !std::isfinite(p.lambda_mc))
    return fail(c, STEREO_EINVAL, "lambda_ad and lambda_mc must be finite and > 0");
  if (p.cost_scale < 1 || p.cost_scale > 1024)
    return fail(c, STEREO_EINVAL, "cost_scale %d outside 1..1024", p.cost_scale);
  if (p.color_delta < 0 || p.color_delta > 256)
    return fail(c, STEREO_EINVAL, "color_delta %d outside 0..256", p.color_delta);
  if (p.arm_x_r == -1) p.arm_x_r = p.arm_x;
  if (p.arm_x < 0 || p.arm_x > 127 || p.arm_y < 0 || p.arm_y > 127 || p.arm_x_r < 0 ||
      p.arm_x_r > 127)
    return fail(c, STEREO_EINVAL, "arm caps must be in 0..127 (arm_x_r: -1 or 0..127)");
  if (p.fill_mode < 0 || p.fill_mode > 2) return fail(c, STEREO_EINVAL, "fill_mode %d outside 0..2", p.fill_mode);
  if (p.fill_T < 0 || p.fill_T > 1023) return fail(c, STEREO_EINVAL, "fill_T outside 0..1023");
  uint16_t ad[256], mc[7];
  build_tables(p, ad, mc);
  const double cmax = (double)ad[255] + mc[6];
  const int ax = std::max(p.arm_x, p.arm_x_r), dbits = key_dbits(D);
  const double bound = (2.0 * ax + 1) * (2.0 * p.arm_y + 1) * cmax;
  if (bound >= std::ldexp(1.0, 32 - dbits))
    return fail(c, STEREO_EINVAL,
                "(2 arm_x + 1)(2 arm_y + 1) C_max = %.0f must be < 2^%d for D = %d "
                "(lower cost_scale or the arm caps)", bound, 32 - dbits, D);
  return 0;
}

void free_plan(Plan* pl) {
  if (!pl) return;
  if (pl->block) (void)hipFree(pl->block);
  if (pl->dbg_block) (void)hipFree(pl->dbg_block);
  delete pl;
}


// Modelled k_match time, in units of one disparity of one workgroup, for
// d-chunks of cs disparities: each XCD's workgroups, in k_match's order of
// positions, go to dispatch queue (position % kXcdQueues), where each takes
// the CU of that queue that frees first; a workgroup costs its disparities
// plus ovh units of set-up and drain (cost table, arms, key stores).
// Remainder chunks are placed as k_match places them.  The queue structure
// (4 queues of 8 CUs per XCD, filled in turn) is what measurement of these
// placements shows: a workgroup past the first round waits for a CU of its
// own queue, not for the first CU to free.
double match_makespan(int groups, int D, int cs, int cus_per_xcd, double ovh) {
  const int nfull = D / cs, rem = D - nfull * cs, nchunk = nfull + (rem > 0);
  const int nloc = (groups + kXcds - 1) / kXcds, T = nloc * nchunk;
  const int per_q = std::max(1, cus_per_xcd / kXcdQueues);
  const bool stacked = nchunk != nfull && kXcdQueues * (nloc - 1) <= T - 1;
  double worst = 0.0;
  std::vector<double> cu((size_t)kXcdQueues * per_q);
  for (int x = 0; x < kXcds && x < groups; ++x) {
    std::fill(cu.begin(), cu.end(), 0.0);
    for (int j = 0; j < T; ++j) {
      int local, chunk;
      const int q = T - 1 - j;
      if (stacked && q % kXcdQueues == 0 && q / kXcdQueues < nloc) {
        local = nloc - 1 - q / kXcdQueues;
        chunk = nfull;
      } else if (stacked) {
        const int i = j - std::max(0, nloc - (q / kXcdQueues + 1));
        local = i / nfull;
        chunk = i - local * nfull;
      } else {
        local = j < nloc * nfull ? j / nfull : j - nloc * nfull;
        chunk = j < nloc * nfull ? j - local * nfull : nfull;
      }
      if (local * kXcds + x >= groups) continue;  // padding workgroup
      double* qb = cu.data() + (size_t)(j % kXcdQueues) * per_q;
      *std::min_element(qb, qb + per_q) += ovh + (chunk < nfull ? cs : rem);
    }
    worst = std::max(worst, *std::max_element(cu.begin(), cu.end()));
  }
  return worst;
}

// Chunk size with the shortest modelled time among ceil(D / n), n = 1..64,
// at most 16 workgroups per CU.  A workgroup's fixed cost (set-up, drain and
// the first disparity's cold reads) is taken as one disparity over
// kSetupRows band rows: fitted to timings of all chunk sizes at 640x480,
// 1436x992, 1920x1080 (1 and 8 pairs) and 2872x1984, where this value picks
// the fastest size or one within 6% of it.
constexpr double kSetupRows = 300.0;

int best_chunk_size(int groups, int D, int rows, int num_cu) {
  const int cus = std::max(1, num_cu / kXcds);
  const double ovh = kSetupRows / std::max(1, rows);
  int best = D;
  double best_t = 1e300;
  for (int n = 1; n <= std::min(D, 64); ++n) {
    const int cs = (D + n - 1) / n;
    if ((long)groups * ((D + cs - 1) / cs) > 16L * num_cu) break;
    const double t = match_makespan(groups, D, cs, cus, ovh);
    if (t < best_t - 1e-9) {  // ties keep the larger chunks (fewer workgroups)
      best_t = t;
      best = cs;
    }
  }
  return best;
}

// Launch geometry: bands keep the k_match LDS plane and the per-thread key
// registers within bounds; d-chunks raise the workgroup count to fill the CUs.
void plan_geometry(Plan& pl, int num_cu, int forced_csize) {
  // the row buffer spans x0 - hx .. x0 + 63 + arm_x, hx = arm_x + 1 rounded up to even
  pl.ns = (66 + 2 * std::max(pl.p.arm_x, pl.p.arm_x_r) + 127) / 128;
  const int pr = plane_rows(pl.ns);
  // Output rows of a band are spread over the 16 waves, KMAX per thread
  // (template steps 8..36).  The finalize of a band reads plane rows up to
  // o0 + 16 KMAX (padding rows included, o0 <= arm_y is the top halo), and
  // the band itself must fit the plane.
  auto kstep = [](int rows_per_thread) {
    for (int s : {8, 16, 24, 32, kKMax})  // kKMax = 34
      if (rows_per_thread <= s) return s;
    return -1;
  };
  int nb = 1, km = 8;
  for (;; ++nb) {
    const int ob = (pl.Y + nb - 1) / nb;
    km = kstep((ob + kWaves - 1) / kWaves);
    if (km < 0) continue;
    const int rows = nb == 1 ? pl.Y : ob + 2 * pl.p.arm_y;
    const int o0max = nb == 1 ? 0 : pl.p.arm_y;
    if (rows <= pr && o0max + kWaves * km <= pr) break;
  }
  pl.kmax = km;
  pl.nbands = nb;
  pl.nstrips = (pl.X + kTX - 1) / kTX;
  // pk padding covers every column a k_match lane loads: x0 - hx - D at the
  // left, x0 - hx + 128 NS - 1 + D < X + 128 NS + D at the right (one more in
  // the shifted copy); pad and the pitch are even, so the pair of columns
  // from an even column is an aligned 32-bit word
  pl.pad = ((128 * pl.ns + pl.D + 2) + 3) & ~3;
  pl.XP = (pl.X + 2 * pl.pad + 63) & ~63;
  pl.XA = pl.nstrips * kTX;
  const int groups = pl.nstrips * pl.nbands * 2 * pl.npair;
  // d-chunks of csize disparities (the last one the remainder): the size
  // with the shortest modelled k_match time, or the one stereo_autotune chose
  const int rows = pl.nbands == 1 ? pl.Y : std::min(pl.Y, (pl.Y + pl.nbands - 1) / pl.nbands + 2 * pl.p.arm_y);
  pl.csize = forced_csize > 0 ? std::min(forced_csize, pl.D) : best_chunk_size(groups, pl.D, rows, num_cu);
  pl.nchunk = (pl.D + pl.csize - 1) / pl.csize;
}

// The d-chunk size stereo_autotune chose for this shape and parameters, or 0.
int tuned_csize(const stereo_ctx* c, int W, int H, int Dmax, int npair, const stereo_params& p) {
  for (const Tuned& t : c->tuned)
    if (t.W == W && t.H == H && t.Dmax == Dmax && t.npair == npair && same_params(t.p, p))
      return t.csize;
  return 0;
}

// Device bytes of a plan's block and of its pixel (pk, both copies) and arm
// planes, for the geometry already in pl.
struct PlanBytes {
  size_t total, pk, arms;  // arms: each of the arms and xoff planes
};

PlanBytes plan_bytes(const Plan& pl) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t n = (size_t)pl.X * pl.Y, npair = pl.npair;
  const size_t npk = (size_t)2 * npair * pl.Y * pl.XP, nar = (size_t)2 * npair * pl.Y * pl.XA;
  const size_t nk = pl.nk;
  PlanBytes b;
  b.pk = 2 * npk * 2;
  b.arms = nar * 4;
  b.total = al(2 * npair * n) + al(b.pk) + 2 * al(b.arms) + al(kTab * 2) +
            al((size_t)npair * pl.nchunk * 2 * nk * 4) + al(2 * npair * nk * 2) +
            al(2 * npair * nk * 4) + al(npair * n) + al(npair * n * 2) + al(npair * n * 2);
  return b;
}

// Shape, tables and launch geometry of a plan (host side only, no device
// memory); rejects shapes whose pixel or arm planes the kernels' 32-bit
// buffer offsets cannot address.
int plan_setup(stereo_ctx* c, Plan& pl, int W, int H, int Dmax, const stereo_params& p,
               int npair, int forced_csize) {
  pl.W = W; pl.H = H; pl.Dmax = Dmax; pl.npair = npair;
  if (full_res(p)) {
    pl.X = W; pl.Y = H; pl.D = Dmax;
  } else {
    pl.X = (W + 1) / 2; pl.Y = (H + 1) / 2; pl.D = (Dmax + 1) / 2;
  }
  pl.dbits = key_dbits(pl.D);
  pl.p = p;
  build_tables(p, pl.lut_ad, pl.lut_mc);
  pl.cmax = pl.lut_ad[255] + pl.lut_mc[6];
  plan_geometry(pl, c->num_cu, forced_csize);
  pl.nk = (int)(((size_t)pl.X * pl.Y + 63) & ~size_t(63));
  const PlanBytes b = plan_bytes(pl);
  if (b.pk >= (size_t(1) << 32) || b.arms >= (size_t(1) << 32))
    return fail(c, STEREO_EINVAL, "%d pairs of %dx%d exceed the 4 GiB pixel or arm planes", npair,
                W, H);
  return 0;
}

// Carves the planes of pl from the device block at base and enqueues their
// set-up on stream s: padding cleared, cost table written (k_plan_init).
void plan_carve_and_init(Plan& pl, void* base, hipStream_t s) {
  const size_t n = (size_t)pl.X * pl.Y, npair = pl.npair, nk = pl.nk;
  const PlanBytes b = plan_bytes(pl);
  char* cur = static_cast<char*>(base);
  pl.half = carve<uint8_t>(cur, 2 * npair * n);
  pl.pk = carve<uint16_t>(cur, b.pk / 2);
  pl.arms = carve<uint32_t>(cur, b.arms / 4);
  pl.xoff = carve<uint32_t>(cur, b.arms / 4);
  pl.tab = carve<uint16_t>(cur, kTab);
  pl.keys = carve<uint32_t>(cur, npair * pl.nchunk * 2 * nk);
  pl.disp = carve<int16_t>(cur, 2 * npair * nk);
  pl.mincost = carve<uint32_t>(cur, 2 * npair * nk);
  pl.gcp = carve<uint8_t>(cur, npair * n);
  pl.med = carve<int16_t>(cur, npair * n);
  pl.filled = carve<int16_t>(cur, npair * n);
  TabArgs t{};
  for (int i = 0; i < 256; ++i) t.ad[i] = pl.lut_ad[i];
  for (int i = 0; i < 7; ++i) t.mc[i] = pl.lut_mc[i];
  t.cmax = (uint16_t)pl.cmax;
  // pk, arms and xoff are adjacent in the block: one cleared range covers them
  const size_t nzero = (size_t)(reinterpret_cast<char*>(pl.xoff) + b.arms -
                                reinterpret_cast<char*>(pl.pk)) / 4;
  const unsigned blocks = (unsigned)std::min<size_t>(2048, (nzero + 1023) / 1024 + 1);
  hipLaunchKernelGGL(k_plan_init, dim3(blocks), dim3(256), 0, s,
                     reinterpret_cast<uint32_t*>(pl.pk), nzero, pl.tab, t);
}

int make_plan(stereo_ctx* c, int W, int H, int Dmax, const stereo_params& p, int npair,
              hipStream_t s, Plan** out) {
  Plan* pl = new Plan();
  int rc = plan_setup(c, *pl, W, H, Dmax, p, npair, tuned_csize(c, W, H, Dmax, npair, p));
  if (rc) {
    delete pl;
    return rc;
  }
  const size_t bytes = plan_bytes(*pl).total;
  if (c->mem_cap && c->used + bytes > c->mem_cap) {
    delete pl;
    return fail(c, STEREO_ENOMEM, "plan needs %zu bytes, cap %zu, in use %zu", bytes, c->mem_cap,
                c->used);
  }
  hipError_t e = hipMalloc(&pl->block, bytes);
  if (e != hipSuccess) {
    delete pl;
    (void)hipGetLastError();
    return fail(c, STEREO_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  pl->bytes = bytes;
  // set-up on the stream the plan serves: later work on that stream follows
  // it, and no other stream or slot is stalled
  plan_carve_and_init(*pl, pl->block, s);
  e = hipGetLastError();
  if (e != hipSuccess) {
    free_plan(pl);
    return fail(c, STEREO_EHIP, "plan initialisation: %s", hipGetErrorString(e));
  }
  c->used += bytes;
  *out = pl;
  return 0;
}

int get_plan(stereo_ctx* c, int W, int H, int Dmax, const stereo_params& p, int npair,
             const void* owner, hipStream_t s, Plan** out) {
  for (Plan* pl : c->plans)
    if (pl->W == W && pl->H == H && pl->Dmax == Dmax && pl->npair >= npair && pl->owner == owner &&
        same_params(pl->p, p)) {
      pl->last_use = ++c->tick;
      *out = pl;
      return 0;
    }
  // a new plan needs an allocation, which a stream under graph capture
  // cannot make
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(c, STEREO_EINVAL,
                "no scratch yet for %dx%d Dmax %d on this stream: make one call outside the "
                "graph capture first (or use stereo_disparity_noalloc)", W, H, Dmax);
  (void)hipGetLastError();
  Plan* pl = nullptr;
  int rc = make_plan(c, W, H, Dmax, p, npair, s, &pl);
  if (rc == STEREO_ENOMEM && !c->plans.empty()) {
    // evict least recently used plans, except the one whose intermediates are
    // kept and those a captured graph still launches into, then retry
    std::sort(c->plans.begin(), c->plans.end(),
              [](Plan* a, Plan* b) { return a->last_use < b->last_use; });
    for (size_t i = 0; i < c->plans.size() && rc == STEREO_ENOMEM;) {
      if (c->plans[i] == c->last || c->plans[i]->pins > 0 || c->plans[i]->captured) {
        ++i;
        continue;
      }
      (void)hipDeviceSynchronize();
      c->used -= c->plans[i]->bytes;
      free_plan(c->plans[i]);
      c->plans.erase(c->plans.begin() + i);
      rc = make_plan(c, W, H, Dmax, p, npair, s, &pl);
    }
  }
  if (rc) return rc;
  pl->last_use = ++c->tick;
  pl->owner = owner;
  c->plans.push_back(pl);
  *out = pl;
  return 0;
}

void drop_plan(stereo_ctx* c, Plan* pl) {
  for (size_t i = 0; i < c->plans.size(); ++i)
    if (c->plans[i] == pl) {
      if (c->last == pl) c->last = nullptr;
      c->used -= pl->bytes;
      free_plan(pl);
      c->plans.erase(c->plans.begin() + i);
      return;
    }
}

// Frees every plan of (W, H, Dmax, p), whatever its owner (after the device
// has finished with them), so that the next call makes it again.
int evict_shape(stereo_ctx* c, int W, int H, int Dmax, const stereo_params& p) {
  for (const Plan* pl : c->plans)
    if (pl->W == W && pl->H == H && pl->Dmax == Dmax && same_params(pl->p, p) &&
        (pl->pins > 0 || pl->captured))
      return fail(c, STEREO_EINVAL, "a captured graph uses the scratch of %dx%d Dmax %d; tune "
                  "before capturing", W, H, Dmax);
  HIP_TRY(c, hipDeviceSynchronize());
  for (size_t i = 0; i < c->plans.size();) {
    Plan* pl = c->plans[i];
    if (pl->W == W && pl->H == H && pl->Dmax == Dmax && same_params(pl->p, p)) {
      if (c->last == pl) c->last = nullptr;
      c->used -= pl->bytes;
      free_plan(pl);
      c->plans.erase(c->plans.begin() + i);
    } else {
      ++i;
    }
  }
  return 0;
}

void set_tuned(stereo_ctx* c, int W, int H, int Dmax, int npair, const stereo_params& p,
               int csize) {
  for (Tuned& t : c->tuned)
    if (t.W == W && t.H == H && t.Dmax == Dmax && t.npair == npair && same_params(t.p, p)) {
      t.csize = csize;
      return;
    }
  c->tuned.push_back(Tuned{W, H, Dmax, npair, p, csize});
}

MatchArgs match_args(const Plan& pl, int dlo, int dhi, int csize) {
  MatchArgs a{};
  a.pk = pl.pk; a.arms = pl.arms; a.xoff = pl.xoff; a.tab = pl.tab; a.keys = pl.keys;
  a.X = pl.X; a.Y = pl.Y; a.XP = pl.XP; a.pad = pl.pad; a.XA = pl.XA; a.nk = pl.nk;
  a.arm_x = pl.p.arm_x; a.arm_x_r = pl.p.arm_x_r; a.arm_y = pl.p.arm_y; a.dbits = pl.dbits;
  a.copy_bytes = (uint32_t)((size_t)2 * pl.npair * pl.Y * pl.XP * 2);
  a.pk_bytes = 2 * a.copy_bytes;
  a.arms_bytes = (uint32_t)((size_t)2 * pl.npair * pl.Y * pl.XA * 4);
  a.nbands = pl.nbands; a.dlo = dlo; a.dhi = dhi;
  a.csize = std::max(1, std::min(csize, dhi - dlo));
  a.nchunk = (dhi - dlo + a.csize - 1) / a.csize;
  return a;
}

// k_match with KMAX = KM: its LDS block holds the plane rows the plan's
// bands write (band rows + 1) or its window step reads (o0 + 16 KMAX + 1),
// whichever is more; the rest of the CU's LDS stays free for other streams.
template <int NS, int KM, bool DBG>
void launch_match_km(const Plan& pl, const MatchArgs& a, dim3 grid, hipStream_t s) {
  const int brows = pl.nbands == 1 ? pl.Y : std::min(pl.Y, (pl.Y + pl.nbands - 1) / pl.nbands + 2 * pl.p.arm_y);
  const int o0max = pl.nbands == 1 ? 0 : pl.p.arm_y;
  const int rows = std::max(brows, o0max + kWaves * KM) + 1;
  // dynamic LDS beyond the default limit needs the attribute (set once per
  // instance); were it refused, the launch below fails and run() reports
  // that launch's error
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&k_match<NS, KM, DBG>),
      hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes - kMatchTabBytes);
  (void)attr;
  hipLaunchKernelGGL((k_match<NS, KM, DBG>), grid, dim3(kThreads),
                     (size_t)match_lds_bytes(NS, rows), s, a);
}

template <int NS, bool DBG>
void launch_match_k(const Plan& pl, const MatchArgs& a, dim3 grid, hipStream_t s) {
  switch (pl.kmax) {
    case 8: launch_match_km<NS, 8, DBG>(pl, a, grid, s); break;
    case 16: launch_match_km<NS, 16, DBG>(pl, a, grid, s); break;
    case 24: launch_match_km<NS, 24, DBG>(pl, a, grid, s); break;
    case 32: launch_match_km<NS, 32, DBG>(pl, a, grid, s); break;
    default: launch_match_km<NS, kKMax, DBG>(pl, a, grid, s); break;
  }
}

void launch_match(const Plan& pl, MatchArgs a, int npair, hipStream_t s) {
  a.nstrips = pl.nstrips;
  a.ngroups = pl.nstrips * pl.nbands * 2 * npair;
  dim3 grid((unsigned)(((a.ngroups + kXcds - 1) / kXcds) * kXcds * a.nchunk));
  const bool dbg = a.dbg_cost != nullptr;
  switch (pl.ns) {
    case 1: dbg ? launch_match_k<1, true>(pl, a, grid, s) : launch_match_k<1, false>(pl, a, grid, s); break;
    case 2: dbg ? launch_match_k<2, true>(pl, a, grid, s) : launch_match_k<2, false>(pl, a, grid, s); break;
    default: dbg ? launch_match_k<3, true>(pl, a, grid, s) : launch_match_k<3, false>(pl, a, grid, s); break;
  }
}

// Events of the next timed call (created on first use, reused after reset).
int timing_events(stereo_ctx* c, hipEvent_t** ev) {
  const size_t per = STEREO_NUM_STAGES + 1, need = (size_t)(c->timed_calls + 1) * per;
  while (c->events.size() < need) {
    hipEvent_t e;
    HIP_TRY(c, hipEventCreate(&e));
    c->events.push_back(e);
  }
  *ev = &c->events[(size_t)c->timed_calls * per];
  return 0;
}

// The whole path for npair pairs already checked against the plan.
int run(stereo_ctx* c, Plan& pl, const PairPtrs& pp, int npair, bool keep, bool timed,
        hipStream_t s) {
  const int X = pl.X, Y = pl.Y;
  hipEvent_t* ev = nullptr;
  if (timed) {
    int rc = timing_events(c, &ev);
    if (rc) return rc;
  }
  auto mark = [&](int i) { if (ev) (void)hipEventRecord(ev[i], s); };
  dim3 b2(64, 4);
  const bool full = full_res(pl.p);
  mark(0);
  if (full)
    hipLaunchKernelGGL(k_gray_full, dim3((X + 255) / 256, Y, 2 * npair), dim3(256), 0, s, pp, X, Y,
                       pl.half);
  else
    hipLaunchKernelGGL(k_prep, dim3((X + 63) / 64, (Y + kPrepRows - 1) / kPrepRows, 2 * npair),
                       b2, 0, s, pp, pl.W, pl.H, X, Y, pl.half);
  mark(1);
  hipLaunchKernelGGL(k_feat, dim3((X + 63) / 64, (Y + kFeatRows - 1) / kFeatRows, 2 * npair),
                     dim3(64, kFeatRows), 0,
                     s, pl.half, X, Y, pl.p.color_delta, pl.p.arm_x, pl.p.arm_x_r, pl.p.arm_y,
                     pl.XP, pl.pad, pl.XA, nullptr, nullptr, pl.arms, pl.xoff, pl.pk,
                     (size_t)2 * npair * Y * pl.XP);
  mark(2);
  launch_match(pl, match_args(pl, 0, pl.D, pl.csize), npair, s);
  mark(3);
  hipLaunchKernelGGL(k_wta, dim3((pl.nk + 1023) / 1024, npair), dim3(256), 0, s, pl.keys,
                     pl.nchunk, pl.nk, pl.dbits, pl.disp, keep ? pl.mincost : nullptr);
  mark(4);
  hipLaunchKernelGGL(k_refine, dim3(Y, npair), dim3(256), 0, s, pl.disp, pl.nk, pl.pk, pl.XP,
                     pl.pad, X, Y, pl.p.fill_T, pl.p.fill_mode, keep ? pl.gcp : nullptr,
                     keep ? pl.med : nullptr, pl.filled);
  mark(5);
  if (full)
    hipLaunchKernelGGL(k_copy_out, dim3((X * Y + 255) / 256, npair), dim3(256), 0, s, pp,
                       pl.filled, X * Y);
  else
    hipLaunchKernelGGL(k_upscale, dim3((X + 63) / 64, (Y + 3) / 4, npair), b2, 0, s, pp,
                       pl.filled, pl.W, pl.H, X, Y, pl.p.fill_T);
  mark(6);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, STEREO_EHIP, "kernel launch: %s", hipGetErrorString(e));
  if (timed) ++c->timed_calls;
  return 0;
}

int common_checks(stereo_ctx* c, int W, int H, int Dmax, const stereo_params* params,
                  stereo_params* p) {
  if (W < 2 || H < 2 || W > STEREO_MAX_SIDE || H > STEREO_MAX_SIDE)
    return fail(c, STEREO_EINVAL, "image size %dx%d outside 2..%d", W, H, STEREO_MAX_SIDE);
  if (Dmax < 1 || Dmax > W || Dmax > STEREO_MAX_DMAX)
    return fail(c, STEREO_EINVAL, "Dmax %d outside 1..min(W=%d, %d)", Dmax, W, STEREO_MAX_DMAX);
  if (params) {
    if (params->size != sizeof(stereo_params))
      return fail(c, STEREO_EINVAL, "params.size %u != %zu", params->size, sizeof(stereo_params));
    *p = *params;
  } else {
    stereo_default_params(p);
  }
  const bool full = (p->flags & STEREO_F_FULL_RES) != 0;
  if (full && W > STEREO_MAX_SIDE / 2)
    return fail(c, STEREO_EINVAL, "full-resolution mode needs W <= %d", STEREO_MAX_SIDE / 2);
  return check_params(c, *p, full ? Dmax : (Dmax + 1) / 2);
}

}  // namespace stereo_host

using namespace stereo_host;

extern "C" {

void stereo_default_params(stereo_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->size = sizeof(stereo_params);
  p->lambda_ad = 0.3f;
  p->lambda_mc = 2.3f;
  p->cost_scale = 1024;
  p->color_delta = 13;
  p->arm_x = 21;
  p->arm_y = 31;
  p->fill_T = 3;
  p->flags = 0;
  p->arm_x_r = -1;
  p->fill_mode = 0;
}

int stereo_create(stereo_ctx** out, int device, size_t mem_cap) {
  if (!out) return STEREO_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return STEREO_EINVAL;
  }
  if (hipSetDevice(device) != hipSuccess) return STEREO_EHIP;
  stereo_ctx* c = new stereo_ctx();
  c->device = device;
  c->mem_cap = mem_cap;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      cu > 0)
    c->num_cu = cu;
  // the device's fixed scratch array, for stereo_disparity_noalloc
  c->noalloc_scratch = noalloc_scratch_of(device, &c->noalloc_err);
  *out = c;
  return 0;
}

void stereo_destroy(stereo_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  for (Plan* pl : c->plans) free_plan(pl);
  free_soft_plans(c->soft_plans);
  for (auto& b : c->l1_blocks) (void)hipFree(b.second);
  delete c;
}

const char* stereo_last_error(const stereo_ctx* c) { return c ? c->err.c_str() : "null context"; }

int stereo_disparity_batch(stereo_ctx* c, const uint8_t* const* left, const uint8_t* const* right,
                           int n, int W, int H, int Dmax, const stereo_params* params,
                           int16_t* const* out_disp, hipStream_t stream) {
  if (!c) return STEREO_EINVAL;
  c->err.clear();
  if (!left || !right || !out_disp || n < 1) return fail(c, STEREO_EINVAL, "null pointer or n < 1");
  for (int i = 0; i < n; ++i)
    if (!left[i] || !right[i] || !out_disp[i]) return fail(c, STEREO_EINVAL, "null image pointer %d", i);
  stereo_params p;
  int rc = common_checks(c, W, H, Dmax, params, &p);
  if (rc) return rc;
  HIP_TRY(c, hipSetDevice(c->device));
  const bool keep = (p.flags & STEREO_F_KEEP_INTERMEDIATES) != 0;
  const int per = std::min(n, kMaxPairs);
  Plan* pl = nullptr;
  rc = get_plan(c, W, H, Dmax, p, per, stream, stream, &pl);
  if (rc) return rc;
  // a graph captured from this call launches into the plan's memory later:
  // the plan is never evicted for another (it is freed by stereo_destroy)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    pl->captured = true;
  (void)hipGetLastError();
  for (int i0 = 0; i0 < n; i0 += kMaxPairs) {
    const int m = std::min(kMaxPairs, n - i0);
    PairPtrs pp{};
    for (int i = 0; i < m; ++i) {
      pp.left[i] = left[i0 + i];
      pp.right[i] = right[i0 + i];
      pp.out[i] = out_disp[i0 + i];
    }
    rc = run(c, *pl, pp, m, keep && i0 == 0, (p.flags & STEREO_F_STAGE_TIMING) != 0, stream);
    if (rc) return rc;
  }
  if (keep) c->last = pl;
  return 0;
}

int stereo_autotune(stereo_ctx* c, const uint8_t* const* left, const uint8_t* const* right, int n,
                    int W, int H, int Dmax, const stereo_params* params, int* chosen,
                    int* sizes, float* times_ms, int max_times, hipStream_t stream) {
  if (!c) return STEREO_EINVAL;
  c->err.clear();
  if (!left || !right || n < 1) return fail(c, STEREO_EINVAL, "null pointer or n < 1");
  const int m = std::min(n, kMaxPairs);
  for (int i = 0; i < m; ++i)
    if (!left[i] || !right[i]) return fail(c, STEREO_EINVAL, "null image pointer %d", i);
  stereo_params p;
  int rc = common_checks(c, W, H, Dmax, params, &p);
  if (rc) return rc;
  p.flags &= ~(STEREO_F_KEEP_INTERMEDIATES | STEREO_F_STAGE_TIMING);
  HIP_TRY(c, hipSetDevice(c->device));
  // the modelled default, then sizes ceil(D / k), k = 1 .. min(D, 32)
  Plan probe{};
  probe.W = W; probe.H = H; probe.Dmax = Dmax; probe.npair = m; probe.p = p;
  probe.X = full_res(p) ? W : (W + 1) / 2;
  probe.Y = full_res(p) ? H : (H + 1) / 2;
  probe.D = full_res(p) ? Dmax : (Dmax + 1) / 2;
  plan_geometry(probe, c->num_cu, 0);
  std::vector<int> cand{probe.csize};
  for (int k = 1; k <= std::min(probe.D, 32); ++k) {
    const int cs = (probe.D + k - 1) / k;
    if (std::find(cand.begin(), cand.end(), cs) == cand.end()) cand.push_back(cs);
  }
  // scratch output maps for the trial runs
  int16_t* outs = nullptr;
  HIP_TRY(c, hipMalloc(&outs, (size_t)m * W * H * 2));
  PairPtrs pp{};
  for (int i = 0; i < m; ++i) {
    pp.left[i] = left[i];
    pp.right[i] = right[i];
    pp.out[i] = outs + (size_t)i * W * H;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = probe.csize;
  float best_ms = 1e30f;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  for (size_t k = 0; k < cand.size() && he == hipSuccess && rc == 0; ++k) {
    set_tuned(c, W, H, Dmax, m, p, cand[k]);
    rc = evict_shape(c, W, H, Dmax, p);
    Plan* pl = nullptr;
    if (!rc) rc = get_plan(c, W, H, Dmax, p, m, stream, stream, &pl);
    if (!rc) rc = run(c, *pl, pp, m, false, false, stream);  // warm
    constexpr int kReps = 5;
    if (!rc) he = hipEventRecord(e0, stream);
    for (int r = 0; r < kReps && !rc && he == hipSuccess; ++r) rc = run(c, *pl, pp, m, false, false, stream);
    if (!rc && he == hipSuccess) he = hipEventRecord(e1, stream);
    if (!rc && he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (!rc && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    ms /= kReps;
    if ((int)k < max_times) {
      if (sizes) sizes[k] = cand[k];
      if (times_ms) times_ms[k] = ms;
    }
    if (!rc && he == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = cand[k];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipDeviceSynchronize();
  (void)hipFree(outs);
  if (!rc && he != hipSuccess) rc = fail(c, STEREO_EHIP, "autotune: %s", hipGetErrorString(he));
  set_tuned(c, W, H, Dmax, m, p, best);
  const int rc2 = evict_shape(c, W, H, Dmax, p);
  if (rc) return rc;
  if (rc2) return rc2;
  if (chosen) *chosen = best;
  if (max_times > (int)cand.size()) {
    if (sizes) sizes[cand.size()] = 0;
    if (times_ms) times_ms[cand.size()] = -1.f;
  }
  return 0;
}

int stereo_disparity(stereo_ctx* c, const uint8_t* left, const uint8_t* right, int W, int H,
                     int Dmax, const stereo_params* params, int16_t* out_disp, hipStream_t stream) {
  if (!c) return STEREO_EINVAL;
  return stereo_disparity_batch(c, &left, &right, 1, W, H, Dmax, params, &out_disp, stream);
}

int stereo_disparity_noalloc(stereo_ctx* c, const uint8_t* left, const uint8_t* right, int W,
                             int H, int Dmax, const stereo_params* params, int16_t* out_disp,
                             hipStream_t stream) {
  if (!c) return STEREO_EINVAL;
  c->err.clear();
  if (!left || !right || !out_disp) return fail(c, STEREO_EINVAL, "null pointer");
  stereo_params p;
  int rc = common_checks(c, W, H, Dmax, params, &p);
  if (rc) return rc;
  if (p.flags & (STEREO_F_KEEP_INTERMEDIATES | STEREO_F_STAGE_TIMING))
    return fail(c, STEREO_EINVAL, "stereo_disparity_noalloc takes neither "
                "STEREO_F_KEEP_INTERMEDIATES nor STEREO_F_STAGE_TIMING");
  if (!c->noalloc_scratch)
    return fail(c, STEREO_EHIP, "no fixed scratch on device %d: %s", c->device,
                c->noalloc_err.c_str());
  // the plan lives on the stack and its memory is the fixed array: geometry
  // and tables are host arithmetic, the set-up (padding cleared, cost table
  // written) is a kernel on the caller's stream
  Plan pl{};
  rc = plan_setup(c, pl, W, H, Dmax, p, 1, tuned_csize(c, W, H, Dmax, 1, p));
  if (rc) return rc;
  const size_t bytes = plan_bytes(pl).total;
  if (bytes > kNoallocBytes)
    return fail(c, STEREO_EINVAL, "%dx%d Dmax %d needs %zu bytes of scratch; the fixed array "
                "holds %zu (use stereo_disparity)", W, H, Dmax, bytes, kNoallocBytes);
  HIP_TRY(c, hipSetDevice(c->device));
  (void)hipGetLastError();
  plan_carve_and_init(pl, c->noalloc_scratch, stream);
  PairPtrs pp{};
  pp.left[0] = left;
  pp.right[0] = right;
  pp.out[0] = out_disp;
  return run(c, pl, pp, 1, false, false, stream);
}

int stereo_stage_times(stereo_ctx* c, double* ms, int* calls, int reset) {
  if (!c) return STEREO_EINVAL;
  c->err.clear();
  if (!ms) return fail(c, STEREO_EINVAL, "null ms");
  HIP_TRY(c, hipSetDevice(c->device));
  for (int i = 0; i < STEREO_NUM_STAGES; ++i) ms[i] = 0.0;
  const size_t per = STEREO_NUM_STAGES + 1;
  for (int k = 0; k < c->timed_calls; ++k) {
    hipEvent_t* ev = &c->events[(size_t)k * per];
    HIP_TRY(c, hipEventSynchronize(ev[STEREO_NUM_STAGES]));
    for (int i = 0; i < STEREO_NUM_STAGES; ++i) {
      float t = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&t, ev[i], ev[i + 1]));
      ms[i] += t;
    }
  }
  if (calls) *calls = c->timed_calls;
  if (reset) c->timed_calls = 0;
  return 0;
}

int stereo_get_intermediate(stereo_ctx* c, int which, int d, void* dst, size_t bytes,
                            hipStream_t stream) {
  if (!c) return STEREO_EINVAL;
  c->err.clear();
  Plan* pl = c->last;
  if (!pl) return fail(c, STEREO_EINVAL, "no call with STEREO_F_KEEP_INTERMEDIATES yet");
  if (!dst) return fail(c, STEREO_EINVAL, "null destination");
  HIP_TRY(c, hipSetDevice(c->device));
  const size_t n = (size_t)pl->X * pl->Y;
  auto need = [&](size_t b) { return bytes >= b; };
  switch (which) {
    case STEREO_I_LUT: {
      if (!need(263 * 2)) break;
      std::memcpy(dst, pl->lut_ad, 256 * 2);
      std::memcpy(static_cast<char*>(dst) + 512, pl->lut_mc, 7 * 2);
      return 0;
    }
    case STEREO_I_HALF_L: case STEREO_I_HALF_R: case STEREO_I_CENSUS_L: case STEREO_I_CENSUS_R: {
      if (!need(n)) break;
      const int img = (which == STEREO_I_HALF_R || which == STEREO_I_CENSUS_R) ? 1 : 0;
      std::vector<uint16_t> tmp(n);
      HIP_TRY(c, hipStreamSynchronize(stream));
      HIP_TRY(c, hipMemcpy2D(tmp.data(), (size_t)pl->X * 2,
                             pl->pk + (size_t)img * pl->Y * pl->XP + pl->pad, (size_t)pl->XP * 2,
                             (size_t)pl->X * 2, pl->Y, hipMemcpyDeviceToHost));
      const bool census = which == STEREO_I_CENSUS_L || which == STEREO_I_CENSUS_R;
      uint8_t* o = static_cast<uint8_t*>(dst);
      for (size_t i = 0; i < n; ++i) o[i] = census ? (uint8_t)(tmp[i] >> 8) : (uint8_t)tmp[i];
      return 0;
    }
    case STEREO_I_ARMS_L: case STEREO_I_ARMS_R: {
      if (!need(4 * n)) break;
      const int img = which == STEREO_I_ARMS_R ? 1 : 0;
      HIP_TRY(c, hipStreamSynchronize(stream));
      HIP_TRY(c, hipMemcpy2D(dst, (size_t)pl->X * 4, pl->arms + (size_t)img * pl->Y * pl->XA,
                             (size_t)pl->XA * 4, (size_t)pl->X * 4, pl->Y, hipMemcpyDeviceToHost));
      return 0;
    }
    case STEREO_I_COST_L_D: case STEREO_I_COST_R_D: case STEREO_I_CAX_L_D: case STEREO_I_CAX_R_D:
    case STEREO_I_CA_L_D: case STEREO_I_CA_R_D: {
      const bool cost = which == STEREO_I_COST_L_D || which == STEREO_I_COST_R_D;
      if (!need(cost ? 2 * n : 4 * n)) break;
      if (d < 0 || d >= pl->D) return fail(c, STEREO_EINVAL, "d %d outside 0..%d", d, pl->D - 1);
      if (!pl->dbg_block) {
        const size_t b = ((2 * n + 255) & ~size_t(255)) + 2 * ((4 * n + 255) & ~size_t(255));
        hipError_t e = hipMalloc(&pl->dbg_block, b);
        if (e != hipSuccess) {
          (void)hipGetLastError();
          return fail(c, STEREO_ENOMEM, "debug planes: %s", hipGetErrorString(e));
        }
        char* cur = static_cast<char*>(pl->dbg_block);
        pl->dbg_cost = carve<uint16_t>(cur, n);
        pl->dbg_cax = carve<uint32_t>(cur, n);
        pl->dbg_ca = carve<uint32_t>(cur, n);
      }
      // one-disparity run of the fused kernel on pair 0 with the debug planes
      // of the wanted base on; it overwrites the first d-chunk keys only
      MatchArgs a = match_args(*pl, d, d + 1, 1);
      a.dbg_cost = pl->dbg_cost; a.dbg_cax = pl->dbg_cax; a.dbg_ca = pl->dbg_ca;
      a.dbg_base = (which == STEREO_I_COST_R_D || which == STEREO_I_CAX_R_D ||
                    which == STEREO_I_CA_R_D) ? 1 : 0;
      launch_match(*pl, a, 1, stream);
      HIP_TRY(c, hipGetLastError());
      HIP_TRY(c, hipStreamSynchronize(stream));
      const void* src = cost ? (const void*)pl->dbg_cost
                      : (which == STEREO_I_CAX_L_D || which == STEREO_I_CAX_R_D)
                            ? (const void*)pl->dbg_cax : (const void*)pl->dbg_ca;
      HIP_TRY(c, hipMemcpy(dst, src, cost ? 2 * n : 4 * n, hipMemcpyDeviceToHost));
      return 0;
    }
    case STEREO_I_MINCOST_L: case STEREO_I_MINCOST_R: {
      if (!need(4 * n)) break;
      HIP_TRY(c, hipStreamSynchronize(stream));
      HIP_TRY(c, hipMemcpy(dst, pl->mincost + (which == STEREO_I_MINCOST_R ? pl->nk : 0), 4 * n,
                           hipMemcpyDeviceToHost));
      return 0;
    }
    case STEREO_I_DISP_L: case STEREO_I_DISP_R: {
      if (!need(2 * n)) break;
      HIP_TRY(c, hipStreamSynchronize(stream));
      HIP_TRY(c, hipMemcpy(dst, pl->disp + (which == STEREO_I_DISP_R ? pl->nk : 0), 2 * n,
                           hipMemcpyDeviceToHost));
      return 0;
    }
    case STEREO_I_GCP: {
      if (!need(n)) break;
      HIP_TRY(c, hipStreamSynchronize(stream));
      HIP_TRY(c, hipMemcpy(dst, pl->gcp, n, hipMemcpyDeviceToHost));
      return 0;
    }
    case STEREO_I_MEDIAN: case STEREO_I_FILLED: {
      if (!need(2 * n)) break;
      HIP_TRY(c, hipStreamSynchronize(stream));
      HIP_TRY(c, hipMemcpy(dst, which == STEREO_I_MEDIAN ? pl->med : pl->filled, 2 * n,
                           hipMemcpyDeviceToHost));
      return 0;
    }
    default:
      return fail(c, STEREO_EINVAL, "unknown intermediate %d", which);
  }
  return fail(c, STEREO_EINVAL, "destination of %zu bytes too small for intermediate %d", bytes,
              which);
}

}  // extern "C"
