// Host-side pipeline of the integer path, shared by the library's sources:
// per-shape plans and the launch sequence of one call.
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"
#include "context.h"
#include "stereo.h"

namespace stereo_host {

// Scratch and launch geometry of the integer path for one (W, H, Dmax,
// params, owner); planes are carved from one device allocation.
struct Plan {
  int W = 0, H = 0, Dmax = 0, X = 0, Y = 0, D = 0, npair = 0;
  stereo_params p{};
  uint16_t lut_ad[256]{}, lut_mc[7]{};
  int cmax = 0;
  int dbits = 8;                // bits of d in the WTA keys
  int ns = 1, kmax = 8, nstrips = 0, nbands = 0;
  int csize = 1, nchunk = 0;    // k_match d-chunk size and chunk count ceil(D / csize)
  int XP = 0, pad = 0, XA = 0;  // padded pitches of pk and arms
  int nk = 0;                   // padded plane stride of keys, disp and mincost
  size_t bytes = 0;
  // device memory, one block carved into planes
  void* block = nullptr;
  uint8_t* half = nullptr;    // [2*npair][Y][X]
  uint16_t* pk = nullptr;     // [2][2*npair][Y][XP]  gray | census<<8, zero padding; the
                              // second copy one column to the right
  uint32_t* arms = nullptr;   // [2*npair][Y][XA]  zero padding
  uint32_t* xoff = nullptr;   // [2*npair][Y][XA]  k_match row-buffer offsets of the
                              // horizontal arm ends, zero padding
  uint16_t* tab = nullptr;    // [7][kTabPitch]
  uint32_t* keys = nullptr;   // [npair][nchunk][2][Y][X]
  int16_t* disp = nullptr;    // [2*npair][Y][X]
  uint32_t* mincost = nullptr;// [2*npair][Y][X]
  uint8_t* gcp = nullptr;     // [npair][Y][X]
  int16_t* med = nullptr;     // [npair][Y][X]
  int16_t* filled = nullptr;  // [npair][Y][X]
  // debug planes, allocated on demand
  void* dbg_block = nullptr;
  uint16_t* dbg_cost = nullptr;
  uint32_t* dbg_cax = nullptr;
  uint32_t* dbg_ca = nullptr;
  uint64_t last_use = 0;
  const void* owner = nullptr;  // stream (or server slot) the plan belongs to
  int pins = 0;                 // server graphs that launch into this plan's memory
  bool captured = false;        // used under a caller's graph capture: kept until destroy
};

// Validates sizes and params (NULL = defaults) into *p.
int common_checks(stereo_ctx* c, int W, int H, int Dmax, const stereo_params* params,
                  stereo_params* p);
// The cached plan of (W, H, Dmax, p, owner) holding at least npair pairs,
// made (and least recently used plans evicted under the memory cap, except
// pinned ones) when missing; a new plan's set-up is enqueued on stream s,
// the stream its work will run on.  Calls with different owners never share
// scratch, so their work may overlap on the device.
int get_plan(stereo_ctx* c, int W, int H, int Dmax, const stereo_params& p, int npair,
             const void* owner, hipStream_t s, Plan** out);
// Frees one plan of the context (the caller has synchronised its work).
void drop_plan(stereo_ctx* c, Plan* pl);
// Enqueues the whole path for npair (<= plan's) pairs on stream s.  Makes no
// allocation, memset or synchronisation, so it may be captured in a graph.
int run(stereo_ctx* c, Plan& pl, const stereo_dev::PairPtrs& pp, int npair, bool keep,
        bool timed, hipStream_t s);

}  // namespace stereo_host
