/*
 * stereo.h - C interface of the MI355X stereo-matching library.
 *
 * The library computes the disparity map of a rectified stereo pair by the
 * method of Chang & Maruyama, "Real-Time High-Quality Stereo Matching System
 * on a GPU" (arXiv 2212.00488): gray-scale and 2x mean-pool downscale
 * (Sec. III-A, Eq. 2), absolute-difference plus mini-census matching cost
 * (Sec. III-B, Eq. 3-6), cross-based aggregation along x then y (Sec. III-C,
 * Eq. 7-8), winner-take-all for the left- and right-based maps (Eq. 9),
 * left/right cross-check into ground control points (Sec. III-D, Eq. 10),
 * median filter and bilateral filling of the other pixels (Sec. III-E,
 * Eq. 11) and bilateral upscale back to full resolution (Sec. IV, Step8).
 *
 * Conventions shared by every entry point
 *   - All image and map pointers are DEVICE pointers (HIP global memory) on
 *     the context's device, row-major, tightly packed (pitch = width).
 *   - Input images are uint8 RGB, interleaved, [H][W][3].  The output is an
 *     int16 full-resolution disparity map [H][W] for the left image, values
 *     in [0, Dmax-1] (even numbers and midpoints of the half-res map).
 *   - Dmax is the full-resolution disparity range: d in [0, Dmax-1] (Sec. II).
 *     The half-resolution search range is D = ceil(Dmax / 2).
 *   - Work is enqueued asynchronously on `stream` (0 = the null stream).  The
 *     caller keeps inputs and outputs alive and unmodified until the stream
 *     has passed the work.  Results are bit-exact and deterministic.
 *   - Every function returns 0 on success or a negative STEREO_E* code.  On
 *     error nothing is enqueued, the context stays usable and
 *     stereo_last_error() describes the failure.
 *   - A context may be used by one host thread at a time.
 */
#ifndef STEREO_H
#define STEREO_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STEREO_OK 0
#define STEREO_EINVAL (-1)  /* bad pointer, size, range or params              */
#define STEREO_ENOMEM (-2)  /* device allocation failed or mem_cap exceeded     */
#define STEREO_EHIP (-3)    /* a HIP runtime call failed                        */
#define STEREO_EUNIMPL (-4) /* not implemented                                  */

/* Largest supported full-resolution image side and disparity range. */
#define STEREO_MAX_SIDE 8192
#define STEREO_MAX_DMAX 512

/* params.flags */
#define STEREO_F_KEEP_INTERMEDIATES 1u /* keep per-call planes for stereo_get_intermediate */
#define STEREO_F_STAGE_TIMING 2u       /* time each stage with HIP events on the stream     */

/* Parameters of the method.  Defaults (stereo_default_params) are the paper's:
 * lambda_AD = 0.3, lambda_MC = 2.3 and T = 3 (Sec. V); arm caps 21 (x) and
 * 31 (y) and colour threshold 13 (Table II footnote, Sec. V). */
typedef struct stereo_params {
  uint32_t size;       /* must equal sizeof(stereo_params)                          */
  float lambda_ad;     /* Eq. 4, on brightness normalised to [0,1]; > 0              */
  float lambda_mc;     /* Eq. 5, on census Hamming distance; > 0                     */
  int32_t cost_scale;  /* fixed-point scale S of the cost tables, 1..1024            */
  int32_t color_delta; /* delta of Sec. III-C: arms take |I(t) - I(centre)| < delta  */
  int32_t arm_x;       /* per-side cap of the horizontal arms m, n; 0..127           */
  int32_t arm_y;       /* per-side cap of the vertical arms M, N; 0..127             */
  int32_t fill_T;      /* T of Sec. III-E (bilateral filling and upscale); >= 0      */
  uint32_t flags;      /* STEREO_F_*                                                 */
} stereo_params;

typedef struct stereo_ctx stereo_ctx; /* opaque, owned by the library */

/* Fills *p with the paper's parameters. */
void stereo_default_params(stereo_params* p);

/* Creates a context on HIP device `device`.  mem_cap bounds the library's
 * device scratch in bytes (0 = no bound).  *out receives the context. */
int stereo_create(stereo_ctx** out, int device, size_t mem_cap);

/* Frees the context and everything it allocated.  NULL is a no-op.  The
 * caller must have synchronised every stream it used with the context. */
void stereo_destroy(stereo_ctx* ctx);

/* Text of the last error on this context ("" if none).  Valid until the next
 * call on the context. */
const char* stereo_last_error(const stereo_ctx* ctx);

/* Disparity map of one pair (the whole path of Sec. III / Sec. IV Step1-8).
 *   left, right : device, uint8 [H][W][3] RGB, rectified so that a left pixel
 *                 (x,y) matches right pixel (x-d, y) (Sec. II).
 *   W, H        : 2..STEREO_MAX_SIDE.
 *   Dmax        : 1..min(W, STEREO_MAX_DMAX).
 *   params      : NULL for the defaults; else size must match and values be
 *                 in range, including (2 arm_x + 1)(2 arm_y + 1) * C_max < 2^24
 *                 where C_max is the largest table cost.
 *   out_disp    : device, int16 [H][W].
 * Scratch for each (W, H, Dmax, params) is allocated on first use and cached. */
int stereo_disparity(stereo_ctx* ctx, const uint8_t* left, const uint8_t* right, int W, int H,
                     int Dmax, const stereo_params* params, int16_t* out_disp,
                     hipStream_t stream);

/* n independent pairs of the same shape in one launch sequence: pair i reads
 * left[i], right[i] and writes out_disp[i] (all device pointers; the pointer
 * arrays themselves are host memory read during the call).  n >= 1. */
int stereo_disparity_batch(stereo_ctx* ctx, const uint8_t* const* left,
                           const uint8_t* const* right, int n, int W, int H, int Dmax,
                           const stereo_params* params, int16_t* const* out_disp,
                           hipStream_t stream);

/* Debug export of one plane of the last stereo_disparity call made with
 * STEREO_F_KEEP_INTERMEDIATES (pair 0 of a batch).  Copies into HOST memory
 * `dst`, which must hold at least `bytes` = the plane size; synchronises
 * `stream`.  Half-resolution planes are [Y][X] with X = ceil(W/2),
 * Y = ceil(H/2).  `d` (half-res disparity, 0..D-1) selects the plane of the
 * *_D items and is ignored otherwise. */
enum stereo_intermediate {
  STEREO_I_HALF_L = 1,    /* uint8  [Y][X] gray, downscaled (Eq. 2)                 */
  STEREO_I_HALF_R = 2,
  STEREO_I_CENSUS_L = 3,  /* uint8  [Y][X] 6-bit mini-census string                 */
  STEREO_I_CENSUS_R = 4,
  STEREO_I_ARMS_L = 5,    /* uint8  [Y][X][4] m, n, M, N                            */
  STEREO_I_ARMS_R = 6,
  STEREO_I_COST_L_D = 7,  /* uint16 [Y][X] C^L(x,y,d) (Eq. 3)                       */
  STEREO_I_COST_R_D = 8,  /* uint16 [Y][X] C^R(x,y,d) (Eq. 6)                       */
  STEREO_I_CAX_L_D = 9,   /* uint32 [Y][X] CA^L_x(x,y,d) (Eq. 7)                    */
  STEREO_I_CAX_R_D = 10,
  STEREO_I_CA_L_D = 11,   /* uint32 [Y][X] CA^L(x,y,d) (Eq. 8)                      */
  STEREO_I_CA_R_D = 12,
  STEREO_I_MINCOST_L = 13,/* uint32 [Y][X] min over d of CA^L                       */
  STEREO_I_MINCOST_R = 14,
  STEREO_I_DISP_L = 15,   /* int16  [Y][X] D^L (Eq. 9)                              */
  STEREO_I_DISP_R = 16,
  STEREO_I_GCP = 17,      /* uint8  [Y][X] 1 for ground control points (Eq. 10)     */
  STEREO_I_MEDIAN = 18,   /* int16  [Y][X] 3x3 median of D^L                        */
  STEREO_I_FILLED = 19,   /* int16  [Y][X] D+ after bilateral filling (Eq. 11)      */
  STEREO_I_LUT = 20       /* uint16 [263]: AD table [256] then census table [7]     */
};
int stereo_get_intermediate(stereo_ctx* ctx, int which, int d, void* dst, size_t bytes,
                            hipStream_t stream);

/* Device time of each stage, in the order of Sec. IV: 0 downscale (Step1),
 * 1 census + arms (Step2, Step4), 2 cost + x/y aggregation + WTA per
 * d-chunk (Step3, Step5), 3 minimum over the d-chunks (Step5), 4 cross-check
 * + median + filling (Step6, Step7), 5 upscale (Step8).  Sums, in milliseconds, over the calls made with
 * STEREO_F_STAGE_TIMING since the last reset, measured by HIP events
 * recorded on each call's stream around each stage's launch.  ms receives
 * STEREO_NUM_STAGES values; *calls (may be NULL) the number of calls.
 * Synchronises with the timed work.  reset != 0 clears the sums after
 * reading them. */
#define STEREO_NUM_STAGES 6
int stereo_stage_times(stereo_ctx* ctx, double* ms, int* calls, int reset);

#ifdef __cplusplus
}
#endif
#endif /* STEREO_H */
