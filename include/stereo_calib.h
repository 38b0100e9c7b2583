/* Peak-rate probes of the device the stereo library runs on.
 *
 * These are measurement tools, not part of the stereo path: they give the
 * denominators of the roofline fractions reported for the path's kernels
 * (LDS read bandwidth for the fused aggregation kernel, whose on-chip
 * traffic the paper's Sec. VI names as the bound; device-memory copy
 * bandwidth for the streaming kernels; the integer vector-ALU issue rate).
 * Each call enqueues one kernel on `stream` and returns at once; the caller
 * times it (HIP events on the same stream).  All pointers are device memory
 * owned by the caller.  Return 0, or STEREO_EINVAL for a bad argument and
 * STEREO_EHIP when the launch fails (include/stereo.h codes). */
#ifndef STEREO_CALIB_H
#define STEREO_CALIB_H

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* LDS reads: `blocks` workgroups of 1024 threads; each thread reads
 * iters x 16 x 16 bytes from a 64 KiB LDS array with 16-byte loads, every
 * wave's load covering 1 KiB of consecutive bytes (no bank conflict).
 * LDS bytes read = blocks * 1024 * iters * 256.  sink: device, uint32
 * [blocks * 1024], written once per thread so no load can be dropped. */
int stereo_calib_lds_read(uint32_t* sink, int blocks, int iters, hipStream_t stream);

/* 32-bit integer VALU: `blocks` workgroups of 1024 threads, each thread
 * runs iters x 256 dependent-free 32-bit integer adds and xors (16
 * independent chains).  Lane operations = blocks * 1024 * iters * 256.
 * sink as for stereo_calib_lds_read. */
int stereo_calib_valu(uint32_t* sink, int blocks, int iters, hipStream_t stream);

/* Device copy of `bytes` (a multiple of 16, both pointers 16-byte aligned)
 * from src to dst with 16-byte loads and stores, a grid of `blocks`
 * workgroups of 256 threads striding over the buffer.  Device-memory bytes
 * moved = 2 * bytes. */
int stereo_calib_copy(const void* src, void* dst, size_t bytes, int blocks, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* STEREO_CALIB_H */
