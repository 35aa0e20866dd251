/* Measurement probes of the device, built as a library of their own (libdirac_probe.so) beside the
 * operator library.  They are not part of the method: they give the measured denominators printed
 * next to the published peaks (sustained copy bandwidth, FMA rate) and the ceiling of the stencils'
 * memory access pattern (one output row from seven input rows) without their arithmetic.
 *
 * Every call times `reps` launches between two HIP events on `stream` (0: the null stream), after
 * one untimed launch, and synchronises with the stream.  All buffers are device memory owned by the
 * caller, 16-byte aligned and not overlapping.  Return codes: 0 success, -1 bad arguments (nothing
 * launched), -3 a HIP call failed. */
#ifndef DIRAC_PROBE_H
#define DIRAC_PROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Copies nbytes (a positive multiple of 16) from src to dst, one 16-byte load and store per lane;
 * returns (read + written bytes) / second. */
int dirac_probe_copy(const void* src, void* dst, size_t nbytes, int reps, double* bytes_per_s, void* stream);

/* A register-resident loop of independent, non-packed fused multiply-adds; fp64 = 0 for FP32, 1 for
 * FP64; 16 work-groups of 256 threads per CU.  Returns flop / second (an FMA counts 2).  sink: at
 * least 8 device bytes the kernel may write (it never does for the inputs used). */
int dirac_probe_fma(int fp64, void* sink, double* flops_per_s, void* stream);

/* The row-gather pattern of the Wilson and staggered row kernels without their arithmetic: over a
 * periodic nx*ny*nz*nt lattice of site blocks of site_bytes bytes (a positive multiple of 16;
 * in and out each hold nx*ny*nz*nt*site_bytes bytes, site-major with x fastest), one work-group per
 * x-row reads its own row and, with nrows = 7, the six rows one step away in +-y, +-z, +-t (all in
 * flight at once, 16 bytes per lane) and writes one row (the exclusive or of the rows read); nrows = 1
 * is a row-by-row copy with the same loads, whose bytes are known exactly (counter calibration).  Rows are taken in the
 * stencils' order: 4 x 4 (y, z) blocks over the whole t range, each of the eight XCDs a contiguous
 * eighth.  Needs ny, nz divisible by 4, ny*nz*nt divisible by 8, nx*site_bytes/16 <= 3072 units.
 * Returns (one read and one write of the vector) / second, the stencils' byte count without links. */
int dirac_probe_row_gather(const void* in, void* out, int nx, int ny, int nz, int nt, int site_bytes, int nrows,
                           int reps, double* bytes_per_s, void* stream);

#ifdef __cplusplus
}
#endif

#endif
