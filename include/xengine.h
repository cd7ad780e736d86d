/*
 * xengine.h -- C ABI of the MI355X (gfx950) 4-bit X-engine correlator.
 *
 * The operation (Klages et al., "GPU Kernels for High-Speed 4-Bit
 * Astrophysical Data Processing"):
 *   For every frequency channel f and every element pair i <= j,
 *     V_f[i][j] = sum over t of x_i(t) * conj(x_j(t))
 *   with the complex product written out in Eq. 1 (Sec. II-A):
 *     Re = xRe*yRe + xIm*yIm,   Im = xIm*yRe - xRe*yIm.
 *   Only the upper triangle is produced: the matrix is Hermitian (Sec. II-A,
 *   Eq. 2 counts N(N+1)/2 entries).
 *
 * Input samples (Sec. III, Excess-8): one byte per complex sample; the high
 * nibble holds Re + 8 and the low nibble Im + 8, each value in [-8, 7].
 *
 * Layouts (all row-major, no padding):
 *   input   uint8_t  in[F][T][N]          channel, time sample, element
 *   output  int32_t  vis[F][N(N+1)/2][2]  (re, im) per entry; entry (i, j),
 *           i <= j, sits at k(i,j) = i*(2N-i+1)/2 + (j-i), so each row i of the
 *           triangle is contiguous.
 *
 * Accumulation (Sec. III-A: new sums are added to the results already held):
 *   accumulate = 0 overwrites vis; accumulate = 1 adds to it. t_prev is the
 *   number of samples already summed into vis (0 when overwriting). Sums are
 *   exact in int32 while t_prev + t <= XENG_MAX_SAMPLES, since one sample
 *   contributes at most 128 in magnitude; beyond that the call is refused.
 *
 * Memory and streams: every d_ pointer is device memory owned by the caller
 * (typically allocated through PyTorch). The library never allocates, frees or
 * keeps device memory. All GPU work is enqueued on the caller's hipStream_t
 * (passed as void*, NULL = the null stream) and returns without waiting;
 * buffers must stay valid until that work completes.
 *
 * Errors: every call returns an xeng_status; nothing throws or aborts across
 * this boundary. xeng_last_error() returns a message for the calling thread's
 * last failed call.
 */
#ifndef XENGINE_H
#define XENGINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XENG_MAX_SAMPLES 16777215LL

typedef enum xeng_status {
  XENG_OK = 0,
  XENG_EINVAL = -1,    /* bad pointer, size, alignment or overlap */
  XENG_ERANGE = -2,    /* t_prev + t would leave the exact int32 range */
  XENG_ENOMEM = -3,    /* host allocation failed, or workspace too small */
  XENG_EDEVICE = -4,   /* a HIP runtime call failed; see xeng_last_error() */
  XENG_EBUSY = -5,     /* admission refused: no memory or slot free now */
  XENG_ENOTFOUND = -6  /* unknown job, ticket or variant */
} xeng_status;

/* Message for the calling thread's most recent failed call ("" if none).
 * The pointer stays valid until the thread's next call into the library. */
const char* xeng_last_error(void);

/* Library version string. */
const char* xeng_version(void);

/* Entries of the packed upper triangle, n(n+1)/2 (Eq. 2); -1 if n < 0. */
int64_t xeng_vis_entries(int n);

/* Packed index k(i,j) = i*(2n-i+1)/2 + (j-i) for 0 <= i <= j < n, else -1. */
int64_t xeng_tri_index(int n, int i, int j);

/* Number of square tiles of edge `tile` that cover the upper triangle of an
 * n x n matrix (Sec. II-C, Fig. 1: 36 tiles of 32 for n = 256); -1 if invalid. */
int64_t xeng_tile_count(int n, int tile);

/*
 * Plain correlation of one job (Sec. II-A, Eq. 1 summed over t; upper
 * triangle per Eq. 2).
 *   d_in   device uint8_t[f][t][n], read only; any alignment.
 *   d_vis  device int32_t[f][n(n+1)/2][2], 8-byte aligned; must not overlap d_in.
 *   n >= 1 elements, f >= 1 channels, t >= 0 samples.
 *   t == 0: zero-fills vis when accumulate == 0, does nothing otherwise.
 * Returns XENG_EINVAL, XENG_ERANGE or XENG_EDEVICE on failure, in which case
 * nothing was enqueued.
 */
xeng_status xeng_correlate(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                           int64_t t_prev, int accumulate, void* hip_stream);

/*
 * Kernel variants, for the autotuner and for tests that compare variants.
 * A variant fixes the tile shape and the samples staged per step; split_t >= 1
 * divides the time axis among that many workgroups per tile (partial sums are
 * combined with exact int32 atomic adds). Every variant gives bit-identical
 * results. variant = -1 lets the library choose (same as xeng_correlate).
 */
int xeng_variant_count(void);
const char* xeng_variant_name(int variant);   /* NULL if out of range */
xeng_status xeng_correlate_variant(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                                   int64_t t_prev, int accumulate, int variant, int split_t,
                                   void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* XENGINE_H */
