/*
 * xcorr_oracle.c -- plain CPU oracle for the 4-bit X-engine cross-correlation.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
 * CPU-baseline leg of the benchmark load this library. The GPU library never
 * links, loads or calls it, and the two share no source, header or table.
 *
 * What it computes (Klages et al., "GPU Kernels for High-Speed 4-Bit
 * Astrophysical Data Processing"):
 *   - Sec. III (Excess-8 encoding): every complex sample is one byte holding
 *     two 4-bit fields, each the value plus 8, so a field in [0,15] stands for
 *     a value in [-8,7]. Reading taken here: the real part is the high nibble,
 *     the imaginary part the low nibble.
 *   - Sec. II-A, Eq. 1: the correlation of elements X and Y at one instant is
 *     X * conj(Y) = (XRe*YRe + XIm*YIm, XIm*YRe - XRe*YIm).
 *   - Sec. II-A: these products are summed over the T time samples of an
 *     integration; the matrix is Hermitian, so only i <= j is kept (Eq. 2).
 *   - Sec. III-A (last step of the kernel description): new sums are added to
 *     the results already held in the output (the accumulate flag).
 *   - Sec. III, Eq. 3: the paper's own route through unsigned products plus
 *     per-element offset sums, kept here as a second, independent route.
 *
 * Input layout: in[f][t][e], one byte per (channel, time, element).
 * Output layout: vis[f][k(i,j)][2] = (re, im) in int64, k(i,j) the row-major
 * packed upper-triangle index i*(2n-i+1)/2 + (j-i).
 *
 * Every sum is held in int64; callers range-check the result into int32.
 * Loops are the plain definition: no blocking, no reordering, no reuse.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Sec. III: a 4-bit field stores value + 8. Real part = high nibble. */
static int64_t field_value(unsigned nibble) { return (int64_t)nibble - 8; }
static int64_t sample_re(uint8_t byte) { return field_value((unsigned)byte >> 4); }
static int64_t sample_im(uint8_t byte) { return field_value((unsigned)byte & 0x0Fu); }

/* Packed row-major upper triangle: row i holds j = i..n-1 contiguously. */
static int64_t tri_index(int64_t n, int64_t i, int64_t j) {
  return i * (2 * n - i + 1) / 2 + (j - i);
}

/* Eq. 1 summed over time: V_ij = sum_t x_i(t) * conj(x_j(t)). */
static void correlate_pair(const uint8_t* chan, int64_t n, int64_t t_count,
                           int64_t i, int64_t j, int64_t* re, int64_t* im) {
  int64_t sum_re = 0, sum_im = 0;
  for (int64_t t = 0; t < t_count; ++t) {
    uint8_t x = chan[t * n + i];
    uint8_t y = chan[t * n + j];
    int64_t x_re = sample_re(x), x_im = sample_im(x);
    int64_t y_re = sample_re(y), y_im = sample_im(y);
    sum_re += x_re * y_re + x_im * y_im;
    sum_im += x_im * y_re - x_re * y_im;
  }
  *re = sum_re;
  *im = sum_im;
}

static int bad_shape(const void* a, const void* b, int n, int f, int t) {
  return a == NULL || b == NULL || n < 1 || f < 1 || t < 0;
}

/* Upper triangle of every channel. accumulate != 0 adds to vis (Sec. III-A). */
int xcorr_oracle_correlate(const uint8_t* in, int64_t* vis, int n, int f, int t,
                           int accumulate) {
  if (bad_shape(in, vis, n, f, t)) return -1;
  const int64_t N = n, T = t, entries = N * (N + 1) / 2;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int64_t ch = 0; ch < f; ++ch) {
    for (int64_t i = 0; i < N; ++i) {
      const uint8_t* chan = in + ch * T * N;
      int64_t* out = vis + 2 * ch * entries;
      for (int64_t j = i; j < N; ++j) {
        int64_t re, im;
        correlate_pair(chan, N, T, i, j, &re, &im);
        int64_t k = tri_index(N, i, j);
        if (accumulate) {
          out[2 * k] += re;
          out[2 * k + 1] += im;
        } else {
          out[2 * k] = re;
          out[2 * k + 1] = im;
        }
      }
    }
  }
  return 0;
}

/* Every (i, j), lower triangle included: full[f][i][j][2]. Used to check the
 * Hermitian property stated in Sec. II-A rather than assume it. */
int xcorr_oracle_full_matrix(const uint8_t* in, int64_t* full, int n, int f, int t) {
  if (bad_shape(in, full, n, f, t)) return -1;
  const int64_t N = n, T = t;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int64_t ch = 0; ch < f; ++ch) {
    for (int64_t i = 0; i < N; ++i) {
      const uint8_t* chan = in + ch * T * N;
      for (int64_t j = 0; j < N; ++j) {
        int64_t* o = full + 2 * ((ch * N + i) * N + j);
        correlate_pair(chan, N, T, i, j, &o[0], &o[1]);
      }
    }
  }
  return 0;
}

/* Selected entries: fij[m][3] = (channel, i, j) with i <= j; out[m][2]. For
 * spot checks of outputs too large to compute in full. */
int xcorr_oracle_entries(const uint8_t* in, int n, int f, int t, const int64_t* fij,
                         int64_t m, int64_t* out) {
  if (bad_shape(in, out, n, f, t) || (m > 0 && fij == NULL)) return -1;
  const int64_t N = n, T = t;
  for (int64_t q = 0; q < m; ++q) {
    int64_t ch = fij[3 * q], i = fij[3 * q + 1], j = fij[3 * q + 2];
    if (ch < 0 || ch >= f || i < 0 || j < i || j >= N) return -1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < m; ++q) {
    int64_t ch = fij[3 * q], i = fij[3 * q + 1], j = fij[3 * q + 2];
    correlate_pair(in + ch * T * N, N, T, i, j, &out[2 * q], &out[2 * q + 1]);
  }
  return 0;
}

/*
 * The paper's own route (Sec. III, Eq. 3), written out as three passes in the
 * order the paper gives them:
 *   1. running sums per element of (XRe + XIm) and (XRe - XIm) over t, taken on
 *      the encoded fields (values in [0,15]);
 *   2. the offset B(X,Y,t) = ( -8*(sum(X+) + sum(Y+)) + 128*t,
 *                               8*(sum(X-) - sum(Y-)) ) seeded into each entry;
 *   3. the products of the encoded fields, combined as in Eq. 1, added on top.
 * It shares the output index with the plain route but not the decode, so a
 * wrong sign or offset in either route shows up as a mismatch.
 */
int xcorr_oracle_offset_route(const uint8_t* in, int64_t* vis, int n, int f, int t) {
  if (bad_shape(in, vis, n, f, t)) return -1;
  const int64_t N = n, T = t, entries = N * (N + 1) / 2;
  int64_t* run_plus = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
  int64_t* run_minus = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
  if (run_plus == NULL || run_minus == NULL) {
    free(run_plus);
    free(run_minus);
    return -2;
  }
  for (int64_t ch = 0; ch < f; ++ch) {
    const uint8_t* chan = in + ch * T * N;
    int64_t* out = vis + 2 * ch * entries;
    /* pass 1: running sums of the encoded fields, per element */
    for (int64_t e = 0; e < N; ++e) {
      int64_t plus = 0, minus = 0;
      for (int64_t s = 0; s < T; ++s) {
        unsigned u = chan[s * N + e];
        int64_t ure = u >> 4, uim = u & 0x0Fu;
        plus += ure + uim;
        minus += ure - uim;
      }
      run_plus[e] = plus;
      run_minus[e] = minus;
    }
    /* pass 2: pre-seed every entry with B(X,Y,t) */
    for (int64_t i = 0; i < N; ++i) {
      for (int64_t j = i; j < N; ++j) {
        int64_t k = tri_index(N, i, j);
        out[2 * k] = -8 * (run_plus[i] + run_plus[j]) + 128 * T;
        out[2 * k + 1] = 8 * (run_minus[i] - run_minus[j]);
      }
    }
    /* pass 3: add the products of the encoded fields (Eq. 1 on [0,15]) */
    for (int64_t i = 0; i < N; ++i) {
      for (int64_t j = i; j < N; ++j) {
        int64_t re = 0, im = 0;
        for (int64_t s = 0; s < T; ++s) {
          unsigned x = chan[s * N + i], y = chan[s * N + j];
          int64_t xr = x >> 4, xi = x & 0x0Fu, yr = y >> 4, yi = y & 0x0Fu;
          re += xr * yr + xi * yi;
          im += xi * yr - xr * yi;
        }
        int64_t k = tri_index(N, i, j);
        out[2 * k] += re;
        out[2 * k + 1] += im;
      }
    }
  }
  free(run_plus);
  free(run_minus);
  return 0;
}

/* Number of OpenMP threads the oracle loops run on (1 without OpenMP). */
int xcorr_oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
