/*
 * mxfft_oracle.h -- interface of the CPU oracle (test infrastructure only).
 *
 * Plain, slow, obviously correct CPU definition of the MX-scaled mixed-precision
 * radix-2 2D FFT (Alg. 1 global prescale, Alg. 2 MX butterfly, Eq. 1 forward and
 * round-trip transforms).  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares nothing with the GPU library.
 *
 * Data: complex values are interleaved FP32 (re, im); an N x N slice is row-major.
 */
#ifndef MXFFT_ORACLE_H
#define MXFFT_ORACLE_H

#include <stdint.h>

enum { ORC_E4M3 = 0, ORC_E5M2 = 1, ORC_FP16 = 2, ORC_BF16 = 3, ORC_E6M23 = 4, ORC_E2M3 = 5, ORC_E3M2 = 6, ORC_NFMT = 7 };
enum { ORC_MODE_MX = 0, ORC_MODE_FP32 = 1, ORC_MODE_FP16 = 2, ORC_MODE_BF16 = 3 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENONFINITE = -4, ORC_ERANGE = -5 };
enum { ORC_NO_PRESCALE = 1u, ORC_KEEP_SCALE = 2u, ORC_NORMALIZE = 4u, ORC_FUSED_RT = 8u, ORC_QUANTIZE_OUT = 32u };

int orc_fmt_info(int f, int* ebits, int* mbits, int* emin, int* emax, double* maxval);
double orc_quantize(int f, double x);
void orc_quantize_array(int f, const double* x, double* q, long n);
int orc_encode_code(int f, double q);
double orc_decode_code(int f, int c);
int orc_mx_encode(int f, const double* vals, int n, double* mant);
void orc_twiddle64(int j, int m, int inverse, double* wr, double* wi);
void orc_mx_butterfly(int f, int cb, const float* u, const float* v, const double* x, int Ew,
                      float* y0, float* y1, int* ev_kr_eo);
int orc_prescale(const float* x, long n, double target, double tau, double tau_min,
                 int kmin, int kmax, int32_t* k_out);
/* op: 0 forward, 1 inverse, 2 round trip.  kp: per-slice prescale exponents,
 * written (forward, round trip, inverse without kp_given) or read (inverse with
 * kp_given).  Returns the first error over the batch. */
int orc_transform(int op, int mode, int fmt, int B, int N, long batch,
                  const float* in, float* out, int32_t* kp, int kp_given,
                  double target, double tau, double tau_min, int kmin, int kmax,
                  unsigned flags, int nthreads);
int orc_pass_lines(int mode, int fmt, int B, int N, int inverse, long lines, float* a, int* trace);
int orc_column_encode(int fmt, int B, int N, const float* a, double* mant, int32_t* E);
int orc_fft2_f64(int N, long batch, int inverse, double* a);
int orc_fft1_f64(int N, long lines, int inverse, double* a);

/* Eq. 1 root-sum-of-squares coil combine (FP32, coils in order) and the mean
 * SSIM (Wang et al. 2004, 11 x 11 Gaussian window, sigma 1.5, FP64). */
int orc_rss(const float* T, long recon, int coils, long nn, float* out);
int orc_ssim(const float* x, const float* y, int N, double L, double* ssim);

#endif
