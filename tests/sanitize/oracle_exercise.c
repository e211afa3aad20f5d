/* oracle_exercise.c -- drives every entry point of the CPU oracle over small
 * inputs (every element format, mode, operation and flag, edge data), for a
 * build with the address and undefined-behaviour sanitizers.  Exit status 0
 * when every call returned; the sanitizers abort on the first finding. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mxfft_oracle.h"

static uint32_t state = 20251204u;
static float rnd(void)
{
    state = state * 1664525u + 1013904223u;
    const float u = (float)((state >> 8) & 0xFFFFFF) / 16777216.0f;
    return ldexpf(u - 0.5f, (int)((state >> 3) % 40) - 20);
}

static int check(int st, int want, const char* what)
{
    if (st != want) {
        fprintf(stderr, "%s: status %d, expected %d\n", what, st, want);
        return 1;
    }
    return 0;
}

int main(void)
{
    int bad = 0;
    const int fmts[] = {ORC_E4M3, ORC_E5M2, ORC_E2M3, ORC_E3M2, ORC_E6M23};
    for (int f = 0; f < ORC_NFMT; f++) {
        int eb, mb, emin, emax;
        double mv;
        if (orc_fmt_info(f, &eb, &mb, &emin, &emax, &mv) != ORC_OK) continue;
        for (int c = 0; c < (1 << (1 + eb + mb)) && c < 4096; c++) {
            const double d = orc_decode_code(f, c);
            if (!isnan(d)) (void)orc_encode_code(f, orc_quantize(f, d));
        }
    }
    for (int N = 2; N <= 64; N *= 2) {
        const long nn = (long)N * N, batch = 3;
        float* x = malloc(sizeof(float) * 2 * nn * batch);
        float* y = malloc(sizeof(float) * 2 * nn * batch);
        int32_t k[3];
        for (long i = 0; i < 2 * nn * batch; i++) x[i] = rnd();
        memset(x + 2 * nn, 0, sizeof(float) * 2 * nn);          /* an all-zero slice */
        for (int fi = 0; fi < 5; fi++)
            for (int B = 2; B <= N && B <= 64; B *= 2)
                for (int op = 0; op < 3; op++)
                    for (int fi2 = 0; fi2 < 5; fi2++) {
                        const unsigned flv[5] = {0u, ORC_NO_PRESCALE | ORC_KEEP_SCALE, ORC_NORMALIZE, ORC_FUSED_RT,
                                                 ORC_QUANTIZE_OUT | ORC_FUSED_RT};
                        const unsigned fl = flv[fi2];
                        if (fmts[fi] == ORC_E6M23 && B > 8) continue;
                        const int st = orc_transform(op, ORC_MODE_MX, fmts[fi], B, N, batch, x, y, k, 0, 128.0, 5.0,
                                                     0.3, INT32_MIN, INT32_MAX, fl, 1);
                        bad |= check(st, ORC_OK, "mx transform");
                    }
        for (int mode = ORC_MODE_FP32; mode <= ORC_MODE_BF16; mode++)
            for (int op = 0; op < 3; op++)
                bad |= check(orc_transform(op, mode, ORC_E4M3, 2, N, batch, x, y, k, 0, 128.0, 5.0, 1.0 / 64,
                                           INT32_MIN, INT32_MAX, 0, 2), ORC_OK, "plain transform");
        /* given k for the inverse, clipped prescale, non-finite input */
        k[0] = 3; k[1] = 0; k[2] = -2;
        bad |= check(orc_transform(1, ORC_MODE_MX, ORC_E4M3, 2, N, batch, x, y, k, 1, 128.0, 5.0, 1.0 / 64, -4, 4, 0, 1),
                     ORC_OK, "inverse with k");
        x[5] = NAN;
        bad |= check(orc_transform(0, ORC_MODE_MX, ORC_E5M2, 2, N, batch, x, y, k, 0, 128.0, 5.0, 1.0 / 64,
                                   INT32_MIN, INT32_MAX, 0, 1), ORC_ENONFINITE, "non-finite");
        x[5] = 1.0f;
        int32_t kp;
        (void)orc_prescale(x, nn, 3.0, 97.5, 1e-3, INT32_MIN, INT32_MAX, &kp);
        int* tr = malloc(sizeof(int) * 3 * 16 * (N > 1 ? N : 1));
        bad |= check(orc_pass_lines(ORC_MODE_MX, ORC_E4M3, 2, N, 0, N, x, tr), ORC_OK, "pass lines");
        double* mant = malloc(sizeof(double) * 2 * nn);
        int32_t* E = malloc(sizeof(int32_t) * nn);
        bad |= check(orc_column_encode(ORC_E4M3, 2, N, x, mant, E), ORC_OK, "column encode");
        double* z = malloc(sizeof(double) * 2 * nn);
        for (long i = 0; i < 2 * nn; i++) z[i] = x[i];
        bad |= check(orc_fft2_f64(N, 1, 0, z), ORC_OK, "fft2 f64");
        bad |= check(orc_fft1_f64(N, N, 1, z), ORC_OK, "fft1 f64");
        float* img = malloc(sizeof(float) * nn);
        bad |= check(orc_rss(x, 1, 3, nn, img), ORC_OK, "rss");
        if (N >= 16) {
            double s;
            bad |= check(orc_ssim(img, img, N, 1.0, &s), ORC_OK, "ssim");
        }
        free(img); free(z); free(E); free(mant); free(tr); free(y); free(x);
    }
    if (!bad) printf("oracle exercise: ok\n");
    return bad;
}
