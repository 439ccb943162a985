/*
 * Plain FP64 CPU oracle for block-DCT filtering (Amin-Naji & Aghagolzadeh,
 * "Block DCT filtering using vector processing").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library.  It shares no code, header, table or helper with the
 * HIP implementation.
 *
 * What it computes is the plain definition the method reaches exactly:
 *   - the orthonormal 2-D DCT-II of an N x N block, BLOCK = C.block.C^t
 *     (Sec. II.A, eq. 1), with C orthogonal so that C^-1 = C^t (eq. 2), and
 *     its inverse block = C^t.BLOCK.C (eq. 3), both written out as the
 *     double sums of their definition;
 *   - the block-local spatial filter of a custom mask W (Sec. II.B, eq. 4-5),
 *     applied as a correlation (mask entry W[p][q] weights the pixel at row
 *     offset p - a_h and column offset q - a_w from the output pixel, with
 *     a = floor((K-1)/2)), reading zeros outside the block (zero padding,
 *     Sec. II.B) or the nearest pixel of the same block (border replication,
 *     Sec. II.C and Fig. 1).  The block never reads a neighbouring block.
 *   - the filtered coefficients DCT(filter(IDCT(X))) that the DCT-domain
 *     method must reproduce (eq. 11 for zero padding, eq. 20 for
 *     replication), and the operator obtained by probing that map with unit
 *     coefficient vectors.
 *   - the filtered pixels filter(IDCT(X)) of coefficient blocks and the
 *     pixel-output operator probed the same way (the filtered result taken
 *     back to the spatial domain, Sec. III);
 *   - the image-level variant: the whole image filtered across block
 *     boundaries (only the image border padded), then cut into blocks again;
 *   - the uint8 conversion of a filtered pixel (Sec. III): the FP64
 *     filtered value rounded half up and saturated to [0, 255]; pixels whose
 *     FP64 value lies within 1e-3 of a .5 boundary are flagged (either
 *     neighbouring integer is accepted for them).
 *
 * Loops over independent blocks carry an OpenMP pragma; nothing else is
 * blocked, fused or reordered.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXN 32
#define OR_BORDER_ZERO 0
#define OR_BORDER_REPLICATE 1

/* Threads used by the loops over blocks (n < 1 restores the default). */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    static int deflt = 0;
    if (deflt == 0)
        deflt = omp_get_max_threads();
    omp_set_num_threads(n >= 1 ? n : deflt);
#else
    (void)n;
#endif
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* C[k][n] = alpha_k cos(pi (2n+1) k / (2N)); alpha_0 = sqrt(1/N), else sqrt(2/N).
 * Orthonormal scaling is the one that makes C^-1 = C^t (eq. 2). */
void or_dct_matrix(int N, double *C)
{
    for (int k = 0; k < N; ++k) {
        double alpha = (k == 0) ? sqrt(1.0 / N) : sqrt(2.0 / N);
        for (int n = 0; n < N; ++n)
            C[k * N + n] = alpha * cos(M_PI * (2.0 * n + 1.0) * k / (2.0 * N));
    }
}

/* Eq. 1: X[u][v] = sum_i sum_j C[u][i] x[i][j] C[v][j]. */
static void dct2_block(int N, const double *C, const double *x, double *X)
{
    for (int u = 0; u < N; ++u)
        for (int v = 0; v < N; ++v) {
            double s = 0.0;
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j)
                    s += C[u * N + i] * x[i * N + j] * C[v * N + j];
            X[u * N + v] = s;
        }
}

/* Eq. 3: x[i][j] = sum_u sum_v C[u][i] X[u][v] C[v][j]. */
static void idct2_block(int N, const double *C, const double *X, double *x)
{
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int u = 0; u < N; ++u)
                for (int v = 0; v < N; ++v)
                    s += C[u * N + i] * X[u * N + v] * C[v * N + j];
            x[i * N + j] = s;
        }
}

static int clamp_index(int v, int n)
{
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

/* Eq. 5 read as a correlation over a block-local neighbourhood. */
static void filter_block(int N, const double *x, const double *W, int kh, int kw,
                         int border, double *f)
{
    int ah = (kh - 1) / 2, aw = (kw - 1) / 2;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int p = 0; p < kh; ++p)
                for (int q = 0; q < kw; ++q) {
                    int r = i + p - ah, c = j + q - aw;
                    double v;
                    if (border == OR_BORDER_ZERO) {
                        if (r < 0 || r >= N || c < 0 || c >= N)
                            continue;
                        v = x[r * N + c];
                    } else {
                        v = x[clamp_index(r, N) * N + clamp_index(c, N)];
                    }
                    s += W[p * kw + q] * v;
                }
            f[i * N + j] = s;
        }
}

/* Sec. III uint8 conversion of the FP64 filtered value. */
static uint8_t to_u8(double f)
{
    double v = floor(f + 0.5);
    if (!(v > 0.0))
        return 0;
    if (v > 255.0)
        return 255;
    return (uint8_t)v;
}

static int near_half(double f)
{
    return fabs(f - floor(f) - 0.5) < 1e-3;
}

static int check_args(int N, int kh, int kw, int border)
{
    if (N < 1 || N > OR_MAXN || kh < 1 || kw < 1 || kh > 2 * N + 1 || kw > 2 * N + 1)
        return -1;
    if (border != OR_BORDER_ZERO && border != OR_BORDER_REPLICATE)
        return -1;
    return 0;
}

/* Batch forward DCT (eq. 1): x [B][N][N] -> X [B][N][N]. */
int or_dct2(int N, int64_t B, const double *x, double *X)
{
    if (N < 1 || N > OR_MAXN || B < 0)
        return -1;
    double C[OR_MAXN * OR_MAXN];
    or_dct_matrix(N, C);
    int64_t nn = (int64_t)N * N;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b)
        dct2_block(N, C, x + b * nn, X + b * nn);
    return 0;
}

/* Batch inverse DCT (eq. 3). */
int or_idct2(int N, int64_t B, const double *X, double *x)
{
    if (N < 1 || N > OR_MAXN || B < 0)
        return -1;
    double C[OR_MAXN * OR_MAXN];
    or_dct_matrix(N, C);
    int64_t nn = (int64_t)N * N;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b)
        idct2_block(N, C, X + b * nn, x + b * nn);
    return 0;
}

/* Batch spatial filter of pixel-domain blocks (eq. 5, Fig. 1). */
int or_filter_spatial(int N, const double *W, int kh, int kw, int border, int64_t B,
                      const double *x, double *f)
{
    if (check_args(N, kh, kw, border) || B < 0)
        return -1;
    int64_t nn = (int64_t)N * N;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b)
        filter_block(N, x + b * nn, W, kh, kw, border, f + b * nn);
    return 0;
}

/* Filtered coefficients from coefficients: Y = DCT(filter(IDCT(X))).
 * This is the map the DCT-domain operator of eq. 11 / eq. 20 applies. */
int or_filter_coeffs(int N, const double *W, int kh, int kw, int border, int64_t B,
                     const double *X, double *Y)
{
    if (check_args(N, kh, kw, border) || B < 0)
        return -1;
    double C[OR_MAXN * OR_MAXN];
    or_dct_matrix(N, C);
    int64_t nn = (int64_t)N * N;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b) {
        double x[OR_MAXN * OR_MAXN], f[OR_MAXN * OR_MAXN];
        idct2_block(N, C, X + b * nn, x);
        filter_block(N, x, W, kh, kw, border, f);
        dct2_block(N, C, f, Y + b * nn);
    }
    return 0;
}

/* Same, evaluated only at selected (block, coefficient) pairs: every listed
 * output is computed on its own from its block, as above. */
int or_filter_coeffs_sampled(int N, const double *W, int kh, int kw, int border,
                             int64_t nsamp, const int64_t *block_idx, const int *coef_idx,
                             const float *X, double *out)
{
    if (check_args(N, kh, kw, border) || nsamp < 0)
        return -1;
    double C[OR_MAXN * OR_MAXN];
    or_dct_matrix(N, C);
    int64_t nn = (int64_t)N * N;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nsamp; ++s) {
        double Xb[OR_MAXN * OR_MAXN], x[OR_MAXN * OR_MAXN], f[OR_MAXN * OR_MAXN];
        double Yb[OR_MAXN * OR_MAXN];
        const float *src = X + block_idx[s] * nn;
        for (int64_t k = 0; k < nn; ++k)
            Xb[k] = (double)src[k];
        idct2_block(N, C, Xb, x);
        filter_block(N, x, W, kh, kw, border, f);
        dct2_block(N, C, f, Yb);
        out[s] = Yb[coef_idx[s]];
    }
    return 0;
}

/* From uint8 pixel blocks: reference coefficients Y = DCT(filter(x)), the
 * uint8 pixels of filter(x) and the near-1/2 flags.  Any output may be NULL. */
int or_filter_pixels(int N, const double *W, int kh, int kw, int border, int64_t B,
                     const uint8_t *px, double *Y, uint8_t *u8, uint8_t *nearhalf)
{
    if (check_args(N, kh, kw, border) || B < 0)
        return -1;
    double C[OR_MAXN * OR_MAXN];
    or_dct_matrix(N, C);
    int64_t nn = (int64_t)N * N;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b) {
        double x[OR_MAXN * OR_MAXN], f[OR_MAXN * OR_MAXN];
        for (int64_t k = 0; k < nn; ++k)
            x[k] = (double)px[b * nn + k];
        filter_block(N, x, W, kh, kw, border, f);
        if (Y)
            dct2_block(N, C, f, Y + b * nn);
        for (int64_t k = 0; k < nn; ++k) {
            if (u8)
                u8[b * nn + k] = to_u8(f[k]);
            if (nearhalf)
                nearhalf[b * nn + k] = (uint8_t)near_half(f[k]);
        }
    }
    return 0;
}

/* uint8 pixels of the inverse DCT of coefficient blocks (eq. 3 then Sec. III). */
int or_idct_u8(int N, int64_t B, const double *Y, uint8_t *u8, uint8_t *nearhalf)
{
    if (N < 1 || N > OR_MAXN || B < 0)
        return -1;
    double C[OR_MAXN * OR_MAXN];
    or_dct_matrix(N, C);
    int64_t nn = (int64_t)N * N;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b) {
        double x[OR_MAXN * OR_MAXN];
        idct2_block(N, C, Y + b * nn, x);
        for (int64_t k = 0; k < nn; ++k) {
            if (u8)
                u8[b * nn + k] = to_u8(x[k]);
            if (nearhalf)
                nearhalf[b * nn + k] = (uint8_t)near_half(x[k]);
        }
    }
    return 0;
}

/* Filtered pixels from coefficients, f = filter(IDCT(X)): the inverse DCT of
 * eq. 3 followed by the block-local filter of eq. 5 / Fig. 1.  This is what
 * the DCT-domain result becomes once it is taken back to the spatial domain
 * and converted to uint8 (Sec. III), and, by the similarity of eq. 7-8,
 * equals IDCT(F) for the filtered coefficients F of eq. 11 / eq. 20.
 * f, u8 and nearhalf may each be NULL. */
int or_filter_coeffs_to_pixels(int N, const double *W, int kh, int kw, int border, int64_t B,
                               const double *X, double *f, uint8_t *u8, uint8_t *nearhalf)
{
    if (check_args(N, kh, kw, border) || B < 0)
        return -1;
    double C[OR_MAXN * OR_MAXN];
    or_dct_matrix(N, C);
    int64_t nn = (int64_t)N * N;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b) {
        double x[OR_MAXN * OR_MAXN], fb[OR_MAXN * OR_MAXN];
        idct2_block(N, C, X + b * nn, x);
        filter_block(N, x, W, kh, kw, border, fb);
        for (int64_t k = 0; k < nn; ++k) {
            if (f)
                f[b * nn + k] = fb[k];
            if (u8)
                u8[b * nn + k] = to_u8(fb[k]);
            if (nearhalf)
                nearhalf[b * nn + k] = (uint8_t)near_half(fb[k]);
        }
    }
    return 0;
}

/* The pixel-output operator probed column by column:
 * G[:, k] = filter(IDCT(e_k)), row index = output pixel i*N+j, column index =
 * input coefficient.  No Kronecker product is formed. */
int or_pixel_operator_probe(int N, const double *W, int kh, int kw, int border, double *G)
{
    if (check_args(N, kh, kw, border))
        return -1;
    double C[OR_MAXN * OR_MAXN];
    or_dct_matrix(N, C);
    int nn = N * N;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nn; ++k) {
        double e[OR_MAXN * OR_MAXN], x[OR_MAXN * OR_MAXN], f[OR_MAXN * OR_MAXN];
        memset(e, 0, sizeof(double) * nn);
        e[k] = 1.0;
        idct2_block(N, C, e, x);
        filter_block(N, x, W, kh, kw, border, f);
        for (int r = 0; r < nn; ++r)
            G[(int64_t)r * nn + k] = f[r];
    }
    return 0;
}

/* The DCT-domain operator probed column by column:
 * H[:, k] = DCT(filter(IDCT(e_k))), row index = output coefficient u*N+v,
 * column index = input coefficient.  No Kronecker product is formed. */
int or_operator_probe(int N, const double *W, int kh, int kw, int border, double *H)
{
    if (check_args(N, kh, kw, border))
        return -1;
    double C[OR_MAXN * OR_MAXN];
    or_dct_matrix(N, C);
    int nn = N * N;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nn; ++k) {
        double e[OR_MAXN * OR_MAXN], x[OR_MAXN * OR_MAXN], f[OR_MAXN * OR_MAXN];
        double Y[OR_MAXN * OR_MAXN];
        memset(e, 0, sizeof(double) * nn);
        e[k] = 1.0;
        idct2_block(N, C, e, x);
        filter_block(N, x, W, kh, kw, border, f);
        dct2_block(N, C, f, Y);
        for (int r = 0; r < nn; ++r)
            H[(int64_t)r * nn + k] = Y[r];
    }
    return 0;
}

/* Image-level filtering of a block-DCT image (the cross-block variant the
 * paper's replication of Fig. 1 stands in for): the Bh x Bw coefficient
 * blocks (raster order) are taken back to one Bh*N x Bw*N pixel image
 * (eq. 3), the mask is correlated over the whole image, reading zeros
 * outside the image (zero padding) or the nearest image pixel
 * (replication), and every block of the result is transformed again
 * (eq. 1).  Blocks now see their neighbours' pixels; only the image border
 * is padded.  nimg images of the same size are stored one after another. */
int or_filter_image_coeffs(int N, const double *W, int kh, int kw, int border, int Bh, int Bw,
                           int nimg, const double *X, double *Y)
{
    if (check_args(N, kh, kw, border) || Bh < 1 || Bw < 1 || nimg < 0)
        return -1;
    double C[OR_MAXN * OR_MAXN];
    or_dct_matrix(N, C);
    const int H = Bh * N, Wd = Bw * N, ah = (kh - 1) / 2, aw = (kw - 1) / 2;
    const int64_t nn = (int64_t)N * N, per = (int64_t)Bh * Bw * nn;
    double *img = (double *)malloc(sizeof(double) * H * Wd);
    double *out = (double *)malloc(sizeof(double) * H * Wd);
    if (!img || !out) {
        free(img);
        free(out);
        return -2;
    }
    for (int im = 0; im < nimg; ++im) {
        const double *Xi = X + im * per;
        double *Yi = Y + im * per;
        /* inverse DCT of every block into the image */
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < (int64_t)Bh * Bw; ++b) {
            double x[OR_MAXN * OR_MAXN];
            idct2_block(N, C, Xi + b * nn, x);
            const int by = (int)(b / Bw), bx = (int)(b % Bw);
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j)
                    img[(int64_t)(by * N + i) * Wd + bx * N + j] = x[i * N + j];
        }
        /* correlation over the image */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < Wd; ++x) {
                double s = 0.0;
                for (int p = 0; p < kh; ++p)
                    for (int q = 0; q < kw; ++q) {
                        int r = y + p - ah, c = x + q - aw;
                        if (border == OR_BORDER_ZERO) {
                            if (r < 0 || r >= H || c < 0 || c >= Wd)
                                continue;
                        } else {
                            r = clamp_index(r, H);
                            c = clamp_index(c, Wd);
                        }
                        s += W[p * kw + q] * img[(int64_t)r * Wd + c];
                    }
                out[(int64_t)y * Wd + x] = s;
            }
        /* forward DCT of every block of the result */
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < (int64_t)Bh * Bw; ++b) {
            double f[OR_MAXN * OR_MAXN];
            const int by = (int)(b / Bw), bx = (int)(b % Bw);
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j)
                    f[i * N + j] = out[(int64_t)(by * N + i) * Wd + bx * N + j];
            dct2_block(N, C, f, Yi + b * nn);
        }
    }
    free(img);
    free(out);
    return 0;
}

/* Cut an h x w uint8 image into N x N blocks in raster (block-row-major)
 * order.  Sides that are not a multiple of N are extended by repeating the
 * last row / column of the image. */
int or_tile_u8(const uint8_t *img, int h, int w, int N, uint8_t *blocks)
{
    if (N < 1 || N > OR_MAXN || h < 1 || w < 1)
        return -1;
    int bh = (h + N - 1) / N, bw = (w + N - 1) / N;
    int64_t nn = (int64_t)N * N;
    for (int by = 0; by < bh; ++by)
        for (int bx = 0; bx < bw; ++bx) {
            uint8_t *dst = blocks + ((int64_t)by * bw + bx) * nn;
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j) {
                    int y = by * N + i, x = bx * N + j;
                    if (y >= h)
                        y = h - 1;
                    if (x >= w)
                        x = w - 1;
                    dst[i * N + j] = img[(int64_t)y * w + x];
                }
        }
    return 0;
}
