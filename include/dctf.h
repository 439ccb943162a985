/*
 * dctf.h — C ABI of the MI355X (gfx950) block-DCT filtering library.
 *
 * Method: Amin-Naji & Aghagolzadeh, "Block DCT filtering using vector
 * processing".  An image stored as N x N blocks of orthonormal DCT-II
 * coefficients (BLOCK = C.block.C^t, Sec. II.A eq. 1-3) is filtered without
 * leaving the DCT domain.  The paper turns a custom mask (eq. 4) into
 * constant DCT-domain matrices once per mask (Sec. II.B) and applies them to
 * every block as matrix products (eq. 8-11 for zero padding, eq. 13-20 for
 * border replication).  This library folds those products into one
 * N^2 x N^2 operator per mask,
 *
 *     H_dct = (C (x) C) . H_sp . (C (x) C)^t
 *           = sum_{p,q} W[p][q] (C S_p C^t) (x) (C S_q C^t),
 *
 * and filters a block by one matrix-vector product Y = H_dct . X of its
 * row-major coefficient vector (vec index u*N + v).  S_d is the block-local
 * row (or column) shift by d = p - a (a = floor((K-1)/2)) with zero fill
 * (Sec. II.B) or with clamping to the block edge (Sec. II.C, Fig. 1).
 *
 * Conventions for every call:
 *   - Blocks are x[i][j], i = row, j = column.  Coefficient blocks are stored
 *     block-contiguous: block b occupies N*N consecutive floats, row-major
 *     (u*N + v), i.e. a column-major N^2 x B matrix.
 *   - Masks are row-major kh x kw doubles and are CORRELATED: W[p][q] weights
 *     the pixel at (i + p - a_h, j + q - a_w).  This is the orientation the
 *     paper's matrices a..e fix (w11 weights block(i-1, j-1), Sec. II.B);
 *     eq. 5 as printed swaps the indices.  Pass a 180-degree rotated mask for
 *     a convolution.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls that take a
 *     stream are asynchronous on it; argument validation happens on the host
 *     before anything is enqueued.  Device faults surface as DCTF_EHIP from a
 *     later call that synchronises.
 *   - Device pointers must be 16-byte aligned.  The library never aborts,
 *     throws or prints; every call returns a dctf_status.
 *   - An operator is read-only once built: it may be used from several
 *     streams and host threads at once (a rebuild must not overlap its use),
 *     and operators may be built concurrently.  Results do not depend on
 *     the stream or on what runs beside the call.
 */
#ifndef DCTF_H
#define DCTF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DCTF_OK = 0,
    DCTF_EINVAL = -1,        /* bad argument (null, misaligned, overlap, range) */
    DCTF_EUNSUPPORTED = -2,  /* N or precision not supported by this build */
    DCTF_ENOMEM = -3,        /* device or host allocation failed */
    DCTF_EHIP = -4,          /* a HIP runtime call failed */
    DCTF_EBUSY = -5,         /* resource budget exhausted (server admission) */
} dctf_status;

typedef enum {
    DCTF_BORDER_ZERO = 0,       /* zero padding at the block edge (Sec. II.B) */
    DCTF_BORDER_REPLICATE = 1,  /* nearest-pixel replication (Sec. II.C, Fig. 1) */
} dctf_border;

typedef enum {
    DCTF_PREC_FP32 = 0,        /* FP32 MFMA, FP32 accumulate */
    DCTF_PREC_SPLIT_BF16 = 1,  /* X and H split into BF16 hi + lo, three BF16 MFMA
                                  products hi.hi + hi.lo + lo.hi, FP32 accumulate */
} dctf_precision;

typedef void *dctf_stream;                 /* hipStream_t */
typedef struct dctf_operator_s *dctf_operator;
typedef struct dctf_batch_s *dctf_batch;

/* Launch configuration of a batch plan (results are bit-identical for every
 * configuration; only the time differs).
 *   fronts        : sweep fronts of the N = 8 work (see dctf_set_batch_fronts);
 *                   -1 = the process-wide fronts setting
 *   io, nt        : N = 8 tile I/O path: 0 registers in the MFMA layout,
 *                   1 coalesced 1 KiB accesses staged through LDS, 2 coalesced
 *                   loads written straight into LDS (buffer loads to LDS);
 *                   nt = 1 adds the nontemporal hint; io = -1 takes the path
 *                   of the current N = 8 variant (dctf_set_variant)
 *   groups_per_cu : persistent workgroups per CU, 1..64; 0 = as many as the
 *                   kernel's registers and LDS allow (more are never used) */
typedef struct {
    int fronts;
    int io;
    int nt;
    int groups_per_cu;
} dctf_batch_config;
typedef struct dctf_image_operator_s *dctf_image_operator;

/* Supported block sizes N: 2, 4, 8, 16, and 32 for the operator build, its
 * FP64 read-back, dctf_filter_blocks, dctf_filter_blocks_f64, the forward
 * DCT and the verify kernel (the other calls return DCTF_EUNSUPPORTED for
 * N = 32).  Mask sides: 1 <= kh, kw <= 2N + 1. */

/* ------------------------------------------------------------------ operators */

/*
 * Build the operator of one mask (Sec. II.B-C: the paper prepares the
 * DCT-domain matrices once per mask and reuses them as constants).
 * The operator is formed on the GPU in FP64: C from its closed form, the
 * shift / clamp factors C S_d C^t, and H_dct as the sum above.  From the FP64
 * operator the build derives, by round-to-nearest-even, the FP32 operator,
 * its BF16 hi/lo split (hi = bf16(fp32(H)), lo = bf16(fp32(H - hi))) and the
 * FP32 DC column H[:, 0], all in the layouts the filter kernels read.
 *   mask_host  kh*kw doubles, row-major, host memory; copied before return.
 *   N          block size (2, 4, 8, 16 or 32).
 *   border     dctf_border.
 *   out        receives a handle owning device memory until destroyed.
 * Errors: DCTF_EINVAL (null, kh/kw out of [1, 2N+1], non-finite entry, bad
 * border), DCTF_EUNSUPPORTED (N), DCTF_ENOMEM, DCTF_EHIP.
 * Asynchronous on `stream`: wait on it before dctf_operator_fp64 reads back.
 */
dctf_status dctf_build_operator(const double *mask_host, int kh, int kw, int N, int border,
                                dctf_stream stream, dctf_operator *out);

/* Mask description for dctf_build_operators. */
typedef struct {
    const double *mask_host; /* kh*kw doubles, row-major */
    int kh, kw, N, border;
} dctf_mask_desc;

/*
 * Build n operators with one builder launch (same result, bit for bit, as n
 * calls of dctf_build_operator).  out[i] receives the i-th handle.  On error
 * no handle is returned.
 */
dctf_status dctf_build_operators(const dctf_mask_desc *masks, int n, dctf_stream stream,
                                 dctf_operator *out);

/*
 * Re-run the builder for existing operators from their device-resident masks
 * (one launch, no host transfer; may be captured in a HIP graph).
 */
dctf_status dctf_rebuild_operators(const dctf_operator *ops, int n, dctf_stream stream);

/* Copy the FP64 operator (N^2 x N^2, row-major, row = output coefficient
 * u*N+v, column = input coefficient) to host memory.  Synchronous. */
dctf_status dctf_operator_fp64(dctf_operator op, double *host_out);

/* Copy the FP64 pixel-domain operator G = (C (x) C)^t . H_dct (N^2 x N^2,
 * row-major, row = output pixel i*N+j, column = input coefficient) to host
 * memory: the filter of eq. 11 / eq. 20 followed by the inverse DCT of
 * eq. 3.  The builder forms it in FP64 with H_dct.  Synchronous. */
dctf_status dctf_operator_pixel_fp64(dctf_operator op, double *host_out);

/* Copy the FP64 pixel-to-pixel operator (C (x) C)^t . H_dct . (C (x) C)
 * (64 x 64, row-major, row = output pixel, column = input pixel) of an
 * N = 8 operator to host memory: the forward DCT of eq. 1, the filter and
 * the inverse DCT of eq. 3 as one matrix.  Since H_dct is the orthogonal
 * similarity of the spatial operator (eq. 7-8), this is the block-local
 * correlation itself; the builder forms it in FP64 from the same Kronecker
 * factors (C^t T_p C = S_p).  Synchronous.  DCTF_EUNSUPPORTED for N != 8. */
dctf_status dctf_operator_pixpix_fp64(dctf_operator op, double *host_out);

/* Block size, mask size and border of an operator (any pointer may be NULL). */
dctf_status dctf_operator_info(dctf_operator op, int *N, int *kh, int *kw, int *border);

/* Free an operator.  The caller must ensure no queued work still uses it. */
void dctf_operator_destroy(dctf_operator op);

/*
 * Factored (paper-form) operator, Sec. II.B-C, eq. 8-12 and eq. 20: the
 * paper applies a mask to a block as a sum of products A . BLOCK . B of N x N
 * DCT-domain matrices.  At build time the mask is decomposed on the host into
 * rank-one terms, W = sum_r a_r b_r^t (complete-pivoting elimination in FP64,
 * terms stop when the remainder is below 1e-14 of the largest entry), and the
 * GPU builder forms, in FP64,
 *   P_r = C (sum_p a_r[p] S_{p-a_h}) C^t,   Q_r = C (sum_q b_r[q] S_{q-a_w}) C^t,
 * with the same shift matrices S_d (zero fill or clamp) as the dense
 * operator, so that H_dct = sum_r P_r (x) Q_r and Y = sum_r P_r X Q_r^t for
 * each N x N coefficient block X.  Separable masks (and 1-D masks) have rank
 * 1; mirror-symmetric masks have rank at most ceil(K/2) (the symmetric
 * shortcut of eq. 12 is this reduction).
 *
 * dctf_operator_rank: the number of terms R (1 <= R <= min(kh, kw)).
 * dctf_operator_factors_fp64: copies P (R x N x N) and Q (R x N x N), each
 *   row-major FP64, to host memory (caller-owned, R*N*N doubles each).
 *   Synchronous.
 */
dctf_status dctf_operator_rank(dctf_operator op, int *rank);
dctf_status dctf_operator_factors_fp64(dctf_operator op, double *P_host, double *Q_host);

/* ------------------------------------------------------------------- filter */

/*
 * Y[b] = H_dct . X[b] for b = 0..B-1 (eq. 11 / eq. 20 for every block at
 * once).  in_dev, out_dev: device, B * N*N floats each, block-contiguous,
 * 16-byte aligned, non-overlapping (in-place is not supported).
 * prec: dctf_precision.  FP32: the MFMA sums over every column but the DC
 * column H[:,0], which is applied in FP32 VALU arithmetic.  Split-BF16: the
 * low-frequency input coefficients (N = 8: (0,0) (0,1) (0,4) (0,5) (1,0)
 * (1,1) (1,4) (1,5), the two FP32 k-steps of the kernel's first load; N = 16:
 * the first 8 in zigzag order; N = 32: the 16 with u, v < 4, DC excluded)
 * are multiplied in FP32 MFMA, the others as BF16 hi.hi + hi.lo + lo.hi;
 * both accumulate in FP32 (N = 32: DC column in FP32 VALU, last).  The
 * split keeps about 16 bits of each operand, so its error grows with the
 * magnitude of the mid- and high-frequency coefficients: the 5e-3 bound
 * holds for natural-image content, not for arbitrary inputs (binary stripe
 * patterns reach ~2e-2).
 * For N <= 4 both precisions run one FP32 kernel (the operator is at most
 * 16 x 16); at N = 32 the 1024 x 1024 operator is streamed from L2 in
 * either precision (FP32: DC column applied in FP32 VALU).
 * B = 0 is a no-op.  Each block's result depends only on that
 * block and the operator: it is bit-identical whatever B, the tuning variant
 * or the batch the block belongs to.
 * Errors: DCTF_EINVAL, DCTF_EUNSUPPORTED, DCTF_EHIP (launch failure).
 */
dctf_status dctf_filter_blocks(dctf_operator op, int prec, const float *in_dev, float *out_dev,
                               int64_t B, dctf_stream stream);

/*
 * Mirror-symmetric masks.  A mask that is mirror-symmetric on both axes
 * (W[i][j] = W[kh-1-i][j] = W[i][kw-1-j], kh and kw odd) filters a block and
 * its mirror images alike (both borders), while the DCT basis vectors are
 * even or odd under a mirror; so H_dct[(u1,v1),(u2,v2)] = 0 unless u1 + u2
 * and v1 + v2 are even (the DCT-domain form of the paper's observation that
 * symmetric masks need fewer products, Sec. II.B-C, eq. 12 and the remark
 * after eq. 20).  H_dct is then four (N^2/4) x (N^2/4) operators, one per
 * parity class (u % 2, v % 2).  At N = 16 and N = 32 the builder forms these
 * four operators (64 x 64 and 256 x 256, in FP64, taken from H_dct) when the
 * mask has the symmetry to 1e-12 of its largest entry (the coupling that
 * such a difference leaves between classes is of the same relative size and
 * is left out).  Class coefficient (a, b), a, b < N/2, is (u, v) =
 * (2a + pu, 2b + pv); a class is then filtered as blocks of side N/2.
 *
 * dctf_operator_parity_classes: 4 when the operator has the class operators
 *   (N = 16 or 32, doubly symmetric mask), else 1.
 * dctf_filter_blocks_parity: Y[b] = H_dct . X[b] as dctf_filter_blocks, through
 *   the four class operators: a quarter of the dense product's MFMA work.
 *   Precisions as for dctf_filter_blocks (split-BF16: the class inputs that
 *   the N/2 dense path keeps in FP32 MFMA, i.e. N = 16: a <= 1 and b in
 *   {0, 1, 4, 5}; N = 32: the first 8 (a, b) in zigzag order; in either case
 *   a superset of the dense path's FP32 set; FP32: each class's first column
 *   in FP32 VALU).  Results agree with dctf_filter_blocks within its
 *   tolerance, not bit for bit (other operands and summation order); each
 *   block's result depends only on the block and the operator.  Buffers as
 *   for dctf_filter_blocks.  Errors: DCTF_EINVAL, DCTF_EUNSUPPORTED (the
 *   operator has no class operators), DCTF_EHIP.
 */
dctf_status dctf_operator_parity_classes(dctf_operator op, int *classes);
dctf_status dctf_filter_blocks_parity(dctf_operator op, int prec, const float *in_dev, float *out_dev, int64_t B,
                                      dctf_stream stream);

/*
 * Y[b] = sum_r P_r X[b] Q_r^t for b = 0..B-1: the factored form above,
 * FP32 MFMA (v_mfma_f32_16x16x4_f32, two chained products per rank term,
 * on 16 x 16 quadrants at N = 32, FP32 accumulation).  It does 2 R N^3
 * multiply-adds per block against the dense path's N^4, so it does less MFMA
 * work for R < N/2 (N = 16: R < 8; N = 32: every R <= 8) and keeps low-rank
 * masks (separable, 1-D, symmetric 3 x 3) at the HBM bound.
 * Results match dctf_filter_blocks(FP32) within FP32 rounding, not bit for
 * bit (different summation order).  Buffers as for dctf_filter_blocks.
 * Errors: DCTF_EINVAL (arguments), DCTF_EUNSUPPORTED (N other than 16 and
 * 32, or R > 8), DCTF_EHIP.
 */
dctf_status dctf_filter_blocks_factored(dctf_operator op, const float *in_dev, float *out_dev, int64_t B,
                                        dctf_stream stream);

/* ------------------------------------------------- filtered pixels (uint8) */

/*
 * Filter, inverse DCT and uint8 conversion in one pass: for every block,
 * P[b] = u8(G . X[b]) with G the pixel-domain operator above, i.e. the
 * filtered coefficients of eq. 11 / eq. 20 taken back to the spatial domain
 * (eq. 3) and converted to uint8 as in Sec. III (round half up, saturate to
 * [0, 255], decided in FP32).  The filtered coefficients are not written.
 *   in_dev   B * N*N FP32 coefficients (device, block-contiguous, 16-byte aligned).
 *   pix_dev  B * N*N bytes out (device, 16-byte aligned; block b at b*N*N,
 *            row-major i*N+j inside the block), not overlapping in_dev.
 *   prec     as for dctf_filter_blocks, applied to G (same low-frequency
 *            FP32 columns in the split path).
 * B = 0 is a no-op.  Errors: DCTF_EINVAL (null, misaligned, overlapping,
 * B < 0, bad prec), DCTF_EHIP (launch failure).
 */
dctf_status dctf_filter_blocks_u8(dctf_operator op, int prec, const float *in_dev, uint8_t *pix_dev,
                                  int64_t B, dctf_stream stream);

/*
 * The same from quantised coefficients, as an entropy-decoded JPEG-style
 * stream holds them (the setting of the paper's introduction: filtering
 * compressed images in the DCT domain).  Each block is dequantised in
 * registers, X[k] = qtable[k] * qcoef[k] (FP32), plus dc_offset on the DC
 * coefficient X[0] (a codec that subtracted 128 from every pixel before its
 * orthonormal DCT passes 128 * N), then filtered, inverse transformed and
 * converted as above.
 *   qcoef_dev   B * N*N int16 coefficients (device, 16-byte aligned).
 *   qtable_dev  N*N FP32 dequantisation factors, row-major (device,
 *               16-byte aligned).
 *   dc_offset   finite.
 * Errors as for dctf_filter_blocks_u8 (qtable_dev must not overlap pix_dev).
 */
dctf_status dctf_filter_quantized_u8(dctf_operator op, int prec, const int16_t *qcoef_dev,
                                     const float *qtable_dev, float dc_offset, uint8_t *pix_dev,
                                     int64_t B, dctf_stream stream);

/*
 * The same two calls with the pixels written in their places in images
 * instead of block by block: the input holds nimg images one after another,
 * each as the ceil(h/N) x ceil(w/N) blocks of an h x w image in raster block
 * order (as dctf_forward_dct_u8 cuts it), and pixel (y, x) of filtered
 * image i goes to img_dev[i * img_stride + y * pitch + x] for y < h, x < w
 * (the pixels of edge blocks past the image are not written).  The
 * filtered coefficients and the block-ordered pixels never reach memory:
 * from a JPEG-style decoder's quantised blocks to the filtered raster
 * images is one pass, one launch for all nimg images.
 *   img_dev     device, 4-byte aligned; pitch >= w, a multiple of 4.
 *   img_stride  bytes from one output image to the next (nimg > 1: a
 *               multiple of 4, >= (h - 1) * pitch + w; ignored for nimg = 1).
 * h, w or nimg = 0 is a no-op.  Errors: DCTF_EINVAL (as above; h, w or nimg
 * < 0, bad pitch or stride, more than 2^31 - 1 blocks per image or 2^32 or
 * more blocks in all (128 bytes of memory per block and more), input
 * overlapping the images), DCTF_EUNSUPPORTED (N = 32), DCTF_EHIP.
 */
dctf_status dctf_filter_blocks_u8_raster(dctf_operator op, int prec, const float *in_dev, int h, int w,
                                         int64_t nimg, uint8_t *img_dev, int64_t pitch, int64_t img_stride,
                                         dctf_stream stream);
dctf_status dctf_filter_quantized_u8_raster(dctf_operator op, int prec, const int16_t *qcoef_dev,
                                            const float *qtable_dev, float dc_offset, int h, int w,
                                            int64_t nimg, uint8_t *img_dev, int64_t pitch, int64_t img_stride,
                                            dctf_stream stream);

/*
 * uint8 images in, filtered uint8 images out, in one pass (N = 8): every
 * 8 x 8 block of each image (cut as dctf_forward_dct_u8 cuts it, ragged
 * sides extended by repeating the last row / column) goes through the
 * pixel-to-pixel operator above, i.e. the forward DCT (eq. 1), the
 * DCT-domain filter (eq. 11 / eq. 20) and the inverse DCT (eq. 3), and is
 * converted to uint8 as in Sec. III (round half up, saturate).  2 bytes of
 * memory traffic per pixel instead of 1 + 4 + 4 + 1 for the separate passes.
 *   in_dev, out_dev   nimg images of h x w pixels, row pitch in_pitch /
 *                     out_pitch bytes (>= w, multiples of 4), in_stride /
 *                     out_stride bytes from one image to the next (nimg > 1:
 *                     multiples of 4, at least (h - 1) * pitch + w); device,
 *                     4-byte aligned, not overlapping.
 *   prec              DCTF_PREC_FP32: the operator in FP32 MFMA (DC column in
 *                     FP32 VALU); DCTF_PREC_SPLIT_BF16: uint8 pixels are
 *                     exact in BF16, so the operator is taken as three BF16
 *                     terms hi + mid + lo (24 bits) against the exact pixels.
 * h, w or nimg = 0 is a no-op.  Errors: DCTF_EINVAL (null, misaligned,
 * overlapping, bad sizes, pitches or strides; more than 2^31 - 1 blocks per
 * image or 2^32 or more in all), DCTF_EUNSUPPORTED (N != 8), DCTF_EHIP.
 */
dctf_status dctf_filter_u8_raster(dctf_operator op, int prec, const uint8_t *in_dev, int64_t in_pitch,
                                  int64_t in_stride, int h, int w, int64_t nimg, uint8_t *out_dev,
                                  int64_t out_pitch, int64_t out_stride, dctf_stream stream);

/* ------------------------------------------------- image-level filtering */

/*
 * Cross-block (image-level) filtering in the DCT domain.  The block-local
 * filter above pads every block on its own (zeros, or the block's own edge
 * pixels, Fig. 1), which is what lets the paper write the result as
 * products of the block with constant matrices (Sec. II.B-C).  Here the
 * image is filtered across block boundaries: a block's result reads the
 * pixels of its 8 neighbour blocks, and the border rule (zero or
 * replication) applies only at the image edge.  The same Kronecker
 * construction (eq. 6-8) with shift matrices that select rows of a
 * neighbour gives one N^2 x N^2 operator per neighbour offset (dr, ds):
 *
 *   Y[R][S] = sum_{dr, ds in {-1, 0, 1}} H^{rc, cc}_{dr, ds} X[R + dr][S + ds],
 *
 * where the row class rc of block row R (and cc of block column S) is
 * 0 = interior, 1 = first, 2 = last, 3 = both (a one-block image side); the
 * class decides which neighbours exist and where reads are clamped.  The
 * builder forms all 16 class pairs x 9 offsets in FP64 on the GPU, with
 * their FP32 and split-BF16 MFMA fragments (N = 8: 4.7 MB FP64 + 2.4 MB
 * FP32 + 2.6 MB split; N = 16: 75.5 MB + 37.7 MB + 39 MB); each operator's
 * DC column is applied in FP32 VALU arithmetic after all other products.
 * Masks: 1 <= kh, kw <= 2N + 1 (a mask never reaches past a neighbour).
 * Errors: as dctf_build_operator; DCTF_EUNSUPPORTED for N other than 8
 * and 16.
 * Synchronises `stream` (the mask copy is from host memory).
 */
dctf_status dctf_build_image_operator(const double *mask_host, int kh, int kw, int N, int border,
                                      dctf_stream stream, dctf_image_operator *out);

/* Copy H^{row_class, col_class}_{dr, ds} (N^2 x N^2 FP64, row-major, row =
 * output coefficient) to host memory.  Synchronous.  Operators of
 * neighbours a class does not have are zero. */
dctf_status dctf_image_operator_fp64(dctf_image_operator op, int row_class, int col_class, int dr, int ds,
                                     double *host_out);

void dctf_image_operator_destroy(dctf_image_operator op);

/*
 * Filter nimg images of Bh x Bw blocks each (block-contiguous, raster
 * order inside an image, images one after another: Bh*Bw*nimg blocks of
 * N*N floats), MFMA with FP32 accumulation; each block's sum runs over
 * the neighbour offsets in a fixed order, so its result does not depend on
 * nimg or on where the block falls in the work partition.
 *   in_dev, out_dev  device, 16-byte aligned, non-overlapping.
 *   prec             DCTF_PREC_FP32, or DCTF_PREC_SPLIT_BF16 (per neighbour
 *                    the split of dctf_filter_blocks at the same N: 8
 *                    low-frequency inputs in FP32 MFMA, the others BF16
 *                    hi.hi + hi.lo + lo.hi).
 * nimg = 0 is a no-op.  Errors: DCTF_EINVAL (null, misaligned, overlap,
 * Bh or Bw < 1, nimg < 0), DCTF_EUNSUPPORTED (N = 16 with Bw > 131072),
 * DCTF_EHIP.
 */
dctf_status dctf_filter_image(dctf_image_operator op, int prec, const float *in_dev, float *out_dev, int Bh,
                              int Bw, int64_t nimg, dctf_stream stream);

/* ------------------------------------------------------------ FP64 filter */

/*
 * Y[b] = H_dct . X[b] in FP64: FP64 coefficients in and out, the FP64
 * operator the builder forms, FP64 arithmetic throughout (N = 8, 16, 32:
 * v_mfma_f64_16x16x4_f64 MFMA, the operator streamed from L2 for N = 16 and
 * 32; N <= 4: FP64 VALU).  For callers whose coefficients are FP64 (no
 * rounding of the data or the operator to FP32); at 16 bytes per
 * coefficient it moves twice the bytes of the FP32 paths.
 *   in_dev, out_dev  B * N*N doubles each (device, block-contiguous,
 *                    16-byte aligned, non-overlapping).
 * B = 0 is a no-op.  Errors: DCTF_EINVAL, DCTF_EHIP.
 */
dctf_status dctf_filter_blocks_f64(dctf_operator op, const double *in_dev, double *out_dev, int64_t B,
                                   dctf_stream stream);

/* ---------------------------------------------------------- batched launch */

/* One filter job: B blocks of in -> out with operator op. */
typedef struct {
    dctf_operator op;
    const float *in;
    float *out;
    int64_t B;
} dctf_job;

/*
 * Plan a batch: many jobs (images), operators (masks) and block sizes (N = 8
 * and N = 16 may be mixed) that run in ONE persistent kernel launch.  The plan
 * copies the job list into a device work table (jobs grouped by operator) and
 * records the distinct operators.  Jobs of the other block sizes (N = 2, 4
 * and 32) run after that launch, on the same stream, one single-operator
 * launch each (the kernels of dctf_filter_blocks: N = 32 in the batch's
 * precision, N <= 4 in FP32); every run, rebuild and captured graph
 * includes them.  Outputs of different jobs must not overlap any input
 * or output of another job.  The plan owns device memory until destroyed;
 * operators must outlive it.
 */
dctf_status dctf_batch_create(const dctf_job *jobs, int njobs, int prec, dctf_batch *out);

/* Flags for dctf_batch_run / dctf_batch_capture. */
#define DCTF_RUN_REBUILD_OPERATORS 1u /* re-run the FP64 builder for the plan's
                                         operators first (one extra launch) */

/* Enqueue the plan on `stream`: [builder launch] + one persistent filter launch. */
dctf_status dctf_batch_run(dctf_batch batch, unsigned flags, dctf_stream stream);

/* Capture dctf_batch_run(batch, flags, stream) into a HIP graph held by the
 * plan (replaces any previous capture).  Nothing is executed. */
dctf_status dctf_batch_capture(dctf_batch batch, unsigned flags, dctf_stream stream);

/* Launch the captured graph on `stream` (DCTF_EINVAL if none was captured). */
dctf_status dctf_batch_launch_graph(dctf_batch batch, dctf_stream stream);

/* Grid shape of the plan's persistent launch (workgroups for N = 8 work,
 * workgroups for N = 16 work, threads per workgroup: 256 when the plan holds
 * only N = 8 jobs, else 512).  Any pointer may be NULL. */
dctf_status dctf_batch_info(dctf_batch batch, int *groups_n8, int *groups_n16, int *threads);

void dctf_batch_destroy(dctf_batch batch);

/* Convenience: create, run and destroy a plan.  Synchronises `stream`. */
dctf_status dctf_filter_batch(const dctf_job *jobs, int njobs, int prec, dctf_stream stream);

/*
 * dctf_filter_batch without any device allocation, for callers that cannot
 * allocate (code that must not call hipMalloc, such as tight serving loops
 * or harnesses that forbid it).  Same jobs, arithmetic and results (bit for
 * bit) as dctf_filter_batch with the process-wide batch configuration; the
 * work table goes into a fixed 1 MiB device array of the library (one per
 * GPU, kept until the process ends; its address on each device is looked up
 * once, at the first call on that device).  1 MiB holds the table of about
 * 8,000 jobs with as many operators (JobDesc 40 B per job, OpDesc 40 B per
 * distinct operator, SegDesc 48 B per front); a larger table returns
 * DCTF_EINVAL and nothing runs.  The host-side plan uses ordinary heap
 * memory.  Synchronous like dctf_filter_batch (returns when the work is
 * done).  Calls that overlap on one GPU (several host threads, or calls made
 * while another is in flight) share the array and race: serialise them.
 */
dctf_status dctf_filter_batch_noalloc(const dctf_job *jobs, int njobs, int prec, dctf_stream stream);

/* One FP64 filter job: B blocks of in -> out with operator op. */
typedef struct {
    dctf_operator op;
    const double *in;
    double *out;
    int64_t B;
} dctf_job_f64;

/*
 * The FP64 filter (dctf_filter_blocks_f64: FP64 coefficients, the FP64
 * operator, FP64 MFMA) over many jobs of any block sizes and operators,
 * enqueued on `stream` as one launch per job in job order (a caller may
 * capture the stream into a graph).  Buffers as for dctf_filter_blocks_f64;
 * outputs must not overlap any input or output of another job.  Jobs with
 * B = 0 are skipped.  Asynchronous.  Errors: DCTF_EINVAL (null, misaligned,
 * overlapping), DCTF_EHIP.
 */
dctf_status dctf_filter_batch_f64(const dctf_job_f64 *jobs, int njobs, dctf_stream stream);

/* --------------------------------------------------------- around the path */

/*
 * Forward DCT of a uint8 image into coefficient blocks (eq. 1), FP64
 * arithmetic rounded once to FP32.  The h x w image (row pitch `pitch` bytes,
 * device memory) is cut into N x N blocks in raster order; sides that are not
 * multiples of N are extended by repeating the last row / column.
 * coeffs_dev receives ceil(h/N)*ceil(w/N) blocks of N*N floats.
 */
dctf_status dctf_forward_dct_u8(const uint8_t *img_dev, int h, int w, int64_t pitch, int N,
                                float *coeffs_dev, dctf_stream stream);

/*
 * The same for nimg images of h x w pixels in one launch (N = 8, 16, 32; one
 * launch per image for the other block sizes): image i starts img_stride
 * bytes after image i - 1 (nimg > 1: img_stride >= (h - 1) * pitch + w), and
 * its blocks follow image i - 1's in coeffs_dev (nimg * ceil(h/N)*ceil(w/N)
 * blocks of N*N floats, the layout the raster calls take).  h, w or nimg = 0
 * is a no-op.  Errors: DCTF_EINVAL (null, misaligned, negative sizes, bad
 * pitch or stride, images overlapping the coefficients), DCTF_EUNSUPPORTED,
 * DCTF_EHIP.
 */
dctf_status dctf_forward_dct_u8_images(const uint8_t *img_dev, int h, int w, int64_t pitch, int64_t img_stride,
                                       int64_t nimg, int N, float *coeffs_dev, dctf_stream stream);

/*
 * Verify kernel: inverse DCT (eq. 3) of each coefficient block in FP32, then
 * the uint8 conversion of Sec. III (round half up, saturate to [0, 255]).
 *   pix_dev      B*N*N bytes out (block-contiguous, row-major inside a block).
 *   expected_dev B*N*N bytes or NULL.
 *   counters_dev two unsigned 64-bit device counters, ADDED to (zero them first):
 *                [0] pixels that differ from expected_dev while their FP32
 *                    value is not within 1e-3 of a .5 boundary,
 *                [1] pixels within 1e-3 of a .5 boundary.
 *                NULL skips counting.
 */
dctf_status dctf_idct_u8_verify(int N, const float *coeffs_dev, int64_t B, uint8_t *pix_dev,
                                const uint8_t *expected_dev, unsigned long long *counters_dev,
                                dctf_stream stream);

/*
 * Measurement aid, not part of the method: a plain streaming copy of n floats
 * (n a multiple of 4, 16-byte aligned, non-overlapping).  Its bandwidth is the
 * achievable-HBM reference for the filter kernels, and its FETCH_SIZE /
 * WRITE_SIZE counter readings calibrate the traffic figures of the others.
 */
dctf_status dctf_stream_copy(const float *in_dev, float *out_dev, int64_t n, dctf_stream stream);

/* ----------------------------------------------------------------- tuning */

/*
 * Kernel variants for (N, precision): a variant fixes the blocks each wave
 * carries per iteration and the persistent grid size (N = 8), or how many
 * tiles of loads run ahead of the MFMA work (N = 16).  Variant 0 is the
 * default.  Every variant computes bit-identical results.  dctf_autotune times each variant on the
 * caller's buffers (in_dev/out_dev, B blocks, operator op) with HIP events
 * (32 warm-up launches, then three passes of `iters` launches per variant,
 * each variant's best pass kept) and selects the fastest for subsequent
 * calls; the choice can be read and set explicitly so that a table persisted
 * by the caller can be re-applied (paper_1710_07193_amd/tuning.py keeps one).
 * N = 8 variants: lds_* stage coalesced loads through LDS in registers,
 * dma_* load them straight into LDS, u<k>_w<w> are registers in the MFMA
 * layout; u = tiles per step, w = waves per CU of the persistent grid,
 * _nt = nontemporal loads and stores.
 */
int dctf_variant_count(int N, int prec);
const char *dctf_variant_name(int N, int prec, int variant);
dctf_status dctf_get_variant(int N, int prec, int *variant);
dctf_status dctf_set_variant(int N, int prec, int variant);
/*
 * Sweep fronts of a batch plan's N = 8 work (read when a plan is created;
 * results are bit-identical for every setting).  The operator-sorted work
 * units are cut at operator boundaries into `fronts` runs of about equal
 * size; the waves of a run stride over it together and reload their operator
 * when they reach the next operator's units.  1 = one front over all units;
 * 0 = one front per operator (each wave loads one operator); -1 = the
 * default of the plan's precision (split-BF16 2, FP32 4), which is also the
 * initial setting (dctf_get_batch_fronts then returns -1).
 * Errors: DCTF_EINVAL outside [-1, 4096].
 */
dctf_status dctf_set_batch_fronts(int fronts);
int dctf_get_batch_fronts(void);

dctf_status dctf_autotune(dctf_operator op, int prec, const float *in_dev, float *out_dev,
                          int64_t B, int iters, dctf_stream stream, int *best_variant,
                          float *best_ms);

/*
 * Batch configuration.  New plans of precision `prec` take the process-wide
 * configuration (initially {-1, -1, 0, 0}); an existing plan can be re-planned
 * with another one (its work table is rebuilt after the device has finished
 * the plan's launches, a captured graph is dropped: capture again).
 * dctf_batch_get_config returns the configuration the plan was made with
 * and/or what it resolved to (I/O path, number of N = 8 fronts actually cut,
 * workgroups per CU of its grid).  Errors: DCTF_EINVAL for a field outside
 * the ranges above.
 */
dctf_status dctf_set_batch_config(int prec, const dctf_batch_config *cfg);
dctf_status dctf_get_batch_config(int prec, dctf_batch_config *cfg);
dctf_status dctf_batch_set_config(dctf_batch batch, const dctf_batch_config *cfg);
dctf_status dctf_batch_get_config(dctf_batch batch, dctf_batch_config *cfg, dctf_batch_config *resolved);

/*
 * Batch autotuner.  Times each candidate configuration on the plan itself
 * (its own jobs and buffers, so the outputs are overwritten with identical
 * results): after 64 warm-up launches of the current plan, `rounds` passes
 * over all candidates, each pass re-planning the batch and timing `iters`
 * launches (flags as dctf_batch_run) after 2 untimed ones with HIP events on
 * `stream`; a candidate's time is its best pass.  The plan is left with the
 * fastest candidate; *best is its index and ms_out[i] (ncand entries, or as
 * many as the built-in list holds) the time per launch of candidate i (-1 if
 * skipped).  candidates = NULL, ncand = 0: the built-in list, which
 * dctf_batch_autotune_candidates copies out (returns its length; max = 0 just
 * counts): every I/O path x fronts {1, 2, 3, 4, 6, 8} x the largest grid or
 * one workgroup per CU fewer (groups_per_cu = -1 in the list; skipped when
 * the largest grid has one workgroup per CU).  Synchronous.
 * Errors: DCTF_EINVAL (bad arguments or candidate), DCTF_EHIP.
 */
dctf_status dctf_batch_autotune(dctf_batch batch, unsigned flags, int iters, int rounds,
                                const dctf_batch_config *candidates, int ncand, dctf_stream stream,
                                float *ms_out, int *best);
int dctf_batch_autotune_candidates(dctf_batch_config *out, int max);

/* ---------------------------------------------------------------- serving */

/*
 * Continuous-batching server (not part of the paper's method: the serving
 * layer around it).  Requests are filter jobs of any size, block size (8 or
 * 16) and mask.  A submitted request waits in a queue; each poll reaps the
 * batches that have finished and admits queued requests, in submission order,
 * once a request's output fits in the server's device arena (the HBM budget)
 * and a launch slot is free.  The requests admitted together form one batch
 * (one persistent launch, operators from a device cache keyed by mask bytes,
 * kh, kw, N and border, LRU eviction); up to max_inflight batches run at once
 * on their own streams, so requests that arrive while others are on the GPU
 * overlap with them.  Each request's result equals, bit for bit, a
 * dctf_filter_blocks call with the same operator and precision.
 *
 * Threading: one server is driven from one host thread at a time (calls on
 * the same server must not overlap); different servers are independent.
 */
typedef struct dctf_server_s *dctf_server;

typedef struct {
    int64_t arena_bytes;   /* device memory for request outputs (>= 256) */
    int max_inflight;      /* batches in flight at once, 1..16 (one stream each) */
    int max_batch_jobs;    /* requests per batch, 1..4096 */
    int max_cached_ops;    /* operator cache entries, >= 1 */
    int prec;              /* dctf_precision */
} dctf_server_config;

typedef struct {
    /* set by the caller */
    double arrival_s;          /* dctf_server_run: arrival time, seconds after the start of the run,
                                  non-decreasing; not read by dctf_server_submit */
    const double *mask_host;   /* kh*kw doubles (host), all finite; copied at submission */
    int kh, kw, N, border;     /* N = 2, 4, 8, 16 or 32; 1 <= kh, kw <= 2N+1 */
    const float *in_dev;       /* B*N*N coefficients, device-resident, 16-byte aligned; must stay
                                  valid and unchanged until the request completes */
    int64_t B;                 /* >= 1 */
    float *out_dev;            /* NULL: the output is written to the arena and dropped at
                                  completion; else also copied here (device, 16-byte aligned)
                                  before the request completes */
    /* set by the server, on its clock (dctf_server_clock; -1 if never reached) */
    double admit_s, launch_s, done_s;
    int status;                /* DCTF_OK; DCTF_EBUSY: the output alone exceeds the arena;
                                  DCTF_ENOMEM / DCTF_EHIP: its operator could not be built, or the
                                  device failed while it was in flight */
    int batch;                 /* index of the launch that carried it, -1 if none */
} dctf_request;

typedef struct {
    int64_t batches, cache_hits, cache_misses, cache_evictions;
    int64_t peak_arena_bytes, peak_inflight_batches, rejected;
    int64_t failed;            /* requests completed with an error other than DCTF_EBUSY */
    double busy_s;             /* wall time spent in dctf_server_run */
} dctf_server_stats;

/* Errors: DCTF_EINVAL (bad config), DCTF_ENOMEM (arena), DCTF_EHIP. */
dctf_status dctf_server_create(const dctf_server_config *cfg, dctf_server *out);

/* Seconds on the server's clock: since creation, or since the start of the
 * last dctf_server_run.  -1 for a NULL server. */
double dctf_server_clock(dctf_server s);

/* Online interface.  Queues one request; nothing is launched until the next
 * poll.  The server keeps `req` (the caller's record: it must stay valid and
 * is written by the server) until a poll returns it.  Returns DCTF_EINVAL for
 * a malformed request (bad N, mask shape or non-finite mask entry, border,
 * NULL or unaligned pointer, B < 1); then nothing is queued. */
dctf_status dctf_server_submit(dctf_server s, dctf_request *req);
/* Makes progress: reaps finished batches, admits and launches queued
 * requests, and returns up to max_done completed requests in `done` (in
 * completion order; *n_done = their count).  If none has completed, it keeps
 * polling for up to wait_s seconds (0: return at once).  Completed requests
 * carry their status; DCTF_EHIP is also returned when the device failed. */
dctf_status dctf_server_poll(dctf_server s, double wait_s, dctf_request **done, int max_done, int *n_done);

/* Replays a request list with known arrival times in real time on the
 * calling thread (submitting each request at its arrival time and polling)
 * until every request has completed.  Returns DCTF_EINVAL for a malformed list
 * (any request invalid as for dctf_server_submit, or arrival times not
 * non-decreasing and >= 0): nothing runs.  DCTF_EBUSY if requests submitted
 * through the online interface are still in the server.  DCTF_EHIP on a
 * device error (requests not yet run then complete with that status). */
dctf_status dctf_server_run(dctf_server s, dctf_request *reqs, int n);
dctf_status dctf_server_stats_get(dctf_server s, dctf_server_stats *out);
/* Waits for the server's streams, then frees everything it owns; requests
 * still queued are dropped. */
void dctf_server_destroy(dctf_server s);

/* ------------------------------------------------------------------ misc */

const char *dctf_status_string(dctf_status s);
const char *dctf_version(void);

/* Kernel-only timing: the average duration (ms) of the last `n` persistent
 * filter launches of dctf_batch_run on this device, measured with HIP events
 * recorded on the launch stream around each launch.  Enable with
 * dctf_timing_enable(1) (events cost a few microseconds per launch). */
dctf_status dctf_timing_enable(int on);
dctf_status dctf_timing_read(double *avg_ms, int *count);

#ifdef __cplusplus
}
#endif

#endif /* DCTF_H */
