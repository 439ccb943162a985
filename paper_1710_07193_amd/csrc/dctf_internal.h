// Internal declarations shared by the HIP sources of libdctf (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/dctf.h"

namespace dctf {

// ---------------------------------------------------------------- operator

// One dense N^2 x N^2 operator (columns = input coefficients) in every form
// the kernels read.
struct DenseImages {
    double *H64;         // N^2 x N^2 row-major, FP64
    float *H32;          // N^2 x N^2 row-major, FP32 (RNE of H64)
    float *frag32;       // FP32 MFMA A-operand fragments (N = 8, 16), DC column zeroed
    uint16_t *frag_hi;   // BF16 hi fragments (N = 8, 16), low-frequency columns zeroed
    uint16_t *frag_lo;   // BF16 lo fragments
    float *frag_lf;      // FP32 A fragments of the low-frequency columns (split path)
    float *h0;           // DC column H[:, 0] in FP32 (N^2 floats)
    uint16_t *frag_lo2;  // pixel-to-pixel set only: third BF16 term (see OpImages::pp)
};

// Device image of one operator, all in a single allocation.
struct OpImages {
    double *mask;        // kh*kw, row-major (device copy of the caller's mask)
    DenseImages dct;     // H_dct: coefficients -> filtered coefficients (row u*N+v)
    DenseImages pix;     // G = (C (x) C)^t H_dct: coefficients -> filtered pixels
                         // (row i*N+j), the filter followed by the inverse DCT
    DenseImages pp;      // N = 8 only: (C (x) C)^t H_dct (C (x) C), pixels -> filtered
                         // pixels (the forward DCT, the filter and the inverse DCT
                         // in one operator); its split images take every column
                         // as three BF16 terms hi + mid + lo (frag_hi, frag_lo,
                         // frag_lo2), since uint8 pixels are exact in BF16
    // Rank factors of the mask, W = sum_r fac_a[r] (outer) fac_b[r], and the
    // matching DCT-domain factors H = sum_r P_r (x) Q_r (paper form F =
    // sum A . BLOCK . B^t): P_r = C (sum_p fac_a[r][p] S_{p-a_h}) C^t over
    // block rows, Q_r likewise over block columns with fac_b[r].
    double *fac_a;       // rank x kh
    double *fac_b;       // rank x kw
    double *P64, *Q64;   // rank x N x N each, row-major, FP64
    float *P32, *Q32;    // FP32 (RNE) copies
};

// Low-frequency input coefficients that the split-BF16 path multiplies in
// FP32 MFMA instead of BF16 (they carry the largest magnitudes of natural
// images, where a two-term BF16 split loses the most absolute precision).
//   N = 8 : the 8 coefficients of the two FP32 k-steps j = 0, 1 of the first
//           load (k = 4g + j, g = 0..3): (0,0) (0,1) (0,4) (0,5) (1,0) (1,1)
//           (1,4) (1,5), slot 2g + j;
//   N = 16: the first 8 in zigzag order: u + v <= 2, then (0, 3), (1, 2).
// Returns the slot of coefficient k (0 .. lf_count(N) - 1), or -1.
__host__ __device__ inline int lf_slot(int N, int k)
{
    if (N == 8)
        return (k < 16 && (k & 3) < 2) ? 2 * (k >> 2) + (k & 3) : -1;
    const int u = k / N, v = k % N, d = u + v;
    if (d <= 2)
        return d * (d + 1) / 2 + u;
    if (d == 3 && u <= 1)
        return 6 + u;
    return -1;
}
__host__ __device__ constexpr int lf_count(int) { return 8; }

// ------------------------------------------- operator fragment layouts
// (written by the builders, read by the MFMA kernels)

// Round an FP32 value to BF16, round-to-nearest-even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t b = __float_as_uint(f);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Position of H[r][c] in the FP32 MFMA fragment layout.
//   N = 8  (v_mfma_f32_16x16x4_f32, whole operator per wave): lane = 16g + m,
//          r = 16t + m, c = 16i + 4g + j -> ((t*4 + i)*64 + lane)*4 + j.
//   N = 16 (weight-stationary, 16 M-tiles over 8 waves): r = 16T + m,
//          c = 16i + 4g + j -> ((T*16 + i)*64 + lane)*4 + j.
//   N = 32 (operator streamed in 16-column chunks): the same with 64 chunks
//          per M-tile, ((T*64 + i)*64 + lane)*4 + j.
__device__ __forceinline__ int frag32_index(int N, int r, int c)
{
    int t = r >> 4, m = r & 15;
    int i = c >> 4, g = (c >> 2) & 3, j = c & 3;
    int lane = 16 * g + m;
    int ni = N * N / 16;   // k-chunks of 16 per M-tile
    return ((t * ni + i) * 64 + lane) * 4 + j;
}

// Position of H[r][c] in the BF16 MFMA fragment layout
// (v_mfma_f32_16x16x32_bf16, 8 BF16 per lane per k-step).
//   N = 8:  c = 16(2s + e) + 4g + j, element 4e + j   -> ((t*2 + s)*64 + lane)*8 + 4e + j.
//   N = 16: c = 32s + 8g + e8, element e8             -> ((T*8 + s)*64 + lane)*8 + e8.
__device__ __forceinline__ int frag16_index(int N, int r, int c)
{
    int t = r >> 4, m = r & 15;
    if (N == 8) {
        int ii = c >> 4, s = ii >> 1, e = ii & 1, g = (c >> 2) & 3, j = c & 3;
        return ((t * 2 + s) * 64 + 16 * g + m) * 8 + 4 * e + j;
    }
    int s = c >> 5, g = (c >> 3) & 3, e8 = c & 7;
    return ((t * 8 + s) * 64 + 16 * g + m) * 8 + e8;
}

}  // namespace dctf

struct dctf_operator_s {
    int N, kh, kw, border;
    int rank;     // terms of the rank factorisation of the mask (>= 1)
    int device;
    void *base;   // owning device allocation
    size_t bytes;
    dctf::OpImages img;
    // N = 16 and 32, masks mirror-symmetric on both axes (odd kh, kw): H_dct
    // couples only coefficients whose row indices and whose column indices
    // have equal parity, so it splits into four (N^2 / 4)-square operators,
    // one per class (pu, pv) of coefficients (u, v) with u % 2 = pu,
    // v % 2 = pv; par[2 pu + pv] holds class (pu, pv) in the fragment images
    // of the N / 2 block size (frag32, h0, frag_hi, frag_lo, frag_lf), class
    // coefficient q = (N / 2) a + b standing for (u, v) = (2a + pu, 2b + pv).
    // parity = 1 when they exist.
    int parity;
    dctf::DenseImages par[4];
};

namespace dctf {

constexpr int kMaxBuildPerLaunch = 16;

struct BuildDesc {
    OpImages img;
    int N, kh, kw, border;
    int rank;
};

// Parts of an operator a builder call forms.
constexpr unsigned kBuildDct = 1u;       // H_dct images (dense filter, batches, server)
constexpr unsigned kBuildPix = 2u;       // pixel-domain images (filter + inverse DCT)
constexpr unsigned kBuildFactors = 4u;   // rank factors P_r, Q_r (factored filter)
constexpr unsigned kBuildPixPix = 8u;    // pixel-to-pixel images (N = 8 one-pass uint8 filter)
constexpr unsigned kBuildParity = 16u;   // parity-class images (N = 16 and 32, symmetric masks), from H_dct
constexpr unsigned kBuildAll = kBuildDct | kBuildPix | kBuildFactors | kBuildPixPix | kBuildParity;

struct BuildArgs {
    BuildDesc d[kMaxBuildPerLaunch];
    int n;
    unsigned parts;   // kBuild* bits
};

// Fragment sizes (elements) per operator.
inline size_t frag_elems(int N) { return (N >= 8) ? (size_t)N * N * N * N : 0; }
inline size_t frag_lf_elems(int N) { return (N >= 8) ? (size_t)N * N * lf_count(N) : 0; }

// builder.hip
hipError_t launch_build(const BuildArgs &args, hipStream_t stream);
// The parity-class images (dctf_operator_s::par) of an N = 16 or 32 operator
// from its FP64 H_dct (N^2 x N^2, row-major).
hipError_t launch_build_parity(int N, const double *H64, const DenseImages *par, hipStream_t stream);

// Rank factorisation of a kh x kw mask (host, FP64): W = sum_r a_r b_r^t with
// a_r (kh values) and b_r (kw values) appended to a and b.  Returns the rank
// (at least 1: a zero mask gives one zero term).
int mask_rank_factors(const double *W, int kh, int kw, std::vector<double> &a, std::vector<double> &b);

// filter.hip — the factored (paper-form) path Y = sum_r P_r X Q_r^t, N = 16
// and 32, FP32, rank <= kFactoredMaxRank; h0 (the DC column of H, N = 32
// only) carries the DC coefficient's term, applied last.
constexpr int kFactoredMaxRank = 8;
hipError_t launch_filter_factored(int N, int rank, const float *P32, const float *Q32, const float *h0,
                                  const float *in, float *out, int64_t B, hipStream_t stream);

// pixels.hip — filter + inverse DCT + uint8 in one pass (pixel-domain images),
// from FP32 coefficients (IN = 0) or from quantised int16 coefficients that
// are dequantised in registers (IN = 1).
// Division of 32-bit block numbers by a launch constant d without a divide:
// M = ceil(2^64 / d) in two 32-bit words (d = 1: M = 0); div_u32 then takes
// the high 64 bits of M * n, which equal n / d for every 32-bit n and d
// (Lemire, Kaser and Kurz, "Faster remainder by direct computation", 2019).
inline void div_magic(uint32_t d, uint32_t *m)
{
    const uint64_t M = d > 1 ? UINT64_MAX / d + 1 : 0;
    m[0] = (uint32_t)M;
    m[1] = (uint32_t)(M >> 32);
}

struct PxArgs {
    const float *in;        // IN = 0: B * N*N FP32 coefficients
    const int16_t *qin;     // IN = 1: B * N*N quantised coefficients
    const float *qtab;      // IN = 1: N*N dequantisation factors (device)
    float dc_offset;        // IN = 1: added to every dequantised DC coefficient
    uint8_t *pix;           // B * N*N filtered pixels (raster = 0), or the h x w image (raster = 1)
    int64_t B;
    DenseImages G;          // the pixel-domain images of the operator
    // raster = 1: the B blocks tile images of h x w pixels in raster order
    // (bpi blocks per image, Bw per block row), images one after another;
    // pixel (y, x) of image i goes to pix[i * img_stride + y * pitch + x]
    // for y < h, x < w
    int raster;
    int h, w, Bw, bpi;
    int64_t pitch, img_stride;
    uint32_t magic[4];      // div_magic of bpi (words 0, 1) and of Bw (words 2, 3); B < 2^32
};
hipError_t launch_filter_px(int N, int prec, int in_kind, const PxArgs &a, hipStream_t stream);
// uint8 raster images in (row pitch in_pitch, in_stride bytes per image) and
// out (a.pix, a.pitch, a.img_stride), N = 8, a.G = the pixel-to-pixel set.
hipError_t launch_filter_u8_raster8(int prec, const PxArgs &a, const uint8_t *in_img, int64_t in_pitch,
                                   int64_t in_stride, hipStream_t stream);

// image.hip — image-level (cross-block) filtering, N = 8.  Operators are
// indexed [class pair cp = 4 cr + cs][offset o = 3 (dr + 1) + (ds + 1)], each
// N^2 x N^2; class bit 0 = first block row / column of the image, bit 1 = last.
constexpr int kImageClassPairs = 16;
constexpr int kImageOffsets = 9;

struct ImageBuildArgs {
    const double *mask;   // kh * kw (device)
    int kh, kw, border;
    double *H64;          // [cp][o] N^2 x N^2, row-major
    float *frag32;        // [cp][o] FP32 MFMA A fragments (layout of the block's N), DC column zeroed
    uint16_t *frag_hi;    // [cp][o] BF16 hi / lo fragments, low-frequency columns zeroed
    uint16_t *frag_lo;
    float *frag_lf;       // [cp][o] FP32 fragments of the low-frequency columns, DC zeroed
    float *h0;            // [cp][o] DC columns H[:, 0], FP32
};

// A rectangle of blocks of one class pair, cut into tiles of up to 16 blocks
// along a block row (dir 0) or, when it is one block wide, a block column
// (dir 1).  `offsets` has bit o set for every neighbour the blocks read.
struct ImageRect {
    int R0, nR, S0, nS;
    int cp, dir, offsets;
    int64_t tiles;        // tiles in the rectangle
    int64_t unit_begin;   // first work unit of the rectangle within its image
};

struct ImageFilterArgs {
    const float *in;
    float *out;
    int Bh, Bw;
    int64_t nimg;
    int nrect;
    ImageRect rect[9];
    int64_t units_per_image;
    const float *frag32;
    const uint16_t *frag_hi;
    const uint16_t *frag_lo;
    const float *frag_lf;
    const float *h0;
};

hipError_t launch_build_image(int N, const ImageBuildArgs &args, hipStream_t stream);
hipError_t launch_filter_image(int N, int prec, const ImageFilterArgs &a, hipStream_t stream);
int image_tiles_per_unit(int N, int prec);
// widest image (blocks) the N = 16 image-level kernel takes
constexpr int kImage16MaxBw = 131072;

// fp64.hip — FP64 filter (N = 8 MFMA, N <= 4 VALU) from the FP64 operator.
hipError_t launch_filter_f64(int N, const double *H64, const double *in, double *out, int64_t B,
                             hipStream_t stream);

// filter.hip — single-operator filter of B blocks.
struct FilterArgs {
    const float *in;
    float *out;
    int64_t B;
    const float *frag32;
    const uint16_t *frag_hi;
    const uint16_t *frag_lo;
    const float *frag_lf;
    const float *h0;
    const float *H32;
};
hipError_t launch_filter(int N, int prec, int variant, const FilterArgs &a, hipStream_t stream);
// The N = 16 / N = 32 filters through the four parity-class operators
// (dctf_operator_s::par).
hipError_t launch_filter_n16_parity(int prec, const DenseImages *par, const float *in, float *out, int64_t B,
                                    hipStream_t stream);
hipError_t launch_filter_n32_parity(int prec, const DenseImages *par, const float *in, float *out, int64_t B,
                                    hipStream_t stream);
// n32.hip — the N = 32 filter, operator streamed from L2: FP32 MFMA (frag32
// and h0 of the DCT-domain images) or split-BF16 (frag_hi / frag_lo in the
// N = 32 layout, frag_lf of n32_lf_elems floats, h0).
hipError_t launch_filter_n32(int prec, const FilterArgs &a, hipStream_t stream);
// The N = 32 split-BF16 images from the FP64 operator (1024 x 1024, row-major).
hipError_t launch_split_n32(const double *H64, uint16_t *hi, uint16_t *lo, float *lf, hipStream_t stream);
constexpr size_t n32_lf_elems = 1024 * 16;
int variant_count(int N, int prec);
const char *variant_name(int N, int prec, int v);
int default_variant(int N, int prec);

// batch.hip — persistent launch over a device work table.
struct JobDesc {
    const float *in;
    float *out;
    int64_t B;
    int64_t unit_begin;   // first work unit of this job within its N class
    int op;               // index into the op table
    int N;
};

struct OpDesc {
    const float *frag32;
    const uint16_t *frag_hi;
    const uint16_t *frag_lo;
    const float *frag_lf;
    const float *h0;
};

// A front: a run of consecutive jobs of one class and the workers that share
// its units: workers [worker_begin, worker_begin + nworkers).
struct SegDesc {
    int64_t unit_begin, unit_end;
    int64_t worker_begin, nworkers;
    int job_begin, job_end;   // [job_begin, job_end) in the class's job table
    int op;                   // operator of the first job
};

struct BatchArgs {
    const JobDesc *jobs8;    // N = 8 jobs, units of kUnitBlocks8 blocks
    const SegDesc *segs8;
    int nsegs8;
    int64_t workers8;        // waves with N = 8 work (<= 8 * groups8)
    const JobDesc *jobs16;   // N = 16 jobs, units of 16 blocks
    const SegDesc *segs16;
    int nsegs16;
    int64_t workers16;       // workgroups with N = 16 work (<= groups16)
    const OpDesc *ops;
    int groups8;             // workgroups [0, groups8) take N = 8 work
    int groups16;            // workgroups [groups8, groups8 + groups16) take N = 16 work
    int prec;
    int io;                  // N = 8 I/O: 0 registers, 1 coalesced through LDS
    bool nt;                 // N = 8: nontemporal global accesses
};

// Sweep fronts for N = 8 batch work (process-wide setting, read at plan creation).
int batch_fronts();
void set_batch_fronts(int fronts);

constexpr int kBatchThreads = 512;    // mixed and N = 16 batch workgroups
constexpr int kBatch8Threads = 256;   // N = 8-only batch workgroups
constexpr int kUnitBlocks8 = 16;    // blocks per N = 8 work unit (one MFMA tile)
constexpr int kUnitBlocks16 = 16;   // blocks per N = 16 work unit
// N = 16 tiles of loads in flight (as the single-operator N = 16 filter: the
// FP32 operator slice leaves room for 2, the split one for 4)
constexpr int batch_depth16(int prec) { return prec == DCTF_PREC_FP32 ? 2 : 4; }

hipError_t launch_batch(const BatchArgs &a, hipStream_t stream);
// Workgroups per CU of the batch kernel for kind 8 (N = 8 only), 16 (N = 16
// only) or 0 (mixed).
int batch_occupancy(int prec, int io, bool nt, int kind);
// Batch planning: validates the jobs, groups them, cuts fronts and sizes the
// grid.  The work table is written to `table`; the pointers in `a` hold
// offsets into it until rebase_batch() adds the table's device address.
// `cfg` fixes the fronts, N = 8 I/O path and grid size (fields < 0 / 0 take
// the process-wide setting of the precision, see dctf_set_batch_config).
dctf_status plan_batch(const dctf_job *jobs, int njobs, int prec, const dctf_batch_config &cfg,
                       std::vector<char> &table, BatchArgs &a, std::vector<dctf_operator> &ops,
                       std::vector<dctf_job> *side);
// The jobs plan_batch set aside (N = 2, 4, 32): one single-operator launch each.
dctf_status launch_side_jobs(const std::vector<dctf_job> &side, int prec, hipStream_t s);
// The process-wide configuration of a precision.
dctf_batch_config batch_config(int prec);
void rebase_batch(BatchArgs &a, const void *dev);

// I/O mode of the current N = 8 variant (used by the batch kernel's N = 8 work).
void variant_io(int N, int prec, int variant, int *io, bool *nt);

// verify.hip
hipError_t launch_idct_u8_verify(int N, const float *Y, int64_t B, uint8_t *pix,
                                 const uint8_t *expected, unsigned long long *counters,
                                 hipStream_t stream);
// nimg images img_stride bytes apart -> their blocks one image after another
hipError_t launch_forward_dct_u8(const uint8_t *img, int h, int w, int64_t pitch, int64_t img_stride,
                                 int64_t nimg, int N, float *coeffs, hipStream_t stream);
hipError_t launch_stream_copy(const float *in, float *out, int64_t n, hipStream_t stream);

// Device properties cached per device.
int cu_count();

// Workgroups of `threads` threads of `kernel` that one CU holds at once (the
// runtime's occupancy for its registers and LDS; at least 1).  Persistent
// grids are sized with it: a workgroup beyond it would start only when
// another ends and run as a tail at low occupancy.
template <typename K>
inline int resident_groups(K kernel, int threads)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1)
        n = 1;
    return n;
}

}  // namespace dctf
