// FP64 filter: Y[b] = H_dct . X[b] with FP64 coefficients and the FP64
// operator the builder forms (eq. 11 / eq. 20 for every block, no rounding
// of the operator or the data to a narrower type).
//
//   N = 8 : k_filter_n8_f64 — v_mfma_f64_16x16x4_f64, the same tiling as the
//           FP32 kernel: one wave holds the whole 64 x 64 operator in VGPRs
//           (64 doubles per lane, read straight from the row-major FP64
//           operator, rows permuted inside each M-tile to match the FP64
//           MFMA's result layout) and computes Y^t = H . X^t for 16 blocks
//           per tile, M = 64 outputs in 4 M-tiles, K = 64 in 16 k-steps; lane
//           (n, g) supplies coefficients 16i + 4g + j of block n and receives
//           outputs 16t + 4g + r, both as 32 contiguous bytes.
//           The blocks move between HBM and the MFMA layout through 8 KiB
//           of wave-private LDS: every load and store instruction covers 1 KiB
//           of contiguous memory (two blocks), where the MFMA layout itself
//           would touch half of every 32-byte span of 16 blocks.
//   N <= 4: k_filter_small_f64 — one thread per block, FP64 VALU.
//   N = 16, 32: k_filter_big_f64 — the operator (256^2 or 1024^2 doubles:
//           512 KiB or 8 MiB) is streamed from L2 as in the FP32 N = 32
//           kernel: a wave owns 4 M-tiles x 2 block tiles and walks K in
//           chunks of 16 coefficients, with the same row permutation inside
//           each M-tile, reading the rows of the FP64 operator directly.
//
// With 8 bytes in and 8 out per coefficient the N = 8 kernel is HBM-bound
// (1 KiB per block against 8192 flop: FP64 MFMA would allow 9.6e9 blocks/s);
// at N = 16 and 32 the FP64 MFMA rate bounds (2 N^4 flop against 16 N^2
// bytes per block: 6.0e8 and 3.7e7 blocks/s at the 78.6 TFLOP/s peak).
#include "mfma_common.h"

namespace dctf {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f64x2 ld2_nt(const double *p)
{
    return __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p));
}

__device__ __forceinline__ void st2_nt(double *p, f64x2 v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<f64x2 *>(p));
}

// LDS image of one 16-block tile: 16 rows of 32 chunks (2 doubles each),
// chunk c of block b at b * 32 + (c ^ b).  A coalesced access of instruction
// k moves blocks 2k and 2k + 1 with lane l at position l of the instruction's
// 64 chunks (global chunk (l % 32) ^ b); an MFMA-layout access of lane (n, g)
// takes one chunk of block n, and the XOR spreads the 16 blocks of a lane
// group over all banks.
__device__ __forceinline__ int f64_pos(int b, int c) { return b * 32 + (c ^ b); }

// Wave w takes tiles (16 blocks) w, w + waves, ...  Two waves per SIMD
// (launch bound): one multiplies while the other waits for its tile.  A
// register double buffer of the next tile would not fit beside the operator
// at that occupancy, and one wave per SIMD with the buffer is slower
// (measured: 0.86 against 0.83 ms for 4,194,304 blocks).
//   IO = 0: blocks loaded and stored in the MFMA layout (0.98 ms);
//   IO = 1: coalesced through LDS.
template <int IO>
__global__ __launch_bounds__(256, 2) void k_filter_n8_f64(const double *H64, const double *in, double *out,
                                                       int64_t B, int64_t tiles, int64_t waves)
{
    __shared__ __attribute__((aligned(16))) f64x2 lds_all[IO ? 4 * 16 * 32 : 1];
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= waves)   // waves <= tiles
        return;
    f64x2 *lds = lds_all + (IO ? (threadIdx.x >> 6) * 16 * 32 : 0);
    // A[t][i][j] = H[16t + s(m)][16i + 4g + j] with m = lane % 16.  The FP64
    // MFMA returns row g + 4r of its 16 x 16 result in register r of lane
    // (n, g); taking A's rows in the order s(m) = 4 (m % 4) + m / 4 makes that
    // row output 16t + 4g + r, so each lane holds four consecutive outputs.
    const int srow = 4 * (n & 3) + (n >> 2);
    double A[4][4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const f64x2 v =
                    *reinterpret_cast<const f64x2 *>(H64 + (16 * t + srow) * 64 + 16 * i + 4 * g + 2 * h);
                A[t][i][2 * h] = v[0];
                A[t][i][2 * h + 1] = v[1];
            }
    // x[k]: IO = 0, chunk 8 (k / 2) + 2g + k % 2 of block n (coefficients
    // 16i + 4g + 2h, 16i + 4g + 2h + 1 with i = k / 2, h = k % 2);
    // IO = 1, position lane of the coalesced instruction k.
    auto load = [&](f64x2 (&x)[8], int64_t tile) {
        if constexpr (IO == 1) {
            const int64_t blk0 = tile * 16;
            const int64_t nv = B - blk0;   // >= 1
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int b = 2 * k + (lane >> 5);
                const int64_t bb = b < nv ? b : nv - 1;   // clamped: its result is never stored
                x[k] = ld2_nt(in + (blk0 + bb) * 64 + 2 * ((lane & 31) ^ b));
            }
        } else {
            int64_t blk = tile * 16 + n;
            blk = blk < B ? blk : B - 1;   // clamped: the store below is masked
            const double *src = in + blk * 64 + 4 * g;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                x[k] = ld2_nt(src + 16 * (k >> 1) + 2 * (k & 1));
        }
    };
    auto compute_store = [&](const f64x2 (&xin)[8], int64_t tile) {
        if constexpr (IO == 1) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                lds[k * 64 + lane] = xin[k];
            wave_lds_sync();
        }
        f64x4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // coefficients 16i + 4g .. 16i + 4g + 3 of block n
            f64x2 x[2];
#pragma unroll
            for (int h = 0; h < 2; ++h)
                x[h] = IO == 1 ? lds[f64_pos(n, 8 * i + 2 * g + h)] : xin[2 * i + h];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[t] = mfma_f64(A[t][i][j], x[j >> 1][j & 1], acc[t]);
        }
        if constexpr (IO == 1) {
            wave_lds_sync();
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                lds[f64_pos(n, 8 * t + 2 * g)] = f64x2{acc[t][0], acc[t][1]};
                lds[f64_pos(n, 8 * t + 2 * g + 1)] = f64x2{acc[t][2], acc[t][3]};
            }
            wave_lds_sync();
            const int64_t blk0 = tile * 16;
            const int64_t nv = B - blk0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int b = 2 * k + (lane >> 5);
                const f64x2 v = lds[k * 64 + lane];
                if (b < nv)
                    st2_nt(out + (blk0 + b) * 64 + 2 * ((lane & 31) ^ b), v);
            }
            wave_lds_sync();
        } else {
            const int64_t blk = tile * 16 + n;
            if (blk < B) {
                double *dst = out + blk * 64 + 4 * g;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    st2_nt(dst + 16 * t, f64x2{acc[t][0], acc[t][1]});
                    st2_nt(dst + 16 * t + 2, f64x2{acc[t][2], acc[t][3]});
                }
            }
        }
    };
    for (int64_t tile = wave; tile < tiles; tile += waves) {
        f64x2 x[8];
        load(x, tile);
        compute_store(x, tile);
    }
}

__global__ __launch_bounds__(256) void k_filter_small_f64(const double *H64, const double *in, double *out,
                                                          int64_t B, int N)
{
    __shared__ double sH[256];
    const int NN = N * N;
    for (int e = threadIdx.x; e < NN * NN; e += blockDim.x)
        sH[e] = H64[e];
    __syncthreads();
    const int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blk >= B)
        return;
    double x[16];
    for (int k = 0; k < NN; ++k)
        x[k] = in[blk * NN + k];
    for (int u = 0; u < NN; ++u) {
        double s = 0.0;
        for (int k = 0; k < NN; ++k)
            s = fma(sH[u * NN + k], x[k], s);
        out[blk * NN + u] = s;
    }
}

// N = 16, 32 (NN = N^2 coefficients per block).  Units: one block group
// (16 NT blocks) x one panel of MT M-tiles, numbered block group first, so
// the waves of a workgroup share a block group (read once through L2) and
// every XCD meets a fixed subset of the panels (N = 32: 4 of 16, 2 MiB).
template <int NN, int MT, int NT>
__global__ __launch_bounds__(256, 2) void k_filter_big_f64(const double *H64, const double *in, double *out,
                                                          int64_t B, int64_t groups, int64_t waves)
{
    constexpr int kPanels = NN / (16 * MT);
    constexpr int kChunks = NN / 16;
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int srow = 4 * (n & 3) + (n >> 2);   // row permutation, as in k_filter_n8_f64
    const int64_t units = groups * kPanels;
    for (int64_t unit = wave; unit < units; unit += waves) {
        const int64_t grp = unit / kPanels;
        const int T0 = (int)(unit % kPanels) * MT;
        int64_t blk[NT];
        const double *xs[NT];
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            blk[s] = grp * (16 * NT) + 16 * s + n;
            const int64_t bb = blk[s] < B ? blk[s] : B - 1;   // clamped: the store is masked
            xs[s] = in + bb * NN + 4 * g;
        }
        const double *ha = H64 + (size_t)(16 * T0 + srow) * NN + 4 * g;
        f64x4 acc[MT][NT];
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int s = 0; s < NT; ++s)
                acc[t][s] = f64x4{0.0, 0.0, 0.0, 0.0};
        // chunk i: A[t] = H[16(T0 + t) + srow][16i + 4g .. + 3], X[s] = coefficients
        // 16i + 4g .. + 3 of block blk[s]
        f64x2 A[MT][2], X[NT][2], An[MT][2], Xn[NT][2];
        auto load = [&](f64x2 (&Ar)[MT][2], f64x2 (&Xr)[NT][2], int i) {
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    Ar[t][h] = *reinterpret_cast<const f64x2 *>(ha + (size_t)16 * t * NN + 16 * i + 2 * h);
#pragma unroll
            for (int s = 0; s < NT; ++s)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    Xr[s][h] = *reinterpret_cast<const f64x2 *>(xs[s] + 16 * i + 2 * h);
        };
        load(A, X, 0);
        for (int i = 0; i < kChunks; ++i) {
            if (i + 1 < kChunks)
                load(An, Xn, i + 1);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int s = 0; s < NT; ++s)
#pragma unroll
                    for (int t = 0; t < MT; ++t)
                        acc[t][s] = mfma_f64(A[t][j >> 1][j & 1], X[s][j >> 1][j & 1], acc[t][s]);
            if (i + 1 < kChunks) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll
                    for (int t = 0; t < MT; ++t)
                        A[t][h] = An[t][h];
#pragma unroll
                    for (int s = 0; s < NT; ++s)
                        X[s][h] = Xn[s][h];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            if (blk[s] < B) {
                double *dst = out + blk[s] * NN + 4 * g;
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    st2_nt(dst + 16 * (T0 + t), f64x2{acc[t][s][0], acc[t][s][1]});
                    st2_nt(dst + 16 * (T0 + t) + 2, f64x2{acc[t][s][2], acc[t][s][3]});
                }
            }
        }
    }
}

constexpr int kF64WavesPerCu = 8;
constexpr int kF64Io = 1;
constexpr int kF64BigMt = 4;
constexpr int kF64BigNt = 2;

template <int NN>
hipError_t launch_big_f64(const double *H64, const double *in, double *out, int64_t B, hipStream_t stream)
{
    const int64_t groups = (B + 16 * kF64BigNt - 1) / (16 * kF64BigNt);
    const int64_t units = groups * (NN / (16 * kF64BigMt));
    int64_t waves = (int64_t)cu_count() * kF64WavesPerCu;
    waves = waves < units ? waves : units;
    const int64_t wgs = (waves + 3) / 4;
    hipLaunchKernelGGL((k_filter_big_f64<NN, kF64BigMt, kF64BigNt>), dim3((unsigned)wgs), dim3(256), 0, stream,
                       H64, in, out, B, groups, waves);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_filter_f64(int N, const double *H64, const double *in, double *out, int64_t B,
                             hipStream_t stream)
{
    if (B <= 0)
        return hipSuccess;
    if (N <= 4) {
        const int64_t groups = (B + 255) / 256;
        hipLaunchKernelGGL(k_filter_small_f64, dim3((unsigned)groups), dim3(256), 0, stream, H64, in, out, B, N);
        return hipGetLastError();
    }
    if (N == 16)
        return launch_big_f64<256>(H64, in, out, B, stream);
    if (N == 32)
        return launch_big_f64<1024>(H64, in, out, B, stream);
    if (N != 8)
        return hipErrorInvalidValue;
    const int64_t tiles = (B + 15) / 16;
    int64_t waves = (int64_t)cu_count() * kF64WavesPerCu;
    waves = waves < tiles ? waves : tiles;
    const int64_t groups = (waves + 3) / 4;
    hipLaunchKernelGGL(k_filter_n8_f64<kF64Io>, dim3((unsigned)groups), dim3(256), 0, stream, H64, in, out, B, tiles,
                       waves);
    return hipGetLastError();
}

}  // namespace dctf
