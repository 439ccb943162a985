// Filter + inverse DCT + uint8 in one pass: P[b] = u8(G . X[b]), where
// G = (C (x) C)^t H_dct is the pixel-domain operator the builder forms in
// FP64 next to H_dct (the DCT-domain filter of eq. 11 / eq. 20 followed by
// the inverse DCT of eq. 3, then the uint8 conversion of Sec. III).  The
// filtered coefficients never reach HBM: 4 bytes in and 1 byte out per
// coefficient instead of 4 + 4 for the filter and 4 + 1 for a separate
// inverse transform.
//
// Inputs: FP32 coefficient blocks (IN = 0), or quantised int16 coefficient
// blocks (IN = 1, the entropy-decoded blocks of a JPEG-style codec) that are
// dequantised in registers, X[k] = q[k] c[k] (+ dc_offset on the DC term):
// 2 bytes in and 1 byte out per coefficient.
//
//   N = 8  : k_filter_px8  — one wave per 16-block tile, G in VGPRs (the
//            layout of the DCT-domain kernel), tiles staged through a
//            wave-private LDS region so that every global access of the
//            wave covers contiguous memory.
//   N = 16 : k_filter_px16 — the weight-stationary 8-wave tile loop of the
//            DCT-domain kernel with the int16 loader / uint8 store.
//   N <= 4 : k_filter_px_small — one thread per block, FP32 VALU.
#include "mfma_common.h"

namespace dctf {
namespace {

// ---------------------------------------------------------------- N = 8

// Tile input held in registers while the previous tile is multiplied.
template <int IN>
struct In8;

template <>
struct In8<0> {
    float4 x[4];   // the coalesced layout of load_tile_coalesced
};

template <>
struct In8<1> {
    u32x4 raw[2];  // 2 KiB tile: lane l, load i holds coefficients 8(l % 8) .. +7 of block 8i + l / 8
};

__device__ __forceinline__ void load8(In8<0> &t, const PxArgs &a, int64_t blk0, int lane)
{
    const int64_t nv = a.B - blk0;
    load_tile_coalesced<true>(t.x, a.in + blk0 * 64, nv, lane);
}

__device__ __forceinline__ void load8(In8<1> &t, const PxArgs &a, int64_t blk0, int lane)
{
    const int64_t nv = a.B - blk0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int64_t b = 8 * i + (lane >> 3);
        const int64_t bb = b < nv ? b : nv - 1;   // clamped: its pixels are never stored
        t.raw[i] = __builtin_nontemporal_load(
            reinterpret_cast<const u32x4 *>(a.qin + (blk0 + bb) * 64 + 8 * (lane & 7)));
    }
}

// Write the tile to the wave's LDS region in the swizzled layout read_mfma
// expects (chunk c of block b at slot 16 b + (c ^ b)).
__device__ __forceinline__ void stage8(const In8<0> &t, float4 *lds, int lane, const float *, float)
{
    stage_in(lds, t.x, lane);
}

__device__ __forceinline__ void stage8(const In8<1> &t, float4 *lds, int lane, const float *qv, float dc)
{
    const int c8 = lane & 7;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int b = 8 * i + (lane >> 3);
        float4 lo, hi;
        dequant8(t.raw[i], qv, dc, lo, hi);
        lds[b * 16 + ((2 * c8) ^ b)] = lo;
        lds[b * 16 + ((2 * c8 + 1) ^ b)] = hi;
    }
}

// Pixels of the tile from the LDS staging (floats, swizzled): lane l writes
// the 16 pixels 16(l % 4) .. +15 of block l / 4, one 16-byte store, so the
// wave's store covers the tile's 1 KiB contiguously.
__device__ __forceinline__ void store_px8(uint8_t *pix, int64_t nvalid, const float4 *lds, int lane)
{
    const int b = lane >> 2, k4 = lane & 3;
    if (b >= nvalid)
        return;
    u32x4 w;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const float4 v = lds[b * 16 + ((4 * k4 + m) ^ b)];
        w[m] = pack_u8x4(v.x, v.y, v.z, v.w);
    }
    __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(pix + (int64_t)b * 64 + 16 * k4));
}

// Wave w takes 16-block tiles w, w + waves, ...; the next tile's loads are in
// flight while the current one is multiplied.
template <int PREC, int IN>
__global__ __launch_bounds__(256) void k_filter_px8(PxArgs a, int64_t units, int64_t waves)
{
    __shared__ __attribute__((aligned(16))) float4 lds_all[4 * 256];
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= waves)   // waves <= units
        return;
    float4 *lds = lds_all + (threadIdx.x >> 6) * 256;

    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs8F32, OpRegs8BF16>::type Regs;
    Regs R;
    if constexpr (PREC == DCTF_PREC_FP32)
        load_op8(R, a.G.frag32, a.G.h0, lane);
    else
        load_op8(R, a.G.frag_hi, a.G.frag_lo, a.G.frag_lf, lane);

    float qv[8];
    float dc = 0.0f;
    if constexpr (IN == 1) {
        const float4 q0 = ld4(a.qtab + 8 * (lane & 7)), q1 = ld4(a.qtab + 8 * (lane & 7) + 4);
        qv[0] = q0.x; qv[1] = q0.y; qv[2] = q0.z; qv[3] = q0.w;
        qv[4] = q1.x; qv[5] = q1.y; qv[6] = q1.z; qv[7] = q1.w;
        dc = (lane & 7) == 0 ? a.dc_offset : 0.0f;
    }

    const int64_t my_units = (units - wave + waves - 1) / waves;
    auto compute_store = [&](const In8<IN> &t, int64_t unit) {
        const int64_t blk0 = unit * 16;
        stage8(t, lds, lane, qv, dc);
        wave_lds_sync();
        float4 xm[4];
        read_mfma(lds, xm, lane);
        f32x4 acc[4];
        tile8(R, xm, lane, acc);
        wave_lds_sync();
        stage_out(lds, acc, lane);
        wave_lds_sync();
        store_px8(a.pix + blk0 * 64, a.B - blk0, lds, lane);
        wave_lds_sync();
    };

    In8<IN> cur, nxt;
    int64_t unit = wave;
    load8(cur, a, unit * 16, lane);
    for (int64_t k = 1; k < my_units; ++k) {
        load8(nxt, a, (unit + waves) * 16, lane);
        compute_store(cur, unit);
        cur = nxt;
        unit += waves;
    }
    compute_store(cur, unit);
}

// ---------------------------------------------------------------- N = 16

struct RefPx16 {
    const float *in;
    const int16_t *qin;
    uint8_t *pix;
    int64_t B;
    int64_t blk0;
    int op;
};

template <int PREC, int IN, int D>
__global__ __launch_bounds__(512) void k_filter_px16(PxArgs a, int64_t tiles)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t wg = blockIdx.x, G = gridDim.x;
    if (wg >= tiles)
        return;
    __shared__ __attribute__((aligned(16))) char smem[PREC == DCTF_PREC_FP32 ? kSmem16F32 : kSmem16Split];
    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs16F32, OpRegs16BF16>::type Regs;
    Regs R;
    const int64_t count = (tiles - wg + G - 1) / G;
    auto ref = [&](int64_t t) {
        RefPx16 r;
        r.in = a.in;
        r.qin = a.qin;
        r.pix = a.pix;
        r.B = a.B;
        r.blk0 = (wg + t * G) * 16;
        r.op = 0;
        return r;
    };
    auto op_load = [&](int) {
        if constexpr (PREC == DCTF_PREC_FP32)
            load_op16(R, a.G.frag32, a.G.h0, wave, lane);
        else
            load_op16(R, a.G.frag_hi, a.G.frag_lo, a.G.frag_lf, wave, lane);
    };
    run_tiles16<PREC, D, RefPx16, IN, 1>(count, ref, op_load, R, smem, a.qtab, a.dc_offset);
}

// ---------------------------------------------------------------- N <= 4

template <int IN>
__global__ __launch_bounds__(256) void k_filter_px_small(PxArgs a, int N)
{
    __shared__ float sG[256];
    const int NN = N * N;
    for (int e = threadIdx.x; e < NN * NN; e += blockDim.x)
        sG[e] = a.G.H32[e];
    __syncthreads();
    const int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blk >= a.B)
        return;
    float x[16];
    for (int k = 0; k < NN; ++k) {
        if constexpr (IN == 0)
            x[k] = a.in[blk * NN + k];
        else
            x[k] = (float)a.qin[blk * NN + k] * a.qtab[k] + (k == 0 ? a.dc_offset : 0.0f);
    }
    for (int r = 0; r < NN; ++r) {
        float s = 0.0f;
        for (int k = 0; k < NN; ++k)
            s = fmaf(sG[r * NN + k], x[k], s);
        a.pix[blk * NN + r] = (uint8_t)pixel_u8(s);
    }
}

// ------------------------------------------------------------- launches

constexpr int kPx8WavesPerCu = 8;
constexpr int kPx16Depth = 2;

template <int PREC, int IN>
hipError_t run_px8(const PxArgs &a, hipStream_t stream)
{
    const int64_t units = (a.B + 15) / 16;
    int64_t waves = (int64_t)cu_count() * kPx8WavesPerCu;
    waves = waves < units ? waves : units;
    const int64_t groups = (waves + 3) / 4;
    hipLaunchKernelGGL((k_filter_px8<PREC, IN>), dim3((unsigned)groups), dim3(256), 0, stream, a, units, waves);
    return hipGetLastError();
}

template <int PREC, int IN>
hipError_t run_px16(const PxArgs &a, hipStream_t stream)
{
    const int64_t tiles = (a.B + 15) / 16;
    int64_t groups = (int64_t)cu_count();
    groups = groups < tiles ? groups : tiles;
    hipLaunchKernelGGL((k_filter_px16<PREC, IN, kPx16Depth>), dim3((unsigned)groups), dim3(512), 0, stream, a,
                       tiles);
    return hipGetLastError();
}

template <int PREC>
hipError_t dispatch_px(int N, int in_kind, const PxArgs &a, hipStream_t stream)
{
    if (N == 8)
        return in_kind ? run_px8<PREC, 1>(a, stream) : run_px8<PREC, 0>(a, stream);
    return in_kind ? run_px16<PREC, 1>(a, stream) : run_px16<PREC, 0>(a, stream);
}

}  // namespace

hipError_t launch_filter_px(int N, int prec, int in_kind, const PxArgs &a, hipStream_t stream)
{
    if (a.B <= 0)
        return hipSuccess;
    if (N <= 4) {
        const int64_t groups = (a.B + 255) / 256;
        if (in_kind)
            hipLaunchKernelGGL(k_filter_px_small<1>, dim3((unsigned)groups), dim3(256), 0, stream, a, N);
        else
            hipLaunchKernelGGL(k_filter_px_small<0>, dim3((unsigned)groups), dim3(256), 0, stream, a, N);
        return hipGetLastError();
    }
    return prec == DCTF_PREC_FP32 ? dispatch_px<DCTF_PREC_FP32>(N, in_kind, a, stream)
                                  : dispatch_px<DCTF_PREC_SPLIT_BF16>(N, in_kind, a, stream);
}

}  // namespace dctf
