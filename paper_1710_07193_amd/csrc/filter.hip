// Single-operator filter kernels: Y[b] = H_dct . X[b] for B blocks
// (eq. 11 / eq. 20 applied to every block as one matrix-vector product).
//
//   N = 8  : k_filter_n8   — one wave per 16-block MFMA tile, operator in VGPRs,
//            U tiles per iteration, loads of the next iteration in flight while
//            the current one is multiplied (software pipelining).
//   N = 16 : k_filter_n16  — 8-wave workgroups, operator split over the waves'
//            VGPRs, tiles double-buffered in LDS.
//   N <= 4 : k_filter_small — one thread per block, FP32 VALU.
#include "mfma_common.h"

#include <mutex>

namespace dctf {
namespace {

// ---------------------------------------------------------------- N = 8

// IO = 0: registers in MFMA layout (each load / store instruction covers 64
//         contiguous bytes of 16 blocks);
// IO = 1: coalesced 1 KiB accesses staged through a wave-private LDS region.
// Tiles go through raw buffer instructions over a resource per tile (ragged
// tiles need no clamping or store branches).  Two register buffers alternate
// (the loop body is unrolled twice), so the loads of the next unit stay in
// flight across the loop back-edge instead of being waited for there.
// IO = 2: coalesced loads straight into LDS (two tile buffers per wave),
//         U = 1.
template <int U, int PREC, bool NT, int IO>
__global__ __launch_bounds__(256) void k_filter_n8(FilterArgs a, int64_t units, int64_t waves)
{
    static_assert(IO != 2 || U == 1, "the LDS-load path takes one tile per step");
    __shared__ __attribute__((aligned(16))) float4 lds_all[IO == 1 ? 4 * U * 256 : 1];
    __shared__ __attribute__((aligned(16))) float4 lds_t0[IO == 2 ? 4 : 1][256];
    __shared__ __attribute__((aligned(16))) float4 lds_t1[IO == 2 ? 4 : 1][256];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wave = uniform_i64((int64_t)blockIdx.x * 4 + wid);
    if (wave >= waves)   // waves <= units
        return;
    float4 *lds = lds_all + (IO == 1 ? wid * U * 256 : 0);

    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs8F32, OpRegs8BF16>::type Regs;
    Regs R;
    if constexpr (PREC == DCTF_PREC_FP32)
        load_op8(R, a.frag32, a.h0, lane);
    else
        load_op8(R, a.frag_hi, a.frag_lo, a.frag_lf, lane);

    const int64_t B = a.B;
    // Units are U*16 consecutive blocks; wave w takes units w, w + waves, ...
    const int64_t my_units = (units - wave + waves - 1) / waves;
    uint32_t off[4];
    if constexpr (IO >= 1)
        coalesced_offsets(off, lane);
    else
        mfma_offsets(off, lane);

    auto load_unit = [&](float4 (&x)[U][4], int64_t unit) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            load_tile_buf<NT>(x[u], tile_rsrc8(a.in, unit * (16 * U) + 16 * u, B), off);
    };
    auto compute_store = [&](float4 (&x)[U][4], int64_t unit) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const rsrc_t out = tile_rsrc8(a.out, unit * (16 * U) + 16 * u, B);
            if constexpr (IO == 1)
                tile8_buf<NT>(R, x[u], lds + u * 256, out, off, lane);
            else
                tile8_buf_direct<NT>(R, x[u], out, off, lane);
        }
    };

    if constexpr (IO == 2) {
        // In flight after a tile's loads when the step reading it waits: the
        // 4 stores of the step before (4 dropped stores before the first
        // step) and the 4 loads of the next tile; 4 in the last step, which
        // loads no next tile.
        float4 *t0 = lds_t0[wid], *t1 = lds_t1[wid];
        auto dma_unit = [&](float4 *t, int64_t unit) { dma_tile8<NT>(t, tile_rsrc8(a.in, unit * 16, B), off); };
        auto compute_lds = [&](auto W, float4 *t, int64_t unit) {
            tile8_from_lds<decltype(W)::value, NT>(R, t, tile_rsrc8(a.out, unit * 16, B), off, lane);
        };
        std::integral_constant<int, 8> steady;
        std::integral_constant<int, 4> final;
        int64_t unit = wave;
        dma_unit(t0, unit);
        dummy_stores8<NT>(a.out, off);
        for (int64_t k = 1;; k += 2) {
            if (k >= my_units) {
                compute_lds(final, t0, unit);
                break;
            }
            dma_unit(t1, unit + waves);
            compute_lds(steady, t0, unit);
            unit += waves;
            if (k + 1 >= my_units) {
                compute_lds(final, t1, unit);
                break;
            }
            dma_unit(t0, unit + waves);
            compute_lds(steady, t1, unit);
            unit += waves;
        }
        return;
    }
    float4 b0[U][4], b1[U][4];
    int64_t unit = wave;
    load_unit(b0, unit);
    for (int64_t k = 1;; k += 2) {
        if (k >= my_units) {
            compute_store(b0, unit);
            break;
        }
        load_unit(b1, unit + waves);
        compute_store(b0, unit);
        unit += waves;
        if (k + 1 >= my_units) {
            compute_store(b1, unit);
            break;
        }
        load_unit(b0, unit + waves);
        compute_store(b1, unit);
        unit += waves;
    }
}

// ---------------------------------------------------------------- N = 16

struct Ref16 {
    const float *in;
    float *out;
    int64_t B;
    int64_t blk0;
    int op;
};

// Workgroup w takes tiles w, w + G, w + 2G, ... (G = grid size); loads run D
// tiles ahead.
template <int PREC, int D>
__global__ __launch_bounds__(512) void k_filter_n16(FilterArgs a, int64_t tiles)
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
        Ref16 r;
        r.in = a.in;
        r.out = a.out;
        r.B = a.B;
        r.blk0 = (wg + t * G) * 16;
        r.op = 0;
        return r;
    };
    auto op_load = [&](int) {
        if constexpr (PREC == DCTF_PREC_FP32)
            load_op16(R, a.frag32, a.h0, wave, lane);
        else
            load_op16(R, a.frag_hi, a.frag_lo, a.frag_lf, wave, lane);
    };
    run_tiles16<PREC, D, Ref16>(count, ref, op_load, R, smem);
}

// ---------------------------------------------------------------- N <= 4

__global__ __launch_bounds__(256) void k_filter_small(FilterArgs a, int N)
{
    __shared__ float sH[256];
    const int NN = N * N;
    for (int e = threadIdx.x; e < NN * NN; e += blockDim.x)
        sH[e] = a.H32[e];
    __syncthreads();
    const int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blk >= a.B)
        return;
    float x[16], y[16];
    const float *src = a.in + blk * NN;
    for (int q = 0; q < NN / 4; ++q) {
        float4 v = ld4(src + 4 * q);
        x[4 * q] = v.x;
        x[4 * q + 1] = v.y;
        x[4 * q + 2] = v.z;
        x[4 * q + 3] = v.w;
    }
    for (int u = 0; u < NN; ++u) {
        float s = 0.0f;
        for (int k = 0; k < NN; ++k)
            s = fmaf(sH[u * NN + k], x[k], s);
        y[u] = s;
    }
    float *dst = a.out + blk * NN;
    for (int q = 0; q < NN / 4; ++q)
        *reinterpret_cast<float4 *>(dst + 4 * q) = make_float4(y[4 * q], y[4 * q + 1], y[4 * q + 2], y[4 * q + 3]);
}

// ------------------------------------------------------------- variants

struct Variant8 {
    int U;
    bool nt;
    int io;             // 0: registers, 1: coalesced through LDS, 2: loaded straight into LDS
    int waves_per_cu;   // persistent grid: CUs * waves_per_cu waves
    const char *name;
};

// One tile per wave step throughout: with two or four tiles per step the
// register allocation of the ping-pong loop gave wrong results once the
// loop ran (GPU tests on inputs long enough for several steps per wave), and
// those shapes had measured slower than one tile per step before.
const Variant8 kVariants8[] = {
    {1, true, 1, 8, "lds_u1_w8_nt"},
    {1, false, 0, 8, "u1_w8"},
    {1, false, 0, 16, "u1_w16"},
    {1, true, 1, 12, "lds_u1_w12_nt"},
    {1, false, 1, 8, "lds_u1_w8"},
    {1, true, 2, 8, "dma_u1_w8_nt"},
    {1, true, 2, 12, "dma_u1_w12_nt"},
    {1, false, 2, 8, "dma_u1_w8"},
};
constexpr int kNumVariants8 = sizeof(kVariants8) / sizeof(kVariants8[0]);

template <int U, int PREC, bool NT, int IO>
hipError_t run8(const FilterArgs &a, int waves_per_cu, hipStream_t stream)
{
    const int64_t units = (a.B + 16 * U - 1) / (16 * U);
    int64_t waves = (int64_t)cu_count() * waves_per_cu;
    waves = waves < units ? waves : units;
    const int64_t groups = (waves + 3) / 4;
    hipLaunchKernelGGL((k_filter_n8<U, PREC, NT, IO>), dim3((unsigned)groups), dim3(256), 0, stream, a,
                       units, waves);
    return hipGetLastError();
}

template <int U, int PREC>
hipError_t dispatch8u(const Variant8 &v, const FilterArgs &a, hipStream_t stream)
{
    if constexpr (U == 1)
        if (v.io == 2)
            return v.nt ? run8<1, PREC, true, 2>(a, v.waves_per_cu, stream) : run8<1, PREC, false, 2>(a, v.waves_per_cu, stream);
    if (v.io)
        return v.nt ? run8<U, PREC, true, 1>(a, v.waves_per_cu, stream) : run8<U, PREC, false, 1>(a, v.waves_per_cu, stream);
    return v.nt ? run8<U, PREC, true, 0>(a, v.waves_per_cu, stream) : run8<U, PREC, false, 0>(a, v.waves_per_cu, stream);
}

template <int PREC>
hipError_t dispatch8(const Variant8 &v, const FilterArgs &a, hipStream_t stream)
{
    return dispatch8u<1, PREC>(v, a, stream);
}

template <int PREC, int D>
hipError_t run16(const FilterArgs &a, hipStream_t stream)
{
    const int64_t tiles = (a.B + 15) / 16;
    int64_t groups = (int64_t)cu_count();
    groups = groups < tiles ? groups : tiles;
    hipLaunchKernelGGL((k_filter_n16<PREC, D>), dim3((unsigned)groups), dim3(512), 0, stream, a, tiles);
    return hipGetLastError();
}

struct Variant16 {
    int depth;   // tiles of global loads in flight ahead of the MFMA work
    const char *name;
};
// The FP32 kernel keeps the whole FP32 operator slice in registers; three
// tiles in flight push it past the register file, so its table stops at two.
// Split (1,036,800 blocks of the N = 16 frames): 4 tiles ahead 0.49 ms, 5:
// 0.49, 3: 0.52, 2: 0.59, 1: 0.62; 6 spills (0.78).  One workgroup per CU
// keeps 16 KiB per tile in flight, so the depth sets the bytes in flight.
const Variant16 kVariants16Split[] = {{4, "wg8_ahead4"}, {5, "wg8_ahead5"}, {3, "wg8_ahead3"}, {2, "wg8_ahead2"},
                                      {1, "wg8_ahead1"}};
const Variant16 kVariants16F32[] = {{2, "wg8_ahead2"}, {1, "wg8_ahead1"}};
constexpr int kNumVariants16Split = sizeof(kVariants16Split) / sizeof(kVariants16Split[0]);
constexpr int kNumVariants16F32 = sizeof(kVariants16F32) / sizeof(kVariants16F32[0]);

const Variant16 &variant16(int prec, int variant)
{
    if (prec == DCTF_PREC_FP32)
        return kVariants16F32[(variant >= 0 && variant < kNumVariants16F32) ? variant : 0];
    return kVariants16Split[(variant >= 0 && variant < kNumVariants16Split) ? variant : 0];
}

hipError_t dispatch16_f32(int variant, const FilterArgs &a, hipStream_t stream)
{
    switch (variant16(DCTF_PREC_FP32, variant).depth) {
    case 1: return run16<DCTF_PREC_FP32, 1>(a, stream);
    default: return run16<DCTF_PREC_FP32, 2>(a, stream);
    }
}

hipError_t dispatch16_split(int variant, const FilterArgs &a, hipStream_t stream)
{
    switch (variant16(DCTF_PREC_SPLIT_BF16, variant).depth) {
    case 1: return run16<DCTF_PREC_SPLIT_BF16, 1>(a, stream);
    case 2: return run16<DCTF_PREC_SPLIT_BF16, 2>(a, stream);
    case 3: return run16<DCTF_PREC_SPLIT_BF16, 3>(a, stream);
    case 4: return run16<DCTF_PREC_SPLIT_BF16, 4>(a, stream);
    default: return run16<DCTF_PREC_SPLIT_BF16, 5>(a, stream);
    }
}

// -------------------------------------- N = 16, mirror-symmetric masks
//
// A mask that is mirror-symmetric on both axes (odd kh and kw) filters a
// block and its mirror images alike, and the DCT basis vectors are even or
// odd under a mirror: H_dct couples coefficient (u, v) only with those whose
// row and column indices have the same parities (the DCT-domain form of the
// paper's remark that symmetric masks need fewer products, Sec. II.B-C).  The
// operator is then four 64 x 64 operators, one per parity class (pu, pv): a
// quarter of the dense 256 x 256 product.
//
// A workgroup of four waves takes 16-block tiles; wave c = 2 pu + pv
// multiplies class (pu, pv) of each block with the N = 8 tile code (its
// operator in VGPRs, N = 8 fragment layout, class coefficient q = 8a + b for
// (u, v) = (2a + pu, 2b + pv)).  The tile passes through LDS in class order:
// every global load and store instruction covers 4 KiB of the tile
// (thread t holds float4 k 256 + t: block 4k + t / 64, row (t / 4) % 16,
// columns 4 (t % 4) .. +3, i.e. two coefficients of class (u % 2, 0) and two
// of class (u % 2, 1)), written to and gathered from LDS as 8-byte pairs.
// In LDS, class c of block n is 16 chunks of 16 bytes (class coefficients
// 4 ch .. 4 ch + 3 in chunk ch), chunk ch stored at slot ch ^ n, so that the
// 16-byte reads of a wave (lane (n, g) takes chunk 4i + g of block n, i.e.
// class coefficients 16i + 4g .. +3 as the N = 8 tile code wants them) fall
// in different banks.  Each wave writes its outputs over its own inputs (no
// other wave touches that class), then the workgroup gathers the natural
// order back for the stores.  The next tile's loads are in flight while the
// current one is multiplied; a ragged tail goes through raw buffer
// instructions over the tile's valid blocks (zeros in, stores dropped).
struct ParArgs {
    const float *in;
    float *out;
    int64_t B;
    DenseImages par[4];
};

__device__ __forceinline__ int par_slot(int cls, int n, int ch) { return (cls * 16 + n) * 16 + (ch ^ n); }

template <int PREC>
__global__ __launch_bounds__(256, 2) void k_filter_n16_par(ParArgs a, int64_t tiles, int64_t groups)
{
    __shared__ __attribute__((aligned(16))) float4 lds[4 * 16 * 16];   // [class][block][chunk slot], 16 KiB
    const int tid = threadIdx.x, lane = tid & 63;
    const int cls = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t wg = blockIdx.x;
    if (wg >= tiles)
        return;
    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs8F32, OpRegs8BF16>::type Regs;
    Regs R;
    const DenseImages &P = a.par[cls];
    if constexpr (PREC == DCTF_PREC_FP32)
        load_op8(R, P.frag32, P.h0, lane);
    else
        load_op8(R, P.frag_hi, P.frag_lo, P.frag_lf, lane);
    const int n = lane & 15, g = lane >> 4;
    // loader role: float4 k of thread tid is block 4k + tid / 64, row u, columns v0 .. v0 + 3
    const int u = (tid >> 2) & 15, pu = u & 1, ch = 2 * (u >> 1) + ((tid & 3) >> 1), half = tid & 1;
    const int64_t my_tiles = (tiles - wg + groups - 1) / groups;
    const int64_t last = wg + (my_tiles - 1) * groups;
    float2 *lds2 = reinterpret_cast<float2 *>(lds);
    float4 gl[4];
    auto load = [&](int64_t t) {
        const rsrc_t r = tile_rsrc(a.in, t * 16, a.B, 1024);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            gl[k] = buf_ld4<true>(r, (uint32_t)(k * 256 + tid) * 16u);
    };
    int64_t tile = wg;
    load(tile);
    for (int64_t it = 0; it < my_tiles; ++it) {
        __syncthreads();   // the previous tile's gathers are done
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int nb = 4 * k + (tid >> 6);
            lds2[2 * par_slot(2 * pu, nb, ch) + half] = make_float2(gl[k].x, gl[k].z);
            lds2[2 * par_slot(2 * pu + 1, nb, ch) + half] = make_float2(gl[k].y, gl[k].w);
        }
        const int64_t nt = tile + groups;
        load(nt < last ? nt : last);   // the last step loads its own tile again: every step loads
        __syncthreads();
        float4 x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            x[i] = lds[par_slot(cls, n, 4 * i + g)];
        f32x4 acc[4];
        tile8(R, x, lane, acc);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            lds[par_slot(cls, n, 4 * t + g)] = make_float4(acc[t][0], acc[t][1], acc[t][2], acc[t][3]);
        __syncthreads();
        const rsrc_t o = tile_rsrc(a.out, tile * 16, a.B, 1024);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int nb = 4 * k + (tid >> 6);
            const float2 e = lds2[2 * par_slot(2 * pu, nb, ch) + half];
            const float2 f = lds2[2 * par_slot(2 * pu + 1, nb, ch) + half];
            buf_st4<true>(o, (uint32_t)(k * 256 + tid) * 16u, f32x4{e.x, f.x, e.y, f.y});
        }
        tile += groups;
    }
}

// -------------------------------------- N = 32, mirror-symmetric masks
//
// The same parity classes at N = 32: four 256 x 256 operators, the size of
// an N = 16 operator, so each class runs through the N = 16 weight-stationary
// tile loop (8 waves holding the class operator in VGPRs) with a loader that
// gathers the class's 256 coefficients of each of a tile's 16 blocks (four
// 32-bit loads per class chunk of four, every other float of a block row; the
// workgroup of the other column parity reads the floats in between, from the
// same cache lines) and stores that write the results back to their places
// (32-bit stores, the other half of each row written by that workgroup).  Workgroup w takes class (w / 8) % 4 and, within it, the place
// (w / 32) 8 + w % 8: the four classes of a tile are on the same XCD (its
// L2 serves the rows the four read) and next to each other in launch order.
// FP32: 32-bit class loads, two tiles ahead; split-BF16 (more operator
// registers): float4 loads of whole 32-byte row pieces, one tile ahead,
// written to LDS after the tile's MFMA work rather than halfway through it
// (a whole tile's work for the loads to land in).
constexpr int kPar32In[2] = {2, 3};
constexpr int kPar32Depth[2] = {2, 1};
constexpr bool kPar32Late[2] = {false, true};
struct RefPar32 {
    const float *in;
    float *out;
    int64_t B;
    int64_t blk0;
    int op;
    int cls;
};

template <int PREC>
__global__ __launch_bounds__(512) void k_filter_n32_par(ParArgs a, int64_t tiles, int64_t per_class)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int w = blockIdx.x;
    const int cls = (w >> 3) & 3;
    const int64_t wg = (int64_t)(w >> 5) * 8 + (w & 7), G = per_class;
    if (wg >= tiles)
        return;
    // the two tile buffers, then 2 KiB per wave for the results on their way out
    __shared__ __attribute__((aligned(16))) char smem[(PREC == DCTF_PREC_FP32 ? kSmem16F32 : kSmem16Split) + 8 * 2048];
    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs16F32, OpRegs16BF16>::type Regs;
    Regs R;
    const int64_t count = (tiles - wg + G - 1) / G;
    auto ref = [&](int64_t t) {
        RefPar32 r;
        r.in = a.in;
        r.out = a.out;
        r.B = a.B;
        r.blk0 = (wg + t * G) * 16;
        r.op = 0;
        r.cls = cls;
        return r;
    };
    const DenseImages &P = a.par[cls];
    auto op_load = [&](int) {
        if constexpr (PREC == DCTF_PREC_FP32)
            load_op16(R, P.frag32, P.h0, wave, lane);
        else
            load_op16(R, P.frag_hi, P.frag_lo, P.frag_lf, wave, lane);
    };
    run_tiles16<PREC, kPar32Depth[PREC], RefPar32, kPar32In[PREC], 3, false, kPar32Late[PREC]>(count, ref, op_load, R,
                                                                                            smem);
}

// ------------------------------------------------- N = 16, factored form
//
// Y = sum_r P_r X Q_r^t per block (the paper's A . BLOCK . B products with
// the mask rows merged into rank terms), FP32 MFMA v_mfma_f32_16x16x4_f32.
// Lane (n, g) of a wave loads X[n][4g..4g+3] (one 16-byte load per lane
// covers the 1 KiB block) and the same slices of P_r and Q_r.  With the
// contraction index of k-step s taken as 4g + s on both operands:
//   stage 1: Z_r = X Q_r^t   (A = X, B = Q_r^t), D: lane (j, g) holds Z_r[4g + i][j];
//   stage 2: Y^t += Z_r^t P_r^t (A = Z_r^t read straight from stage 1's D
//            registers, B = P_r^t), D: lane (u, g) holds Y[u][4g + i],
// which is the load layout again, so the store is one 16-byte access per
// lane.  Each wave carries U blocks per iteration (independent MFMA chains)
// and has the next U blocks' loads in flight.
template <int R, int U>
__global__ __launch_bounds__(256) void k_filter_factored16(const float *in, float *out, int64_t B,
                                                           const float *P32, const float *Q32, int64_t waves)
{
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= waves)
        return;
    const int off = n * 16 + 4 * g;
    float4 P[R], Q[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        P[r] = ld4(P32 + r * 256 + off);
        Q[r] = ld4(Q32 + r * 256 + off);
    }
    const int64_t units = (B + U - 1) / U;
    const int64_t my_units = (units - wave + waves - 1) / waves;
    auto load = [&](float4 (&x)[U], int64_t unit) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t b = unit * U + u;
            b = b < B ? b : B - 1;   // clamped: the store is skipped
            x[u] = ld4_nt(in + b * 256 + off);
        }
    };
    auto compute_store = [&](const float4 (&x)[U], int64_t unit) {
        f32x4 y[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            y[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float q[4] = {Q[r].x, Q[r].y, Q[r].z, Q[r].w};
            const float p[4] = {P[r].x, P[r].y, P[r].z, P[r].w};
            f32x4 z[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float xv[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
                z[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    z[u] = mfma_f32(xv[k], q[k], z[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    y[u] = mfma_f32(z[u][k], p[k], y[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t b = unit * U + u;
            if (b < B)
                st4_nt(out + b * 256 + off, y[u]);
        }
    };
    float4 cur[U], nxt[U];
    int64_t unit = wave;
    load(cur, unit);
    for (int64_t k = 1; k < my_units; ++k) {
        load(nxt, unit + waves);
        compute_store(cur, unit);
#pragma unroll
        for (int u = 0; u < U; ++u)
            cur[u] = nxt[u];
        unit += waves;
    }
    compute_store(cur, unit);
}

template <int R>
hipError_t run_factored16(const float *P32, const float *Q32, const float *in, float *out, int64_t B,
                          hipStream_t stream)
{
    constexpr int U = 4;
    const int64_t units = (B + U - 1) / U;
    static const int per_cu = resident_groups(k_filter_factored16<R, U>, 256);
    int64_t waves = (int64_t)cu_count() * per_cu * 4;
    waves = waves < units ? waves : units;
    const int64_t groups = (waves + 3) / 4;
    hipLaunchKernelGGL((k_filter_factored16<R, U>), dim3((unsigned)groups), dim3(256), 0, stream, in, out, B,
                       P32, Q32, waves);
    return hipGetLastError();
}

// ------------------------------------------------- N = 32, factored form
//
// The same two chained products on 16 x 16 quadrants: block X (32 x 32) is
// X[a][b] with a = 16 alpha + a', b = 16 beta + b'; lane (n, g) holds
// X[16 alpha + n][16 beta + 4g .. +3] of every quadrant (four 16-byte loads
// cover the 4 KiB block).  For each rank term,
//   stage 1: Z[alpha][gamma] = sum_beta X[alpha][beta] Q[gamma][beta]^t
//            (8 MFMAs per quadrant, contraction index 16 beta + 4g + k),
//            D: lane (n, g) holds Z[16 alpha + 4g + i][16 gamma + n];
//   stage 2: Y^t[gamma][delta] += sum_alpha Z[alpha][gamma]^t P[delta][alpha]^t
//            (A read straight from stage 1's D registers),
//            D: lane (n, g) holds Y[16 delta + n][16 gamma + 4g + i],
// the load layout of quadrant (delta, gamma).  The DC coefficient X[0][0]
// (the block's largest, up to 4096 for uint8 pixels) is taken out of the
// products and applied last in FP32 VALU with the operator's DC column
// H[:, 0] (Y += X[0][0] H[:, 0]), as the dense FP32 path does: in the MFMA
// chains it would set the rounding step of every other term.  The factors (R terms of two
// 32 x 32 FP32 matrices, up to 64 KiB) are staged in LDS once per
// workgroup with rows padded to 36 floats, which keeps the 16 rows a wave
// reads at once on distinct banks.
constexpr int kFac32Ld = 36;

template <int R, int U>
__global__ __launch_bounds__(256) void k_filter_factored32(const float *in, float *out, int64_t B,
                                                           const float *P32, const float *Q32, const float *h0,
                                                           int64_t waves)
{
    __shared__ __attribute__((aligned(16))) float sP[R * 32 * kFac32Ld];
    __shared__ __attribute__((aligned(16))) float sQ[R * 32 * kFac32Ld];
    for (int e = threadIdx.x; e < R * 32 * 8; e += blockDim.x) {   // 16-byte chunks
        const int r = e / 256, row = (e / 8) % 32, c4 = e % 8;
        *reinterpret_cast<float4 *>(sP + (r * 32 + row) * kFac32Ld + 4 * c4) = ld4(P32 + r * 1024 + row * 32 + 4 * c4);
        *reinterpret_cast<float4 *>(sQ + (r * 32 + row) * kFac32Ld + 4 * c4) = ld4(Q32 + r * 1024 + row * 32 + 4 * c4);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= waves)
        return;
    // offset of the lane's piece of quadrant (a, b) in a block / in a factor
    auto blk_off = [&](int a, int b) { return (16 * a + n) * 32 + 16 * b + 4 * g; };
    auto fac_off = [&](int r, int a, int b) { return (r * 32 + 16 * a + n) * kFac32Ld + 16 * b + 4 * g; };
    // the lane's pieces of the DC column, as quadrants [gamma][delta] of Y
    float4 hd[2][2];
#pragma unroll
    for (int ga = 0; ga < 2; ++ga)
#pragma unroll
        for (int de = 0; de < 2; ++de)
            hd[ga][de] = ld4(h0 + blk_off(de, ga));
    const int64_t units = (B + U - 1) / U;
    const int64_t my_units = (units - wave + waves - 1) / waves;
    auto load = [&](float4 (&x)[U][2][2], int64_t unit) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t b = unit * U + u;
            b = b < B ? b : B - 1;   // clamped: the store is skipped
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    x[u][a][c] = ld4_nt(in + b * 1024 + blk_off(a, c));
        }
    };
    auto compute_store = [&](const float4 (&x)[U][2][2], int64_t unit) {
        // The factor reads are the same for every unit; an opaque zero offset
        // keeps the compiler from hoisting them out of the loop (all R terms
        // would then stay in VGPRs and cut the waves per SIMD).
        int fbase = 0;
        asm volatile("" : "+s"(fbase));
        f32x4 y[U][2][2];   // [gamma][delta]
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    y[u][a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float4 q[2][2], p[2][2];   // q[gamma][beta], p[delta][alpha]
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    q[a][c] = *reinterpret_cast<const float4 *>(sQ + fbase + fac_off(r, a, c));
                    p[a][c] = *reinterpret_cast<const float4 *>(sP + fbase + fac_off(r, a, c));
                }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                f32x4 z[2][2];   // [alpha][gamma]
#pragma unroll
                for (int al = 0; al < 2; ++al)
#pragma unroll
                    for (int ga = 0; ga < 2; ++ga) {
                        z[al][ga] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int be = 0; be < 2; ++be) {
                            // lane 0 holds X[0][0] in quadrant (0, 0): it enters as zero
                            const float x0 = (al == 0 && be == 0 && lane == 0) ? 0.0f : x[u][al][be].x;
                            const float xv[4] = {x0, x[u][al][be].y, x[u][al][be].z, x[u][al][be].w};
                            const float qv[4] = {q[ga][be].x, q[ga][be].y, q[ga][be].z, q[ga][be].w};
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                z[al][ga] = mfma_f32(xv[k], qv[k], z[al][ga]);
                        }
                    }
#pragma unroll
                for (int ga = 0; ga < 2; ++ga)
#pragma unroll
                    for (int de = 0; de < 2; ++de)
#pragma unroll
                        for (int al = 0; al < 2; ++al) {
                            const float pv[4] = {p[de][al].x, p[de][al].y, p[de][al].z, p[de][al].w};
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                y[u][ga][de] = mfma_f32(z[al][ga][k], pv[k], y[u][ga][de]);
                        }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // X[0][0] of the block, held by lane 0
            const float x00 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x[u][0][0].x)));
#pragma unroll
            for (int ga = 0; ga < 2; ++ga)
#pragma unroll
                for (int de = 0; de < 2; ++de) {
                    y[u][ga][de][0] = fmaf(hd[ga][de].x, x00, y[u][ga][de][0]);
                    y[u][ga][de][1] = fmaf(hd[ga][de].y, x00, y[u][ga][de][1]);
                    y[u][ga][de][2] = fmaf(hd[ga][de].z, x00, y[u][ga][de][2]);
                    y[u][ga][de][3] = fmaf(hd[ga][de].w, x00, y[u][ga][de][3]);
                }
            const int64_t b = unit * U + u;
            if (b < B)
#pragma unroll
                for (int ga = 0; ga < 2; ++ga)
#pragma unroll
                    for (int de = 0; de < 2; ++de)
                        st4_nt(out + b * 1024 + blk_off(de, ga), y[u][ga][de]);
        }
    };
    float4 cur[U][2][2], nxt[U][2][2];
    int64_t unit = wave;
    load(cur, unit);
    for (int64_t k = 1; k < my_units; ++k) {
        load(nxt, unit + waves);
        compute_store(cur, unit);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    cur[u][a][c] = nxt[u][a][c];
        unit += waves;
    }
    compute_store(cur, unit);
}

template <int R>
hipError_t run_factored32(const float *P32, const float *Q32, const float *h0, const float *in, float *out,
                          int64_t B, hipStream_t stream)
{
    constexpr int U = 2;
    const int64_t units = (B + U - 1) / U;
    static const int per_cu = resident_groups(k_filter_factored32<R, U>, 256);
    int64_t waves = (int64_t)cu_count() * per_cu * 4;
    waves = waves < units ? waves : units;
    const int64_t groups = (waves + 3) / 4;
    hipLaunchKernelGGL((k_filter_factored32<R, U>), dim3((unsigned)groups), dim3(256), 0, stream, in, out, B,
                       P32, Q32, h0, waves);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_filter_factored(int N, int rank, const float *P32, const float *Q32, const float *h0,
                                  const float *in, float *out, int64_t B, hipStream_t stream)
{
    if (B <= 0)
        return hipSuccess;
    if ((N != 16 && N != 32) || rank < 1 || rank > kFactoredMaxRank)
        return hipErrorInvalidValue;
    if (N == 32) {
        switch (rank) {
        case 1: return run_factored32<1>(P32, Q32, h0, in, out, B, stream);
        case 2: return run_factored32<2>(P32, Q32, h0, in, out, B, stream);
        case 3: return run_factored32<3>(P32, Q32, h0, in, out, B, stream);
        case 4: return run_factored32<4>(P32, Q32, h0, in, out, B, stream);
        case 5: return run_factored32<5>(P32, Q32, h0, in, out, B, stream);
        case 6: return run_factored32<6>(P32, Q32, h0, in, out, B, stream);
        case 7: return run_factored32<7>(P32, Q32, h0, in, out, B, stream);
        default: return run_factored32<8>(P32, Q32, h0, in, out, B, stream);
        }
    }
    switch (rank) {
    case 1: return run_factored16<1>(P32, Q32, in, out, B, stream);
    case 2: return run_factored16<2>(P32, Q32, in, out, B, stream);
    case 3: return run_factored16<3>(P32, Q32, in, out, B, stream);
    case 4: return run_factored16<4>(P32, Q32, in, out, B, stream);
    case 5: return run_factored16<5>(P32, Q32, in, out, B, stream);
    case 6: return run_factored16<6>(P32, Q32, in, out, B, stream);
    case 7: return run_factored16<7>(P32, Q32, in, out, B, stream);
    default: return run_factored16<8>(P32, Q32, in, out, B, stream);
    }
}

int variant_count(int N, int prec)
{
    if (N == 8)
        return kNumVariants8;
    if (N == 16)
        return prec == DCTF_PREC_FP32 ? kNumVariants16F32 : kNumVariants16Split;
    return 1;
}

const char *variant_name(int N, int prec, int v)
{
    if (N == 8 && v >= 0 && v < kNumVariants8)
        return kVariants8[v].name;
    if (N == 16 && v >= 0 && v < variant_count(16, prec))
        return variant16(prec, v).name;
    if (N <= 4 && v == 0)
        return "valu";
    return nullptr;
}

void variant_io(int N, int prec, int variant, int *io, bool *nt)
{
    (void)prec;
    *io = 0;
    *nt = false;
    if (N == 8 && variant >= 0 && variant < kNumVariants8) {
        *io = kVariants8[variant].io;
        *nt = kVariants8[variant].nt;
    }
}

int default_variant(int N, int prec)
{
    (void)N;
    (void)prec;
    return 0;
}

hipError_t launch_filter_n16_parity(int prec, const DenseImages *par, const float *in, float *out, int64_t B,
                                    hipStream_t stream)
{
    if (B <= 0)
        return hipSuccess;
    ParArgs a;
    a.in = in;
    a.out = out;
    a.B = B;
    for (int c = 0; c < 4; ++c)
        a.par[c] = par[c];
    const int64_t tiles = (B + 15) / 16;
    // two 4-wave workgroups per CU (three or four measured 7-10 % slower,
    // split-BF16)
    const int64_t want = (int64_t)cu_count() * 2;
    const int64_t groups = tiles < want ? tiles : want;
    if (prec == DCTF_PREC_FP32)
        hipLaunchKernelGGL(k_filter_n16_par<DCTF_PREC_FP32>, dim3((unsigned)groups), dim3(256), 0, stream, a, tiles,
                           groups);
    else
        hipLaunchKernelGGL(k_filter_n16_par<DCTF_PREC_SPLIT_BF16>, dim3((unsigned)groups), dim3(256), 0, stream, a,
                           tiles, groups);
    return hipGetLastError();
}

hipError_t launch_filter_n32_parity(int prec, const DenseImages *par, const float *in, float *out, int64_t B,
                                    hipStream_t stream)
{
    if (B <= 0)
        return hipSuccess;
    ParArgs a;
    a.in = in;
    a.out = out;
    a.B = B;
    for (int c = 0; c < 4; ++c)
        a.par[c] = par[c];
    const int64_t tiles = (B + 15) / 16;
    // one 8-wave workgroup per CU, a quarter of them per class, in groups of 8
    int64_t per_class = ((int64_t)cu_count() / 4 + 7) / 8 * 8;
    const int64_t need = (tiles + 7) / 8 * 8;
    per_class = per_class < need ? per_class : need;
    const unsigned grid = (unsigned)(4 * per_class);
    if (prec == DCTF_PREC_FP32)
        hipLaunchKernelGGL((k_filter_n32_par<DCTF_PREC_FP32>), dim3(grid), dim3(512), 0, stream, a, tiles,
                           per_class);
    else
        hipLaunchKernelGGL((k_filter_n32_par<DCTF_PREC_SPLIT_BF16>), dim3(grid), dim3(512), 0, stream,
                           a, tiles, per_class);
    return hipGetLastError();
}

hipError_t launch_filter(int N, int prec, int variant, const FilterArgs &a, hipStream_t stream)
{
    if (a.B <= 0)
        return hipSuccess;
    if (N <= 4) {
        const int64_t groups = (a.B + 255) / 256;
        hipLaunchKernelGGL(k_filter_small, dim3((unsigned)groups), dim3(256), 0, stream, a, N);
        return hipGetLastError();
    }
    if (N == 8) {
        const Variant8 &v = kVariants8[(variant >= 0 && variant < kNumVariants8) ? variant : 0];
        return prec == DCTF_PREC_FP32 ? dispatch8<DCTF_PREC_FP32>(v, a, stream)
                                      : dispatch8<DCTF_PREC_SPLIT_BF16>(v, a, stream);
    }
    return prec == DCTF_PREC_FP32 ? dispatch16_f32(variant, a, stream) : dispatch16_split(variant, a, stream);
}

}  // namespace dctf
