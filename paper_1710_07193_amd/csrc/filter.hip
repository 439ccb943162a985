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

template <int U, int PREC, bool NT>
__global__ __launch_bounds__(256) void k_filter_n8(FilterArgs a, int64_t units, int64_t waves)
{
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= waves)   // waves <= units
        return;

    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs8F32, OpRegs8BF16>::type Regs;
    Regs R;
    if constexpr (PREC == DCTF_PREC_FP32)
        load_op8(R, a.frag32, a.h0, lane);
    else
        load_op8(R, a.frag_hi, a.frag_lo, a.frag_lf, lane);

    const int64_t B = a.B;
    // Units are U*16 consecutive blocks; wave w takes units w, w + waves, ...
    const int64_t my_units = (units - wave + waves - 1) / waves;

    auto load_unit = [&](float4 (&x)[U][4], int64_t unit) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t blk = unit * (16 * U) + 16 * u + n;
            blk = blk < B ? blk : B - 1;   // clamped: the store below is masked
            const float *src = a.in + blk * 64 + 4 * g;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                x[u][i] = NT ? ld4_nt(src + 16 * i) : ld4(src + 16 * i);
        }
    };
    auto compute_store = [&](float4 (&x)[U][4], int64_t unit) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            f32x4 acc[4];
            tile8(R, x[u], lane, acc);
            const int64_t blk = unit * (16 * U) + 16 * u + n;
            if (blk < B) {
                float *dst = a.out + blk * 64 + 4 * g;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (NT)
                        st4_nt(dst + 16 * t, acc[t]);
                    else
                        st4(dst + 16 * t, acc[t]);
                }
            }
        }
    };

    float4 cur[U][4], nxt[U][4];
    int64_t unit = wave;
    load_unit(cur, unit);
    for (int64_t k = 1; k < my_units; ++k) {
        load_unit(nxt, unit + waves);
        compute_store(cur, unit);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                cur[u][i] = nxt[u][i];
        unit += waves;
    }
    compute_store(cur, unit);
}

// ---------------------------------------------------------------- N = 16

template <int PREC>
__global__ __launch_bounds__(512) void k_filter_n16(FilterArgs a, int64_t tiles)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int64_t B = a.B;
    if ((int64_t)blockIdx.x >= tiles)
        return;

    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs16F32, OpRegs16BF16>::type Regs;
    Regs R;
    if constexpr (PREC == DCTF_PREC_FP32)
        load_op16(R, a.frag32, a.h0, wave, lane);
    else
        load_op16(R, a.frag_hi, a.frag_lo, a.frag_lf, wave, lane);

    constexpr int kF32 = 16 * kLd16F32;           // floats per FP32 buffer
    constexpr int kB16 = 16 * kLd16BF16;          // BF16 per hi (or lo) buffer
    __shared__ __attribute__((aligned(16))) char smem[PREC == DCTF_PREC_FP32 ? 2 * kTile16BytesF32
                                                                             : 2 * kTile16BytesSplit];
    float *lf = reinterpret_cast<float *>(smem);
    uint16_t *lhi = reinterpret_cast<uint16_t *>(smem);
    uint16_t *llo = lhi + 2 * kB16;
    float *llf = reinterpret_cast<float *>(llo + 2 * kB16);

    const int64_t step = gridDim.x;
    int64_t tile = blockIdx.x;
    Stage16 S;
    stage16_load(S, a.in, B, tile, tid);
    if constexpr (PREC == DCTF_PREC_FP32)
        stage16_store(S, lf, tid);
    else
        stage16_store(S, lhi, llo, llf, tid);
    __syncthreads();

    int buf = 0;
    for (;;) {
        const int64_t next = tile + step;
        const bool more = next < tiles;
        if (more)
            stage16_load(S, a.in, B, next, tid);
        f32x4 acc[2];
        if constexpr (PREC == DCTF_PREC_FP32)
            tile16(R, lf + buf * kF32, lane, acc);
        else
            tile16(R, lhi + buf * kB16, llo + buf * kB16, llf + buf * 16 * kLd16Lf, lane, acc);
        const int64_t blk = tile * 16 + n;
        if (blk < B) {
            float *dst = a.out + blk * 256 + 32 * wave + 4 * g;
            st4(dst, acc[0]);
            st4(dst + 16, acc[1]);
        }
        if (!more)
            break;
        if constexpr (PREC == DCTF_PREC_FP32)
            stage16_store(S, lf + (buf ^ 1) * kF32, tid);
        else
            stage16_store(S, lhi + (buf ^ 1) * kB16, llo + (buf ^ 1) * kB16, llf + (buf ^ 1) * 16 * kLd16Lf, tid);
        __syncthreads();
        buf ^= 1;
        tile = next;
    }
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
    int waves_per_cu;   // persistent grid: CUs * waves_per_cu waves
    const char *name;
};

const Variant8 kVariants8[] = {
    {2, false, 8, "u2_w8"},
    {1, false, 8, "u1_w8"},
    {4, false, 4, "u4_w4"},
    {2, true, 8, "u2_w8_nt"},
    {1, false, 16, "u1_w16"},
    {2, false, 16, "u2_w16"},
    {4, true, 4, "u4_w4_nt"},
};
constexpr int kNumVariants8 = sizeof(kVariants8) / sizeof(kVariants8[0]);

template <int U, int PREC, bool NT>
hipError_t run8(const FilterArgs &a, int waves_per_cu, hipStream_t stream)
{
    const int64_t units = (a.B + 16 * U - 1) / (16 * U);
    int64_t waves = (int64_t)cu_count() * waves_per_cu;
    waves = waves < units ? waves : units;
    const int64_t groups = (waves + 3) / 4;
    hipLaunchKernelGGL((k_filter_n8<U, PREC, NT>), dim3((unsigned)groups), dim3(256), 0, stream, a,
                       units, waves);
    return hipGetLastError();
}

template <int PREC>
hipError_t dispatch8(const Variant8 &v, const FilterArgs &a, hipStream_t stream)
{
    if (v.U == 1)
        return v.nt ? run8<1, PREC, true>(a, v.waves_per_cu, stream) : run8<1, PREC, false>(a, v.waves_per_cu, stream);
    if (v.U == 2)
        return v.nt ? run8<2, PREC, true>(a, v.waves_per_cu, stream) : run8<2, PREC, false>(a, v.waves_per_cu, stream);
    return v.nt ? run8<4, PREC, true>(a, v.waves_per_cu, stream) : run8<4, PREC, false>(a, v.waves_per_cu, stream);
}

template <int PREC>
hipError_t run16(const FilterArgs &a, int groups_per_cu, hipStream_t stream)
{
    const int64_t tiles = (a.B + 15) / 16;
    int64_t groups = (int64_t)cu_count() * groups_per_cu;
    groups = groups < tiles ? groups : tiles;
    hipLaunchKernelGGL((k_filter_n16<PREC>), dim3((unsigned)groups), dim3(512), 0, stream, a, tiles);
    return hipGetLastError();
}

}  // namespace

int variant_count(int N, int prec)
{
    (void)prec;
    if (N == 8)
        return kNumVariants8;
    return 1;
}

const char *variant_name(int N, int prec, int v)
{
    (void)prec;
    if (N == 8 && v >= 0 && v < kNumVariants8)
        return kVariants8[v].name;
    if (N == 16 && v == 0)
        return "wg8_lds2";
    if (N <= 4 && v == 0)
        return "valu";
    return nullptr;
}

int default_variant(int N, int prec)
{
    (void)N;
    (void)prec;
    return 0;
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
    return prec == DCTF_PREC_FP32 ? run16<DCTF_PREC_FP32>(a, 1, stream)
                                  : run16<DCTF_PREC_SPLIT_BF16>(a, 1, stream);
}

}  // namespace dctf
