// N = 32 filter: Y[b] = H_dct . X[b] with the 1024 x 1024 operator (4 MiB in
// FP32), too large for any register or LDS residency.  The product over
// all blocks is a matrix product Y^t = H . X^t (M = 1024 output coefficients,
// K = 1024, one column per block) with the operator streamed from L2:
//
//   a wave owns a unit of MT M-tiles (16 output rows each) x NT N-tiles (16
//   blocks each) and walks K in 64 chunks of 16 coefficients, from the
//   highest frequencies to the lowest (FP32 accuracy: the large
//   low-frequency products enter the sum last); per chunk it
//   loads one 16-byte fragment per M-tile (the builder's frag32 layout,
//   ((T*64 + i)*64 + lane)*4 + j) and one 16-byte slice per block
//   (coefficients 16i + 4g .. +3 of block n), then issues 4 x MT x NT
//   v_mfma_f32_16x16x4_f32.  The next chunk's loads are in flight while the
//   current one is multiplied.
//
// Units are numbered block group first and dealt to the workgroups in
// order, which the dispatcher spreads round-robin over the 8 XCDs: each XCD
// sees 4 of the 16 operator panels (1 MiB, L2-resident) and each block group
// is read by 4 XCDs.  Handing a group's 16 panels to one XCD instead (the
// XCD order of the image-level kernel) reads each block once but makes every
// XCD stream the whole 4 MiB operator through its 4 MB L2: measured 7.3 GB
// of fetches per launch against 5.3 GB, at the same speed (the kernel is
// MFMA-bound).
// The DC column is zeroed in the MFMA image and applied in FP32 VALU after
// the AC products (the DC product is the largest term of the sum).
#include "mfma_common.h"

namespace dctf {
namespace {

constexpr int kNN32 = 1024;
constexpr int kChunks32 = kNN32 / 16;   // k-chunks of 16 coefficients

template <int MT, int NT>
__global__ __launch_bounds__(256) void k_filter_n32(FilterArgs a, int64_t groups, int64_t waves)
{
    constexpr int kPanels = 64 / MT;   // M-tile panels per block group
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t units = groups * kPanels;
    const int64_t B = a.B;
    for (int64_t unit = wave; unit < units; unit += waves) {
        const int64_t grp = unit / kPanels;
        const int T0 = (int)(unit % kPanels) * MT;
        int64_t blk[NT];
        const float *xs[NT];
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            blk[s] = grp * (16 * NT) + 16 * s + n;
            const int64_t bb = blk[s] < B ? blk[s] : B - 1;   // clamped: the store is masked
            xs[s] = a.in + bb * kNN32 + 4 * g;
        }
        const float *fa = a.frag32 + ((size_t)T0 * kChunks32 * 64 + lane) * 4;
        f32x4 acc[MT][NT];
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int s = 0; s < NT; ++s)
                acc[t][s] = f32x4{0.f, 0.f, 0.f, 0.f};
        float4 A[MT], X[NT], An[MT], Xn[NT];
        auto load = [&](float4 (&Ar)[MT], float4 (&Xr)[NT], int i) {
#pragma unroll
            for (int t = 0; t < MT; ++t)
                Ar[t] = ld4(fa + ((size_t)t * kChunks32 + i) * 256);
#pragma unroll
            for (int s = 0; s < NT; ++s)
                Xr[s] = ld4(xs[s] + 16 * i);
        };
        // Chunks from the highest to the lowest frequency: the accumulator stays
        // small while the many small high-frequency products are added, and
        // only the last chunks (rows u < 4 of the block) add large terms.
        load(A, X, kChunks32 - 1);
        float x0[NT];
        for (int i = kChunks32 - 1; i >= 0; --i) {
            if (i > 0)
                load(An, Xn, i - 1);
            if (i == 0)
#pragma unroll
                for (int s = 0; s < NT; ++s)
                    x0[s] = lane_read(X[s].x, n);   // coefficient 0 of block n (lane (n, 0), chunk 0)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
#pragma unroll
                for (int s = 0; s < NT; ++s) {
                    const float xv = j == 0 ? X[s].x : (j == 1 ? X[s].y : (j == 2 ? X[s].z : X[s].w));
#pragma unroll
                    for (int t = 0; t < MT; ++t) {
                        const float av = j == 0 ? A[t].x : (j == 1 ? A[t].y : (j == 2 ? A[t].z : A[t].w));
                        acc[t][s] = mfma_f32(av, xv, acc[t][s]);
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < MT; ++t)
                A[t] = An[t];
#pragma unroll
            for (int s = 0; s < NT; ++s)
                X[s] = Xn[s];
        }
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            const float4 h = ld4(a.h0 + 16 * (T0 + t) + 4 * g);
#pragma unroll
            for (int s = 0; s < NT; ++s) {
                acc[t][s][0] = fmaf(h.x, x0[s], acc[t][s][0]);
                acc[t][s][1] = fmaf(h.y, x0[s], acc[t][s][1]);
                acc[t][s][2] = fmaf(h.z, x0[s], acc[t][s][2]);
                acc[t][s][3] = fmaf(h.w, x0[s], acc[t][s][3]);
            }
        }
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            if (blk[s] < B) {
                float *dst = a.out + blk[s] * kNN32 + 4 * g;
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    st4(dst + 16 * (T0 + t), acc[t][s]);
            }
        }
    }
}

constexpr int kN32Mt = 4;
constexpr int kN32Nt = 2;
constexpr int kN32WavesPerCu = 16;

}  // namespace

hipError_t launch_filter_n32(const FilterArgs &a, hipStream_t stream)
{
    if (a.B <= 0)
        return hipSuccess;
    const int64_t groups = (a.B + 16 * kN32Nt - 1) / (16 * kN32Nt);
    const int64_t units = groups * (64 / kN32Mt);
    int64_t waves = (int64_t)cu_count() * kN32WavesPerCu;
    waves = waves < units ? waves : units;
    const int64_t wgs = (waves + 3) / 4;
    hipLaunchKernelGGL((k_filter_n32<kN32Mt, kN32Nt>), dim3((unsigned)wgs), dim3(256), 0, stream, a, groups, waves);
    return hipGetLastError();
}

}  // namespace dctf
