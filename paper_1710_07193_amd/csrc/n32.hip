// N = 32 filter: Y[b] = H_dct . X[b] with the 1024 x 1024 operator (4 MiB in
// FP32), too large for any register or LDS residency.  The product over
// all blocks is a matrix product Y^t = H . X^t (M = 1024 output coefficients,
// K = 1024, one column per block) with the operator streamed from L2.
//
// FP32 (k_filter_n32; the split-BF16 kernel k_filter_n32s is described
// with its code below):
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

// ---------------------------------------------------------------- split-BF16
//
// The same product with the operator in BF16 hi + lo (products hi.hi +
// hi.lo + lo.hi, FP32 accumulation): three BF16 MFMAs cost less than a
// quarter of one FP32 MFMA of the same K, which moves N = 32 from the FP32
// MFMA bound towards the HBM bound.  The 16 lowest-frequency coefficients
// (u, v < 4: the large terms of smooth image content) are multiplied in
// FP32 MFMA, and the DC column in FP32 VALU, after all the others.
//
// Operator images (from the FP64 operator, k_split32):
//   hi / lo  A operands of v_mfma_f32_16x16x32_bf16 for k-step s (the 32
//            coefficients of block row u = s): lane (m, g) of M-tile T holds
//            H[16T + m][32s + 8g + e], e < 8, at ((T*32 + s)*64 + 16g + m)*8 + e;
//            hi = bf16(fp32(H)), lo = bf16(fp32(H - hi)); the low-frequency
//            columns are zero.
//   lf       A operand of v_mfma_f32_16x16x4_f32 for the low-frequency
//            columns: k-step j, lane (m, g) holds H[16T + m][32g + j] at
//            (T*64 + 16g + m)*4 + j; the DC column (g = j = 0) is zero.
//
// Work: a workgroup of 4 waves takes a unit of 128 blocks (8 tiles of 16) x
// one 256-row panel P of the operator (wave w: M-tiles 16P + 4w .. + 3).  Per
// k-step (32 coefficients) the workgroup loads the unit's 128 x 32 FP32
// coefficients once (1 KiB rows of 8 contiguous float4 per block), splits
// them into BF16 hi / lo and stores them in LDS, double-buffered with one
// barrier per k-step, while every wave streams its 4 M-tiles of hi / lo
// from L2 (the next k-step's fragments in flight during the current one).
// LDS rows (one block, 32 BF16 = four 16-byte chunks, chunk g holding
// coefficients 8g .. 8g + 7) are XOR-swizzled, chunk g of block b at
// g ^ ((b / 4) % 4), which keeps the 16-byte MFMA reads of 16 blocks free
// of bank conflicts.
//
// XCD placement: XCD x serves panels 2 (x / 4) and 2 (x / 4) + 1 (2 MiB of
// hi / lo, L2-resident) for the block groups g = x (mod 4); the two panels
// of a group run on neighbouring workgroups of one XCD, so the group's
// coefficients are read from HBM by two XCDs, once each.
constexpr int kSteps32 = kNN32 / 32;          // BF16 k-steps

__device__ __forceinline__ bool low_freq32(int c) { return c < 128 && (c & 31) < 4; }

__global__ __launch_bounds__(256) void k_split32(const double *H64, uint16_t *hi, uint16_t *lo, float *lf)
{
    const int r = blockIdx.x, T = r >> 4, m = r & 15;
    for (int c = threadIdx.x; c < kNN32; c += 256) {
        const double h = H64[(size_t)r * kNN32 + c];
        const float h32 = __double2float_rn(h);
        const int s = c >> 5, g = (c >> 3) & 3, e = c & 7;
        uint16_t vh = 0, vl = 0;
        if (low_freq32(c))
            lf[(T * 64 + 16 * s + m) * 4 + (c & 3)] = c == 0 ? 0.0f : h32;
        else {
            vh = bf16_rne(h32);
            vl = bf16_rne(__double2float_rn(h - (double)bf16_to_f32(vh)));
        }
        const size_t fi = (((size_t)T * kSteps32 + s) * 64 + 16 * g + m) * 8 + e;
        hi[fi] = vh;
        lo[fi] = vl;
    }
}

// position (in BF16) of chunk g of block b in an LDS hi or lo array
__device__ __forceinline__ int s32_chunk(int b, int g) { return b * 32 + 8 * (g ^ ((b >> 2) & 3)); }

// NT block tiles per unit (16 NT blocks); ADB: the next k-step's operator
// fragments are loaded during the current one; XPF: the next tile's LDS
// read is issued before the current tile's MFMAs; OCC: waves per SIMD the
// registers are allocated for.
// MT M-tiles per wave and W waves per workgroup cover the 256-row panel
// (MT W = 16).
template <int MT, int W, int NT, bool ADB, bool XPF, int OCC>
__global__ __launch_bounds__(64 * W, OCC) void k_filter_n32s(FilterArgs a, int64_t groups)
{
    static_assert(MT * W == 16, "a workgroup covers one 256-row panel");
    constexpr int kThreads = 64 * W;
    constexpr int kBlocks = 16 * NT;               // blocks per unit
    constexpr int kQ = kBlocks * 8 / kThreads;     // loader float4 per thread and k-step
    constexpr int kBuf = 2 * kBlocks * 32;         // BF16 per LDS buffer (hi, lo)
    static_assert(kQ * kThreads == kBlocks * 8, "the loader covers the unit");
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * kBuf];
    const int tid = threadIdx.x, lane = tid & 63, n = lane & 15, g = lane >> 4, w = tid >> 6;
    const int xcd = blockIdx.x % 8;
    const int64_t L = gridDim.x / 8, l = blockIdx.x / 8;
    const int64_t B = a.B;
    const u32x4 *fhi = reinterpret_cast<const u32x4 *>(a.frag_hi);
    const u32x4 *flo = reinterpret_cast<const u32x4 *>(a.frag_lo);
    for (int64_t j = l;; j += L) {
        const int64_t grp = (xcd & 3) + 4 * (j >> 1);
        if (grp >= groups)
            break;
        const int P = 2 * (xcd >> 2) + (int)(j & 1);
        const int64_t blk0 = grp * kBlocks;
        const int T0 = 16 * P + MT * w;
        // loader: thread t moves float4 c8 = t % 8 (coefficients 4 c8 .. + 3
        // of the k-step) of blocks (kThreads / 8) q + t / 8, q < kQ
        const float *src[kQ];
        int ldpos[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int b = (kThreads / 8) * q + (tid >> 3), c8 = tid & 7;
            int64_t bb = blk0 + b;
            bb = bb < B ? bb : B - 1;   // clamped: its results are never stored
            src[q] = a.in + bb * kNN32 + 4 * c8;
            ldpos[q] = s32_chunk(b, c8 >> 1) + 4 * (c8 & 1);
        }
        auto load_x = [&](float4 (&xr)[kQ], int s) {
#pragma unroll
            for (int q = 0; q < kQ; ++q)
                xr[q] = ld4(src[q] + 32 * s);
        };
        auto stage_x = [&](const float4 (&xr)[kQ], int buf) {
            uint16_t *H = lds + buf * kBuf, *Lo = H + kBlocks * 32;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                uint32_t h01, h23, l01, l23;
                split_bf16(xr[q], h01, h23, l01, l23);
                *reinterpret_cast<uint2 *>(H + ldpos[q]) = make_uint2(h01, h23);
                *reinterpret_cast<uint2 *>(Lo + ldpos[q]) = make_uint2(l01, l23);
            }
        };
        auto load_a = [&](u32x4 (&ah)[MT], u32x4 (&al)[MT], int s) {
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const size_t fi = ((size_t)(T0 + t) * kSteps32 + s) * 64 + lane;
                ah[t] = fhi[fi];
                al[t] = flo[fi];
            }
        };
        f32x4 acc[MT][NT];
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int q = 0; q < NT; ++q)
                acc[t][q] = f32x4{0.f, 0.f, 0.f, 0.f};
        // k-steps from the highest block row (u = 31) to the lowest
        float4 xr[kQ];
        u32x4 ah[MT], al[MT], nh[ADB ? MT : 1], nl[ADB ? MT : 1];
        load_x(xr, kSteps32 - 1);
        if constexpr (ADB)
            load_a(ah, al, kSteps32 - 1);
        stage_x(xr, 0);   // the previous unit's reads of both buffers ended at its last barrier
        __syncthreads();
        for (int k = 0; k < kSteps32; ++k) {
            const int s = kSteps32 - 1 - k;
            if constexpr (!ADB)
                load_a(ah, al, s);
            if (s > 0) {
                load_x(xr, s - 1);
                if constexpr (ADB)
                    load_a(nh, nl, s - 1);
            }
            const uint16_t *H = lds + (k & 1) * kBuf, *Lo = H + kBlocks * 32;
            u32x4 xh, xl;
            if constexpr (XPF) {
                const int pos = s32_chunk(n, g);
                xh = *reinterpret_cast<const u32x4 *>(H + pos);
                xl = *reinterpret_cast<const u32x4 *>(Lo + pos);
            }
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                u32x4 yh, yl;
                if constexpr (XPF) {
                    if (q + 1 < NT) {
                        const int pos = s32_chunk(16 * (q + 1) + n, g);
                        yh = *reinterpret_cast<const u32x4 *>(H + pos);
                        yl = *reinterpret_cast<const u32x4 *>(Lo + pos);
                    }
                } else {
                    const int pos = s32_chunk(16 * q + n, g);
                    xh = *reinterpret_cast<const u32x4 *>(H + pos);
                    xl = *reinterpret_cast<const u32x4 *>(Lo + pos);
                }
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    acc[t][q] = mfma_bf16(ah[t], xh, acc[t][q]);
                    acc[t][q] = mfma_bf16(ah[t], xl, acc[t][q]);
                    acc[t][q] = mfma_bf16(al[t], xh, acc[t][q]);
                }
                if constexpr (XPF) {
                    if (q + 1 < NT) {
                        xh = yh;
                        xl = yl;
                    }
                }
            }
            if (s > 0) {
                stage_x(xr, (k + 1) & 1);
                if constexpr (ADB)
#pragma unroll
                    for (int t = 0; t < MT; ++t) {
                        ah[t] = nh[t];
                        al[t] = nl[t];
                    }
            }
            __syncthreads();
        }
        // low-frequency coefficients (u = g, v = 0 .. 3) in FP32 MFMA, then DC
        float4 alf[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t)
            alf[t] = ld4(a.frag_lf + ((size_t)(T0 + t) * 64 + lane) * 4);
        float x0[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            int64_t bb = blk0 + 16 * q + n;
            bb = bb < B ? bb : B - 1;
            const float4 xv = ld4(a.in + bb * kNN32 + 32 * g);
            x0[q] = lane_read(xv.x, n);   // coefficient 0 of block n (lane (n, 0))
            const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    const float av = jj == 0 ? alf[t].x : (jj == 1 ? alf[t].y : (jj == 2 ? alf[t].z : alf[t].w));
                    acc[t][q] = mfma_f32(av, xs[jj], acc[t][q]);
                }
        }
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            const float4 h = ld4(a.h0 + 16 * (T0 + t) + 4 * g);
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                acc[t][q][0] = fmaf(h.x, x0[q], acc[t][q][0]);
                acc[t][q][1] = fmaf(h.y, x0[q], acc[t][q][1]);
                acc[t][q][2] = fmaf(h.z, x0[q], acc[t][q][2]);
                acc[t][q][3] = fmaf(h.w, x0[q], acc[t][q][3]);
            }
        }
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int64_t blk = blk0 + 16 * q + n;
            if (blk < B) {
                float *dst = a.out + blk * kNN32 + 4 * g;
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    st4(dst + 16 * (T0 + t), acc[t][q]);
            }
        }
    }
}

}  // namespace

// Launch shape of the split kernel, measured over 261,120 blocks (ms):
// NT = 8 at two waves per SIMD 1.62-1.64; the same with the LDS prefetch
// 1.62; NT = 6 / 4 with the operator double buffer 1.68 / 1.84 (more
// operator traffic per block); one wave per SIMD with every prefetch and
// 256 accumulators in AGPRs, NT = 16 / 8: 1.96 / 2.21 (the second wave
// hides the latencies better than the in-wave pipeline); 8 waves of 2
// M-tiles per workgroup with both prefetches, NT = 8 / 16: 2.03 / 1.61.
constexpr int kSMt = 4;
constexpr int kSW = 4;
constexpr int kSNt = 8;
constexpr bool kSAdb = false;
constexpr bool kSXpf = false;
constexpr int kSOcc = 2;

hipError_t launch_split_n32(const double *H64, uint16_t *hi, uint16_t *lo, float *lf, hipStream_t stream)
{
    hipLaunchKernelGGL(k_split32, dim3(kNN32), dim3(256), 0, stream, H64, hi, lo, lf);
    return hipGetLastError();
}

hipError_t launch_filter_n32(int prec, const FilterArgs &a, hipStream_t stream)
{
    if (a.B <= 0)
        return hipSuccess;
    if (prec == DCTF_PREC_SPLIT_BF16) {
        const int64_t groups = (a.B + 16 * kSNt - 1) / (16 * kSNt);
        // kSOcc waves per SIMD (4 kSOcc / kSW workgroups per CU), a multiple of
        // the 8 XCDs; the workgroups past the last unit of their XCD find no work
        int64_t wgs = (int64_t)cu_count() * kSOcc * 4 / kSW;
        // XCD x has 2 ceil((groups - x % 4) / 4) units: at most that many workgroups each
        const int64_t need = 8 * 2 * ((groups + 3) / 4);
        wgs = wgs < need ? wgs : need;
        wgs = (wgs + 7) / 8 * 8;
        hipLaunchKernelGGL((k_filter_n32s<kSMt, kSW, kSNt, kSAdb, kSXpf, kSOcc>), dim3((unsigned)wgs),
                           dim3(64 * kSW), 0, stream, a, groups);
        return hipGetLastError();
    }
    const int64_t groups = (a.B + 16 * kN32Nt - 1) / (16 * kN32Nt);
    const int64_t units = groups * (64 / kN32Mt);
    // as many waves as are resident at once (3 per SIMD: 5.56 -> 5.15 ms against 16 per CU)
    static const int per_cu = resident_groups(k_filter_n32<kN32Mt, kN32Nt>, 256);
    int64_t waves = (int64_t)cu_count() * per_cu * 4;
    waves = waves < units ? waves : units;
    const int64_t wgs = (waves + 3) / 4;
    hipLaunchKernelGGL((k_filter_n32<kN32Mt, kN32Nt>), dim3((unsigned)wgs), dim3(256), 0, stream, a, groups, waves);
    return hipGetLastError();
}

}  // namespace dctf
