// Persistent batched filter: one launch over many jobs (images), operators
// (masks) and both MFMA block sizes.
//
// The host groups jobs by N and, within N, by operator, and numbers work
// units consecutively across the jobs of each class (JobDesc::unit_begin):
//   N = 8 : a unit is 32 blocks (two 16-block MFMA tiles), done by one wave;
//   N = 16: a unit is 16 blocks, done by one 8-wave workgroup.
// Workgroups [0, groups8) take the N = 8 units, the rest the N = 16 units.
// Each wave (N = 8) or workgroup (N = 16) takes one contiguous range of
// units, so it crosses few job and operator boundaries; its operator
// fragments are reloaded only when the operator changes.  The per-block
// arithmetic is the one of the single-operator kernels, so every block's
// result is bit-identical to filtering its job alone.
#include "mfma_common.h"

namespace dctf {
namespace {

constexpr int kU8 = kUnitBlocks8 / 16;   // MFMA tiles per N = 8 unit

struct UnitRef {
    const float *in;
    float *out;
    int64_t B;      // blocks of the job
    int64_t blk0;   // first block of the unit within the job
    int op;
};

__device__ __forceinline__ int find_job(const JobDesc *jobs, int njobs, int64_t unit)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].unit_begin <= unit)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ UnitRef resolve(const JobDesc *jobs, int njobs, int &j, int64_t unit,
                                           int blocks_per_unit)
{
    while (j + 1 < njobs && jobs[j + 1].unit_begin <= unit)
        ++j;
    const JobDesc &d = jobs[j];
    UnitRef r;
    r.in = d.in;
    r.out = d.out;
    r.B = d.B;
    r.blk0 = (unit - d.unit_begin) * blocks_per_unit;
    r.op = d.op;
    return r;
}

template <int PREC>
__device__ void worker8(const BatchArgs &a, int64_t gw, int64_t nwaves, int lane)
{
    const int64_t u_begin = gw * a.units8 / nwaves;
    const int64_t u_end = (gw + 1) * a.units8 / nwaves;
    if (u_begin >= u_end)
        return;
    const int n = lane & 15, g = lane >> 4;
    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs8F32, OpRegs8BF16>::type Regs;
    Regs R;
    int loaded_op = -1;

    auto load_unit = [&](float4 (&x)[kU8][4], const UnitRef &r) {
#pragma unroll
        for (int u = 0; u < kU8; ++u) {
            int64_t blk = r.blk0 + 16 * u + n;
            blk = blk < r.B ? blk : r.B - 1;
            const float *src = r.in + blk * 64 + 4 * g;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                x[u][i] = ld4(src + 16 * i);
        }
    };
    auto compute_store = [&](float4 (&x)[kU8][4], const UnitRef &r) {
        if (r.op != loaded_op) {
            const OpDesc &o = a.ops[r.op];
            if constexpr (PREC == DCTF_PREC_FP32)
                load_op8(R, o.frag32, o.h0, lane);
            else
                load_op8(R, o.frag_hi, o.frag_lo, o.frag_lf, lane);
            loaded_op = r.op;
        }
#pragma unroll
        for (int u = 0; u < kU8; ++u) {
            f32x4 acc[4];
            tile8(R, x[u], lane, acc);
            const int64_t blk = r.blk0 + 16 * u + n;
            if (blk < r.B) {
                float *dst = r.out + blk * 64 + 4 * g;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    st4(dst + 16 * t, acc[t]);
            }
        }
    };

    int j = find_job(a.jobs8, a.njobs8, u_begin);
    UnitRef rc = resolve(a.jobs8, a.njobs8, j, u_begin, kUnitBlocks8);
    float4 cur[kU8][4], nxt[kU8][4];
    load_unit(cur, rc);
    for (int64_t u = u_begin + 1; u < u_end; ++u) {
        const UnitRef rn = resolve(a.jobs8, a.njobs8, j, u, kUnitBlocks8);
        load_unit(nxt, rn);
        compute_store(cur, rc);
#pragma unroll
        for (int q = 0; q < kU8; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                cur[q][i] = nxt[q][i];
        rc = rn;
    }
    compute_store(cur, rc);
}

template <int PREC>
__device__ void worker16(const BatchArgs &a, int64_t wg, int64_t ngroups, char *smem)
{
    const int64_t t_begin = wg * a.units16 / ngroups;
    const int64_t t_end = (wg + 1) * a.units16 / ngroups;
    if (t_begin >= t_end)
        return;   // uniform over the workgroup
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs16F32, OpRegs16BF16>::type Regs;
    Regs R;
    int loaded_op = -1;

    constexpr int kF32 = 16 * kLd16F32;
    constexpr int kB16 = 16 * kLd16BF16;
    float *lf = reinterpret_cast<float *>(smem);
    uint16_t *lhi = reinterpret_cast<uint16_t *>(smem);
    uint16_t *llo = lhi + 2 * kB16;
    float *llf = reinterpret_cast<float *>(llo + 2 * kB16);

    auto stage = [&](Stage16 &S, const UnitRef &r) {
        stage16_load(S, r.in + r.blk0 * 256, r.B - r.blk0, 0, tid);
    };
    auto put = [&](const Stage16 &S, int buf) {
        if constexpr (PREC == DCTF_PREC_FP32)
            stage16_store(S, lf + buf * kF32, tid);
        else
            stage16_store(S, lhi + buf * kB16, llo + buf * kB16, llf + buf * 16 * kLd16Lf, tid);
    };

    int j = find_job(a.jobs16, a.njobs16, t_begin);
    UnitRef rc = resolve(a.jobs16, a.njobs16, j, t_begin, kUnitBlocks16);
    Stage16 S;
    stage(S, rc);
    put(S, 0);
    __syncthreads();
    int buf = 0;
    for (int64_t t = t_begin;; ++t) {
        const bool more = t + 1 < t_end;
        UnitRef rn = rc;
        if (more) {
            rn = resolve(a.jobs16, a.njobs16, j, t + 1, kUnitBlocks16);
            stage(S, rn);
        }
        if (rc.op != loaded_op) {
            const OpDesc &o = a.ops[rc.op];
            if constexpr (PREC == DCTF_PREC_FP32)
                load_op16(R, o.frag32, o.h0, wave, lane);
            else
                load_op16(R, o.frag_hi, o.frag_lo, o.frag_lf, wave, lane);
            loaded_op = rc.op;
        }
        f32x4 acc[2];
        if constexpr (PREC == DCTF_PREC_FP32)
            tile16(R, lf + buf * kF32, lane, acc);
        else
            tile16(R, lhi + buf * kB16, llo + buf * kB16, llf + buf * 16 * kLd16Lf, lane, acc);
        const int64_t blk = rc.blk0 + n;
        if (blk < rc.B) {
            float *dst = rc.out + blk * 256 + 32 * wave + 4 * g;
            st4(dst, acc[0]);
            st4(dst + 16, acc[1]);
        }
        if (!more)
            break;
        put(S, buf ^ 1);
        __syncthreads();
        buf ^= 1;
        rc = rn;
    }
}

template <int PREC>
__global__ __launch_bounds__(kBatchThreads) void k_batch(BatchArgs a)
{
    constexpr int kBytes = PREC == DCTF_PREC_FP32 ? 2 * kTile16BytesF32 : 2 * kTile16BytesSplit;
    __shared__ __attribute__((aligned(16))) char smem[kBytes];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if ((int)blockIdx.x < a.groups8) {
        const int64_t nw = (int64_t)a.groups8 * (kBatchThreads / 64);
        worker8<PREC>(a, (int64_t)blockIdx.x * (kBatchThreads / 64) + wave, nw, lane);
    } else {
        worker16<PREC>(a, (int64_t)blockIdx.x - a.groups8, a.groups16, smem);
    }
}

}  // namespace

hipError_t launch_batch(const BatchArgs &a, hipStream_t stream)
{
    const int groups = a.groups8 + a.groups16;
    if (groups <= 0)
        return hipSuccess;
    if (a.prec == DCTF_PREC_FP32)
        hipLaunchKernelGGL(k_batch<DCTF_PREC_FP32>, dim3(groups), dim3(kBatchThreads), 0, stream, a);
    else
        hipLaunchKernelGGL(k_batch<DCTF_PREC_SPLIT_BF16>, dim3(groups), dim3(kBatchThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace dctf

namespace dctf {

int batch_occupancy(int prec)
{
    int nb = 0;
    hipError_t e = (prec == DCTF_PREC_FP32)
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<DCTF_PREC_FP32>, kBatchThreads, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<DCTF_PREC_SPLIT_BF16>, kBatchThreads, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace dctf
