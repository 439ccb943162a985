// Persistent batched filter: one launch over many jobs (images), operators
// (masks) and both MFMA block sizes.
//
// The host groups jobs by N and, within N, by operator, and numbers work
// units consecutively across the jobs of each class (JobDesc::unit_begin):
//   N = 8 : a unit is one 16-block MFMA tile, done by one wave;
//   N = 16: a unit is one 16-block tile, done by one 8-wave workgroup.
// Workgroups [0, groups8) take the N = 8 units, the rest the N = 16 units.
// The units of a class are cut into "fronts": N = 8 work into a few runs of
// operator segments (one sweep front each: fewer fronts stream HBM better,
// more fronts mean fewer operator reloads per wave), N = 16 work into one
// front per operator.  Each front owns a contiguous range of workers (waves
// for N = 8, workgroups for N = 16) in proportion to its units, and they
// stride over its units front to back.  The per-block arithmetic is the one
// of the single-operator kernels, so every block's result is bit-identical
// to filtering its job alone.
#include "mfma_common.h"

namespace dctf {
namespace {

struct UnitRef {
    const float *in;
    float *out;
    int64_t B;      // blocks of the job
    int64_t blk0;   // first block of the unit within the job
    int op;
};

// Segment of worker w: the last segment whose worker_begin <= w.
__device__ __forceinline__ int find_segment(const SegDesc *segs, int nsegs, int64_t w)
{
    int lo = 0, hi = nsegs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].worker_begin <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Walks the job table forward as the unit index grows.  The end of the
// current job follows from its own descriptor.  The next job's descriptor is
// requested by refill() with a vector load (lane k loads dword k) issued just
// before a step's data loads: a scalar load would share its wait counter with
// the LDS accesses of the tile pipeline and stall them, while the vector load
// completes in order ahead of the data it precedes.  At the crossing the
// fields are read back from the lanes.
template <int BPU>   // blocks per work unit
struct JobCursor {
    static_assert(sizeof(JobDesc) == 40, "JobDesc is 10 dwords");
    static constexpr int blocks_per_unit = BPU;
    const JobDesc *jobs;
    int end, j;
    JobDesc cur;
    int64_t cur_end;   // first unit after the current job
    uint32_t nextv;    // lane k < 10: dword k of jobs[j + 1]
    bool have_next;

    __device__ __forceinline__ int64_t units_of(const JobDesc &d) const
    {
        return (d.B + blocks_per_unit - 1) / blocks_per_unit;
    }
    __device__ __forceinline__ void start(const JobDesc *t, int job_begin, int job_end, int64_t unit)
    {
        jobs = t;
        end = job_end;
        j = job_begin;
        cur = t[j];
        cur_end = cur.unit_begin + units_of(cur);
        have_next = false;
        at(unit);
    }
    __device__ __forceinline__ void refill()
    {
        if (!have_next && j + 1 < end) {
            const uint32_t *p = reinterpret_cast<const uint32_t *>(jobs + j + 1);
            const int lane = __lane_id();
            nextv = p[lane < 10 ? lane : 0];
            have_next = true;
        }
    }
    __device__ __forceinline__ JobDesc unpack() const
    {
        uint32_t w[10];
#pragma unroll
        for (int k = 0; k < 10; ++k)
            w[k] = (uint32_t)__builtin_amdgcn_readlane((int)nextv, k);
        JobDesc d;
        __builtin_memcpy(&d, w, sizeof(d));
        return d;
    }
    __device__ __forceinline__ UnitRef at(int64_t unit)
    {
        while (unit >= cur_end && j + 1 < end) {
            refill();   // no-op when the descriptor was requested earlier
            cur = unpack();
            ++j;
            have_next = false;
            cur_end = cur.unit_begin + units_of(cur);
        }
        UnitRef r;
        r.in = cur.in;
        r.out = cur.out;
        r.B = cur.B;
        r.blk0 = (unit - cur.unit_begin) * blocks_per_unit;
        r.op = cur.op;
        return r;
    }
};

// The waves of a front (a run of consecutive segments) stride over its
// units together; a wave reloads its operator fragments when the unit it
// reaches belongs to another operator.
template <int PREC, int IO, bool NT>
__device__ void worker8(const BatchArgs &a, int64_t gw, int lane, float4 *lds)
{
    if (gw >= a.workers8)
        return;
    const SegDesc &sg = a.segs8[find_segment(a.segs8, a.nsegs8, gw)];
    const int64_t first = sg.unit_begin + (gw - sg.worker_begin);
    const int64_t stride = sg.nworkers, end = sg.unit_end;
    const int job_begin = sg.job_begin, job_end = sg.job_end;
    if (first >= end)
        return;
    const int64_t my_units = (end - first + stride - 1) / stride;
    const int n = lane & 15, g = lane >> 4;

    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs8F32, OpRegs8BF16>::type Regs;
    Regs R;
    int loaded_op = -1;
    auto op_load = [&](int op) {
        const OpDesc &o = a.ops[op];
        if constexpr (PREC == DCTF_PREC_FP32)
            load_op8(R, o.frag32, o.h0, lane);
        else
            load_op8(R, o.frag_hi, o.frag_lo, o.frag_lf, lane);
        loaded_op = op;
    };

    auto load_unit = [&](float4 (&x)[4], const UnitRef &r) {
        if constexpr (IO == 1) {
            load_tile_coalesced<NT>(x, r.in + r.blk0 * 64, r.B - r.blk0, lane);
        } else {
            int64_t blk = r.blk0 + n;
            blk = blk < r.B ? blk : r.B - 1;
            const float *src = r.in + blk * 64 + 4 * g;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                x[i] = NT ? ld4_nt(src + 16 * i) : ld4(src + 16 * i);
        }
    };
    // Operator fragments are requested before the data loads of the unit
    // after, so the wait for them does not also drain that unit's loads.
    auto ensure_op = [&](int op) {
        if (op != loaded_op)
            op_load(op);
    };
    auto compute_store = [&](float4 (&x)[4], const UnitRef &r) {
        if constexpr (IO == 1) {
            tile8_coalesced<NT>(R, x, lds, r.out + r.blk0 * 64, r.B - r.blk0, lane);
        } else {
            f32x4 acc[4];
            tile8(R, x, lane, acc);
            const int64_t blk = r.blk0 + n;
            if (blk < r.B) {
                float *dst = r.out + blk * 64 + 4 * g;
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

    JobCursor<kUnitBlocks8> jc;
    int64_t unit = first;
    jc.start(a.jobs8, job_begin, job_end, unit);
    UnitRef rc = jc.at(unit);
    float4 cur[4], nxt[4];
    ensure_op(rc.op);
    load_unit(cur, rc);
    for (int64_t k = 1; k < my_units; ++k) {
        unit += stride;
        const UnitRef rn = jc.at(unit);
        jc.refill();
        ensure_op(rc.op);
        load_unit(nxt, rn);
        compute_store(cur, rc);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            cur[i] = nxt[i];
        rc = rn;
    }
    ensure_op(rc.op);
    compute_store(cur, rc);
}

template <int PREC, int D>
__device__ void worker16(const BatchArgs &a, int64_t wg, char *smem)
{
    if (wg >= a.workers16)
        return;   // uniform over the workgroup
    const SegDesc &sg = a.segs16[find_segment(a.segs16, a.nsegs16, wg)];
    const int64_t first = sg.unit_begin + (wg - sg.worker_begin);
    if (first >= sg.unit_end)
        return;
    const int64_t stride = sg.nworkers;
    const int64_t count = (sg.unit_end - first + stride - 1) / stride;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs16F32, OpRegs16BF16>::type Regs;
    Regs R;
    JobCursor<kUnitBlocks16> jc;
    jc.start(a.jobs16, sg.job_begin, sg.job_end, first);
    auto ref = [&](int64_t t) {
        const UnitRef r = jc.at(first + t * stride);
        jc.refill();   // ahead of the tile's data loads
        return r;
    };
    auto op_load = [&](int op) {
        const OpDesc &o = a.ops[op];
        if constexpr (PREC == DCTF_PREC_FP32)
            load_op16(R, o.frag32, o.h0, wave, lane);
        else
            load_op16(R, o.frag_hi, o.frag_lo, o.frag_lf, wave, lane);
    };
    run_tiles16<PREC, D, UnitRef>(count, ref, op_load, R, smem);
}

template <int PREC, int IO, bool NT>
__global__ __launch_bounds__(kBatchThreads) void k_batch(BatchArgs a)
{
    // N = 16 workgroups use the LDS for their double-buffered tiles, N = 8
    // workgroups for the per-wave staging of the coalesced I/O.
    constexpr int k16 = PREC == DCTF_PREC_FP32 ? kSmem16F32 : kSmem16Split;
    constexpr int k8 = IO ? (kBatchThreads / 64) * 256 * 16 : 0;
    constexpr int kBytes = k16 > k8 ? k16 : k8;
    __shared__ __attribute__((aligned(16))) char smem[kBytes];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if ((int)blockIdx.x < a.groups8) {
        float4 *lds = reinterpret_cast<float4 *>(smem) + (IO ? wave * 256 : 0);
        worker8<PREC, IO, NT>(a, (int64_t)blockIdx.x * (kBatchThreads / 64) + wave, lane, lds);
    } else {
        worker16<PREC, batch_depth16(PREC)>(a, (int64_t)blockIdx.x - a.groups8, smem);
    }
}

// Batches of one block size run a kernel holding only that worker, so the
// register allocation and schedule are those of the worker alone.
template <int PREC, int IO, bool NT>
__global__ __launch_bounds__(kBatch8Threads) void k_batch8(BatchArgs a)
{
    __shared__ __attribute__((aligned(16))) float4 lds_all[IO ? (kBatch8Threads / 64) * 256 : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    worker8<PREC, IO, NT>(a, (int64_t)blockIdx.x * (kBatch8Threads / 64) + wave, lane, lds_all + (IO ? wave * 256 : 0));
}

template <int PREC>
__global__ __launch_bounds__(kBatchThreads) void k_batch16(BatchArgs a)
{
    __shared__ __attribute__((aligned(16))) char smem[PREC == DCTF_PREC_FP32 ? kSmem16F32 : kSmem16Split];
    worker16<PREC, batch_depth16(PREC)>(a, blockIdx.x, smem);
}

template <int PREC, int IO, bool NT>
hipError_t launch_batch_t(const BatchArgs &a, hipStream_t stream)
{
    if (a.groups16 == 0)
        hipLaunchKernelGGL((k_batch8<PREC, IO, NT>), dim3(a.groups8), dim3(kBatch8Threads), 0, stream, a);
    else if (a.groups8 == 0)
        hipLaunchKernelGGL((k_batch16<PREC>), dim3(a.groups16), dim3(kBatchThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((k_batch<PREC, IO, NT>), dim3(a.groups8 + a.groups16), dim3(kBatchThreads), 0, stream, a);
    return hipGetLastError();
}

template <typename K>
int occ(K kernel, int threads)
{
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

template <int PREC, int IO, bool NT>
int occupancy_t(int kind)
{
    if (kind == 8)
        return occ(k_batch8<PREC, IO, NT>, kBatch8Threads);
    if (kind == 16)
        return occ(k_batch16<PREC>, kBatchThreads);
    return occ(k_batch<PREC, IO, NT>, kBatchThreads);
}

}  // namespace

hipError_t launch_batch(const BatchArgs &a, hipStream_t stream)
{
    const int groups = a.groups8 + a.groups16;
    if (groups <= 0)
        return hipSuccess;
    const bool f32 = a.prec == DCTF_PREC_FP32;
    switch (a.io * 2 + (a.nt ? 1 : 0)) {
    case 0: return f32 ? launch_batch_t<DCTF_PREC_FP32, 0, false>(a, stream) : launch_batch_t<DCTF_PREC_SPLIT_BF16, 0, false>(a, stream);
    case 1: return f32 ? launch_batch_t<DCTF_PREC_FP32, 0, true>(a, stream) : launch_batch_t<DCTF_PREC_SPLIT_BF16, 0, true>(a, stream);
    case 2: return f32 ? launch_batch_t<DCTF_PREC_FP32, 1, false>(a, stream) : launch_batch_t<DCTF_PREC_SPLIT_BF16, 1, false>(a, stream);
    default: return f32 ? launch_batch_t<DCTF_PREC_FP32, 1, true>(a, stream) : launch_batch_t<DCTF_PREC_SPLIT_BF16, 1, true>(a, stream);
    }
}

int batch_occupancy(int prec, int io, bool nt, int kind)
{
    const bool f32 = prec == DCTF_PREC_FP32;
    switch (io * 2 + (nt ? 1 : 0)) {
    case 0: return f32 ? occupancy_t<DCTF_PREC_FP32, 0, false>(kind) : occupancy_t<DCTF_PREC_SPLIT_BF16, 0, false>(kind);
    case 1: return f32 ? occupancy_t<DCTF_PREC_FP32, 0, true>(kind) : occupancy_t<DCTF_PREC_SPLIT_BF16, 0, true>(kind);
    case 2: return f32 ? occupancy_t<DCTF_PREC_FP32, 1, false>(kind) : occupancy_t<DCTF_PREC_SPLIT_BF16, 1, false>(kind);
    default: return f32 ? occupancy_t<DCTF_PREC_FP32, 1, true>(kind) : occupancy_t<DCTF_PREC_SPLIT_BF16, 1, true>(kind);
    }
}

}  // namespace dctf
