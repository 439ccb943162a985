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
// requested by refill() with a vector load (lane k loads dword k) issued once
// per step, unconditionally, just before the step's data loads: a scalar load
// would share its wait counter with the LDS accesses of the tile pipeline and
// stall them, while the vector load completes in order ahead of the data it
// precedes; and since it is issued at the same point of every step, the
// compiler can wait for it alone at a crossing (a conditional request would
// make it wait for every load in flight).  At the crossing the fields are
// read back from the lanes.
template <int BPU>   // blocks per work unit
struct JobCursor {
    static_assert(sizeof(JobDesc) == 40, "JobDesc is 10 dwords");
    static constexpr int blocks_per_unit = BPU;
    const JobDesc *jobs;
    int end, j;
    JobDesc cur;
    int64_t cur_end;   // first unit after the current job
    uint32_t nextv;    // lane k < 10: dword k of jobs[min(j + 1, end - 1)] as of the last refill()

    __device__ __forceinline__ int64_t units_of(const JobDesc &d) const
    {
        return (d.B + blocks_per_unit - 1) / blocks_per_unit;
    }
    // Positions the cursor on the job of `unit` (reading the table directly),
    // then requests the descriptor after it: refill() must always follow the
    // last move, or a crossing would take a stale descriptor.
    __device__ __forceinline__ void start(const JobDesc *t, int job_begin, int job_end, int64_t unit)
    {
        jobs = t;
        end = job_end;
        j = job_begin;
        cur = t[j];
        cur_end = cur.unit_begin + units_of(cur);
        while (unit >= cur_end && j + 1 < end) {
            ++j;
            cur = t[j];
            cur_end = cur.unit_begin + units_of(cur);
        }
        refill();
    }
    __device__ __forceinline__ void refill()
    {
        const int nj = j + 1 < end ? j + 1 : j;
        const uint32_t *p = reinterpret_cast<const uint32_t *>(jobs + nj);
        const int lane = __lane_id();
        nextv = ldg_u32(p + (lane < 10 ? lane : 0));
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
    __device__ __forceinline__ void advance()
    {
        cur = unpack();
        ++j;
        cur_end = cur.unit_begin + units_of(cur);
    }
    __device__ __forceinline__ UnitRef at(int64_t unit)
    {
        if (unit >= cur_end && j + 1 < end) {
            advance();   // the descriptor the last refill() requested
            while (unit >= cur_end && j + 1 < end) {
                refill();   // the unit skipped a whole job: read the next descriptor now
                advance();
            }
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
__device__ __forceinline__ void worker8(const BatchArgs &a, int64_t gw, int lane, float4 *lds, float4 *t0,
                                        float4 *t1)
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

    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs8F32, OpRegs8BF16>::type Regs;
    Regs R;
    auto op_load = [&](int op) {
        const OpDesc &o = a.ops[op];
        if constexpr (PREC == DCTF_PREC_FP32)
            load_op8(R, o.frag32, o.h0, lane);
        else
            load_op8(R, o.frag_hi, o.frag_lo, o.frag_lf, lane);
    };

    uint32_t off[4];
    if constexpr (IO >= 1)
        coalesced_offsets(off, lane);
    else
        mfma_offsets(off, lane);

    if constexpr (IO == 2) {
        // Tiles loaded straight into LDS: the wave's two tile buffers t0, t1
        // alternate.  A run of one operator is code of its own for each
        // buffer its first unit sits in, so that every access names its
        // buffer statically (the compiler then waits for that buffer's loads
        // only); a run returns the buffer of the next run's first unit.
        // In flight after a tile's loads when the step reading it waits: the
        // 4 stores of the step before (4 dropped stores before the first
        // step), the job descriptor request and the 4 loads of the next tile
        // (every step issues them; past the wave's last unit an empty tile).
        // Operator loads at the start of a run add to them and are waited
        // for as well.
        auto dma_unit = [&](float4 *t, const UnitRef &r) { dma_tile8<NT>(t, tile_rsrc8(r.in, r.blk0, r.B), off); };
        auto compute_lds = [&](float4 *t, const UnitRef &r) {
            tile8_from_lds<9, NT>(R, t, tile_rsrc8(r.out, r.blk0, r.B), off, lane);
        };
        JobCursor<kUnitBlocks8> jc;
        int64_t unit = first, k = 0;
        jc.start(a.jobs8, job_begin, job_end, unit);
        UnitRef rc = jc.at(unit), rn;
        dma_unit(t0, rc);
        dummy_stores8<NT>(rc.out, off);
        auto step = [&](float4 *cb, float4 *nb) -> bool {
            const bool more = k + 1 < my_units;
            if (more) {
                unit += stride;
                rn = jc.at(unit);
            } else {
                rn = rc;
                rn.B = 0;   // past the wave's last unit: an empty tile
            }
            jc.refill();
            dma_unit(nb, rn);
            compute_lds(cb, rc);
            ++k;
            rc = rn;
            return more;
        };
        auto run = [&](auto P) -> int {
            constexpr int p = decltype(P)::value;
            float4 *ta = p ? t1 : t0, *tb = p ? t0 : t1;
            const int op = rc.op;
            op_load(op);
            if (!step(ta, tb))
                return -1;
            if (rc.op != op)
                return 1 - p;
            for (;;) {
                if (!step(tb, ta))
                    return -1;
                if (rc.op != op)
                    return p;
                if (!step(ta, tb))
                    return -1;
                if (rc.op != op)
                    return 1 - p;
            }
        };
        for (int par = 0; par >= 0;)
            par = par ? run(std::integral_constant<int, 1>()) : run(std::integral_constant<int, 0>());
        return;
    }

    auto load_unit = [&](float4 (&x)[4], const UnitRef &r) {
        load_tile_buf<NT>(x, tile_rsrc8(r.in, r.blk0, r.B), off);
    };
    auto compute_store = [&](float4 (&x)[4], const UnitRef &r) {
        const rsrc_t out = tile_rsrc8(r.out, r.blk0, r.B);
        if constexpr (IO == 1)
            tile8_buf<NT>(R, x, lds, out, off, lane);
        else
            tile8_buf_direct<NT>(R, x, out, off, lane);
    };

    // The wave's units form runs of one operator.  Each run starts with the
    // operator's fragments loaded (requested after the data loads of the
    // run's first unit and before those of the unit after, so the wait for
    // them does not drain that unit's loads); that first step is peeled off
    // the loop, so the loop never waits for operator loads.  Inside a run two
    // register buffers alternate (the body is unrolled twice): the loads of
    // the next unit stay in flight across the loop back-edge, and the
    // operator registers are not carried around the loop (a conditional
    // reload there would make the compiler copy all of them, and wait for
    // the copies, on every iteration).  Every step issues the same loads
    // (past the wave's last unit, an empty tile that loads nothing), so the
    // compiler's memory-counter waits are exact.  A run that ends on the
    // second buffer hands its next unit to the first one with a copy.
    JobCursor<kUnitBlocks8> jc;
    int64_t unit = first, k = 0;
    jc.start(a.jobs8, job_begin, job_end, unit);
    UnitRef rc = jc.at(unit), rn;
    float4 b0[4], b1[4];
    load_unit(b0, rc);
    auto step = [&](float4 (&cb)[4], float4 (&nb)[4]) -> bool {
        const bool more = k + 1 < my_units;
        if (more) {
            unit += stride;
            rn = jc.at(unit);
        } else {
            rn = rc;
            rn.B = 0;
        }
        jc.refill();
        load_unit(nb, rn);
        compute_store(cb, rc);
        ++k;
        rc = rn;
        return more;
    };
    for (;;) {
        const int op = rc.op;
        op_load(op);
        if (!step(b0, b1))
            return;
        if (rc.op != op) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                b0[i] = b1[i];
            continue;
        }
        for (;;) {
            if (!step(b1, b0))
                return;
            if (rc.op != op)
                break;
            if (!step(b0, b1))
                return;
            if (rc.op != op) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    b0[i] = b1[i];
                break;
            }
        }
    }
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
    run_tiles16<PREC, D, UnitRef, 0, 0, true>(count, ref, op_load, R, smem);
}

template <int PREC, int IO, bool NT>
__global__ __launch_bounds__(kBatchThreads) void k_batch(BatchArgs a)
{
    static_assert(IO != 2, "the mixed kernel stages N = 8 tiles through registers");
    // N = 16 workgroups use the LDS for their double-buffered tiles, N = 8
    // workgroups for the per-wave staging of the coalesced I/O.
    constexpr int k16 = PREC == DCTF_PREC_FP32 ? kSmem16F32 : kSmem16Split;
    constexpr int k8 = IO ? (kBatchThreads / 64) * 256 * 16 : 0;
    constexpr int kBytes = k16 > k8 ? k16 : k8;
    __shared__ __attribute__((aligned(16))) char smem[kBytes];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if ((int)blockIdx.x < a.groups8) {
        float4 *lds = reinterpret_cast<float4 *>(smem) + (IO ? wave * 256 : 0);
        worker8<PREC, IO, NT>(a, uniform_i64((int64_t)blockIdx.x * (kBatchThreads / 64) + wave), lane, lds, nullptr,
                              nullptr);
    } else {
        worker16<PREC, batch_depth16(PREC)>(a, (int64_t)blockIdx.x - a.groups8, smem);
    }
}

// Batches of one block size run a kernel holding only that worker, so the
// register allocation and schedule are those of the worker alone.
template <int PREC, int IO, bool NT>
__global__ __launch_bounds__(kBatch8Threads) void k_batch8(BatchArgs a)
{
    constexpr int W = kBatch8Threads / 64;
    __shared__ __attribute__((aligned(16))) float4 lds_all[IO == 1 ? W * 256 : 1];
    __shared__ __attribute__((aligned(16))) float4 lds_t0[IO == 2 ? W : 1][256];
    __shared__ __attribute__((aligned(16))) float4 lds_t1[IO == 2 ? W : 1][256];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    worker8<PREC, IO, NT>(a, uniform_i64((int64_t)blockIdx.x * W + wave), lane, lds_all + (IO == 1 ? wave * 256 : 0),
                          lds_t0[IO == 2 ? wave : 0], lds_t1[IO == 2 ? wave : 0]);
}

template <int PREC>
__global__ __launch_bounds__(kBatchThreads) void k_batch16(BatchArgs a)
{
    __shared__ __attribute__((aligned(16))) char smem[PREC == DCTF_PREC_FP32 ? kSmem16F32 : kSmem16Split];
    worker16<PREC, batch_depth16(PREC)>(a, blockIdx.x, smem);
}

// The mixed kernel has no LDS-load path: a plan of both block sizes runs
// its N = 8 work through the LDS-staged register path instead.
constexpr int mixed_io(int io) { return io == 2 ? 1 : io; }

template <int PREC, int IO, bool NT>
hipError_t launch_batch_t(const BatchArgs &a, hipStream_t stream)
{
    if (a.groups16 == 0)
        hipLaunchKernelGGL((k_batch8<PREC, IO, NT>), dim3(a.groups8), dim3(kBatch8Threads), 0, stream, a);
    else if (a.groups8 == 0)
        hipLaunchKernelGGL((k_batch16<PREC>), dim3(a.groups16), dim3(kBatchThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((k_batch<PREC, mixed_io(IO), NT>), dim3(a.groups8 + a.groups16), dim3(kBatchThreads), 0,
                           stream, a);
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
    return occ(k_batch<PREC, mixed_io(IO), NT>, kBatchThreads);
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
    case 3: return f32 ? launch_batch_t<DCTF_PREC_FP32, 1, true>(a, stream) : launch_batch_t<DCTF_PREC_SPLIT_BF16, 1, true>(a, stream);
    case 4: return f32 ? launch_batch_t<DCTF_PREC_FP32, 2, false>(a, stream) : launch_batch_t<DCTF_PREC_SPLIT_BF16, 2, false>(a, stream);
    default: return f32 ? launch_batch_t<DCTF_PREC_FP32, 2, true>(a, stream) : launch_batch_t<DCTF_PREC_SPLIT_BF16, 2, true>(a, stream);
    }
}

int batch_occupancy(int prec, int io, bool nt, int kind)
{
    const bool f32 = prec == DCTF_PREC_FP32;
    switch (io * 2 + (nt ? 1 : 0)) {
    case 0: return f32 ? occupancy_t<DCTF_PREC_FP32, 0, false>(kind) : occupancy_t<DCTF_PREC_SPLIT_BF16, 0, false>(kind);
    case 1: return f32 ? occupancy_t<DCTF_PREC_FP32, 0, true>(kind) : occupancy_t<DCTF_PREC_SPLIT_BF16, 0, true>(kind);
    case 2: return f32 ? occupancy_t<DCTF_PREC_FP32, 1, false>(kind) : occupancy_t<DCTF_PREC_SPLIT_BF16, 1, false>(kind);
    case 3: return f32 ? occupancy_t<DCTF_PREC_FP32, 1, true>(kind) : occupancy_t<DCTF_PREC_SPLIT_BF16, 1, true>(kind);
    case 4: return f32 ? occupancy_t<DCTF_PREC_FP32, 2, false>(kind) : occupancy_t<DCTF_PREC_SPLIT_BF16, 2, false>(kind);
    default: return f32 ? occupancy_t<DCTF_PREC_FP32, 2, true>(kind) : occupancy_t<DCTF_PREC_SPLIT_BF16, 2, true>(kind);
    }
}

}  // namespace dctf
