// Host side of the C ABI declared in include/dctf.h: argument validation,
// operator lifetime, dispatch to the kernels, batch plans (work tables,
// persistent launch, HIP graph capture), variant selection and timing.
#include "dctf_internal.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <mutex>
#include <new>
#include <vector>

namespace dctf {


namespace {

constexpr int kMaxDevices = 64;
std::atomic<int> g_cu[kMaxDevices];

std::mutex g_variant_mu;
int g_variant[17][2];   // [N][prec]; zero-initialised = default variant 0
std::atomic<int> g_batch_fronts{-1};   // -1: the default of each precision
std::mutex g_batch_cfg_mu;
// Process-wide batch configuration per precision ([prec]); -1 / 0 fields:
// fronts from dctf_set_batch_fronts (or the precision's default), I/O path
// of the current N = 8 variant, as many workgroups per CU as fit.
dctf_batch_config g_batch_cfg[2] = {{-1, -1, 0, 0}, {-1, -1, 0, 0}};

// Block sizes of the kernels around the filter (forward DCT, verify,
// tuning) and of every operator path but the N = 32 dense filter.
bool supported_n(int N) { return N == 2 || N == 4 || N == 8 || N == 16; }
// Block sizes an operator can be built for.
bool supported_op_n(int N) { return supported_n(N) || N == 32; }

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb)
{
    uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return na > 0 && nb > 0 && a0 < b0 + nb && b0 < a0 + na;
}

dctf_status hip_status(hipError_t e)
{
    if (e == hipSuccess)
        return DCTF_OK;
    if (e == hipErrorOutOfMemory)
        return DCTF_ENOMEM;
    return DCTF_EHIP;
}

int current_variant(int N, int prec)
{
    std::lock_guard<std::mutex> lk(g_variant_mu);
    return g_variant[N][prec];
}

// ------------------------------------------------------------- timing
struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> ev;   // pairs
    int used = 0;                 // pairs recorded since the last read
};
Timing g_timing;
constexpr int kTimingPairs = 512;

void timing_begin(hipStream_t s, int *slot)
{
    *slot = -1;
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (!g_timing.on || g_timing.used >= kTimingPairs)
        return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return;
    if (g_timing.ev.empty()) {
        g_timing.ev.resize(2 * kTimingPairs);
        for (auto &e : g_timing.ev)
            if (hipEventCreate(&e) != hipSuccess)
                e = nullptr;
    }
    *slot = g_timing.used++;
    hipEventRecord(g_timing.ev[2 * *slot], s);
}

void timing_end(hipStream_t s, int slot)
{
    if (slot < 0)
        return;
    hipEventRecord(g_timing.ev[2 * slot + 1], s);
}

}  // namespace

int cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return 256;
    int v = g_cu[dev].load();
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        g_cu[dev].store(v);
    }
    return v;
}

int batch_fronts() { return g_batch_fronts.load(); }

// Fronts for a plan of the given precision: the set value, or the default
// (split-BF16 2, FP32 4: the FP32 batch reloads a larger operator at each
// crossing and prefers more, shorter fronts).
static int plan_fronts(int prec)
{
    const int f = batch_fronts();
    return f >= 0 ? f : (prec == DCTF_PREC_FP32 ? 4 : 2);
}
void set_batch_fronts(int fronts) { g_batch_fronts.store(fronts); }

dctf_batch_config batch_config(int prec)
{
    std::lock_guard<std::mutex> lk(g_batch_cfg_mu);
    return g_batch_cfg[prec == DCTF_PREC_FP32 ? 0 : 1];
}

}  // namespace dctf

using namespace dctf;

// ================================================================ operators

static dctf_status validate_mask(const double *mask, int kh, int kw, int N, int border)
{
    if (!supported_op_n(N))
        return (N > 0 && N <= 64) ? DCTF_EUNSUPPORTED : DCTF_EINVAL;
    if (mask == nullptr || kh < 1 || kw < 1 || kh > 2 * N + 1 || kw > 2 * N + 1)
        return DCTF_EINVAL;
    if (border != DCTF_BORDER_ZERO && border != DCTF_BORDER_REPLICATE)
        return DCTF_EINVAL;
    for (int i = 0; i < kh * kw; ++i)
        if (!isfinite(mask[i]))
            return DCTF_EINVAL;
    return DCTF_OK;
}

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Complete-pivoting elimination of the mask: each step takes the largest
// remaining entry as pivot and removes the rank-one term through it (column
// times row / pivot), until the remainder is below 1e-14 of the largest mask
// entry.  The two vectors of a term are scaled to equal largest magnitude.
int dctf::mask_rank_factors(const double *W, int kh, int kw, std::vector<double> &a, std::vector<double> &b)
{
    std::vector<double> E(W, W + (size_t)kh * kw);
    double wmax = 0.0;
    for (double v : E)
        wmax = std::max(wmax, std::fabs(v));
    int rank = 0;
    while (wmax > 0.0 && rank < std::min(kh, kw)) {
        int pi = 0, pj = 0;
        double best = -1.0;
        for (int i = 0; i < kh; ++i)
            for (int j = 0; j < kw; ++j)
                if (std::fabs(E[(size_t)i * kw + j]) > best) {
                    best = std::fabs(E[(size_t)i * kw + j]);
                    pi = i;
                    pj = j;
                }
        if (best <= 1e-14 * wmax)
            break;
        const double piv = E[(size_t)pi * kw + pj];
        std::vector<double> col(kh), row(kw);
        for (int i = 0; i < kh; ++i)
            col[i] = E[(size_t)i * kw + pj];
        for (int j = 0; j < kw; ++j)
            row[j] = E[(size_t)pi * kw + j] / piv;
        for (int i = 0; i < kh; ++i)
            for (int j = 0; j < kw; ++j)
                E[(size_t)i * kw + j] -= col[i] * row[j];
        double ca = 0.0, rb = 0.0;
        for (double v : col)
            ca = std::max(ca, std::fabs(v));
        for (double v : row)
            rb = std::max(rb, std::fabs(v));
        const double f = std::sqrt(rb / ca);   // ca, rb > 0: both contain the pivot
        for (double v : col)
            a.push_back(v * f);
        for (double v : row)
            b.push_back(v / f);
        ++rank;
    }
    if (rank == 0) {
        a.insert(a.end(), kh, 0.0);
        b.insert(b.end(), kw, 0.0);
        rank = 1;
    }
    return rank;
}

// Mirror-symmetric on both axes with odd sides: then the correlation window
// is centred and the block's mirror images are filtered alike.  Entries may
// differ from their mirror images by 1e-12 of the largest entry (a mask
// averaged with its mirror images in floating point); the coupling between
// parity classes that this leaves is of the same relative size, far below
// FP32 rounding, and the class operators leave it out.
static bool mask_doubly_symmetric(const double *W, int kh, int kw)
{
    if (kh % 2 == 0 || kw % 2 == 0)
        return false;
    double m = 0.0;
    for (int e = 0; e < kh * kw; ++e)
        m = std::max(m, std::fabs(W[e]));
    const double tol = 1e-12 * m;
    for (int i = 0; i < kh; ++i)
        for (int j = 0; j < kw; ++j)
            if (std::fabs(W[i * kw + j] - W[(kh - 1 - i) * kw + j]) > tol ||
                std::fabs(W[i * kw + j] - W[i * kw + (kw - 1 - j)]) > tol)
                return false;
    return true;
}

static dctf_status alloc_operator(int N, int kh, int kw, int border, int rank, bool parity, dctf_operator *out)
{
    const size_t NN = (size_t)N * N, N4 = NN * NN, F = frag_elems(N);
    // split-BF16 images exist for N = 8, 16 and 32; the pixel-domain set for N <= 16
    const bool split = N == 8 || N == 16 || N == 32;
    const size_t FS = split ? F : 0;
    const size_t FL = N == 32 ? n32_lf_elems : split ? frag_lf_elems(N) : 0;
    // DCT-domain H for every N, the pixel-domain G for N <= 16, the
    // pixel-to-pixel set for N = 8
    const int domains = N == 8 ? 3 : (N <= 16 ? 2 : 1);
    size_t off = 0;
    const size_t o_mask = off; off = align_up(off + sizeof(double) * kh * kw);
    // one dense image set per domain
    size_t o_h64[3], o_h32[3], o_f32[3], o_fhi[3], o_flo[3], o_flf[3], o_h0[3], o_flo2 = 0;
    for (int d = 0; d < domains; ++d) {
        o_h64[d] = off; off = align_up(off + sizeof(double) * N4);
        o_h32[d] = off; off = align_up(off + sizeof(float) * N4);
        o_f32[d] = off; off = align_up(off + sizeof(float) * F);
        o_fhi[d] = off; off = align_up(off + sizeof(uint16_t) * FS);
        o_flo[d] = off; off = align_up(off + sizeof(uint16_t) * FS);
        o_flf[d] = off; off = align_up(off + sizeof(float) * FL);
        o_h0[d] = off;  off = align_up(off + sizeof(float) * NN);
        if (d == 2) {
            o_flo2 = off; off = align_up(off + sizeof(uint16_t) * FS);
        }
    }
    const size_t o_fa = off;   off = align_up(off + sizeof(double) * rank * kh);
    const size_t o_fb = off;   off = align_up(off + sizeof(double) * rank * kw);
    const size_t o_p64 = off;  off = align_up(off + sizeof(double) * rank * NN);
    const size_t o_q64 = off;  off = align_up(off + sizeof(double) * rank * NN);
    const size_t o_p32 = off;  off = align_up(off + sizeof(float) * rank * NN);
    const size_t o_q32 = off;  off = align_up(off + sizeof(float) * rank * NN);
    // parity-class images (N = 16 and 32, doubly symmetric masks): four sets
    // of the N / 2 block size's images (K = N^2 / 4 class coefficients)
    parity = parity && (N == 16 || N == 32);
    const size_t K = NN / 4;
    size_t o_par = off;
    const size_t par_f32 = align_up(sizeof(float) * (K * K + K + K * lf_count(N / 2)));
    const size_t par_bytes = par_f32 + 2 * align_up(sizeof(uint16_t) * K * K);
    if (parity)
        off += 4 * par_bytes;

    dctf_operator op = new (std::nothrow) dctf_operator_s();
    if (!op)
        return DCTF_ENOMEM;
    void *base = nullptr;
    hipError_t e = hipMalloc(&base, off);
    if (e != hipSuccess) {
        delete op;
        return hip_status(e);
    }
    char *b = static_cast<char *>(base);
    op->N = N;
    op->kh = kh;
    op->kw = kw;
    op->border = border;
    hipGetDevice(&op->device);
    op->base = base;
    op->bytes = off;
    op->img.mask = reinterpret_cast<double *>(b + o_mask);
    op->img.dct = DenseImages{};
    op->img.pix = DenseImages{};
    op->img.pp = DenseImages{};
    for (int d = 0; d < domains; ++d) {
        DenseImages &D = d == 0 ? op->img.dct : (d == 1 ? op->img.pix : op->img.pp);
        D.H64 = reinterpret_cast<double *>(b + o_h64[d]);
        D.H32 = reinterpret_cast<float *>(b + o_h32[d]);
        D.frag32 = F ? reinterpret_cast<float *>(b + o_f32[d]) : nullptr;
        D.frag_hi = FS ? reinterpret_cast<uint16_t *>(b + o_fhi[d]) : nullptr;
        D.frag_lo = FS ? reinterpret_cast<uint16_t *>(b + o_flo[d]) : nullptr;
        D.frag_lf = FL ? reinterpret_cast<float *>(b + o_flf[d]) : nullptr;
        D.h0 = reinterpret_cast<float *>(b + o_h0[d]);
        D.frag_lo2 = d == 2 ? reinterpret_cast<uint16_t *>(b + o_flo2) : nullptr;
    }
    op->rank = rank;
    op->img.fac_a = reinterpret_cast<double *>(b + o_fa);
    op->img.fac_b = reinterpret_cast<double *>(b + o_fb);
    op->img.P64 = reinterpret_cast<double *>(b + o_p64);
    op->img.Q64 = reinterpret_cast<double *>(b + o_q64);
    op->img.P32 = reinterpret_cast<float *>(b + o_p32);
    op->img.Q32 = reinterpret_cast<float *>(b + o_q32);
    op->parity = parity ? 1 : 0;
    for (int c = 0; c < 4; ++c) {
        DenseImages &P = op->par[c];
        P = DenseImages{};
        if (!parity)
            continue;
        char *q = b + o_par + c * par_bytes;
        P.frag32 = reinterpret_cast<float *>(q);
        P.h0 = P.frag32 + K * K;
        P.frag_lf = P.h0 + K;
        q += par_f32;
        P.frag_hi = reinterpret_cast<uint16_t *>(q);
        P.frag_lo = reinterpret_cast<uint16_t *>(q + align_up(sizeof(uint16_t) * K * K));
    }
    *out = op;
    return DCTF_OK;
}

static dctf_status launch_rebuild(const dctf_operator *ops, int n, hipStream_t s, unsigned parts)
{
    for (int first = 0; first < n; first += kMaxBuildPerLaunch) {
        BuildArgs args;
        memset(&args, 0, sizeof(args));
        args.n = std::min(kMaxBuildPerLaunch, n - first);
        args.parts = parts;
        for (int i = 0; i < args.n; ++i) {
            const dctf_operator op = ops[first + i];
            args.d[i].img = op->img;
            args.d[i].N = op->N;
            args.d[i].kh = op->kh;
            args.d[i].kw = op->kw;
            args.d[i].border = op->border;
            args.d[i].rank = op->rank;
        }
        dctf_status st = hip_status(launch_build(args, s));
        if (st != DCTF_OK)
            return st;
    }
    // the N = 32 split-BF16 images and the N = 16 and 32 parity-class images, from
    // the FP64 operator just built (batches, which rebuild only what they
    // read, leave the parity classes alone)
    for (int i = 0; i < n && (parts & kBuildDct); ++i) {
        const DenseImages &D = ops[i]->img.dct;
        dctf_status st = DCTF_OK;
        if (ops[i]->N == 32)
            st = hip_status(launch_split_n32(D.H64, D.frag_hi, D.frag_lo, D.frag_lf, s));
        if (st == DCTF_OK && ops[i]->parity && (parts & kBuildParity))
            st = hip_status(launch_build_parity(ops[i]->N, D.H64, ops[i]->par, s));
        if (st != DCTF_OK)
            return st;
    }
    return DCTF_OK;
}

extern "C" dctf_status dctf_build_operators(const dctf_mask_desc *masks, int n, dctf_stream stream,
                                            dctf_operator *out)
{
    if (n < 0 || (n > 0 && (masks == nullptr || out == nullptr)))
        return DCTF_EINVAL;
    for (int i = 0; i < n; ++i) {
        dctf_status st = validate_mask(masks[i].mask_host, masks[i].kh, masks[i].kw, masks[i].N,
                                       masks[i].border);
        if (st != DCTF_OK)
            return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<dctf_operator> ops(n, nullptr);
    // host-side rank factors, kept alive until the stream has consumed them
    std::vector<std::vector<double>> fa(n), fb(n);
    dctf_status st = DCTF_OK;
    for (int i = 0; i < n && st == DCTF_OK; ++i) {
        const int kh = masks[i].kh, kw = masks[i].kw;
        const int rank = mask_rank_factors(masks[i].mask_host, kh, kw, fa[i], fb[i]);
        st = alloc_operator(masks[i].N, kh, kw, masks[i].border, rank,
                            mask_doubly_symmetric(masks[i].mask_host, kh, kw), &ops[i]);
        if (st == DCTF_OK)
            st = hip_status(hipMemcpyAsync(ops[i]->img.mask, masks[i].mask_host, sizeof(double) * kh * kw,
                                           hipMemcpyHostToDevice, s));
        if (st == DCTF_OK)
            st = hip_status(hipMemcpyAsync(ops[i]->img.fac_a, fa[i].data(), sizeof(double) * rank * kh,
                                           hipMemcpyHostToDevice, s));
        if (st == DCTF_OK)
            st = hip_status(hipMemcpyAsync(ops[i]->img.fac_b, fb[i].data(), sizeof(double) * rank * kw,
                                           hipMemcpyHostToDevice, s));
    }
    if (st == DCTF_OK)
        st = launch_rebuild(ops.data(), n, s, kBuildAll);
    // The mask and factor copies are from pageable memory: make them complete
    // before the caller may free its masks.
    if (st == DCTF_OK)
        st = hip_status(hipStreamSynchronize(s));
    if (st != DCTF_OK) {
        for (auto op : ops)
            dctf_operator_destroy(op);
        return st;
    }
    for (int i = 0; i < n; ++i)
        out[i] = ops[i];
    return DCTF_OK;
}

extern "C" dctf_status dctf_build_operator(const double *mask_host, int kh, int kw, int N, int border,
                                           dctf_stream stream, dctf_operator *out)
{
    if (out == nullptr)
        return DCTF_EINVAL;
    dctf_mask_desc d = {mask_host, kh, kw, N, border};
    return dctf_build_operators(&d, 1, stream, out);
}

extern "C" dctf_status dctf_rebuild_operators(const dctf_operator *ops, int n, dctf_stream stream)
{
    if (n < 0 || (n > 0 && ops == nullptr))
        return DCTF_EINVAL;
    for (int i = 0; i < n; ++i)
        if (ops[i] == nullptr)
            return DCTF_EINVAL;
    return launch_rebuild(ops, n, static_cast<hipStream_t>(stream), kBuildAll);
}

extern "C" dctf_status dctf_operator_fp64(dctf_operator op, double *host_out)
{
    if (op == nullptr || host_out == nullptr)
        return DCTF_EINVAL;
    const size_t NN = (size_t)op->N * op->N;
    return hip_status(hipMemcpy(host_out, op->img.dct.H64, sizeof(double) * NN * NN, hipMemcpyDeviceToHost));
}

extern "C" dctf_status dctf_operator_pixel_fp64(dctf_operator op, double *host_out)
{
    if (op == nullptr || host_out == nullptr)
        return DCTF_EINVAL;
    if (op->img.pix.H64 == nullptr)
        return DCTF_EUNSUPPORTED;
    const size_t NN = (size_t)op->N * op->N;
    return hip_status(hipMemcpy(host_out, op->img.pix.H64, sizeof(double) * NN * NN, hipMemcpyDeviceToHost));
}

extern "C" dctf_status dctf_operator_info(dctf_operator op, int *N, int *kh, int *kw, int *border)
{
    if (op == nullptr)
        return DCTF_EINVAL;
    if (N)
        *N = op->N;
    if (kh)
        *kh = op->kh;
    if (kw)
        *kw = op->kw;
    if (border)
        *border = op->border;
    return DCTF_OK;
}

extern "C" void dctf_operator_destroy(dctf_operator op)
{
    if (op == nullptr)
        return;
    if (op->base)
        hipFree(op->base);
    delete op;
}

// =================================================================== filter

static dctf_status validate_io(int N, const float *in, const float *out, int64_t B)
{
    if (B < 0)
        return DCTF_EINVAL;
    if (B == 0)
        return DCTF_OK;
    if (in == nullptr || out == nullptr || !aligned16(in) || !aligned16(out))
        return DCTF_EINVAL;
    const size_t bytes = (size_t)B * N * N * sizeof(float);
    if (ranges_overlap(in, bytes, out, bytes))
        return DCTF_EINVAL;
    return DCTF_OK;
}

static FilterArgs filter_args(dctf_operator op, const float *in, float *out, int64_t B)
{
    FilterArgs a;
    a.in = in;
    a.out = out;
    a.B = B;
    a.frag32 = op->img.dct.frag32;
    a.frag_hi = op->img.dct.frag_hi;
    a.frag_lo = op->img.dct.frag_lo;
    a.frag_lf = op->img.dct.frag_lf;
    a.h0 = op->img.dct.h0;
    a.H32 = op->img.dct.H32;
    return a;
}

extern "C" dctf_status dctf_filter_blocks(dctf_operator op, int prec, const float *in_dev, float *out_dev,
                                          int64_t B, dctf_stream stream)
{
    if (op == nullptr)
        return DCTF_EINVAL;
    if (prec != DCTF_PREC_FP32 && prec != DCTF_PREC_SPLIT_BF16)
        return DCTF_EINVAL;
    dctf_status st = validate_io(op->N, in_dev, out_dev, B);
    if (st != DCTF_OK || B == 0)
        return st;
    const FilterArgs a = filter_args(op, in_dev, out_dev, B);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int slot;
    timing_begin(s, &slot);
    if (op->N == 32)
        st = hip_status(launch_filter_n32(prec, a, s));
    else
        st = hip_status(launch_filter(op->N, prec, current_variant(op->N, prec), a, s));
    timing_end(s, slot);
    return st;
}

extern "C" dctf_status dctf_operator_parity_classes(dctf_operator op, int *classes)
{
    if (op == nullptr || classes == nullptr)
        return DCTF_EINVAL;
    *classes = op->parity ? 4 : 1;
    return DCTF_OK;
}

extern "C" dctf_status dctf_filter_blocks_parity(dctf_operator op, int prec, const float *in_dev, float *out_dev,
                                                 int64_t B, dctf_stream stream)
{
    if (op == nullptr || (prec != DCTF_PREC_FP32 && prec != DCTF_PREC_SPLIT_BF16))
        return DCTF_EINVAL;
    dctf_status st = validate_io(op->N, in_dev, out_dev, B);
    if (st != DCTF_OK)
        return st;
    if (!op->parity)
        return DCTF_EUNSUPPORTED;
    if (B == 0)
        return DCTF_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int slot;
    timing_begin(s, &slot);
    st = hip_status(op->N == 16 ? launch_filter_n16_parity(prec, op->par, in_dev, out_dev, B, s)
                                : launch_filter_n32_parity(prec, op->par, in_dev, out_dev, B, s));
    timing_end(s, slot);
    return st;
}

extern "C" dctf_status dctf_operator_rank(dctf_operator op, int *rank)
{
    if (op == nullptr || rank == nullptr)
        return DCTF_EINVAL;
    *rank = op->rank;
    return DCTF_OK;
}

extern "C" dctf_status dctf_operator_factors_fp64(dctf_operator op, double *P_host, double *Q_host)
{
    if (op == nullptr || P_host == nullptr || Q_host == nullptr)
        return DCTF_EINVAL;
    const size_t bytes = sizeof(double) * op->rank * op->N * op->N;
    dctf_status st = hip_status(hipMemcpy(P_host, op->img.P64, bytes, hipMemcpyDeviceToHost));
    if (st == DCTF_OK)
        st = hip_status(hipMemcpy(Q_host, op->img.Q64, bytes, hipMemcpyDeviceToHost));
    return st;
}

extern "C" dctf_status dctf_filter_blocks_factored(dctf_operator op, const float *in_dev, float *out_dev,
                                                   int64_t B, dctf_stream stream)
{
    if (op == nullptr)
        return DCTF_EINVAL;
    if ((op->N != 16 && op->N != 32) || op->rank > kFactoredMaxRank)
        return DCTF_EUNSUPPORTED;
    dctf_status st = validate_io(op->N, in_dev, out_dev, B);
    if (st != DCTF_OK || B == 0)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int slot;
    timing_begin(s, &slot);
    st = hip_status(launch_filter_factored(op->N, op->rank, op->img.P32, op->img.Q32, op->img.dct.h0, in_dev,
                                           out_dev, B, s));
    timing_end(s, slot);
    return st;
}

extern "C" dctf_status dctf_filter_blocks_f64(dctf_operator op, const double *in_dev, double *out_dev, int64_t B,
                                              dctf_stream stream)
{
    if (op == nullptr || B < 0)
        return DCTF_EINVAL;
    if (B == 0)
        return DCTF_OK;
    const size_t bytes = (size_t)B * op->N * op->N * sizeof(double);
    if (in_dev == nullptr || out_dev == nullptr || !aligned16(in_dev) || !aligned16(out_dev) ||
        ranges_overlap(in_dev, bytes, out_dev, bytes))
        return DCTF_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int slot;
    timing_begin(s, &slot);
    dctf_status st = hip_status(launch_filter_f64(op->N, op->img.dct.H64, in_dev, out_dev, B, s));
    timing_end(s, slot);
    return st;
}

// ============================================================ pixel output

// raster: the pixels go into the h x w image `pix` (row pitch `pitch`)
// instead of block by block; B is then the image's block count.
struct RasterOut {
    int h = 0, w = 0;
    int64_t pitch = 0;
    int64_t nimg = 1, img_stride = 0;
};

static dctf_status filter_px(dctf_operator op, int prec, int in_kind, const void *in, const float *qtab,
                             float dc_offset, uint8_t *pix, int64_t B, dctf_stream stream,
                             const RasterOut *raster = nullptr)
{
    if (op == nullptr)
        return DCTF_EINVAL;
    if (op->img.pix.H64 == nullptr)
        return DCTF_EUNSUPPORTED;
    if (prec != DCTF_PREC_FP32 && prec != DCTF_PREC_SPLIT_BF16)
        return DCTF_EINVAL;
    if (B < 0 || !std::isfinite(dc_offset))
        return DCTF_EINVAL;
    if (B == 0)
        return DCTF_OK;
    const size_t nn = (size_t)op->N * op->N;
    const size_t in_bytes = (size_t)B * nn * (in_kind ? sizeof(int16_t) : sizeof(float));
    // bytes of the output: block by block, or the raster image up to its last pixel
    const size_t out_bytes = raster ? (size_t)(raster->nimg - 1) * raster->img_stride +
                                          (size_t)(raster->h - 1) * raster->pitch + raster->w
                                    : (size_t)B * nn;
    const bool out_aligned = raster ? reinterpret_cast<uintptr_t>(pix) % 4 == 0 : aligned16(pix);
    if (in == nullptr || pix == nullptr || !aligned16(in) || !out_aligned)
        return DCTF_EINVAL;
    if (in_kind && (qtab == nullptr || !aligned16(qtab) || ranges_overlap(qtab, nn * sizeof(float), pix, out_bytes)))
        return DCTF_EINVAL;
    if (ranges_overlap(in, in_bytes, pix, out_bytes))
        return DCTF_EINVAL;
    PxArgs a;
    a.raster = raster ? 1 : 0;
    a.h = raster ? raster->h : 0;
    a.w = raster ? raster->w : 0;
    a.Bw = raster ? (raster->w + op->N - 1) / op->N : 0;
    a.bpi = raster ? (int)(B / raster->nimg) : 0;
    a.pitch = raster ? raster->pitch : 0;
    a.img_stride = raster ? raster->img_stride : 0;
    div_magic((uint32_t)(raster ? a.bpi : 1), a.magic);
    div_magic((uint32_t)(raster ? a.Bw : 1), a.magic + 2);
    a.in = in_kind ? nullptr : static_cast<const float *>(in);
    a.qin = in_kind ? static_cast<const int16_t *>(in) : nullptr;
    a.qtab = qtab;
    a.dc_offset = dc_offset;
    a.pix = pix;
    a.B = B;
    a.G = op->img.pix;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int slot;
    timing_begin(s, &slot);
    dctf_status st = hip_status(launch_filter_px(op->N, prec, in_kind, a, s));
    timing_end(s, slot);
    return st;
}

extern "C" dctf_status dctf_filter_blocks_u8(dctf_operator op, int prec, const float *in_dev, uint8_t *pix_dev,
                                             int64_t B, dctf_stream stream)
{
    return filter_px(op, prec, 0, in_dev, nullptr, 0.0f, pix_dev, B, stream);
}

extern "C" dctf_status dctf_filter_quantized_u8(dctf_operator op, int prec, const int16_t *qcoef_dev,
                                                const float *qtable_dev, float dc_offset, uint8_t *pix_dev,
                                                int64_t B, dctf_stream stream)
{
    return filter_px(op, prec, 1, qcoef_dev, qtable_dev, dc_offset, pix_dev, B, stream);
}

// The raster forms: the block count follows from the image size; the images
// must fit the kernels' 32-bit block and row arithmetic (fewer than 2^32
// blocks in all: at 128 bytes of input and output per block or more, more
// than the memory of the device could hold).
static dctf_status filter_px_raster(dctf_operator op, int prec, int in_kind, const void *in, const float *qtab,
                                    float dc_offset, int h, int w, int64_t nimg, uint8_t *img, int64_t pitch,
                                    int64_t img_stride, dctf_stream stream)
{
    if (op == nullptr || h < 0 || w < 0 || nimg < 0 || pitch < w || pitch % 4 != 0)
        return DCTF_EINVAL;
    if (h == 0 || w == 0 || nimg == 0)
        return DCTF_OK;
    // images one after another, not overlapping, each 4-byte aligned
    if (nimg > 1 && (img_stride % 4 != 0 || img_stride < (int64_t)(h - 1) * pitch + w))
        return DCTF_EINVAL;
    const int64_t bpi = (int64_t)((h + op->N - 1) / op->N) * ((w + op->N - 1) / op->N);
    if (bpi > INT32_MAX || nimg > (int64_t)UINT32_MAX / bpi)
        return DCTF_EINVAL;
    RasterOut r;
    r.h = h;
    r.w = w;
    r.pitch = pitch;
    r.nimg = nimg;
    r.img_stride = nimg > 1 ? img_stride : 0;
    return filter_px(op, prec, in_kind, in, qtab, dc_offset, img, bpi * nimg, stream, &r);
}

extern "C" dctf_status dctf_filter_blocks_u8_raster(dctf_operator op, int prec, const float *in_dev, int h, int w,
                                                    int64_t nimg, uint8_t *img_dev, int64_t pitch,
                                                    int64_t img_stride, dctf_stream stream)
{
    return filter_px_raster(op, prec, 0, in_dev, nullptr, 0.0f, h, w, nimg, img_dev, pitch, img_stride, stream);
}

extern "C" dctf_status dctf_filter_quantized_u8_raster(dctf_operator op, int prec, const int16_t *qcoef_dev,
                                                       const float *qtable_dev, float dc_offset, int h, int w,
                                                       int64_t nimg, uint8_t *img_dev, int64_t pitch,
                                                       int64_t img_stride, dctf_stream stream)
{
    return filter_px_raster(op, prec, 1, qcoef_dev, qtable_dev, dc_offset, h, w, nimg, img_dev, pitch, img_stride,
                            stream);
}

// One pass from uint8 images to filtered uint8 images (N = 8).
extern "C" dctf_status dctf_filter_u8_raster(dctf_operator op, int prec, const uint8_t *in_dev, int64_t in_pitch,
                                             int64_t in_stride, int h, int w, int64_t nimg, uint8_t *out_dev,
                                             int64_t out_pitch, int64_t out_stride, dctf_stream stream)
{
    if (op == nullptr || (prec != DCTF_PREC_FP32 && prec != DCTF_PREC_SPLIT_BF16))
        return DCTF_EINVAL;
    if (op->N != 8 || op->img.pp.H64 == nullptr)
        return DCTF_EUNSUPPORTED;
    if (h < 0 || w < 0 || nimg < 0 || in_pitch < w || out_pitch < w || in_pitch % 4 != 0 || out_pitch % 4 != 0)
        return DCTF_EINVAL;
    if (h == 0 || w == 0 || nimg == 0)
        return DCTF_OK;
    const int64_t span = (int64_t)(h - 1) * in_pitch + w, ospan = (int64_t)(h - 1) * out_pitch + w;
    if (nimg > 1 && (in_stride % 4 != 0 || out_stride % 4 != 0 || in_stride < span || out_stride < ospan))
        return DCTF_EINVAL;
    if (in_dev == nullptr || out_dev == nullptr || reinterpret_cast<uintptr_t>(in_dev) % 4 != 0 ||
        reinterpret_cast<uintptr_t>(out_dev) % 4 != 0)
        return DCTF_EINVAL;
    const int64_t bpi = (int64_t)((h + 7) / 8) * ((w + 7) / 8);
    if (bpi > INT32_MAX || nimg > (int64_t)UINT32_MAX / bpi)
        return DCTF_EINVAL;
    const int64_t istr = nimg > 1 ? in_stride : 0, ostr = nimg > 1 ? out_stride : 0;
    if (ranges_overlap(in_dev, (size_t)((nimg - 1) * istr + span), out_dev, (size_t)((nimg - 1) * ostr + ospan)))
        return DCTF_EINVAL;
    PxArgs a;
    memset(&a, 0, sizeof(a));
    a.pix = out_dev;
    a.B = bpi * nimg;
    a.G = op->img.pp;
    a.raster = 1;
    a.h = h;
    a.w = w;
    a.Bw = (w + 7) / 8;
    a.bpi = (int)bpi;
    a.pitch = out_pitch;
    a.img_stride = ostr;
    div_magic((uint32_t)a.bpi, a.magic);
    div_magic((uint32_t)a.Bw, a.magic + 2);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int slot;
    timing_begin(s, &slot);
    dctf_status st = hip_status(launch_filter_u8_raster8(prec, a, in_dev, in_pitch, istr, s));
    timing_end(s, slot);
    return st;
}

extern "C" dctf_status dctf_operator_pixpix_fp64(dctf_operator op, double *host_out)
{
    if (op == nullptr || host_out == nullptr)
        return DCTF_EINVAL;
    if (op->img.pp.H64 == nullptr)
        return DCTF_EUNSUPPORTED;
    return hip_status(hipMemcpy(host_out, op->img.pp.H64, sizeof(double) * 4096, hipMemcpyDeviceToHost));
}

// ============================================================ image level

struct dctf_image_operator_s {
    int N, kh, kw, border;
    void *base = nullptr;
    double *mask = nullptr;
    double *H64 = nullptr;
    float *frag32 = nullptr;
    float *h0 = nullptr;
    uint16_t *frag_hi = nullptr;
    uint16_t *frag_lo = nullptr;
    float *frag_lf = nullptr;
};

extern "C" dctf_status dctf_build_image_operator(const double *mask_host, int kh, int kw, int N, int border,
                                                 dctf_stream stream, dctf_image_operator *out)
{
    if (out == nullptr)
        return DCTF_EINVAL;
    dctf_status st = validate_mask(mask_host, kh, kw, N, border);
    if (st != DCTF_OK)
        return st;
    if (N != 8 && N != 16)
        return DCTF_EUNSUPPORTED;
    const size_t NN = (size_t)N * N, nops = (size_t)kImageClassPairs * kImageOffsets;
    size_t off = 0;
    const size_t o_mask = off; off = align_up(off + sizeof(double) * kh * kw);
    const size_t o_h64 = off;  off = align_up(off + sizeof(double) * nops * NN * NN);
    const size_t o_f32 = off;  off = align_up(off + sizeof(float) * nops * NN * NN);
    const size_t o_h0 = off;   off = align_up(off + sizeof(float) * nops * NN);
    const size_t o_fhi = off;  off = align_up(off + sizeof(uint16_t) * nops * NN * NN);
    const size_t o_flo = off;  off = align_up(off + sizeof(uint16_t) * nops * NN * NN);
    const size_t o_flf = off;  off = align_up(off + sizeof(float) * nops * NN * lf_count(N));
    dctf_image_operator op = new (std::nothrow) dctf_image_operator_s();
    if (!op)
        return DCTF_ENOMEM;
    hipError_t e = hipMalloc(&op->base, off);
    if (e != hipSuccess) {
        delete op;
        return hip_status(e);
    }
    char *b = static_cast<char *>(op->base);
    op->N = N;
    op->kh = kh;
    op->kw = kw;
    op->border = border;
    op->mask = reinterpret_cast<double *>(b + o_mask);
    op->H64 = reinterpret_cast<double *>(b + o_h64);
    op->frag32 = reinterpret_cast<float *>(b + o_f32);
    op->h0 = reinterpret_cast<float *>(b + o_h0);
    op->frag_hi = reinterpret_cast<uint16_t *>(b + o_fhi);
    op->frag_lo = reinterpret_cast<uint16_t *>(b + o_flo);
    op->frag_lf = reinterpret_cast<float *>(b + o_flf);
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = hip_status(hipMemcpyAsync(op->mask, mask_host, sizeof(double) * kh * kw, hipMemcpyHostToDevice, s));
    if (st == DCTF_OK) {
        ImageBuildArgs a;
        a.mask = op->mask;
        a.kh = kh;
        a.kw = kw;
        a.border = border;
        a.H64 = op->H64;
        a.frag32 = op->frag32;
        a.frag_hi = op->frag_hi;
        a.frag_lo = op->frag_lo;
        a.frag_lf = op->frag_lf;
        a.h0 = op->h0;
        st = hip_status(launch_build_image(N, a, s));
    }
    // the mask copy is from pageable memory: complete it before returning
    if (st == DCTF_OK)
        st = hip_status(hipStreamSynchronize(s));
    if (st != DCTF_OK) {
        dctf_image_operator_destroy(op);
        return st;
    }
    *out = op;
    return DCTF_OK;
}

extern "C" dctf_status dctf_image_operator_fp64(dctf_image_operator op, int row_class, int col_class, int dr,
                                                int ds, double *host_out)
{
    if (op == nullptr || host_out == nullptr || row_class < 0 || row_class > 3 || col_class < 0 ||
        col_class > 3 || dr < -1 || dr > 1 || ds < -1 || ds > 1)
        return DCTF_EINVAL;
    const size_t NN = (size_t)op->N * op->N;
    const size_t idx = (size_t)(4 * row_class + col_class) * kImageOffsets + 3 * (dr + 1) + (ds + 1);
    return hip_status(hipMemcpy(host_out, op->H64 + idx * NN * NN, sizeof(double) * NN * NN,
                                hipMemcpyDeviceToHost));
}

extern "C" void dctf_image_operator_destroy(dctf_image_operator op)
{
    if (op == nullptr)
        return;
    if (op->base)
        hipFree(op->base);
    delete op;
}

namespace {

struct Run {
    int begin, len, cls;
};

// Runs of equal class along one axis of n blocks (first, interior, last; or
// one block that is both).
int class_runs(int n, Run out[3])
{
    if (n == 1) {
        out[0] = {0, 1, 3};
        return 1;
    }
    int k = 0;
    out[k++] = {0, 1, 1};
    if (n > 2)
        out[k++] = {1, n - 2, 0};
    out[k++] = {n - 1, 1, 2};
    return k;
}

// Neighbour offsets a block of classes (cr, cs) reads: the neighbour exists
// and the mask reaches into it.
int image_offsets(int cr, int cs, int kh, int kw)
{
    const int ah = (kh - 1) / 2, aw = (kw - 1) / 2;
    const bool up = !(cr & 1) && ah > 0, down = !(cr & 2) && kh - 1 - ah > 0;
    const bool left = !(cs & 1) && aw > 0, right = !(cs & 2) && kw - 1 - aw > 0;
    int mask = 0;
    for (int o = 0; o < kImageOffsets; ++o) {
        const int dr = o / 3 - 1, ds = o % 3 - 1;
        const bool rok = dr == 0 || (dr < 0 ? up : down);
        const bool cok = ds == 0 || (ds < 0 ? left : right);
        if (rok && cok)
            mask |= 1 << o;
    }
    return mask;
}

}  // namespace

extern "C" dctf_status dctf_filter_image(dctf_image_operator op, int prec, const float *in_dev, float *out_dev,
                                         int Bh, int Bw, int64_t nimg, dctf_stream stream)
{
    if (op == nullptr || Bh < 1 || Bw < 1 || nimg < 0)
        return DCTF_EINVAL;
    if (prec != DCTF_PREC_FP32 && prec != DCTF_PREC_SPLIT_BF16)
        return DCTF_EINVAL;
    // N = 16 addresses a tile's blocks with 32-bit byte offsets from the tile's
    // first block (16 blocks a block row apart: 16 KiB per block of width)
    if (op->N == 16 && Bw > kImage16MaxBw)
        return DCTF_EUNSUPPORTED;
    const int64_t B = (int64_t)Bh * Bw * nimg;
    dctf_status st = validate_io(op->N, in_dev, out_dev, B);
    if (st != DCTF_OK || B == 0)
        return st;
    ImageFilterArgs a;
    memset(&a, 0, sizeof(a));
    a.in = in_dev;
    a.out = out_dev;
    a.Bh = Bh;
    a.Bw = Bw;
    a.nimg = nimg;
    a.frag32 = op->frag32;
    a.frag_hi = op->frag_hi;
    a.frag_lo = op->frag_lo;
    a.frag_lf = op->frag_lf;
    a.h0 = op->h0;
    Run rr[3], cr[3];
    const int nr = class_runs(Bh, rr), nc = class_runs(Bw, cr);
    const int T = image_tiles_per_unit(op->N, prec);
    int64_t units = 0;
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nc; ++j) {
            ImageRect &r = a.rect[a.nrect++];
            r.R0 = rr[i].begin;
            r.nR = rr[i].len;
            r.S0 = cr[j].begin;
            r.nS = cr[j].len;
            r.cp = 4 * rr[i].cls + cr[j].cls;
            r.dir = (r.nS > 1 || r.nR == 1) ? 0 : 1;
            r.offsets = image_offsets(rr[i].cls, cr[j].cls, op->kh, op->kw);
            r.tiles = r.dir == 0 ? (int64_t)r.nR * ((r.nS + 15) / 16) : (int64_t)r.nS * ((r.nR + 15) / 16);
            r.unit_begin = units;
            units += (r.tiles + T - 1) / T;
        }
    a.units_per_image = units;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int slot;
    timing_begin(s, &slot);
    st = hip_status(launch_filter_image(op->N, prec, a, s));
    timing_end(s, slot);
    return st;
}

// ==================================================================== batch

struct dctf_batch_s {
    int prec = 0;
    std::vector<dctf_job> jobs;       // the caller's jobs (kept for re-planning)
    dctf_batch_config cfg{};          // configuration of the current plan
    std::vector<dctf_operator> ops;   // distinct operators, in table order (then those of side jobs)
    std::vector<dctf_job> side;       // jobs of N = 2, 4 and 32: one launch each after the persistent one
    void *dev = nullptr;              // JobDesc[njobs8] | JobDesc[njobs16] | OpDesc[nops]
    size_t dev_bytes = 0;
    BatchArgs args{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

struct Interval {
    uintptr_t a, b;
    bool out;
};

// Whether an output range overlaps any other range (inputs may overlap
// each other).
bool intervals_conflict(std::vector<Interval> &iv)
{
    std::sort(iv.begin(), iv.end(), [](const Interval &x, const Interval &y) { return x.a < y.a; });
    uintptr_t end_all = 0, end_out = 0;
    for (const auto &v : iv) {
        if (v.out ? v.a < end_all : v.a < end_out)
            return true;
        end_all = std::max(end_all, v.b);
        if (v.out)
            end_out = std::max(end_out, v.b);
    }
    return false;
}

template <typename Job>
bool jobs_conflict_t(const Job *jobs, int n, size_t elem_bytes)
{
    std::vector<Interval> iv;
    iv.reserve(2 * n);
    for (int i = 0; i < n; ++i) {
        if (jobs[i].B == 0)
            continue;
        const size_t bytes = (size_t)jobs[i].B * jobs[i].op->N * jobs[i].op->N * elem_bytes;
        iv.push_back({(uintptr_t)jobs[i].in, (uintptr_t)jobs[i].in + bytes, false});
        iv.push_back({(uintptr_t)jobs[i].out, (uintptr_t)jobs[i].out + bytes, true});
    }
    return intervals_conflict(iv);
}

bool jobs_conflict(const dctf_job *jobs, int n) { return jobs_conflict_t(jobs, n, sizeof(float)); }

}  // namespace

namespace dctf {

dctf_status plan_batch(const dctf_job *jobs, int njobs, int prec, const dctf_batch_config &cfg,
                       std::vector<char> &table, BatchArgs &a, std::vector<dctf_operator> &ops,
                       std::vector<dctf_job> *side)
{
    if (njobs < 0 || (njobs > 0 && jobs == nullptr))
        return DCTF_EINVAL;
    if (prec != DCTF_PREC_FP32 && prec != DCTF_PREC_SPLIT_BF16)
        return DCTF_EINVAL;
    for (int i = 0; i < njobs; ++i) {
        const dctf_job &j = jobs[i];
        if (j.op == nullptr)
            return DCTF_EINVAL;
        if (j.op->N != 8 && j.op->N != 16 && side == nullptr)
            return DCTF_EUNSUPPORTED;
        dctf_status st = validate_io(j.op->N, j.in, j.out, j.B);
        if (st != DCTF_OK)
            return st;
    }
    if (jobs_conflict(jobs, njobs))
        return DCTF_EINVAL;

    // Group by N, then operator (stable in the caller's order otherwise);
    // jobs of the other block sizes run after the persistent launch.
    std::vector<int> order;
    if (side)
        side->clear();
    for (int i = 0; i < njobs; ++i) {
        if (jobs[i].B <= 0)
            continue;
        if (jobs[i].op->N == 8 || jobs[i].op->N == 16)
            order.push_back(i);
        else
            side->push_back(jobs[i]);
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (jobs[x].op->N != jobs[y].op->N)
            return jobs[x].op->N < jobs[y].op->N;
        return jobs[x].op < jobs[y].op;
    });
    ops.clear();
    std::vector<JobDesc> j8, j16;
    std::vector<OpDesc> od;
    int64_t u8 = 0, u16 = 0, blocks8 = 0, blocks16 = 0;
    for (int idx : order) {
        const dctf_job &j = jobs[idx];
        int opi = -1;
        if (!ops.empty() && ops.back() == j.op)   // jobs are grouped by operator
            opi = (int)ops.size() - 1;
        if (opi < 0) {
            opi = (int)ops.size();
            ops.push_back(j.op);
            const DenseImages &D = j.op->img.dct;
            od.push_back({D.frag32, D.frag_hi, D.frag_lo, D.frag_lf, D.h0});
        }
        JobDesc d;
        d.in = j.in;
        d.out = j.out;
        d.B = j.B;
        d.op = opi;
        d.N = j.op->N;
        if (d.N == 8) {
            d.unit_begin = u8;
            u8 += (j.B + kUnitBlocks8 - 1) / kUnitBlocks8;
            blocks8 += j.B;
            j8.push_back(d);
        } else {
            d.unit_begin = u16;
            u16 += (j.B + kUnitBlocks16 - 1) / kUnitBlocks16;
            blocks16 += j.B;
            j16.push_back(d);
        }
    }

    a = BatchArgs{};
    a.prec = prec;
    if (cfg.io >= 0) {
        a.io = cfg.io;
        a.nt = cfg.nt != 0;
    } else {
        variant_io(8, prec, current_variant(8, prec), &a.io, &a.nt);
    }

    // One block size: a kernel holding only that worker, one persistent
    // grid.  Both: the combined kernel, its grid split in proportion to the
    // estimated time (bytes for the HBM-bound cases, MFMA work for N = 16 in
    // FP32).
    const int kind = (u16 == 0) ? 8 : (u8 == 0 ? 16 : 0);
    int occ = std::max(1, batch_occupancy(prec, a.io, a.nt, kind));
    if (cfg.groups_per_cu > 0)
        occ = std::min(occ, cfg.groups_per_cu);
    const int G = std::max(1, cu_count() * occ);
    const int wpg8 = (kind == 8 ? kBatch8Threads : kBatchThreads) / 64;   // waves per N = 8 workgroup
    const double c16 = (prec == DCTF_PREC_FP32) ? 16.0 : 4.0;
    const double w8 = (double)blocks8, w16 = c16 * (double)blocks16;
    int g16 = 0;
    if (u16 > 0)
        g16 = (u8 > 0) ? (int)std::lround(G * w16 / (w8 + w16)) : G;
    if (u16 > 0 && g16 < 1)
        g16 = 1;
    if (u8 > 0 && g16 > G - 1)
        g16 = G - 1;
    const int g8 = (u8 > 0) ? G - g16 : 0;

    // Fronts: runs of consecutive jobs (N = 8: `fronts` runs cut at operator
    // boundaries with about equal units; N = 16: one run per operator), with
    // workers in proportion to their units.
    auto cut = [](const std::vector<JobDesc> &js, int64_t units, int64_t workers, int fronts) {
        std::vector<size_t> starts;   // first job of each operator segment
        for (size_t i = 0; i < js.size(); ++i)
            if (i == 0 || js[i].op != js[i - 1].op)
                starts.push_back(i);
        std::vector<size_t> cuts{0};
        if (fronts > 0) {
            for (int f = 1; f < fronts; ++f) {
                const int64_t target = units * f / fronts;
                size_t best = cuts.back();
                for (size_t st : starts)
                    if (st > cuts.back() && js[st].unit_begin <= target)
                        best = st;
                if (best > cuts.back())
                    cuts.push_back(best);
            }
        } else {
            cuts = starts;
        }
        std::vector<SegDesc> segs;
        int64_t next_worker = 0;
        for (size_t c = 0; c < cuts.size(); ++c) {
            const size_t i = cuts[c], e = (c + 1 < cuts.size()) ? cuts[c + 1] : js.size();
            SegDesc sd;
            sd.unit_begin = js[i].unit_begin;
            sd.unit_end = (e < js.size()) ? js[e].unit_begin : units;
            const int64_t su = sd.unit_end - sd.unit_begin;
            int64_t w = (int64_t)std::llround((double)workers * (double)su / (double)units);
            w = std::max<int64_t>(1, std::min(w, su));
            sd.worker_begin = next_worker;
            sd.nworkers = w;
            next_worker += w;
            sd.job_begin = (int)i;
            sd.job_end = (int)e;
            sd.op = js[i].op;
            segs.push_back(sd);
        }
        return segs;
    };
    const std::vector<SegDesc> s8 = j8.empty() ? std::vector<SegDesc>()
                                               : cut(j8, u8, (int64_t)g8 * wpg8,
                                                     cfg.fronts >= 0 ? cfg.fronts : plan_fronts(prec));
    const std::vector<SegDesc> s16 = j16.empty() ? std::vector<SegDesc>() : cut(j16, u16, g16, 0);
    const int64_t workers8 = s8.empty() ? 0 : s8.back().worker_begin + s8.back().nworkers;
    const int64_t workers16 = s16.empty() ? 0 : s16.back().worker_begin + s16.back().nworkers;

    // Table layout: JobDesc[j8] | JobDesc[j16] | SegDesc[s8] | SegDesc[s16] | OpDesc[ops].
    table.clear();
    auto put = [&](const void *src, size_t n) -> uintptr_t {
        const uintptr_t off = table.size();
        table.resize(off + n);
        if (n)
            memcpy(table.data() + off, src, n);
        return off;
    };
    a.jobs8 = reinterpret_cast<const JobDesc *>(put(j8.data(), sizeof(JobDesc) * j8.size()));
    a.jobs16 = reinterpret_cast<const JobDesc *>(put(j16.data(), sizeof(JobDesc) * j16.size()));
    a.segs8 = reinterpret_cast<const SegDesc *>(put(s8.data(), sizeof(SegDesc) * s8.size()));
    a.segs16 = reinterpret_cast<const SegDesc *>(put(s16.data(), sizeof(SegDesc) * s16.size()));
    a.ops = reinterpret_cast<const OpDesc *>(put(od.data(), sizeof(OpDesc) * od.size()));
    a.nsegs8 = (int)s8.size();
    a.nsegs16 = (int)s16.size();
    a.workers8 = workers8;
    a.workers16 = workers16;
    a.groups8 = (int)((workers8 + wpg8 - 1) / wpg8);
    a.groups16 = (int)workers16;
    // the operators of the other jobs, after those of the table (rebuilt with them)
    if (side)
        for (const dctf_job &j : *side)
            if (std::find(ops.begin(), ops.end(), j.op) == ops.end())
                ops.push_back(j.op);
    return DCTF_OK;
}

dctf_status launch_side_jobs(const std::vector<dctf_job> &side, int prec, hipStream_t s)
{
    for (const dctf_job &j : side) {
        const FilterArgs fa = filter_args(j.op, j.in, j.out, j.B);
        const hipError_t e = j.op->N == 32 ? launch_filter_n32(prec, fa, s)
                                           : launch_filter(j.op->N, prec, current_variant(j.op->N, prec), fa, s);
        if (e != hipSuccess)
            return hip_status(e);
    }
    return DCTF_OK;
}

void rebase_batch(BatchArgs &a, const void *dev)
{
    const uintptr_t base = (uintptr_t)dev;
    a.jobs8 = reinterpret_cast<const JobDesc *>(base + (uintptr_t)a.jobs8);
    a.jobs16 = reinterpret_cast<const JobDesc *>(base + (uintptr_t)a.jobs16);
    a.segs8 = reinterpret_cast<const SegDesc *>(base + (uintptr_t)a.segs8);
    a.segs16 = reinterpret_cast<const SegDesc *>(base + (uintptr_t)a.segs16);
    a.ops = reinterpret_cast<const OpDesc *>(base + (uintptr_t)a.ops);
}

}  // namespace dctf

static bool batch_config_valid(const dctf_batch_config *c)
{
    return c != nullptr && c->fronts >= -1 && c->fronts <= 4096 && c->io >= -1 && c->io <= 2 &&
           (c->nt == 0 || c->nt == 1) && c->groups_per_cu >= 0 && c->groups_per_cu <= 64;
}

// Plans `b` with `cfg` and uploads its work table (the previous table and
// any captured graph are released).
static dctf_status batch_plan(dctf_batch b, const dctf_batch_config &cfg)
{
    std::vector<char> table;
    BatchArgs a;
    std::vector<dctf_operator> ops;
    std::vector<dctf_job> side;
    dctf_status st = plan_batch(b->jobs.data(), (int)b->jobs.size(), b->prec, cfg, table, a, ops, &side);
    if (st != DCTF_OK)
        return st;
    if (b->exec) {
        hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    if (b->dev) {
        // A re-plan: launches of the previous plan may still read its table.
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess)
            return hip_status(e);
    }
    if (table.size() > b->dev_bytes) {
        if (b->dev)
            (void)hipFree(b->dev);
        b->dev = nullptr;
        b->dev_bytes = 0;
        hipError_t e = hipMalloc(&b->dev, table.size());
        if (e != hipSuccess) {
            b->dev = nullptr;
            return hip_status(e);
        }
        b->dev_bytes = table.size();
    }
    if (!table.empty()) {
        hipError_t e = hipMemcpy(b->dev, table.data(), table.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return hip_status(e);
    }
    rebase_batch(a, b->dev);
    b->args = a;
    b->ops = ops;
    b->side = side;
    b->cfg = cfg;
    return DCTF_OK;
}

extern "C" dctf_status dctf_batch_create(const dctf_job *jobs, int njobs, int prec, dctf_batch *out)
{
    if (out == nullptr || njobs < 0 || (njobs > 0 && jobs == nullptr))
        return DCTF_EINVAL;
    dctf_batch b = new (std::nothrow) dctf_batch_s();
    if (!b)
        return DCTF_ENOMEM;
    b->prec = prec;
    try {
        b->jobs.assign(jobs, jobs + njobs);
    } catch (...) {
        delete b;
        return DCTF_ENOMEM;
    }
    dctf_status st = batch_plan(b, batch_config(prec));
    if (st != DCTF_OK) {
        dctf_batch_destroy(b);
        return st;
    }
    *out = b;
    return DCTF_OK;
}

extern "C" dctf_status dctf_set_batch_config(int prec, const dctf_batch_config *cfg)
{
    if ((prec != DCTF_PREC_FP32 && prec != DCTF_PREC_SPLIT_BF16) || !batch_config_valid(cfg))
        return DCTF_EINVAL;
    std::lock_guard<std::mutex> lk(g_batch_cfg_mu);
    g_batch_cfg[prec == DCTF_PREC_FP32 ? 0 : 1] = *cfg;
    return DCTF_OK;
}

extern "C" dctf_status dctf_get_batch_config(int prec, dctf_batch_config *cfg)
{
    if ((prec != DCTF_PREC_FP32 && prec != DCTF_PREC_SPLIT_BF16) || cfg == nullptr)
        return DCTF_EINVAL;
    *cfg = batch_config(prec);
    return DCTF_OK;
}

extern "C" dctf_status dctf_batch_set_config(dctf_batch b, const dctf_batch_config *cfg)
{
    if (b == nullptr || !batch_config_valid(cfg))
        return DCTF_EINVAL;
    return batch_plan(b, *cfg);
}

extern "C" dctf_status dctf_batch_get_config(dctf_batch b, dctf_batch_config *cfg, dctf_batch_config *resolved)
{
    if (b == nullptr || (cfg == nullptr && resolved == nullptr))
        return DCTF_EINVAL;
    if (cfg)
        *cfg = b->cfg;
    if (resolved) {
        // What the plan runs: its N = 8 I/O path, the number of N = 8 fronts
        // it cut and its workgroups per CU.
        resolved->io = b->args.io;
        resolved->nt = b->args.nt ? 1 : 0;
        resolved->fronts = b->args.nsegs8;
        const int groups = b->args.groups8 + b->args.groups16;
        resolved->groups_per_cu = groups > 0 ? (groups + cu_count() - 1) / cu_count() : 0;
    }
    return DCTF_OK;
}

static dctf_status batch_enqueue(dctf_batch b, unsigned flags, hipStream_t s)
{
    if (flags & DCTF_RUN_REBUILD_OPERATORS) {
        dctf_status st = launch_rebuild(b->ops.data(), (int)b->ops.size(), s, kBuildDct);
        if (st != DCTF_OK)
            return st;
    }
    int slot;
    timing_begin(s, &slot);
    dctf_status st = hip_status(launch_batch(b->args, s));
    timing_end(s, slot);
    if (st == DCTF_OK)
        st = launch_side_jobs(b->side, b->prec, s);
    return st;
}

extern "C" dctf_status dctf_batch_run(dctf_batch b, unsigned flags, dctf_stream stream)
{
    if (b == nullptr || (flags & ~DCTF_RUN_REBUILD_OPERATORS))
        return DCTF_EINVAL;
    return batch_enqueue(b, flags, static_cast<hipStream_t>(stream));
}

extern "C" dctf_status dctf_batch_capture(dctf_batch b, unsigned flags, dctf_stream stream)
{
    if (b == nullptr || stream == nullptr || (flags & ~DCTF_RUN_REBUILD_OPERATORS))
        return DCTF_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->exec) {
        hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return hip_status(e);
    dctf_status st = batch_enqueue(b, flags, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (st != DCTF_OK || e != hipSuccess) {
        if (g)
            hipGraphDestroy(g);
        return st != DCTF_OK ? st : hip_status(e);
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return hip_status(e);
    }
    b->graph = g;
    b->exec = x;
    return DCTF_OK;
}

extern "C" dctf_status dctf_batch_launch_graph(dctf_batch b, dctf_stream stream)
{
    if (b == nullptr || b->exec == nullptr)
        return DCTF_EINVAL;
    return hip_status(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
}

extern "C" dctf_status dctf_batch_info(dctf_batch b, int *groups_n8, int *groups_n16, int *threads)
{
    if (b == nullptr)
        return DCTF_EINVAL;
    if (groups_n8)
        *groups_n8 = b->args.groups8;
    if (groups_n16)
        *groups_n16 = b->args.groups16;
    if (threads)
        *threads = (b->args.groups16 == 0) ? kBatch8Threads : kBatchThreads;
    return DCTF_OK;
}

extern "C" void dctf_batch_destroy(dctf_batch b)
{
    if (b == nullptr)
        return;
    if (b->exec)
        hipGraphExecDestroy(b->exec);
    if (b->graph)
        hipGraphDestroy(b->graph);
    if (b->dev)
        hipFree(b->dev);
    delete b;
}

extern "C" dctf_status dctf_filter_batch(const dctf_job *jobs, int njobs, int prec, dctf_stream stream)
{
    dctf_batch b = nullptr;
    dctf_status st = dctf_batch_create(jobs, njobs, prec, &b);
    if (st != DCTF_OK)
        return st;
    st = dctf_batch_run(b, 0, stream);
    dctf_status st2 = hip_status(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    dctf_batch_destroy(b);
    return st != DCTF_OK ? st : st2;
}

extern "C" dctf_status dctf_filter_batch_f64(const dctf_job_f64 *jobs, int njobs, dctf_stream stream)
{
    if (njobs < 0 || (njobs > 0 && jobs == nullptr))
        return DCTF_EINVAL;
    for (int i = 0; i < njobs; ++i) {
        const dctf_job_f64 &j = jobs[i];
        if (j.op == nullptr || j.B < 0)
            return DCTF_EINVAL;
        if (j.B > 0 && (j.in == nullptr || j.out == nullptr || !aligned16(j.in) || !aligned16(j.out)))
            return DCTF_EINVAL;
    }
    if (jobs_conflict_t(jobs, njobs, sizeof(double)))
        return DCTF_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < njobs; ++i) {
        const dctf_job_f64 &j = jobs[i];
        if (j.B == 0)
            continue;
        const dctf_status st = hip_status(launch_filter_f64(j.op->N, j.op->img.dct.H64, j.in, j.out, j.B, s));
        if (st != DCTF_OK)
            return st;
    }
    return DCTF_OK;
}

// ------------------------------------------- one-shot batch, no allocation
//
// The work table of dctf_filter_batch_noalloc lives in a file-scope device
// array (one copy per GPU, held until the process ends).  In host code the
// array's name is not a device address: its address on each device comes
// from hipGetSymbolAddress, taken once per device with that device current,
// and only that address is used (copy target, kernel argument).

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(1) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

dctf_status scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_status(e);
    if (dev < 0 || dev >= kMaxDevices)
        return DCTF_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return e != hipSuccess ? hip_status(e) : DCTF_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DCTF_OK;
}

}  // namespace

extern "C" dctf_status dctf_filter_batch_noalloc(const dctf_job *jobs, int njobs, int prec, dctf_stream stream)
{
    std::vector<char> table;
    BatchArgs a;
    std::vector<dctf_operator> ops;
    std::vector<dctf_job> side;
    dctf_status st = plan_batch(jobs, njobs, prec, batch_config(prec), table, a, ops, &side);
    if (st != DCTF_OK)
        return st;
    if (table.size() > kNoAllocScratchBytes)
        return DCTF_EINVAL;   // work table beyond the fixed scratch: use dctf_filter_batch
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!table.empty()) {
        void *dev = nullptr;
        st = scratch_address(&dev);
        if (st != DCTF_OK)
            return st;
        hipError_t e = hipMemcpyAsync(dev, table.data(), table.size(), hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return hip_status(e);
        rebase_batch(a, dev);
        st = hip_status(launch_batch(a, s));
    }
    if (st == DCTF_OK)
        st = launch_side_jobs(side, prec, s);   // their kernels use no scratch
    if (table.empty() && side.empty())
        return st;   // no blocks: nothing was launched
    // The host table must outlive the copy, and the next call may rewrite
    // the scratch: return once this call's work is done.
    const dctf_status st2 = hip_status(hipStreamSynchronize(s));
    return st != DCTF_OK ? st : st2;
}

// ============================================================ around the path

extern "C" dctf_status dctf_forward_dct_u8(const uint8_t *img_dev, int h, int w, int64_t pitch, int N,
                                           float *coeffs_dev, dctf_stream stream)
{
    if (!supported_op_n(N))
        return (N > 0 && N <= 64) ? DCTF_EUNSUPPORTED : DCTF_EINVAL;
    if (img_dev == nullptr || coeffs_dev == nullptr || h < 1 || w < 1 || pitch < w || !aligned16(coeffs_dev))
        return DCTF_EINVAL;
    return hip_status(launch_forward_dct_u8(img_dev, h, w, pitch, 0, 1, N, coeffs_dev,
                                            static_cast<hipStream_t>(stream)));
}

extern "C" dctf_status dctf_forward_dct_u8_images(const uint8_t *img_dev, int h, int w, int64_t pitch,
                                                  int64_t img_stride, int64_t nimg, int N, float *coeffs_dev,
                                                  dctf_stream stream)
{
    if (!supported_op_n(N))
        return (N > 0 && N <= 64) ? DCTF_EUNSUPPORTED : DCTF_EINVAL;
    if (nimg < 0 || h < 0 || w < 0)
        return DCTF_EINVAL;
    if (nimg == 0 || h == 0 || w == 0)
        return DCTF_OK;
    if (img_dev == nullptr || coeffs_dev == nullptr || pitch < w || !aligned16(coeffs_dev))
        return DCTF_EINVAL;
    const int64_t span = (int64_t)(h - 1) * pitch + w;
    if (nimg > 1 && img_stride < span)
        return DCTF_EINVAL;
    const int64_t bpi = (int64_t)((h + N - 1) / N) * ((w + N - 1) / N);
    if (nimg > INT64_MAX / (bpi * N * N * 4) || nimg > INT64_MAX / std::max<int64_t>(img_stride, 1))
        return DCTF_EINVAL;
    const int64_t istr = nimg > 1 ? img_stride : 0;
    if (ranges_overlap(img_dev, (size_t)((nimg - 1) * istr + span), coeffs_dev, (size_t)(nimg * bpi * N * N * 4)))
        return DCTF_EINVAL;
    return hip_status(launch_forward_dct_u8(img_dev, h, w, pitch, istr, nimg, N, coeffs_dev,
                                            static_cast<hipStream_t>(stream)));
}

extern "C" dctf_status dctf_idct_u8_verify(int N, const float *coeffs_dev, int64_t B, uint8_t *pix_dev,
                                           const uint8_t *expected_dev, unsigned long long *counters_dev,
                                           dctf_stream stream)
{
    if (!supported_op_n(N))
        return (N > 0 && N <= 64) ? DCTF_EUNSUPPORTED : DCTF_EINVAL;
    if (B < 0)
        return DCTF_EINVAL;
    if (B == 0)
        return DCTF_OK;
    if (coeffs_dev == nullptr || pix_dev == nullptr || !aligned16(coeffs_dev))
        return DCTF_EINVAL;
    if (counters_dev != nullptr && ((uintptr_t)counters_dev & 7u))
        return DCTF_EINVAL;
    return hip_status(launch_idct_u8_verify(N, coeffs_dev, B, pix_dev, expected_dev, counters_dev,
                                            static_cast<hipStream_t>(stream)));
}

extern "C" dctf_status dctf_stream_copy(const float *in_dev, float *out_dev, int64_t n, dctf_stream stream)
{
    if (n < 0 || (n & 3))
        return DCTF_EINVAL;
    if (n == 0)
        return DCTF_OK;
    if (in_dev == nullptr || out_dev == nullptr || !aligned16(in_dev) || !aligned16(out_dev))
        return DCTF_EINVAL;
    if (ranges_overlap(in_dev, (size_t)n * 4, out_dev, (size_t)n * 4))
        return DCTF_EINVAL;
    return hip_status(launch_stream_copy(in_dev, out_dev, n, static_cast<hipStream_t>(stream)));
}

// =================================================================== tuning

extern "C" int dctf_variant_count(int N, int prec)
{
    if (!supported_n(N) || (prec != DCTF_PREC_FP32 && prec != DCTF_PREC_SPLIT_BF16))
        return 0;
    return variant_count(N, prec);
}

extern "C" const char *dctf_variant_name(int N, int prec, int v)
{
    if (dctf_variant_count(N, prec) <= v || v < 0)
        return nullptr;
    return variant_name(N, prec, v);
}

extern "C" dctf_status dctf_get_variant(int N, int prec, int *variant)
{
    if (variant == nullptr || dctf_variant_count(N, prec) == 0)
        return DCTF_EINVAL;
    *variant = current_variant(N, prec);
    return DCTF_OK;
}

extern "C" dctf_status dctf_set_variant(int N, int prec, int variant)
{
    if (variant < 0 || variant >= dctf_variant_count(N, prec))
        return DCTF_EINVAL;
    std::lock_guard<std::mutex> lk(g_variant_mu);
    g_variant[N][prec] = variant;
    return DCTF_OK;
}

extern "C" dctf_status dctf_set_batch_fronts(int fronts)
{
    if (fronts < -1 || fronts > 4096)
        return DCTF_EINVAL;
    set_batch_fronts(fronts);
    return DCTF_OK;
}

extern "C" int dctf_get_batch_fronts(void) { return batch_fronts(); }

extern "C" dctf_status dctf_autotune(dctf_operator op, int prec, const float *in_dev, float *out_dev,
                                     int64_t B, int iters, dctf_stream stream, int *best_variant,
                                     float *best_ms)
{
    if (op == nullptr || iters < 1 || B <= 0)
        return DCTF_EINVAL;
    if (prec != DCTF_PREC_FP32 && prec != DCTF_PREC_SPLIT_BF16)
        return DCTF_EINVAL;
    if (!supported_n(op->N))   // the N = 32 filter has one launch shape
        return DCTF_EUNSUPPORTED;
    dctf_status st = validate_io(op->N, in_dev, out_dev, B);
    if (st != DCTF_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const FilterArgs a = filter_args(op, in_dev, out_dev, B);
    const int nv = variant_count(op->N, prec);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            hipEventDestroy(e0);
        return DCTF_EHIP;
    }
    // Warm-up (the chip raises its clocks under a new load over tens of
    // launches), then three passes over all variants, each variant's best
    // pass kept, so that a clock drift over the sweep favours no variant.
    for (int w = 0; w < 32 && st == DCTF_OK; ++w)
        st = hip_status(launch_filter(op->N, prec, 0, a, s));
    std::vector<float> t(nv, 0.0f);
    for (int r = 0; r < 3 && st == DCTF_OK; ++r)
        for (int v = 0; v < nv && st == DCTF_OK; ++v) {
            for (int w = 0; w < 2 && st == DCTF_OK; ++w)
                st = hip_status(launch_filter(op->N, prec, v, a, s));
            if (st == DCTF_OK)
                st = hip_status(hipEventRecord(e0, s));
            for (int i = 0; i < iters && st == DCTF_OK; ++i)
                st = hip_status(launch_filter(op->N, prec, v, a, s));
            if (st == DCTF_OK)
                st = hip_status(hipEventRecord(e1, s));
            if (st == DCTF_OK)
                st = hip_status(hipEventSynchronize(e1));
            float ms = 0.0f;
            if (st == DCTF_OK)
                st = hip_status(hipEventElapsedTime(&ms, e0, e1));
            ms /= iters;
            if (st == DCTF_OK && (r == 0 || ms < t[v]))
                t[v] = ms;
        }
    int best = -1;
    float best_t = 0.0f;
    for (int v = 0; v < nv && st == DCTF_OK; ++v)
        if (best < 0 || t[v] < best_t) {
            best = v;
            best_t = t[v];
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != DCTF_OK)
        return st;
    dctf_set_variant(op->N, prec, best);
    if (best_variant)
        *best_variant = best;
    if (best_ms)
        *best_ms = best_t;
    return DCTF_OK;
}

// Candidates of the batch tuner: every N = 8 I/O path (registers in the MFMA
// layout, LDS-staged coalesced, loaded straight into LDS; with and without
// the nontemporal hint where it applies) x fronts 1, 2, 3, 4, 6, 8 x the
// largest grid or one workgroup per CU less.
static std::vector<dctf_batch_config> batch_candidates()
{
    std::vector<dctf_batch_config> c;
    const int io_nt[][2] = {{1, 1}, {2, 1}, {2, 0}, {1, 0}, {0, 0}};
    const int fronts[] = {1, 2, 3, 4, 6, 8};
    for (const auto &p : io_nt)
        for (int f : fronts)
            for (int g : {0, -1})
                c.push_back({f, p[0], p[1], g});
    return c;
}

extern "C" dctf_status dctf_batch_autotune(dctf_batch b, unsigned flags, int iters, int rounds,
                                           const dctf_batch_config *candidates, int ncand, dctf_stream stream,
                                           float *ms_out, int *best)
{
    if (b == nullptr || iters < 1 || rounds < 1 || ncand < 0 || (ncand > 0 && candidates == nullptr) ||
        (flags & ~DCTF_RUN_REBUILD_OPERATORS))
        return DCTF_EINVAL;
    std::vector<dctf_batch_config> cand;
    if (ncand > 0)
        cand.assign(candidates, candidates + ncand);
    else
        cand = batch_candidates();
    // groups_per_cu = -1 in the built-in list: one workgroup per CU fewer
    // than the occupancy allows (skipped where that is 1).
    std::vector<int> usable(cand.size(), 1);
    for (size_t i = 0; i < cand.size(); ++i) {
        if (!batch_config_valid(&cand[i]) && cand[i].groups_per_cu != -1)
            return DCTF_EINVAL;
        if (cand[i].groups_per_cu == -1) {
            const dctf_batch_config probe = {cand[i].fronts, cand[i].io, cand[i].nt, 0};
            dctf_status st = batch_plan(b, probe);
            if (st != DCTF_OK)
                return st;
            const int groups = b->args.groups8 + b->args.groups16;
            const int per_cu = (groups + cu_count() - 1) / cu_count();
            cand[i].groups_per_cu = per_cu - 1;
            usable[i] = per_cu > 1;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            hipEventDestroy(e0);
        return DCTF_EHIP;
    }
    const dctf_batch_config orig = b->cfg;
    std::vector<float> t(cand.size(), 0.0f);
    dctf_status st = DCTF_OK;
    // Warm-up: the chip raises its clocks under a new load over tens of
    // launches; the first candidate would otherwise run in that phase.
    for (int i = 0; i < 64 && st == DCTF_OK; ++i)
        st = batch_enqueue(b, flags, s);
    // Rounds over all candidates, each candidate's best round kept, so that a
    // drift of the clock over the sweep does not favour one end of the list.
    for (int r = 0; r < rounds && st == DCTF_OK; ++r)
        for (size_t i = 0; i < cand.size() && st == DCTF_OK; ++i) {
            if (!usable[i])
                continue;
            st = batch_plan(b, cand[i]);
            for (int w = 0; w < 2 && st == DCTF_OK; ++w)
                st = batch_enqueue(b, flags, s);
            if (st == DCTF_OK)
                st = hip_status(hipEventRecord(e0, s));
            for (int k = 0; k < iters && st == DCTF_OK; ++k)
                st = batch_enqueue(b, flags, s);
            if (st == DCTF_OK)
                st = hip_status(hipEventRecord(e1, s));
            if (st == DCTF_OK)
                st = hip_status(hipEventSynchronize(e1));
            float ms = 0.0f;
            if (st == DCTF_OK)
                st = hip_status(hipEventElapsedTime(&ms, e0, e1));
            ms /= iters;
            if (st == DCTF_OK && (r == 0 || ms < t[i]))
                t[i] = ms;
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != DCTF_OK) {
        (void)batch_plan(b, orig);
        return st;
    }
    int bi = -1;
    for (size_t i = 0; i < cand.size(); ++i)
        if (usable[i] && (bi < 0 || t[i] < t[bi]))
            bi = (int)i;
    if (ms_out)
        for (size_t i = 0; i < cand.size(); ++i)
            ms_out[i] = usable[i] ? t[i] : -1.0f;
    if (best)
        *best = bi;
    return batch_plan(b, bi >= 0 ? cand[bi] : orig);
}

extern "C" int dctf_batch_autotune_candidates(dctf_batch_config *out, int max)
{
    const std::vector<dctf_batch_config> c = batch_candidates();
    if (out)
        for (int i = 0; i < max && i < (int)c.size(); ++i)
            out[i] = c[i];
    return (int)c.size();
}

// ===================================================================== misc

extern "C" const char *dctf_status_string(dctf_status s)
{
    switch (s) {
    case DCTF_OK: return "ok";
    case DCTF_EINVAL: return "invalid argument";
    case DCTF_EUNSUPPORTED: return "unsupported block size or precision";
    case DCTF_ENOMEM: return "out of memory";
    case DCTF_EHIP: return "HIP runtime error";
    case DCTF_EBUSY: return "resource budget exhausted";
    }
    return "unknown status";
}

extern "C" const char *dctf_version(void) { return "dctf 0.1.0 (gfx950)"; }

extern "C" dctf_status dctf_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.on = on != 0;
    g_timing.used = 0;
    return DCTF_OK;
}

extern "C" dctf_status dctf_timing_read(double *avg_ms, int *count)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    double total = 0.0;
    int n = 0;
    for (int i = 0; i < g_timing.used; ++i) {
        hipEvent_t a = g_timing.ev[2 * i], b = g_timing.ev[2 * i + 1];
        if (!a || !b)
            continue;
        if (hipEventSynchronize(b) != hipSuccess)
            return DCTF_EHIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, a, b) != hipSuccess)
            return DCTF_EHIP;
        total += ms;
        ++n;
    }
    g_timing.used = 0;
    if (avg_ms)
        *avg_ms = n ? total / n : 0.0;
    if (count)
        *count = n;
    return DCTF_OK;
}
