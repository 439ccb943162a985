// FP64 operator builder (gfx950).
//
// For a kh x kw mask W, block size N and border mode, forms
//
//   H[(u,v),(k,l)] = sum_p sum_q W[p][q] T_{p-a_h}[u][k] T_{q-a_w}[v][l],
//   T_d = C S_d C^t,  T_d[u][k] = sum_i C[u][i] C[k][s_d(i)],
//
// where C is the orthonormal DCT-II matrix (Sec. II.A, eq. 1-2) and s_d(i)
// the source row of output row i under a shift by d: i + d with zero fill
// outside the block (zero padding, Sec. II.B) or clamp(i + d, 0, N-1) (border
// replication, Sec. II.C / Fig. 1).  This is the Kronecker form of the
// paper's DCT-domain products A.BLOCK.B (eq. 6-8): a row selector a = S_d
// becomes A = C a C^t (eq. 7), and a horizontal band of mask row p becomes
// B_p = sum_q W[p][q] T_q^t.  Summing over every mask row reproduces eq. 11
// (zero padding) and, with the clamped selectors, the corner / lateral terms
// of eq. 13-19 that eq. 20 adds.
//
// The sum over q is taken first: G_p[j][l] = sum_q W[p][q] C[l][s_q(j)],
// B_p = C G_p (so B_p[v][l] = sum_q W[p][q] T_q[v][l]); then
// H += T_p (x) B_p for each mask row p.
//
// The same launch also forms the pixel-domain operator G = (C (x) C)^t H,
// the map from coefficients to filtered pixels (the filtered block taken
// back to the spatial domain, eq. 3).  Because C^t C = I, its factors are
// C^t T_p = S_p C^t and C^t B_p = G_p, so
//   G[(i,j),(k,l)] = sum_p [s_{p-a_h}(i) valid] C[k][s_{p-a_h}(i)] G_p[j][l],
// built in the same loop with T_p replaced by S_p C^t and B_p by G_p.  Mask rows are processed in chunks
// that fit in LDS (all rows at once for the usual mask sizes), three barriers
// per chunk.  Everything is FP64.  One workgroup owns 16 rows of H (all N^2
// columns) for one operator and writes every image of those rows: FP64,
// FP32, the MFMA fragments and the DC column.
//
// Fragment layouts (lane = 16 g + m of a 64-lane wave, M-tile t = row / 16,
// m = row % 16):
//   frag32  FP32 A operand of v_mfma_f32_16x16x4_f32, DC column zeroed
//   frag_hi / frag_lo  BF16 A operands of v_mfma_f32_16x16x32_bf16, with the
//           low-frequency columns zeroed
//   frag_lf FP32 A operand for the low-frequency columns (lf_slot()): slot
//           q = 2 g + j at ((t * 64 + lane) * 2 + j), j the k-step (two k-steps
//           for N = 8 and N = 16)
#include "dctf_internal.h"

#include <math.h>

namespace dctf {
namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerGroup = 16;
constexpr int kMaxN = 16;
constexpr int kMaxK = 2 * kMaxN + 1;
constexpr int kMaxFacN = 32;   // the factors are built for every block size

// Source index of row (or column) i under a shift by d.  The returned index
// is always inside the block (clamped); in zero mode *valid tells whether the
// unclamped index was inside (otherwise the term is zero).
__device__ inline int src_index(int i, int d, int N, int border, bool *valid)
{
    const int m = i + d;
    *valid = (border != DCTF_BORDER_ZERO) || (m >= 0 && m < N);
    return m < 0 ? 0 : (m >= N ? N - 1 : m);
}

// LDS budget for the per-chunk matrices: T_p, G_p and B_p (3 N x N FP64
// each) for up to kChunk(N) mask rows at once.
template <int N>
constexpr int chunk_rows() { return N >= 32 ? 1 : (N >= 16 ? 8 : (N == 8 ? 17 : 33)); }

// Split-BF16 images of entry H[r][c] = h (h32 = fp32(h)) of an operator on
// N x N blocks (N = 8 or 16): the low-frequency columns (DC included) go to
// the FP32 MFMA image frag_lf (slot 2g + j of k-step j, 2 steps); every other
// column is split into BF16 hi = bf16(fp32(H)), lo = bf16(fp32(H - hi)).
__device__ __forceinline__ void write_split_entry(const DenseImages &D, int N, int r, int c, double h, float h32)
{
    const int q = lf_slot(N, c);
    uint16_t hi = 0, lo = 0;
    if (q >= 0) {
        const int t = r >> 4, m = r & 15;
        const int steps = lf_count(N) / 4, lane = 16 * (q / steps) + m;
        D.frag_lf[(t * 64 + lane) * steps + q % steps] = h32;
    } else {
        hi = bf16_rne(h32);
        lo = bf16_rne(__double2float_rn(h - (double)bf16_to_f32(hi)));
    }
    const int fi = frag16_index(N, r, c);
    D.frag_hi[fi] = hi;
    D.frag_lo[fi] = lo;
}

template <int N>
__device__ void build_op(const BuildDesc &d, int r0, double *lds, int domain)
{
    constexpr int NN = N * N;
    constexpr int P = chunk_rows<N>();
    constexpr int rows = NN < kRowsPerGroup ? NN : kRowsPerGroup;   // H rows of this group
    constexpr int owned = rows * NN;                                 // H entries of this group
    constexpr int per_thread = (owned + kThreads - 1) / kThreads;
    const int kh = d.kh, kw = d.kw, border = d.border;
    const int ah = (kh - 1) / 2, aw = (kw - 1) / 2;
    // domain 1: pixel-domain G (coefficients -> pixels); domain 2 (N = 8):
    // pixels -> pixels, whose factors are S_p and sum_q W[p][q] S_q
    // (C^t T_p C = S_p), the spatial operator the method's H_dct is the
    // orthogonal similarity of
    const bool pix = domain >= 1;
    const bool pp = domain == 2;
    const DenseImages &out = pp ? d.img.pp : (pix ? d.img.pix : d.img.dct);

    // N = 32 masks (up to 65 x 65) are read from global memory instead of LDS
    constexpr bool kMaskInLds = N <= 16;
    double *sC = lds;                                   // NN
    double *sW = sC + NN;                               // kh * kw (<= 33 * 33), N <= 16
    double *sT = sW + (kMaskInLds ? kMaxK * kMaxK : 0); // P * NN
    double *sG = sT + P * NN;                           // P * NN
    double *sB = sG + P * NN;                           // P * NN
    const double *Wm = kMaskInLds ? sW : d.img.mask;

    const int tid = threadIdx.x;
    for (int e = tid; e < NN; e += kThreads) {
        const int k = e / N, n = e % N;
        const double alpha = (k == 0) ? sqrt(1.0 / N) : sqrt(2.0 / N);
        sC[e] = alpha * cos(M_PI * (2.0 * n + 1.0) * k / (2.0 * N));
    }
    if constexpr (kMaskInLds)
        for (int e = tid; e < kh * kw; e += kThreads)
            sW[e] = d.img.mask[e];

    double acc[per_thread];
#pragma unroll
    for (int o = 0; o < per_thread; ++o)
        acc[o] = 0.0;
    __syncthreads();

    for (int p0 = 0; p0 < kh; p0 += P) {
        const int np = kh - p0 < P ? kh - p0 : P;
        // T_p[u][k] = sum_i C[u][i] C[k][s_{p-ah}(i)];  G_p[j][l] = sum_q W[p][q] C[l][s_{q-aw}(j)]
        for (int e = tid; e < 2 * np * NN; e += kThreads) {
            const int which = e / (np * NN), rest = e % (np * NN);
            const int pr = rest / NN, idx = rest % NN;
            const int a = idx / N, b = idx % N;
            double s = 0.0;
            if (which == 0) {
                const int dp = p0 + pr - ah;
                if (pp) {
                    // S_p[i][m] with (i, m) = (a, b)
                    bool ok;
                    const int m = src_index(a, dp, N, border, &ok);
                    s = (ok && m == b) ? 1.0 : 0.0;
                } else if (pix) {
                    // (S_p C^t)[i][k] with (i, k) = (a, b)
                    bool ok;
                    const int m = src_index(a, dp, N, border, &ok);
                    s = ok ? sC[b * N + m] : 0.0;
                } else {
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        bool ok;
                        const int m = src_index(i, dp, N, border, &ok);
                        s += ok ? sC[a * N + i] * sC[b * N + m] : 0.0;
                    }
                }
                sT[pr * NN + idx] = s;
            } else {
                const double *w = Wm + (p0 + pr) * kw;
                for (int q = 0; q < kw; ++q) {
                    bool ok;
                    const int m = src_index(a, q - aw, N, border, &ok);
                    // pixels in: sum_q W[p][q] S_q[j][n] instead of C[l][s_q(j)]
                    s += ok ? w[q] * (pp ? (m == b ? 1.0 : 0.0) : sC[b * N + m]) : 0.0;
                }
                sG[pr * NN + idx] = s;
            }
        }
        __syncthreads();
        // B_p[v][l] = sum_j C[v][j] G_p[j][l] (the pixel domain uses G_p itself)
        if (!pix) {
            for (int e = tid; e < np * NN; e += kThreads) {
                const int pr = e / NN, idx = e % NN, v = idx / N, l = idx % N;
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j)
                    s += sC[v * N + j] * sG[pr * NN + j * N + l];
                sB[e] = s;
            }
        }
        __syncthreads();
        // H[(u,v),(k,l)] += sum_p T_p[u][k] B_p[v][l]  (pixel domain: (S_p C^t)[i][k] G_p[j][l])
        const double *sR = pix ? sG : sB;
#pragma unroll
        for (int o = 0; o < per_thread; ++o) {
            const int e = tid + o * kThreads;
            if (e < owned) {
                const int r = r0 + e / NN, c = e % NN;
                const int u = r / N, v = r % N, k = c / N, l = c % N;
                double s = acc[o];
                for (int pr = 0; pr < np; ++pr)
                    s += sT[pr * NN + u * N + k] * sR[pr * NN + v * N + l];
                acc[o] = s;
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int o = 0; o < per_thread; ++o) {
        const int e = tid + o * kThreads;
        if (e >= owned)
            continue;
        const int r = r0 + e / NN, c = e % NN;
        const double h = acc[o];
        const float h32 = __double2float_rn(h);
        out.H64[(size_t)r * NN + c] = h;
        out.H32[(size_t)r * NN + c] = h32;
        if (c == 0)
            out.h0[r] = h32;
        if constexpr (N >= 8)
            // FP32 MFMA image: the operator without its DC column, which the
            // FP32 filter applies separately in VALU arithmetic.
            out.frag32[frag32_index(N, r, c)] = (c == 0) ? 0.0f : h32;
        if (pp) {
            // pixels -> pixels: every column as three BF16 terms (pixels are
            // exact in BF16, so the operator's 24 bits carry the precision)
            const uint16_t hi = bf16_rne(h32);
            const double r1 = h - (double)bf16_to_f32(hi);
            const uint16_t mid = bf16_rne(__double2float_rn(r1));
            const uint16_t lo = bf16_rne(__double2float_rn(r1 - (double)bf16_to_f32(mid)));
            const int fi = frag16_index(N, r, c);
            out.frag_hi[fi] = hi;
            out.frag_lo[fi] = mid;
            out.frag_lo2[fi] = lo;
        } else if constexpr (N == 8 || N == 16) {
            write_split_entry(out, N, r, c, h, h32);
        }
    }
}

constexpr int lds_doubles(int N)
{
    return N * N + (N <= 16 ? kMaxK * kMaxK : 0) + 3 * (N >= 32 ? 1 : (N >= 16 ? 8 : (N == 8 ? 17 : 33))) * N * N;
}
constexpr int max3(int a, int b, int c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }
constexpr int kLdsDoubles = max3(lds_doubles(4), lds_doubles(8), lds_doubles(16));

__global__ __launch_bounds__(kThreads) void k_build(BuildArgs args)
{
    const int op = blockIdx.y;
    if (op >= args.n)
        return;
    const BuildDesc &d = args.d[op];
    const int NN = d.N * d.N;
    const int rows_per_group = NN < kRowsPerGroup ? NN : kRowsPerGroup;
    const int r0 = blockIdx.x * rows_per_group;
    if (r0 >= NN)
        return;
    __shared__ double lds[kLdsDoubles];
    // z enumerates the requested domains in the order H_dct, pixel-domain G,
    // pixels -> pixels (that one for N = 8 only)
    const bool want[3] = {(args.parts & kBuildDct) != 0, (args.parts & kBuildPix) != 0,
                          (args.parts & kBuildPixPix) != 0};
    int domain = -1;
    for (int k = 0, z = 0; k < 3; ++k)
        if (want[k] && z++ == (int)blockIdx.z)
            domain = k;
    if (domain < 0 || (domain == 2 && d.N != 8))
        return;
    switch (d.N) {
    case 2: build_op<2>(d, r0, lds, domain); break;
    case 4: build_op<4>(d, r0, lds, domain); break;
    case 8: build_op<8>(d, r0, lds, domain); break;
    case 16: build_op<16>(d, r0, lds, domain); break;
    default: break;   // N = 32: k_build32
    }
}

// N = 32 operators (H_dct images only: no split-BF16 or pixel-domain set).
// A kernel of its own: its 64 FP64 accumulators per thread would otherwise
// set the register allocation, and so the occupancy, of every block size.
__global__ __launch_bounds__(kThreads) void k_build32(BuildArgs args)
{
    const int op = blockIdx.y;
    if (op >= args.n || args.d[op].N != 32)
        return;
    __shared__ double lds[lds_doubles(32)];
    build_op<32>(args.d[op], blockIdx.x * kRowsPerGroup, lds, 0);
}

// Factored (paper-form) operator: for rank term r and axis x (0: block rows
// with fac_a and the kh anchor, 1: block columns with fac_b and kw),
//   F = C M C^t,  M[i][m] = sum_p coef[p] [s_{p-a}(i) = m]  (valid shifts only),
// i.e. F = sum_p coef[p] T_{p-a}: the DCT-domain matrices A (eq. 7) of the
// mask's rank-one terms, so that H = sum_r P_r (x) Q_r and every block
// becomes Y = sum_r P_r X Q_r^t (eq. 8, 11, 20 with the mask rows merged
// into rank terms).  FP64 throughout; one workgroup per (operator, r, axis).
__global__ __launch_bounds__(kThreads) void k_build_factors(BuildArgs args)
{
    const int op = blockIdx.y;
    if (op >= args.n)
        return;
    const BuildDesc &d = args.d[op];
    const int r = blockIdx.x >> 1, axis = blockIdx.x & 1;
    if (r >= d.rank)
        return;
    const int N = d.N, NN = N * N, tid = threadIdx.x;
    const int K = axis ? d.kw : d.kh, anchor = (K - 1) / 2;
    const double *coef = axis ? d.img.fac_b + (size_t)r * d.kw : d.img.fac_a + (size_t)r * d.kh;
    __shared__ double sC[kMaxFacN * kMaxFacN], sM[kMaxFacN * kMaxFacN], sT[kMaxFacN * kMaxFacN];
    for (int e = tid; e < NN; e += kThreads) {
        const int k = e / N, n = e % N;
        const double alpha = (k == 0) ? sqrt(1.0 / N) : sqrt(2.0 / N);
        sC[e] = alpha * cos(M_PI * (2.0 * n + 1.0) * k / (2.0 * N));
        const int i = e / N, m = e % N;
        double acc = 0.0;
        for (int p = 0; p < K; ++p) {
            bool ok;
            const int src = src_index(i, p - anchor, N, d.border, &ok);
            acc += (ok && src == m) ? coef[p] : 0.0;
        }
        sM[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < NN; e += kThreads) {   // T = C M
        const int u = e / N, m = e % N;
        double acc = 0.0;
        for (int i = 0; i < N; ++i)
            acc += sC[u * N + i] * sM[i * N + m];
        sT[e] = acc;
    }
    __syncthreads();
    double *F64 = (axis ? d.img.Q64 : d.img.P64) + (size_t)r * NN;
    float *F32 = (axis ? d.img.Q32 : d.img.P32) + (size_t)r * NN;
    for (int e = tid; e < NN; e += kThreads) {   // F = T C^t
        const int u = e / N, k = e % N;
        double acc = 0.0;
        for (int m = 0; m < N; ++m)
            acc += sT[u * N + m] * sC[k * N + m];
        F64[e] = acc;
        F32[e] = __double2float_rn(acc);
    }
}

// Parity classes of an N = 16 or 32 operator (mask mirror-symmetric on both
// axes): with M = N / 2, entry [r][c] of class (pu, pv), r = M a + b and
// c = M a' + b', is H_dct[(2a + pu) N + 2b + pv][(2a' + pu) N + 2b' + pv],
// written into the class's images as the builder writes an operator on
// M x M blocks.
struct ParityOut {
    DenseImages par[4];
};

template <int N>
__global__ __launch_bounds__(kThreads) void k_build_parity(const double *H64, ParityOut out)
{
    constexpr int M = N / 2, K = M * M;
    const int e = blockIdx.x * kThreads + threadIdx.x;   // 4 classes x K x K
    if (e >= 4 * K * K)
        return;
    const int cls = e / (K * K), r = (e / K) % K, c = e % K;
    const int pu = cls >> 1, pv = cls & 1;
    const int R = (2 * (r / M) + pu) * N + 2 * (r % M) + pv;
    const int C = (2 * (c / M) + pu) * N + 2 * (c % M) + pv;
    const double h = H64[(size_t)R * (N * N) + C];
    const float h32 = __double2float_rn(h);
    const DenseImages &D = out.par[cls];
    if (c == 0)
        D.h0[r] = h32;
    D.frag32[frag32_index(M, r, c)] = (c == 0) ? 0.0f : h32;
    write_split_entry(D, M, r, c, h, h32);
}

}  // namespace

hipError_t launch_build_parity(int N, const double *H64, const DenseImages *par, hipStream_t stream)
{
    ParityOut o;
    for (int c = 0; c < 4; ++c)
        o.par[c] = par[c];
    if (N == 16)
        hipLaunchKernelGGL(k_build_parity<16>, dim3(4 * 4096 / kThreads), dim3(kThreads), 0, stream, H64, o);
    else
        hipLaunchKernelGGL(k_build_parity<32>, dim3(4 * 65536 / kThreads), dim3(kThreads), 0, stream, H64, o);
    return hipGetLastError();
}

hipError_t launch_build(const BuildArgs &args, hipStream_t stream)
{
    if (args.n <= 0)
        return hipSuccess;
    int maxN = 0, maxRank = 0;
    bool has32 = false;
    for (int i = 0; i < args.n; ++i) {
        if (args.d[i].N == 32)
            has32 = true;
        else
            maxN = args.d[i].N > maxN ? args.d[i].N : maxN;
        maxRank = args.d[i].rank > maxRank ? args.d[i].rank : maxRank;
    }
    const int groups = (maxN * maxN + kRowsPerGroup - 1) / kRowsPerGroup;
    const int domains = ((args.parts & kBuildDct) ? 1 : 0) + ((args.parts & kBuildPix) ? 1 : 0) +
                        ((args.parts & kBuildPixPix) ? 1 : 0);
    if (domains > 0 && maxN > 0) {
        hipLaunchKernelGGL(k_build, dim3(groups, args.n, domains), dim3(kThreads), 0, stream, args);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (has32 && (args.parts & kBuildDct)) {
        hipLaunchKernelGGL(k_build32, dim3(32 * 32 / kRowsPerGroup, args.n), dim3(kThreads), 0, stream, args);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (!(args.parts & kBuildFactors) || maxRank <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_build_factors, dim3(2 * maxRank, args.n), dim3(kThreads), 0, stream, args);
    return hipGetLastError();
}

}  // namespace dctf
