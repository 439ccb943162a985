// Kernels around the filter path:
//   k_forward_dct_mfma   uint8 image -> FP32 coefficient blocks (eq. 1) for
//                        N = 8, 16, 32: FP64 MFMA, rounded once to FP32
//   k_forward_dct_u8     the same for N = 2, 4: one thread per pixel, FP64
//   k_idct_u8_verify8    FP32 coefficients -> uint8 pixels (eq. 3 in FP32, then
//                        the Sec. III uint8 conversion) with mismatch / near-1/2
//                        counters, N = 8: one block per lane
//   k_idct_u8_verify_mfma  the same for N = 16, 32 on FP32 MFMA
//   k_idct_u8_verify     the same for N = 2, 4 and unaligned N = 8 buffers
// The N x N DCT matrix is formed in LDS from its closed form.
#include <atomic>

#include "mfma_common.h"

#include <math.h>

namespace dctf {
namespace {

constexpr int kThreads = 256;

template <typename T>
__device__ inline void fill_dct(T *sC, int N)
{
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        int k = e / N, n = e % N;
        double alpha = (k == 0) ? sqrt(1.0 / N) : sqrt(2.0 / N);
        sC[e] = (T)(alpha * cos(M_PI * (2.0 * n + 1.0) * k / (2.0 * N)));
    }
}

// One output x_k = sum_v C[v][k] z_v of the 8-point inverse DCT along one axis
// (eq. 3), from the symmetries of the DCT basis.  C[v][7 - k] = (-1)^v C[v][k]
// splits the sum into an even part (z0, z2, z4, z6) and an odd part
// (z1, z3, z5, z7), both shared by outputs k and 7 - k; within the even part
// C[2w][3 - h] = (-1)^w C[2w][h] splits it again into (z0, z4) and (z2, z6),
// shared by h and 3 - h.  With h = min(k, 7 - k) and m = min(h, 3 - h):
//   ce = C[0][m], C[4][m], C[2][m], C[6][m];  co = C[1][h], C[3][h], C[5][h], C[7][h];
//   neg_e = (h >= 2), neg_o = (k >= 4).
// 36 operations per 8 outputs against 64 products for the plain sum.  Every
// 8-point inverse transform below evaluates an output in exactly this order,
// so the kernels give the same pixels bit for bit.
__device__ __forceinline__ float idct8_point(const float z[8], const float ce[4], const float co[4], bool neg_e,
                                             bool neg_o)
{
    const float ee = fmaf(z[4], ce[1], z[0] * ce[0]);
    const float eo = fmaf(z[6], ce[3], z[2] * ce[2]);
    const float e = neg_e ? ee - eo : ee + eo;
    const float o = fmaf(z[7], co[3], fmaf(z[5], co[2], fmaf(z[3], co[1], z[1] * co[0])));
    return neg_o ? e - o : e + o;
}

// The coefficients and signs of idct8_point for output k, from C[v * 8 + n] = C[v][n].
template <typename Tab>
__device__ __forceinline__ void idct8_coeffs(const Tab &C, int k, float ce[4], float co[4], bool &neg_e,
                                             bool &neg_o)
{
    const int h = k < 4 ? k : 7 - k, m = h < 2 ? h : 3 - h;
    ce[0] = C[m];
    ce[1] = C[32 + m];
    ce[2] = C[16 + m];
    ce[3] = C[48 + m];
    co[0] = C[8 + h];
    co[1] = C[24 + h];
    co[2] = C[40 + h];
    co[3] = C[56 + h];
    neg_e = h >= 2;
    neg_o = k >= 4;
}

// X[u][v] = sum_i C[u][i] (sum_j x[i][j] C[v][j]) in FP64, rounded once to FP32.
// One thread per pixel; workgroups of max(256, N*N) threads.
constexpr int kMaxDctThreads = 1024;
__global__ __launch_bounds__(kMaxDctThreads) void k_forward_dct_u8(const uint8_t *img, int h, int w,
                                                                   int64_t pitch, int N, float *coeffs,
                                                                   int64_t nblocks)
{
    __shared__ double sC[kMaxDctThreads];
    __shared__ double sx[kMaxDctThreads];
    __shared__ double st[kMaxDctThreads];
    fill_dct(sC, N);
    const int NN = N * N;
    const int per = blockDim.x / NN;
    const int local = threadIdx.x / NN, e = threadIdx.x % NN;
    const int i = e / N, j = e % N;
    const int64_t blk = (int64_t)blockIdx.x * per + local;
    const bool active = local < per && blk < nblocks;
    const int bw = (w + N - 1) / N;
    if (active) {
        const int64_t by = blk / bw, bx = blk % bw;
        int64_t y = by * N + i, x = bx * N + j;
        y = y < h ? y : h - 1;
        x = x < w ? x : w - 1;
        sx[threadIdx.x] = (double)img[y * pitch + x];
    }
    __syncthreads();
    const int base = local * NN;
    if (active) {
        // t[i][v] with (i, v) = (i, j) of this thread
        double s = 0.0;
        for (int jj = 0; jj < N; ++jj)
            s += sx[base + i * N + jj] * sC[j * N + jj];
        st[threadIdx.x] = s;
    }
    __syncthreads();
    if (active) {
        // X[u][v] with (u, v) = (i, j) of this thread
        double s = 0.0;
        for (int ii = 0; ii < N; ++ii)
            s += sC[i * N + ii] * st[base + ii * N + j];
        coeffs[blk * NN + e] = __double2float_rn(s);
    }
}

// v from lane 15 - i of the lane's 16-lane row (DPP row_mirror)
__device__ __forceinline__ float row_mirror(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xf, 0xf, false));
}

__device__ __forceinline__ f32x4 row_mirror4(f32x4 v)
{
    return f32x4{row_mirror(v[0]), row_mirror(v[1]), row_mirror(v[2]), row_mirror(v[3])};
}

typedef double f64x4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4v mfma_f64x4(double a, double b, f64x4v c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Forward DCT for N = 8, 16 and 32 on FP64 MFMA 16x16x4, one unit of S x S
// pixels per wave at a time (S = 16 for N = 8 and 16, 32 for N = 32), no data
// moved between lanes.  The MFMA returns row g + 4r of its 16 x 16 result in
// register r of lane (n, g) = (lane % 16, lane / 16).  Pass 1, T = x C^t:
// lane (n, g) supplies pixels x[n][4g + s] of a 16 x 16 tile as the A operand
// of k-step s and C[sigma(n)][4g + s] as B, sigma(m) = 4 (m % 4) + m / 4, so
// register r holds T[g + 4r][sigma(n)].  That is the A operand of k-step r of
// pass 2, X^t = T^t C^t, with C[n][g + 4r] as B; its register r then holds
// X[n][sigma(g + 4r)] = X[n][4g + r]: four consecutive coefficients, stored as
// one 16-byte write.  N = 32: a block is 2 x 2 tiles (8 k-steps per output
// tile).  N = 8: a unit is 2 x 2 blocks and C is diag(C8, C8), so the tile's
// result holds the four blocks' coefficients in the same arrangement (the
// off-diagonal products add exact zeros).  Pixels past the image repeat the
// last row / column; blocks past the block grid (N = 8, odd counts) are not
// stored.  A unit inside the image reads its four pixels per lane and tile
// row as one 32-bit load when the image and its pitch are 4-byte aligned
// (aligned4), others pixel by pixel with clamped indices.  FP64 products and
// sums, rounded once to FP32.  Several images (img_stride bytes apart, upi
// units each) go through one launch: the units are numbered across them, and
// image i's blocks follow image i - 1's in the output.
template <int N, int NB>
__global__ __launch_bounds__(kThreads) void k_forward_dct_mfma(const uint8_t *img, int h, int w, int64_t pitch,
                                                               float *coeffs, int64_t bh, int64_t bw, int64_t ubw,
                                                               int64_t units, int aligned4, int64_t upi,
                                                               int64_t img_stride)
{
    constexpr int S = N < 16 ? 16 : N, NT = S / 16;
    __shared__ double sC[N * N];
    fill_dct(sC, N);
    __syncthreads();
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int sn = 4 * (n & 3) + (n >> 2);
    // element (a, b) of C (N = 8: of diag(C8, C8))
    auto cval = [&](int a, int b) -> double {
        if constexpr (N == 8)
            return (a >> 3) == (b >> 3) ? sC[(a & 7) * 8 + (b & 7)] : 0.0;
        else
            return sC[a * N + b];
    };
    // c1[J][V][s] (N = 32: c1[0][P][s] = C[2 sigma(n) + P][4g + s], the even / odd
    // halves of pass 1), c2[I][U][r]
    double c1[NT][NT][4], c2[NT][NT][4];
#pragma unroll
    for (int P = 0; P < NT; ++P)
#pragma unroll
        for (int Q = 0; Q < NT; ++Q)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if constexpr (N == 32)
                    c1[P][Q][k] = cval(2 * sn + Q, 4 * g + k);
                else
                    c1[P][Q][k] = cval(16 * Q + sn, 16 * P + 4 * g + k);
                c2[P][Q][k] = cval(16 * Q + n, 16 * P + g + 4 * k);
            }
    // the wave index as a scalar: the unit bookkeeping below runs on the scalar unit
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    const int64_t waves = (int64_t)gridDim.x * 4;
    // per lane, relative to a unit's corner: pixel (16 I + n, 16 J + 4g) and the
    // output place of X[16 U + n][16 V + 4g]
    int64_t loff[NT][NT], soff[NT][NT];
#pragma unroll
    for (int P = 0; P < NT; ++P)
#pragma unroll
        for (int Q = 0; Q < NT; ++Q) {
            // N = 32: word Q = 1 holds the mirror columns 28 - 4g .. 31 - 4g
            loff[P][Q] = (int64_t)(16 * P + n) * pitch + (N == 32 && Q == 1 ? 28 - 4 * g : 16 * Q + 4 * g);
            if constexpr (N == 8)
                soff[P][Q] = ((n >> 3) * bw + (g >> 1)) * 64 + (n & 7) * 8 + 4 * (g & 1);
            else
                soff[P][Q] = (16 * P + n) * N + 16 * Q + 4 * g;
        }
    const int64_t ubh = upi / ubw, bpi_floats = bh * bw * (N * N);
    for (int64_t unit0 = wave * NB; unit0 < units; unit0 += waves * NB) {
        const int64_t im0 = unit0 / upi, r0 = unit0 - im0 * upi;
        const int64_t uy0 = r0 / ubw, ux0 = r0 % ubw;
        // px[b][I][J] byte s = pixel (16 I + n, 16 J + 4g + s) of unit unit0 + b: four pixels
        // per register, so that many units' loads fit in flight
        uint32_t px[NB][NT][NT];
        {
            int64_t im = im0, uy = uy0, ux = ux0;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const bool live = unit0 + b < units;
                // a unit past the end reads unit 0
                const int64_t ly = live ? uy : 0, lx = live ? ux : 0, li = live ? im : 0;
                const uint8_t *ibase = img + li * img_stride;
                if (aligned4 && (ly + 1) * S <= h && (lx + 1) * S <= w) {   // uniform over the wave
                    const uint8_t *base = ibase + ly * S * pitch + lx * S;
#pragma unroll
                    for (int I = 0; I < NT; ++I)
#pragma unroll
                        for (int J = 0; J < NT; ++J)
                            px[b][I][J] = *reinterpret_cast<const uint32_t *>(base + loff[I][J]);
                } else {
#pragma unroll
                    for (int I = 0; I < NT; ++I) {
                        int64_t row = ly * S + 16 * I + n;
                        row = row < h ? row : h - 1;
#pragma unroll
                        for (int J = 0; J < NT; ++J) {
                            uint32_t v = 0;
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                int64_t col = lx * S + (N == 32 && J == 1 ? 28 - 4 * g : 16 * J + 4 * g) + k;
                                col = col < w ? col : w - 1;
                                v |= (uint32_t)ibase[row * pitch + col] << (8 * k);
                            }
                            px[b][I][J] = v;
                        }
                    }
                }
                if (++ux == ubw) {
                    ux = 0;
                    if (++uy == ubh) {
                        uy = 0;
                        ++im;
                    }
                }
            }
        }
        int64_t im = im0, uy = uy0, ux = ux0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const bool live = unit0 + b < units;
            const int64_t ci = im, cy = uy, cx = ux;
            if (++ux == ubw) {
                ux = 0;
                if (++uy == ubh) {
                    uy = 0;
                    ++im;
                }
            }
            f64x4v t[NT][NT];   // t[I][V]; N = 32: t[I][P], columns v = 2 sigma(n) + P
            if constexpr (N == 32) {
                // x[j] + x[31 - j] and x[j] - x[31 - j] for j = 4g + s < 16 (exact integers)
#pragma unroll
                for (int I = 0; I < 2; ++I) {
                    t[I][0] = f64x4v{0.0, 0.0, 0.0, 0.0};
                    t[I][1] = t[I][0];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int xa = (int)((px[b][I][0] >> (8 * k)) & 0xffu);
                        const int xm = (int)((px[b][I][1] >> (8 * (3 - k))) & 0xffu);
                        t[I][0] = mfma_f64x4((double)(xa + xm), c1[0][0][k], t[I][0]);
                        t[I][1] = mfma_f64x4((double)(xa - xm), c1[0][1][k], t[I][1]);
                    }
                }
            } else {
#pragma unroll
                for (int I = 0; I < NT; ++I)
#pragma unroll
                    for (int V = 0; V < NT; ++V) {
                        t[I][V] = f64x4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int J = 0; J < NT; ++J)
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                t[I][V] = mfma_f64x4((double)((px[b][I][J] >> (8 * k)) & 0xffu), c1[J][V][k],
                                                     t[I][V]);
                    }
            }
            if (!live)
                continue;
            float *out = coeffs + ci * bpi_floats + (N == 8 ? (2 * cy * bw + 2 * cx) * 64 : (cy * bw + cx) * (N * N));
            const bool mine = N != 8 || (2 * cy + (n >> 3) < bh && 2 * cx + (g >> 1) < bw);
            if constexpr (N == 32) {
#pragma unroll
                for (int U = 0; U < 2; ++U) {
                    f64x4v p[2];   // p[P]: X[16 U + n][8g + 2r + P]
#pragma unroll
                    for (int P = 0; P < 2; ++P) {
                        p[P] = f64x4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int I = 0; I < 2; ++I)
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                p[P] = mfma_f64x4(t[I][P][k], c2[I][U][k], p[P]);
                    }
                    float *dst = out + (16 * U + n) * 32 + 8 * g;
                    *reinterpret_cast<float4 *>(dst) =
                        make_float4((float)p[0][0], (float)p[1][0], (float)p[0][1], (float)p[1][1]);
                    *reinterpret_cast<float4 *>(dst + 4) =
                        make_float4((float)p[0][2], (float)p[1][2], (float)p[0][3], (float)p[1][3]);
                }
            } else {
#pragma unroll
                for (int V = 0; V < NT; ++V)
#pragma unroll
                    for (int U = 0; U < NT; ++U) {
                        f64x4v p = f64x4v{0.0, 0.0, 0.0, 0.0};   // X[16 U + n][16 V + 4g + r]
#pragma unroll
                        for (int I = 0; I < NT; ++I)
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                p = mfma_f64x4(t[I][V][k], c2[I][U][k], p);
                        if (mine)
                            *reinterpret_cast<float4 *>(out + soff[U][V]) =
                                make_float4((float)p[0], (float)p[1], (float)p[2], (float)p[3]);
                    }
            }
        }
    }
}

// pix[i][j] = sum_u C[u][i] (sum_v Y[u][v] C[v][j]) in FP32.  Each thread
// owns V consecutive coefficients (V = min(N, 4)) of one row of two blocks;
// a workgroup step covers G blocks and the workgroups stride over the
// steps, so the DCT matrix is formed once per workgroup and the counters
// are reduced once per wave at the end.  Two register buffers take turns:
// each is refilled with the step two strides ahead as soon as its rows are
// staged in LDS, so every load has two steps of work to hide in (the kernel
// is bound by the bytes it keeps in flight).  For N <= 4 the thread's part
// of the DCT matrix (C[v][j0 .. j0 + V - 1] and C[u][i], for all u, v) sits
// in registers instead of being read from LDS in both passes; N = 8 keeps
// the coefficients of idct8_point for its outputs there and uses it in both
// passes.
template <int N>
__global__ __launch_bounds__(kThreads) void k_idct_u8_verify(const float *Y, int64_t B, uint8_t *pix,
                                                             const uint8_t *expected,
                                                             unsigned long long *counters, int vec_bytes)
{
    // V coefficients per thread and block row, TPB threads per block, R blocks
    // per thread and step, G = R kThreads / TPB blocks per step
    constexpr int NN = N * N, V = N < 4 ? N : 4, TPB = NN / V, R = 2, GR = kThreads / TPB, G = R * GR;
    constexpr bool kCreg = N <= 4, kBfly = N == 8;
    __shared__ __attribute__((aligned(16))) float sC[NN];
    __shared__ __attribute__((aligned(16))) float sy[G * NN];
    __shared__ __attribute__((aligned(16))) float st[G * NN];
    fill_dct(sC, N);
    __syncthreads();
    const int local = threadIdx.x / TPB, e0 = (threadIdx.x % TPB) * V;
    const int i = e0 / N, j0 = e0 % N;
    float crow[kCreg ? N : 1][V], ccol[kCreg ? N : 1];   // C[v][j0 + q], C[u][i]
    if constexpr (kCreg) {
#pragma unroll
        for (int v = 0; v < N; ++v) {
#pragma unroll
            for (int q = 0; q < V; ++q)
                crow[v][q] = sC[v * N + j0 + q];
            ccol[v] = sC[v * N + i];
        }
    }
    // N = 8: outputs j0 + q of the first pass, output i of the second
    float ce1[kBfly ? V : 1][4], co1[kBfly ? V : 1][4], ce2[4], co2[4];
    bool ne1[kBfly ? V : 1], no1[kBfly ? V : 1], ne2 = false, no2 = false;
    if constexpr (kBfly) {
#pragma unroll
        for (int q = 0; q < V; ++q)
            idct8_coeffs(sC, j0 + q, ce1[q], co1[q], ne1[q], no1[q]);
        idct8_coeffs(sC, i, ce2, co2, ne2, no2);
    }
    unsigned long long bad = 0, near = 0;
    const int64_t steps = (B + G - 1) / G;
    // block of row r of this thread in a step: step G + r GR + local
    auto load = [&](float (&y)[R][V], int64_t step) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t blk = step * G + r * GR + local;
            if (blk < B) {
                if constexpr (V == 4) {
                    const float4 v = *reinterpret_cast<const float4 *>(Y + blk * NN + e0);
                    y[r][0] = v.x;
                    y[r][1] = v.y;
                    y[r][2] = v.z;
                    y[r][3] = v.w;
                } else {
#pragma unroll
                    for (int q = 0; q < V; ++q)
                        y[r][q] = Y[blk * NN + e0 + q];
                }
            }
        }
    };
    const int64_t stride = gridDim.x;
    // One step: stage y in LDS, refill y with the step two strides ahead (its
    // load stays in flight through this step and the next), transform.
    auto process = [&](float (&y)[R][V], int64_t step) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int base = (r * GR + local) * NN;
            if (step * G + r * GR + local < B) {
#pragma unroll
                for (int q = 0; q < V; ++q)
                    sy[base + e0 + q] = y[r][q];
            }
        }
        if (step + 2 * stride < steps)
            load(y, step + 2 * stride);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int base = (r * GR + local) * NN;
            if (step * G + r * GR + local >= B)
                continue;
            float t[V];
            if constexpr (kBfly) {
                float z[8];
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    z[v] = sy[base + i * 8 + v];
#pragma unroll
                for (int q = 0; q < V; ++q)
                    t[q] = idct8_point(z, ce1[q], co1[q], ne1[q], no1[q]);
            } else {
#pragma unroll
                for (int q = 0; q < V; ++q)
                    t[q] = 0.0f;
#pragma unroll
                for (int v = 0; v < N; ++v) {
                    const float yv = sy[base + i * N + v];
#pragma unroll
                    for (int q = 0; q < V; ++q)
                        t[q] = fmaf(yv, kCreg ? crow[v][q] : sC[v * N + j0 + q], t[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < V; ++q)
                st[base + e0 + q] = t[q];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int base = (r * GR + local) * NN;
            const int64_t blk = step * G + r * GR + local;
            if (blk >= B)
                continue;
            const int64_t off = blk * NN + e0;
            uint8_t qv[V];
            bool nh[V];
            float pv[V];
            if constexpr (kBfly) {
                float z[8][V];
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int q = 0; q < V; ++q)
                        z[u][q] = st[base + u * 8 + j0 + q];
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    const float zc[8] = {z[0][q], z[1][q], z[2][q], z[3][q], z[4][q], z[5][q], z[6][q], z[7][q]};
                    pv[q] = idct8_point(zc, ce2, co2, ne2, no2);
                }
            } else {
#pragma unroll
                for (int q = 0; q < V; ++q)
                    pv[q] = 0.0f;
#pragma unroll
                for (int u = 0; u < N; ++u) {
                    const float c = kCreg ? ccol[u] : sC[u * N + i];
#pragma unroll
                    for (int q = 0; q < V; ++q)
                        pv[q] = fmaf(c, st[base + u * N + j0 + q], pv[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const float p = pv[q];
                const float rr = floorf(p + 0.5f);
                qv[q] = (uint8_t)(rr > 0.0f ? (rr > 255.0f ? 255.0f : rr) : 0.0f);
                nh[q] = fabsf(p - floorf(p) - 0.5f) < 1e-3f;
                near += nh[q] ? 1 : 0;
            }
            if (V == 4 && vec_bytes) {
                const uint32_t packed = (uint32_t)qv[0] | ((uint32_t)qv[1] << 8) | ((uint32_t)qv[2] << 16) |
                                        ((uint32_t)qv[3] << 24);
                *reinterpret_cast<uint32_t *>(pix + off) = packed;
                if (expected != nullptr) {
                    const uint32_t ex = *reinterpret_cast<const uint32_t *>(expected + off);
#pragma unroll
                    for (int q = 0; q < V; ++q)
                        bad += (!nh[q] && (uint8_t)(ex >> (8 * q)) != qv[q]) ? 1 : 0;
                }
            } else {
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    pix[off + q] = qv[q];
                    if (expected != nullptr)
                        bad += (!nh[q] && expected[off + q] != qv[q]) ? 1 : 0;
                }
            }
        }
        // the next step writes sy before its first barrier: every read of
        // sy in this step happened before this step's second barrier
    };
    // two register buffers used in turn, so no load result is ever copied
    // (a copy would wait for the load)
    float ya[R][V], yb[R][V];
    if (blockIdx.x < steps)
        load(ya, blockIdx.x);
    if (blockIdx.x + stride < steps)
        load(yb, blockIdx.x + stride);
    for (int64_t step = blockIdx.x; step < steps; step += 2 * stride) {
        process(ya, step);
        if (step + stride < steps)
            process(yb, step + stride);
    }
    if (counters != nullptr) {
        // per-wave sums, one atomic per wave and counter
        for (int d = 32; d >= 1; d >>= 1) {
            bad += __shfl_xor(bad, d);
            near += __shfl_xor(near, d);
        }
        if ((threadIdx.x & 63) == 0) {
            if (bad)
                atomicAdd(&counters[0], bad);
            if (near)
                atomicAdd(&counters[1], near);
        }
    }
}

// N = 16 and 32: both passes on FP32 MFMA 16x16x4, one 16 x 16 tile per wave
// at a time, no data moved between lanes.  Lane (n, g) = (lane % 16,
// lane / 16) loads Y[n][4g .. 4g + 3] of the tile (one 16-byte load): those
// are the A operand of the four k-steps s of T = Y C, k-step s taking
// contraction index 4g + s from lane group g; the B operand is C[4g + s][n],
// constants of the lane.  The result holds T[4g + r][n] in lane (n, g), which
// is the A operand of k-step r of P^t = T^t C, again with C[4g + s][n] as B;
// that result holds
// P[n][4g .. 4g + 3], four consecutive pixels of row n, converted and stored as
// one 32-bit word (four bytes when the pixel buffers are not 4-byte aligned).
// N = 16: a tile is a block.  N = 32: a block is 2 x 2 tiles, and each pass
// uses the basis symmetry C[v][31 - j] = (-1)^v C[v][j]: the even and odd
// contraction slices (k-steps 0, 2 and 1, 3 of each tile, the same C[16V +
// 4g + k][n] as B) give E and O for output columns j < 16, and then
// T[.][j] = E + O and T[.][31 - j] = E - O; column 31 - j sits in lane
// 15 - j of the other tile, so that half moves across the lane's 16-lane
// row (DPP row_mirror).  16 MFMAs per pass instead of 32.  NB blocks per
// wave step: all their loads are issued first.  The sums run in a fixed
// order, so every call gives the same pixels.
template <int N, int NB, bool COUNT>
__global__ __launch_bounds__(kThreads) void k_idct_u8_verify_mfma(const float *Y, int64_t B, uint8_t *pix,
                                                                  const uint8_t *expected,
                                                                  unsigned long long *counters, int vec)
{
    constexpr int NT = N / 16, NN = N * N;
    __shared__ float sC[NN];
    fill_dct(sC, N);
    __syncthreads();
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    float cb[NT][NT][4];   // C[16 V + 4g + s][16 J + n]
#pragma unroll
    for (int V = 0; V < NT; ++V)
#pragma unroll
        for (int J = 0; J < NT; ++J)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                cb[V][J][k] = sC[(16 * V + 4 * g + k) * N + 16 * J + n];
    // this lane's element offset in tile (U, V) of a block
    auto offset = [&](int U, int V) { return (16 * U + n) * N + 16 * V + 4 * g; };
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), waves = (int64_t)gridDim.x * 4;
    const int64_t units = (B + NB - 1) / NB;
    unsigned bad = 0, near = 0;
    for (int64_t unit = wave; unit < units; unit += waves) {
        f32x4 y[NB][NT][NT];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            int64_t blk = unit * NB + b;
            blk = blk < B ? blk : B - 1;   // clamped: nothing is stored for it
#pragma unroll
            for (int U = 0; U < NT; ++U)
#pragma unroll
                for (int V = 0; V < NT; ++V)
                    y[b][U][V] = *reinterpret_cast<const f32x4 *>(Y + blk * NN + offset(U, V));
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int64_t blk = unit * NB + b;
            f32x4 t[NT][NT];   // tile (U, J) of T = Y C
            f32x4 pt[NT][NT];  // tile (J, I) of P^t = T^t C
            if constexpr (N == 32) {
#pragma unroll
                for (int U = 0; U < 2; ++U) {
                    f32x4 e = f32x4{0.f, 0.f, 0.f, 0.f}, o = e;
#pragma unroll
                    for (int V = 0; V < 2; ++V)
#pragma unroll
                        for (int k = 0; k < 4; k += 2) {
                            e = mfma_f32(y[b][U][V][k], cb[V][0][k], e);
                            o = mfma_f32(y[b][U][V][k + 1], cb[V][0][k + 1], o);
                        }
                    t[U][0] = e + o;
                    t[U][1] = row_mirror4(e - o);
                }
#pragma unroll
                for (int J = 0; J < 2; ++J) {
                    f32x4 e = f32x4{0.f, 0.f, 0.f, 0.f}, o = e;
#pragma unroll
                    for (int U = 0; U < 2; ++U)
#pragma unroll
                        for (int k = 0; k < 4; k += 2) {
                            e = mfma_f32(t[U][J][k], cb[U][0][k], e);
                            o = mfma_f32(t[U][J][k + 1], cb[U][0][k + 1], o);
                        }
                    pt[J][0] = e + o;
                    pt[J][1] = row_mirror4(e - o);
                }
            } else {
#pragma unroll
                for (int U = 0; U < NT; ++U)
#pragma unroll
                    for (int J = 0; J < NT; ++J) {
                        t[U][J] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int V = 0; V < NT; ++V)
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                t[U][J] = mfma_f32(y[b][U][V][k], cb[V][J][k], t[U][J]);
                    }
#pragma unroll
                for (int J = 0; J < NT; ++J)
#pragma unroll
                    for (int I = 0; I < NT; ++I) {
                        pt[J][I] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int U = 0; U < NT; ++U)
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                pt[J][I] = mfma_f32(t[U][J][k], cb[U][I][k], pt[J][I]);
                    }
            }
#pragma unroll
            for (int J = 0; J < NT; ++J)
#pragma unroll
                for (int I = 0; I < NT; ++I) {
                    const f32x4 p = pt[J][I];
                    if (blk >= B)
                        continue;
                    // P[16 I + n][16 J + 4g + r]: tile (I, J) of the block
                    const int64_t off = blk * NN + offset(I, J);
                    const uint32_t w = pack_u8x4(p[0], p[1], p[2], p[3]);
                    uint32_t ex = 0;
                    if (vec) {
                        *reinterpret_cast<uint32_t *>(pix + off) = w;
                        if (COUNT && expected != nullptr)
                            ex = *reinterpret_cast<const uint32_t *>(expected + off);
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            pix[off + r] = (uint8_t)(w >> (8 * r));
                            if (COUNT && expected != nullptr)
                                ex |= (uint32_t)expected[off + r] << (8 * r);
                        }
                    }
                    if constexpr (COUNT) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const unsigned nh = fabsf(p[r] - floorf(p[r]) - 0.5f) < 1e-3f ? 1u : 0u;
                            near += nh;
                            if (expected != nullptr)
                                bad += ((((ex ^ w) >> (8 * r)) & 0xffu) != 0u ? 1u : 0u) & (nh ^ 1u);
                        }
                    }
                }
        }
    }
    if (COUNT && counters != nullptr) {
        for (int d = 32; d >= 1; d >>= 1) {
            bad += __shfl_xor(bad, d);
            near += __shfl_xor(near, d);
        }
        if (lane == 0) {
            if (bad)
                atomicAdd(&counters[0], (unsigned long long)bad);
            if (near)
                atomicAdd(&counters[1], (unsigned long long)near);
        }
    }
}

// units per wave step of k_forward_dct_mfma: N = 8 and 16 (16 x 16 pixels
// each; 4 and 32 were 2-8 % slower), N = 32 (32 x 32; 2 and 8 were slower)
constexpr int kFdctNb = 8;
constexpr int kFdctNb32 = 4;
// blocks per wave step of k_idct_u8_verify_mfma
constexpr int kVerifyNb16 = 4;
constexpr int kVerifyNb32 = 2;

// Plain streaming copy: each wave moves 4 KiB per step (4 x 1 KiB contiguous
// 16-byte-per-lane accesses, nontemporal), waves stride over the buffer.
typedef float f32x4c __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const f32x4c *__restrict__ in, f32x4c *__restrict__ out,
                                                     int64_t n4)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int64_t base = wave * 256;
    for (; base + 256 <= n4; base += nw * 256) {
        f32x4c v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            v[k] = __builtin_nontemporal_load(&in[base + 64 * k + lane]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            __builtin_nontemporal_store(v[k], &out[base + 64 * k + lane]);
    }
    // tail (fewer than 256 float4 left for this wave)
    for (int64_t i = base + lane; i < n4 && i < base + 256; i += 64)
        out[i] = in[i];
}

// N = 8: one block per lane, 64 blocks per wave.  The blocks move between
// HBM and the lanes through 16 KiB of wave-private LDS with 1 KiB coalesced
// accesses (float4 k of block b at 16 b + (k ^ b mod 16)), and each lane
// runs its block's two passes in registers with the DCT matrix in scalar
// registers: no barrier, and LDS carries each byte once in and once out.
// The arithmetic is that of k_idct_u8_verify (idct8_point for every output
// of both passes), so pixels and counters are identical.  The kernel is
// bound by VALU issue (a wave64 instruction takes 4 cycles of a 16-lane
// SIMD), so COUNT = false, for calls without counters, leaves out the
// near-1/2 and mismatch tests.
template <bool COUNT>
__global__ __launch_bounds__(kThreads) void k_idct_u8_verify8(const float *Y, int64_t B, uint8_t *pix,
                                                              const uint8_t *expected,
                                                              unsigned long long *counters)
{
    __shared__ float sC[64];
    __shared__ __attribute__((aligned(16))) float4 lds_all[4 * 64 * 16];
    fill_dct(sC, 8);
    __syncthreads();
    float C[64];
#pragma unroll
    for (int k = 0; k < 64; ++k)
        C[k] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sC[k])));
    const int lane = threadIdx.x & 63;
    float4 *lds = lds_all + (threadIdx.x >> 6) * 64 * 16;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), waves = (int64_t)gridDim.x * 4;
    const int64_t units = (B + 63) / 64;
    unsigned bad = 0, near = 0;   // per lane: at most 64 pixels per unit
    for (int64_t unit = wave; unit < units; unit += waves) {
        const int64_t blk0 = unit * 64;
        const int nv = (int)(B - blk0 < 64 ? B - blk0 : 64);
        // instruction m moves blocks 4m .. 4m + 3 (lane l: float4 l % 16 of block
        // 4m + l / 16); all 16 loads are issued before the first LDS write (a
        // branch per load would wait for each in turn), past the last block
        // clamped to it (those slots are never stored)
        float4 xin[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int b = 4 * m + (lane >> 4), k = lane & 15;
            const int bb = b < nv ? b : nv - 1;
            xin[m] = *reinterpret_cast<const float4 *>(Y + (blk0 + bb) * 64 + 4 * k);
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int b = 4 * m + (lane >> 4), k = lane & 15;
            lds[b * 16 + (k ^ (b & 15))] = xin[m];
        }
        wave_lds_sync();
        float y[64];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const float4 v = lds[lane * 16 + (k ^ (lane & 15))];
            y[4 * k] = v.x;
            y[4 * k + 1] = v.y;
            y[4 * k + 2] = v.z;
            y[4 * k + 3] = v.w;
        }
        wave_lds_sync();
        // t[u][j] = sum_v Y[u][v] C[v][j], row by row in place
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            float z[8], t[8];
#pragma unroll
            for (int v = 0; v < 8; ++v)
                z[v] = y[8 * u + v];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                float ce[4], co[4];
                bool ne, no;
                idct8_coeffs(C, j, ce, co, ne, no);
                t[j] = idct8_point(z, ce, co, ne, no);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
                y[8 * u + j] = t[j];
        }
        // p[i][j] = sum_u C[u][i] t[u][j], column by column in place
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float z[8], pc[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                z[u] = y[8 * u + j];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                float ce[4], co[4];
                bool ne, no;
                idct8_coeffs(C, i, ce, co, ne, no);
                pc[i] = idct8_point(z, ce, co, ne, no);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i)
                y[8 * i + j] = pc[i];
        }
        // uint8 and the counters
        const unsigned mine = lane < nv ? 1u : 0u;
        uint32_t packed[16];
        uint4 ex[4] = {};
        if (COUNT && expected != nullptr) {
            const int bl = lane < nv ? lane : nv - 1;   // clamped: counted only for lane < nv
#pragma unroll
            for (int h = 0; h < 4; ++h)
                ex[h] = *reinterpret_cast<const uint4 *>(expected + (blk0 + bl) * 64 + 16 * h);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float *pv = y + 8 * i;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // the same bytes as the general kernel's clamp for every finite value
                const uint32_t w = pack_u8x4(pv[4 * h], pv[4 * h + 1], pv[4 * h + 2], pv[4 * h + 3]);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if constexpr (COUNT) {
                        const float pq = pv[4 * h + q];
                        const uint32_t qv = (w >> (8 * q)) & 0xffu;
                        const unsigned nh = fabsf(pq - floorf(pq) - 0.5f) < 1e-3f ? 1u : 0u;
                        near += nh & mine;
                        if (expected != nullptr) {
                            const int e = 8 * i + 4 * h + q;   // pixel index in the block
                            const uint4 x4 = ex[e >> 4];
                            const uint32_t xw = (e & 15) < 4 ? x4.x : (e & 15) < 8 ? x4.y : (e & 15) < 12 ? x4.z : x4.w;
                            bad += (((xw >> (8 * (e & 3))) & 0xffu) != qv ? 1u : 0u) & (nh ^ 1u) & mine;
                        }
                    }
                }
                packed[2 * i + h] = w;
            }
        }
        // out: 64 B per lane through LDS (uint4 h of block b at 4 b + (h ^ b mod 4)), then
        // instruction m stores blocks 16m .. 16m + 15 (lane l: uint4 l % 4 of block 16m + l / 4)
        uint4 *ldo = reinterpret_cast<uint4 *>(lds);
#pragma unroll
        for (int h = 0; h < 4; ++h)
            ldo[lane * 4 + (h ^ (lane & 3))] =
                make_uint4(packed[4 * h], packed[4 * h + 1], packed[4 * h + 2], packed[4 * h + 3]);
        wave_lds_sync();
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int b = 16 * m + (lane >> 2), h = lane & 3;
            if (b < nv)
                *reinterpret_cast<uint4 *>(pix + (blk0 + b) * 64 + 16 * h) = ldo[b * 4 + (h ^ (b & 3))];
        }
        wave_lds_sync();
    }
    if (COUNT && counters != nullptr) {
        for (int d = 32; d >= 1; d >>= 1) {
            bad += __shfl_xor(bad, d);
            near += __shfl_xor(near, d);
        }
        if (lane == 0) {
            if (bad)
                atomicAdd(&counters[0], (unsigned long long)bad);
            if (near)
                atomicAdd(&counters[1], (unsigned long long)near);
        }
    }
}

}  // namespace

hipError_t launch_stream_copy(const float *in, float *out, int64_t n, hipStream_t stream)
{
    const int64_t n4 = n / 4;
    // up to one step per wave: a launch of many short-lived workgroups keeps
    // more loads in flight as waves end than a few long grid-stride loops
    // (1 GiB, 4 KiB per wave and step: 6.23 TB/s at 256 workgroups per CU
    // (one step), 6.15 at 64, 5.98 at 16, 5.88 at the resident 8)
    int64_t groups = (int64_t)cu_count() * 256;
    const int64_t need = (n4 + 1023) / 1024;   // 4 waves x 256 float4 per group and step
    groups = groups < need ? groups : need;
    if (groups <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)groups), dim3(256), 0, stream,
                       reinterpret_cast<const f32x4c *>(in), reinterpret_cast<f32x4c *>(out), n4);
    return hipGetLastError();
}

hipError_t launch_forward_dct_u8(const uint8_t *img, int h, int w, int64_t pitch, int64_t img_stride,
                                 int64_t nimg, int N, float *coeffs, hipStream_t stream)
{
    if (N == 8 || N == 16 || N == 32) {
        const int64_t bh = (h + N - 1) / N, bw = (w + N - 1) / N;
        const int64_t ubh = N == 8 ? (bh + 1) / 2 : bh, ubw = N == 8 ? (bw + 1) / 2 : bw;
        const int64_t upi = ubh * ubw, units = upi * nimg;
        // 32-bit pixel loads need every image's rows 4-byte aligned
        const int aligned4 = ((uintptr_t)img & 3u) == 0 && (pitch & 3) == 0 && (nimg == 1 || (img_stride & 3) == 0);
        auto launch = [&](auto kernel, int nb, int slot_id) {
            static std::atomic<int> resident[4];
            std::atomic<int> &slot = resident[slot_id];
            int per_cu = slot.load(std::memory_order_relaxed);
            if (per_cu == 0) {
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess ||
                    per_cu < 1)
                    per_cu = 1;
                slot.store(per_cu, std::memory_order_relaxed);
            }
            int64_t groups = (int64_t)cu_count() * per_cu;
            const int64_t need = (units + 4 * nb - 1) / (4 * nb);
            groups = groups < need ? groups : need;
            hipLaunchKernelGGL(kernel, dim3((unsigned)groups), dim3(kThreads), 0, stream, img, h, w, pitch, coeffs,
                               bh, bw, ubw, units, aligned4, upi, img_stride);
        };
        // images too small to give every resident wave a few steps of kFdctNb
        // units (one 2048 x 2048 image at N = 8 is 16,384 units) take two units
        // per step: more waves share the image, and each waits on fewer loads
        const bool small = units < (int64_t)cu_count() * 64 * kFdctNb;
        if (N == 8 && small)
            launch(k_forward_dct_mfma<8, 2>, 2, 3);
        else if (N == 8)
            launch(k_forward_dct_mfma<8, kFdctNb>, kFdctNb, 0);
        else if (N == 16)
            launch(k_forward_dct_mfma<16, kFdctNb>, kFdctNb, 1);
        else
            launch(k_forward_dct_mfma<32, kFdctNb32>, kFdctNb32, 2);
        return hipGetLastError();
    }
    const int64_t nblocks = (int64_t)((h + N - 1) / N) * ((w + N - 1) / N);
    const int threads = N * N > kThreads ? N * N : kThreads;   // <= kMaxDctThreads (N <= 32)
    const int per = threads / (N * N);
    const int64_t groups = (nblocks + per - 1) / per;
    for (int64_t i = 0; i < nimg; ++i) {   // small blocks: one launch per image
        hipLaunchKernelGGL(k_forward_dct_u8, dim3((unsigned)groups), dim3(threads), 0, stream, img + i * img_stride,
                           h, w, pitch, N, coeffs + i * nblocks * N * N, nblocks);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_idct_u8_verify(int N, const float *Y, int64_t B, uint8_t *pix,
                                 const uint8_t *expected, unsigned long long *counters,
                                 hipStream_t stream)
{
    const int V = N < 4 ? N : 4;
    const int64_t G = 2 * (kThreads / (N * N / V));   // blocks per step (R = 2 per thread)
    const int64_t steps = (B + G - 1) / G;
    const int vec = ((uintptr_t)pix & 3u) == 0 && ((uintptr_t)expected & 3u) == 0;
    // A persistent grid: as many workgroups as can be resident at once (the
    // block sizes differ in registers per thread, so in occupancy).
    // (queried once per block size; concurrent first calls store the same value)
    static std::atomic<int> resident[6];
    auto launch = [&](auto kernel) {
        std::atomic<int> &slot = resident[__builtin_ctz((unsigned)N)];
        int per_cu = slot.load(std::memory_order_relaxed);
        if (per_cu == 0) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess ||
                per_cu < 1)
                per_cu = 1;
            slot.store(per_cu, std::memory_order_relaxed);
        }
        int64_t groups = (int64_t)cu_count() * per_cu;
        groups = groups < steps ? groups : steps;
        hipLaunchKernelGGL(kernel, dim3((unsigned)groups), dim3(kThreads), 0, stream, Y, B, pix, expected, counters,
                           vec);
    };
    if (N == 16 || N == 32) {
        // every call of these sizes, aligned or not, runs the MFMA kernel (same pixels)
        const bool count = counters != nullptr;
        static std::atomic<int> resident_m[4];
        auto launch_m = [&](auto kernel, int slot_id, int nb) {
            std::atomic<int> &slot = resident_m[slot_id];
            int per_cu = slot.load(std::memory_order_relaxed);
            if (per_cu == 0) {
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess ||
                    per_cu < 1)
                    per_cu = 1;
                slot.store(per_cu, std::memory_order_relaxed);
            }
            const int64_t units = (B + nb - 1) / nb;
            int64_t groups = (int64_t)cu_count() * per_cu;
            const int64_t need = (units + 3) / 4;
            groups = groups < need ? groups : need;
            hipLaunchKernelGGL(kernel, dim3((unsigned)groups), dim3(kThreads), 0, stream, Y, B, pix, expected,
                               counters, vec);
        };
        if (N == 16) {
            if (count)
                launch_m(k_idct_u8_verify_mfma<16, kVerifyNb16, true>, 0, kVerifyNb16);
            else
                launch_m(k_idct_u8_verify_mfma<16, kVerifyNb16, false>, 1, kVerifyNb16);
        } else {
            if (count)
                launch_m(k_idct_u8_verify_mfma<32, kVerifyNb32, true>, 2, kVerifyNb32);
            else
                launch_m(k_idct_u8_verify_mfma<32, kVerifyNb32, false>, 3, kVerifyNb32);
        }
        return hipGetLastError();
    }
    const bool aligned = ((uintptr_t)pix & 15u) == 0 && ((uintptr_t)expected & 15u) == 0;
    if (N == 8 && aligned) {
        // the counting kernel when counters are asked for (a mismatch count needs them)
        const bool count = counters != nullptr;
        static std::atomic<int> resident8[2];
        std::atomic<int> &slot = resident8[count ? 1 : 0];
        int per_cu = slot.load(std::memory_order_relaxed);
        if (per_cu == 0) {
            const hipError_t e =
                count ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_idct_u8_verify8<true>, kThreads, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_idct_u8_verify8<false>, kThreads, 0);
            if (e != hipSuccess || per_cu < 1)
                per_cu = 1;
            slot.store(per_cu, std::memory_order_relaxed);
        }
        const int64_t units = (B + 63) / 64;
        int64_t groups = (int64_t)cu_count() * per_cu;
        const int64_t need = (units + 3) / 4;
        groups = groups < need ? groups : need;
        if (count)
            hipLaunchKernelGGL(k_idct_u8_verify8<true>, dim3((unsigned)groups), dim3(kThreads), 0, stream, Y, B, pix,
                               expected, counters);
        else
            hipLaunchKernelGGL(k_idct_u8_verify8<false>, dim3((unsigned)groups), dim3(kThreads), 0, stream, Y, B,
                               pix, expected, counters);
        return hipGetLastError();
    }
    switch (N) {
    case 2: launch(k_idct_u8_verify<2>); break;
    case 4: launch(k_idct_u8_verify<4>); break;
    default: launch(k_idct_u8_verify<8>); break;
    }
    return hipGetLastError();
}

}  // namespace dctf
