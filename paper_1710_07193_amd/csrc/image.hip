// Image-level filtering in the DCT domain: every output block is a sum over
// its 3 x 3 block neighbourhood,
//
//   Y[R][S] = sum_{dr, ds in {-1, 0, 1}} H^{c(R), c(S)}_{dr, ds} . X[R + dr][S + ds],
//
// the image filtered across block boundaries (the variant the paper's
// block-edge replication of Fig. 1 approximates), with zero padding or
// replication only at the image border.  H_{dr,ds} is the Kronecker form of
// the paper's DCT-domain products (eq. 6-8) with shift matrices that may
// select rows of the neighbour block:
//
//   H^{cr,cs}_{dr,ds} = sum_{p,q} W[p][q] A^{cr}_{dr, p-a_h} (x) A^{cs}_{ds, q-a_w},
//   A^{c}_{d,e} = C S^{c}_{d,e} C^t,
//
// where S^{c}_{d,e}[i][m] = 1 if output row i, shifted by e, reads row m of
// the neighbour at offset d.  The class c of a block row (or column) says
// which neighbours exist: bit 0 = it is the first one (no neighbour before:
// reads before it are dropped (zero) or clamped to its row 0 (replication)),
// bit 1 = it is the last one.  The builder forms all 4 x 4 class pairs x 9
// offsets in FP64 (N = 8), with their FP32 and split-BF16 MFMA fragments
// (the split path of the block-local filter: 8 low-frequency columns in
// FP32, the others as BF16 hi.hi + hi.lo + lo.hi); each operator's DC
// column is kept out of the MFMA images and applied in FP32 VALU after all
// AC products (the nine DC products are the largest terms of a sum that
// cancels: in the MFMA chain they would set the rounding step of every
// later addition).
//
// The filter kernel partitions each image into at most 9 rectangles of one
// class pair (interior, 4 edges, 4 corners) and those into tiles of 16 blocks
// along a block row (or, for a one-block-wide rectangle, a block column).
// A wave takes T tiles of one rectangle, loads the fragments of one
// neighbour operator at a time into VGPRs and accumulates its product over
// the T tiles before moving to the next neighbour (the operator is read
// once per T tiles, the neighbour blocks come from L2).  Units are handed
// out in XCD order (xcd_wave), so the units that share block rows run on
// the same XCD and read those rows through one L2.
#include "mfma_common.h"

namespace dctf {
namespace {

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup g runs on
// XCD g % 8), and each XCD has its own L2.  xcd_wave() renumbers the waves of
// a grid whose workgroup count is a multiple of 8 so that consecutive
// numbers run on the same XCD: XCD x holds numbers [x W/8, (x + 1) W/8)
// (W = all waves).  Kernels whose neighbouring work units share input hand
// units out in this order, so the sharing happens inside one L2.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_wave(int waves_per_group)
{
    const int64_t per_xcd = gridDim.x / kXcds;
    return ((int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds) * waves_per_group +
           (threadIdx.x >> 6);
}

// Workgroups for `waves` waves of `per` waves each, rounded up to a multiple
// of the XCD count (as xcd_wave() needs).
inline int64_t xcd_groups(int64_t waves, int per)
{
    const int64_t g = (waves + per - 1) / per;
    return (g + kXcds - 1) / kXcds * kXcds;
}

constexpr int kThreads = 256;
constexpr int kN = 8;
constexpr int kNN = kN * kN;

// Source of output row i shifted by e in a block of class c: the neighbour
// offset d (-1, 0, 1) and its row m; false if the source is dropped (zero
// padding outside the image).
template <int N>
__device__ inline bool image_source(int i, int e, int c, int border, int *d, int *m)
{
    int y = i + e;
    if (y < 0 && (c & 1)) {
        if (border == DCTF_BORDER_ZERO)
            return false;
        y = 0;
    }
    if (y >= N && (c & 2)) {
        if (border == DCTF_BORDER_ZERO)
            return false;
        y = N - 1;
    }
    *d = y < 0 ? -1 : (y >= N ? 1 : 0);
    *m = y - *d * N;
    return true;
}

// One workgroup per (class pair, offset, 16 output rows).  The mask rows p
// are taken in chunks of PC (T_p, G_p and B_p of a chunk in LDS); the sum
// over p runs in increasing p in every case, so the chunking does not change
// a result.  N = 8 takes all rows in one chunk; N = 16 takes 8 at a time
// (three N^2 arrays of 8 FP64 matrices: 48 KiB).
template <int N, int PC>
__global__ __launch_bounds__(kThreads) void k_build_image(ImageBuildArgs args)
{
    constexpr int NN = N * N, MaxK = 2 * N + 1;
    constexpr int E = 16 * NN / kThreads;   // entries per thread
    const int cp = blockIdx.y, o = blockIdx.z;
    const int cr = cp >> 2, cs = cp & 3, dr = o / 3 - 1, ds = o % 3 - 1;
    const int r0 = blockIdx.x * 16;
    const ImageBuildArgs &d = args;
    const int kh = d.kh, kw = d.kw, ah = (kh - 1) / 2, aw = (kw - 1) / 2;
    __shared__ double sC[NN];
    __shared__ double sW[MaxK * MaxK];
    __shared__ double sT[PC * NN];   // T_p = A^{cr}_{dr, p - ah}
    __shared__ double sG[PC * NN];   // G_p[j][l] = sum_q W[p][q] [row j reads m at ds] C[l][m]
    __shared__ double sB[PC * NN];   // B_p = C G_p
    const int tid = threadIdx.x;
    for (int e = tid; e < NN; e += kThreads) {
        const int k = e / N, n = e % N;
        const double alpha = (k == 0) ? sqrt(1.0 / N) : sqrt(2.0 / N);
        sC[e] = alpha * cos(M_PI * (2.0 * n + 1.0) * k / (2.0 * N));
    }
    for (int e = tid; e < kh * kw; e += kThreads)
        sW[e] = d.mask[e];
    double acc[E];
#pragma unroll
    for (int j = 0; j < E; ++j)
        acc[j] = 0.0;
    for (int p0 = 0; p0 < kh; p0 += PC) {
        const int np = kh - p0 < PC ? kh - p0 : PC;
        __syncthreads();
        for (int e = tid; e < 2 * np * NN; e += kThreads) {
            const int which = e / (np * NN), rest = e % (np * NN);
            const int pl = rest / NN, p = p0 + pl, idx = rest % NN, a = idx / N, b = idx % N;
            double s = 0.0;
            if (which == 0) {
                // T_p[u][k] = sum_i C[u][i] C[k][m(i)] over rows i that read neighbour dr
                for (int i = 0; i < N; ++i) {
                    int dd, m;
                    if (image_source<N>(i, p - ah, cr, d.border, &dd, &m) && dd == dr)
                        s += sC[a * N + i] * sC[b * N + m];
                }
                sT[pl * NN + idx] = s;
            } else {
                // G_p[j][l] with (j, l) = (a, b)
                for (int q = 0; q < kw; ++q) {
                    int dd, m;
                    if (image_source<N>(a, q - aw, cs, d.border, &dd, &m) && dd == ds)
                        s += sW[p * kw + q] * sC[b * N + m];
                }
                sG[pl * NN + idx] = s;
            }
        }
        __syncthreads();
        for (int e = tid; e < np * NN; e += kThreads) {
            const int pl = e / NN, idx = e % NN, v = idx / N, l = idx % N;
            double s = 0.0;
            for (int j = 0; j < N; ++j)
                s += sC[v * N + j] * sG[pl * NN + j * N + l];
            sB[e] = s;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int e = tid + j * kThreads;
            const int r = r0 + e / NN, c = e % NN;
            const int u = r / N, v = r % N, k = c / N, l = c % N;
            double s = acc[j];
            for (int pl = 0; pl < np; ++pl)
                s += sT[pl * NN + u * N + k] * sB[pl * NN + v * N + l];
            acc[j] = s;
        }
    }
    const size_t opi = (size_t)cp * 9 + o;
    double *H64 = d.H64 + opi * NN * NN;
    float *F32 = d.frag32 + opi * NN * NN;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int e = tid + j * kThreads;
        const int r = r0 + e / NN, c = e % NN;
        const double s = acc[j];
        H64[(size_t)r * NN + c] = s;
        // the DC column goes to h0 (FP32 VALU in the filter), not to the MFMA images
        const float h32 = __double2float_rn(s);
        F32[frag32_index(N, r, c)] = c == 0 ? 0.0f : h32;
        if (c == 0)
            d.h0[opi * NN + r] = h32;
        // split images: low-frequency columns (DC zeroed) in FP32, the rest as
        // BF16 hi = bf16(fp32(H)), lo = bf16(fp32(H - hi))
        const int q = lf_slot(N, c);
        uint16_t hi = 0, lo = 0;
        if (q >= 0) {
            const int t = r >> 4, m = r & 15, lane = 16 * (q >> 1) + m;
            d.frag_lf[opi * NN * lf_count(N) + (t * 64 + lane) * 2 + (q & 1)] = c == 0 ? 0.0f : h32;
        } else {
            hi = bf16_rne(h32);
            lo = bf16_rne(__double2float_rn(s - (double)bf16_to_f32(hi)));
        }
        const size_t fi = opi * NN * NN + frag16_index(N, r, c);
        d.frag_hi[fi] = hi;
        d.frag_lo[fi] = lo;
    }
}

// ------------------------------------------------------------- filter

// Tile t of rectangle `rc` in image `img`: the first block's (R, S), the
// step between its blocks (1 along a row, Bw along a column) and the count.
struct TileRef {
    int64_t blk0;     // raster index of the tile's first block within the image
    int64_t step;
    int count;
};

__device__ inline TileRef tile_ref(const ImageRect &rc, int64_t t, int Bw)
{
    TileRef r;
    if (rc.dir == 0) {
        const int64_t tps = (rc.nS + 15) / 16;
        const int64_t row = rc.R0 + t / tps, seg = t % tps;
        r.blk0 = row * Bw + rc.S0 + 16 * seg;
        r.step = 1;
        r.count = (int)min((int64_t)16, (int64_t)rc.nS - 16 * seg);
    } else {
        const int64_t tps = (rc.nR + 15) / 16;
        const int64_t col = rc.S0 + t / tps, seg = t % tps;
        r.blk0 = (rc.R0 + 16 * seg) * Bw + col;
        r.step = Bw;
        r.count = (int)min((int64_t)16, (int64_t)rc.nR - 16 * seg);
    }
    return r;
}

// Wave w takes units w, w + waves, ...; a unit is up to T consecutive tiles
// of one rectangle of one image.
//
// LOPS (split path): the workgroup (8 waves, one per CU) first copies the
// fragments of the 8 non-centre neighbour operators of class pair lds_cp
// (the interior, which holds nearly every block) into LDS, 144 KiB, and its
// units of that class pair read them from there; the centre operator and
// every other class pair come from L2 as before.  Fragment traffic from L2,
// which bounds the kernel, drops from 9 to 1 operator per unit.
constexpr int kOpHalf = 4 * 2 * 64 * 8;   // BF16 of one operator's hi (or lo) fragments
constexpr int kOpLf = 4 * 64 * 2;         // floats of its low-frequency fragments
constexpr int kLdsOps = 8;                // resident operators: offsets 0-3, 5-8

template <int PREC, int T, bool LOPS>
__global__ __launch_bounds__(LOPS ? 512 : 256) void k_filter_image8(ImageFilterArgs a, int64_t units, int64_t waves,
                                                                    int lds_cp)
{
    __shared__ __attribute__((aligned(16))) uint16_t s_hl[LOPS ? kLdsOps * 2 * kOpHalf : 8];
    __shared__ __attribute__((aligned(16))) float s_lf[LOPS ? kLdsOps * kOpLf : 4];
    if constexpr (LOPS) {
        if (lds_cp >= 0) {
            // slot q holds offset q < 4 ? q : q + 1: hi at 2q kOpHalf, lo after it
            for (int e = threadIdx.x; e < kLdsOps * 2 * kOpHalf / 8; e += blockDim.x) {
                const int q = e / (2 * kOpHalf / 8), r = e % (2 * kOpHalf / 8);
                const size_t opi = (size_t)lds_cp * 9 + (q < 4 ? q : q + 1);
                const uint16_t *src = r < kOpHalf / 8 ? a.frag_hi + opi * kNN * kNN + 8 * r
                                                      : a.frag_lo + opi * kNN * kNN + 8 * (r - kOpHalf / 8);
                reinterpret_cast<u32x4 *>(s_hl)[e] = *reinterpret_cast<const u32x4 *>(src);
            }
            for (int e = threadIdx.x; e < kLdsOps * kOpLf / 4; e += blockDim.x) {
                const int q = e / (kOpLf / 4), r = e % (kOpLf / 4);
                const size_t opi = (size_t)lds_cp * 9 + (q < 4 ? q : q + 1);
                reinterpret_cast<float4 *>(s_lf)[e] =
                    *reinterpret_cast<const float4 *>(a.frag_lf + opi * kNN * lf_count(kN) + 4 * r);
            }
        }
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    // consecutive units (the same and adjacent block rows) run on one XCD
    // a scalar: the unit decode below (image, rectangle, tiles) runs on the scalar unit
    const int64_t wave = __builtin_amdgcn_readfirstlane((int)xcd_wave(LOPS ? 8 : 4));
    if (wave >= waves)
        return;
    const int64_t per_img_blocks = (int64_t)a.Bh * a.Bw;
    for (int64_t unit = wave; unit < units; unit += waves) {
        const int64_t img = unit / a.units_per_image;
        const int64_t lu = unit % a.units_per_image;
        int ri = 0;
        while (ri + 1 < a.nrect && a.rect[ri + 1].unit_begin <= lu)
            ++ri;
        const ImageRect &rc = a.rect[ri];
        const int64_t t0 = (lu - rc.unit_begin) * T;
        const int nt = (int)min((int64_t)T, rc.tiles - t0);
        const float *X = a.in + img * per_img_blocks * kNN;
        float *Y = a.out + img * per_img_blocks * kNN;
        // this lane's block of each tile (clamped to the tile's first block past the count)
        int64_t blk[T];
        bool valid[T];
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            if (tt < nt) {
                const TileRef r = tile_ref(rc, t0 + tt, a.Bw);
                valid[tt] = n < r.count;
                blk[tt] = r.blk0 + (valid[tt] ? n : 0) * r.step;
            } else {
                valid[tt] = false;
                blk[tt] = 0;
            }
        }
        f32x4 acc[T][4];
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[tt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
        float x0s[T][9];
        // tile tt of the neighbour at offset o.  FP32 path: the first tile of each
        // offset is loaded during the last tile of the offset before (no wait at the
        // switch; 3.18 -> 3.11 ms); the split path has no registers left for it (3
        // spilled, slower) and loads it at the switch.
        constexpr bool kCross = PREC == DCTF_PREC_FP32;
        auto shift_of = [&](int o) { return (int64_t)(o / 3 - 1) * a.Bw + (o % 3 - 1); };
        auto load = [&](float4 (&x)[4], int tt, int64_t shift) {
            const float *src = X + (blk[tt] + shift) * kNN + 4 * g;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                x[i] = ld4(src + 16 * i);
        };
        float4 cur[4], nxt[4];
        if constexpr (kCross)
            load(cur, 0, shift_of(__builtin_ctz((unsigned)rc.offsets)));   // the centre is always present
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            if (!((rc.offsets >> o) & 1))
                continue;
            const int64_t shift = shift_of(o);
            const unsigned rest = (unsigned)rc.offsets >> (o + 1);   // offsets still to come
            const size_t opi = (size_t)rc.cp * 9 + o;
            float A[4][4][4];
            OpRegs8BF16 R;
            if constexpr (PREC == DCTF_PREC_FP32) {
                const float *F = a.frag32 + opi * kNN * kNN;
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float4 v = ld4(F + ((t * 4 + i) * 64 + lane) * 4);
                        A[t][i][0] = v.x;
                        A[t][i][1] = v.y;
                        A[t][i][2] = v.z;
                        A[t][i][3] = v.w;
                    }
            } else if (LOPS && rc.cp == lds_cp && o != 4) {
                const int q = o < 4 ? o : o - 1;
                load_op8_lds(R, s_hl + 2 * q * kOpHalf, s_hl + (2 * q + 1) * kOpHalf, s_lf + q * kOpLf, lane);
            } else {
                load_op8(R, a.frag_hi + opi * kNN * kNN, a.frag_lo + opi * kNN * kNN,
                         a.frag_lf + opi * kNN * lf_count(kN), lane);
            }
            if constexpr (!kCross)
                load(cur, 0, shift);
#pragma unroll
            for (int tt = 0; tt < T; ++tt) {
                if (tt >= nt)
                    break;
                if (tt + 1 < nt)
                    load(nxt, tt + 1, shift);
                else if (kCross && rest != 0)
                    load(nxt, 0, shift_of(o + 1 + __builtin_ctz(rest)));
                // DC of the neighbour block (lane (n, 0) holds coefficient 0 of block n),
                // applied after every AC product
                x0s[tt][o] = lane_read(cur[0].x, n);
                if constexpr (PREC == DCTF_PREC_FP32) {
                    // rows u = 7, 6 first, u = 1, 0 last (FP32 accuracy)
#pragma unroll
                    for (int i = 3; i >= 0; --i) {
                        const float xv[4] = {cur[i].x, cur[i].y, cur[i].z, cur[i].w};
#pragma unroll
                        for (int j = 0; j < 4; ++j)
#pragma unroll
                            for (int t = 0; t < 4; ++t)
                                acc[tt][t] = mfma_f32(A[t][i][j], xv[j], acc[tt][t]);
                    }
                } else {
                    tile8_acc(R, cur, acc[tt]);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    cur[i] = nxt[i];
            }
        }
        // the DC columns, in FP32 VALU, in offset order
#pragma unroll
        for (int o = 0; o < 9; ++o) {
            if (!((rc.offsets >> o) & 1))
                continue;
            const float *D = a.h0 + ((size_t)rc.cp * 9 + o) * kNN + 4 * g;
            float4 h0[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                h0[t] = ld4(D + 16 * t);
#pragma unroll
            for (int tt = 0; tt < T; ++tt)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    acc[tt][t][0] = fmaf(h0[t].x, x0s[tt][o], acc[tt][t][0]);
                    acc[tt][t][1] = fmaf(h0[t].y, x0s[tt][o], acc[tt][t][1]);
                    acc[tt][t][2] = fmaf(h0[t].z, x0s[tt][o], acc[tt][t][2]);
                    acc[tt][t][3] = fmaf(h0[t].w, x0s[tt][o], acc[tt][t][3]);
                }
        }
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            if (tt < nt && valid[tt]) {
                float *dst = Y + blk[tt] * kNN + 4 * g;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    st4(dst + 16 * t, acc[tt][t]);
            }
        }
    }
}

// tiles per unit (each neighbour operator is loaded once per unit): FP32 4,
// the most the register file holds; split 3, the most beside the LDS-resident
// operators' addressing without spills (measured 1.77 ms against 1.84 for 2)
constexpr int kImageT32 = 4;
constexpr int kImageTSplit = 3;
constexpr int kImageWavesPerCu = 8;

// ------------------------------------------------------- filter, N = 16
//
// A workgroup of 8 waves holds one 256 x 256 neighbour operator in VGPRs
// (wave w: output rows 32w .. 32w + 31), as the block-local N = 16 kernel
// does.  A unit is up to T tiles of 16 blocks of one rectangle; one step is
// one neighbour offset of a unit: its T neighbour tiles are in LDS together
// (two sets of T tile buffers: the next step's tiles are loaded while this
// step's are multiplied), and the MFMA work runs k-step by k-step over the
// T tiles, so that each k-step's operator fragments are free once that
// k-step is done: they are reloaded with the next step's operator (256 KiB
// per workgroup, from L2: the 9 operators of the interior class pair,
// 2.25 MiB, stay in each XCD's L2) while the later k-steps run.  Every step
// issues the same loads (past the last unit: empty tiles and the current
// operator again), so no step waits for more than its own data.  The DC
// coefficients of the neighbour blocks are kept in LDS when a tile set is
// staged and applied with the operators' DC columns in FP32 VALU after every
// MFMA product, in offset order.  Workgroups take units in XCD order, so the
// units of neighbouring block rows share an L2.

struct ImgOp16F32 {
    float A[2][16][4];
};

__device__ __forceinline__ void load_img_op16_all(ImgOp16F32 &R, const float *frag32, int wave, int lane)
{
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float4 v = ld4(frag32 + (((2 * wave + t) * 16 + i) * 64 + lane) * 4);
            R.A[t][i][0] = v.x;
            R.A[t][i][1] = v.y;
            R.A[t][i][2] = v.z;
            R.A[t][i][3] = v.w;
        }
}

constexpr int kBlk16Bytes = 256 * 4;

// Resource over the `count` blocks of a tile that starts at block `first` of
// an image and steps `step` blocks (count = 0: an empty resource).  Block b
// of the tile is at byte b * step * 1 KiB; blocks b >= count fall outside.
__device__ __forceinline__ rsrc_t tile16_rsrc(const float *img, int64_t first, int64_t step, int count)
{
    const int bytes = count <= 0 ? 0 : (int)(((int64_t)(count - 1) * step + 1) * kBlk16Bytes);
    const float *p = img + (count <= 0 ? 0 : first * 256);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), (short)0, bytes, kRsrcWord3);
}

// Thread q of the workgroup loads chunk (block q / 64, coefficients
// 4(q % 64) .. +3) and the chunk q + 512 (the layout stage16_store takes).
__device__ __forceinline__ void stage16_load_strided(Stage16<0> &S, rsrc_t r, uint32_t step_bytes, int tid)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = tid + 512 * h;
        S.v[h] = buf_ld4<false>(r, (uint32_t)(q >> 6) * step_bytes + 16 * (q & 63));
    }
}

// One unit: image base block, its tiles (first block and valid count; count
// 0 past the unit's tiles), the block step inside a tile, class pair and
// neighbour offsets.
template <int T>
struct Unit16 {
    int64_t base;
    int64_t blk0[T];
    int cnt[T];
    int64_t step;
    int cp, offsets, nt;
};

template <int T>
__device__ __forceinline__ Unit16<T> decode_unit16(const ImageFilterArgs &a, int64_t unit)
{
    Unit16<T> u;
    const int64_t img = unit / a.units_per_image;
    const int64_t lu = unit % a.units_per_image;
    int ri = 0;
    while (ri + 1 < a.nrect && a.rect[ri + 1].unit_begin <= lu)
        ++ri;
    const ImageRect &rc = a.rect[ri];
    const int64_t t0 = (lu - rc.unit_begin) * T;
    u.nt = (int)min((int64_t)T, rc.tiles - t0);
    u.base = img * a.Bh * a.Bw;
    u.cp = rc.cp;
    u.offsets = rc.offsets;
    u.step = 1;
#pragma unroll
    for (int tt = 0; tt < T; ++tt) {
        const TileRef r = tile_ref(rc, t0 + (tt < u.nt ? tt : 0), a.Bw);
        u.blk0[tt] = r.blk0;
        u.cnt[tt] = tt < u.nt ? r.count : 0;
        u.step = r.step;
    }
    return u;
}

// tiles per unit (N = 16): the unit's accumulators (8 VGPRs per tile) and
// its tiles in flight (8 VGPRs each) share the register file with one
// operator (128-132 VGPRs); 4 tiles spill
constexpr int kImage16T = 3;

template <int PREC, int T>
constexpr int image16_smem()
{
    return 2 * T * (PREC == DCTF_PREC_FP32 ? kTile16BytesF32 : kTile16BytesSplit) + 64 * 4 + 3 * 9 * T * 16 * 4;
}

template <int PREC, int T>
__global__ __launch_bounds__(512) void k_filter_image16(ImageFilterArgs a, int64_t units)
{
    constexpr int kB16 = 16 * kLd16BF16;   // BF16 of one hi (or lo) tile
    constexpr int kTileBytes = PREC == DCTF_PREC_FP32 ? kTile16BytesF32 : kTile16BytesSplit;
    __shared__ __attribute__((aligned(16))) char smem[image16_smem<PREC, T>()];
    // [2][T] tile buffers, then 64 floats of `trash`, then sx0[3][9 T][16]:
    // the DC coefficient of each staged neighbour block, for three units in
    // turn (a unit's DC pass reads its third while the next two units' tiles
    // are staged into the others)
    float *trash = reinterpret_cast<float *>(smem + 2 * T * kTileBytes);
    float *sx0 = trash + 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    typedef typename std::conditional<PREC == DCTF_PREC_FP32, ImgOp16F32, OpRegs16BF16>::type Regs;
    Regs R;
    const int64_t G = gridDim.x;
    // consecutive numbers run on one XCD (G is a multiple of 8)
    int64_t unit = (int64_t)(blockIdx.x % kXcds) * (G / kXcds) + blockIdx.x / kXcds;
    if (unit >= units)
        return;
    const uint32_t out_off = (uint32_t)(4 * (32 * wave + 4 * g));
    auto shift_of = [&](int o) { return (int64_t)(o / 3 - 1) * a.Bw + (o % 3 - 1); };
    auto tile_lds = [&](int b, int tt) { return smem + (b * T + tt) * kTileBytes; };
    // neighbour tile tt of unit u at offset o (live = false: an empty tile)
    auto src = [&](const Unit16<T> &u, int o, int tt, bool live) {
        return tile16_rsrc(a.in + u.base * 256, u.blk0[tt] + shift_of(o), u.step, live ? u.cnt[tt] : 0);
    };
    auto load_tiles = [&](Stage16<0> (&S)[T], const Unit16<T> &u, int o, bool live) {
        const uint32_t sb = (uint32_t)(u.step * kBlk16Bytes);
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
            stage16_load_strided(S[tt], src(u, o, tt, live), sb, tid);
    };
    // tile tt of the stages into tile set b, its DC coefficients into sx0 third par, slot
    auto put_tile = [&](const Stage16<0> &St, int b, int tt, int par, int slot) {
        char *base = tile_lds(b, tt);
        if constexpr (PREC == DCTF_PREC_FP32) {
            stage16_store<0>(St, reinterpret_cast<float *>(base), tid, nullptr, 0.0f);
        } else {
            uint16_t *lhi = reinterpret_cast<uint16_t *>(base);
            stage16_store<0>(St, lhi, lhi + kB16, reinterpret_cast<float *>(lhi + 2 * kB16), trash, tid, nullptr,
                             0.0f);
        }
        // the thread holding coefficients 0..3 of blocks q / 64 and q / 64 + 8
        if ((tid & 63) == 0) {
            float *x0 = sx0 + ((par * 9 * T) + slot) * 16;
            x0[tid >> 6] = St.v[0].x;
            x0[(tid >> 6) + 8] = St.v[1].x;
        }
    };
    auto load_op = [&](int cp, int o) {
        const size_t opi = (size_t)cp * 9 + o;
        if constexpr (PREC == DCTF_PREC_FP32)
            load_img_op16_all(R, a.frag32 + opi * 65536, wave, lane);
        else
            load_op16(R, a.frag_hi + opi * 65536, a.frag_lo + opi * 65536, a.frag_lf + opi * 256 * lf_count(16),
                      wave, lane);
    };
    f32x4 acc[T][2];
    // The MFMA work of one step over tile set b (nt tiles).  Each k-step's
    // operator fragments are reloaded from operator (cp, o) once that k-step
    // is done, and the stages S go into tile set pb (DC coefficients into
    // third ppar from slot pslot) one tile after each of the last T k-steps,
    // so the conversion runs beside the MFMA work.
    auto compute = [&](int b, int nt, int cp, int o, const Stage16<0> (&S)[T], int pb, int ppar, int pslot) {
        const size_t opi = (size_t)cp * 9 + o;
        if constexpr (PREC == DCTF_PREC_FP32) {
            const float *F = a.frag32 + opi * 65536;
#pragma unroll
            for (int i = 15; i >= 0; --i) {
#pragma unroll
                for (int tt = 0; tt < T; ++tt) {
                    if (tt < nt) {
                        const float *lf = reinterpret_cast<const float *>(tile_lds(b, tt));
                        const float4 xv4 = *reinterpret_cast<const float4 *>(lf + f32_chunk(n, 4 * i + g));
                        const float xv[4] = {xv4.x, xv4.y, xv4.z, xv4.w};
#pragma unroll
                        for (int j = 0; j < 4; ++j)
#pragma unroll
                            for (int t = 0; t < 2; ++t)
                                acc[tt][t] = mfma_f32(R.A[t][i][j], xv[j], acc[tt][t]);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const float4 v = ld4(F + (((2 * wave + t) * 16 + i) * 64 + lane) * 4);
                    R.A[t][i][0] = v.x;
                    R.A[t][i][1] = v.y;
                    R.A[t][i][2] = v.z;
                    R.A[t][i][3] = v.w;
                }
                if (i < T)
                    put_tile(S[T - 1 - i], pb, T - 1 - i, ppar, pslot + T - 1 - i);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            const uint16_t *fhi = a.frag_hi + opi * 65536, *flo = a.frag_lo + opi * 65536;
#pragma unroll
            for (int s = 7; s >= 0; --s) {
#pragma unroll
                for (int tt = 0; tt < T; ++tt) {
                    if (tt < nt) {
                        const uint16_t *lhi = reinterpret_cast<const uint16_t *>(tile_lds(b, tt));
                        const u32x4 bh = *reinterpret_cast<const u32x4 *>(lhi + bf16_chunk(n, 4 * s + g));
                        const u32x4 bl = *reinterpret_cast<const u32x4 *>(lhi + kB16 + bf16_chunk(n, 4 * s + g));
#pragma unroll
                        for (int t = 0; t < 2; ++t)
                            acc[tt][t] = mfma_bf16(R.lo[t][s], bh, acc[tt][t]);
#pragma unroll
                        for (int t = 0; t < 2; ++t)
                            acc[tt][t] = mfma_bf16(R.hi[t][s], bl, acc[tt][t]);
#pragma unroll
                        for (int t = 0; t < 2; ++t)
                            acc[tt][t] = mfma_bf16(R.hi[t][s], bh, acc[tt][t]);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int T2 = 2 * wave + t;
                    R.hi[t][s] = ldg_u32x4(fhi + ((T2 * 8 + s) * 64 + lane) * 8);
                    R.lo[t][s] = ldg_u32x4(flo + ((T2 * 8 + s) * 64 + lane) * 8);
                }
                if (s < T)
                    put_tile(S[T - 1 - s], pb, T - 1 - s, ppar, pslot + T - 1 - s);
                __builtin_amdgcn_sched_barrier(0);
            }
            // the low-frequency coefficients in FP32 (the DC columns are zero here)
#pragma unroll
            for (int tt = 0; tt < T; ++tt) {
                if (tt < nt) {
                    const float *llf = reinterpret_cast<const float *>(tile_lds(b, tt) + 2 * kB16 * 2);
                    const float2 lv = *reinterpret_cast<const float2 *>(llf + (g * 16 + n) * 2);
                    const float lfv[2] = {lv.x, lv.y};
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int t = 0; t < 2; ++t)
                            acc[tt][t] = mfma_f32(R.lf[t][j], lfv[j], acc[tt][t]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            const float *flf = a.frag_lf + opi * 256 * lf_count(16);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const f32x2 v = ldg_f32x2(flf + ((2 * wave + t) * 64 + lane) * 2);
                R.lf[t][0] = v[0];
                R.lf[t][1] = v[1];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    Unit16<T> cu = decode_unit16<T>(a, unit);
    int par = 0;   // sx0 third of the current unit
    int b = 0;     // tile set of the current step
    Stage16<0> S[T];
    {
        const int o = __builtin_ctz((unsigned)cu.offsets);   // the centre is always present
        load_tiles(S, cu, o, true);
        load_op(cu.cp, o);
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
            put_tile(S[tt], 0, tt, 0, tt);
        // nothing in flight at the loop's entry: its waits then count only the
        // loads the loop itself issues (the operator reloads of the step before)
        wait_vm_all();
        __syncthreads();
    }
    for (;;) {
        const int64_t nunit = unit + G;
        const bool more = nunit < units;
        const Unit16<T> nu = more ? decode_unit16<T>(a, nunit) : cu;
        const int nfirst = __builtin_ctz((unsigned)nu.offsets);
        const int npar = par == 2 ? 0 : par + 1;
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            acc[tt][0] = f32x4{0.f, 0.f, 0.f, 0.f};
            acc[tt][1] = acc[tt][0];
        }
        unsigned rem = (unsigned)cu.offsets;
        int o = __builtin_ctz(rem);
        rem &= rem - 1;
        // every step but the unit's last: the next offset's tiles into the other set
        for (int oi = 0; rem != 0; ++oi) {
            const int on = __builtin_ctz(rem);
            rem &= rem - 1;
            load_tiles(S, cu, on, true);
            compute(b, cu.nt, cu.cp, on, S, b ^ 1, par, (oi + 1) * T);
            __syncthreads();
            b ^= 1;
            o = on;
        }
        // the unit's last step: the next unit's first tiles and operator (or,
        // past the last unit, empty tiles and this operator again)
        load_tiles(S, nu, more ? nfirst : o, more);
        compute(b, cu.nt, more ? nu.cp : cu.cp, more ? nfirst : o, S, b ^ 1, npar, 0);
        __syncthreads();
        // the operators' DC columns, in offset order
        {
            unsigned r2 = (unsigned)cu.offsets;
            int i = 0;
            while (r2) {
                const int od = __builtin_ctz(r2);
                r2 &= r2 - 1;
                const float *D0 = a.h0 + ((size_t)cu.cp * 9 + od) * 256 + 32 * wave + 4 * g;
                const float4 h0[2] = {ld4(D0), ld4(D0 + 16)};
#pragma unroll
                for (int tt = 0; tt < T; ++tt) {
                    const float x0 = sx0[((par * 9 * T) + i * T + tt) * 16 + n];
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        acc[tt][t][0] = fmaf(h0[t].x, x0, acc[tt][t][0]);
                        acc[tt][t][1] = fmaf(h0[t].y, x0, acc[tt][t][1]);
                        acc[tt][t][2] = fmaf(h0[t].z, x0, acc[tt][t][2]);
                        acc[tt][t][3] = fmaf(h0[t].w, x0, acc[tt][t][3]);
                    }
                }
                ++i;
            }
        }
        {
            float *Y = a.out + cu.base * 256;
            const uint32_t sb = (uint32_t)(cu.step * kBlk16Bytes);
#pragma unroll
            for (int tt = 0; tt < T; ++tt) {
                const rsrc_t out = tile16_rsrc(Y, cu.blk0[tt], cu.step, cu.cnt[tt]);
                buf_st4<false>(out, (uint32_t)n * sb + out_off, acc[tt][0]);
                buf_st4<false>(out, (uint32_t)n * sb + out_off + 64, acc[tt][1]);
            }
        }
        if (!more)
            break;
        b ^= 1;
        par = npar;
        unit = nunit;
        cu = nu;
    }
}

}  // namespace

hipError_t launch_build_image(int N, const ImageBuildArgs &args, hipStream_t stream)
{
    if (N == 8)
        hipLaunchKernelGGL((k_build_image<8, 17>), dim3(64 / 16, 16, 9), dim3(kThreads), 0, stream, args);
    else
        hipLaunchKernelGGL((k_build_image<16, 8>), dim3(256 / 16, 16, 9), dim3(kThreads), 0, stream, args);
    return hipGetLastError();
}

int image_tiles_per_unit(int N, int prec)
{
    if (N == 16)
        return kImage16T;
    return prec == DCTF_PREC_FP32 ? kImageT32 : kImageTSplit;
}

hipError_t launch_filter_image(int N, int prec, const ImageFilterArgs &a, hipStream_t stream)
{
    const int64_t units = a.units_per_image * a.nimg;
    if (units <= 0)
        return hipSuccess;
    if (N == 16) {
        // one 8-wave workgroup per CU (the operator takes most of the registers)
        const int64_t groups = xcd_groups(units < cu_count() ? units : cu_count(), 1);
        if (prec == DCTF_PREC_FP32)
            hipLaunchKernelGGL((k_filter_image16<DCTF_PREC_FP32, kImage16T>), dim3((unsigned)groups), dim3(512), 0,
                               stream, a, units);
        else
            hipLaunchKernelGGL((k_filter_image16<DCTF_PREC_SPLIT_BF16, kImage16T>), dim3((unsigned)groups),
                               dim3(512), 0, stream, a, units);
        return hipGetLastError();
    }
    int64_t waves = (int64_t)cu_count() * kImageWavesPerCu;
    waves = waves < units ? waves : units;
    if (prec == DCTF_PREC_FP32) {
        const int64_t groups = xcd_groups(waves, 4);
        waves = groups * 4;   // waves past the last unit find no work
        hipLaunchKernelGGL((k_filter_image8<DCTF_PREC_FP32, kImageT32, false>), dim3((unsigned)groups), dim3(256), 0,
                           stream, a, units, waves, -1);
    } else {
        // the class pair with the most tiles keeps its neighbour operators in LDS
        int lds_cp = -1;
        int64_t best = 0;
        for (int r = 0; r < a.nrect; ++r)
            if (a.rect[r].tiles > best) {
                best = a.rect[r].tiles;
                lds_cp = a.rect[r].cp;
            }
        const int64_t groups = xcd_groups(waves, 8);
        waves = groups * 8;
        hipLaunchKernelGGL((k_filter_image8<DCTF_PREC_SPLIT_BF16, kImageTSplit, true>), dim3((unsigned)groups),
                           dim3(512), 0, stream, a, units, waves, lds_cp);
    }
    return hipGetLastError();
}

}  // namespace dctf
