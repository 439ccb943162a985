// Filter + inverse DCT + uint8 in one pass: P[b] = u8(G . X[b]), where
// G = (C (x) C)^t H_dct is the pixel-domain operator the builder forms in
// FP64 next to H_dct (the DCT-domain filter of eq. 11 / eq. 20 followed by
// the inverse DCT of eq. 3, then the uint8 conversion of Sec. III).  The
// filtered coefficients never reach HBM: 4 bytes in and 1 byte out per
// coefficient instead of 4 + 4 for the filter and 4 + 1 for a separate
// inverse transform.
//
// Outputs: the pixels block by block (N*N bytes per block), or in their
// places in one h x w raster image (row pitch in bytes).
//
// Inputs: FP32 coefficient blocks (IN = 0), or quantised int16 coefficient
// blocks (IN = 1, the entropy-decoded blocks of a JPEG-style codec) that are
// dequantised in registers, X[k] = q[k] c[k] (+ dc_offset on the DC term):
// 2 bytes in and 1 byte out per coefficient.
//
//   N = 8  : k_filter_px8  — one wave per 16-block tile, G in VGPRs (the
//            layout of the DCT-domain kernel), tiles staged through a
//            wave-private LDS region so that every global access of the
//            wave covers contiguous memory.
//   N = 16 : k_filter_px16 — the weight-stationary 8-wave tile loop of the
//            DCT-domain kernel with the int16 loader / uint8 store.
//   N <= 4 : k_filter_px_small — one thread per block, FP32 VALU.
#include "mfma_common.h"

namespace dctf {
namespace {

// ---------------------------------------------------------------- N = 8
//
// Loads (LI): 1 = coalesced through the wave's LDS region (every load
// instruction covers contiguous memory, the tile is then re-read in MFMA
// layout); 0 = straight into the MFMA layout (lane (n, g) loads coefficients
// 16i + 4g .. +3 of block n).  Stores (SO): 1 = through LDS, one 16-byte
// store per lane covering the tile's 1 KiB; 0 = straight from the MFMA
// result layout (lane (n, g) stores pixels 16t + 4g .. +3 of block n, four
// bytes).  U tiles per iteration; the next iteration's loads are in flight
// while the current one is multiplied.

// Tile input held in registers while the previous tile is multiplied.
template <int IN, int LI>
struct In8;

template <int LI>
struct In8<0, LI> {
    float4 x[4];   // LI = 1: the layout of load_tile_coalesced; LI = 0: MFMA layout
};

template <>
struct In8<1, 1> {
    u32x4 raw[2];  // 2 KiB tile: lane l, load i holds coefficients 8(l % 8) .. +7 of block 8i + l / 8
};

template <>
struct In8<1, 0> {
    uint2 raw[4];  // lane (n, g), load i: coefficients 16i + 4g .. +3 of block n
};

template <int LI>
__device__ __forceinline__ void load8(In8<0, LI> &t, const PxArgs &a, int64_t blk0, int lane)
{
    const int64_t nv = a.B - blk0;
    if constexpr (LI == 1) {
        load_tile_coalesced<true>(t.x, a.in + blk0 * 64, nv, lane);
    } else {
        const int64_t n = lane & 15;
        const float *src = a.in + (blk0 + (n < nv ? n : nv - 1)) * 64 + 4 * (lane >> 4);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            t.x[i] = ld4_nt(src + 16 * i);
    }
}

__device__ __forceinline__ void load8(In8<1, 1> &t, const PxArgs &a, int64_t blk0, int lane)
{
    const int64_t nv = a.B - blk0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int64_t b = 8 * i + (lane >> 3);
        const int64_t bb = b < nv ? b : nv - 1;   // clamped: its pixels are never stored
        t.raw[i] = __builtin_nontemporal_load(
            reinterpret_cast<const u32x4 *>(a.qin + (blk0 + bb) * 64 + 8 * (lane & 7)));
    }
}

__device__ __forceinline__ void load8(In8<1, 0> &t, const PxArgs &a, int64_t blk0, int lane)
{
    const int64_t nv = a.B - blk0;
    const int64_t n = lane & 15;
    const int16_t *src = a.qin + (blk0 + (n < nv ? n : nv - 1)) * 64 + 4 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        t.raw[i] = *reinterpret_cast<const uint2 *>(src + 16 * i);
}

// The tile in MFMA layout (xm), through the wave's LDS region where the
// loads were coalesced (chunk c of block b at slot 16 b + (c ^ b)).
// q: the dequantisation factors this lane needs (IN = 1), dc the DC offset.
template <int LI>
__device__ __forceinline__ void to_mfma8(const In8<0, LI> &t, float4 *lds, int lane, const float *, float,
                                         float4 xm[4])
{
    if constexpr (LI == 1) {
        stage_in(lds, t.x, lane);
        wave_lds_sync();
        read_mfma(lds, xm, lane);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            xm[i] = t.x[i];
    }
}

// LI = 1: q[e] is the factor of coefficient 8(lane % 8) + e.
__device__ __forceinline__ void to_mfma8(const In8<1, 1> &t, float4 *lds, int lane, const float *q, float dc,
                                         float4 xm[4])
{
    const int c8 = lane & 7;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int b = 8 * i + (lane >> 3);
        float4 lo, hi;
        dequant8(t.raw[i], q, dc, lo, hi);
        lds[b * 16 + ((2 * c8) ^ b)] = lo;
        lds[b * 16 + ((2 * c8 + 1) ^ b)] = hi;
    }
    wave_lds_sync();
    read_mfma(lds, xm, lane);
}

// LI = 0: q[4i + j] is the factor of coefficient 16i + 4(lane / 16) + j.
__device__ __forceinline__ void to_mfma8(const In8<1, 0> &t, float4 *, int, const float *q, float dc,
                                         float4 xm[4])
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint2 r = t.raw[i];
        xm[i] = make_float4((float)(int16_t)(r.x & 0xffffu) * q[4 * i],
                            (float)((int32_t)r.x >> 16) * q[4 * i + 1],
                            (float)(int16_t)(r.y & 0xffffu) * q[4 * i + 2],
                            (float)((int32_t)r.y >> 16) * q[4 * i + 3]);
    }
    xm[0].x += dc;
}

// SO = 1: lane l writes the 16 pixels 16(l % 4) .. +15 of block l / 4 from
// the LDS staging (floats, swizzled), one 16-byte store per lane.
__device__ __forceinline__ void store_px8_lds(uint8_t *pix, int64_t nvalid, const float4 *lds, int lane)
{
    const int b = lane >> 2, k4 = lane & 3;
    if (b >= nvalid)
        return;
    u32x4 w;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const float4 v = lds[b * 16 + ((4 * k4 + m) ^ b)];
        w[m] = pack_u8x4(v.x, v.y, v.z, v.w);
    }
    __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(pix + (int64_t)b * 64 + 16 * k4));
}

// SO = 0: lane (n, g) holds pixels 16t + 4g + r of block n.
__device__ __forceinline__ void store_px8_direct(uint8_t *pix, int64_t nvalid, const f32x4 acc[4], int lane)
{
    const int n = lane & 15, g = lane >> 4;
    if (n >= nvalid)
        return;
    uint32_t *dst = reinterpret_cast<uint32_t *>(pix + (int64_t)n * 64 + 4 * g);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        dst[4 * t] = pack_u8x4(acc[t][0], acc[t][1], acc[t][2], acc[t][3]);
}

// SO = 0 into a raster image: lane (n, g) holds pixels 4(g % 2) .. +3 of
// rows 2t + g / 2 of block n.
__device__ __forceinline__ void store_px8_raster(const PxArgs &a, int64_t blk0, int64_t nvalid, const f32x4 acc[4],
                                                 int lane)
{
    const int n = lane & 15, g = lane >> 4;
    if (n >= nvalid)
        return;
    int64_t img;
    int by, bx;
    raster_place((uint32_t)(blk0 + n), a.bpi, a.Bw, a.magic, img, by, bx);
    uint8_t *base = a.pix + img * a.img_stride;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        store_px_raster4(base, a.pitch, a.h, a.w, 8 * by + 2 * t + (g >> 1), 8 * bx + 4 * (g & 1),
                         pack_u8x4(acc[t][0], acc[t][1], acc[t][2], acc[t][3]));
}

// Wave w takes units (U tiles of 16 blocks) w, w + waves, ...
// RAST: pixels into the raster image (SO = 0 only).
template <int PREC, int IN, int U, int LI, int SO, bool RAST = false>
__global__ __launch_bounds__(256) void k_filter_px8(PxArgs a, int64_t units, int64_t waves)
{
    constexpr bool kLds = LI == 1 || SO == 1;
    __shared__ __attribute__((aligned(16))) float4 lds_all[kLds ? 4 * U * 256 : 1];
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= waves)   // waves <= units
        return;
    float4 *lds = lds_all + (kLds ? (threadIdx.x >> 6) * U * 256 : 0);

    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs8F32, OpRegs8BF16>::type Regs;
    Regs R;
    if constexpr (PREC == DCTF_PREC_FP32)
        load_op8(R, a.G.frag32, a.G.h0, lane);
    else
        load_op8(R, a.G.frag_hi, a.G.frag_lo, a.G.frag_lf, lane);

    constexpr int kQ = IN == 0 ? 1 : (LI == 1 ? 8 : 16);
    float q[kQ];
    float dc = 0.0f;
    if constexpr (IN == 1) {
        if constexpr (LI == 1) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                q[e] = a.qtab[8 * (lane & 7) + e];
            dc = (lane & 7) == 0 ? a.dc_offset : 0.0f;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    q[4 * i + j] = a.qtab[16 * i + 4 * (lane >> 4) + j];
            dc = (lane >> 4) == 0 ? a.dc_offset : 0.0f;
        }
    }

    const int64_t B = a.B;
    const int64_t my_units = (units - wave + waves - 1) / waves;
    auto load_unit = [&](In8<IN, LI> (&t)[U], int64_t unit) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t blk0 = unit * (16 * U) + 16 * u;
            load8(t[u], a, blk0 < B ? blk0 : B - 1, lane);   // an empty tail tile re-reads the last block
        }
    };
    auto compute_store = [&](const In8<IN, LI> (&t)[U], int64_t unit) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t blk0 = unit * (16 * U) + 16 * u;
            if (blk0 >= B)
                break;
            float4 *L = lds + (kLds ? u * 256 : 0);
            float4 xm[4];
            to_mfma8(t[u], L, lane, q, dc, xm);
            f32x4 acc[4];
            tile8(R, xm, lane, acc);
            static_assert(!RAST || SO == 0, "raster stores go straight from the MFMA layout");
            if constexpr (RAST) {
                store_px8_raster(a, blk0, B - blk0, acc, lane);
            } else if constexpr (SO == 1) {
                wave_lds_sync();
                stage_out(L, acc, lane);
                wave_lds_sync();
                store_px8_lds(a.pix + blk0 * 64, B - blk0, L, lane);
            } else {
                store_px8_direct(a.pix + blk0 * 64, B - blk0, acc, lane);
            }
            if constexpr (kLds)
                wave_lds_sync();
        }
    };

    In8<IN, LI> cur[U], nxt[U];
    int64_t unit = wave;
    load_unit(cur, unit);
    for (int64_t k = 1; k < my_units; ++k) {
        load_unit(nxt, unit + waves);
        compute_store(cur, unit);
#pragma unroll
        for (int u = 0; u < U; ++u)
            cur[u] = nxt[u];
        unit += waves;
    }
    compute_store(cur, unit);
}

// ------------------------------------------ N = 8, uint8 raster in and out
//
// One pass from uint8 images to filtered uint8 images: the operator is the
// pixel-to-pixel set (the forward DCT, the filter and the inverse DCT in one
// 64 x 64 matrix), held in VGPRs as in the kernels above.  Lane (n, g) of a
// 16-block tile reads pixels 16i + 4g .. +3 of block n (row 2i + g / 2,
// columns 4(g % 2) .. +3: one 32-bit load, bytes at the right edge, rows and
// columns past the image repeat the last one, as the forward DCT extends
// them), converts them to FP32 (exact), and the result goes to the output
// image with the raster stores.  Split path: the pixels are exact in BF16,
// so Y = G_hi x + G_mid x + G_lo x carries the operator's 24 bits.

struct OpRegs8PP {
    u32x4 hi[4][2];
    u32x4 mid[4][2];
    u32x4 lo[4][2];
};

__device__ __forceinline__ void load_op8_pp(OpRegs8PP &R, const DenseImages &D, int lane)
{
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int o = ((t * 2 + s) * 64 + lane) * 8;
            R.hi[t][s] = ldg_u32x4(D.frag_hi + o);
            R.mid[t][s] = ldg_u32x4(D.frag_lo + o);
            R.lo[t][s] = ldg_u32x4(D.frag_lo2 + o);
        }
}

// acc = init + G . x, three BF16 terms per k-step, the smallest first.
__device__ __forceinline__ void tile8_pp(const OpRegs8PP &R, const float4 x[4], f32x4 acc[4], float init)
{
    u32x4 b[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        uint32_t h0, h1, h2, h3, l0, l1, l2, l3;   // the lo halves are zero (exact pixels)
        split_bf16(x[2 * s], h0, h1, l0, l1);
        split_bf16(x[2 * s + 1], h2, h3, l2, l3);
        b[s] = u32x4{h0, h1, h2, h3};
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
        acc[t] = f32x4{init, init, init, init};
#pragma unroll
    for (int s = 1; s >= 0; --s) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = mfma_bf16(R.lo[t][s], b[s], acc[t]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = mfma_bf16(R.mid[t][s], b[s], acc[t]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = mfma_bf16(R.hi[t][s], b[s], acc[t]);
    }
}

// acc = init + G . x, FP32 path (the operator's first column in VALU
// arithmetic last, as in tile8).
__device__ __forceinline__ void tile8_f32_init(const OpRegs8F32 &R, const float4 x[4], int lane, f32x4 acc[4],
                                               float init)
{
    const int n = lane & 15;
    const float x0 = lane_read(x[0].x, n);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        acc[t] = f32x4{init, init, init, init};
#pragma unroll
    for (int i = 3; i >= 0; --i) {
        const float xv[4] = {x[i].x, x[i].y, x[i].z, x[i].w};
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t] = mfma_f32(R.A[t][i][j], xv[j], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            acc[t][r] = fmaf(R.h0[t][r], x0, acc[t][r]);
}

// Four pixels already biased by +1/2 (the accumulators start at 1/2) -> one
// little-endian word: floor, then V_CVT_PK_U8_F32 as in pack_u8x4.
__device__ __forceinline__ uint32_t pack_u8x4_biased(f32x4 v)
{
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w = __builtin_amdgcn_cvt_pk_u8_f32(floorf(v[k]), k, w);
    return w;
}

struct RasterIn {
    const uint8_t *img;
    int64_t pitch, img_stride;
    // BUF: bytes from img (resp. the output's first pixel) to the end of the
    // last input (output) image, rounded up to a multiple of 4; both < 2^31
    int64_t in_bytes, out_bytes;
};

// The lane's block: image, block row, block column (block blk0 + n, or the
// last block of the tile's valid ones).
struct U8rPlace {
    int64_t img;
    int by, bx;
};

__device__ __forceinline__ U8rPlace u8r_place(const PxArgs &a, int64_t blk0, int lane)
{
    const int n = lane & 15;
    const int64_t nv = a.B - blk0;
    U8rPlace p;
    raster_place((uint32_t)(blk0 + (n < nv ? n : nv - 1)), a.bpi, a.Bw, a.magic, p.img, p.by, p.bx);
    return p;
}

// Byte selector for the columns of a ragged image: the aligned word at
// xa = min(x0, (w - 1) & ~3) holds pixels min(x0 + e, w - 1), e = 0..3
// (an aligned word that holds a pixel of the image lies in the page of that
// pixel; the bytes past w it may cover are not used).
__device__ __forceinline__ uint32_t edge_select(int x0, int w, int &xa)
{
    xa = min(x0, (w - 1) & ~3);
    const int d = min(x0 - xa, 3), m = min(w - 1 - xa, 3);
    return (uint32_t)min(d, m) | (uint32_t)min(d + 1, m) << 8 | (uint32_t)min(d + 2, m) << 16 |
           (uint32_t)min(d + 3, m) << 24;
}

// Lane (n, g) of a 16-block tile holds pixels 16i + 4g .. +3 of block n: row
// 2i + g/2, columns 4(g % 2) .. +3 of the block, one 32-bit word per i; its
// outputs t = 0..3 are the same pixels of row 2t + g/2.  ALIGNED (h and w
// multiples of 8): every pixel of every block is in its image.  Otherwise
// rows past the image repeat the last one and columns past it the last
// column (the forward DCT's extension), and only pixels inside the image
// are stored.
//
// BUF (the images within 2^31 bytes): raw buffer instructions over the input
// and the output, 32-bit offsets, the rows of a block 2 pitch apart through
// the instruction's scalar offset; ragged stores go out as a word, a short
// and a byte whose offsets point past the buffer where they have nothing to
// store (dropped), so that no store is conditional.
template <bool ALIGNED, bool BUF>
struct U8rIO {
    rsrc_t rin, rout;
    int32_t srow_in[4], srow_out[4];   // 2 i pitch (uniform)

    __device__ __forceinline__ void init(const PxArgs &a, const RasterIn &in)
    {
        if constexpr (BUF) {
            rin = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(in.img), (short)0, (int)in.in_bytes,
                                                    kRsrcWord3);
            rout = __builtin_amdgcn_make_buffer_rsrc(a.pix, (short)0, (int)in.out_bytes, kRsrcWord3);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                srow_in[i] = (int32_t)(2 * i * in.pitch);
                srow_out[i] = (int32_t)(2 * i * a.pitch);
            }
        }
    }

    // loads the lane's 16 pixels of the tile at blk0; returns what the
    // later steps of the same tile need: ALIGNED && BUF: the output offset
    // of the lane's row 0 pixels; ragged: the byte selector, applied to the
    // words when they are used (not here, where that would wait for them)
    __device__ __forceinline__ uint32_t load(const PxArgs &a, const RasterIn &in, int64_t blk0, int lane,
                                             uint32_t w4[4]) const
    {
        const int g = lane >> 4;
        const U8rPlace p = u8r_place(a, blk0, lane);
        const int x0 = 8 * p.bx + 4 * (g & 1), y0 = 8 * p.by + (g >> 1);
        if constexpr (ALIGNED && BUF) {
            const uint32_t off = (uint32_t)p.img * (uint32_t)in.img_stride + (uint32_t)y0 * (uint32_t)in.pitch + x0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                w4[i] = __builtin_amdgcn_raw_buffer_load_b32(rin, off, srow_in[i], 0);
            return (uint32_t)p.img * (uint32_t)a.img_stride + (uint32_t)y0 * (uint32_t)a.pitch + x0;
        } else if constexpr (ALIGNED) {
            const uint8_t *base = in.img + p.img * in.img_stride + (int64_t)y0 * in.pitch + x0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                w4[i] = *reinterpret_cast<const uint32_t *>(base + 2 * i * in.pitch);
            return 0;
        } else {
            int xa;
            const uint32_t sel = edge_select(x0, a.w, xa);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = min(y0 + 2 * i, a.h - 1);
                if constexpr (BUF)
                    w4[i] = __builtin_amdgcn_raw_buffer_load_b32(
                        rin, (uint32_t)p.img * (uint32_t)in.img_stride + (uint32_t)y * (uint32_t)in.pitch + xa, 0, 0);
                else
                    w4[i] = *reinterpret_cast<const uint32_t *>(in.img + p.img * in.img_stride +
                                                                (int64_t)y * in.pitch + xa);
            }
            return sel;
        }
    }

    // the tile's pixels as FP32 (exact), from the words and what load returned
    __device__ __forceinline__ void unpack(const uint32_t w4[4], uint32_t aux, float4 x[4]) const
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t w = ALIGNED ? w4[i] : __builtin_amdgcn_perm(w4[i], w4[i], aux);
            x[i] = make_float4((float)(w & 0xffu), (float)((w >> 8) & 0xffu), (float)((w >> 16) & 0xffu),
                               (float)(w >> 24));
        }
    }

    // stores the tile's pixels (acc biased by +1/2); lanes past the tile's
    // last valid block hold that block's pixels and store them again
    __device__ __forceinline__ void store(const PxArgs &a, int64_t blk0, int lane, uint32_t out_off,
                                          const f32x4 acc[4]) const
    {
        if constexpr (ALIGNED && BUF) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                __builtin_amdgcn_raw_buffer_store_b32(pack_u8x4_biased(acc[t]), rout, out_off, srow_out[t], 0);
            return;
        }
        const int g = lane >> 4;
        const U8rPlace p = u8r_place(a, blk0, lane);
        const int x0 = 8 * p.bx + 4 * (g & 1), y0 = 8 * p.by + (g >> 1);
        if constexpr (ALIGNED) {
            uint8_t *base = a.pix + p.img * a.img_stride + (int64_t)y0 * a.pitch + x0;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                *reinterpret_cast<uint32_t *>(base + 2 * t * a.pitch) = pack_u8x4_biased(acc[t]);
        } else if constexpr (BUF) {
            constexpr uint32_t kPast = 0x80000000u;   // >= out_bytes: dropped
            const int c = min(max(a.w - x0, 0), 4);    // pixels of the word inside the image
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t word = pack_u8x4_biased(acc[t]);
                const bool row = y0 + 2 * t < a.h;
                const uint32_t off =
                    (uint32_t)p.img * (uint32_t)a.img_stride + (uint32_t)(y0 + 2 * t) * (uint32_t)a.pitch + x0;
                __builtin_amdgcn_raw_buffer_store_b32(word, rout, row && c == 4 ? off : kPast, 0, 0);
                __builtin_amdgcn_raw_buffer_store_b16((uint16_t)word, rout, row && (c == 2 || c == 3) ? off : kPast,
                                                      0, 0);
                // c = 1: byte 0 at off; c = 3: byte 2 at off + 2
                const uint32_t b = (uint32_t)(c & 2);
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(word >> (8 * b)), rout,
                                                     row && (c & 1) ? off + b : kPast, 0, 0);
            }
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                store_px_raster4(a.pix + p.img * a.img_stride, a.pitch, a.h, a.w, y0 + 2 * t, x0,
                                 pack_u8x4_biased(acc[t]));
        }
    }
};

// Wave w takes tiles w, w + waves, ...; the pixels of the next D tiles are in
// flight while the current one is multiplied (a ring of D register slots,
// the loop unrolled D times so that every slot is a fixed register set).
// The wave's step count is rounded up to a multiple of D: the extra steps
// filter its last tile again and store the same bytes, so the loop has no
// exit but its end and every step issues the same loads and stores (the
// waits for a slot then count exactly the operations issued after it).
template <int PREC, bool ALIGNED, bool BUF, int D>
__global__ __launch_bounds__(256, 2) void k_filter_u8r8(PxArgs a, RasterIn in, int64_t tiles, int64_t waves)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = uniform_i64((int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    if (wave >= waves)   // waves <= tiles
        return;
    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs8F32, OpRegs8PP>::type Regs;
    Regs R;
    if constexpr (PREC == DCTF_PREC_FP32)
        load_op8(R, a.G.frag32, a.G.h0, lane);
    else
        load_op8_pp(R, a.G, lane);
    U8rIO<ALIGNED, BUF> io;
    io.init(a, in);
    const int64_t my_tiles = (tiles - wave + waves - 1) / waves;
    const int64_t last = wave + (my_tiles - 1) * waves;
    uint32_t ring[D][4], ring_aux[D];
    int64_t tile = wave;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int64_t t = tile + j * waves;
        ring_aux[j] = io.load(a, in, (t < last ? t : last) * 16, lane, ring[j]);
    }
    auto round = [&]() {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int64_t cur = tile < last ? tile : last;
            float4 x[4];
            io.unpack(ring[j], ring_aux[j], x);
            const uint32_t out_off = ring_aux[j];
            const int64_t t = tile + D * waves;
            ring_aux[j] = io.load(a, in, (t < last ? t : last) * 16, lane, ring[j]);
            // keep the slot's next loads ahead of this tile's products
            __builtin_amdgcn_sched_barrier(0);
            f32x4 acc[4];
            if constexpr (PREC == DCTF_PREC_FP32)
                tile8_f32_init(R, x, lane, acc, 0.5f);
            else
                tile8_pp(R, x, acc, 0.5f);
            io.store(a, cur * 16, lane, out_off, acc);
            __builtin_amdgcn_sched_barrier(0);
            tile += waves;
        }
    };
    // the first round outside the loop: the loop is then entered with the
    // same operations in flight as at its back-edge
    round();
    for (int64_t k = D; k < my_tiles; k += D)
        round();
}

// ---------------------------------------------------------------- N = 16

struct RefPx16 {
    const float *in;
    const int16_t *qin;
    uint8_t *pix;
    int64_t B;
    int64_t blk0;
    int op;
    int h, w, Bw, bpi;   // raster output
    int64_t pitch, img_stride;
    uint32_t magic[4];
};

template <int PREC, int IN, int D, bool RAST = false>
__global__ __launch_bounds__(512) void k_filter_px16(PxArgs a, int64_t tiles)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t wg = blockIdx.x, G = gridDim.x;
    if (wg >= tiles)
        return;
    __shared__ __attribute__((aligned(16))) char smem[PREC == DCTF_PREC_FP32 ? kSmem16F32 : kSmem16Split];
    typedef typename std::conditional<PREC == DCTF_PREC_FP32, OpRegs16F32, OpRegs16BF16>::type Regs;
    Regs R;
    const int64_t count = (tiles - wg + G - 1) / G;
    auto ref = [&](int64_t t) {
        RefPx16 r;
        r.in = a.in;
        r.qin = a.qin;
        r.pix = a.pix;
        r.B = a.B;
        r.blk0 = (wg + t * G) * 16;
        r.op = 0;
        r.h = a.h;
        r.w = a.w;
        r.Bw = a.Bw;
        r.bpi = a.bpi;
        r.pitch = a.pitch;
        r.img_stride = a.img_stride;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            r.magic[i] = a.magic[i];
        return r;
    };
    auto op_load = [&](int) {
        if constexpr (PREC == DCTF_PREC_FP32)
            load_op16(R, a.G.frag32, a.G.h0, wave, lane);
        else
            load_op16(R, a.G.frag_hi, a.G.frag_lo, a.G.frag_lf, wave, lane);
    };
    run_tiles16<PREC, D, RefPx16, IN, RAST ? 2 : 1>(count, ref, op_load, R, smem, a.qtab, a.dc_offset);
}

// ---------------------------------------------------------------- N <= 4

template <int IN>
__global__ __launch_bounds__(256) void k_filter_px_small(PxArgs a, int N)
{
    // (raster output: pixel r of block blk goes to its place in the image)
    __shared__ float sG[256];
    const int NN = N * N;
    for (int e = threadIdx.x; e < NN * NN; e += blockDim.x)
        sG[e] = a.G.H32[e];
    __syncthreads();
    const int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blk >= a.B)
        return;
    float x[16];
    for (int k = 0; k < NN; ++k) {
        if constexpr (IN == 0)
            x[k] = a.in[blk * NN + k];
        else
            x[k] = (float)a.qin[blk * NN + k] * a.qtab[k] + (k == 0 ? a.dc_offset : 0.0f);
    }
    // (per thread: blk differs between the lanes of a wave)
    int64_t img = 0;
    int by = 0, bx = 0;
    if (a.raster)
        raster_place((uint32_t)blk, a.bpi, a.Bw, a.magic, img, by, bx);
    for (int r = 0; r < NN; ++r) {
        float s = 0.0f;
        for (int k = 0; k < NN; ++k)
            s = fmaf(sG[r * NN + k], x[k], s);
        if (!a.raster) {
            a.pix[blk * NN + r] = (uint8_t)pixel_u8(s);
        } else {
            const int y = by * N + r / N, xx = bx * N + r % N;
            if (y < a.h && xx < a.w)
                a.pix[img * a.img_stride + (int64_t)y * a.pitch + xx] = (uint8_t)pixel_u8(s);
        }
    }
}

// ------------------------------------------------------------- launches

// N = 8 launch shape: tiles per iteration, load / store paths, waves per CU.
constexpr int kPx8U = 2;
constexpr int kPx8Li = 1;
constexpr int kPx8So = 0;
constexpr int kPx8WavesPerCu = 8;
// one-pass uint8 kernel: waves per CU (two per SIMD; three measured no
// faster) and tiles of pixels in flight per wave (2, 3 and 4 measured 0.126,
// 0.138 and 0.134 ms on 64 2048^2 images, split-BF16)
constexpr int kU8rWavesPerCu = 8;
constexpr int kU8rDepth = 2;
constexpr int kPx16Depth = 2;

template <int PREC, int IN>
hipError_t run_px8(const PxArgs &a, hipStream_t stream)
{
    const int64_t units = (a.B + 16 * kPx8U - 1) / (16 * kPx8U);
    int64_t waves = (int64_t)cu_count() * kPx8WavesPerCu;
    waves = waves < units ? waves : units;
    const int64_t groups = (waves + 3) / 4;
    if (a.raster)
        hipLaunchKernelGGL((k_filter_px8<PREC, IN, kPx8U, kPx8Li, 0, true>), dim3((unsigned)groups), dim3(256), 0,
                           stream, a, units, waves);
    else
        hipLaunchKernelGGL((k_filter_px8<PREC, IN, kPx8U, kPx8Li, kPx8So>), dim3((unsigned)groups), dim3(256), 0,
                           stream, a, units, waves);
    return hipGetLastError();
}

template <int PREC, int IN>
hipError_t run_px16(const PxArgs &a, hipStream_t stream)
{
    const int64_t tiles = (a.B + 15) / 16;
    int64_t groups = (int64_t)cu_count();
    groups = groups < tiles ? groups : tiles;
    if (a.raster)
        hipLaunchKernelGGL((k_filter_px16<PREC, IN, kPx16Depth, true>), dim3((unsigned)groups), dim3(512), 0,
                           stream, a, tiles);
    else
        hipLaunchKernelGGL((k_filter_px16<PREC, IN, kPx16Depth>), dim3((unsigned)groups), dim3(512), 0, stream, a,
                           tiles);
    return hipGetLastError();
}

template <int PREC>
hipError_t dispatch_px(int N, int in_kind, const PxArgs &a, hipStream_t stream)
{
    if (N == 8)
        return in_kind ? run_px8<PREC, 1>(a, stream) : run_px8<PREC, 0>(a, stream);
    return in_kind ? run_px16<PREC, 1>(a, stream) : run_px16<PREC, 0>(a, stream);
}

}  // namespace

hipError_t launch_filter_u8_raster8(int prec, const PxArgs &a, const uint8_t *in_img, int64_t in_pitch,
                                   int64_t in_stride, hipStream_t stream)
{
    if (a.B <= 0)
        return hipSuccess;
    RasterIn in;
    in.img = in_img;
    in.pitch = in_pitch;
    in.img_stride = in_stride;
    const int64_t nimg = a.B / a.bpi;
    in.in_bytes = ((nimg - 1) * in_stride + (int64_t)(a.h - 1) * in_pitch + a.w + 3) / 4 * 4;
    in.out_bytes = ((nimg - 1) * a.img_stride + (int64_t)(a.h - 1) * a.pitch + a.w + 3) / 4 * 4;
    const int64_t tiles = (a.B + 15) / 16;
    int64_t waves = (int64_t)cu_count() * kU8rWavesPerCu;
    waves = waves < tiles ? waves : tiles;
    const int64_t groups = (waves + 3) / 4;
    const bool aligned = a.h % 8 == 0 && a.w % 8 == 0;
    const bool buf = in.in_bytes < ((int64_t)1 << 31) && in.out_bytes < ((int64_t)1 << 31);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(256), 0, stream, a, in, tiles, waves);
    };
    constexpr int D = kU8rDepth;
    if (prec == DCTF_PREC_FP32) {
        if (aligned)
            buf ? go(k_filter_u8r8<DCTF_PREC_FP32, true, true, D>) : go(k_filter_u8r8<DCTF_PREC_FP32, true, false, D>);
        else
            buf ? go(k_filter_u8r8<DCTF_PREC_FP32, false, true, D>) : go(k_filter_u8r8<DCTF_PREC_FP32, false, false, D>);
    } else {
        if (aligned)
            buf ? go(k_filter_u8r8<DCTF_PREC_SPLIT_BF16, true, true, D>)
                : go(k_filter_u8r8<DCTF_PREC_SPLIT_BF16, true, false, D>);
        else
            buf ? go(k_filter_u8r8<DCTF_PREC_SPLIT_BF16, false, true, D>)
                : go(k_filter_u8r8<DCTF_PREC_SPLIT_BF16, false, false, D>);
    }
    return hipGetLastError();
}

hipError_t launch_filter_px(int N, int prec, int in_kind, const PxArgs &a, hipStream_t stream)
{
    if (a.B <= 0)
        return hipSuccess;
    if (N <= 4) {
        const int64_t groups = (a.B + 255) / 256;
        if (in_kind)
            hipLaunchKernelGGL(k_filter_px_small<1>, dim3((unsigned)groups), dim3(256), 0, stream, a, N);
        else
            hipLaunchKernelGGL(k_filter_px_small<0>, dim3((unsigned)groups), dim3(256), 0, stream, a, N);
        return hipGetLastError();
    }
    return prec == DCTF_PREC_FP32 ? dispatch_px<DCTF_PREC_FP32>(N, in_kind, a, stream)
                                  : dispatch_px<DCTF_PREC_SPLIT_BF16>(N, in_kind, a, stream);
}

}  // namespace dctf
