// Device helpers shared by the filter kernels: MFMA operand types, the
// FP32 -> BF16 hi/lo split and the per-tile compute of the N = 8 and N = 16
// paths.  Everything here targets gfx950 (64-lane waves, 16x16 MFMA tiles).
#pragma once

#include "dctf_internal.h"

namespace dctf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two FP32 values -> packed BF16 pair (low half = a), round-to-nearest-even.
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b)
{
    f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// x = hi + lo + r with hi = bf16(x), lo = bf16(x - hi); x - hi is exact in FP32.
__device__ __forceinline__ void split_bf16(float4 x, uint32_t &h01, uint32_t &h23, uint32_t &l01,
                                           uint32_t &l23)
{
    h01 = pack_bf16x2(x.x, x.y);
    h23 = pack_bf16x2(x.z, x.w);
    float hx = __uint_as_float(h01 << 16), hy = __uint_as_float(h01 & 0xffff0000u);
    float hz = __uint_as_float(h23 << 16), hw = __uint_as_float(h23 & 0xffff0000u);
    l01 = pack_bf16x2(x.x - hx, x.y - hy);
    l23 = pack_bf16x2(x.z - hz, x.w - hw);
}

__device__ __forceinline__ f32x4 mfma_bf16(u32x4 a, u32x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Value of `v` held by lane `src` (within the wave).
__device__ __forceinline__ float lane_read(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// Accesses of device (global) memory.  The pointers reach the kernels inside
// argument structures and work tables, where the compiler cannot tell their
// address space; the explicit global space keeps them off the flat path,
// whose loads also count against the LDS wait counter (every LDS wait would
// then wait for the loads in flight as well).
typedef __attribute__((address_space(1))) f32x4 g_f32x4;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;
typedef __attribute__((address_space(1))) f32x2 g_f32x2;
typedef __attribute__((address_space(1))) uint32_t g_u32;

__device__ __forceinline__ const g_f32x4 *gp4(const float *p) { return (const g_f32x4 *)p; }
__device__ __forceinline__ g_f32x4 *gp4(float *p) { return (g_f32x4 *)p; }

__device__ __forceinline__ float4 ld4(const float *p)
{
    const f32x4 v = *gp4(p);
    return make_float4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ float4 ld4_nt(const float *p)
{
    const f32x4 v = __builtin_nontemporal_load(gp4(p));
    return make_float4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ void st4(float *p, f32x4 v) { *gp4(p) = v; }

__device__ __forceinline__ void st4_nt(float *p, f32x4 v) { __builtin_nontemporal_store(v, gp4(p)); }

// 16 bytes / 8 bytes / 4 bytes of device memory.
__device__ __forceinline__ u32x4 ldg_u32x4(const void *p) { return *(const g_u32x4 *)p; }
__device__ __forceinline__ f32x2 ldg_f32x2(const float *p) { return *(const g_f32x2 *)p; }
__device__ __forceinline__ uint32_t ldg_u32(const void *p) { return *(const g_u32 *)p; }

// uint8 conversion of a filtered pixel (Sec. III): round half up, saturate
// to [0, 255], decided in FP32 (NaN gives 0).
__device__ __forceinline__ uint32_t pixel_u8(float p)
{
    const float r = floorf(p + 0.5f);
    return (uint32_t)(r > 0.0f ? (r > 255.0f ? 255.0f : r) : 0.0f);
}

// Four pixels -> one little-endian word (first pixel in the low byte), the
// rule of pixel_u8 for finite values: floor(p + 1/2) is an exact integer,
// which V_CVT_PK_U8_F32 converts and packs into its byte.  The CDNA ISA
// reference defines that opcode's conversion as float -> unsigned byte with
// the destination's range, i.e. the clamp the ISA's float-to-integer
// conversions apply (out-of-range values saturate to 0 or 255, NaN gives 0),
// so no separate clamp is needed.  The GPU tests check the saturating cases
// (256, 300, 1e9, +inf -> 255; -0.5, -300, -inf -> 0; NaN -> 0).
__device__ __forceinline__ uint32_t pack_u8x4(float a, float b, float c, float d)
{
    const float v[4] = {a, b, c, d};
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w = __builtin_amdgcn_cvt_pk_u8_f32(floorf(v[k] + 0.5f), k, w);
    return w;
}

// Four pixels (one little-endian word, first pixel at column x) into row y
// of an h x w raster image with row pitch `pitch` bytes (a multiple of 4):
// one word store where all four columns are inside the image, byte stores
// at the right edge, nothing below the last row.
__device__ __forceinline__ void store_px_raster4(uint8_t *img, int64_t pitch, int h, int w, int y, int x,
                                                 uint32_t word)
{
    if (y >= h)
        return;
    uint8_t *row = img + (int64_t)y * pitch;
    if (x + 3 < w) {
        *reinterpret_cast<uint32_t *>(row + x) = word;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (x + e < w)
                row[x + e] = (uint8_t)(word >> (8 * e));
    }
}

// Eight quantised coefficients (one 16-byte load, little-endian int16) times
// their dequantisation factors q[0..7]; `dc` is added to the first one.
__device__ __forceinline__ void dequant8(u32x4 raw, const float q[8], float dc, float4 &lo, float4 &hi)
{
    float x[8];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        x[2 * w] = (float)(int16_t)(raw[w] & 0xffffu) * q[2 * w];
        x[2 * w + 1] = (float)((int32_t)raw[w] >> 16) * q[2 * w + 1];
    }
    x[0] += dc;
    lo = make_float4(x[0], x[1], x[2], x[3]);
    hi = make_float4(x[4], x[5], x[6], x[7]);
}

// ------------------------------------------------------------------ N = 8
//
// One wave holds the whole 64 x 64 operator in VGPRs as MFMA A fragments and
// computes Y^t = H . X^t for 16 blocks per MFMA tile: M = 64 output
// coefficients (4 M-tiles of 16), N = 16 blocks, K = 64 input coefficients.
// Lane (n, g) = (lane % 16, lane / 16) loads X[n][16i + 4g + j] (i, j in
// 0..3) with four 16-byte loads, so each load instruction covers 64
// contiguous bytes of 16 blocks.  The MFMA contraction index is permuted to
// match (the builder wrote H's columns in the same permutation).  Lane (n, g)
// receives Y[n][16t + 4g + r], r = 0..3, and stores it as one 16-byte store
// per M-tile.

struct OpRegs8F32 {
    float A[4][4][4];   // [t][i][j]
    float h0[4][4];     // [t][r] = H[16t + 4g + r][0]
};

struct OpRegs8BF16 {
    u32x4 hi[4][2];     // [t][s]
    u32x4 lo[4][2];
    float lf[4][2];     // [t][j]: FP32 A operand of the two low-frequency k-steps
};

__device__ __forceinline__ void load_op8(OpRegs8F32 &R, const float *frag32, const float *h0, int lane)
{
    const int g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float4 v = ld4(frag32 + ((t * 4 + i) * 64 + lane) * 4);
            R.A[t][i][0] = v.x;
            R.A[t][i][1] = v.y;
            R.A[t][i][2] = v.z;
            R.A[t][i][3] = v.w;
        }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float4 v = ld4(h0 + 16 * t + 4 * g);
        R.h0[t][0] = v.x;
        R.h0[t][1] = v.y;
        R.h0[t][2] = v.z;
        R.h0[t][3] = v.w;
    }
}

// From device memory (the operator's fragment images).
__device__ __forceinline__ void load_op8(OpRegs8BF16 &R, const uint16_t *fhi, const uint16_t *flo,
                                         const float *flf, int lane)
{
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            R.hi[t][s] = ldg_u32x4(fhi + ((t * 2 + s) * 64 + lane) * 8);
            R.lo[t][s] = ldg_u32x4(flo + ((t * 2 + s) * 64 + lane) * 8);
        }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x2 v = ldg_f32x2(flf + (t * 64 + lane) * 2);
        R.lf[t][0] = v[0];
        R.lf[t][1] = v[1];
    }
}

// The same fragments from copies in LDS (the pointers point into __shared__
// arrays; device-memory loads must not be used on them).
typedef __attribute__((address_space(3))) const u32x4 l_u32x4;
typedef __attribute__((address_space(3))) const f32x2 l_f32x2;

__device__ __forceinline__ void load_op8_lds(OpRegs8BF16 &R, const uint16_t *fhi, const uint16_t *flo,
                                             const float *flf, int lane)
{
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            R.hi[t][s] = *(l_u32x4 *)(fhi + ((t * 2 + s) * 64 + lane) * 8);
            R.lo[t][s] = *(l_u32x4 *)(flo + ((t * 2 + s) * 64 + lane) * 8);
        }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x2 v = *(l_f32x2 *)(flf + (t * 64 + lane) * 2);
        R.lf[t][0] = v[0];
        R.lf[t][1] = v[1];
    }
}

// Y for one 16-block tile held in x[4] (lane layout above); DC in FP32.
__device__ __forceinline__ void tile8(const OpRegs8F32 &R, float4 x[4], int lane, f32x4 acc[4])
{
    const int n = lane & 15;
    const float x0 = lane_read(x[0].x, n);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // rows u = 7, 6 first and u = 1, 0 last: the large low-frequency
    // products enter the FP32 sum after the many small ones
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

// Split path.  Components x, y of load 0 (k-steps j = 0, 1: coefficients
// 4g and 4g + 1 of rows u = 0, 1, DC included) are multiplied in FP32 MFMA;
// the other 56 coefficients are split into BF16 hi + lo and multiplied as
// hi.hi + hi.lo + lo.hi (the low-frequency columns of the BF16 fragments are
// zero, and those inputs enter the BF16 products as zeros).  The BF16
// products come first, from the higher-frequency k-step down, and the large
// low-frequency FP32 products last.
// acc += H . x for one tile, split path (the order and operands of tile8
// below, without clearing acc first).
__device__ __forceinline__ void tile8_acc(const OpRegs8BF16 &R, const float4 x[4], f32x4 acc[4])
{
    u32x4 bh[2], bl[2];
    {
        // BF16 operand element 4e + j of k-step s is coefficient 16(2s + e) + 4g + j
        uint32_t h0, h1, h2, h3, l0, l1, l2, l3;
        split_bf16(make_float4(0.0f, 0.0f, x[0].z, x[0].w), h0, h1, l0, l1);
        split_bf16(x[1], h2, h3, l2, l3);
        bh[0] = u32x4{0u, h1, h2, h3};
        bl[0] = u32x4{0u, l1, l2, l3};
        split_bf16(x[2], h0, h1, l0, l1);
        split_bf16(x[3], h2, h3, l2, l3);
        bh[1] = u32x4{h0, h1, h2, h3};
        bl[1] = u32x4{l0, l1, l2, l3};
    }
    // higher-frequency k-step first; the FP32 low-frequency part last
#pragma unroll
    for (int s = 1; s >= 0; --s) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = mfma_bf16(R.lo[t][s], bh[s], acc[t]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = mfma_bf16(R.hi[t][s], bl[s], acc[t]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = mfma_bf16(R.hi[t][s], bh[s], acc[t]);
    }
    const float x0[2] = {x[0].x, x[0].y};
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = mfma_f32(R.lf[t][j], x0[j], acc[t]);
}

__device__ __forceinline__ void tile8(const OpRegs8BF16 &R, float4 x[4], int lane, f32x4 acc[4])
{
    (void)lane;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    tile8_acc(R, x, acc);
}

// ------------------------------------------------- N = 8, coalesced I/O
//
// Optional staging of a 16-block tile (4 KiB) through a wave-private LDS
// region so that every global load and store instruction of the wave covers
// 1 KiB of contiguous memory (four whole blocks).  Chunk c (16 bytes,
// coefficients 4c..4c+3) of block b lives in LDS slot b*16 + (c ^ b):
//   - global side: instruction i, lane l handles block b = 4i + l/16, chunk
//     (l % 16) ^ b, i.e. LDS slot i*64 + l (a permutation inside the same
//     1 KiB, so the access stays fully coalesced);
//   - MFMA side: lane (n, g) reads chunk 4j + g of block n (the register
//     layout of tile8), slot n*16 + ((4j + g) ^ n): the 16 lanes of a phase
//     hit 16 different bank groups.
// LDS accesses of one wave execute in order; wave_lds_sync() only keeps the
// compiler from moving them across each other.

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool NT>
__device__ __forceinline__ void load_tile_coalesced(float4 x[4], const float *tile, int64_t nvalid, int lane)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int b = 4 * i + (lane >> 4);
        const int c = (lane & 15) ^ b;
        const int64_t bb = b < nvalid ? b : nvalid - 1;   // clamped: its result is never stored
        const float *p = tile + bb * 64 + 4 * c;
        x[i] = NT ? ld4_nt(p) : ld4(p);
    }
}

__device__ __forceinline__ void stage_in(float4 *lds, const float4 x[4], int lane)
{
#pragma unroll
    for (int i = 0; i < 4; ++i)
        lds[i * 64 + lane] = x[i];
}

__device__ __forceinline__ void read_mfma(const float4 *lds, float4 x[4], int lane)
{
    const int n = lane & 15, g = lane >> 4;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        x[j] = lds[n * 16 + ((4 * j + g) ^ n)];
}

__device__ __forceinline__ void stage_out(float4 *lds, const f32x4 acc[4], int lane)
{
    const int n = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        lds[n * 16 + ((4 * t + g) ^ n)] = make_float4(acc[t][0], acc[t][1], acc[t][2], acc[t][3]);
}

template <bool NT>
__device__ __forceinline__ void store_tile_coalesced(float *tile, int64_t nvalid, const float4 *lds, int lane)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int b = 4 * i + (lane >> 4);
        const int c = (lane & 15) ^ b;
        const float4 v = lds[i * 64 + lane];
        if (b < nvalid) {
            const f32x4 w = {v.x, v.y, v.z, v.w};
            if (NT)
                st4_nt(tile + (int64_t)b * 64 + 4 * c, w);
            else
                st4(tile + (int64_t)b * 64 + 4 * c, w);
        }
    }
}

// One 16-block tile through the coalesced path: registers x (coalesced
// layout) -> LDS -> MFMA -> LDS -> global.
template <bool NT, typename Regs>
__device__ __forceinline__ void tile8_coalesced(const Regs &R, const float4 xin[4], float4 *lds, float *tile,
                                                int64_t nvalid, int lane)
{
    stage_in(lds, xin, lane);
    wave_lds_sync();
    float4 xm[4];
    read_mfma(lds, xm, lane);
    f32x4 acc[4];
    tile8(R, xm, lane, acc);
    wave_lds_sync();
    stage_out(lds, acc, lane);
    wave_lds_sync();
    store_tile_coalesced<NT>(tile, nvalid, lds, lane);
    wave_lds_sync();
}

// ------------------------------------------- N = 8, buffer-resource tile I/O
//
// The same tile layouts through raw buffer instructions over a resource that
// covers exactly the valid blocks of the tile: loads past the end return
// zeros and stores past the end are dropped by the hardware, so a ragged
// tile needs neither clamped addresses nor branches around its stores.  The
// tile base lives in scalar registers and every lane's byte offset is a
// constant of the lane, which leaves no 64-bit address arithmetic in the
// loop; and since every store is issued on every path, the memory counter
// waits stay exact (a skipped store would make the compiler wait for all).

typedef __amdgpu_buffer_rsrc_t rsrc_t;
// Descriptor word 3 of a raw buffer (32-bit data format) on gfx9-family chips.
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int64_t uniform_i64(int64_t v) { return (int64_t)uniform_u64((uint64_t)v); }

// n / d from the two words of div_magic(d) (see there).
__device__ __forceinline__ uint32_t div_u32(uint32_t n, const uint32_t *m)
{
    const uint64_t p = (uint64_t)m[1] * n + __umulhi(m[0], n);
    return (m[0] | m[1]) ? (uint32_t)(p >> 32) : n;
}

// Image, block row and block column of block `blk` (< 2^32) of images of bpi
// blocks, Bw per block row; magic = div_magic of bpi, then of Bw.
__device__ __forceinline__ void raster_place(uint32_t blk, int bpi, int Bw, const uint32_t *magic, int64_t &img,
                                             int &by, int &bx)
{
    const uint32_t i = div_u32(blk, magic);
    const uint32_t lb = blk - i * (uint32_t)bpi;
    const uint32_t r = div_u32(lb, magic + 2);
    img = i;
    by = (int)r;
    bx = (int)(lb - r * (uint32_t)Bw);
}

// Resource over the blocks [blk0, min(blk0 + 16, B)) of an array of blocks of
// `block_bytes` bytes; empty when blk0 >= B (and, as a guard, when blk0 < 0).
// Arguments are wave-uniform.
__device__ __forceinline__ rsrc_t tile_rsrc(const void *base, int64_t blk0, int64_t B, int block_bytes)
{
    const int64_t nv = B - blk0;
    const bool ok = nv > 0 && blk0 >= 0;
    const int bytes = !ok ? 0 : (nv >= 16 ? 16 * block_bytes : (int)nv * block_bytes);
    const char *p = static_cast<const char *>(base) + (ok ? blk0 : 0) * block_bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, bytes, kRsrcWord3);
}

// N = 8 blocks of FP32 coefficients (256 bytes).
__device__ __forceinline__ rsrc_t tile_rsrc8(const float *base, int64_t blk0, int64_t B)
{
    return tile_rsrc(base, blk0, B, 256);
}

// Waits until at most n vector memory accesses of the wave are in flight
// (they complete in issue order for this count).
template <int n>
__device__ __forceinline__ void wait_vm()
{
    static_assert(n >= 0 && n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | 0x70 | 0xF00);
}

// Waits for every vector memory access of the wave in flight.  After a
// conditional reload (operator fragments), this lets the compiler know at
// the join that nothing of it is pending: otherwise it would wait for all
// loads at the next use of those registers on every path.
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// 16 bytes at byte offset `off` of the resource (the b128 buffer builtins
// move four 32-bit words; the floats are reinterpreted, not converted).
template <bool NT>
__device__ __forceinline__ float4 buf_ld4(rsrc_t r, uint32_t off)
{
    const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, NT ? 2 : 0));
    return make_float4(v[0], v[1], v[2], v[3]);
}

template <bool NT>
__device__ __forceinline__ void buf_st4(rsrc_t r, uint32_t off, f32x4 v)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, NT ? 2 : 0);
}

// Byte offsets of a lane's four 16-byte chunks in the coalesced layout
// (instruction i: block b = 4i + lane/16, chunk (lane % 16) ^ b) ...
__device__ __forceinline__ void coalesced_offsets(uint32_t off[4], int lane)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int b = 4 * i + (lane >> 4);
        off[i] = (uint32_t)(b * 256 + 16 * ((lane & 15) ^ b));
    }
}

// ... and in the MFMA layout (chunk 4i + g of block n).
__device__ __forceinline__ void mfma_offsets(uint32_t off[4], int lane)
{
#pragma unroll
    for (int i = 0; i < 4; ++i)
        off[i] = (uint32_t)((lane & 15) * 256 + 64 * i + 16 * (lane >> 4));
}

template <bool NT>
__device__ __forceinline__ void load_tile_buf(float4 x[4], rsrc_t r, const uint32_t off[4])
{
#pragma unroll
    for (int i = 0; i < 4; ++i)
        x[i] = buf_ld4<NT>(r, off[i]);
}

// One 16-block tile through the coalesced path with buffer I/O: registers
// (coalesced layout) -> LDS -> MFMA -> LDS -> device memory.
template <bool NT, typename Regs>
__device__ __forceinline__ void tile8_buf(const Regs &R, const float4 xin[4], float4 *lds, rsrc_t out,
                                         const uint32_t off[4], int lane)
{
    stage_in(lds, xin, lane);
    wave_lds_sync();
    float4 xm[4];
    read_mfma(lds, xm, lane);
    f32x4 acc[4];
    tile8(R, xm, lane, acc);
    wave_lds_sync();
    stage_out(lds, acc, lane);
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float4 v = lds[i * 64 + lane];
        buf_st4<NT>(out, off[i], f32x4{v.x, v.y, v.z, v.w});
    }
    wave_lds_sync();
}

// The same tile with loads and stores in the MFMA layout (no LDS).
template <bool NT, typename Regs>
__device__ __forceinline__ void tile8_buf_direct(const Regs &R, float4 x[4], rsrc_t out, const uint32_t off[4],
                                                 int lane)
{
    f32x4 acc[4];
    tile8(R, x, lane, acc);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        buf_st4<NT>(out, off[t], acc[t]);
}

// ------------------------------------------- N = 8, tiles loaded into LDS
//
// The coalesced-layout loads can write LDS directly (buffer_load ... lds):
// lane l of instruction i deposits its 16 bytes at slot i*64 + l of the
// wave's tile buffer, the layout stage_in() writes, without passing through
// VGPRs.  The tile then goes LDS -> MFMA layout -> MFMA -> LDS -> device
// memory as in tile8_buf.  Two LDS tile buffers per wave alternate; they are
// separate __shared__ arrays, so the compiler can tell a read of one from
// the loads in flight into the other and waits for the right loads only.
typedef __attribute__((address_space(3))) void lds_void_t;

// The loads are kept ahead of everything after them (the scheduler would
// otherwise sink them below the next tile's LDS reads, shortening the time
// they have to arrive).
// Four stores into an empty resource (dropped by the hardware; they still
// count as vector memory accesses): they stand in for the stores of a step
// before the first, so that every step finds the same count in flight.
template <bool NT>
__device__ __forceinline__ void dummy_stores8(const float *base, const uint32_t off[4])
{
    const rsrc_t none = tile_rsrc8(base, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        buf_st4<NT>(none, off[i], f32x4{0.f, 0.f, 0.f, 0.f});
    __builtin_amdgcn_sched_barrier(0);
}

template <bool NT>
__device__ __forceinline__ void dma_tile8(float4 *lds, rsrc_t r, const uint32_t off[4])
{
#pragma unroll
    for (int i = 0; i < 4; ++i)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t *)(lds + i * 64), 16, off[i], 0, 0, NT ? 2 : 0);
    __builtin_amdgcn_sched_barrier(0);
}

// The compiler does not reliably order reads of a tile buffer after the
// loads into it (its tracking of loads to LDS missed some of the reads of a
// tile, which then read stale data), so the tile loop waits itself: it keeps
// the number of vector memory accesses issued after a tile's loads fixed
// (the stores of the step before, the next tile's loads, and per-step
// extras), and each step waits with that count (WAIT) before reading its
// tile.
template <int WAIT, bool NT, typename Regs>
__device__ __forceinline__ void tile8_from_lds(const Regs &R, float4 *lds, rsrc_t out, const uint32_t off[4],
                                               int lane)
{
    wait_vm<WAIT>();
    __builtin_amdgcn_sched_barrier(0);
    float4 xm[4];
    read_mfma(lds, xm, lane);
    f32x4 acc[4];
    tile8(R, xm, lane, acc);
    wave_lds_sync();
    stage_out(lds, acc, lane);
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float4 v = lds[i * 64 + lane];
        buf_st4<NT>(out, off[i], f32x4{v.x, v.y, v.z, v.w});
    }
    wave_lds_sync();
}

// ----------------------------------------------------------------- N = 16
//
// Weight-stationary: a workgroup of 8 waves holds the 256 x 256 operator in
// VGPRs, wave w owning output rows [32w, 32w + 32) (two M-tiles).  A tile of
// 16 blocks is staged in LDS once and read by all 8 waves.  Rows (one block
// each) are split into 16-byte chunks stored XOR-swizzled by the row index,
// chunk c of row b at position c ^ b, which keeps the 16-byte MFMA-layout
// reads of a wave free of bank conflicts (padded rows are not, on gfx950):
//   FP32: [16][256] floats; lane (n, g) reads chunk 4i + g of row n, i = 0..15.
//   BF16: hi / lo [16][256] BF16, split once when written; lane (n, g) reads
//         chunk 4s + g (8 BF16), s = 0..7.  The 8 low-frequency coefficients
//         (lf_slot) go to an FP32 array [4][16][2] instead (slots 2g, 2g + 1
//         of row n at (g*16 + n)*2) and are multiplied in FP32 MFMA.

constexpr int kLd16F32 = 256;    // floats per LDS row (FP32 path)
constexpr int kLd16BF16 = 256;   // BF16 per LDS row (split path)
constexpr int kLd16Lf = 8;       // floats per block of the low-frequency FP32 part

// LDS bytes of one 16-block tile buffer.
constexpr int kTile16BytesF32 = 16 * kLd16F32 * 4;
constexpr int kTile16BytesSplit = 2 * 16 * kLd16BF16 * 2 + 16 * kLd16Lf * 4;
// LDS of the tile loop: two tiles, plus (split path) 64 floats that the
// loader's lanes without a low-frequency coefficient write instead, so that
// the extraction has no branches.
constexpr int kSmem16F32 = 2 * kTile16BytesF32;
constexpr int kSmem16Split = 2 * kTile16BytesSplit + 64 * 4;

// Element offsets of 16-byte chunk c of row b.
__device__ __forceinline__ int f32_chunk(int b, int c) { return b * kLd16F32 + 4 * (c ^ b); }
__device__ __forceinline__ int bf16_chunk(int b, int c) { return b * kLd16BF16 + 8 * (c ^ b); }

struct OpRegs16F32 {
    float A[2][16][4];
    float h0[2][4];
};

struct OpRegs16BF16 {
    u32x4 hi[2][8];
    u32x4 lo[2][8];
    float lf[2][2];     // [t][j]: FP32 A operand of the two low-frequency k-steps
};

__device__ __forceinline__ void load_op16(OpRegs16F32 &R, const float *frag32, const float *h0,
                                          int wave, int lane)
{
    const int g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int T = 2 * wave + t;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            float4 v = ld4(frag32 + ((T * 16 + i) * 64 + lane) * 4);
            R.A[t][i][0] = v.x;
            R.A[t][i][1] = v.y;
            R.A[t][i][2] = v.z;
            R.A[t][i][3] = v.w;
        }
        float4 v = ld4(h0 + 16 * T + 4 * g);
        R.h0[t][0] = v.x;
        R.h0[t][1] = v.y;
        R.h0[t][2] = v.z;
        R.h0[t][3] = v.w;
    }
}

__device__ __forceinline__ void load_op16(OpRegs16BF16 &R, const uint16_t *fhi, const uint16_t *flo,
                                          const float *flf, int wave, int lane)
{
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int T = 2 * wave + t;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            R.hi[t][s] = ldg_u32x4(fhi + ((T * 8 + s) * 64 + lane) * 8);
            R.lo[t][s] = ldg_u32x4(flo + ((T * 8 + s) * 64 + lane) * 8);
        }
        const f32x2 v = ldg_f32x2(flf + (T * 64 + lane) * 2);
        R.lf[t][0] = v[0];
        R.lf[t][1] = v[1];
    }
}

// LDS staging of one 16-block tile.  Each thread holds two 16-byte FP32
// chunks of the tile (stage16_pos): from FP32 coefficients (IN = 0) thread q
// of the workgroup holds chunk (block q / 64, coefficients 4(q % 64) .. +3)
// and the chunk q + 512; from quantised int16 coefficients (IN = 1) its one
// 16-byte load is coefficients 8(q % 32) .. +7 of block q / 32, kept raw in
// registers and dequantised into the two chunks 2(q % 32), 2(q % 32) + 1
// when the tile is written to LDS.
template <int IN>
struct Stage16;

template <>
struct Stage16<0> {
    float4 v[2];
};

template <>
struct Stage16<1> {
    u32x4 raw;
};

// IN = 2, 3: one parity class (pu, pv) of N = 32 blocks as blocks of 256
// coefficients in class order (q = 16a + b for (u, v) = (2a + pu, 2b + pv)):
// class chunk c (coefficients 4c .. 4c + 3) is every other float of the 8
// from column 8(c % 4) of row 2(c / 4) + pu.  IN = 2 loads the four with
// 32-bit loads; IN = 3 loads all 8 as two float4s (half the load
// instructions and cache-line lookups, twice the registers) and picks the
// class's four when the tile is written to LDS.
template <>
struct Stage16<2> {
    float4 v[2];
};

template <>
struct Stage16<3> {
    float4 v[2][2];
    int pv;
};

__device__ __forceinline__ void stage16_chunks(const Stage16<0> &S, const float *, float, float4 v[2])
{
    v[0] = S.v[0];
    v[1] = S.v[1];
}

// qv: the thread's eight dequantisation factors; dc: the offset of the DC
// coefficient (non-zero only in the thread holding it).
__device__ __forceinline__ void stage16_chunks(const Stage16<1> &S, const float *qv, float dc, float4 v[2])
{
    dequant8(S.raw, qv, dc, v[0], v[1]);
}

__device__ __forceinline__ void stage16_chunks(const Stage16<2> &S, const float *, float, float4 v[2])
{
    v[0] = S.v[0];
    v[1] = S.v[1];
}

__device__ __forceinline__ void stage16_chunks(const Stage16<3> &S, const float *, float, float4 v[2])
{
#pragma unroll
    for (int h = 0; h < 2; ++h)
        v[h] = S.pv ? make_float4(S.v[h][0].y, S.v[h][0].w, S.v[h][1].y, S.v[h][1].w)
                    : make_float4(S.v[h][0].x, S.v[h][0].z, S.v[h][1].x, S.v[h][1].z);
}

template <int IN>
__device__ __forceinline__ void stage16_pos(int tid, int h, int &b, int &c)
{
    if constexpr (IN != 1) {
        const int q = tid + 512 * h;
        b = q >> 6;
        c = q & 63;
    } else {
        b = tid >> 5;
        c = 2 * (tid & 31) + h;
    }
}

// Tile loads through a resource over the tile's valid blocks (blocks past
// the end read as zeros; their results are never stored).
__device__ __forceinline__ void stage16_load_q(Stage16<1> &S, rsrc_t r, int tid)
{
    // int16 block: 512 bytes; thread q: coefficients 8(q % 32) .. +7 of block q / 32
    S.raw = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                          r, (uint32_t)((tid >> 5) * 512 + 16 * (tid & 31)), 0, 2));
}

// class cls = 2 pu + pv of a tile of 16 N = 32 blocks (4 KiB each)
__device__ __forceinline__ void stage16_load_cls(Stage16<2> &S, rsrc_t r, int tid, int cls)
{
    const int pu = cls >> 1, pv = cls & 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = tid + 512 * h, c = q & 63;
        const uint32_t off = (uint32_t)((q >> 6) * 4096 + ((2 * (c >> 2) + pu) * 32 + 8 * (c & 3) + pv) * 4);
        S.v[h] = make_float4(__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0)),
                             __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off + 8, 0, 0)),
                             __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off + 16, 0, 0)),
                             __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off + 24, 0, 0)));
    }
}

__device__ __forceinline__ void stage16_load_cls(Stage16<3> &S, rsrc_t r, int tid, int cls)
{
    const int pu = cls >> 1;
    S.pv = cls & 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = tid + 512 * h, c = q & 63;
        const uint32_t off = (uint32_t)((q >> 6) * 4096 + ((2 * (c >> 2) + pu) * 32 + 8 * (c & 3)) * 4);
        S.v[h][0] = buf_ld4<false>(r, off);
        S.v[h][1] = buf_ld4<false>(r, off + 16);
    }
}

__device__ __forceinline__ void stage16_load(Stage16<0> &S, rsrc_t r, int tid)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = tid + 512 * h;
        S.v[h] = buf_ld4<false>(r, (uint32_t)((q >> 6) * 1024 + 16 * (q & 63)));
    }
}

template <int IN>
__device__ __forceinline__ void stage16_store(const Stage16<IN> &S, float *lds, int tid, const float *qv, float dc)
{
    float4 v[2];
    stage16_chunks(S, qv, dc, v);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        int b, c;
        stage16_pos<IN>(tid, h, b, c);
        *reinterpret_cast<float4 *>(lds + f32_chunk(b, c)) = v[h];
    }
}

// Split path: the low-frequency coefficients go to the FP32 array llf (slot
// order of lf_slot) and enter the BF16 arrays as zeros.  Every element is
// written somewhere (other lanes' values to their word of `trash`), so the
// extraction is branch-free.
template <int IN>
__device__ __forceinline__ void stage16_store(const Stage16<IN> &S, uint16_t *lhi, uint16_t *llo,
                                              float *llf, float *trash, int tid, const float *qv, float dc)
{
    float4 v[2];
    stage16_chunks(S, qv, dc, v);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        int b, c;
        stage16_pos<IN>(tid, h, b, c);
        float xv[4] = {v[h].x, v[h].y, v[h].z, v[h].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int slot = lf_slot(16, 4 * c + e);
            const bool lf = slot >= 0;
            float *dst = lf ? llf + ((slot >> 1) * 16 + b) * 2 + (slot & 1) : trash + (tid & 63);
            *dst = xv[e];
            xv[e] = lf ? 0.0f : xv[e];
        }
        uint32_t h01, h23, l01, l23;
        split_bf16(make_float4(xv[0], xv[1], xv[2], xv[3]), h01, h23, l01, l23);
        const int off = bf16_chunk(b, c >> 1) + 4 * (c & 1);
        *reinterpret_cast<uint2 *>(lhi + off) = make_uint2(h01, h23);
        *reinterpret_cast<uint2 *>(llo + off) = make_uint2(l01, l23);
    }
}

// `mid` runs once in the middle of the k-steps (the tile loop stages the next
// tile into the other LDS buffer there, beside the MFMA work).
struct NoMid {
    __device__ void operator()() const {}
};

template <typename Mid = NoMid>
__device__ __forceinline__ void tile16(const OpRegs16F32 &R, const float *lds, int lane, f32x4 acc[2],
                                       const Mid &mid = Mid())
{
    const int n = lane & 15, g = lane >> 4;
    acc[0] = f32x4{0.f, 0.f, 0.f, 0.f};
    acc[1] = acc[0];
    // highest-frequency rows first, rows u = 0, 1 last (FP32 accuracy)
#pragma unroll
    for (int i = 15; i >= 0; --i) {
        const float4 xv4 = *reinterpret_cast<const float4 *>(lds + f32_chunk(n, 4 * i + g));
        const float xv[4] = {xv4.x, xv4.y, xv4.z, xv4.w};
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[t] = mfma_f32(R.A[t][i][j], xv[j], acc[t]);
        if (i == 8)
            mid();
    }
    const float x0 = lds[f32_chunk(n, 0)];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            acc[t][r] = fmaf(R.h0[t][r], x0, acc[t][r]);
}

template <typename Mid = NoMid>
__device__ __forceinline__ void tile16(const OpRegs16BF16 &R, const uint16_t *lhi, const uint16_t *llo,
                                       const float *llf, int lane, f32x4 acc[2], const Mid &mid = Mid())
{
    const int n = lane & 15, g = lane >> 4;
    acc[0] = f32x4{0.f, 0.f, 0.f, 0.f};
    acc[1] = acc[0];
    // BF16 products from the highest-frequency k-step down, then the large
    // low-frequency FP32 products last
#pragma unroll
    for (int s = 7; s >= 0; --s) {
        const u32x4 bh = *reinterpret_cast<const u32x4 *>(lhi + bf16_chunk(n, 4 * s + g));
        const u32x4 bl = *reinterpret_cast<const u32x4 *>(llo + bf16_chunk(n, 4 * s + g));
#pragma unroll
        for (int t = 0; t < 2; ++t)
            acc[t] = mfma_bf16(R.lo[t][s], bh, acc[t]);
#pragma unroll
        for (int t = 0; t < 2; ++t)
            acc[t] = mfma_bf16(R.hi[t][s], bl, acc[t]);
#pragma unroll
        for (int t = 0; t < 2; ++t)
            acc[t] = mfma_bf16(R.hi[t][s], bh, acc[t]);
        if (s == 4)
            mid();
    }
    // low-frequency slots 2g + j of block n, FP32
    const float2 lv = *reinterpret_cast<const float2 *>(llf + (g * 16 + n) * 2);
    const float lfv[2] = {lv.x, lv.y};
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int t = 0; t < 2; ++t)
            acc[t] = mfma_f32(R.lf[t][j], lfv[j], acc[t]);
}

// ----------------------------------------------- N = 16 tile loop (shared)
//
// Runs `count` tiles of one workgroup through the weight-stationary path.
// Global loads run D tiles ahead of the MFMA work (a ring of D register
// stages); LDS tiles are double-buffered with one barrier per tile.
// With one operator, the next tile is written to the other LDS buffer halfway
// through a tile's MFMA work, so its conversion (the BF16 split) runs beside
// the MFMAs.
// ref(t) returns the UnitRef-like descriptor of the t-th tile (called in
// increasing t, also for t >= count: such a tile must be past the end of its
// job, so that it reads nothing); op_load(op) loads the operator fragments
// into R.  MULTI_OP = false: every tile has the operator of tile 0, loaded
// once before the loop; true: a tile of another operator reloads it (then
// every load in flight is waited for, so that no later wait has to assume
// the reload pending).  Every step issues the same loads and stores (past
// the end, through empty resources), so the compiler's memory-counter waits
// let the D tiles ahead stay in flight.
// IN = 0: FP32 coefficients from r.in; IN = 1: int16 coefficients from
// r.qin, dequantised with qtab (N*N factors) and dc_offset on the DC term;
// IN = 2: parity class r.cls of N = 32 blocks from r.in (Stage16<2>).
// OUT = 0: FP32 results to r.out; OUT = 1: uint8 pixels to r.pix (the
// operator is then the pixel-domain one); OUT = 2: the same pixels into the
// raster images at r.pix (r.h x r.w, row pitch r.pitch, r.Bw blocks per row,
// r.bpi blocks and r.img_stride bytes per image); OUT = 3: FP32 results of
// parity class r.cls back to their places in the N = 32 blocks at r.out.
template <int PREC, int D, typename Ref, int IN = 0, int OUT = 0, bool MULTI_OP = false, bool LATE_PUT = false,
          typename RefFn, typename OpFn, typename Regs>
__device__ __forceinline__ void run_tiles16(int64_t count, RefFn ref, OpFn op_load, Regs &R, char *smem,
                                            const float *qtab = nullptr, float dc_offset = 0.0f)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    float qv[8];
    float dc = 0.0f;
    if constexpr (IN == 1) {
        const float4 q0 = ld4(qtab + 8 * (tid & 31)), q1 = ld4(qtab + 8 * (tid & 31) + 4);
        qv[0] = q0.x; qv[1] = q0.y; qv[2] = q0.z; qv[3] = q0.w;
        qv[4] = q1.x; qv[5] = q1.y; qv[6] = q1.z; qv[7] = q1.w;
        dc = (tid & 31) == 0 ? dc_offset : 0.0f;
    }
    constexpr int kF32 = 16 * kLd16F32;
    constexpr int kB16 = 16 * kLd16BF16;
    float *lf = reinterpret_cast<float *>(smem);
    uint16_t *lhi = reinterpret_cast<uint16_t *>(smem);
    uint16_t *llo = lhi + 2 * kB16;
    float *llf = reinterpret_cast<float *>(llo + 2 * kB16);
    float *trash = llf + 2 * 16 * kLd16Lf;   // split path only: 64 floats past the two tiles
    auto put = [&](const Stage16<IN> &S, int buf) {
        if constexpr (PREC == DCTF_PREC_FP32)
            stage16_store<IN>(S, lf + buf * kF32, tid, qv, dc);
        else
            stage16_store<IN>(S, lhi + buf * kB16, llo + buf * kB16, llf + buf * 16 * kLd16Lf, trash, tid, qv,
                              dc);
    };
    auto stage = [&](Stage16<IN> &S, const Ref &r) {
        if constexpr (IN == 0)
            stage16_load(S, tile_rsrc(r.in, r.blk0, r.B, 1024), tid);
        else if constexpr (IN == 1)
            stage16_load_q(S, tile_rsrc(r.qin, r.blk0, r.B, 512), tid);
        else
            stage16_load_cls(S, tile_rsrc(r.in, r.blk0, r.B, 4096), tid, r.cls);
    };
    // Output offsets of the lane (block n, rows 32 wave + 4g .. and + 16).
    const uint32_t out_off = (uint32_t)(n * (OUT == 0 ? 1024 : 256) + (OUT == 0 ? 4 : 1) * (32 * wave + 4 * g));

    Stage16<IN> S[D];
    Ref Rf[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        Rf[d] = ref(d);
        stage(S[d], Rf[d]);
    }
    int loaded_op = -1;
    if constexpr (!MULTI_OP) {
        op_load(Rf[0].op);
        loaded_op = Rf[0].op;
        wait_vm_all();   // the loop then never waits for the operator loads
    }
    put(S[0], 0);
    __syncthreads();
    // One tile: (operator reload,) loads of the tile D ahead into its free
    // stage, MFMA work from LDS, stores, and (unless it is the last tile) the
    // next tile's stage into the other LDS buffer.
    auto step = [&](auto P, int64_t t, bool last) {
        constexpr int p = decltype(P)::value;
        const Ref rc = Rf[p];
        if constexpr (MULTI_OP) {
            if (rc.op != loaded_op) {
                op_load(rc.op);
                loaded_op = rc.op;
                wait_vm_all();
            }
        }
        // S[p] is free (its tile is in LDS): load the tile D ahead into it,
        // kept ahead of the MFMA work by a scheduling barrier
        Rf[p] = ref(t + D);
        stage(S[p], Rf[p]);
        __builtin_amdgcn_sched_barrier(0);
        const int buf = (int)(t & 1);
        f32x4 acc[2];
        // the next tile's stage goes into the other buffer (free since the
        // last barrier) halfway through this tile's MFMA work (single-operator
        // loops; with operator reloads the registers are too tight for it, and
        // LATE_PUT defers it to the end of the tile, which gives loads issued
        // one tile ahead the whole tile's work to land)
        auto mid = [&]() {
            if (!MULTI_OP && !LATE_PUT && !last)
                put(S[(p + 1) % D], buf ^ 1);
        };
        if constexpr (PREC == DCTF_PREC_FP32)
            tile16(R, lf + buf * kF32, lane, acc, mid);
        else
            tile16(R, lhi + buf * kB16, llo + buf * kB16, llf + buf * 16 * kLd16Lf, lane, acc, mid);
        if constexpr (OUT == 0) {
            const rsrc_t o = tile_rsrc(rc.out, rc.blk0, rc.B, 1024);
            buf_st4<false>(o, out_off, acc[0]);
            buf_st4<false>(o, out_off + 64, acc[1]);
        } else if constexpr (OUT == 3) {
            // The wave's results are the class rows a = 2 wave + t (all 16 b)
            // of the 16 blocks: 32 row pieces.  They pass through the wave's
            // own 2 KiB of LDS (row piece 16 t + n, lane (n, g) holding
            // b = 4g .. 4g + 3; LDS accesses of a wave complete in order, so
            // no barrier) and leave with 16 lanes per row piece: b = j at
            // (u, v) = (4 wave + 2t + pu, 2j + pv), four rows per store
            // instruction instead of sixteen.
            float *ost = reinterpret_cast<float *>(smem + (PREC == DCTF_PREC_FP32 ? kSmem16F32 : kSmem16Split)) +
                         wave * 512;
#pragma unroll
            for (int t = 0; t < 2; ++t)
                *reinterpret_cast<f32x4 *>(ost + (16 * t + n) * 16 + 4 * g) = acc[t];
            __builtin_amdgcn_wave_barrier();
            const rsrc_t o = tile_rsrc(rc.out, rc.blk0, rc.B, 4096);
            const int j = lane & 15;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int rp = 4 * i + (lane >> 4), t = rp >> 4, blk = rp & 15;
                const uint32_t off = (uint32_t)(blk * 4096 + ((4 * wave + 2 * t + (rc.cls >> 1)) * 32 + 2 * j + (rc.cls & 1)) * 4);
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(ost[rp * 16 + j]), o, off, 0, 0);
            }
            __builtin_amdgcn_wave_barrier();
        } else if constexpr (OUT == 1) {
            const rsrc_t o = tile_rsrc(rc.pix, rc.blk0, rc.B, 256);
            __builtin_amdgcn_raw_buffer_store_b32(pack_u8x4(acc[0][0], acc[0][1], acc[0][2], acc[0][3]), o,
                                                  out_off, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(pack_u8x4(acc[1][0], acc[1][1], acc[1][2], acc[1][3]), o,
                                                  out_off + 16, 0, 0);
        } else {
            // raster image: pixels 4g .. 4g + 3 of rows 2 wave and 2 wave + 1 of block n
            if (rc.blk0 + n < rc.B) {
                int64_t img;
                int by, bx;
                raster_place((uint32_t)(rc.blk0 + n), rc.bpi, rc.Bw, rc.magic, img, by, bx);
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    store_px_raster4(rc.pix + img * rc.img_stride, rc.pitch, rc.h, rc.w, 16 * by + 2 * wave + t,
                                     16 * bx + 4 * g, pack_u8x4(acc[t][0], acc[t][1], acc[t][2], acc[t][3]));
            }
        }
        if (!last) {
            if constexpr (MULTI_OP || LATE_PUT)
                put(S[(p + 1) % D], buf ^ 1);
            __syncthreads();
        }
    };
    // Whole rounds of D tiles that are all followed by another tile: a loop
    // without exits in its body (an exit there would join the loop's latch
    // and make the compiler's waits assume the exit path's counts); then the
    // last 1..D tiles.
    const int64_t full = (count - 1) / D;
    int64_t t0 = 0;
    for (int64_t it = 0; it < full; ++it, t0 += D) {
        step(std::integral_constant<int, 0>(), t0, false);
        if constexpr (D > 1)
            step(std::integral_constant<int, (1 % D)>(), t0 + 1, false);
        if constexpr (D > 2)
            step(std::integral_constant<int, (2 % D)>(), t0 + 2, false);
        if constexpr (D > 3)
            step(std::integral_constant<int, (3 % D)>(), t0 + 3, false);
        if constexpr (D > 4)
            step(std::integral_constant<int, (4 % D)>(), t0 + 4, false);
    }
    static_assert(D >= 1 && D <= 5, "tiles ahead: 1 to 5");
    bool last = t0 + 1 >= count;
    step(std::integral_constant<int, 0>(), t0, last);
    if (last)
        return;
    if constexpr (D > 1) {
        last = t0 + 2 >= count;
        step(std::integral_constant<int, (1 % D)>(), t0 + 1, last);
        if (last)
            return;
    }
    if constexpr (D > 2) {
        last = t0 + 3 >= count;
        step(std::integral_constant<int, (2 % D)>(), t0 + 2, last);
        if (last)
            return;
    }
    if constexpr (D > 3) {
        last = t0 + 4 >= count;
        step(std::integral_constant<int, (3 % D)>(), t0 + 3, last);
        if (last)
            return;
    }
    if constexpr (D > 4)
        step(std::integral_constant<int, (4 % D)>(), t0 + 4, true);
}

}  // namespace dctf
