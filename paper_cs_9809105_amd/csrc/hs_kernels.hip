// hs_kernels.hip -- HIP kernels for gfx950 (CDNA4) implementing the
// hyper-systolic matrix product (Sec. 5.2.2, Algorithm HYPER-SYSTOLIC) on one
// GPU, with p virtual processors realised as groups of workgroups.
//
// Kernels
//   pack_kernel      operand preparation: copies (or splits, or quantises) a
//                    row-major operand into the packed tile layout described
//                    in hs_internal.h; HBM bound.
//   pack_mn_kernel   the same for an MN-major FP32 source, read as 16-byte
//                    runs of 4 rows and transposed through LDS.
//   mm_kernel        the hot loop: one workgroup holds an output tile of
//                    G stripes of one residue class mod K and is the
//                    collector of the back-shift (base C = (0,1,..,1)): it
//                    visits the partials c^{K-1}, .., c^0 (the auxiliary
//                    arrays C^l of Sec. 5.2.2) and forms each on the spot as
//                    the virtual processor that owns it: K~ steps over the
//                    travelling blocks kb = (v + jK) mod p (base
//                    A = (0,K,..,K)), fetched through registers and a
//                    double-buffered LDS ring, times the pre-shifted static
//                    block (base B = (0,-1,..,-1)), on MFMA, into one
//                    accumulator that never leaves the registers.
//   backshift_kernel the collector of the all-pairs interaction (hs_nbody):
//                    sums K partial planes in FP64, fixed order.
//   gemv_kernel      y = A x with the same index map, collector form: one
//                    wave owns a row and combines the K partial dot products
//                    in the back-shift order (gemv_c32_kernel: complex64).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "hs_internal.h"

namespace hs {

#define DEVI __device__ __forceinline__

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 16 bytes, a native vector
typedef int i32x8 __attribute__((ext_vector_type(8)));             // 32 fp8 values

// ---------------------------------------------------------------------------
// number formats
// ---------------------------------------------------------------------------
// Eight floats -> the 16-byte units of their three BF16 pieces,
// x = a0 + a1 + a2 with a0 = bf16(x), a1 = bf16(x - a0), a2 = bf16(x - a0 - a1):
// round to nearest even, two values per conversion instruction
// (v_cvt_pk_bf16_f32), residuals exact in FP32.  Word j of a unit holds
// elements 2j (low half) and 2j + 1.  The instruction was compared with a
// software round-to-nearest-even on 24 million values (random bit patterns,
// every exponent, exact ties, denormals): no difference.
DEVI void split3_units(const float (&x)[8], u32x4 &p0, u32x4 &p1, u32x4 &p2) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const f32x2 v = {x[2 * j], x[2 * j + 1]};
        const uint32_t w0 = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
        const f32x2 r1 = v - f32x2{__uint_as_float(w0 << 16), __uint_as_float(w0 & 0xffff0000u)};
        const uint32_t w1 = __builtin_bit_cast(uint32_t, __builtin_convertvector(r1, bf16x2));
        const f32x2 r2 = r1 - f32x2{__uint_as_float(w1 << 16), __uint_as_float(w1 & 0xffff0000u)};
        p0[j] = w0;
        p1[j] = w1;
        p2[j] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r2, bf16x2));
    }
}

// float -> e4m3 (OCP FP8: 1 sign, 4 exponent bits with bias 7, 3 mantissa
// bits; largest finite 448, no infinities), round to nearest, ties to even,
// saturating at 448 (subnormals m * 2^-9, m = 1..7), four values at a time:
// gfx950's conversion instruction on values clamped to [-448, 448].  The
// instruction's rounding was compared with a software round-to-nearest-even
// encoder on every e4m3 value, every midpoint between neighbours and the
// floats next to each midpoint, both signs, values below the smallest
// subnormal and 8 million random ones: no difference.  The tests compare
// the quantisation bit for bit with the oracle's encoder.
DEVI uint32_t e4m3x4(float x0, float x1, float x2, float x3) {
    auto c = [](float x) { return fminf(fmaxf(x, -448.0f), 448.0f); };
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(c(x0), c(x1), 0, false);     // bytes 0, 1
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c(x2), c(x3), w, true);          // bytes 2, 3
    return (uint32_t)w;
}
// byte B of a word of four e4m3 codes -> float (exact)
template <int B> DEVI float e4m3_byte_to_f32(uint32_t w) { return __builtin_amdgcn_cvt_f32_fp8((int)w, B); }

// Largest e with amax * 2^e <= 448 (0 for an all-zero tile), clamped so that
// the block-scale byte 127 - e stays a finite E8M0 value.
DEVI int fp8_exponent(float amax) {
    if (!(amax > 0.0f) || !(amax < 3.0e38f)) return 0;
    int E;
    const float m = frexpf(amax, &E);                      // amax = m 2^E, m in [0.5, 1)
    int e = (m <= 0.875f ? 9 : 8) - E;                     // 448 = 0.875 * 2^9
    return e < -126 ? -126 : (e > 126 ? 126 : e);
}

// ---------------------------------------------------------------------------
// pack
// ---------------------------------------------------------------------------
// One workgroup per 128 x 128 scale tile: amax of the tile, then (with
// refinement) amax of the residuals a 2^e - q0, both turned into exponents.
// The tile is 128 lines of 128 contiguous floats in memory (rows of a
// K-major source, contraction rows of an MN-major one); each of the 512
// threads holds 8 float4 of it in registers (one read of the tile), line
// t * 16 + tid / 32, float4 tid % 32, so a wave reads two 512-byte lines per
// load.  VEC: rows are 16-byte aligned (ld % 4 == 0, 16-byte aligned base).
DEVI float wave_max(float m) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) m = fmaxf(m, __shfl_xor(m, s, 64));
    return m;
}

template <int VEC>
__global__ __launch_bounds__(512) void fp8_tile_exp_kernel(Fp8ExpArgs a) {
    __shared__ float red[2][8];
    const int64_t tr = blockIdx.x / a.tiles_k, tc = blockIdx.x % a.tiles_k;
    const int tid = threadIdx.x, wave = tid >> 6;
    // memory lines (outer index) and contiguous positions (inner index)
    const int64_t o0 = (a.kmajor ? tr : tc) * FP8_TILE, i0 = (a.kmajor ? tc : tr) * FP8_TILE;
    const int64_t olim = a.kmajor ? a.R : a.Kd, ilim = a.kmajor ? a.Kd : a.R;
    const int64_t ib = i0 + (tid & 31) * 4;
    float4 v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int64_t o = o0 + t * 16 + (tid >> 5);
        const float *q = a.src + o * a.ld + ib;
        if (VEC && o < olim && ib + 3 < ilim) {
            v[t] = *(const float4 *)q;
        } else {
            const bool ol = o < olim;
            v[t].x = ol && ib < ilim ? q[0] : 0.f;
            v[t].y = ol && ib + 1 < ilim ? q[1] : 0.f;
            v[t].z = ol && ib + 2 < ilim ? q[2] : 0.f;
            v[t].w = ol && ib + 3 < ilim ? q[3] : 0.f;
        }
    }
    auto block_max = [&](float m, float (&r)[8]) {
        m = wave_max(m);
        if ((tid & 63) == 0) r[wave] = m;
        __syncthreads();
        float x = r[0];
#pragma unroll
        for (int w = 1; w < 8; ++w) x = fmaxf(x, r[w]);
        return x;
    };
    float m = 0.f;
#pragma unroll
    for (int t = 0; t < 8; ++t)
        m = fmaxf(m, fmaxf(fmaxf(fabsf(v[t].x), fabsf(v[t].y)), fmaxf(fabsf(v[t].z), fabsf(v[t].w))));
    const float amax = block_max(m, red[0]);
    const int e = fp8_exponent(amax);
    int e1 = 0;
    if (a.refine) {
        float mr = 0.f;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            // a 2^e is exact; its residual after rounding to e4m3 is exact too
            const float x0 = ldexpf(v[t].x, e), x1 = ldexpf(v[t].y, e), x2 = ldexpf(v[t].z, e),
                        x3 = ldexpf(v[t].w, e);
            const uint32_t q = e4m3x4(x0, x1, x2, x3);
            mr = fmaxf(mr, fmaxf(fmaxf(fabsf(x0 - e4m3_byte_to_f32<0>(q)), fabsf(x1 - e4m3_byte_to_f32<1>(q))),
                                 fmaxf(fabsf(x2 - e4m3_byte_to_f32<2>(q)), fabsf(x3 - e4m3_byte_to_f32<3>(q)))));
        }
        const float rmax = block_max(mr, red[1]);
        e1 = rmax > 0.0f ? fp8_exponent(rmax) : 0;
        if (e1 > 127 - e) e1 = 127 - e;                    // keep 127 - e - e1 >= 0
        if (e1 < -127 - e) e1 = -127 - e;
    }
    if (tid == 0) {
        a.exps[blockIdx.x * 2] = e;
        a.exps[blockIdx.x * 2 + 1] = e1;
    }
}

// Scale exponent of an operand row from its amax bits: the largest e with
// amax 2^e < 2^15 is 15 - frexp_exp(amax) (frexp_exp(0) = 0: any e suits
// a row of zeros).
DEVI int row_scale_exp(uint32_t amax_bits) { return 15 - __builtin_amdgcn_frexp_expf(__uint_as_float(amax_bits)); }

// Eight floats of one row -> the 16-byte units of their two FP16 pieces,
// x' = x 2^e, a0 = f16(x'), a1 = f16(x' - a0): round to nearest even, the
// residual exact in FP32 (a0 is within a factor 2 of x', or both lie below
// 2^-14 on the 2^-24 grid).  Word j holds elements 2j (low half), 2j + 1.
DEVI void split2_f16_units(const float (&x)[8], int e, u32x4 &p0, u32x4 &p1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const f32x2 v = {ldexpf(x[2 * j], e), ldexpf(x[2 * j + 1], e)};   // exact
        const f16x2 h0 = __builtin_convertvector(v, f16x2);
        const f32x2 r = v - __builtin_convertvector(h0, f32x2);
        p0[j] = __builtin_bit_cast(uint32_t, h0);
        p1[j] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, f16x2));
    }
}

template <int KIND> struct PackTraits;
template <> struct PackTraits<PK_F64> { typedef double S; static const int UE = 2; static const int ESZ = 8; static const int NP = 1; };
template <> struct PackTraits<PK_F32> { typedef float S; static const int UE = 4; static const int ESZ = 4; static const int NP = 1; };
template <> struct PackTraits<PK_B16> { typedef uint16_t S; static const int UE = 8; static const int ESZ = 2; static const int NP = 1; };
template <> struct PackTraits<PK_SPLIT3> { typedef float S; static const int UE = 8; static const int ESZ = 2; static const int NP = 3; };
template <> struct PackTraits<PK_FP8> { typedef float S; static const int UE = 16; static const int ESZ = 1; static const int NP = 2; };
template <> struct PackTraits<PK_SPLIT2F16> { typedef float S; static const int UE = 8; static const int ESZ = 2; static const int NP = 2; };

// Write one 16-byte unit (of each piece) of the packed image: row rr of
// group grp, block kb, chunk ch, plane half, from the unit's values.
template <int KIND>
DEVI void pack_emit(const PackArgs &a, uint32_t grp, uint32_t kb, uint32_t ch, uint32_t half, uint32_t rr,
                    int64_t row, bool rvalid, int64_t kk0, const float *vals_f, const double *vals_d,
                    const uint16_t *vals_h) {
    const OperandGeom &g = a.g;
    const uint32_t nch = (uint32_t)g.nch, gr = (uint32_t)g.grp_rows;
    // chunk = UPR planes of 16 bytes per row: [plane][row][16 bytes]
    // [group][piece][block][chunk][plane][row][16 bytes]
    const int64_t inner = ((int64_t)kb * nch + ch) * gr * g.chunk_bytes + ((int64_t)half * gr + rr) * 16;
    uint8_t *dst = (uint8_t *)a.dst + (int64_t)grp * g.group_bytes + inner;
    auto put = [&](int64_t at, const u32x4 &w) { *(u32x4 *)(dst + at) = w; };
    if constexpr (KIND == PK_F64) {
        put(0, __builtin_bit_cast(u32x4, make_double2(vals_d[0], vals_d[1])));
    } else if constexpr (KIND == PK_F32) {
        put(0, u32x4{__float_as_uint(vals_f[0]), __float_as_uint(vals_f[1]), __float_as_uint(vals_f[2]),
                     __float_as_uint(vals_f[3])});
    } else if constexpr (KIND == PK_B16) {
        u32x4 w;
        w[0] = vals_h[0] | ((uint32_t)vals_h[1] << 16);
        w[1] = vals_h[2] | ((uint32_t)vals_h[3] << 16);
        w[2] = vals_h[4] | ((uint32_t)vals_h[5] << 16);
        w[3] = vals_h[6] | ((uint32_t)vals_h[7] << 16);
        put(0, w);
    } else if constexpr (KIND == PK_FP8) {
        // all 16 elements of the unit lie in one 128 x 128 scale tile
        int e = 0, e1 = 0;
        if (rvalid && kk0 < g.Kd) {
            const int64_t t2 = ((row / FP8_TILE) * a.exp_tiles_k + kk0 / FP8_TILE) * 2;
            e = a.exps[t2];
            e1 = a.exps[t2 + 1];
        }
        u32x4 w0, w1 = {0, 0, 0, 0};
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            float xs[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) xs[i] = ldexpf(vals_f[4 * d + i], e);   // exact
            w0[d] = e4m3x4(xs[0], xs[1], xs[2], xs[3]);
            if (a.refine) {
                // the residual a 2^e - q0 is exact; scaled by 2^e1, rounded again
                const uint32_t q = w0[d];
                w1[d] = e4m3x4(ldexpf(xs[0] - e4m3_byte_to_f32<0>(q), e1), ldexpf(xs[1] - e4m3_byte_to_f32<1>(q), e1),
                               ldexpf(xs[2] - e4m3_byte_to_f32<2>(q), e1), ldexpf(xs[3] - e4m3_byte_to_f32<3>(q), e1));
            }
        }
        put(0, w0);
        if (a.refine) put(g.piece_bytes, w1);
    } else if constexpr (KIND == PK_SPLIT2F16) {
        const int e = rvalid ? row_scale_exp(((const uint32_t *)a.exps)[row]) : 0;
        u32x4 w0, w1;
        split2_f16_units(*(const float(*)[8])vals_f, e, w0, w1);
        put(0, w0);
        put(g.piece_bytes, w1);
    } else {   // PK_SPLIT3: a0 = bf16(a), a1 = bf16(a - a0), a2 = bf16(a - a0 - a1)
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = vals_f[e];
        u32x4 w0, w1, w2;
        split3_units(x, w0, w1, w2);
        put(0, w0);
        put(g.piece_bytes, w1);
        put(2 * g.piece_bytes, w2);
    }
}

// Row amax of the two-piece FP16 split, K-major source: one wave per row,
// 16-byte loads when VEC (ld % 4 == 0, 16-byte aligned base).  NaNs are
// skipped (fmaxf); they reach the product through the values themselves.
template <int VEC>
__global__ __launch_bounds__(256) void row_amax_k_kernel(RowAmaxArgs a) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= a.R) return;
    const float *q = a.src + (a.embed == EMB_BLOCKS_H ? row >> 1 : row) * a.ld;
    float m = 0.f;
    int64_t k = 0;
    if (VEC) {
        const int64_t k4 = a.Kd / 4 * 4;
#pragma unroll 4
        for (k = lane * 4; k < k4; k += 256) {
            const float4 v = *(const float4 *)(q + k);
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
        k = k4;
    }
    for (int64_t kk = k + lane; kk < a.Kd; kk += 64) m = fmaxf(m, fabsf(q[kk]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if (lane == 0) a.amax[row] = __float_as_uint(m);
}

// Row amax, MN-major source (element (kk, c) of the float view at
// src[kk ld + c]): thread columns (4 per thread when VEC) over a slab of
// 256 contraction rows, then one atomic max per column into its row (two
// for EMB_BLOCKS); the host zero-fills amax first.  Workgroup b takes column
// block b % ncb of slab b / ncb.
DEVI void amax_into_rows(const RowAmaxArgs &a, int64_t c, float m) {
    const uint32_t bits = __float_as_uint(m);
    if (a.embed == EMB_BLOCKS) {
        atomicMax(a.amax + (c & ~(int64_t)1), bits);
        atomicMax(a.amax + (c | 1), bits);
    } else if (a.embed == EMB_TRANS || a.embed == EMB_CONJ) {
        atomicMax(a.amax + (c >> 1), bits);
    } else {
        atomicMax(a.amax + c, bits);
    }
}

template <int VEC>
__global__ __launch_bounds__(256) void row_amax_mn_kernel(RowAmaxArgs a) {
    constexpr int CW = VEC ? 4 : 1;
    // the float view's columns and contraction rows
    const int64_t ncol = (a.embed == EMB_TRANS || a.embed == EMB_CONJ) ? 2 * a.R : a.R;
    const int64_t nk = a.embed == EMB_NONE ? a.Kd : a.Kd / 2;
    const int64_t ncb = (ncol + 256 * CW - 1) / (256 * CW);
    const int64_t r0 = ((int64_t)(blockIdx.x % ncb) * 256 + threadIdx.x) * CW;
    if (r0 >= ncol) return;
    const int64_t k0 = (int64_t)(blockIdx.x / ncb) * 256;
    const int64_t k1 = k0 + 256 < nk ? k0 + 256 : nk;
    float m[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) m[j] = 0.f;
    bool done = false;
    if constexpr (VEC) {
        if (r0 + 3 < ncol) {
#pragma unroll 4
            for (int64_t kk = k0; kk < k1; ++kk) {
                const float4 v = *(const float4 *)(a.src + kk * a.ld + r0);
                m[0] = fmaxf(m[0], fabsf(v.x));
                m[1] = fmaxf(m[1], fabsf(v.y));
                m[2] = fmaxf(m[2], fabsf(v.z));
                m[3] = fmaxf(m[3], fabsf(v.w));
            }
            done = true;
        }
    }
    if (!done) {
        for (int64_t kk = k0; kk < k1; ++kk)
#pragma unroll
            for (int j = 0; j < CW; ++j)
                if (r0 + j < ncol) m[j] = fmaxf(m[j], fabsf(a.src[kk * a.ld + r0 + j]));
    }
#pragma unroll
    for (int j = 0; j < CW; ++j)
        if (r0 + j < ncol) amax_into_rows(a, r0 + j, m[j]);
}

// An MN-major unit of pack_kernel's numbering: row rr of group grp, block
// kb, chunk ch, plane half, and where its elements lie in the source.
struct MnUnit {
    uint32_t rr, half, ch, kb, grp;
    int64_t row, kin0, kk0;
    bool rvalid;
};

template <int KIND>
DEVI MnUnit mn_decode(uint32_t u, const OperandGeom &g) {
    typedef PackTraits<KIND> T;
    const int KC = g.chunk_bytes / T::ESZ;
    const uint32_t UPR = (uint32_t)(g.chunk_bytes / 16), nch = (uint32_t)g.nch, p = (uint32_t)g.p;
    const uint32_t gr = (uint32_t)g.grp_rows;
    MnUnit d;
    uint32_t t = u;
    d.rr = t % gr;    t /= gr;
    d.half = t % UPR; t /= UPR;
    d.ch = t % nch;   t /= nch;
    d.kb = t % p;
    d.grp = t / p;
    if (g.striped) {
        const int64_t stripe = d.grp / g.GS, msub = d.grp % g.GS;
        const int64_t within = msub * gr + d.rr;
        d.row = stripe * g.S_r + within;
        d.rvalid = within < g.S_r && d.row < g.R;
    } else {
        d.row = (int64_t)d.grp * gr + d.rr;
        d.rvalid = d.row < g.R;
    }
    d.kin0 = (int64_t)d.ch * KC + d.half * T::UE;
    d.kk0 = (int64_t)d.kb * g.S_k + d.kin0;
    return d;
}

// MN-major FP32 source (copy, split and FP8 kinds), transposed through LDS:
// the workgroup's 256 units (pack_kernel's numbering: rows fastest) are read
// as 16-byte runs of 4 rows per contraction index -- 64 lanes read 64 runs,
// one contiguous stretch per group -- into an [element][unit] tile, then each
// thread packs and writes its own unit as pack_kernel does, so consecutive
// threads still write consecutive 16-byte rows.  Host: ld % 4 == 0, source
// 16-byte aligned, grp_rows % 4 == 0, S_r % 4 == 0 for a striped operand;
// total_units is a multiple of 4.
template <int KIND>
__global__ __launch_bounds__(256) void pack_mn_kernel(PackArgs a) {
    typedef PackTraits<KIND> T;
    constexpr int UE = T::UE;                   // 4, 8 or 16 elements per unit
    __shared__ float tile[UE][256];
    const OperandGeom &g = a.g;
    const float *src = (const float *)a.src;
    const uint32_t base = blockIdx.x * 256u;    // host: total_units < 2^31
#pragma unroll
    for (int i = 0; i < UE / 4; ++i) {
        const uint32_t q = threadIdx.x + 256u * i;
        const uint32_t quad = q % 64, e = q / 64;
        const uint32_t u = base + quad * 4;     // units u .. u+3: rows rr .. rr+3 of one group
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (u < (uint32_t)a.total_units) {
            const MnUnit d = mn_decode<KIND>(u, g);
            const int64_t kk = d.kk0 + e;
            if (d.kin0 + e < g.S_k && kk < g.Kd) {
                bool rv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (g.striped) {
                        const int64_t within = (int64_t)(d.grp % g.GS) * g.grp_rows + d.rr + r;
                        rv[r] = within < g.S_r && d.row + r < g.R;
                    } else {
                        rv[r] = d.row + r < g.R;
                    }
                }
                const float *q4 = src + kk * a.ld + d.row;
                if (rv[0] && rv[1] && rv[2] && rv[3]) {
                    v = *(const float4 *)q4;
                } else {
                    v.x = rv[0] ? q4[0] : 0.f;
                    v.y = rv[1] ? q4[1] : 0.f;
                    v.z = rv[2] ? q4[2] : 0.f;
                    v.w = rv[3] ? q4[3] : 0.f;
                }
            }
        }
        *(float4 *)&tile[e][quad * 4] = v;
    }
    __syncthreads();
    const uint32_t u = base + threadIdx.x;
    if (u >= (uint32_t)a.total_units) return;
    const MnUnit d = mn_decode<KIND>(u, g);
    float vals_f[UE];
    double vals_d[1] = {0.0};
    uint16_t vals_h[1] = {0};
#pragma unroll
    for (int e = 0; e < UE; ++e) vals_f[e] = tile[e][threadIdx.x];
    pack_emit<KIND>(a, d.grp, d.kb, d.ch, d.half, d.rr, d.row, d.rvalid, d.kk0, vals_f, vals_d, vals_h);
}

// One thread makes one 16-byte unit of the packed image (for the split form,
// the same unit of each of the three pieces).  Consecutive threads take
// consecutive rows of one (group, block, chunk, plane), so the packed writes
// are contiguous; for a row-major (MN-major) source the reads are contiguous
// too, for a K-major source each thread reads its own 16-32 bytes of a row.
template <int KIND, int KMAJOR>
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a) {
    typedef PackTraits<KIND> T;
    typedef typename T::S S;
    const OperandGeom &g = a.g;
    const uint32_t u = blockIdx.x * 256u + threadIdx.x;     // host: total_units < 2^31
    if (u >= (uint32_t)a.total_units) return;
    const int KC = g.chunk_bytes / T::ESZ;      // elements per chunk row
    const uint32_t UPR = (uint32_t)(g.chunk_bytes / 16);  // 16-byte planes per chunk row
    const uint32_t nch = (uint32_t)g.nch, p = (uint32_t)g.p, gr = (uint32_t)g.grp_rows;
    uint32_t t = u, rr, half, ch, kb, grp;
    if (KMAJOR) {
        // 8 x 8 blocks of (row, unit along the contraction): a wave reads 8
        // rows x 8 consecutive units (128-256 contiguous bytes per row) and
        // writes, per (chunk, plane), 8 consecutive rows (128 bytes).
        const uint32_t nu = nch * UPR;                  // units along one block row
        const uint32_t nkg = (nu + 7) / 8, nrg = (gr + 7) / 8;
        const uint32_t uu = t % 8;  t /= 8;
        const uint32_t rlo = t % 8; t /= 8;
        const uint32_t kg = t % nkg; t /= nkg;
        const uint32_t rhi = t % nrg; t /= nrg;
        kb = t % p;
        grp = t / p;
        const uint32_t ku = kg * 8 + uu;
        rr = rhi * 8 + rlo;
        if (ku >= nu || rr >= gr) return;
        ch = ku / UPR;
        half = ku % UPR;
    } else {
        rr = t % gr;    t /= gr;
        half = t % UPR; t /= UPR;
        ch = t % nch;   t /= nch;
        kb = t % p;
        grp = t / p;
    }
    int64_t row;
    bool rvalid;
    if (g.striped) {
        const int64_t stripe = grp / g.GS, msub = grp % g.GS;
        const int64_t within = msub * gr + rr;
        row = stripe * g.S_r + within;
        rvalid = within < g.S_r && row < g.R;
    } else {
        row = (int64_t)grp * gr + rr;
        rvalid = row < g.R;
    }
    const int64_t kin0 = (int64_t)ch * KC + half * T::UE;
    const int64_t kk0 = (int64_t)kb * g.S_k + kin0;
    const S *src = (const S *)a.src;
    float vals_f[T::UE];
    double vals_d[T::UE];
    uint16_t vals_h[T::UE];
    if (KMAJOR && a.vec) {
        // the unit's elements are contiguous, 16-byte aligned, all valid or all padding
        const bool ok = rvalid && kin0 < g.S_k && kk0 < g.Kd;
        const S *q = src + row * a.ld + kk0;
        constexpr int SB = (int)sizeof(S);             // source element bytes
        constexpr int NV = T::UE * SB / 16;            // 16-byte loads per unit
        u32x4 w[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) w[i] = ok ? *(const u32x4 *)(q + i * (16 / SB)) : u32x4{0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < T::UE; ++e) {
            const int byte = e * SB;
            const uint32_t word = w[byte / 16][(byte % 16) / 4];
            if constexpr (KIND == PK_F64) {
                vals_d[e] = __hiloint2double((int)w[byte / 16][(byte % 16) / 4 + 1], (int)word);
            } else if constexpr (KIND == PK_B16) {
                vals_h[e] = (uint16_t)(word >> ((byte % 4) * 8));
            } else {
                vals_f[e] = __uint_as_float(word);
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < T::UE; ++e) {
            const int64_t kin = kin0 + e;
            const int64_t kk = kk0 + e;
            const bool ok = rvalid && kin < g.S_k && kk < g.Kd;
            int64_t idx = KMAJOR ? row * a.ld + kk : kk * a.ld + row;
            bool neg = false;
            if constexpr (KIND == PK_F32 || KIND == PK_SPLIT3 || KIND == PK_SPLIT2F16) {
                // complex sources: sr = kk % 2 and c = row % 2 pick the entry
                // of the 2 x 2 block [[re, im], [-im, re]]
                const int64_t sr = kk & 1, c = row & 1;
                if (!KMAJOR && a.embed == EMB_BLOCKS) {
                    idx = (kk >> 1) * a.ld + (row - c) + (sr ^ c);
                    neg = sr == 1 && c == 0;
                } else if (KMAJOR && a.embed == EMB_BLOCKS_H) {
                    // conj(x): the im entries change sign
                    idx = (row >> 1) * a.ld + 2 * (kk >> 1) + (sr ^ c);
                    neg = sr == 0 && c == 1;
                } else if (!KMAJOR && (a.embed == EMB_CONJ || a.embed == EMB_TRANS)) {
                    idx = (kk >> 1) * a.ld + 2 * row + sr;
                    neg = a.embed == EMB_CONJ && sr == 1;
                }
            }
            if constexpr (KIND == PK_F64) vals_d[e] = ok ? (double)src[idx] : 0.0;
            else if constexpr (KIND == PK_B16) vals_h[e] = ok ? (uint16_t)src[idx] : (uint16_t)0;
            else vals_f[e] = ok ? (neg ? -(float)src[idx] : (float)src[idx]) : 0.0f;
        }
    }
    pack_emit<KIND>(a, grp, kb, ch, half, rr, row, rvalid, kk0, vals_f, vals_d, vals_h);
}

// ---------------------------------------------------------------------------
// the hyper-systolic main loop on MFMA
// ---------------------------------------------------------------------------
// FORM 0: one piece per operand, one product.  FORM 1: three bf16 pieces,
// the six products a_i b_j with i + j <= 2, smallest first.  FORM 2: two
// f16 pieces of the row-scaled operands, the three products a_i b_j with
// i + j <= 1, smallest first; the epilogue removes the row scales.
template <int FORM> struct Form;
template <> struct Form<0> { static const int NP = 1; static const int NPROD = 1; };
template <> struct Form<1> { static const int NP = 3; static const int NPROD = 6; };
template <> struct Form<2> { static const int NP = 2; static const int NPROD = 3; };

template <int FAM> struct Mfma;
template <> struct Mfma<FAM_F64> { static const int T = 16; typedef f64x4 Acc; };
template <> struct Mfma<FAM_F32> { static const int T = 32; typedef f32x16 Acc; };
template <> struct Mfma<FAM_BF16> { static const int T = 32; typedef f32x16 Acc; };
template <> struct Mfma<FAM_F16> { static const int T = 32; typedef f32x16 Acc; };
template <> struct Mfma<FAM_FP8> { static const int T = 32; typedef f32x16 Acc; };

// Pieces per operand: split-BF16 3, two-piece FP16 2, refined FP8 2 (q0,
// q1), otherwise 1.
template <int FAM, int FORM>
struct Pieces { static const int NP = FAM == FAM_FP8 ? (FORM ? 2 : 1) : Form<FORM>::NP; };

template <int FAM, int FORM, int BM, int BN, int CPS, int WAVES>
struct MmCfg {
    static const int NP = Pieces<FAM, FORM>::NP;
    static const int NT = 64 * WAVES;                   // threads per workgroup
    static const int CB = FAM == FAM_FP8 ? 64 : 32;     // bytes per chunk row
    static const int NPL = CB / 16;                     // 16-byte planes per chunk row
    static const int A_STAGE = NP * CPS * BM * CB;      // LDS bytes per stage
    static const int B_STAGE = NP * CPS * BN * CB;
    static const int UA = NP * CPS * BM * NPL / NT;     // 16-byte loads per thread
    static const int UB = NP * CPS * BN * NPL / NT;
    static_assert(UA * NT == NP * CPS * BM * NPL && UB * NT == NP * CPS * BN * NPL, "tile/threads");
    static const int WM = BM / 2, WN = BN / (WAVES / 2); // waves: 2 along rows, WAVES/2 along columns
    static const int MT = Mfma<FAM>::T;
    static const int TM = WM / MT, TN = WN / MT;
    static const int STAGE = A_STAGE + B_STAGE;         // one slot of the LDS ring
    static const int LPS = UA + UB;                     // DMA loads per thread per stage
    // One wave per SIMD (4 waves of 128 x 128 on the 256 x 256 tile): both
    // operands through LDS, two slots of static LDS, the stage interleaved
    // by hand (FP32, plain BF16 and FP16)
    static const bool W1 = WAVES == 4 && BM == 256;
    // B fragments straight from memory into registers (32x32 families)
    static const bool BD = FAM != FAM_F64 && FAM != FAM_FP8 && !W1;
    static const int LDS_BYTES = W1 ? 0 : 2 * (BD ? A_STAGE : STAGE);   // dynamic LDS: two slots
};

// One pipeline stage of block products from LDS: for every chunk of the
// stage, the wave's MFMA tiles accumulate A_rows x B_cols.
// For FP8, sa[c][P][mi] / sb[c][P][ni] are the E8M0 block-scale bytes of
// chunk c, piece P, row / column tile (uniform across the wave).
template <int FAM, int FORM, int BM, int BN, int CPS, int WAVES, typename AccArr, typename SA, typename SB>
DEVI void mm_compute(AccArr &acc, const uint8_t *Ab, const uint8_t *Bb, int lane, int wm, int wn,
                     const SA &sa, const SB &sb) {
    typedef MmCfg<FAM, FORM, BM, BN, CPS, WAVES> C;
#pragma unroll
    for (int c = 0; c < CPS; ++c) {
        if constexpr (FAM == FAM_FP8) {
            // lane group g holds contraction elements 32g..32g+31 of the
            // 64-element chunk: planes 2g and 2g+1 of the row
            const int r32 = lane & 31, g = lane >> 5;
            i32x8 bv[C::NP][C::TN];
#pragma unroll
            for (int P = 0; P < C::NP; ++P)
#pragma unroll
                for (int ni = 0; ni < C::TN; ++ni) {
                    const uint8_t *q = Bb + (P * CPS + c) * BN * C::CB + (2 * g) * BN * 16 + (wn * C::WN + ni * 32 + r32) * 16;
                    const u32x4 lo = *(const u32x4 *)q, hi = *(const u32x4 *)(q + BN * 16);
                    bv[P][ni] = i32x8{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
                }
#pragma unroll
            for (int mi = 0; mi < C::TM; ++mi) {
                i32x8 av[C::NP];
#pragma unroll
                for (int P = 0; P < C::NP; ++P) {
                    const uint8_t *q = Ab + (P * CPS + c) * BM * C::CB + (2 * g) * BM * 16 + (wm * C::WM + mi * 32 + r32) * 16;
                    const u32x4 lo = *(const u32x4 *)q, hi = *(const u32x4 *)(q + BM * 16);
                    av[P] = i32x8{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
                }
#pragma unroll
                for (int ni = 0; ni < C::TN; ++ni) {
                    if constexpr (C::NP == 2) {
                        // q1 q0', q0 q1', q0 q0': smallest first
                        acc[mi][ni] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            av[1], bv[0][ni], acc[mi][ni], 0, 0, 0, sa[c][1][mi], 0, sb[c][0][ni]);
                        acc[mi][ni] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            av[0], bv[1][ni], acc[mi][ni], 0, 0, 0, sa[c][0][mi], 0, sb[c][1][ni]);
                    }
                    acc[mi][ni] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        av[0], bv[0][ni], acc[mi][ni], 0, 0, 0, sa[c][0][mi], 0, sb[c][0][ni]);
                }
            }
        } else if constexpr (FAM == FAM_F64) {
            const int r16 = lane & 15, g = lane >> 4;
            double av[C::TM], bv[C::TN];
#pragma unroll
            for (int mi = 0; mi < C::TM; ++mi)
                av[mi] = *(const double *)(Ab + (c * 2 + (g >> 1)) * BM * 16 + (wm * C::WM + mi * 16 + r16) * 16 + (g & 1) * 8);
#pragma unroll
            for (int ni = 0; ni < C::TN; ++ni)
                bv[ni] = *(const double *)(Bb + (c * 2 + (g >> 1)) * BN * 16 + (wn * C::WN + ni * 16 + r16) * 16 + (g & 1) * 8);
#pragma unroll
            for (int mi = 0; mi < C::TM; ++mi)
#pragma unroll
                for (int ni = 0; ni < C::TN; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mi], bv[ni], acc[mi][ni], 0, 0, 0);
        } else {
            const int r32 = lane & 31, g = lane >> 5;
            // all B fragments of the chunk, then one row tile of A at a time
            u32x4 bv[C::NP][C::TN];
#pragma unroll
            for (int P = 0; P < C::NP; ++P)
#pragma unroll
                for (int ni = 0; ni < C::TN; ++ni)
                    bv[P][ni] = *(const u32x4 *)(Bb + (P * CPS + c) * BN * C::CB + g * BN * 16 +
                                                 (wn * C::WN + ni * 32 + r32) * 16);
#pragma unroll
            for (int mi = 0; mi < C::TM; ++mi) {
                u32x4 av[C::NP];
#pragma unroll
                for (int P = 0; P < C::NP; ++P)
                    av[P] = *(const u32x4 *)(Ab + (P * CPS + c) * BM * C::CB + g * BM * 16 +
                                             (wm * C::WM + mi * 32 + r32) * 16);
#pragma unroll
                for (int ni = 0; ni < C::TN; ++ni) {
                    if constexpr (FAM == FAM_F32) {
                        // lane group g holds contraction elements 4g..4g+3 of
                        // the chunk; MFMA t takes element t of A and B alike
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                                __uint_as_float(av[0][t]), __uint_as_float(bv[0][ni][t]), acc[mi][ni], 0, 0, 0);
                    } else if constexpr (FAM == FAM_F16) {
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(f16x8, av[0]), __builtin_bit_cast(f16x8, bv[0][ni]), acc[mi][ni], 0, 0, 0);
                    } else if constexpr (FORM == 0) {
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, av[0]), __builtin_bit_cast(bf16x8, bv[0][ni]), acc[mi][ni], 0, 0, 0);
                    } else {
                        // a2 b0, a1 b1, a0 b2, a1 b0, a0 b1, a0 b0: smallest first
#pragma unroll
                        for (int q = 0; q < 6; ++q) {
                            const int pa = q < 3 ? 2 - q : (q == 3 ? 1 : 0);
                            const int pb = q < 3 ? q : (q == 4 ? 1 : 0);
                            acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, av[pa]), __builtin_bit_cast(bf16x8, bv[pb][ni]), acc[mi][ni], 0, 0, 0);
                        }
                    }
                }
            }
        }
    }
}

// Fragment reads and MFMA tile products of the 32x32 families (FP32,
// BF16, FP16, split-BF16) for the B-direct stage below.  Lane group g
// = lane / 32 holds plane g of a chunk row (16 bytes); lane & 31 the row.
template <int FAM, int FORM, int BM, int BN, int CPS, int WAVES, typename AV>
DEVI void read_a_frags(AV &av, const uint8_t *Ab, int c, int mi, int lane, int wm) {
    typedef MmCfg<FAM, FORM, BM, BN, CPS, WAVES> C;
    const int r32 = lane & 31, g = lane >> 5;
#pragma unroll
    for (int P = 0; P < C::NP; ++P)
        av[P] = *(const u32x4 *)(Ab + (P * CPS + c) * BM * C::CB + g * BM * 16 + (wm * C::WM + mi * 32 + r32) * 16);
}

template <int FAM, int FORM, int TN, typename AccRow, typename AV, typename BV>
DEVI void mfma_row(AccRow &accr, const AV &av, const BV &bv) {
#pragma unroll
    for (int ni = 0; ni < TN; ++ni) {
        if constexpr (FAM == FAM_F32) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                accr[ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(av[0][t]), __uint_as_float(bv[0][ni][t]),
                                                               accr[ni], 0, 0, 0);
        } else if constexpr (FAM == FAM_F16 && FORM == 2) {
            // a1 b0, a0 b1, a0 b0: smallest first
            accr[ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av[1]),
                                                              __builtin_bit_cast(f16x8, bv[0][ni]), accr[ni], 0, 0, 0);
            accr[ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av[0]),
                                                              __builtin_bit_cast(f16x8, bv[1][ni]), accr[ni], 0, 0, 0);
            accr[ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av[0]),
                                                              __builtin_bit_cast(f16x8, bv[0][ni]), accr[ni], 0, 0, 0);
        } else if constexpr (FAM == FAM_F16) {
            accr[ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av[0]),
                                                              __builtin_bit_cast(f16x8, bv[0][ni]), accr[ni], 0, 0, 0);
        } else if constexpr (FORM == 0) {
            accr[ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av[0]),
                                                               __builtin_bit_cast(bf16x8, bv[0][ni]), accr[ni], 0, 0, 0);
        } else {
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int pa = q < 3 ? 2 - q : (q == 3 ? 1 : 0);
                const int pb = q < 3 ? q : (q == 4 ? 1 : 0);
                accr[ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av[pa]),
                                                                   __builtin_bit_cast(bf16x8, bv[pb][ni]), accr[ni], 0, 0, 0);
            }
        }
    }
}

// One stage of a 32x32 family whose B fragments are already in registers
// (bq[chunk][piece][column tile]); A fragments come from the LDS slot.
template <int FAM, int FORM, int BM, int BN, int CPS, int WAVES, typename AccArr, typename BQ>
DEVI void mm_compute_bd(AccArr &acc, const uint8_t *Ab, const BQ &bq, int lane, int wm) {
    typedef MmCfg<FAM, FORM, BM, BN, CPS, WAVES> C;
#pragma unroll
    for (int c = 0; c < CPS; ++c)
#pragma unroll
        for (int mi = 0; mi < C::TM; ++mi) {
            u32x4 av[C::NP];
            read_a_frags<FAM, FORM, BM, BN, CPS, WAVES>(av, Ab, c, mi, lane, wm);
            mfma_row<FAM, FORM, C::TN>(acc[mi], av, bq[c]);
        }
}

// Buffer resource over a packed operand (raw buffer, byte addressed; the
// third dword is the gfx9 default format word).
DEVI __amdgpu_buffer_rsrc_t packed_rsrc(const uint8_t *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, 0x00020000);
}

// Global -> registers for one stage: 16-byte buffer loads of the K static
// blocks and of the travelling block.  The per-thread part of each address
// is a constant 32-bit offset; the stage part is wave-uniform (SGPR).
template <int UA, int UB>
DEVI void stage_load(u32x4 (&r)[UA + UB], __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rb,
                     const uint32_t (&a_off)[UA], const uint32_t (&b_off)[UB], uint32_t ach, uint32_t bch) {
#pragma unroll
    for (int q = 0; q < UA; ++q)
        r[q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, (int)a_off[q], (int)ach, 0));
#pragma unroll
    for (int q = 0; q < UB; ++q)
        r[UA + q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rb, (int)b_off[q], (int)bch, 0));
}

// Registers -> LDS slot.  The LDS image of a stage is
// [slab = (piece, chunk)][plane][row][16 bytes]: unit ui = tid + NT q lands
// at ui * 16, so consecutive lanes write consecutive 16 bytes, and the 32
// lanes of an MFMA lane group later read 512 contiguous bytes of one plane.
template <int UA, int UB, int A_STAGE, int NT>
DEVI void stage_store(const u32x4 (&r)[UA + UB], uint8_t *slot, int tid) {
#pragma unroll
    for (int q = 0; q < UA; ++q) *(u32x4 *)(slot + (tid + NT * q) * 16) = r[q];
#pragma unroll
    for (int q = 0; q < UB; ++q) *(u32x4 *)(slot + A_STAGE + (tid + NT * q) * 16) = r[UA + q];
}

template <int UA>
DEVI void stage_load_a(u32x4 (&r)[UA], __amdgpu_buffer_rsrc_t ra, const uint32_t (&a_off)[UA], uint32_t ach) {
#pragma unroll
    for (int q = 0; q < UA; ++q)
        r[q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, (int)a_off[q], (int)ach, 0));
}

template <int UA, int NT>
DEVI void stage_store_a(const u32x4 (&r)[UA], uint8_t *slot, int tid) {
#pragma unroll
    for (int q = 0; q < UA; ++q) *(u32x4 *)(slot + (tid + NT * q) * 16) = r[q];
}

template <int FAM, int FORM, int BM, int BN, int CPS, int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(WAVES / 4, WAVES / 4)))
void mm_kernel(MainArgs a) {
    typedef MmCfg<FAM, FORM, BM, BN, CPS, WAVES> C;
    typedef typename Mfma<FAM>::Acc Acc;
    extern __shared__ __attribute__((aligned(16))) uint8_t ring[];   // C::LDS_BYTES

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    // workgroup -> (class c, stripe group sg, stripe sub-group msub, column
    // tile).  The tile's rows are sub-group msub of the G stripes
    // r0 + i K (i < ng), r0 = c + sg G K: all of residue class c mod K, so
    // they need the same travelling block at every step (see the step order
    // below).  Workgroups are dealt to the 8 XCDs round robin; renumber them
    // so each XCD runs a contiguous range.  Inside it, 32 consecutive
    // workgroups (one per CU of the XCD) take G_V members of one class times
    // G_T column tiles, so the XCD's L2 serves each travelling tile to G_V
    // workgroups and each static tile to G_T of them.
    // With a.nsplit > 1 (launches with fewer output tiles than CUs) the grid
    // holds nsplit copies of the tile grid; copy q walks only stages
    // [q per, (q + 1) per) of the step order and leaves its sums in plane q
    // of a.part (a fixed-order FP64 sum of the planes follows).
    int64_t bid = blockIdx.x;
    {
        const int64_t nwg = gridDim.x, xcd = bid % 8, per = nwg / 8, rem = nwg % 8;
        bid = xcd * per + (xcd < rem ? xcd : rem) + bid / 8;
    }
    const int split = (int)(bid / (gridDim.x / a.nsplit));
    bid %= gridDim.x / a.nsplit;
    const int p = a.p, K = a.K, Kt = a.Kt, MS = a.MS, G = a.G;
    int64_t ntile, msub;
    int c_class, r0, ng;
    {
        const int64_t t_lo = bid % a.grp_t;  bid /= a.grp_t;
        const int64_t u_lo = bid % a.grp_v;  bid /= a.grp_v;
        const int64_t tg = bid % a.n_tg;     bid /= a.n_tg;
        const int64_t ug = bid % a.n_ug;
        c_class = (int)(bid / a.n_ug);
        ntile = tg * a.grp_t + t_lo;
        const int64_t u = ug * a.grp_v + u_lo;        // member of the class: (sg, msub)
        const int nsg = (Kt + G - 1) / G;              // stripe groups per class
        if (ntile >= a.n_ntiles || u >= (int64_t)nsg * a.GS) return;   // grid padding
        msub = u % a.GS;
        const int sg = (int)(u / a.GS);
        r0 = c_class + sg * G * K;
        ng = Kt - sg * G < G ? Kt - sg * G : G;        // stripes of this tile
    }

    const int64_t nch = a.nch;
    const int spb = (int)(nch / CPS);                   // stages per contraction block
    // this workgroup's stages of the p spb (< 2^31, host) of the step order
    const int s_begin = split * a.split_stages;
    const int nstages = p * spb - s_begin < a.split_stages ? p * spb - s_begin : a.split_stages;

    // Each workgroup addresses its own region of the packed operands with
    // 32-bit offsets: for the static operand the G groups msub of stripes
    // r0, r0 + K, .., which sit K GS groups apart; for the travelling operand
    // its group of BN columns.  The host keeps each region below 4 GiB,
    // whatever the size of the operands.  Per-thread load descriptors are
    // offsets that do not depend on the step (group, row, half-row, piece,
    // chunk); units past the tile's ng groups re-read offset 0: their tile
    // rows are never stored.
    uint32_t a_off[C::UA];
#pragma unroll
    for (int q = 0; q < C::UA; ++q) {
        const int ui = tid + C::NT * q;              // unit: [slab][plane][row]
        const int slab = ui / (BM * C::NPL);
        const int within = ui % (BM * C::NPL);
        const int plane = within / BM, rho = within % BM;
        const int P = slab / CPS, c = slab % CPS;
        const int i = rho / MS, ir = rho % MS;
        a_off[q] = i < ng ? (uint32_t)((int64_t)i * K * a.GS * a.a_group + (int64_t)P * a.a_piece +
                                       (int64_t)c * MS * C::CB + (int64_t)(plane * MS + ir) * 16)
                          : 0u;
    }
    uint32_t b_off[C::UB];
#pragma unroll
    for (int q = 0; q < C::UB; ++q) {
        const int ui = tid + C::NT * q;
        const int slab = ui / (BN * C::NPL);
        const int within = ui % (BN * C::NPL);
        const int P = slab / CPS, c = slab % CPS;
        b_off[q] = (uint32_t)((int64_t)P * a.b_piece + (int64_t)c * BN * C::CB + (int64_t)within * 16);
    }
    const __amdgpu_buffer_rsrc_t rsA = packed_rsrc(a.A + ((int64_t)r0 * a.GS + msub) * a.a_group, (uint32_t)a.a_span);
    const __amdgpu_buffer_rsrc_t rsB = packed_rsrc(a.B + ntile * a.b_group, (uint32_t)a.b_group);

    // The step order.  The collector visits the partials l = K-1, .., 0
    // (t = K-1-l).  Partial l of stripe s is virtual processor v = s + l's
    // work: its steps visit the travelling blocks kb = (v + jK) mod p,
    // j = 0..K~-1 (base A = (0, K, .., K)), a cycle of stride K through the
    // residue class (c + l) mod K, which is the same for every stripe of the
    // tile; the cycle is entered at its smallest block (c + l) mod K, so all
    // workgroups of class c hold the same block at the same time.  cs counts
    // the stages inside a block.  Past the last stage the position stays put,
    // so the surplus fetches re-read the last stage (never used).
    struct Pos { int kb, cs, j, t, n; };
    auto advance = [&](Pos &q) {
        if (++q.n >= nstages) return;
        if (++q.cs < spb) return;
        q.cs = 0;
        if (++q.j < Kt) {                               // next step: shift by K along the ring
            q.kb += K;
            return;
        }
        q.j = 0;                                        // next partial of the collector
        ++q.t;
        q.kb = (c_class + K - 1 - q.t) % K;
    };
    // position of stage s_begin: partial t, step j, stage cs of the block
    Pos start;
    {
        const int per_t = Kt * spb;
        start.t = s_begin / per_t;
        start.j = (s_begin % per_t) / spb;
        start.cs = s_begin % spb;
        start.kb = (c_class + K - 1 - start.t) % K + start.j * K;
        start.n = 0;
    }
    const uint32_t a_stage = (uint32_t)(MS * C::CB), b_stage = (uint32_t)(BN * C::CB);
    // first chunk of the stage at q, then advance q by one stage
    auto next_chunk = [&](Pos &q) -> uint32_t {
        // wave-uniform by construction; readfirstlane keeps the stage
        // offsets in SGPRs whatever the compiler's uniformity analysis finds
        const uint32_t ch = (uint32_t)__builtin_amdgcn_readfirstlane((int)((uint32_t)q.kb * (uint32_t)nch + (uint32_t)(q.cs * CPS)));
        advance(q);
        return ch;
    };
    Pos pa = start;
    auto fetch_offsets = [&](uint32_t &ach, uint32_t &bch) {
        const uint32_t ch = next_chunk(pa);
        ach = ch * a_stage;
        bch = ch * b_stage;
    };

    // FP8: block-scale bytes of the stage being multiplied.  Every 32-row
    // (32-column) MFMA tile and every 64-deep chunk lies inside one 128 x 128
    // scale tile (the host checks the alignment), so each scale is uniform
    // across the wave: 127 - e for q0, 127 - e - e1 for q1.
    int sa[CPS][C::NP][C::TM], sb[CPS][C::NP][C::TN];
    Pos pc = start;                                     // stage being multiplied
    int tra[C::TM], trb[C::TN];
    if constexpr (FAM == FAM_FP8) {
#pragma unroll
        for (int mi = 0; mi < C::TM; ++mi) {
            const int rho0 = wm * C::WM + mi * 32;
            const int i = rho0 / MS, i0 = rho0 % MS;
            // rows of the groups past ng are never stored: any valid scale
            int64_t row0 = (int64_t)(r0 + (i < ng ? i : 0) * K) * a.S_r + msub * MS + i0;
            row0 = row0 < a.M ? row0 : a.M - 1;
            tra[mi] = (int)(row0 / FP8_TILE);
        }
#pragma unroll
        for (int ni = 0; ni < C::TN; ++ni) {
            int64_t col0 = ntile * BN + wn * C::WN + ni * 32;
            col0 = col0 < a.N ? col0 : a.N - 1;
            trb[ni] = (int)(col0 / FP8_TILE);
        }
    }
    auto stage_scales = [&]() {
        if constexpr (FAM == FAM_FP8) {
            typedef const __attribute__((address_space(4))) int32_t cint;
            cint *ea = (cint *)a.a_exps;
            cint *eb = (cint *)a.b_exps;
#pragma unroll
            for (int c = 0; c < CPS; ++c) {
                int64_t kk = (int64_t)pc.kb * a.S_k + (int64_t)(pc.cs * CPS + c) * 64;
                kk = kk < a.Kd ? kk : a.Kd - 1;         // padding chunks hold zeros
                const int tc = __builtin_amdgcn_readfirstlane((int)(kk / FP8_TILE));
#pragma unroll
                for (int mi = 0; mi < C::TM; ++mi) {
                    const int t = __builtin_amdgcn_readfirstlane((int)((tra[mi] * a.a_tiles_k + tc) * 2));
                    const int e = ea[t], e1 = ea[t + 1];
                    sa[c][0][mi] = 127 - e;
                    if constexpr (C::NP == 2) sa[c][1][mi] = 127 - e - e1;
                }
#pragma unroll
                for (int ni = 0; ni < C::TN; ++ni) {
                    const int t = __builtin_amdgcn_readfirstlane((int)((trb[ni] * a.b_tiles_k + tc) * 2));
                    const int e = eb[t], e1 = eb[t + 1];
                    sb[c][0][ni] = 127 - e;
                    if constexpr (C::NP == 2) sb[c][1][ni] = 127 - e - e1;
                }
            }
            advance(pc);
        }
    };

    Acc acc[C::TM][C::TN];
#pragma unroll
    for (int mi = 0; mi < C::TM; ++mi)
#pragma unroll
        for (int ni = 0; ni < C::TN; ++ni) acc[mi][ni] = Acc{};

    uint32_t ach, bch;
    if constexpr (C::BD) {
        // The travelling operand skips LDS: each wave loads its own MFMA
        // fragments of B (the packed layout already is the fragment layout:
        // 32 lanes read 512 contiguous bytes of one plane) one stage ahead,
        // into one of two register sets.  Only the static blocks go
        // through LDS (two slots, loaded two stages ahead, written one
        // stage ahead, one barrier per stage), which halves the LDS writes
        // and cuts the LDS reads by a third.
        const int r32 = lane & 31, g = lane >> 5;
        const uint32_t b_lane = (uint32_t)((int64_t)g * BN * 16 + (int64_t)(wn * C::WN + r32) * 16);
        const uint32_t b_piece = (uint32_t)a.b_piece;
        typedef u32x4 BQ[CPS][C::NP][C::TN];
        auto load_b = [&](BQ &bq, uint32_t ch) {
            const uint32_t bst = ch * b_stage;
#pragma unroll
            for (int c = 0; c < CPS; ++c)
#pragma unroll
                for (int P = 0; P < C::NP; ++P)
#pragma unroll
                    for (int ni = 0; ni < C::TN; ++ni)
                        bq[c][P][ni] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                            rsB, (int)(b_lane + ni * 32 * 16), (int)(bst + P * b_piece + c * BN * C::CB), 0));
        };
        u32x4 r0s[C::UA], r1s[C::UA];
        BQ q0, q1;
        Pos pb = start;
        fetch_offsets(ach, bch);
        stage_load_a<C::UA>(r0s, rsA, a_off, ach);
        fetch_offsets(ach, bch);
        stage_load_a<C::UA>(r1s, rsA, a_off, ach);
        load_b(q0, next_chunk(pb));
        stage_store_a<C::UA, C::NT>(r0s, ring, tid);
        __syncthreads();
#define HS_PIPE_STEP(RLOAD, RSTORE, QUSE, QLOAD)                                               \
    {                                                                                          \
        const int slot = (int)(s & 1);                                                         \
        fetch_offsets(ach, bch);                                                               \
        stage_load_a<C::UA>(RLOAD, rsA, a_off, ach);                                           \
        load_b(QLOAD, next_chunk(pb));                                                         \
        stage_store_a<C::UA, C::NT>(RSTORE, ring + (slot ^ 1) * C::A_STAGE, tid);              \
        __builtin_amdgcn_sched_barrier(0);                                                     \
        mm_compute_bd<FAM, FORM, BM, BN, CPS, WAVES>(acc, ring + slot * C::A_STAGE, QUSE, lane, wm); \
        __syncthreads();                                                                       \
        if (++s >= nstages) break;                                                             \
    }
        for (int s = 0; s < nstages;) {
            HS_PIPE_STEP(r0s, r1s, q0, q1)
            HS_PIPE_STEP(r1s, r0s, q1, q0)
        }
#undef HS_PIPE_STEP
    } else if constexpr (C::W1) {
        // One wave per SIMD, so nothing else on the SIMD hides a wait: the
        // stage is laid out by hand.  Each LDS slot is a static array of
        // its own, which lets the compiler place the reads of one slot
        // between the writes to the other.  The one barrier per stage sits
        // before its last chunk: until then the wave multiplies chunk c
        // (fragments already in registers) while it reads chunk c + 1,
        // issues the loads of stage s + 2 and writes stage s + 1 (loaded a
        // stage earlier) into the other slot; after it the wave multiplies
        // the last chunk while it reads chunk 0 of stage s + 1 from the other
        // slot.  A slot is rewritten only after the barrier that follows its
        // last read.
        static_assert(CPS >= 2, "at least two chunks per stage");
        __shared__ __attribute__((aligned(16))) uint8_t slot0[C::STAGE];
        __shared__ __attribute__((aligned(16))) uint8_t slot1[C::STAGE];
        u32x4 r0s[C::LPS], r1s[C::LPS];
        const int r32 = lane & 31, g = lane >> 5;
        const int a_rd = g * BM * 16 + (wm * C::WM + r32) * 16;
        const int b_rd = C::A_STAGE + g * BN * 16 + (wn * C::WN + r32) * 16;
        u32x4 fa0[C::TM], fb0[C::TN], fa1[C::TM], fb1[C::TN];
        auto read_chunk = [&](const uint8_t *sl, int c, u32x4 (&fa)[C::TM], u32x4 (&fb)[C::TN]) {
#pragma unroll
            for (int ni = 0; ni < C::TN; ++ni) fb[ni] = *(const u32x4 *)(sl + b_rd + c * BN * C::CB + ni * 32 * 16);
#pragma unroll
            for (int mi = 0; mi < C::TM; ++mi) fa[mi] = *(const u32x4 *)(sl + a_rd + c * BM * C::CB + mi * 32 * 16);
        };
        auto mfma_chunk = [&](const u32x4 (&fa)[C::TM], const u32x4 (&fb)[C::TN]) {
#pragma unroll
            for (int mi = 0; mi < C::TM; ++mi) {
                u32x4 av[1] = {fa[mi]};
                u32x4 bv[1][C::TN];
#pragma unroll
                for (int ni = 0; ni < C::TN; ++ni) bv[0][ni] = fb[ni];
                mfma_row<FAM, FORM, C::TN>(acc[mi], av, bv);
            }
        };
        fetch_offsets(ach, bch);
        stage_load<C::UA, C::UB>(r0s, rsA, rsB, a_off, b_off, ach, bch);
        fetch_offsets(ach, bch);
        stage_load<C::UA, C::UB>(r1s, rsA, rsB, a_off, b_off, ach, bch);
        stage_store<C::UA, C::UB, C::A_STAGE, C::NT>(r0s, slot0, tid);
        __syncthreads();
        read_chunk(slot0, 0, fa0, fb0);
        // sched_group_barrier masks: 0x008 MFMA, 0x020 global load, 0x100
        // LDS read, 0x200 LDS write.  A chunk has W1_RD fragment reads and
        // W1_PER MFMAs per read (2 for BF16/FP16, 8 for FP32's 32x32x2).
        // Before the barrier, W1_SLOTS times: MFMA, read, (write), W1_PER - 1
        // MFMAs, (load), the LPS loads and writes on the first slots; after
        // it, W1_RD times: MFMA, read, W1_PER - 1 MFMAs.
        constexpr int W1_RD = C::TM + C::TN;
        constexpr int W1_PER = C::TM * C::TN * (FAM == FAM_F32 ? 4 : 1) / W1_RD;
        constexpr int W1_SLOTS = (CPS - 1) * W1_RD;          // reads before the barrier
        static_assert(C::LPS <= W1_SLOTS && W1_PER >= 2, "interleave pattern");
        // Before the barrier: chunks 0 .. CPS-2 (each while reading the next
        // chunk of this slot), the loads of stage s + 2 and the LDS writes of
        // stage s + 1 into the other slot.  After it: the last chunk, while
        // reading chunk 0 of stage s + 1 from the other slot.  Every read of
        // this slot precedes the barrier, so the next stage may rewrite it.
        auto first_part = [&](const uint8_t *X, uint8_t *Y, u32x4 (&RLOAD)[C::LPS], const u32x4 (&RSTORE)[C::LPS]) {
#pragma unroll
            for (int c = 0; c + 1 < CPS; ++c) {
                if (c % 2 == 0) { mfma_chunk(fa0, fb0); read_chunk(X, c + 1, fa1, fb1); }
                else { mfma_chunk(fa1, fb1); read_chunk(X, c + 1, fa0, fb0); }
            }
            stage_load<C::UA, C::UB>(RLOAD, rsA, rsB, a_off, b_off, ach, bch);
            stage_store<C::UA, C::UB, C::A_STAGE, C::NT>(RSTORE, Y, tid);
#pragma unroll
            for (int i = 0; i < W1_SLOTS; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                if (i < C::LPS) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, W1_PER - 1, 0);
                if (i < C::LPS) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
            }
        };
        auto last_part = [&](const uint8_t *Y) {
            if constexpr ((CPS - 1) % 2 == 0) { mfma_chunk(fa0, fb0); read_chunk(Y, 0, fa0, fb0); }
            else { mfma_chunk(fa1, fb1); read_chunk(Y, 0, fa0, fb0); }
#pragma unroll
            for (int i = 0; i < W1_RD; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, W1_PER - 1, 0);
            }
        };
#define HS_W1_STEP(X, Y, RLOAD, RSTORE)                                                        \
    {                                                                                          \
        fetch_offsets(ach, bch);                                                               \
        first_part(X, Y, RLOAD, RSTORE);                                                       \
        __syncthreads();                                                                       \
        last_part(Y);                                                                          \
        if (++s >= nstages) break;                                                             \
    }
        for (int s = 0; s < nstages;) {
            HS_W1_STEP(slot0, slot1, r0s, r1s)
            HS_W1_STEP(slot1, slot0, r1s, r0s)
        }
#undef HS_W1_STEP
    } else {
        // Both operands through LDS, two slots: the global loads for stage
        // s + 2 are issued at the top of stage s into one of two register
        // sets; the LDS image of stage s + 1 is written into the other slot
        // at the top of stage s, and one barrier closes each stage.
        u32x4 r0s[C::LPS], r1s[C::LPS];
        fetch_offsets(ach, bch);
        stage_load<C::UA, C::UB>(r0s, rsA, rsB, a_off, b_off, ach, bch);
        fetch_offsets(ach, bch);
        stage_load<C::UA, C::UB>(r1s, rsA, rsB, a_off, b_off, ach, bch);
        stage_store<C::UA, C::UB, C::A_STAGE, C::NT>(r0s, ring, tid);
        __syncthreads();
#define HS_PIPE_STEP(RLOAD, RSTORE)                                                            \
    {                                                                                          \
        const int slot = (int)(s & 1);                                                         \
        fetch_offsets(ach, bch);                                                               \
        stage_load<C::UA, C::UB>(RLOAD, rsA, rsB, a_off, b_off, ach, bch);                     \
        stage_store<C::UA, C::UB, C::A_STAGE, C::NT>(RSTORE, ring + (slot ^ 1) * C::STAGE, tid); \
        stage_scales();                                                                        \
        __builtin_amdgcn_sched_barrier(0);                                                     \
        mm_compute<FAM, FORM, BM, BN, CPS, WAVES>(acc, ring + slot * C::STAGE,                 \
                                           ring + slot * C::STAGE + C::A_STAGE, lane, wm, wn,  \
                                           sa, sb);                                            \
        __syncthreads();                                                                       \
        if (++s >= nstages) break;                                                             \
    }
        for (int s = 0; s < nstages;) {
            HS_PIPE_STEP(r0s, r1s)
            HS_PIPE_STEP(r1s, r0s)
        }
#undef HS_PIPE_STEP
    }

    // epilogue: the collector has absorbed every partial; tile row rho is
    // row msub MS + (rho mod MS) of stripe r0 + (rho / MS) K.  One tile row
    // at a time (row index computed once, then its columns).
    const int64_t S_r = a.S_r;
    constexpr int NE = (int)(sizeof(Acc) / sizeof(acc[0][0][0]));
    // two-piece FP16: the tile holds C' = sum a' b' of the scaled operands;
    // C = C' 2^-(e_row + e_col) (exact unless the result is subnormal)
    constexpr bool ROWSCALE = FAM == FAM_F16 && FORM == 2;
    int ecol[C::TN];
#pragma unroll
    for (int ni = 0; ni < C::TN; ++ni) {
        ecol[ni] = 0;
        if constexpr (ROWSCALE) {
            const int64_t col = ntile * BN + wn * C::WN + ni * C::MT + (lane & 31);
            if (col < a.N) ecol[ni] = row_scale_exp(((const uint32_t *)a.b_exps)[col]);
        }
    }
#pragma unroll
    for (int mi = 0; mi < C::TM; ++mi) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            int rho;
            if constexpr (FAM == FAM_F64)      // 16x16x4 f64: element e of lane -> row 4e + lane/16
                rho = wm * C::WM + mi * 16 + 4 * e + (lane >> 4);
            else                               // 32x32 f32 accumulators
                rho = wm * C::WM + mi * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
            const int i = rho / MS, ir = rho % MS;
            const int64_t within = msub * MS + ir;
            const int64_t row = (int64_t)(r0 + i * K) * S_r + within;
            const bool rok = i < ng && within < S_r && row < a.M;
            const int64_t cbase = ntile * BN + wn * C::WN + (FAM == FAM_F64 ? (lane & 15) : (lane & 31));
            int erow = 0;
            if constexpr (ROWSCALE) erow = rok ? row_scale_exp(((const uint32_t *)a.a_exps)[row]) : 0;
            // the element's destination: C, or plane `split` of a.part (rows of N)
            const bool to_part = a.nsplit > 1;
            const int64_t obase = to_part ? ((int64_t)split * a.M + row) * a.N + cbase : row * a.ldo + cbase;
            void *dst = to_part ? a.part : a.out;
#pragma unroll
            for (int ni = 0; ni < C::TN; ++ni) {
                const bool ok = rok && cbase + ni * C::MT < a.N;
                if (ok) {
                    if (a.out_f64) ((double *)dst)[obase + ni * C::MT] = (double)acc[mi][ni][e];
                    else if constexpr (ROWSCALE)
                        ((float *)dst)[obase + ni * C::MT] = ldexpf((float)acc[mi][ni][e], -(erow + ecol[ni]));
                    else ((float *)dst)[obase + ni * C::MT] = (float)acc[mi][ni][e];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// back-shift and accumulation (fixed order, FP64)
// ---------------------------------------------------------------------------
// Each thread sums 4 consecutive columns of one row over the K partial
// planes, c^{K-1} first: S = c^l + S for l = K-2 .. 0 (back-shift order).
// VEC: N % 4 == 0 (16-byte partial loads); VST: 16-byte stores into C legal.
template <typename PT, typename OT, int VEC, int VST>
__global__ __launch_bounds__(256) void backshift_kernel(const PT *W, int64_t plane, int K,
                                                        int64_t M, int64_t N, OT *Cout, int64_t ldc) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n4 = (N + 3) / 4;
    if (idx >= M * n4) return;
    const int64_t row = idx / n4, c0 = (idx % n4) * 4;
    const int cnt = (int)((N - c0) < 4 ? (N - c0) : 4);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int l = K - 1; l >= 0; --l) {
        const PT *wl = W + (int64_t)l * plane + row * N + c0;
        PT x[4];
        if constexpr (VEC && sizeof(PT) == 4) {
            const float4 v = *(const float4 *)wl;
            x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
        } else if constexpr (VEC) {
            const double2 v0 = *(const double2 *)wl, v1 = *(const double2 *)(wl + 2);
            x[0] = v0.x; x[1] = v0.y; x[2] = v1.x; x[3] = v1.y;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) x[e] = e < cnt ? wl[e] : (PT)0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) s[e] = (l == K - 1) ? (double)x[e] : (double)x[e] + s[e];
    }
    OT *c = Cout + row * ldc + c0;
    if constexpr (VST && sizeof(OT) == 4) {
        *(float4 *)c = make_float4((float)s[0], (float)s[1], (float)s[2], (float)s[3]);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (e < cnt) c[e] = (OT)s[e];
    }
}

template <typename OT>
__global__ __launch_bounds__(256) void fill_zero_kernel(OT *Cout, int64_t M, int64_t N, int64_t ldc) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= M * N) return;
    Cout[(idx / N) * ldc + idx % N] = (OT)0;
}

// ---------------------------------------------------------------------------
// matrix-vector product
// ---------------------------------------------------------------------------
template <typename T, int VE>
__global__ __launch_bounds__(256) void gemv_kernel(GemvArgs a) {
    typedef typename std::conditional<VE == 4, float4, typename std::conditional<VE == 2, double2, T>::type>::type V;
    constexpr int U = 4;                       // loads in flight per lane
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= a.m) return;
    const T *Ar = (const T *)a.A + row * a.lda;
    const T *x = (const T *)a.x;
    const int p = a.p, K = a.K;
    const int rs = (int)(row / a.S_r);
    const int S_k = (int)a.S_k;                // host: S_k * p fits in 32 bits
    const int total = a.Kt * S_k;
    double S = 0.0;
    for (int l = K - 1; l >= 0; --l) {         // collector: c^{K-1} first
        const int v = (rs + l) % p;            // the virtual processor holding partial l
        // lane position: element e of the partial's sequence lies in step
        // j = e / S_k (block kb = (v + j K) mod p) at offset e mod S_k
        int e = lane * VE, j = e / S_k, off = e % S_k;
        int kb = (int)(((int64_t)v + (int64_t)j * K) % p);
        auto advance = [&]() {
            e += 64 * VE;
            off += 64 * VE;
            while (off >= S_k) {
                off -= S_k;
                kb += K;
                if (kb >= p) kb -= p;
            }
        };
        T acc = 0;
        while (e < total) {
            V av[U], xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t col = (int64_t)kb * S_k + off;
                const bool ok = e < total && col < a.n;
                if (ok) {
                    av[u] = *(const V *)(Ar + col);
                    xv[u] = *(const V *)(x + col);
                } else {
                    av[u] = V{};
                    xv[u] = V{};
                }
                advance();
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if constexpr (VE == 4) {
                    acc += av[u].x * xv[u].x;
                    acc += av[u].y * xv[u].y;
                    acc += av[u].z * xv[u].z;
                    acc += av[u].w * xv[u].w;
                } else if constexpr (VE == 2) {
                    acc += av[u].x * xv[u].x;
                    acc += av[u].y * xv[u].y;
                } else {
                    acc += av[u] * xv[u];
                }
            }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
        S = (double)acc + S;
    }
    if (lane == 0) ((T *)a.y)[row] = (T)S;
}

// Complex y = A x (complex64, interleaved re/im): the map and collector
// order of gemv_kernel, positions in complex elements; each lane keeps the
// real and imaginary partial sums, combined in FP64 in the back-shift order.
// VE complex elements per load: 2 (16 bytes) or 1.
template <int VE>
__global__ __launch_bounds__(256) void gemv_c32_kernel(GemvArgs a) {
    typedef typename std::conditional<VE == 2, float4, float2>::type V;
    constexpr int U = 4;                       // loads in flight per lane
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= a.m) return;
    const float *Ar = (const float *)a.A + row * a.lda * 2;
    const float *x = (const float *)a.x;
    const int p = a.p, K = a.K;
    const int rs = (int)(row / a.S_r);
    const int S_k = (int)a.S_k;                // host: S_k * p fits in 32 bits
    const int total = a.Kt * S_k;
    double Sr = 0.0, Si = 0.0;
    for (int l = K - 1; l >= 0; --l) {         // collector: c^{K-1} first
        const int v = (rs + l) % p;
        int e = lane * VE, j = e / S_k, off = e % S_k;
        int kb = (int)(((int64_t)v + (int64_t)j * K) % p);
        auto advance = [&]() {
            e += 64 * VE;
            off += 64 * VE;
            while (off >= S_k) {
                off -= S_k;
                kb += K;
                if (kb >= p) kb -= p;
            }
        };
        float re = 0.f, im = 0.f;
        while (e < total) {
            V av[U], xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t col = (int64_t)kb * S_k + off;
                const bool ok = e < total && col < a.n;
                if (ok) {
                    av[u] = *(const V *)(Ar + 2 * col);
                    xv[u] = *(const V *)(x + 2 * col);
                } else {
                    av[u] = V{};
                    xv[u] = V{};
                }
                advance();
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                re = __builtin_fmaf(av[u].x, xv[u].x, re);
                re = __builtin_fmaf(-av[u].y, xv[u].y, re);
                im = __builtin_fmaf(av[u].x, xv[u].y, im);
                im = __builtin_fmaf(av[u].y, xv[u].x, im);
                if constexpr (VE == 2) {
                    re = __builtin_fmaf(av[u].z, xv[u].z, re);
                    re = __builtin_fmaf(-av[u].w, xv[u].w, re);
                    im = __builtin_fmaf(av[u].z, xv[u].w, im);
                    im = __builtin_fmaf(av[u].w, xv[u].z, im);
                }
            }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            re += __shfl_xor(re, m, 64);
            im += __shfl_xor(im, m, 64);
        }
        Sr = (double)re + Sr;
        Si = (double)im + Si;
    }
    if (lane == 0) ((float2 *)a.y)[row] = make_float2((float)Sr, (float)Si);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblocks(int64_t work) { return (unsigned)((work + 255) / 256); }

// Events of the next timed launch (hs_profile_begin / hs_profile_end): the
// dispatch itself records them (hipExtLaunchKernel), so they bracket the
// kernel's execution alone, without the gaps that separate event records
// add around a short kernel.
static hipEvent_t g_timed_start = nullptr, g_timed_stop = nullptr;
static bool g_timed_used = false;
void set_timed_launch(hipEvent_t start, hipEvent_t stop) {
    g_timed_start = start;
    g_timed_stop = stop;
    g_timed_used = false;
}
bool take_timed_launch(hipEvent_t *start, hipEvent_t *stop) {
    if (!g_timed_start) return false;
    *start = g_timed_start;
    *stop = g_timed_stop;
    g_timed_start = g_timed_stop = nullptr;
    g_timed_used = true;
    return true;
}
// true if the events set last were taken by a launch; clears them
bool timed_launch_done() {
    const bool used = g_timed_used;
    g_timed_start = g_timed_stop = nullptr;
    g_timed_used = false;
    return used;
}
#define HS_LAUNCH_TIMED(KERNEL, GRID, BLOCK, SHM, ST, ...)                                    \
    do {                                                                                     \
        hipEvent_t ts_, te_;                                                                 \
        if (take_timed_launch(&ts_, &te_))                                                   \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, ST, ts_, te_, 0, __VA_ARGS__);   \
        else                                                                                 \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, ST, __VA_ARGS__);                   \
    } while (0)

hipError_t launch_pack(int kind, int kmajor, const PackArgs &a, hipStream_t st) {
    if (a.total_units == 0) return hipSuccess;
    const unsigned nb = nblocks(a.total_units);
#define HS_PACK(K_, M_) hipLaunchKernelGGL((pack_kernel<K_, M_>), dim3(nb), dim3(256), 0, st, a)
    switch (kind * 2 + (kmajor ? 1 : 0)) {
        case PK_F64 * 2: HS_PACK(PK_F64, 0); break;
        case PK_F64 * 2 + 1: HS_PACK(PK_F64, 1); break;
        case PK_F32 * 2: HS_PACK(PK_F32, 0); break;
        case PK_F32 * 2 + 1: HS_PACK(PK_F32, 1); break;
        case PK_B16 * 2: HS_PACK(PK_B16, 0); break;
        case PK_B16 * 2 + 1: HS_PACK(PK_B16, 1); break;
        case PK_SPLIT3 * 2: HS_PACK(PK_SPLIT3, 0); break;
        case PK_SPLIT3 * 2 + 1: HS_PACK(PK_SPLIT3, 1); break;
        case PK_FP8 * 2: HS_PACK(PK_FP8, 0); break;
        case PK_FP8 * 2 + 1: HS_PACK(PK_FP8, 1); break;
        case PK_SPLIT2F16 * 2: HS_PACK(PK_SPLIT2F16, 0); break;
        case PK_SPLIT2F16 * 2 + 1: HS_PACK(PK_SPLIT2F16, 1); break;
        default: return hipErrorInvalidValue;
    }
#undef HS_PACK
    return hipGetLastError();
}

template <int FAM, int FORM, int BM, int BN, int CPS, int WAVES>
static hipError_t launch_mm_t(const MainArgs &a, hipStream_t st) {
    typedef MmCfg<FAM, FORM, BM, BN, CPS, WAVES> C;
    // the dynamic LDS limit is a per-device function attribute: set it once
    // on each device the kernel runs on (setting it twice is harmless)
    static bool attr_set[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    if (dev < 0 || dev >= 64 || !attr_set[dev]) {
        hipError_t e = hipFuncSetAttribute((const void *)mm_kernel<FAM, FORM, BM, BN, CPS, WAVES>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS_BYTES);
        if (e != hipSuccess) return e;
        if (dev >= 0 && dev < 64) attr_set[dev] = true;
    }
    const int64_t nwg = (int64_t)a.K * a.n_ug * a.n_tg * a.grp_v * a.grp_t * a.nsplit;
    HS_LAUNCH_TIMED((mm_kernel<FAM, FORM, BM, BN, CPS, WAVES>), dim3((unsigned)nwg), dim3(C::NT), C::LDS_BYTES, st, a);
    return hipGetLastError();
}

// Tile shapes per family: rows of the workgroup tile (K groups of MS rows),
// columns, and chunks per pipeline stage.
int mm_tile_rows(int fam) { return fam == FAM_F64 ? 64 : 256; }
int mm_tile_cols(int fam) { return fam == FAM_F64 ? 64 : 256; }
int mm_chunks_per_stage(int fam, int form) {
    if (fam == FAM_F64) return 4;
    if (fam == FAM_FP8) return form == 1 ? 1 : 2;
    if (fam == FAM_F32) return 2;
    // split forms one 16-deep chunk per stage (split-BF16: 48 MFMAs per wave;
    // two-piece FP16: 24, measured 2.45 ms against 2.60 with two chunks at
    // n = 8192), BF16 and FP16 four (64 per wave; 0.915 against 0.934 ms for
    // BF16 with two at n = 8192)
    return form == 1 || form == 2 ? 1 : 4;
}

// 8 waves (2 per SIMD) for the split forms' and FP8's 256 x 256 tiles, 4
// (one per SIMD) for FP32, plain BF16 and FP16 (measured at n = 8192 on
// one box against 8 waves: FP32 7.33 against 7.61 ms, BF16 0.930 against
// 0.970 ms, FP16 0.970 against 1.008 ms, with two chunks per stage) and for
// FP64's 64 x 64.
hipError_t launch_mm(int fam, int form, const MainArgs &a, hipStream_t st) {
    if (fam == FAM_F64) return launch_mm_t<FAM_F64, 0, 64, 64, 4, 4>(a, st);
    if (fam == FAM_F32) return launch_mm_t<FAM_F32, 0, 256, 256, 2, 4>(a, st);
    if (fam == FAM_F16 && form == 0) return launch_mm_t<FAM_F16, 0, 256, 256, 4, 4>(a, st);
    if (fam == FAM_F16 && form == 2) return launch_mm_t<FAM_F16, 2, 256, 256, 1, 8>(a, st);
    if (fam == FAM_BF16 && form == 0) return launch_mm_t<FAM_BF16, 0, 256, 256, 4, 4>(a, st);
    if (fam == FAM_BF16 && form == 1) return launch_mm_t<FAM_BF16, 1, 256, 256, 1, 8>(a, st);
    if (fam == FAM_FP8 && form == 0) return launch_mm_t<FAM_FP8, 0, 256, 256, 2, 8>(a, st);
    if (fam == FAM_FP8 && form == 1) return launch_mm_t<FAM_FP8, 1, 256, 256, 1, 8>(a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_pack_mn(int kind, const PackArgs &a, hipStream_t st) {
    if (a.total_units == 0) return hipSuccess;
    const unsigned nb = nblocks(a.total_units);
    switch (kind) {
        case PK_F32: hipLaunchKernelGGL((pack_mn_kernel<PK_F32>), dim3(nb), dim3(256), 0, st, a); break;
        case PK_SPLIT3: hipLaunchKernelGGL((pack_mn_kernel<PK_SPLIT3>), dim3(nb), dim3(256), 0, st, a); break;
        case PK_FP8: hipLaunchKernelGGL((pack_mn_kernel<PK_FP8>), dim3(nb), dim3(256), 0, st, a); break;
        case PK_SPLIT2F16: hipLaunchKernelGGL((pack_mn_kernel<PK_SPLIT2F16>), dim3(nb), dim3(256), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fill_zero(int f64, void *Cout, int64_t M, int64_t N, int64_t ldc, hipStream_t st);

hipError_t launch_row_amax(const RowAmaxArgs &a, hipStream_t st) {
    if (a.R == 0) return hipSuccess;
    const bool vec = a.ld % 4 == 0 && ((uintptr_t)a.src % 16) == 0;
    if (a.kmajor) {
        const dim3 grid((unsigned)((a.R + 3) / 4));
        if (vec) hipLaunchKernelGGL(row_amax_k_kernel<1>, grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL(row_amax_k_kernel<0>, grid, dim3(256), 0, st, a);
        return hipGetLastError();
    }
    hipError_t e = launch_fill_zero(0, a.amax, 1, a.R, a.R, st);   // zero bits = 0.0f
    if (e != hipSuccess || a.Kd == 0) return e;
    // the float view (see RowAmaxArgs); R Kd < 2^34 (the packing limit), so blocks < 2^19
    const int64_t ncol = (a.embed == EMB_TRANS || a.embed == EMB_CONJ) ? 2 * a.R : a.R;
    const int64_t nk = a.embed == EMB_NONE ? a.Kd : a.Kd / 2;
    const int64_t slabs = (nk + 255) / 256;
    if (vec) hipLaunchKernelGGL(row_amax_mn_kernel<1>, dim3((unsigned)((ncol + 1023) / 1024 * slabs)), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(row_amax_mn_kernel<0>, dim3((unsigned)((ncol + 255) / 256 * slabs)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fp8_exps(const Fp8ExpArgs &a, int64_t tiles, hipStream_t st) {
    if (tiles == 0) return hipSuccess;
    const bool vec = a.ld % 4 == 0 && ((uintptr_t)a.src % 16) == 0;
    if (vec) hipLaunchKernelGGL(fp8_tile_exp_kernel<1>, dim3((unsigned)tiles), dim3(512), 0, st, a);
    else hipLaunchKernelGGL(fp8_tile_exp_kernel<0>, dim3((unsigned)tiles), dim3(512), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_backshift(int f64, const void *W, int64_t plane, int K, int64_t M, int64_t N,
                            void *Cout, int64_t ldc, hipStream_t st) {
    const int64_t work = M * ((N + 3) / 4);
    if (work == 0) return hipSuccess;
    const bool vec = N % 4 == 0;
    const bool vst = vec && ldc % 4 == 0 && ((uintptr_t)Cout % 16) == 0;
    const dim3 grid(nblocks(work)), block(256);
    if (f64) {
        if (vec) hipLaunchKernelGGL((backshift_kernel<double, double, 1, 0>), grid, block, 0, st,
                                    (const double *)W, plane, K, M, N, (double *)Cout, ldc);
        else hipLaunchKernelGGL((backshift_kernel<double, double, 0, 0>), grid, block, 0, st,
                                (const double *)W, plane, K, M, N, (double *)Cout, ldc);
    } else {
        if (vst) hipLaunchKernelGGL((backshift_kernel<float, float, 1, 1>), grid, block, 0, st,
                                    (const float *)W, plane, K, M, N, (float *)Cout, ldc);
        else if (vec) hipLaunchKernelGGL((backshift_kernel<float, float, 1, 0>), grid, block, 0, st,
                                         (const float *)W, plane, K, M, N, (float *)Cout, ldc);
        else hipLaunchKernelGGL((backshift_kernel<float, float, 0, 0>), grid, block, 0, st,
                                (const float *)W, plane, K, M, N, (float *)Cout, ldc);
    }
    return hipGetLastError();
}

hipError_t launch_fill_zero(int f64, void *Cout, int64_t M, int64_t N, int64_t ldc, hipStream_t st) {
    if (M * N == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL((fill_zero_kernel<double>), dim3(nblocks(M * N)), dim3(256), 0, st, (double *)Cout, M, N, ldc);
    else
        hipLaunchKernelGGL((fill_zero_kernel<float>), dim3(nblocks(M * N)), dim3(256), 0, st, (float *)Cout, M, N, ldc);
    return hipGetLastError();
}

hipError_t launch_gemv(int f64, const GemvArgs &a, hipStream_t st) {
    const unsigned nb = (unsigned)((a.m + 3) / 4);
    if (nb == 0) return hipSuccess;
    if (a.cplx) {
        if (a.vec) HS_LAUNCH_TIMED((gemv_c32_kernel<2>), dim3(nb), dim3(256), 0, st, a);
        else HS_LAUNCH_TIMED((gemv_c32_kernel<1>), dim3(nb), dim3(256), 0, st, a);
    } else if (f64) {
        if (a.vec) HS_LAUNCH_TIMED((gemv_kernel<double, 2>), dim3(nb), dim3(256), 0, st, a);
        else HS_LAUNCH_TIMED((gemv_kernel<double, 1>), dim3(nb), dim3(256), 0, st, a);
    } else {
        if (a.vec) HS_LAUNCH_TIMED((gemv_kernel<float, 4>), dim3(nb), dim3(256), 0, st, a);
        else HS_LAUNCH_TIMED((gemv_kernel<float, 1>), dim3(nb), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace hs
