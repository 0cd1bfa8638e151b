// hs_kernels.hip -- HIP kernels for gfx950 (CDNA4) implementing the
// hyper-systolic matrix product (Sec. 5.2.2, Algorithm HYPER-SYSTOLIC) on one
// GPU, with p virtual processors realised as groups of workgroups.
//
// Kernels
//   pack_kernel      operand preparation: copies (or splits, or quantises) a
//                    row-major operand into the packed tile layout described
//                    in hs_internal.h; HBM bound.
//   mm_kernel        the hot loop: one workgroup is virtual processor v for
//                    one (stripe sub-group, column tile).  For step j it
//                    fetches block kb = (v + jK) mod p of the travelling
//                    operand (base A = (0,K,..,K)) through a double-buffered
//                    LDS ring and multiplies it, on MFMA, with the K static
//                    blocks of stripes v, v-1, .., v-K+1 (pre-shift base
//                    B = (0,-1,..,-1)) into K partial accumulators (the
//                    auxiliary arrays C^l of Sec. 5.2.2).
//   backshift_kernel the back-shift and accumulation phase (base
//                    C = (0,1,..,1)): C[r] = c^0_r + (c^1_{r+1} + (..)), in
//                    FP64, fixed order.
//   gemv_kernel      y = A x with the same index map, collector form: one
//                    wave owns a row and combines the K partial dot products
//                    in the back-shift order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hs_internal.h"

namespace hs {

#define DEVI __device__ __forceinline__

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// number formats
// ---------------------------------------------------------------------------
// float -> bfloat16, round to nearest, ties to even; NaN stays NaN.
DEVI uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
DEVI float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// pack
// ---------------------------------------------------------------------------
template <int KIND> struct PackTraits;
template <> struct PackTraits<PK_F64> { typedef double S; static const int UE = 2; static const int ESZ = 8; static const int NP = 1; };
template <> struct PackTraits<PK_F32> { typedef float S; static const int UE = 4; static const int ESZ = 4; static const int NP = 1; };
template <> struct PackTraits<PK_B16> { typedef uint16_t S; static const int UE = 8; static const int ESZ = 2; static const int NP = 1; };
template <> struct PackTraits<PK_SPLIT3> { typedef float S; static const int UE = 8; static const int ESZ = 2; static const int NP = 3; };

template <int KIND, int KMAJOR>
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a) {
    typedef PackTraits<KIND> T;
    typedef typename T::S S;
    const OperandGeom &g = a.g;
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u >= a.total_units) return;
    const int KC = g.chunk_bytes / T::ESZ;      // elements per chunk row
    const int UPR = g.chunk_bytes / 16;         // 16-byte units per chunk row
    const int64_t nch = g.nch, p = g.p, gr = g.grp_rows;
    int64_t t, rr, half, ch, kb, grp;
    if (KMAJOR) {   // consecutive threads walk along the contraction of one row
        half = u % UPR; t = u / UPR;
        ch = t % nch;   t /= nch;
        kb = t % p;     t /= p;
        rr = t % gr;    grp = t / gr;
    } else {        // consecutive threads walk along the rows
        rr = u % gr;    t = u / gr;
        half = t % UPR; t /= UPR;
        ch = t % nch;   t /= nch;
        kb = t % p;     grp = t / p;
    }
    int64_t row;
    bool rvalid;
    if (g.striped) {
        const int64_t stripe = grp / g.GS, msub = grp % g.GS;
        const int64_t within = msub * gr + rr;
        row = stripe * g.S_r + within;
        rvalid = within < g.S_r && row < g.R;
    } else {
        row = grp * gr + rr;
        rvalid = row < g.R;
    }
    const int64_t kin0 = ch * KC + half * T::UE;
    const S *src = (const S *)a.src;
    float vals_f[T::UE];
    double vals_d[T::UE];
    uint16_t vals_h[T::UE];
#pragma unroll
    for (int e = 0; e < T::UE; ++e) {
        const int64_t kin = kin0 + e;
        const int64_t kk = kb * g.S_k + kin;
        const bool ok = rvalid && kin < g.S_k && kk < g.Kd;
        const int64_t idx = KMAJOR ? row * a.ld + kk : kk * a.ld + row;
        if constexpr (KIND == PK_F64) vals_d[e] = ok ? (double)src[idx] : 0.0;
        else if constexpr (KIND == PK_B16) vals_h[e] = ok ? (uint16_t)src[idx] : (uint16_t)0;
        else vals_f[e] = ok ? (float)src[idx] : 0.0f;
    }
    const int64_t off = (((grp * p + kb) * nch + ch) * gr + rr) * g.chunk_bytes + half * 16;
    uint8_t *dst = (uint8_t *)a.dst + off;
    if constexpr (KIND == PK_F64) {
        *(double2 *)dst = make_double2(vals_d[0], vals_d[1]);
    } else if constexpr (KIND == PK_F32) {
        *(float4 *)dst = make_float4(vals_f[0], vals_f[1], vals_f[2], vals_f[3]);
    } else if constexpr (KIND == PK_B16) {
        uint4 w;
        w.x = vals_h[0] | ((uint32_t)vals_h[1] << 16);
        w.y = vals_h[2] | ((uint32_t)vals_h[3] << 16);
        w.z = vals_h[4] | ((uint32_t)vals_h[5] << 16);
        w.w = vals_h[6] | ((uint32_t)vals_h[7] << 16);
        *(uint4 *)dst = w;
    } else {   // PK_SPLIT3: a0 = bf16(a), a1 = bf16(a - a0), a2 = bf16(a - a0 - a1)
        uint16_t p0[8], p1[8], p2[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float x = vals_f[e];
            p0[e] = f32_to_bf16_rne(x);
            const float r1 = x - bf16_to_f32(p0[e]);      // exact in fp32
            p1[e] = f32_to_bf16_rne(r1);
            const float r2 = r1 - bf16_to_f32(p1[e]);     // exact in fp32
            p2[e] = f32_to_bf16_rne(r2);
        }
        uint16_t *pc[3] = {p0, p1, p2};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const uint16_t *h = pc[q];
            uint4 w;
            w.x = h[0] | ((uint32_t)h[1] << 16);
            w.y = h[2] | ((uint32_t)h[3] << 16);
            w.z = h[4] | ((uint32_t)h[5] << 16);
            w.w = h[6] | ((uint32_t)h[7] << 16);
            *(uint4 *)(dst + q * g.piece_bytes) = w;
        }
    }
}

// ---------------------------------------------------------------------------
// the hyper-systolic main loop on MFMA
// ---------------------------------------------------------------------------
// FORM 0: one piece per operand, one product.  FORM 1: three bf16 pieces,
// the six products a_i b_j with i + j <= 2, smallest first.
template <int FORM> struct Form;
template <> struct Form<0> { static const int NP = 1; static const int NPROD = 1; };
template <> struct Form<1> { static const int NP = 3; static const int NPROD = 6; };

template <int FAM> struct Mfma;
template <> struct Mfma<FAM_F64> { static const int T = 16; typedef f64x4 Acc; };
template <> struct Mfma<FAM_F32> { static const int T = 32; typedef f32x16 Acc; };
template <> struct Mfma<FAM_BF16> { static const int T = 32; typedef f32x16 Acc; };
template <> struct Mfma<FAM_F16> { static const int T = 32; typedef f32x16 Acc; };

template <int FAM, int FORM, int BM, int BN, int CPS>
struct MmCfg {
    static const int NP = Form<FORM>::NP;
    static const int CB = 32;                           // bytes per chunk row
    static const int A_STAGE = NP * CPS * BM * CB;      // LDS bytes per stage
    static const int B_STAGE = NP * CPS * BN * CB;
    static const int UA = NP * CPS * BM * 2 / 256;      // 16-byte loads per thread
    static const int UB = NP * CPS * BN * 2 / 256;
    static const int WM = BM / 2, WN = BN / 2;          // 2 x 2 waves
    static const int MT = Mfma<FAM>::T;
    static const int TM = WM / MT, TN = WN / MT;
    static const int LDS = 2 * (A_STAGE + B_STAGE);
};

// One pipeline stage of block products from LDS: for every chunk of the
// stage, the wave's MFMA tiles accumulate A_rows x B_cols.
template <int FAM, int FORM, int BM, int BN, int CPS, typename AccArr>
DEVI void mm_compute(AccArr &acc, const uint8_t *Ab, const uint8_t *Bb, int lane, int wm, int wn) {
    typedef MmCfg<FAM, FORM, BM, BN, CPS> C;
#pragma unroll
    for (int c = 0; c < CPS; ++c) {
        if constexpr (FAM == FAM_F64) {
            const int r16 = lane & 15, g = lane >> 4;
            double av[C::TM], bv[C::TN];
#pragma unroll
            for (int mi = 0; mi < C::TM; ++mi)
                av[mi] = *(const double *)(Ab + (c * BM + wm * C::WM + mi * 16 + r16) * C::CB + g * 8);
#pragma unroll
            for (int ni = 0; ni < C::TN; ++ni)
                bv[ni] = *(const double *)(Bb + (c * BN + wn * C::WN + ni * 16 + r16) * C::CB + g * 8);
#pragma unroll
            for (int mi = 0; mi < C::TM; ++mi)
#pragma unroll
                for (int ni = 0; ni < C::TN; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mi], bv[ni], acc[mi][ni], 0, 0, 0);
        } else {
            const int r32 = lane & 31, g = lane >> 5;
            uint4 av[C::NP][C::TM], bv[C::NP][C::TN];
#pragma unroll
            for (int P = 0; P < C::NP; ++P) {
#pragma unroll
                for (int mi = 0; mi < C::TM; ++mi)
                    av[P][mi] = *(const uint4 *)(Ab + ((P * CPS + c) * BM + wm * C::WM + mi * 32 + r32) * C::CB + g * 16);
#pragma unroll
                for (int ni = 0; ni < C::TN; ++ni)
                    bv[P][ni] = *(const uint4 *)(Bb + ((P * CPS + c) * BN + wn * C::WN + ni * 32 + r32) * C::CB + g * 16);
            }
#pragma unroll
            for (int mi = 0; mi < C::TM; ++mi)
#pragma unroll
                for (int ni = 0; ni < C::TN; ++ni) {
                    if constexpr (FAM == FAM_F32) {
                        // lane group g holds contraction elements 4g..4g+3 of
                        // the chunk; MFMA t takes element t of A and B alike
                        const float4 x = __builtin_bit_cast(float4, av[0][mi]);
                        const float4 y = __builtin_bit_cast(float4, bv[0][ni]);
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(x.x, y.x, acc[mi][ni], 0, 0, 0);
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(x.y, y.y, acc[mi][ni], 0, 0, 0);
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(x.z, y.z, acc[mi][ni], 0, 0, 0);
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(x.w, y.w, acc[mi][ni], 0, 0, 0);
                    } else if constexpr (FAM == FAM_F16) {
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(f16x8, av[0][mi]), __builtin_bit_cast(f16x8, bv[0][ni]), acc[mi][ni], 0, 0, 0);
                    } else if constexpr (FORM == 0) {
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, av[0][mi]), __builtin_bit_cast(bf16x8, bv[0][ni]), acc[mi][ni], 0, 0, 0);
                    } else {
                        // a2 b0, a1 b1, a0 b2, a1 b0, a0 b1, a0 b0: smallest first
#pragma unroll
                        for (int q = 0; q < 6; ++q) {
                            const int pa = q < 3 ? 2 - q : (q == 3 ? 1 : 0);
                            const int pb = q < 3 ? q : (q == 4 ? 1 : 0);
                            acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, av[pa][mi]), __builtin_bit_cast(bf16x8, bv[pb][ni]), acc[mi][ni], 0, 0, 0);
                        }
                    }
                }
        }
    }
}

// Global -> registers for one stage: the travelling block kb held at step j
// and the K static blocks of the same contraction range.
template <int UA, int UB>
DEVI void mm_load(uint4 (&ra)[UA], uint4 (&rb)[UB], const uint8_t *A, const uint8_t *B,
                  const int64_t (&a_off)[UA], const int64_t (&b_off)[UB], int64_t ach, int64_t bch) {
#pragma unroll
    for (int q = 0; q < UA; ++q) ra[q] = *(const uint4 *)(A + (a_off[q] >= 0 ? a_off[q] + ach : 0));
#pragma unroll
    for (int q = 0; q < UB; ++q) rb[q] = *(const uint4 *)(B + b_off[q] + bch);
}

template <int UA, int UB>
DEVI void mm_store(const uint4 (&ra)[UA], const uint4 (&rb)[UB], uint8_t *As, uint8_t *Bs, int tid) {
#pragma unroll
    for (int q = 0; q < UA; ++q) *(uint4 *)(As + (tid + 256 * q) * 16) = ra[q];
#pragma unroll
    for (int q = 0; q < UB; ++q) *(uint4 *)(Bs + (tid + 256 * q) * 16) = rb[q];
}

template <int FAM, int FORM, int BM, int BN, int CPS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void mm_kernel(MainArgs a) {
    typedef MmCfg<FAM, FORM, BM, BN, CPS> C;
    typedef typename Mfma<FAM>::Acc Acc;
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    uint8_t *As = smem;
    uint8_t *Bs = smem + 2 * C::A_STAGE;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    // workgroup -> (virtual processor v, stripe sub-group msub, column tile)
    int64_t bid = blockIdx.x;
    const int64_t ntile = bid % a.n_ntiles;
    bid /= a.n_ntiles;
    const int64_t msub = bid % a.GS;
    const int v = (int)(bid / a.GS);

    const int p = a.p, K = a.K, MS = a.MS;
    const int64_t nch = a.nch;
    const int64_t SPB = nch / CPS;            // stages per contraction block
    const int64_t nstages = (int64_t)a.Kt * SPB;

    // per-thread load descriptors: byte offsets that do not depend on the
    // step (group of the static operand, row, half-row, piece, chunk).  Units
    // past the K groups (only when K * MS < BM) re-read offset 0: their tile
    // rows are never stored.
    int64_t a_off[C::UA];
#pragma unroll
    for (int q = 0; q < C::UA; ++q) {
        const int ui = tid + 256 * q;
        const int slab = ui / (BM * 2);
        const int within = ui % (BM * 2);
        const int rho = within >> 1, half = within & 1;
        const int P = slab / CPS, c = slab % CPS;
        const int l = rho / MS, i = rho % MS;
        const int64_t grp = (int64_t)((v - l + p) % p) * a.GS + msub;
        a_off[q] = l < K ? (int64_t)P * a.a_piece + grp * (int64_t)p * nch * MS * C::CB +
                               (int64_t)c * MS * C::CB + (int64_t)i * C::CB + half * 16
                         : (int64_t)-1;
    }
    int64_t b_off[C::UB];
#pragma unroll
    for (int q = 0; q < C::UB; ++q) {
        const int ui = tid + 256 * q;
        const int slab = ui / (BN * 2);
        const int within = ui % (BN * 2);
        const int P = slab / CPS, c = slab % CPS;
        b_off[q] = (int64_t)P * a.b_piece + ntile * (int64_t)p * nch * BN * C::CB +
                   (int64_t)c * BN * C::CB + (int64_t)within * 16;
    }
    // Stage position: step j holds travelling block kb = (v + jK) mod p
    // (base A = (0, K, .., K)); cs counts the stages inside that block.
    int kb = v, cs = 0;
    const int spb = (int)SPB;

    Acc acc[C::TM][C::TN];
#pragma unroll
    for (int mi = 0; mi < C::TM; ++mi)
#pragma unroll
        for (int ni = 0; ni < C::TN; ++ni) acc[mi][ni] = Acc{};

    uint4 ra[C::UA], rb[C::UB];
    {
        const int64_t ch = (int64_t)kb * nch + cs * CPS;
        mm_load<C::UA, C::UB>(ra, rb, a.A, a.B, a_off, b_off, ch * MS * C::CB, ch * BN * C::CB);
        mm_store<C::UA, C::UB>(ra, rb, As, Bs, tid);
    }
    __syncthreads();

    for (int64_t s = 0; s + 1 < nstages; ++s) {
        const int buf = (int)(s & 1);
        if (++cs == spb) {           // next step: shift by K along the ring
            cs = 0;
            kb += K;
            if (kb >= p) kb -= p;
        }
        const int64_t ch = (int64_t)kb * nch + cs * CPS;
        mm_load<C::UA, C::UB>(ra, rb, a.A, a.B, a_off, b_off, ch * MS * C::CB, ch * BN * C::CB);
        mm_compute<FAM, FORM, BM, BN, CPS>(acc, As + buf * C::A_STAGE, Bs + buf * C::B_STAGE, lane, wm, wn);
        mm_store<C::UA, C::UB>(ra, rb, As + (buf ^ 1) * C::A_STAGE, Bs + (buf ^ 1) * C::B_STAGE, tid);
        __syncthreads();
    }
    {
        const int buf = (int)((nstages - 1) & 1);
        mm_compute<FAM, FORM, BM, BN, CPS>(acc, As + buf * C::A_STAGE, Bs + buf * C::B_STAGE, lane, wm, wn);
    }

    // epilogue: partial l of the tile row rho goes to output stripe (v - l).
    // One tile row at a time (row index computed once, then its columns).
    const int64_t S_r = a.S_r;
    constexpr int NE = (int)(sizeof(Acc) / sizeof(acc[0][0][0]));
#pragma unroll
    for (int mi = 0; mi < C::TM; ++mi) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            int rho;
            if constexpr (FAM == FAM_F64)      // 16x16x4 f64: element e of lane -> row 4e + lane/16
                rho = wm * C::WM + mi * 16 + 4 * e + (lane >> 4);
            else                               // 32x32 f32 accumulators
                rho = wm * C::WM + mi * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
            const int l = rho / MS, i = rho % MS;
            const int64_t within = msub * MS + i;
            const int64_t row = (int64_t)((v - l + p) % p) * S_r + within;
            const bool rok = l < K && within < S_r && row < a.M;
            const int64_t obase = (int64_t)l * a.plane + row * a.ldo + ntile * BN + wn * C::WN +
                                  (FAM == FAM_F64 ? (lane & 15) : (lane & 31));
            const int64_t cbase = ntile * BN + wn * C::WN + (FAM == FAM_F64 ? (lane & 15) : (lane & 31));
#pragma unroll
            for (int ni = 0; ni < C::TN; ++ni) {
                const bool ok = rok && cbase + ni * C::MT < a.N;
                if (ok) {
                    if (a.out_f64) ((double *)a.out)[obase + ni * C::MT] = (double)acc[mi][ni][e];
                    else ((float *)a.out)[obase + ni * C::MT] = (float)acc[mi][ni][e];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// back-shift and accumulation (fixed order, FP64)
// ---------------------------------------------------------------------------
template <typename PT, typename OT>
__global__ __launch_bounds__(256) void backshift_kernel(const PT *W, int64_t plane, int K,
                                                        int64_t M, int64_t N, OT *Cout, int64_t ldc) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n4 = (N + 3) / 4;
    if (idx >= M * n4) return;
    const int64_t row = idx / n4, c0 = (idx % n4) * 4;
    const int cnt = (int)((N - c0) < 4 ? (N - c0) : 4);
    double s[4];
    const PT *w = W + (int64_t)(K - 1) * plane + row * N + c0;
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] = e < cnt ? (double)w[e] : 0.0;
    for (int l = K - 2; l >= 0; --l) {       // c^l + (c^{l+1} + ...)
        const PT *wl = W + (int64_t)l * plane + row * N + c0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (e < cnt) s[e] = (double)wl[e] + s[e];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (e < cnt) Cout[row * ldc + c0 + e] = (OT)s[e];
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
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= a.m) return;
    const T *Ar = (const T *)a.A + row * a.lda;
    const T *x = (const T *)a.x;
    const int64_t rs = row / a.S_r;
    const int64_t S_k = a.S_k;
    const int64_t total = (int64_t)a.Kt * S_k;
    double S = 0.0;
    for (int l = a.K - 1; l >= 0; --l) {      // collector: c^{K-1} first
        const int64_t v = (rs + l) % a.p;      // the virtual processor holding partial l
        T acc = 0;
        int64_t e0 = (int64_t)lane * VE;
        int64_t j = e0 / S_k, off = e0 % S_k;
        for (int64_t e = e0; e < total; e += 64 * VE) {
            const int64_t kb = (v + j * a.K) % a.p;   // block held at step j
            const int64_t col = kb * S_k + off;
            if (col < a.n) {
                if constexpr (VE == 4) {
                    const float4 av = *(const float4 *)(Ar + col);
                    const float4 xv = *(const float4 *)(x + col);
                    acc += av.x * xv.x;
                    acc += av.y * xv.y;
                    acc += av.z * xv.z;
                    acc += av.w * xv.w;
                } else if constexpr (VE == 2) {
                    const double2 av = *(const double2 *)(Ar + col);
                    const double2 xv = *(const double2 *)(x + col);
                    acc += av.x * xv.x;
                    acc += av.y * xv.y;
                } else {
                    acc += Ar[col] * x[col];
                }
            }
            off += 64 * VE;
            while (off >= S_k) { off -= S_k; ++j; }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
        S = (double)acc + S;
    }
    if (lane == 0) ((T *)a.y)[row] = (T)S;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblocks(int64_t work) { return (unsigned)((work + 255) / 256); }

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
        default: return hipErrorInvalidValue;
    }
#undef HS_PACK
    return hipGetLastError();
}

template <int FAM, int FORM, int BM, int BN, int CPS>
static hipError_t launch_mm_t(const MainArgs &a, hipStream_t st) {
    typedef MmCfg<FAM, FORM, BM, BN, CPS> C;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)mm_kernel<FAM, FORM, BM, BN, CPS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t nwg = (int64_t)a.p * a.GS * a.n_ntiles;
    hipLaunchKernelGGL((mm_kernel<FAM, FORM, BM, BN, CPS>), dim3((unsigned)nwg), dim3(256), C::LDS, st, a);
    return hipGetLastError();
}

// Tile shapes per family: rows of the workgroup tile (K groups of MS rows),
// columns, and chunks per pipeline stage.
int mm_tile_rows(int fam) { return fam == FAM_F64 ? 64 : 256; }
int mm_tile_cols(int fam) { return fam == FAM_F64 ? 64 : 256; }
int mm_chunks_per_stage(int fam, int form) {
    if (fam == FAM_F64) return 4;
    if (fam == FAM_F32) return 2;
    return form == 1 ? 1 : 2;
}

hipError_t launch_mm(int fam, int form, const MainArgs &a, hipStream_t st) {
    if (fam == FAM_F64) return launch_mm_t<FAM_F64, 0, 64, 64, 4>(a, st);
    if (fam == FAM_F32) return launch_mm_t<FAM_F32, 0, 256, 256, 2>(a, st);
    if (fam == FAM_F16) return launch_mm_t<FAM_F16, 0, 256, 256, 2>(a, st);
    if (fam == FAM_BF16 && form == 0) return launch_mm_t<FAM_BF16, 0, 256, 256, 2>(a, st);
    if (fam == FAM_BF16 && form == 1) return launch_mm_t<FAM_BF16, 1, 256, 256, 1>(a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_backshift(int f64, const void *W, int64_t plane, int K, int64_t M, int64_t N,
                            void *Cout, int64_t ldc, hipStream_t st) {
    const int64_t work = M * ((N + 3) / 4);
    if (work == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL((backshift_kernel<double, double>), dim3(nblocks(work)), dim3(256), 0, st,
                           (const double *)W, plane, K, M, N, (double *)Cout, ldc);
    else
        hipLaunchKernelGGL((backshift_kernel<float, float>), dim3(nblocks(work)), dim3(256), 0, st,
                           (const float *)W, plane, K, M, N, (float *)Cout, ldc);
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
    if (f64) {
        if (a.vec) hipLaunchKernelGGL((gemv_kernel<double, 2>), dim3(nb), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((gemv_kernel<double, 1>), dim3(nb), dim3(256), 0, st, a);
    } else {
        if (a.vec) hipLaunchKernelGGL((gemv_kernel<float, 4>), dim3(nb), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((gemv_kernel<float, 1>), dim3(nb), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace hs
