// hs_nbody.hip -- the all-pairs gravitational interaction of n bodies (the
// prototype n^2-problem of Sec. 2.2) on the two-array hyper-systolic recipe
// of Sec. 4.1 with the regular bases of Def. REGULARBASE2.
//
// The bodies are cut into p blocks of S = ceil(n / p); virtual processor v
// owns block v.  With 0-based indices and K * K~ = p:
//
//   replicas  x^_t = block (v + t) mod p,   t = 0..K-1   (A = (0, 1, .., 1))
//   travel    step j: z = block (v + j K) mod p, j = 0..K~-1   (B = (0, K, .., K))
//   results   y^_t(v) += f(x^_t, z) over every step
//   collector y(b) = y^_0 + (y^_1 + ( .. + y^_{K-1}))   for body block b,
//             where y^_t comes from processor (b - t) mod p
//
// f(x, z) adds, for target body x and source body z (z != x),
//   a   += m_z (r_z - r_x) / (|r_z - r_x|^2 + eps2)^(3/2)
//   phi -= m_z / (|r_z - r_x|^2 + eps2)^(1/2).
// Every ordered pair of bodies meets exactly once (the base pair is complete
// and K K~ = p, so no multiplicity table is needed); the only pairs of a body
// with itself occur for replica t = 0 at step j = 0, where they are skipped.
//
// On the GPU a virtual processor is a group of workgroups.  A thread holds
// one body position i of the stripe in KR of the K replicas (registers), and
// reads the travelling block body by body with wave-uniform loads, so each
// travelling body feeds KR interactions per lane.  The collector's moves by
// -1 become addressing: replica t of processor v writes its results into
// partial plane t at the rows of the bodies it belongs to (block v + t), and
// the back-shift kernel sums the K planes per body in the order above, in
// FP64.  K = 1 (the systolic special case) writes the result directly.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hs_internal.h"

namespace hs {

#define DEVI __device__ __forceinline__

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    typedef float4 type;
};
template <>
struct Vec4<double> {
    typedef double4 type;
};

DEVI float inv_sqrt(float s) { return __builtin_amdgcn_rsqf(s); }
DEVI double inv_sqrt(double s) { return 1.0 / sqrt(s); }
DEVI float fma3(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
DEVI double fma3(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One travelling body (zx, zy, zz, zm) against the thread's KR replicas.
// SELF: this is step j = 0 of the thread group holding replica t = 0, where
// source position jj equals the thread's own position i for that replica.
// 14 VALU instructions per pair (one v_rsq_f32).  The potential takes its
// own fused multiply-add from inv, independent of m / s^(1/2): forming that
// product once and subtracting it measured 15 % slower.
template <typename T, int KR, bool SELF>
DEVI void interact(const T zx, const T zy, const T zz, const T zm, const int jj, const int i,
                   const T eps2, const T (&px)[KR], const T (&py)[KR], const T (&pz)[KR], T (&ax)[KR],
                   T (&ay)[KR], T (&az)[KR], T (&ph)[KR]) {
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const T dx = zx - px[r];
        const T dy = zy - py[r];
        const T dz = zz - pz[r];
        const T s = fma3(dz, dz, fma3(dy, dy, fma3(dx, dx, eps2)));
        T inv = inv_sqrt(s);
        if (SELF && r == 0) inv = (jj == i) ? (T)0 : inv;
        ph[r] = fma3(-zm, inv, ph[r]);          // phi -= m / s^(1/2)
        const T w = (zm * inv) * (inv * inv);   // m / s^(3/2)
        ax[r] = fma3(w, dx, ax[r]);
        ay[r] = fma3(w, dy, ay[r]);
        az[r] = fma3(w, dz, az[r]);
    }
}

// The travelling block src[0..cnt) against the replicas, UB bodies per
// round of wave-uniform loads.
template <typename T, int KR, bool SELF>
DEVI void travel(const T *__restrict__ src, const int cnt, const int i, const T eps2, const T (&px)[KR],
                 const T (&py)[KR], const T (&pz)[KR], T (&ax)[KR], T (&ay)[KR], T (&az)[KR], T (&ph)[KR]) {
    constexpr int UB = 8;
    int jj = 0;
    for (; jj + UB <= cnt; jj += UB) {
        T z[UB][4];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
#pragma unroll
            for (int c = 0; c < 4; ++c) z[u][c] = src[(int64_t)(jj + u) * 4 + c];
        }
#pragma unroll
        for (int u = 0; u < UB; ++u)
            interact<T, KR, SELF>(z[u][0], z[u][1], z[u][2], z[u][3], jj + u, i, eps2, px, py, pz, ax, ay, az, ph);
    }
    for (; jj < cnt; ++jj) {
        const T *z = src + (int64_t)jj * 4;
        interact<T, KR, SELF>(z[0], z[1], z[2], z[3], jj, i, eps2, px, py, pz, ax, ay, az, ph);
    }
}

// Grid: p * sub * tgroups workgroups of 256 threads (host-checked).
// Workgroup w: thread group tg = w % tgroups (replicas tg*KR .. tg*KR+KR-1),
// slice s = (w / tgroups) % sub (positions s*256 .. s*256+255 of the block),
// virtual processor v = w / (tgroups * sub).
template <typename T, int KR>
__global__ __launch_bounds__(256) void nbody_kernel(const T *__restrict__ bodies, T *__restrict__ out,
                                                    NbodyArgs a) {
    typedef typename Vec4<T>::type V4;
    const int w = blockIdx.x;
    const int tg = w % a.tgroups;
    const int rest = w / a.tgroups;
    const int s = rest % a.sub;
    const int v = rest / a.sub;
    const int i = s * 256 + (int)threadIdx.x;   // position in the stripe
    const int p = a.p, K = a.K, S = a.S;
    const int t0 = tg * KR;
    const T eps2 = (T)a.eps2;

    T px[KR], py[KR], pz[KR], ax[KR], ay[KR], az[KR], ph[KR];
    int64_t row[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int blk = (v + t0 + r) % p;             // replica t = t0 + r: block v + t
        row[r] = (int64_t)blk * S + i;
        const bool ok = i < S && row[r] < a.n;
        if (ok) {
            const V4 b = ((const V4 *)bodies)[row[r]];
            px[r] = b.x;
            py[r] = b.y;
            pz[r] = b.z;
        } else {
            px[r] = py[r] = pz[r] = (T)0;
        }
        ax[r] = ay[r] = az[r] = ph[r] = (T)0;
    }

    for (int j = 0; j < a.Kt; ++j) {
        const int blk = (v + j * K) % p;              // travelling block after j shifts by K
        const int64_t base = (int64_t)blk * S;
        const int64_t left = a.n - base;
        const int cnt = left <= 0 ? 0 : (left < S ? (int)left : S);
        const T *src = bodies + base * 4;
        if (j == 0 && t0 == 0)
            travel<T, KR, true>(src, cnt, i, eps2, px, py, pz, ax, ay, az, ph);
        else
            travel<T, KR, false>(src, cnt, i, eps2, px, py, pz, ax, ay, az, ph);
    }

    if (i >= S) return;
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        if (row[r] >= a.n) continue;
        V4 o;
        o.x = ax[r];
        o.y = ay[r];
        o.z = az[r];
        o.w = ph[r];
        const int64_t plane = (int64_t)(t0 + r) * a.n;   // K == 1: plane 0 is the result
        ((V4 *)out)[plane + row[r]] = o;
    }
}

bool take_timed_launch(hipEvent_t *start, hipEvent_t *stop);   // hs_kernels.hip

hipError_t launch_nbody(int f64, const void *bodies, void *out, const NbodyArgs &a, int kr, hipStream_t st) {
    const int64_t nwg = (int64_t)a.p * a.sub * a.tgroups;
    if (nwg == 0) return hipSuccess;
    const dim3 grid((unsigned)nwg), block(256);
    hipEvent_t ts, te;
    const bool timed = take_timed_launch(&ts, &te);   // hs_profile_*: events recorded by the dispatch
#define HS_NB(T, R)                                                                                           \
    do {                                                                                                      \
        if (timed)                                                                                            \
            hipExtLaunchKernelGGL((nbody_kernel<T, R>), grid, block, 0, st, ts, te, 0, (const T *)bodies,      \
                                  (T *)out, a);                                                               \
        else                                                                                                  \
            hipLaunchKernelGGL((nbody_kernel<T, R>), grid, block, 0, st, (const T *)bodies, (T *)out, a);     \
    } while (0)
    // kr: replicas per thread, 2 (K even) or 1 (K odd)
    if (f64) {
        if (kr == 2) HS_NB(double, 2);
        else HS_NB(double, 1);
    } else {
        if (kr == 2) HS_NB(float, 2);
        else HS_NB(float, 1);
    }
#undef HS_NB
    return hipGetLastError();
}

}  // namespace hs
