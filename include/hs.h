/*
 * hs.h -- hyper-systolic matrix products on AMD MI355X (gfx950): C ABI.
 *
 * The method (Lippert, Petkov, Palazzari, Schilling, "Hyper-Systolic Matrix
 * Multiplication", Sec. 5, Algorithm HYPER-SYSTOLIC) computes the ordinary
 * product c_ij = sum_k a_ik b_kj (Sec. 3.1, Eq. PRODUCT) on a ring of p
 * processors with K * K~ = p.  Here the p processors are virtual: groups of
 * workgroups on one GPU.  Virtual processor v owns row stripe v of A and C;
 * the row stripes of B travel.  With 0-based indices:
 *
 *   step j = 0..K~-1 : v holds B stripe kb = (v + j K) mod p
 *                      (base A = (0, K, .., K), Sec. 5.2.1)
 *   l = 0..K-1       : c^l_v += A[(v - l) mod p, kb] . B[kb, :]
 *                      (pre-shift base B = (0, -1, .., -1))
 *   back-shift       : C[r, :] = c^0_r + (c^1_{r+1} + ( .. + c^{K-1}_{r+K-1}))
 *                      (base C = (0, 1, .., 1))
 *
 * This is Algorithm HYPER-SYSTOLIC applied to C^T = B^T A^T (the paper moves
 * A and keeps columns; here rows are kept and B moves).  The "cshift" of a
 * stripe is the order in which its tiles are fetched from HBM into registers
 * and a double-buffered LDS ring.  The back-shift is done by a collector:
 * the workgroup that owns an output tile of stripe r visits the virtual
 * processors r + K - 1, .., r (base C reversed), forms each one's partial
 * c^l on the spot and accumulates it into the same registers, so the K
 * auxiliary arrays C^l never exist in memory.  Each virtual processor enters
 * its cycle of K~ steps (stride K) at block v mod K rather than at block v,
 * so that all processors of a residue class hold the same travelling block
 * at the same time and share it in cache; every processor still forms
 * exactly the block products listed above.
 *
 * Conventions for every entry point
 *  - All matrices are dense and row-major; a leading dimension (ld*) is the
 *    element distance between consecutive rows and must be >= the row length.
 *  - Every pointer is a DEVICE pointer owned by the caller (the outputs of
 *    the backward call may be NULL).  The library never allocates or frees
 *    device memory and never synchronises the stream: work is
 *    enqueued on `stream` (a hipStream_t; NULL means the null stream) and
 *    completes asynchronously.  Device faults surface at the caller's next
 *    synchronisation.
 *  - `ws` is a caller-owned device workspace of at least
 *    hs_workspace_size(...) bytes, 256-byte aligned (NULL allowed when that
 *    size is 0).  Its contents on return are unspecified; two calls that
 *    overlap in time must not share one workspace.
 *  - All argument checks (shapes, schedule, pointers, alignment, dtype,
 *    workspace size) run on the host before any launch; on failure nothing
 *    is enqueued and a non-zero hs_status is returned.  The library never
 *    aborts the process.  A launch error reported by the runtime is returned
 *    as HS_ERR_LAUNCH_FAILED.
 *  - The schedule: 1 <= p <= 4096, K divides p (K = 0 selects the divisor of
 *    p that minimises the shift count K + p/K - 1, i.e. K = sqrt(p) when p
 *    is a perfect square; Sec. 4.4, Thm. on minimal length).  Stripes are
 *    ceil(rows / p) high; a ragged last stripe and contraction blocks are
 *    padded with zeros, which does not change the product.
 *  - Results are deterministic: the schedule and every summation order are
 *    fixed, so the same inputs give the same bits on every run.
 *  - Calls may be captured into a HIP graph: every entry point enqueues
 *    kernels on `stream` only and no memset (zero fills are kernels).  The
 *    workspace must then stay allocated for as long as the graph is
 *    replayed.  The hs_profile_* timing calls are not for use under capture.
 */
#ifndef HS_H
#define HS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic forms.  "in" is the storage type of A, B (and G, x); "out" that
 * of C (and dA, dB, y).
 *  HS_F64          in f64,  out f64.  FP64 MFMA (v_mfma_f64_16x16x4).
 *  HS_F32          in f32,  out f32.  FP32 MFMA (v_mfma_f32_32x32x2).
 *  HS_BF16         in bf16, out f32.  BF16 MFMA, FP32 accumulation.
 *  HS_F16          in f16,  out f32.  FP16 MFMA, FP32 accumulation.
 *  HS_SPLIT3_BF16  in f32,  out f32.  a = a0 + a1 + a2 with bf16 pieces
 *                  (round-to-nearest-even, exact residuals); the six products
 *                  a_i b_j with i + j <= 2 on BF16 MFMA, smallest first, one
 *                  FP32 accumulator per output element.
 *  HS_FP8_E4M3     in f32,  out f32.  a ~= q0 / s with q0 = e4m3(a s) and a
 *                  power-of-two s per 128 x 128 tile of the operand; one
 *                  FP8 MFMA product with hardware block scales.
 *  HS_FP8_E4M3_R1  in f32,  out f32.  One refinement step: a ~= (q0 + q1/s1)/s
 *                  with q1 = e4m3((a s - q0) s1), s1 a power of two per tile;
 *                  products q0 q0', q0 q1', q1 q0'.
 *  HS_C32          in complex64, out complex64 (interleaved re, im FP32
 *                  pairs; ld* in complex elements).  The
 *                  complex product (the complex-data workload of Sec. 7) as
 *                  one real product on FP32 MFMA: A read as an m x 2k real
 *                  matrix, B embedded as the 2k x 2n real matrix whose
 *                  2 x 2 block (t, j) is [[re, im], [-im, re]] of b_tj, C
 *                  written as m x 2n = interleaved complex.  4 real
 *                  multiplications per complex one (no 3M rewrite: it
 *                  cancels).  Also hs_gemm_tn (A^T as m x 2k reals, no
 *                  conjugation), hs_gemv (FP32 complex arithmetic) and
 *                  hs_gemm_backward (dA = G B^H, dB = A^H G).
 *  HS_C32_SPLIT3_BF16  the same with the split-BF16 arithmetic of
 *                  HS_SPLIT3_BF16 (FP32-accurate).  hs_gemm, hs_gemm_tn and
 *                  hs_gemm_backward.
 *  HS_SPLIT2_F16   in f32,  out f32.  Each operand row r (its non-contraction
 *                  index) is scaled by 2^e_r, e_r the largest integer with
 *                  max|row| 2^e_r < 2^15, and split as a' = a0 + a1 with f16
 *                  pieces a0 = f16(a'), a1 = f16(a' - a0) (round to nearest
 *                  even; 22 significant bits); the three products a0 b0,
 *                  a0 b1, a1 b0 on FP16 MFMA into one FP32 accumulator, the
 *                  result scaled back by 2^-(e_row + e_col).  FP32-level
 *                  accuracy with half the MFMA work of HS_SPLIT3_BF16.
 *                  hs_gemm, hs_gemm_tn and hs_gemm_backward.
 *  HS_C32_SPLIT2_F16  HS_C32 with the arithmetic of HS_SPLIT2_F16 (the row
 *                  scales are those of the real operands of the embedding:
 *                  a 2 x 2 block's two rows share the scale of the complex
 *                  column or row they come from).  hs_gemm, hs_gemm_tn and
 *                  hs_gemm_backward.
 *
 * The entry points take the dtype (and hs_workspace_size its op) as a plain
 * int, so that any value a caller passes is well defined: one that is not
 * an hs_dtype gives HS_ERR_NOT_SUPPORTED (SIZE_MAX from hs_workspace_size). */
typedef enum {
    HS_F64 = 0,
    HS_F32 = 1,
    HS_BF16 = 2,
    HS_F16 = 3,
    HS_SPLIT3_BF16 = 4,
    HS_FP8_E4M3 = 5,
    HS_FP8_E4M3_R1 = 6,
    HS_C32 = 7,
    HS_C32_SPLIT3_BF16 = 8,
    HS_SPLIT2_F16 = 9,
    HS_C32_SPLIT2_F16 = 10
} hs_dtype;

typedef enum {
    HS_OK = 0,
    HS_ERR_INVALID_VALUE = 1,       /* bad shape, ld, pointer, schedule */
    HS_ERR_NOT_SUPPORTED = 2,       /* dtype not available for this call, or a
                                       size the kernels cannot address (a
                                       dimension of 2^31 or more, or one
                                       workgroup's packed region above 4 GiB) */
    HS_ERR_WORKSPACE_TOO_SMALL = 3, /* ws_bytes < hs_workspace_size(...) */
    HS_ERR_LAUNCH_FAILED = 4,       /* the HIP runtime rejected a launch */
    HS_ERR_EXCEEDS_SCRATCH = 5      /* hs_gemm_noalloc: the call needs more
                                       workspace than the static scratch holds */
} hs_status;

/* Which call a workspace is sized for. */
typedef enum {
    HS_OP_GEMM = 0,
    HS_OP_GEMM_TN = 1,
    HS_OP_GEMV = 2,
    HS_OP_BACKWARD = 3,
    HS_OP_NBODY = 4          /* m = number of bodies; n, k ignored */
} hs_op;

/* p virtual processors on a logical ring, K * K~ = p (Sec. 5.2).
 * K == 0 selects the default described above. */
typedef struct {
    int32_t p;
    int32_t K;
} hs_schedule;

/* Human-readable name of a status code (static string, never NULL).  Takes
 * any int, so that a caller may pass whatever it received: a value that is
 * not an hs_status gives "unknown hs_status". */
const char *hs_status_string(int status);

/* Resolve K == 0 to its default and validate the schedule.
 * Host only.  Returns HS_ERR_INVALID_VALUE if p < 1, p > 4096, K < 0 or
 * K does not divide p. */
hs_status hs_schedule_resolve(hs_schedule in, hs_schedule *out);

/* The index map of Algorithm HYPER-SYSTOLIC in row orientation (host only,
 * for inspection and tests).  Writes, for v = 0..p-1, j = 0..K~-1,
 * l = 0..K-1 in that nesting order, the pair (r, kb): output stripe
 * r = (v - l) mod p and contraction block kb = (v + j K) mod p, into out[]
 * (2 * p * K~ * K = 2 p^2 int32 values).  Returns HS_ERR_INVALID_VALUE if
 * cap (in int32 elements) is too small or the schedule is invalid. */
hs_status hs_schedule_table(hs_schedule s, int32_t *out, size_t cap);

/* Bytes of device workspace that `op` needs for these sizes (m, n, k as in
 * the corresponding call; for HS_OP_GEMV k is ignored).  Returns 0 if none
 * is needed, and SIZE_MAX if the arguments are invalid. */
size_t hs_workspace_size(int op, int64_t m, int64_t n, int64_t k,
                         int dtype, hs_schedule s);

/* C[m, n] = A[m, k] . B[k, n]  (Eq. PRODUCT; Algorithm HYPER-SYSTOLIC).
 * A: m x k, lda >= k.  B: k x n, ldb >= n.  C: m x n, ldc >= n (written,
 * never read).  All dtypes, the complex ones included (m, n, k and ld* then
 * count complex elements; pointers 8-byte aligned).  m, n or k may be 0
 * (k == 0 writes zeros).  hs_workspace_size(HS_OP_GEMM, m, n, k, ...) of a
 * complex dtype is that of the real product m x 2k times 2k x 2n. */
hs_status hs_gemm(int64_t m, int64_t n, int64_t k, int dtype, hs_schedule s,
                  const void *A, int64_t lda, const void *B, int64_t ldb,
                  void *C, int64_t ldc, void *ws, size_t ws_bytes, void *stream);

/* C[m, n] = A^T . B with A stored k x m (lda >= m), B k x n (ldb >= n).
 * The transposed product, which the paper says runs as efficiently (Abstract,
 * Sec. 8): the same schedule, with A's tiles read along its columns.
 * All dtypes; for the complex ones C = A^T B (transposed, not conjugated),
 * sizes and ld* in complex elements, pointers 8-byte aligned, and the
 * workspace of the real product m x 2k times 2k x 2n. */
hs_status hs_gemm_tn(int64_t m, int64_t n, int64_t k, int dtype, hs_schedule s,
                     const void *A, int64_t lda, const void *B, int64_t ldb,
                     void *C, int64_t ldc, void *ws, size_t ws_bytes, void *stream);

/* y[m] = A[m, n] . x[n]  (the matrix-vector product of the Abstract and
 * Sec. 8).  Virtual processor v owns row stripe v of A and y; x stripes
 * travel in the order of base A; the K partial vectors are combined in the
 * back-shift order, in FP64 for HS_F32.  dtype: HS_F32, HS_F64 or HS_C32
 * (complex64 A, x, y; lda in complex elements; pointers 8-byte aligned; the
 * real and imaginary partial sums combined in FP64).  lda >= n.
 * Needs no workspace (ws may be NULL). */
hs_status hs_gemv(int64_t m, int64_t n, int dtype, hs_schedule s,
                  const void *A, int64_t lda, const void *x, void *y,
                  void *ws, size_t ws_bytes, void *stream);

/* Backward of C = A . B for L = sum(C * G):
 *   dA[m, k] = G . B^T   (contraction over n; B's tiles read along rows)
 *   dB[k, n] = A^T . G   (contraction over m; the transposed product)
 * A: m x k (lda >= k), B: k x n (ldb >= n), G: m x n (ldg >= n),
 * dA: m x k (ldda >= k), dB: k x n (lddb >= n).  Either output may be NULL
 * to skip it.  Both products follow the same schedule `s`, run one after
 * the other on `stream` and may share the workspace.  Storage types as for
 * hs_gemm (G has the input type).  For the complex dtypes the gradients are
 * dA = G . B^H and dB = A^H . G (conjugate transposes; G = dL/dC in the
 * convention where a real loss L has gradient dL/dre + i dL/dim). */
hs_status hs_gemm_backward(int64_t m, int64_t n, int64_t k, int dtype, hs_schedule s,
                           const void *A, int64_t lda, const void *B, int64_t ldb,
                           const void *G, int64_t ldg,
                           void *dA, int64_t ldda, void *dB, int64_t lddb,
                           void *ws, size_t ws_bytes, void *stream);

/* All-pairs gravitational interaction of n bodies: the prototype
 * n^2-problem of Sec. 2.2, computed with the two-array hyper-systolic recipe
 * of Sec. 4.1 on the regular bases of Def. REGULARBASE2 (both data streams
 * are the bodies).  With G = 1, for every body i:
 *
 *   a_i   =  sum_{j != i} m_j (r_j - r_i) / (|r_j - r_i|^2 + eps2)^(3/2)
 *   phi_i = -sum_{j != i} m_j / (|r_j - r_i|^2 + eps2)^(1/2)
 *
 * The bodies are cut into p blocks of ceil(n / p); virtual processor v holds
 * the K replicas block (v + t) mod p, t < K (base A = (0, 1, .., 1)), the
 * travelling block is (v + j K) mod p at step j < K~ (base B = (0, K, .., K)),
 * and the K intermediate results of each body are combined in the
 * collector's order y^0 + (y^1 + ( .. + y^{K-1})), in FP64.  That is
 * 2K + K~ - 3 shifts on a real ring (Thm. GAIN2, Eq. COMPLEXR).
 *
 * bodies: n x 4 values (x, y, z, m), row-major, contiguous; out: n x 4
 * (ax, ay, az, phi), written, never read; out must not overlap bodies.
 * dtype HS_F32 (float; eps2 is rounded to float, rsqrt is the hardware's
 * 1-ulp reciprocal square root) or HS_F64 (double; correctly rounded sqrt
 * and divide).  Both pointers aligned to one body (16 bytes F32, 32 F64).
 * eps2 >= 0 and finite; with eps2 == 0 no two distinct bodies may share a
 * position (their term is infinite).  n == 0 is a no-op; n < 2^31.
 * Workspace: hs_workspace_size(HS_OP_NBODY, n, 0, 0, dtype, s) bytes
 * (K n 4 values; none for K == 1). */
hs_status hs_nbody(int64_t n, int dtype, hs_schedule s, const void *bodies, double eps2, void *out,
                   void *ws, size_t ws_bytes, void *stream);

/* Bytes of the static scratch array of hs_gemm_noalloc (per device). */
#define HS_NOALLOC_SCRATCH_BYTES (64u << 20)

/* hs_gemm without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation): the same product, kernels and results (bit for
 * bit) as hs_gemm, with the workspace taken from a scratch array of
 * HS_NOALLOC_SCRATCH_BYTES that the library's code object holds on every
 * device it runs on, for the life of the process.  Neither this call nor
 * anything it calls allocates or frees device memory.
 * Arguments as for hs_gemm.  Returns HS_ERR_EXCEEDS_SCRATCH, before any
 * launch, when hs_workspace_size(HS_OP_GEMM, m, n, k, dtype, s) exceeds
 * HS_NOALLOC_SCRATCH_BYTES (for instance split-BF16 beyond about
 * m = n = k = 2300, FP32 beyond about 2800), and HS_ERR_LAUNCH_FAILED if the
 * runtime cannot give the scratch array's device address.  All calls on one
 * device share its scratch array: calls that overlap in time on one device
 * race and must be ordered by the caller (one stream, or events). */
hs_status hs_gemm_noalloc(int64_t m, int64_t n, int64_t k, int dtype, hs_schedule s,
                          const void *A, int64_t lda, const void *B, int64_t ldb,
                          void *C, int64_t ldc, void *stream);

/* Kernel timing for measurement.  Between hs_profile_begin() and
 * hs_profile_end(), every launch of the main kernel of any call made from
 * this process (the MFMA kernel of a product, the matrix-vector kernel of
 * hs_gemv, the interaction kernel of hs_nbody) carries a pair of HIP events
 * that its dispatch records itself (hipExtLaunchKernel), so they time the
 * kernel's execution alone.  hs_profile_end() waits for those events and
 * returns the summed elapsed milliseconds and the number of launches.  Not
 * thread-safe, not for use under stream capture; host only.
 * Returns HS_ERR_INVALID_VALUE if profiling was not begun. */
hs_status hs_profile_begin(void);
hs_status hs_profile_end(double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* HS_H */
