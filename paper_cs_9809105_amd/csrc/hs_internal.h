// hs_internal.h -- structures shared by the host API and the HIP kernels.
//
// Packed operand layout ("pack").  A product C[M,N] = sum_k X[M,k] Y[k,N]
// sees two operands, each as a matrix of R "rows" (the non-contraction
// dimension) by Kd contraction elements:
//   * the static operand X (R = M) is cut into p row stripes of S_r rows
//     (virtual processor v owns stripe v, Sec. 5.2.2); each stripe into GS
//     groups of MS rows, zero padded; stripe s's groups sit at positions
//     s GS .. s GS + GS - 1;
//   * the travelling operand Y (R = N, one row per output column) is cut into
//     groups of BN rows (the workgroup column tile);
//   * the contraction is cut into p blocks of S_k elements (block kb is the
//     stripe of Y that a virtual processor holds after kb-v shifts), each
//     padded with zeros to nch chunks of KC elements (32 or 64 bytes).
// Packed bytes: [group][piece][kb][chunk][plane][row in group][16 bytes].
// One (group, kb, chunk) is therefore a contiguous run of rows x 32 bytes,
// which is exactly one HBM->LDS fetch of a pipeline stage.
#pragma once
#include <stdint.h>
#include <stddef.h>

namespace hs {

enum Family : int { FAM_F64 = 0, FAM_F32 = 1, FAM_BF16 = 2, FAM_F16 = 3, FAM_FP8 = 4 };

// What the pack kernel converts from/to.
enum PackKind : int {
    PK_F64 = 0,      // f64 -> f64
    PK_F32 = 1,      // f32 -> f32
    PK_B16 = 2,      // 16-bit -> same 16-bit (bf16 or f16 copy)
    PK_SPLIT3 = 3,   // f32 -> three bf16 pieces
    PK_FP8 = 4,      // f32 -> e4m3 q0 (+ q1) with per-tile power-of-two scales
    PK_SPLIT2F16 = 5 // f32 -> two f16 pieces of x 2^e, e per operand row
};

// Two-piece FP16 split: each operand row (non-contraction index) r gets the
// scale 2^e_r, e_r = the largest integer with amax_r 2^e_r < 2^15, found
// from the row's amax (kept as its float bits, which order like unsigned
// integers for amax >= 0): e_r = 15 - frexp_exp(amax_r) (15 for amax 0).
// Complex sources (embed, see PackEmbed) are scanned as their float view
// (ld in floats): EMB_NONE reads the operand itself; EMB_BLOCKS_H (K-major)
// takes row r from float row r / 2 of the Kd floats of a complex row;
// EMB_BLOCKS (MN-major, Kd / 2 rows of R floats) folds float column c into
// rows c & ~1 and c | 1; EMB_TRANS and EMB_CONJ (MN-major, Kd / 2 rows of
// 2R floats) fold float column c into row c / 2.
struct RowAmaxArgs {
    const float *src;
    int64_t ld;
    int kmajor;               // 1: row r is contiguous along the contraction
    int64_t R, Kd;
    uint32_t *amax;           // [R] float bits of max |x| over the row
    int embed;
};

// FP8 scale tiles: 128 x 128 blocks of the logical operand (rows x
// contraction); per tile two int32 exponents {e, e1}: q0 = e4m3(a 2^e) and,
// with refinement, q1 = e4m3((a 2^e - q0) 2^e1).
const int FP8_TILE = 128;

struct Fp8ExpArgs {
    const float *src;
    int64_t ld;
    int kmajor;
    int64_t R, Kd;
    int64_t tiles_k;          // tiles along the contraction
    int refine;
    int32_t *exps;            // [tile_r][tile_k][2]
};

struct OperandGeom {
    int64_t R;        // logical rows
    int64_t Kd;       // contraction length
    int striped;      // 1: p stripes of S_r rows, groups of MS; 0: groups of grp_rows
    int64_t S_r;      // stripe height (striped) -- ceil(R / p)
    int grp_rows;     // rows per group (MS or BN)
    int64_t GS;       // groups per stripe (striped) or total groups (tiles)
    int64_t n_groups; // logical groups (p GS striped, GS otherwise)
    int p;
    int64_t S_k;      // contraction block length -- ceil(Kd / p)
    int64_t nch;      // chunks per block (padded)
    int chunk_bytes;  // 32 (f64, f32, 16-bit) or 64 (fp8)
    int pieces;       // planes written
    int64_t piece_bytes;  // one piece of one group: p blocks x nch chunks x grp_rows x chunk_bytes
    int64_t group_bytes;  // one group, all pieces
};

struct PackArgs {
    const void *src;
    int64_t ld;
    OperandGeom g;
    void *dst;
    int64_t total_units;     // < 2^31
    int vec;                 // K-major source: 16-byte vector loads are legal
    const int32_t *exps;     // fp8: tile exponents (Fp8ExpArgs); two-piece FP16:
                             // the rows' amax bits (RowAmaxArgs), as uint32
    int64_t exp_tiles_k;
    int refine;              // fp8 only: write q1 as the second piece
    int embed;               // complex sources (interleaved re, im; ld in
                             // floats), see PackEmbed
};

// How the pack kernel reads a complex source (element (kk, row) of the real
// operand; kk the contraction index, row the output row or column).
enum PackEmbed {
    EMB_NONE = 0,      // real source, or complex already laid out as reals
    EMB_BLOCKS = 1,    // MN-major source X[t][j] (t = kk/2, j = row/2): the real
                       // 2 x 2 block embedding [[re x, im x], [-im x, re x]]
    EMB_BLOCKS_H = 2,  // K-major source X[t][j] (t = row/2, j = kk/2): the block
                       // embedding of conj(X[t][j]), i.e. of X^H
    EMB_CONJ = 3,      // MN-major source X[i][t] (i = kk/2, t = row): conj(X)^T
                       // as reals, kk = 2i + (0 re, 1 im)
    EMB_TRANS = 4      // the same read without the conjugation: X^T as reals
};

// One workgroup computes an output tile of G stripe groups -- stripes
// r0, r0 + K, .., r0 + (G-1) K, all of one residue class mod K, sub-group
// msub of each -- by BN columns, and acts as the collector of the back-shift
// (base C = (0, 1, .., 1)): it visits the partials c^{K-1}, .., c^0 in that
// order, computing each on the spot (partial l of stripe s is the work of
// virtual processor s + l: travelling blocks (s + l + jK) mod p, static
// blocks of stripe s) and accumulating it into the same registers.
struct MainArgs {
    const uint8_t *A;        // packed static operand (layout [group][piece][block][chunk]...)
    int64_t a_piece;         // bytes between pieces inside a group
    int64_t a_group;         // bytes between groups
    const uint8_t *B;        // packed travelling operand
    int64_t b_piece;
    int64_t b_group;
    int64_t a_span;          // bytes one workgroup addresses from its first group, < 4 GiB
    const int32_t *a_exps;   // fp8: tile exponents of each operand; two-piece
    const int32_t *b_exps;   // FP16: each operand's row amax bits (uint32)
    int64_t a_tiles_k, b_tiles_k;
    int64_t S_k;             // contraction block length (fp8 scale lookup)
    int64_t Kd;              // contraction length
    void *out;               // the result C
    int64_t ldo;             // row stride of out (elements)
    int p, K, Kt;
    int MS;                  // static-operand rows per group
    int G;                   // stripes per workgroup tile (one residue class)
    int64_t GS;              // groups per stripe
    int64_t nch;             // chunks per contraction block
    int64_t S_r;             // stripe height
    int64_t M, N;
    int64_t n_ntiles;        // column tiles
    int out_f64;             // out element type: 1 double, 0 float
    // workgroup groups: grp_v class members x grp_t column tiles run together
    int64_t grp_v, grp_t, n_ug, n_tg;
    // launches with fewer output tiles than CUs: nsplit workgroups per tile,
    // each over split_stages consecutive stages of the step order, their sums
    // in planes [nsplit][M][N] of part (element type as out), summed after
    int nsplit;
    int split_stages;
    void *part;
};

struct GemvArgs {
    const void *A;
    int64_t lda;
    const void *x;
    void *y;
    int64_t m, n;
    int p, K, Kt;
    int64_t S_r, S_k;
    int vec;                 // 1: 16-byte loads are legal
    int cplx;                // 1: complex64 A, x, y (lda in complex elements)
};

// All-pairs n-body interaction on the two-array recipe (hs_nbody.hip).
struct NbodyArgs {
    int64_t n;               // bodies
    double eps2;             // softening, >= 0 (rounded to float for FP32)
    int p, K, Kt;            // ring of p virtual processors, K * Kt == p
    int S;                   // bodies per block, ceil(n / p)
    int sub;                 // workgroups along one block: ceil(S / 256)
    int tgroups;             // thread groups per position: K / KR
};

}  // namespace hs
