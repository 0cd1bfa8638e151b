// hs_api.cpp -- host side of the C ABI declared in include/hs.h: argument
// validation, the schedule (bases of Sec. 5.2.1), workspace planning and the
// launch sequence pack -> main loop (whose workgroups also collect the
// back-shift) on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <utility>
#include <vector>

#include "hs.h"
#include "hs_internal.h"

namespace hs {
hipError_t launch_pack(int kind, int kmajor, const PackArgs &a, hipStream_t st);
hipError_t launch_pack_mn(int kind, const PackArgs &a, hipStream_t st);
hipError_t launch_mm(int fam, int form, const MainArgs &a, hipStream_t st);
hipError_t launch_backshift(int f64, const void *W, int64_t plane, int K, int64_t M, int64_t N,
                            void *Cout, int64_t ldc, hipStream_t st);
hipError_t launch_fill_zero(int f64, void *Cout, int64_t M, int64_t N, int64_t ldc, hipStream_t st);
hipError_t launch_gemv(int f64, const GemvArgs &a, hipStream_t st);
hipError_t launch_fp8_exps(const Fp8ExpArgs &a, int64_t tiles, hipStream_t st);
hipError_t launch_row_amax(const RowAmaxArgs &a, hipStream_t st);
void set_timed_launch(hipEvent_t start, hipEvent_t stop);
bool timed_launch_done();
hipError_t launch_nbody(int f64, const void *bodies, void *out, const NbodyArgs &a, int kr, hipStream_t st);
int mm_tile_rows(int fam);
int mm_tile_cols(int fam);
int mm_chunks_per_stage(int fam, int form);
}  // namespace hs

using namespace hs;

namespace {

const int kMaxP = 4096;
const size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct FormInfo {
    int fam, form, pack, in_esz, out_f64, packed_esz;
};

bool form_info(int dt, FormInfo *f) {
    switch (dt) {
        case HS_F64: *f = {FAM_F64, 0, PK_F64, 8, 1, 8}; return true;
        case HS_F32: *f = {FAM_F32, 0, PK_F32, 4, 0, 4}; return true;
        case HS_BF16: *f = {FAM_BF16, 0, PK_B16, 2, 0, 2}; return true;
        case HS_F16: *f = {FAM_F16, 0, PK_B16, 2, 0, 2}; return true;
        case HS_SPLIT3_BF16: *f = {FAM_BF16, 1, PK_SPLIT3, 4, 0, 2}; return true;
        case HS_FP8_E4M3: *f = {FAM_FP8, 0, PK_FP8, 4, 0, 1}; return true;
        case HS_FP8_E4M3_R1: *f = {FAM_FP8, 1, PK_FP8, 4, 0, 1}; return true;
        case HS_SPLIT2_F16: *f = {FAM_F16, 2, PK_SPLIT2F16, 4, 0, 2}; return true;
        default: return false;
    }
}

// The complex dtypes run as one real product of their base form.
bool complex_base(int dt, hs_dtype *base) {
    if (dt == HS_C32) { *base = HS_F32; return true; }
    if (dt == HS_C32_SPLIT3_BF16) { *base = HS_SPLIT3_BF16; return true; }
    if (dt == HS_C32_SPLIT2_F16) { *base = HS_SPLIT2_F16; return true; }
    return false;
}

// Default K: the divisor of p minimising the shift count K + p/K - 1
// (Thm. on minimal length, Sec. 4.4); ties go to the smaller K.
int default_K(int p) {
    int best = 1, cost = std::numeric_limits<int>::max();
    for (int K = 1; K <= p; ++K)
        if (p % K == 0 && K + p / K - 1 < cost) { cost = K + p / K - 1; best = K; }
    return best;
}

struct Plan {
    FormInfo f;
    int p, K, Kt;
    int64_t M, N, Kd;
    OperandGeom ga, gb;
    size_t off_a, off_b, total;
    int G;                            // stripes per workgroup tile (one residue class)
    int64_t a_span;                   // bytes of a workgroup's static-operand region
    size_t off_ea, off_eb;            // fp8: tile exponents of each operand
    int64_t tiles_k, tiles_ra, tiles_rb;
    int nsplit, split_stages;         // workgroups per output tile, stages each
    size_t off_part;                  // their partial planes (nsplit > 1)
};

// Compute units of the MI355X: a launch with fewer output tiles than this
// leaves CUs idle unless each tile's stage sequence is split.
const int64_t kCUs = 256;

// Threads of the pack kernel: one per 16-byte unit; a K-major source is
// walked in 8 x 8 (row, unit) blocks, so both counts round up to 8.
int64_t pack_units(const OperandGeom &g, int kmajor) {
    const int64_t nu = g.nch * (g.chunk_bytes / 16);
    if (kmajor) return g.n_groups * g.p * ((nu + 7) / 8 * 8) * ((g.grp_rows + 7) / 8 * 8);
    return g.n_groups * g.p * nu * g.grp_rows;
}

// Geometry of one product C[M,N] = X[M,Kd] Y[Kd,N] under schedule (p, K).
hs_status make_plan(int64_t M, int64_t N, int64_t Kd, int dt, hs_schedule s, Plan *P) {
    if (!form_info(dt, &P->f)) return HS_ERR_NOT_SUPPORTED;
    hs_schedule r;
    hs_status st = hs_schedule_resolve(s, &r);
    if (st != HS_OK) return st;
    if (M < 0 || N < 0 || Kd < 0) return HS_ERR_INVALID_VALUE;
    // every dimension below 2^31 keeps the products of two of them, and so
    // every count and byte size below, inside 64 bits
    const int64_t kMaxDim = std::numeric_limits<int32_t>::max();
    if (M > kMaxDim || N > kMaxDim || Kd > kMaxDim) return HS_ERR_NOT_SUPPORTED;
    P->p = r.p; P->K = r.K; P->Kt = r.p / r.K;
    P->M = M; P->N = N; P->Kd = Kd;
    const int BMT = mm_tile_rows(P->f.fam), BNT = mm_tile_cols(P->f.fam);
    const int CPS = mm_chunks_per_stage(P->f.fam, P->f.form);
    const int p = P->p;
    const bool fp8 = P->f.fam == FAM_FP8;
    const int CBY = fp8 ? 64 : 32;                  // chunk bytes
    const int KC = CBY / P->f.packed_esz;
    const int64_t S_r = std::max<int64_t>(1, ceil_div(M, p));
    const int64_t S_k = std::max<int64_t>(1, ceil_div(Kd, p));
    const int64_t nch = ceil_div(ceil_div(S_k, KC), CPS) * CPS;
    // a workgroup tile stacks G stripe groups of MS rows, all stripes of one
    // residue class mod K (they share every travelling block)
    const int MS = (int)std::min<int64_t>(BMT, S_r);
    P->G = (int)std::max<int64_t>(1, std::min<int64_t>(P->Kt, BMT / MS));
    const int NP = fp8 ? (P->f.form == 1 ? 2 : 1) : (P->f.form == 1 ? 3 : P->f.form == 2 ? 2 : 1);
    const bool rowscale = P->f.pack == PK_SPLIT2F16;
    if (fp8) {
        // every 32-row / 32-column MFMA tile and every 64-deep chunk must lie
        // inside one 128 x 128 scale tile: whole 64-chunks per block, 32-row
        // aligned stripes and groups
        if (S_k % 64 != 0 || S_r % 32 != 0 || MS % 32 != 0) return HS_ERR_NOT_SUPPORTED;
    }

    OperandGeom &a = P->ga;
    a.R = M; a.Kd = Kd; a.striped = 1; a.S_r = S_r; a.grp_rows = MS;
    a.GS = ceil_div(S_r, MS); a.n_groups = (int64_t)p * a.GS; a.p = p;
    a.S_k = S_k; a.nch = nch; a.chunk_bytes = CBY; a.pieces = NP;
    a.piece_bytes = (int64_t)p * nch * MS * CBY;
    a.group_bytes = NP * a.piece_bytes;

    OperandGeom &b = P->gb;
    b.R = N; b.Kd = Kd; b.striped = 0; b.S_r = 0; b.grp_rows = BNT;
    b.GS = ceil_div(N, BNT); b.n_groups = b.GS; b.p = p;
    b.S_k = S_k; b.nch = nch; b.chunk_bytes = CBY; b.pieces = NP;
    b.piece_bytes = (int64_t)p * nch * BNT * CBY;
    b.group_bytes = NP * b.piece_bytes;

    // grid (with padding to whole workgroup groups) must fit in 32 bits
    const int64_t nwg = (int64_t)p * a.GS * b.GS * 2 + 64;
    if (nwg > std::numeric_limits<int32_t>::max()) return HS_ERR_NOT_SUPPORTED;
    // a workgroup addresses its region of each packed operand with 32-bit
    // offsets: G groups K GS groups apart of the static operand (fewer
    // stripes per tile where that region would pass 4 GiB), one group of
    // the travelling
    const int64_t kMaxPacked = (int64_t)0xFFFFFFF0;
    auto span = [&](int G) { return ((int64_t)(G - 1) * P->K * a.GS + 1) * a.group_bytes; };
    while (P->G > 1 && span(P->G) > kMaxPacked) --P->G;
    P->a_span = span(P->G);
    if (P->a_span > kMaxPacked || b.group_bytes > kMaxPacked) return HS_ERR_NOT_SUPPORTED;
    // 32-bit indexing of the pack kernel and of the stage counter
    if (pack_units(a, 1) >= (int64_t)1 << 31 || pack_units(b, 1) >= (int64_t)1 << 31) return HS_ERR_NOT_SUPPORTED;
    if ((int64_t)p * nch >= (int64_t)1 << 31) return HS_ERR_NOT_SUPPORTED;

    // Output tiles under the CU count: split each tile's step order over
    // nsplit workgroups (at most 4, at least 64 stages each), whose sums a
    // fixed-order FP64 pass adds (the planes below)
    {
        const int64_t nstages = (int64_t)p * (nch / CPS);
        const int64_t tiles = (int64_t)P->K * ceil_div(P->Kt, P->G) * a.GS * b.GS;
        int64_t ns = 1;
        if (tiles > 0 && tiles < kCUs) ns = std::min<int64_t>({4, kCUs / tiles, nstages / 64});
        if (ns < 2) ns = 1;
        P->split_stages = (int)ceil_div(nstages, ns);
        P->nsplit = (int)ceil_div(nstages, P->split_stages);
    }

    // workspace: the two packed operands (no partial planes: the collector
    // keeps every partial in registers), the FP8 tile exponents or the
    // two-piece FP16 row amaxes, and the split planes
    size_t off = 0;
    P->off_a = off; off = align_up(off + (size_t)(a.n_groups * a.group_bytes));
    P->off_b = off; off = align_up(off + (size_t)(b.n_groups * b.group_bytes));
    P->tiles_k = ceil_div(Kd, FP8_TILE);
    P->tiles_ra = ceil_div(M, FP8_TILE);
    P->tiles_rb = ceil_div(N, FP8_TILE);
    P->off_ea = P->off_eb = off;
    if (fp8) {
        P->off_ea = off; off = align_up(off + (size_t)P->tiles_ra * P->tiles_k * 2 * sizeof(int32_t));
        P->off_eb = off; off = align_up(off + (size_t)P->tiles_rb * P->tiles_k * 2 * sizeof(int32_t));
    }
    if (rowscale) {
        P->off_ea = off; off = align_up(off + (size_t)M * sizeof(uint32_t));
        P->off_eb = off; off = align_up(off + (size_t)N * sizeof(uint32_t));
    }
    P->off_part = off;
    if (P->nsplit > 1) off = align_up(off + (size_t)P->nsplit * M * N * (P->f.out_f64 ? 8 : 4));
    P->total = (M == 0 || N == 0 || Kd == 0) ? 0 : off;
    return HS_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// ---------------------------------------------------------------------------
// kernel timing (hs_profile_begin / hs_profile_end)
// ---------------------------------------------------------------------------
bool g_prof = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;

// Two new events handed to the next timed launch, which records them itself.
bool timing_events(hipEvent_t *ev0, hipEvent_t *ev1) {
    if (hipEventCreate(ev0) != hipSuccess) return false;
    if (hipEventCreate(ev1) != hipSuccess) {
        (void)hipEventDestroy(*ev0);
        return false;
    }
    set_timed_launch(*ev0, *ev1);
    return true;
}

// After the launch call: keep the pair if a kernel took it (an empty
// problem launches nothing), else release it.
void keep_timing(hipEvent_t ev0, hipEvent_t ev1) {
    if (timed_launch_done()) {
        g_events.push_back({ev0, ev1});
    } else {
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
}

struct Operand {
    const void *ptr;
    int64_t ld;
    int kmajor;   // 1: contraction index contiguous
    int embed;    // how a complex source is read (PackEmbed)
};

hs_status launch_status(hipError_t e) { return e == hipSuccess ? HS_OK : HS_ERR_LAUNCH_FAILED; }

// A K-major source may be read 16 bytes at a time when every unit's
// elements are contiguous, aligned and either all inside or all outside
// the matrix and its contraction block.
int pack_vec_ok(const Plan &P, const Operand &X) {
    if (!X.kmajor || X.embed != EMB_NONE) return 0;
    const int64_t ue = 16 / P.f.packed_esz;          // source elements per unit
    const int64_t in = P.f.in_esz;
    if (P.f.pack == PK_SPLIT3 || P.f.pack == PK_SPLIT2F16) {   // 8 fp32 per unit (two loads)
        return (X.ld % 4 == 0 && aligned(X.ptr, 16) && P.ga.S_k % 8 == 0 && P.Kd % 8 == 0) ? 1 : 0;
    }
    if (P.f.pack == PK_FP8) {                        // 16 fp32 per unit (four loads)
        return (X.ld % 4 == 0 && aligned(X.ptr, 16) && P.ga.S_k % 16 == 0 && P.Kd % 16 == 0) ? 1 : 0;
    }
    return (X.ld * in % 16 == 0 && aligned(X.ptr, 16) && P.ga.S_k % ue == 0 && P.Kd % ue == 0) ? 1 : 0;
}

// An MN-major FP32 source goes through pack_mn_kernel (16-byte loads of 4
// rows, transposed in LDS) when its rows are 16-byte aligned and every
// 4-row run of a group lies in one stripe.
bool pack_mn_ok(const Plan &P, const Operand &X, const OperandGeom &g) {
    if (X.kmajor || X.embed != EMB_NONE) return false;
    if (P.f.pack != PK_F32 && P.f.pack != PK_SPLIT3 && P.f.pack != PK_FP8 && P.f.pack != PK_SPLIT2F16)
        return false;
    return X.ld % 4 == 0 && aligned(X.ptr, 16) && g.grp_rows % 4 == 0 && (!g.striped || g.S_r % 4 == 0);
}

hipError_t pack_operand(const Plan &P, const Operand &X, const PackArgs &pa, const OperandGeom &g, hipStream_t st) {
    if (pack_mn_ok(P, X, g)) return launch_pack_mn(P.f.pack, pa, st);
    return launch_pack(P.f.pack, X.kmajor, pa, st);
}

// One product through the hyper-systolic path.  The plan must come from
// make_plan with the same sizes; ws holds at least plan.total bytes.
hs_status run_product(const Plan &P, const Operand &X, const Operand &Y, void *out, int64_t ldo,
                      void *ws, hipStream_t stream) {
    const int f64 = P.f.out_f64;
    if (P.M == 0 || P.N == 0) return HS_OK;
    if (P.Kd == 0) return launch_status(launch_fill_zero(f64, out, P.M, P.N, ldo, stream));
    uint8_t *w = (uint8_t *)ws;
    const bool fp8 = P.f.fam == FAM_FP8;
    int32_t *ea = (int32_t *)(w + P.off_ea), *eb = (int32_t *)(w + P.off_eb);
    if (fp8) {   // per-tile exponents of both operands (operand preparation)
        Fp8ExpArgs xa{(const float *)X.ptr, X.ld, X.kmajor, P.M, P.Kd, P.tiles_k, P.f.form, ea};
        Fp8ExpArgs xb{(const float *)Y.ptr, Y.ld, Y.kmajor, P.N, P.Kd, P.tiles_k, P.f.form, eb};
        if (launch_fp8_exps(xa, P.tiles_ra * P.tiles_k, stream) != hipSuccess ||
            launch_fp8_exps(xb, P.tiles_rb * P.tiles_k, stream) != hipSuccess)
            return HS_ERR_LAUNCH_FAILED;
    }
    if (P.f.pack == PK_SPLIT2F16) {   // row amaxes of both operands (their scales)
        RowAmaxArgs xa{(const float *)X.ptr, X.ld, X.kmajor, P.M, P.Kd, (uint32_t *)ea, X.embed};
        RowAmaxArgs xb{(const float *)Y.ptr, Y.ld, Y.kmajor, P.N, P.Kd, (uint32_t *)eb, Y.embed};
        if (launch_row_amax(xa, stream) != hipSuccess || launch_row_amax(xb, stream) != hipSuccess)
            return HS_ERR_LAUNCH_FAILED;
    }

    PackArgs pa{};
    pa.src = X.ptr; pa.ld = X.ld; pa.g = P.ga; pa.dst = w + P.off_a;
    pa.total_units = pack_units(P.ga, X.kmajor);
    pa.vec = pack_vec_ok(P, X);
    pa.exps = ea; pa.exp_tiles_k = P.tiles_k; pa.refine = P.f.form;
    pa.embed = X.embed;
    hipError_t e = pack_operand(P, X, pa, P.ga, stream);
    if (e != hipSuccess) return HS_ERR_LAUNCH_FAILED;
    PackArgs pb{};
    pb.src = Y.ptr; pb.ld = Y.ld; pb.g = P.gb; pb.dst = w + P.off_b;
    pb.total_units = pack_units(P.gb, Y.kmajor);
    pb.vec = pack_vec_ok(P, Y);
    pb.exps = eb; pb.exp_tiles_k = P.tiles_k; pb.refine = P.f.form;
    pb.embed = Y.embed;
    e = pack_operand(P, Y, pb, P.gb, stream);
    if (e != hipSuccess) return HS_ERR_LAUNCH_FAILED;

    MainArgs m{};
    m.A = w + P.off_a; m.a_piece = P.ga.piece_bytes; m.a_group = P.ga.group_bytes;
    m.B = w + P.off_b; m.b_piece = P.gb.piece_bytes; m.b_group = P.gb.group_bytes;
    m.a_span = P.a_span;
    m.p = P.p; m.K = P.K; m.Kt = P.Kt;
    m.MS = P.ga.grp_rows; m.G = P.G; m.GS = P.ga.GS; m.nch = P.ga.nch; m.S_r = P.ga.S_r;
    m.M = P.M; m.N = P.N; m.out_f64 = f64;
    m.a_exps = ea; m.b_exps = eb; m.a_tiles_k = P.tiles_k; m.b_tiles_k = P.tiles_k;
    m.S_k = P.ga.S_k; m.Kd = P.Kd;
    m.out = out;
    m.ldo = ldo;
    m.n_ntiles = P.gb.GS;
    m.nsplit = P.nsplit;
    m.split_stages = P.split_stages;
    m.part = w + P.off_part;
    {   // 32 workgroups per XCD: grp_v class members x grp_t column tiles
        const int64_t nt = P.gb.GS;
        int64_t gt = 1;
        while (gt * 2 <= 8 && gt * 2 <= nt) gt *= 2;
        const int64_t members = ceil_div(P.Kt, P.G) * P.ga.GS;
        int64_t gv = 32 / gt;
        while (gv > 1 && gv / 2 >= members) gv /= 2;
        m.grp_t = gt; m.grp_v = gv;
        m.n_tg = ceil_div(nt, gt);
        m.n_ug = ceil_div(members, gv);
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (g_prof && !timing_events(&ev0, &ev1)) return HS_ERR_LAUNCH_FAILED;
    e = launch_mm(P.f.fam, P.f.form, m, stream);
    if (g_prof) keep_timing(ev0, ev1);
    if (e == hipSuccess && P.nsplit > 1)   // C = the planes' sum, fixed order, FP64
        e = launch_backshift(f64, m.part, P.M * P.N, P.nsplit, P.M, P.N, out, ldo, stream);
    return launch_status(e);
}

hs_status check_mat(const void *p, int64_t rows, int64_t cols, int64_t ld, size_t esz) {
    if (rows < 0 || cols < 0) return HS_ERR_INVALID_VALUE;
    if (ld < std::max<int64_t>(1, cols)) return HS_ERR_INVALID_VALUE;
    if (rows > 0 && cols > 0) {
        if (!p) return HS_ERR_INVALID_VALUE;
        if (!aligned(p, esz)) return HS_ERR_INVALID_VALUE;
    }
    return HS_OK;
}

hs_status check_ws(const Plan &P, const void *ws, size_t ws_bytes) {
    if (P.total == 0) return HS_OK;
    if (!ws) return HS_ERR_WORKSPACE_TOO_SMALL;
    if (!aligned(ws, kAlign)) return HS_ERR_INVALID_VALUE;
    if (ws_bytes < P.total) return HS_ERR_WORKSPACE_TOO_SMALL;
    return HS_OK;
}

#define HS_TRY(x)                          \
    do {                                   \
        hs_status _s = (x);                \
        if (_s != HS_OK) return _s;        \
    } while (0)

}  // namespace

// The n-body call's launch shape and workspace.  Replicas per thread (KR):
// the largest power of two up to 2 that divides K.  Two replicas per thread
// (56 VGPRs, 8 waves per SIMD) measured fastest at n = 2^18, K = 8:
// 3.48 T pairs/s against 3.34 (4) and 3.17 (8).
const int kNbodyKR = 2;
hs_status nbody_plan(int64_t n, int dtype, hs_schedule s, double eps2, NbodyArgs *a, int *kr,
                     size_t *ws) {
    if (dtype != HS_F32 && dtype != HS_F64) return HS_ERR_NOT_SUPPORTED;
    hs_schedule r;
    HS_TRY(hs_schedule_resolve(s, &r));
    if (n < 0 || !std::isfinite(eps2) || eps2 < 0.0) return HS_ERR_INVALID_VALUE;
    if (dtype == HS_F32 && eps2 > (double)std::numeric_limits<float>::max()) return HS_ERR_INVALID_VALUE;
    if (n >= ((int64_t)1 << 31)) return HS_ERR_NOT_SUPPORTED;     // 32-bit positions in a block
    const int f64 = dtype == HS_F64;
    *a = NbodyArgs{};
    a->n = n;
    a->eps2 = eps2;
    a->p = r.p;
    a->K = r.K;
    a->Kt = r.p / r.K;
    a->S = (int)std::max<int64_t>(1, ceil_div(n, r.p));
    a->sub = (int)ceil_div(a->S, 256);
    int k = kNbodyKR;
    while (r.K % k != 0) k /= 2;
    *kr = k;
    a->tgroups = r.K / k;
    if ((int64_t)a->p * a->sub * a->tgroups > std::numeric_limits<int32_t>::max()) return HS_ERR_NOT_SUPPORTED;
    const size_t esz = f64 ? 8 : 4;
    *ws = r.K > 1 ? align_up((size_t)r.K * (size_t)n * 4 * esz) : 0;
    return HS_OK;
}

extern "C" {

const char *hs_status_string(int status) {
    switch (status) {
        case HS_OK: return "HS_OK";
        case HS_ERR_INVALID_VALUE: return "HS_ERR_INVALID_VALUE: invalid argument";
        case HS_ERR_NOT_SUPPORTED: return "HS_ERR_NOT_SUPPORTED: dtype or size not supported for this call";
        case HS_ERR_WORKSPACE_TOO_SMALL: return "HS_ERR_WORKSPACE_TOO_SMALL: workspace smaller than hs_workspace_size()";
        case HS_ERR_LAUNCH_FAILED: return "HS_ERR_LAUNCH_FAILED: the HIP runtime rejected a launch";
        case HS_ERR_EXCEEDS_SCRATCH:
            return "HS_ERR_EXCEEDS_SCRATCH: the call needs more workspace than hs_gemm_noalloc's static scratch holds";
    }
    return "unknown hs_status";
}

hs_status hs_schedule_resolve(hs_schedule in, hs_schedule *out) {
    if (!out) return HS_ERR_INVALID_VALUE;
    if (in.p < 1 || in.p > kMaxP || in.K < 0) return HS_ERR_INVALID_VALUE;
    int K = in.K == 0 ? default_K(in.p) : in.K;
    if (K > in.p || in.p % K != 0) return HS_ERR_INVALID_VALUE;
    out->p = in.p;
    out->K = K;
    return HS_OK;
}

hs_status hs_schedule_table(hs_schedule s, int32_t *out, size_t cap) {
    hs_schedule r;
    HS_TRY(hs_schedule_resolve(s, &r));
    const int p = r.p, K = r.K, Kt = p / K;
    if (!out || cap < (size_t)2 * p * p) return HS_ERR_INVALID_VALUE;
    size_t t = 0;
    for (int v = 0; v < p; ++v)
        for (int j = 0; j < Kt; ++j)
            for (int l = 0; l < K; ++l) {
                out[t++] = ((v - l) % p + p) % p;   // output stripe: partial c^l of v
                out[t++] = (v + j * K) % p;         // travelling block after j shifts by K
            }
    return HS_OK;
}

size_t hs_workspace_size(int op, int64_t m, int64_t n, int64_t k, int dtype, hs_schedule s) {
    const size_t bad = std::numeric_limits<size_t>::max();
    Plan P;
    switch (op) {
        case HS_OP_GEMM: {
            hs_dtype base;
            if (complex_base(dtype, &base)) {
                if (m < 0 || n < 0 || k < 0 || make_plan(m, 2 * n, 2 * k, base, s, &P) != HS_OK) return bad;
                return P.total;
            }
            if (make_plan(m, n, k, dtype, s, &P) != HS_OK) return bad;
            return P.total;
        }
        case HS_OP_GEMM_TN: {
            hs_dtype base;
            if (complex_base(dtype, &base)) {
                if (m < 0 || n < 0 || k < 0 || make_plan(m, 2 * n, 2 * k, base, s, &P) != HS_OK) return bad;
                return P.total;
            }
            if (make_plan(m, n, k, dtype, s, &P) != HS_OK) return bad;
            return P.total;
        }
        case HS_OP_GEMV: {
            if (dtype != HS_F32 && dtype != HS_F64 && dtype != HS_C32) return bad;
            hs_schedule r;
            if (hs_schedule_resolve(s, &r) != HS_OK || m < 0 || n < 0) return bad;
            return 0;
        }
        case HS_OP_NBODY: {
            NbodyArgs a;
            int kr;
            size_t ws;
            if (nbody_plan(m, dtype, s, 0.0, &a, &kr, &ws) != HS_OK) return bad;
            return ws;
        }
        case HS_OP_BACKWARD: {
            Plan Pa, Pb;
            hs_dtype base;
            if (complex_base(dtype, &base)) {
                if (m < 0 || n < 0 || k < 0) return bad;
                if (make_plan(m, 2 * k, 2 * n, base, s, &Pa) != HS_OK) return bad;
                if (make_plan(k, 2 * n, 2 * m, base, s, &Pb) != HS_OK) return bad;
                return std::max(Pa.total, Pb.total);
            }
            if (make_plan(m, k, n, dtype, s, &Pa) != HS_OK) return bad;
            if (make_plan(k, n, m, dtype, s, &Pb) != HS_OK) return bad;
            return std::max(Pa.total, Pb.total);
        }
    }
    return bad;
}

hs_status hs_gemm(int64_t m, int64_t n, int64_t k, int dtype, hs_schedule s,
                  const void *A, int64_t lda, const void *B, int64_t ldb,
                  void *C, int64_t ldc, void *ws, size_t ws_bytes, void *stream) {
    hs_dtype base;
    if (complex_base(dtype, &base)) {
        // one real product: A as m x 2k, B embedded as 2k x 2n, C as m x 2n
        if (m < 0 || n < 0 || k < 0) return HS_ERR_INVALID_VALUE;
        Plan P;
        HS_TRY(make_plan(m, 2 * n, 2 * k, base, s, &P));
        HS_TRY(check_mat(A, m, k, lda, 8));
        HS_TRY(check_mat(B, k, n, ldb, 8));
        HS_TRY(check_mat(C, m, n, ldc, 8));
        HS_TRY(check_ws(P, ws, ws_bytes));
        return run_product(P, Operand{A, 2 * lda, 1, EMB_NONE}, Operand{B, 2 * ldb, 0, EMB_BLOCKS}, C, 2 * ldc, ws,
                           (hipStream_t)stream);
    }
    Plan P;
    HS_TRY(make_plan(m, n, k, dtype, s, &P));
    HS_TRY(check_mat(A, m, k, lda, P.f.in_esz));
    HS_TRY(check_mat(B, k, n, ldb, P.f.in_esz));
    HS_TRY(check_mat(C, m, n, ldc, P.f.out_f64 ? 8 : 4));
    HS_TRY(check_ws(P, ws, ws_bytes));
    return run_product(P, Operand{A, lda, 1, EMB_NONE}, Operand{B, ldb, 0, EMB_NONE}, C, ldc, ws, (hipStream_t)stream);
}

hs_status hs_gemm_tn(int64_t m, int64_t n, int64_t k, int dtype, hs_schedule s,
                     const void *A, int64_t lda, const void *B, int64_t ldb,
                     void *C, int64_t ldc, void *ws, size_t ws_bytes, void *stream) {
    hs_dtype base;
    if (complex_base(dtype, &base)) {
        // A^T as m x 2k reals, read along A's columns; B embedded as 2k x 2n
        if (m < 0 || n < 0 || k < 0) return HS_ERR_INVALID_VALUE;
        Plan P;
        HS_TRY(make_plan(m, 2 * n, 2 * k, base, s, &P));
        HS_TRY(check_mat(A, k, m, lda, 8));
        HS_TRY(check_mat(B, k, n, ldb, 8));
        HS_TRY(check_mat(C, m, n, ldc, 8));
        HS_TRY(check_ws(P, ws, ws_bytes));
        return run_product(P, Operand{A, 2 * lda, 0, EMB_TRANS}, Operand{B, 2 * ldb, 0, EMB_BLOCKS}, C, 2 * ldc, ws,
                           (hipStream_t)stream);
    }
    Plan P;
    HS_TRY(make_plan(m, n, k, dtype, s, &P));
    HS_TRY(check_mat(A, k, m, lda, P.f.in_esz));
    HS_TRY(check_mat(B, k, n, ldb, P.f.in_esz));
    HS_TRY(check_mat(C, m, n, ldc, P.f.out_f64 ? 8 : 4));
    HS_TRY(check_ws(P, ws, ws_bytes));
    return run_product(P, Operand{A, lda, 0, EMB_NONE}, Operand{B, ldb, 0, EMB_NONE}, C, ldc, ws, (hipStream_t)stream);
}

hs_status hs_gemv(int64_t m, int64_t n, int dtype, hs_schedule s,
                  const void *A, int64_t lda, const void *x, void *y,
                  void *ws, size_t ws_bytes, void *stream) {
    (void)ws;
    (void)ws_bytes;
    if (dtype != HS_F32 && dtype != HS_F64 && dtype != HS_C32) return HS_ERR_NOT_SUPPORTED;
    hs_schedule r;
    HS_TRY(hs_schedule_resolve(s, &r));
    const int cplx = dtype == HS_C32;
    const size_t esz = dtype == HS_F32 ? 4 : 8;
    if (m > std::numeric_limits<int32_t>::max()) return HS_ERR_NOT_SUPPORTED;   // 4 rows per workgroup, 32-bit grid
    HS_TRY(check_mat(A, m, n, lda, esz));
    if (n > 0 && m > 0 && (!x || !aligned(x, esz))) return HS_ERR_INVALID_VALUE;
    if (m > 0 && (!y || !aligned(y, esz))) return HS_ERR_INVALID_VALUE;
    if (m == 0) return HS_OK;
    hipStream_t st = (hipStream_t)stream;
    const int f64 = dtype == HS_F64;
    if (n == 0) return launch_status(cplx ? launch_fill_zero(0, y, m, 2, 2, st) : launch_fill_zero(f64, y, m, 1, 1, st));
    GemvArgs g{};
    g.cplx = cplx;
    g.A = A; g.lda = lda; g.x = x; g.y = y; g.m = m; g.n = n;
    g.p = r.p; g.K = r.K; g.Kt = r.p / r.K;
    g.S_r = std::max<int64_t>(1, ceil_div(m, r.p));
    g.S_k = std::max<int64_t>(1, ceil_div(n, r.p));
    if (g.S_k * r.p >= ((int64_t)1 << 31)) return HS_ERR_NOT_SUPPORTED;   // 32-bit positions
    const int VE = (f64 || cplx) ? 2 : 4;         // elements per 16-byte load
    g.vec = (g.S_k % VE == 0 && lda % VE == 0 && n % VE == 0 && aligned(A, 16) && aligned(x, 16)) ? 1 : 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (g_prof && !timing_events(&ev0, &ev1)) return HS_ERR_LAUNCH_FAILED;
    hipError_t e = launch_gemv(f64, g, st);
    if (g_prof) keep_timing(ev0, ev1);
    return launch_status(e);
}

hs_status hs_gemm_backward(int64_t m, int64_t n, int64_t k, int dtype, hs_schedule s,
                           const void *A, int64_t lda, const void *B, int64_t ldb,
                           const void *G, int64_t ldg,
                           void *dA, int64_t ldda, void *dB, int64_t lddb,
                           void *ws, size_t ws_bytes, void *stream) {
    hs_dtype base;
    if (complex_base(dtype, &base)) {
        // dA = G . B^H: G as m x 2n reals, B^H as the 2n x 2k block embedding
        // of conj(B)^T; dB = A^H . G: conj(A)^T as k x 2m reals, G as the
        // 2m x 2n block embedding.  Outputs as interleaved complex.
        if (m < 0 || n < 0 || k < 0) return HS_ERR_INVALID_VALUE;
        Plan Pa, Pb;
        HS_TRY(make_plan(m, 2 * k, 2 * n, base, s, &Pa));
        HS_TRY(make_plan(k, 2 * n, 2 * m, base, s, &Pb));
        HS_TRY(check_mat(G, m, n, ldg, 8));
        if (dA) {
            HS_TRY(check_mat(B, k, n, ldb, 8));
            HS_TRY(check_mat(dA, m, k, ldda, 8));
            HS_TRY(check_ws(Pa, ws, ws_bytes));
        }
        if (dB) {
            HS_TRY(check_mat(A, m, k, lda, 8));
            HS_TRY(check_mat(dB, k, n, lddb, 8));
            HS_TRY(check_ws(Pb, ws, ws_bytes));
        }
        hipStream_t st = (hipStream_t)stream;
        if (dA) HS_TRY(run_product(Pa, Operand{G, 2 * ldg, 1, EMB_NONE}, Operand{B, 2 * ldb, 1, EMB_BLOCKS_H},
                                   dA, 2 * ldda, ws, st));
        if (dB) HS_TRY(run_product(Pb, Operand{A, 2 * lda, 0, EMB_CONJ}, Operand{G, 2 * ldg, 0, EMB_BLOCKS},
                                   dB, 2 * lddb, ws, st));
        return HS_OK;
    }
    Plan Pa, Pb;
    HS_TRY(make_plan(m, k, n, dtype, s, &Pa));   // dA[m,k] = G[m,n] . B[k,n]^T
    HS_TRY(make_plan(k, n, m, dtype, s, &Pb));   // dB[k,n] = A[m,k]^T . G[m,n]
    const size_t oesz = Pa.f.out_f64 ? 8 : 4;
    HS_TRY(check_mat(G, m, n, ldg, Pa.f.in_esz));
    if (dA) {
        HS_TRY(check_mat(B, k, n, ldb, Pa.f.in_esz));
        HS_TRY(check_mat(dA, m, k, ldda, oesz));
        HS_TRY(check_ws(Pa, ws, ws_bytes));
    }
    if (dB) {
        HS_TRY(check_mat(A, m, k, lda, Pb.f.in_esz));
        HS_TRY(check_mat(dB, k, n, lddb, oesz));
        HS_TRY(check_ws(Pb, ws, ws_bytes));
    }
    hipStream_t st = (hipStream_t)stream;
    if (dA) HS_TRY(run_product(Pa, Operand{G, ldg, 1, EMB_NONE}, Operand{B, ldb, 1, EMB_NONE}, dA, ldda, ws, st));
    if (dB) HS_TRY(run_product(Pb, Operand{A, lda, 0, EMB_NONE}, Operand{G, ldg, 0, EMB_NONE}, dB, lddb, ws, st));
    return HS_OK;
}

hs_status hs_nbody(int64_t n, int dtype, hs_schedule s, const void *bodies, double eps2, void *out,
                   void *ws, size_t ws_bytes, void *stream) {
    NbodyArgs a;
    int kr;
    size_t need;
    HS_TRY(nbody_plan(n, dtype, s, eps2, &a, &kr, &need));
    if (n == 0) return HS_OK;
    const int f64 = dtype == HS_F64;
    const size_t row = f64 ? 32 : 16;             // one body: 4 values
    if (!bodies || !out || !aligned(bodies, row) || !aligned(out, row)) return HS_ERR_INVALID_VALUE;
    const uintptr_t b0 = (uintptr_t)bodies, o0 = (uintptr_t)out, len = (uintptr_t)n * row;
    if (b0 < o0 + len && o0 < b0 + len) return HS_ERR_INVALID_VALUE;   // out must not overlap bodies
    if (need > 0) {
        if (!ws) return HS_ERR_WORKSPACE_TOO_SMALL;
        if (!aligned(ws, kAlign)) return HS_ERR_INVALID_VALUE;
        if (ws_bytes < need) return HS_ERR_WORKSPACE_TOO_SMALL;
    }
    hipStream_t st = (hipStream_t)stream;
    void *dst = a.K > 1 ? ws : out;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (g_prof && !timing_events(&ev0, &ev1)) return HS_ERR_LAUNCH_FAILED;
    hipError_t e = launch_nbody(f64, bodies, dst, a, kr, st);
    if (g_prof) keep_timing(ev0, ev1);
    if (e != hipSuccess) return HS_ERR_LAUNCH_FAILED;
    if (a.K > 1) return launch_status(launch_backshift(f64, ws, 4 * n, a.K, n, 4, out, 4, st));
    return HS_OK;
}

hs_status hs_profile_begin(void) {
    g_prof = true;
    return HS_OK;
}

hs_status hs_profile_end(double *total_ms, int64_t *launches) {
    if (!g_prof) return HS_ERR_INVALID_VALUE;
    g_prof = false;
    double tot = 0.0;
    int64_t n = 0;
    hs_status st = HS_OK;
    for (auto &pr : g_events) {
        float ms = 0.f;
        if (hipEventSynchronize(pr.second) != hipSuccess ||
            hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess)
            st = HS_ERR_LAUNCH_FAILED;
        tot += ms;
        ++n;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    g_events.clear();
    if (total_ms) *total_ms = tot;
    if (launches) *launches = n;
    return st;
}

}  // extern "C"
