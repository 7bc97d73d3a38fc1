// Batched exact objective on int8 matrix cores (the evaluation the paper moves
// to the GPU, Introduction and Pseudocode section):
//
//     Y = X Q  (int8 x int8 -> int32, v_mfma_i32_32x32x32_i8),
//     f_m = sum_j x_mj Y_mj  (int64)
//
// X is bit-packed (1 bit per variable, the A operand is expanded to int8 0/1 in
// registers), Q is a resident int8 plane [n_pad][n_pad].  Q is symmetric, so
// column j of Q is row j: both operands are K-contiguous and the B fragment of
// a lane is 16 consecutive bytes of one Q row.
//
// The objective uses only the lower triangle of Q (Q is symmetric):
//     f_m = sum_j x_mj (2 acc_mj - q_jj),  acc_mj = sum_{i <= j} x_mi q_ij,
// so a tile of columns [n0, n0 + 128) contracts K over [0, n0 + 128) only, half
// the dense work overall (the Delta initialisation needs the full Y and keeps
// the full K range).
//
// Exactness: |acc_mj| <= 128 n <= 2^20 for n <= 8192, inside int32; the row dot
// is summed per 128-column tile in int32 (< 2^31) and accumulated across tiles
// and planes with int64 atomics (integer, so the order does not matter).
//
// Workgroup tile BM x BN = 256 x 128: four waves of 64 rows x 128 columns
// (2 x 4 blocks of 32 x 32), so each expanded A fragment feeds 4 MFMAs.  K is
// staged through LDS KC = 128 at a time, double buffered (the tail of the last
// step reads zeros); 48 KB of LDS and under 256 registers per wave let two
// workgroups share a CU, which hides the global-load latency of the staging.
// Inside a K step the fragments of substep s+1 are read (and the A bits
// expanded) while the MFMAs of substep s run, interleaved by scheduling groups.
// Other epilogues store Y rows or the ascent's keys (the Delta initialisation,
// on gathered passer rows).
#include "ubqp_internal.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int BM = 256, THR = 256;  // workgroup rows (one staged X row per thread)

// Workgroup tile geometry: BM x BN, the four waves arranged WR x WC, each wave
// WTM x WTN = (BM / WR) x (BN / WC) in 32 x 32 MFMA blocks.  In use: BN = 128, WR = 4,
// waves of 64 x 128 (two workgroups per CU for KC <= 128).  The body also accepts
// BN = 256 (waves of 64 x 256 or 128 x 128: column tiles may reach past n_pad),
// which was measured slower.
template <int BN_, int WR_> struct Geom {
    static constexpr int BN = BN_, WR = WR_, WC = 4 / WR_;
    static constexpr int WTM = BM / WR, WTN = BN / WC;
    static constexpr int FM = WTM / 32, FN = WTN / 32;
    static_assert(WR * WC == 4 && (WTN == 128 || WTN == 256), "four waves, 128 or 256 columns per wave");
};

// 16 bits -> 16 bytes of 0/1: nibble v spreads to bytes by v * 0x00204081
// (bit i lands at 8i, no carries because the copies are 7 bits apart).
__device__ inline v4i expand16(uint32_t bits)
{
    v4i r;
    r[0] = (int)(((bits & 0xFu) * 0x00204081u) & 0x01010101u);
    r[1] = (int)((((bits >> 4) & 0xFu) * 0x00204081u) & 0x01010101u);
    r[2] = (int)((((bits >> 8) & 0xFu) * 0x00204081u) & 0x01010101u);
    r[3] = (int)((((bits >> 12) & 0xFu) * 0x00204081u) & 0x01010101u);
    return r;
}

// Sum over the 16 lanes of each DPP row (every lane gets its row's sum).
__device__ inline int32_t row16_sum(int32_t v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0, v, 0x124, 0xF, 0xF, false);  // row_ror:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror:8
    return v;
}


// Epilogues of the contraction.
enum { EPI_ROWDOT = 0, EPI_Y = 1, EPI_KEYS = 2 };

// Scheduling groups (the instruction classes of __builtin_amdgcn_sched_group_barrier).
#define SG_VALU 0x002
#define SG_MFMA 0x008
#define SG_DSR 0x100

__device__ inline int word0_of(int col) { return col >> 6; }

// Consecutive workgroups go round-robin to the 8 XCDs: give each XCD a
// contiguous run of tiles, a bijection on [0, total).  Tiles are numbered
// n-tile-major, so the workgroups resident on one XCD share a Q column block in
// its L2.
__device__ inline int64_t xcd_tile(int64_t b, int64_t total)
{
    const int64_t xcd = b % 8, j = b / 8, per = total / 8, rem = total % 8;
    return xcd * per + (xcd < rem ? xcd : rem) + j;
}

// LDS of one workgroup: the double-buffered K step of Q (B) and X (A), and for the
// key epilogue the X words of the tile's columns.  One set per (EPI, KC, BN): the
// split and unsplit bodies of one kernel share it.
template <int EPI, int KC, int BN> struct EvalLds {
    static constexpr bool KEYS_LDS = EPI == EPI_KEYS && KC <= BN && BN % KC == 0;
    static constexpr int B = BN * (KC + 16), A = BM * (KC / 64 + 1), X = KEYS_LDS ? BM * (BN / 64) : 1;
    __device__ static int8_t (&bs())[2][B]
    {
        __shared__ __align__(16) int8_t v[2][B];
        return v;
    }
    __device__ static uint64_t (&as())[2][A]
    {
        __shared__ __align__(16) uint64_t v[2][A];
        return v;
    }
    __device__ static uint64_t (&xt())[X]
    {
        __shared__ uint64_t v[X];
        return v;
    }
};

// SPLIT: the Y / key epilogues' split-K body (a share of the K range, raw partial rows).
template <int EPI, int KC, int BN_, int WR_, bool SPLIT>
__device__ void eval_body(const EvalArgs &a, int64_t tile)
{
    using GM = Geom<BN_, WR_>;
    constexpr int BN = GM::BN, WC = GM::WC, WTM = GM::WTM, WTN = GM::WTN, FM = GM::FM, FN = GM::FN;
    // a column tile wider than the padding granularity can reach past n_pad: its
    // Q rows there read as zero and the waves whose columns lie there store nothing
    constexpr bool ROWGUARD = BN > UBQP_NPAD_ALIGN;
    constexpr bool STORE_Y = EPI != EPI_ROWDOT;
    // The objective needs only the lower triangle of the symmetric Q:
    //     f = sum_j x_j (2 acc_j - q_jj),   acc_j = sum_{i <= j} q_ij x_i,
    // so the row-dot tile of columns [n0, n0 + BN) contracts K over [0, n0 + BN)
    // with the entries k > j of its diagonal block zeroed when they are staged.
    constexpr bool TRI = EPI == EPI_ROWDOT;
    constexpr int BPITCH = KC + 16;       // bytes per staged Q row (16-byte skew: conflict-free reads)
    constexpr int APITCH = KC / 64 + 1;   // words per staged X row (odd: conflict-free 8-byte reads)
    constexpr int NSUB = KC / 32;         // 32-deep MFMA substeps per K step
    constexpr int BCH = BN * KC / 16 / THR;  // 16-byte Q chunks each thread stages per K step
    constexpr int BROWS = THR / (KC / 16);   // Q rows covered by one pass of the threads
    auto &Bs = EvalLds<EPI, KC, BN_>::bs();
    auto &As = EvalLds<EPI, KC, BN_>::as();
    static_assert(sizeof(Bs[0]) == BN * BPITCH && sizeof(As[0]) == BM * APITCH * 8, "LDS layout");

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WC, wc = wave % WC;
    const int64_t T = (int64_t)a.m_tiles * a.n_tiles;
    const int plane = (int)(tile / T);
    const int64_t t = tile - plane * T;
    // tile order: n-tile-major (workgroups adjacent in t share a Q column block)
    // or m-tile-major (they share an X row block)
    int nt = a.order ? (int)(t % a.n_tiles) : (int)(t / a.m_tiles);
    int mt = a.order ? (int)(t / a.n_tiles) : (int)(t % a.m_tiles);
    if (TRI) {
        // column tile nt costs nt + 1 K blocks: pair long and short tiles
        // (N-1, 0, N-2, 1, ...) so that every XCD's contiguous run of tiles holds
        // a balanced share of the work
        nt = (nt & 1) ? (nt >> 1) : a.n_tiles - 1 - (nt >> 1);
    }

    // rows in use: the gathered list's device length (Y / key epilogues), or for
    // the row dot an optional device row count (rows beyond it are skipped)
    int64_t Mrows = a.M;
    if (STORE_Y || a.nrows_d) { const int64_t k = *a.nrows_d - a.offset; Mrows = k < a.M ? k : a.M; }
    // Split K (few gathered rows, the team ascent consuming them): of each column
    // tile's row-tile slots, the first S R take (part ks of the K range, row tile mt)
    // -- slots spread over the grid like the active tiles of an unsplit launch, so
    // over all XCDs -- and part ks stores its raw partial rows prow = ks R 256 rows
    // further down the Y workspace.
    int nks = 1, ks = 0;
    int64_t prow = 0;
    if constexpr (SPLIT) {
        nks = ubqp_dinit_split(Mrows, a.M, a.n_pad, a.planes, a.split_team_max, a.split_target);
        const int R = (int)((Mrows + BM - 1) / BM);
        if (mt >= nks * R) return;
        ks = mt / R;
        mt -= ks * R;
        prow = (int64_t)ks * R * BM;
    }
    const int64_t m0 = (int64_t)mt * BM;
    if (m0 >= Mrows) return;
    const int n0 = nt * BN;
    const int8_t *qp = a.q + plane * a.plane_stride;

    // staging assignment: thread tid loads X row m0 + tid (KC/64 words) and BCH
    // 16-byte chunks of the Q block (rows tid / (KC/16) + BROWS i, chunk tid % (KC/16))
    const int64_t arow = m0 + tid;
    const uint64_t *xrow = nullptr;
    if (arow < Mrows) {
        const int64_t r = STORE_Y ? (int64_t)a.rows[arow] : arow;
        if (r >= 0 && r < a.x_rows) xrow = a.X + r * a.W;
    }
    const int brow = tid / (KC / 16), bc16 = tid % (KC / 16);
    const int8_t *qsrc = qp + (int64_t)(n0 + brow) * a.n_pad + bc16 * 16;

    uint64_t aw[KC / 64];
    uint4 br[BCH];
    // Key epilogue with KC dividing BN: the X words of this tile's columns pass
    // through the staging registers at the K steps kc = n0 / KC + s; a copy goes to
    // LDS after the loop for the epilogue (the same gathered rows, zero where the
    // staging is zero).
    constexpr bool KEYS_LDS = EvalLds<EPI, KC, BN_>::KEYS_LDS && !SPLIT;
    uint64_t xt[BN / 64] = {};
    int32_t dg[FN] = {};  // key epilogue: q_jj of the lane's columns, loaded early
    if constexpr (EPI == EPI_KEYS) {
#pragma unroll
        for (int ni = 0; ni < FN; ni++) {
            const int col = n0 + wc * WTN + ni * 32 + (tid & 31);
            dg[ni] = col < a.n_pad ? a.diag[col] : 0;
        }
    }
    const int nk_full = (a.n_pad + KC - 1) / KC;
    // this workgroup's K steps [kb, ke)
    const int kb = nk_full * ks / nks;
    const int ke = TRI ? min(nk_full, (n0 + BN + KC - 1) / KC) : nk_full * (ks + 1) / nks;
    // global -> registers for K step kc; columns past n_pad (the tail of the last step) read as 0
#define EVAL_LOAD_STAGE(kc)                                                                   \
    do {                                                                                      \
        _Pragma("unroll") for (int w_ = 0; w_ < KC / 64; w_++) {                              \
            const int wi_ = (kc) * (KC / 64) + w_;                                            \
            aw[w_] = (xrow && wi_ < a.W) ? ubqp_ldg8(xrow + wi_) : 0ull;                      \
        }                                                                                     \
        if (KEYS_LDS) {                                                                       \
            _Pragma("unroll") for (int s_ = 0; s_ < BN / KC; s_++) {                          \
                if ((kc) * KC == n0 + s_ * KC) {                                              \
                    _Pragma("unroll") for (int w_ = 0; w_ < KC / 64; w_++)                    \
                        xt[s_ * (KC / 64) + w_] = aw[w_];                                     \
                }                                                                             \
            }                                                                                 \
        }                                                                                     \
        const bool kin_ = (kc) * KC + bc16 * 16 < a.n_pad;                                    \
        _Pragma("unroll") for (int i_ = 0; i_ < BCH; i_++) {                                  \
            const bool rin_ = !ROWGUARD || n0 + brow + BROWS * i_ < a.n_pad;                  \
            br[i_] = (kin_ && rin_) ? ubqp_ldg16(qsrc + (int64_t)(BROWS * i_) * a.n_pad + (kc) * KC) \
                                    : uint4{0u, 0u, 0u, 0u};                                  \
        }                                                                                     \
        if (TRI && (kc) * KC + KC > n0) {                                                     \
            /* diagonal block: keep bytes with k <= j (j = column, k = byte's K index) */     \
            _Pragma("unroll") for (int i_ = 0; i_ < BCH; i_++) {                              \
                const int lim_ = n0 + brow + BROWS * i_ - ((kc) * KC + bc16 * 16) + 1;        \
                uint32_t m_[4];                                                               \
                _Pragma("unroll") for (int d_ = 0; d_ < 4; d_++) {                            \
                    const int v_ = min(max(lim_ - 4 * d_, 0), 4);                             \
                    m_[d_] = v_ >= 4 ? 0xFFFFFFFFu : ((1u << (8 * v_)) - 1u);                 \
                }                                                                             \
                br[i_].x &= m_[0];                                                            \
                br[i_].y &= m_[1];                                                            \
                br[i_].z &= m_[2];                                                            \
                br[i_].w &= m_[3];                                                            \
            }                                                                                 \
        }                                                                                     \
    } while (0)
    // registers -> LDS buffer buf
#define EVAL_STORE_STAGE(buf)                                                                 \
    do {                                                                                      \
        _Pragma("unroll") for (int w_ = 0; w_ < KC / 64; w_++) As[buf][tid * APITCH + w_] = aw[w_]; \
        _Pragma("unroll") for (int i_ = 0; i_ < BCH; i_++)                                    \
            *(uint4 *)(&Bs[buf][(brow + BROWS * i_) * BPITCH + bc16 * 16]) = br[i_];          \
    } while (0)

    v16i acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
        for (int k = 0; k < FN; k++)
#pragma unroll
            for (int e = 0; e < 16; e++) acc[i][k][e] = 0;

    // Fragments of a 32-deep substep: lane l holds row / column l%32 and the 16
    // consecutive k starting at 16 (l/32) -- the same k for A and B.
    const int r32 = lane & 31, h = lane >> 5;
    v4i afc[FM], afn[FM], bfc[FN], bfn[FN];
    uint64_t awd[FM];
#define EVAL_READ_A(buf, w)                                                                   \
    _Pragma("unroll") for (int mi = 0; mi < FM; mi++)                                         \
        awd[mi] = As[buf][(wr * WTM + mi * 32 + r32) * APITCH + (w)]
#define EVAL_EXPAND_A(dst, half)                                                              \
    _Pragma("unroll") for (int mi = 0; mi < FM; mi++)                                         \
        dst[mi] = expand16((uint32_t)(awd[mi] >> (32 * (half) + 16 * h)) & 0xFFFFu)
#define EVAL_READ_B(dst, buf, sub)                                                            \
    _Pragma("unroll") for (int ni = 0; ni < FN; ni++)                                         \
        dst[ni] = *(const v4i *)(&Bs[buf][(wc * WTN + ni * 32 + r32) * BPITCH + 32 * (sub) + 16 * h])

    EVAL_LOAD_STAGE(kb);
    EVAL_STORE_STAGE(0);
    __syncthreads();
    EVAL_READ_A(0, 0);
    EVAL_READ_B(bfc, 0, 0);
    EVAL_EXPAND_A(afc, 0);
    const int nk = ke - kb;
    for (int kk = 0; kk < nk; kk++) {
        const int kc = kb + kk, cur = kk & 1;
        const bool more = kk + 1 < nk;
        if (more) EVAL_LOAD_STAGE(kc + 1);
#pragma unroll
        for (int sub = 0; sub < NSUB; sub++) {
            if (sub + 1 < NSUB) {
                // next substep's fragments: reads first, MFMAs, then the A expansion
                if (((sub + 1) & 1) == 0) EVAL_READ_A(cur, (sub + 1) >> 1);
                EVAL_READ_B(bfn, cur, sub + 1);
            }
            // the substep's matrix ops at raised wave priority: the SIMD's other wave
            // (another workgroup) gets the issue slots of its loads and expansion
            // in between instead of competing with this burst (5% faster measured)
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int ni = 0; ni < FN; ni++)
#pragma unroll
                for (int mi = 0; mi < FM; mi++)
                    acc[mi][ni] = __builtin_amdgcn_mfma_i32_32x32x32_i8(afc[mi], bfc[ni], acc[mi][ni], 0, 0, 0);
            if (sub + 1 < NSUB) {
                EVAL_EXPAND_A(afn, (sub + 1) & 1);
                // interleave: one MFMA, one LDS read, three VALU
#pragma unroll
                for (int i = 0; i < FM * FN; i++) {
                    __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(SG_DSR, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(SG_VALU, 3, 0);
                }
#pragma unroll
                for (int mi = 0; mi < FM; mi++) afc[mi] = afn[mi];
#pragma unroll
                for (int ni = 0; ni < FN; ni++) bfc[ni] = bfn[ni];
            }
            __builtin_amdgcn_s_setprio(0);
        }
        if (more) {
            EVAL_STORE_STAGE(cur ^ 1);
            __syncthreads();
            EVAL_READ_A(cur ^ 1, 0);
            EVAL_READ_B(bfc, cur ^ 1, 0);
            EVAL_EXPAND_A(afc, 0);
        }
    }
#undef EVAL_LOAD_STAGE
#undef EVAL_STORE_STAGE
#undef EVAL_READ_A
#undef EVAL_EXPAND_A
#undef EVAL_READ_B

    // D layout of a 32x32 block: accumulator e of lane l is row 8 (e/4) + 4 (l/32) + e%4,
    // column l%32.  The wave's columns [c0, c0 + WTN) are X words c0/64 + k; column
    // quarter ni (32 columns) is half ni%2 of word ni/2.  n_pad is a multiple of 128,
    // so a 64-column word lies wholly inside or wholly past n_pad; columns past n_pad
    // (only in a tile wider than the padding granularity) hold zeros and are
    // neither counted nor stored.
    auto &Xt = EvalLds<EPI, KC, BN_>::xt();
    if constexpr (KEYS_LDS) {
        // the staged X words of the tile's columns, for the key epilogue
#pragma unroll
        for (int w = 0; w < BN / 64; w++) Xt[tid * (BN / 64) + w] = xt[w];
        __syncthreads();
    }
    constexpr int NWD = WTN / 64;  // X words of the wave's columns
    const int c0 = n0 + wc * WTN;
    if (c0 >= a.n_pad) return;
    bool wok[NWD];
#pragma unroll
    for (int k = 0; k < NWD; k++) wok[k] = c0 + 64 * k < a.n_pad;
    if constexpr (EPI == EPI_ROWDOT) {
        const int64_t wgt = plane == 0 ? a.weight0 : 1;
        // The triangle's K range ends at n0 + BN, so when the tile's columns span at
        // most two K steps they are the last two, whose LDS buffers are not written
        // after their barriers: the staged X words of the columns and the staged Q
        // block's diagonal (q_jj, kept by the k <= j mask) are read from LDS.
        constexpr bool LDS_EPI = TRI && ((KC >= BN && KC % BN == 0) || (BN <= 2 * KC && BN % KC == 0));
        int wbuf[NWD], woff[NWD];  // LDS buffer and word index of each 64-column group
#pragma unroll
        for (int k = 0; k < NWD; k++) {
            const int col = c0 + 64 * k, ks = col / KC;
            wbuf[k] = ks & 1;
            woff[k] = (col - ks * KC) >> 6;
        }
        int32_t dq[FN];  // this plane's q_jj of the lane's columns
#pragma unroll
        for (int ni = 0; ni < FN; ni++) {
            const int col = c0 + ni * 32 + r32;
            dq[ni] = 0;
            if (wok[ni >> 1]) {
                if constexpr (LDS_EPI)
                    dq[ni] = Bs[wbuf[ni >> 1]][(wc * WTN + ni * 32 + r32) * BPITCH + woff[ni >> 1] * 64 + (ni & 1) * 32 + r32];
                else
                    dq[ni] = ubqp_ldg1(qp + (int64_t)col * a.n_pad + col);
            }
        }
#pragma unroll
        for (int mi = 0; mi < FM; mi++) {
            int32_t sv[16];
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int rl = wr * WTM + mi * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                const int64_t row = m0 + rl;
                uint64_t xw[NWD];
#pragma unroll
                for (int k = 0; k < NWD; k++) {
                    xw[k] = 0;
                    if constexpr (LDS_EPI) {
                        if (wok[k]) xw[k] = As[wbuf[k]][rl * APITCH + woff[k]];
                    } else if (row < Mrows && wok[k] && word0_of(c0) + k < a.W) {
                        xw[k] = ubqp_ldg8(a.X + row * a.W + word0_of(c0) + k);
                    }
                }
                int s = 0;
#pragma unroll
                for (int ni = 0; ni < FN; ni++) {
                    const uint32_t q32 = (uint32_t)(xw[ni >> 1] >> (32 * (ni & 1)));
                    s += ((q32 >> r32) & 1u) ? 2 * acc[mi][ni][e] - dq[ni] : 0;
                }
                sv[e] = s;
            }
            // |s| <= 8 (2 * 128 n + 128) < 2^25: the 32-lane sums stay inside int32.
            // The 16 rows are reduced in lockstep so that the DPP steps of different
            // rows fill each other's wait states.  Every lane of a quad permutation or
            // a row rotation has a source lane, so bound_ctrl changes nothing but lets
            // the old value go unused.
#pragma unroll
            for (int e = 0; e < 16; e++) sv[e] += __builtin_amdgcn_update_dpp(0, sv[e], 0xB1, 0xF, 0xF, true);
#pragma unroll
            for (int e = 0; e < 16; e++) sv[e] += __builtin_amdgcn_update_dpp(0, sv[e], 0x4E, 0xF, 0xF, true);
#pragma unroll
            for (int e = 0; e < 16; e++) sv[e] += __builtin_amdgcn_update_dpp(0, sv[e], 0x124, 0xF, 0xF, true);
#pragma unroll
            for (int e = 0; e < 16; e++) sv[e] += __builtin_amdgcn_update_dpp(0, sv[e], 0x128, 0xF, 0xF, true);
#pragma unroll
            for (int e = 0; e < 16; e++) sv[e] += __shfl_xor(sv[e], 16);
            if (r32 == 0) {
#pragma unroll
                for (int e = 0; e < 16; e++) {
                    const int64_t row = m0 + wr * WTM + mi * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                    if (row < Mrows && sv[e] != 0) ubqp_atomic_add_i64(&a.f[row], wgt * (int64_t)sv[e]);
                }
            }
        }
    } else if constexpr (EPI == EPI_Y || SPLIT) {
        // rows of x Q per plane, or (split K) this part's raw partial rows
        int32_t *Yp = a.Y + (int64_t)plane * a.M * a.n_pad + prow * a.n_pad;
#pragma unroll
        for (int mi = 0; mi < FM; mi++) {
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int64_t row = m0 + wr * WTM + mi * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                if (row < Mrows) {
#pragma unroll
                    for (int ni = 0; ni < FN; ni++)
                        if (wok[ni >> 1]) Yp[row * a.n_pad + c0 + ni * 32 + r32] = acc[mi][ni][e];
                }
            }
        }
    } else if constexpr (EPI == EPI_KEYS) {
        // Ascent keys of the single-plane problem: with y = (x Q)_j and s = 1 - 2 x_j,
        // Delta_j = q_jj + 2 s y_j, key_j = Delta_j * 256 + 32 (7 - j / 1024) +
        // 2 (15 - j mod 16) + x_j (the ascent lane's block of 1024 columns above the
        // column's place in its 16).
        int32_t tb[FN];
#pragma unroll
        for (int ni = 0; ni < FN; ni++) {
            const int col = c0 + ni * 32 + r32;
            tb[ni] = 32 * (7 - (col >> 10)) + 2 * (15 - (col & 15));
        }
#pragma unroll
        for (int mi = 0; mi < FM; mi++) {
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int rl = wr * WTM + mi * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                const int64_t row = m0 + rl;
                if (row < Mrows) {
                    uint64_t xw[NWD];
#pragma unroll
                    for (int k = 0; k < NWD; k++) {
                        if constexpr (KEYS_LDS) {
                            xw[k] = Xt[rl * (BN / 64) + wc * NWD + k];
                        } else {
                            const int64_t xr = a.rows[row];
                            const bool ok = xr >= 0 && xr < a.x_rows && word0_of(c0) + k < a.W;
                            xw[k] = ok ? a.X[xr * a.W + word0_of(c0) + k] : 0ull;
                        }
                    }
#pragma unroll
                    for (int ni = 0; ni < FN; ni++) {
                        if (!wok[ni >> 1]) continue;
                        const int col = c0 + ni * 32 + r32;
                        const uint32_t q32 = (uint32_t)(xw[ni >> 1] >> (32 * (ni & 1)));
                        const int32_t xj = (int32_t)((q32 >> r32) & 1u);
                        const int32_t y2 = 2 * acc[mi][ni][e];
                        const int32_t delta = dg[ni] + (xj ? -y2 : y2);
                        a.Y[row * a.n_pad + col] = delta * 256 + tb[ni] + xj;
                    }
                }
            }
        }
    }
}

// The Delta initialisation splits K (ubqp_dinit_split) for this launch's device row count.
template <int EPI> __device__ inline bool eval_split_of(const EvalArgs &a)
{
    if constexpr (EPI == EPI_ROWDOT) {
        return false;
    } else {
        if (a.split_target <= 0) return false;
        const int64_t k = *a.nrows_d - a.offset, P = k < a.M ? k : a.M;
        return ubqp_dinit_split(P, a.M, a.n_pad, a.planes, a.split_team_max, a.split_target) > 1;
    }
}

// Narrow tiles (BN = 128) with KC = 64 and 128 fit two workgroups per CU (LDS 28 /
// 48 KB); KC = 256 (90 KB) one.  Wide tiles (BN = 256) hold 256 accumulators per
// lane: one workgroup per CU.
template <int KC, int BN> constexpr int eval_min_blocks() { return (BN == 128 && KC <= 128) ? 2 : 1; }

template <int EPI, int KC, int BN, int WR>
__global__ __launch_bounds__(THR, (eval_min_blocks<KC, BN>())) void eval_kernel(EvalArgs a, int64_t total)
{
    const int64_t tile = xcd_tile(blockIdx.x, total);
    if (eval_split_of<EPI>(a)) eval_body<EPI, KC, BN, WR, true>(a, tile);
    else eval_body<EPI, KC, BN, WR, false>(a, tile);
}

template <int EPI, int KC, int BN, int WR>
__global__ __launch_bounds__(THR, (eval_min_blocks<KC, BN>())) void eval_batched(const EvalArgs *args,
                                                                              const int64_t *prefix, int count,
                                                                              int64_t total)
{
    const int64_t t = xcd_tile(blockIdx.x, total);
    const int i = ubqp_find_inst(prefix, count, t);
    const EvalArgs a = args[i];  // a local copy: fields stay in registers across stores
    if (eval_split_of<EPI>(a)) eval_body<EPI, KC, BN, WR, true>(a, t - prefix[i]);
    else eval_body<EPI, KC, BN, WR, false>(a, t - prefix[i]);
}

// f[c] = bias * popcount(X_c)^2 (the constant part of the split planes) or 0.
__device__ void eval_init_body(const EvalArgs &a, int64_t bid)
{
    const int64_t c = bid * 256 + threadIdx.x;
    if (c >= a.M) return;
    int64_t v = 0;
    if (a.bias) {
        int64_t k = 0;
        for (int w = 0; w < a.W; w++) k += __popcll(a.X[c * a.W + w]);
        v = a.bias * k * k;
    }
    a.f[c] = v;
}

__global__ __launch_bounds__(256) void eval_init(EvalArgs a) { eval_init_body(a, blockIdx.x); }

__global__ __launch_bounds__(256) void eval_init_batched(const EvalArgs *args, const int64_t *prefix, int count)
{
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const EvalArgs a = args[i];
    eval_init_body(a, blockIdx.x - prefix[i]);
}

// K depth and tile geometry of the Delta-initialisation contractions (Y rows and keys).
#ifndef EVAL_KC
#define EVAL_KC 128
#endif
#ifndef YROWS_BN
#define YROWS_BN 128
#endif
#define YROWS_WR (YROWS_BN == 128 ? 4 : 2)

}  // namespace

EvalArgs ubqp_eval_args(const ubqp_problem *p, const uint64_t *X, int64_t M, int64_t *f)
{
    EvalArgs a{};
    a.q = p->q;
    a.plane_stride = (int64_t)p->n_pad * p->n_pad;
    a.n_pad = p->n_pad;
    a.planes = p->planes;
    a.X = X;
    a.W = p->W;
    a.M = M;
    a.x_rows = M;
    a.f = f;
    a.weight0 = p->weight0;
    a.bias = p->bias;
    a.m_tiles = (int32_t)((M + BM - 1) / BM);
    a.n_tiles = p->n_pad / UBQP_NPAD_ALIGN;  // column tiles of 128; ubqp_eval_set_variant sets a variant's
    return a;
}

EvalArgs ubqp_yrows_args(const ubqp_problem *p, const uint64_t *X, int64_t x_rows, const int32_t *rows,
                         const int64_t *nrows_d, int64_t offset, int64_t cap, int32_t *Y)
{
    EvalArgs a = ubqp_eval_args(p, X, cap, nullptr);
    a.x_rows = x_rows;
    a.rows = rows + offset;
    a.nrows_d = nrows_d;
    a.offset = offset;
    a.Y = Y;
    a.diag = p->diag;
    a.n_tiles = (p->n_pad + YROWS_BN - 1) / YROWS_BN;
    return a;
}

int64_t ubqp_eval_tiles(const EvalArgs &a) { return (int64_t)a.m_tiles * a.n_tiles * a.planes; }
int64_t ubqp_yrows_tiles(const EvalArgs &a)
{
    return (int64_t)a.m_tiles * a.n_tiles * (a.planes == 1 ? 1 : a.planes);
}
int64_t ubqp_eval_init_blocks(const EvalArgs &a) { return (a.M + 255) / 256; }

// Variants of the row-dot contraction: tiles of 256 x 128 (waves of 64 x 128)
// staging K 64, 128 or 256 deep; even variants order tiles n-tile-major, odd ones
// m-tile-major.  (Tiles of 256 x 256 columns with waves of 64 x 256 or 128 x 128,
// one workgroup per CU, compute the same integers but were measured slower at
// every n from 1024 to 8192, 0.56 against 0.49 ms at n = 7000, M = 16384: with one
// wave per SIMD the staging and the per-K-step barrier are no longer hidden.)
int ubqp_eval_variant_kc(int variant) { return variant / 2 == 0 ? 64 : variant / 2 == 1 ? 128 : 256; }
int ubqp_eval_variant_bn(int variant)
{
    (void)variant;
    return 128;
}

void ubqp_eval_set_variant(EvalArgs &a, int variant)
{
    a.order = variant & 1;
    const int bn = ubqp_eval_variant_bn(variant);
    a.n_tiles = (a.n_pad + bn - 1) / bn;
}

#define EVAL_VARIANT_SWITCH(LAUNCH)                 \
    switch (variant) {                              \
    case 0: case 1: LAUNCH(64, 128, 4); break;      \
    case 2: case 3: LAUNCH(128, 128, 4); break;     \
    default: LAUNCH(256, 128, 4); break;            \
    }

hipError_t ubqp_launch_eval_v(hipStream_t st, EvalArgs a, int variant)
{
    ubqp_eval_set_variant(a, variant);
    hipLaunchKernelGGL(eval_init, dim3((unsigned)ubqp_eval_init_blocks(a)), dim3(256), 0, st, a);
    const int64_t T = ubqp_eval_tiles(a);
#define L(KC, BN, WR) hipLaunchKernelGGL((eval_kernel<EPI_ROWDOT, KC, BN, WR>), dim3((unsigned)T), dim3(THR), 0, st, a, T)
    EVAL_VARIANT_SWITCH(L)
#undef L
    return hipGetLastError();
}

hipError_t ubqp_launch_eval_rowdot_batch(hipStream_t st, int variant, const EvalArgs *args, const int64_t *prefix,
                                         int count, int64_t tiles)
{
    if (tiles <= 0) return hipSuccess;
    const dim3 g((unsigned)tiles), b(THR);
#define L(KC, BN, WR) hipLaunchKernelGGL((eval_batched<EPI_ROWDOT, KC, BN, WR>), g, b, 0, st, args, prefix, count, tiles)
    EVAL_VARIANT_SWITCH(L)
#undef L
    return hipGetLastError();
}

hipError_t ubqp_launch_yrows(hipStream_t st, const EvalArgs &a)
{
    const int64_t T = ubqp_yrows_tiles(a);
    if (a.planes == 1)
        hipLaunchKernelGGL((eval_kernel<EPI_KEYS, EVAL_KC, YROWS_BN, YROWS_WR>), dim3((unsigned)T), dim3(THR), 0, st, a, T);
    else
        hipLaunchKernelGGL((eval_kernel<EPI_Y, EVAL_KC, YROWS_BN, YROWS_WR>), dim3((unsigned)T), dim3(THR), 0, st, a, T);
    return hipGetLastError();
}

hipError_t ubqp_launch_eval_init_batch(hipStream_t st, const EvalArgs *args, const int64_t *prefix, int count,
                                       int64_t blocks)
{
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(eval_init_batched, dim3((unsigned)blocks), dim3(256), 0, st, args, prefix, count);
    return hipGetLastError();
}

hipError_t ubqp_launch_eval_batch(hipStream_t st, int epilogue, const EvalArgs *args, const int64_t *prefix,
                                  int count, int64_t tiles)
{
    if (tiles <= 0) return hipSuccess;
    switch (epilogue) {
    case EPI_ROWDOT:
        hipLaunchKernelGGL((eval_batched<EPI_ROWDOT, EVAL_KC, 128, 4>), dim3((unsigned)tiles), dim3(THR), 0, st, args,
                           prefix, count, tiles);
        break;
    case EPI_Y:
        hipLaunchKernelGGL((eval_batched<EPI_Y, EVAL_KC, YROWS_BN, YROWS_WR>), dim3((unsigned)tiles), dim3(THR), 0, st,
                           args, prefix, count, tiles);
        break;
    default:
        hipLaunchKernelGGL((eval_batched<EPI_KEYS, EVAL_KC, YROWS_BN, YROWS_WR>), dim3((unsigned)tiles), dim3(THR), 0,
                           st, args, prefix, count, tiles);
        break;
    }
    return hipGetLastError();
}

extern "C" int ubqp_eval_ops(const ubqp_problem *p, int64_t M, double *executed, double *dense)
{
    if (!p || M < 1 || M > UBQP_MAX_M) return UBQP_EINVAL;
    const int v = ubqp_eval_variant_for(p, M);
    const int KC = ubqp_eval_variant_kc(v), BN = ubqp_eval_variant_bn(v);
    const int64_t rows = (M + BM - 1) / BM * BM;  // whole row tiles run their matrix ops
    const int nk_full = (p->n_pad + KC - 1) / KC;
    double macs = 0.0;
    for (int nt = 0; nt * BN < p->n_pad; nt++) {
        const int nk = min(nk_full, (nt * BN + BN + KC - 1) / KC);  // lower triangle: K over [0, n0 + BN)
        macs += (double)BN * nk * KC;  // every wave runs the K loop, columns past n_pad included
    }
    if (executed) *executed = 2.0 * macs * (double)rows * p->planes;
    if (dense) *dense = 2.0 * (double)p->n * p->n * (double)M * p->planes;
    return UBQP_OK;
}
