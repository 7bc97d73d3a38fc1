// Steepest 1-flip ascent of the screened candidates (Pseudocode section; the
// 1-flip deltas of Glover et al. 2002), one wave64 per candidate, every flip
// on-chip: one Q row read per flip, no LDS, no barrier.
//
// With s_i = 1 - 2 x_i and Delta_i = f(x xor e_i) - f(x), flipping x_k (whose
// old sign is d = s_k) changes Delta_i by 2 q_ik s_i d for i != k and negates
// Delta_k.  The matrix read per flip is Q with a zero diagonal (the "ascent
// matrix", built once at upload) so the row update leaves Delta_k to the
// explicit negation.
//
// int8 Q (ascent_i8): lane l owns the columns 1024 b + 16 l + t (block b < NB,
// t < 16), so each 16-byte row load of the wave is one contiguous KB, and keeps
// for each of them the 32-bit key
//     key_i = Delta_i * 256 + 32 (7 - b) + 2 (15 - t) + x_i     (|Delta_i| < 2^21)
// and the sign s_i as a signed byte (four per VGPR).  A flip is
//     key_i += (q_ik * s_i) * 512 d  -- one SDWA v_mul_i32_i24 (byte x byte,
//                                       both sign-extended) and one v_mad_i32_i24
// with 512 d in an SGPR, so the lane's best key is a v_max3 tree (the largest
// Delta, then the lowest block, then the lowest t), the wave's best (Delta, block)
// one DPP max of key >> 5, and the lowest column attaining the largest Delta the
// lowest lane attaining that pair (ballot + ffs), with t and the old x_k read from
// its key.  The flipped variable's key and sign are rewritten through one
// uniform-indexed register access per block.
//
// int16 Q (ascend_i16): lane l owns the contiguous columns [l PL, (l+1) PL),
// PL = 16 NB, keeps Delta_i itself (|Delta_i| < 2^30 leaves no room for a column
// in 32 bits) and s_i as a byte, and finds the lowest column attaining the largest
// Delta by the lowest lane, then that lane's lowest block and column.
//
// The starting deltas come from Y = X Q on the passers (the matrix-core kernel):
//     y_i = w0 Y0_i + Y1_i + bias * popcount(x)   (bias / Y1 only when split)
//     g_i = 2 y_i + q_ii (1 - 2 x_i).
#include "ubqp_internal.h"

namespace {

// s_waitcnt vmcnt(0) lgkmcnt(0) (expcnt left at its maximum), as the builtin's
// immediate.  Issued before a flip loop: flat accesses still in flight there
// (argument tables, the previous candidate's results) would otherwise make the
// compiler wait for every load in flight at each flip instead of for the row
// block it needs.
constexpr unsigned WAIT_VM_LGKM_0 = 0x0070;


typedef int32_t v16i __attribute__((ext_vector_type(16)));



// Eight keys of one 16-column block (columns 8 h .. 8 h + 7): key += (q * s) * step
// for q the signed bytes of q01 = {w0, w1} and s the signed bytes of the sign words
// {u0, u1}.  One asm statement per eight columns, so no wait states are inserted
// between the multiply-add pairs, and four products in flight.
__device__ inline void update_keys8(int32_t &k0, int32_t &k1, int32_t &k2, int32_t &k3, int32_t &k4, int32_t &k5,
                                    int32_t &k6, int32_t &k7, uint32_t w0, uint32_t w1, uint32_t u0, uint32_t u1,
                                    int32_t step)
{
    int32_t t0, t1, t2, t3;
    asm("v_mul_i32_i24_sdwa %8, sext(%12), sext(%14) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_0 src1_sel:BYTE_0\n\t"
        "v_mul_i32_i24_sdwa %9, sext(%12), sext(%14) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_1 src1_sel:BYTE_1\n\t"
        "v_mul_i32_i24_sdwa %10, sext(%12), sext(%14) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_2 src1_sel:BYTE_2\n\t"
        "v_mul_i32_i24_sdwa %11, sext(%12), sext(%14) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_3 src1_sel:BYTE_3\n\t"
        "v_mad_i32_i24 %0, %8, %16, %0\n\t"
        "v_mad_i32_i24 %1, %9, %16, %1\n\t"
        "v_mad_i32_i24 %2, %10, %16, %2\n\t"
        "v_mad_i32_i24 %3, %11, %16, %3\n\t"
        "v_mul_i32_i24_sdwa %8, sext(%13), sext(%15) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_0 src1_sel:BYTE_0\n\t"
        "v_mul_i32_i24_sdwa %9, sext(%13), sext(%15) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_1 src1_sel:BYTE_1\n\t"
        "v_mul_i32_i24_sdwa %10, sext(%13), sext(%15) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_2 src1_sel:BYTE_2\n\t"
        "v_mul_i32_i24_sdwa %11, sext(%13), sext(%15) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_3 src1_sel:BYTE_3\n\t"
        "v_mad_i32_i24 %4, %8, %16, %4\n\t"
        "v_mad_i32_i24 %5, %9, %16, %5\n\t"
        "v_mad_i32_i24 %6, %10, %16, %6\n\t"
        "v_mad_i32_i24 %7, %11, %16, %7"
        : "+v"(k0), "+v"(k1), "+v"(k2), "+v"(k3), "+v"(k4), "+v"(k5), "+v"(k6), "+v"(k7), "=&v"(t0), "=&v"(t1),
          "=&v"(t2), "=&v"(t3)
        : "v"(w0), "v"(w1), "v"(u0), "v"(u1), "s"(step));
}

// Largest of 16 values: a balanced tree of three-input maxima.
__device__ inline int32_t max16(const v16i &v)
{
    const int32_t a = max(max(v[0], v[1]), v[2]), b = max(max(v[3], v[4]), v[5]);
    const int32_t c = max(max(v[6], v[7]), v[8]), d = max(max(v[9], v[10]), v[11]);
    const int32_t e = max(max(v[12], v[13]), v[14]);
    const int32_t ab = max(max(a, b), c), de = max(max(d, e), v[15]);
    return max(ab, de);
}

// Largest of the lane's 16 NB keys: chains of three-input maxima over groups of
// 15 keys (each maximum takes two new keys) and a group of the rest, then a tree
// over the groups' results -- ceil((16 NB - 1) / 2) instructions in all.
template <int NB> __device__ inline int32_t lane_max(const v16i (&kk)[NB])
{
    constexpr int N = 16 * NB, G = N / 15, R = N - 15 * G;
    int32_t acc[G + 1];
#pragma unroll
    for (int g = 0; g <= G; g++) {
        const int lo = 15 * g, cnt = g < G ? 15 : R;
        if (cnt == 0) continue;
        int32_t m = kk[lo / 16][lo % 16];
        int k = 1;
        if (cnt % 2 == 0) {
            m = max(m, kk[(lo + 1) / 16][(lo + 1) % 16]);
            k = 2;
        }
#pragma unroll
        for (; k + 1 < cnt + 1; k += 2)
            m = max(max(m, kk[(lo + k) / 16][(lo + k) % 16]), kk[(lo + k + 1) / 16][(lo + k + 1) % 16]);
        acc[g] = m;
    }
    constexpr int A = R > 0 ? G + 1 : G;
    int32_t best = acc[0];
    int a = 1;
    if (A % 2 == 0) {
        best = max(best, acc[1]);
        a = 2;
    }
#pragma unroll
    for (; a + 1 < A + 1; a += 2) best = max(max(best, acc[a]), acc[a + 1]);
    return best;
}

// Largest value over the wave (DPP within rows of 16, then across rows by row broadcasts).
// Lanes a step does not write (the rows outside a broadcast's row mask) take
// INT32_MIN, the identity of max, so each step compiles to one v_max_i32 with a DPP
// operand rather than a copy, a DPP move and a maximum.
__device__ inline int32_t wave_max_i32(int32_t v)
{
    constexpr int32_t LO = INT32_MIN;
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0x124, 0xF, 0xF, false));  // row_ror:4
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0x128, 0xF, 0xF, false));  // row_ror:8
    // every lane holds its row's maximum; fold the rows into the last one
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0x142, 0xA, 0xF, false));  // row_bcast:15 into rows 1, 3
    v = max(v, __builtin_amdgcn_update_dpp(LO, v, 0x143, 0xC, 0xF, false));  // row_bcast:31 into rows 2, 3
    return __builtin_amdgcn_readlane(v, 63);
}

// Column ownership of the int8 ascent: lane l owns 1024 b + 16 l + t.  The block
// sits in the key above t, so the lowest column attaining the largest Delta is the
// lowest (block, lane, t) and needs no reduction beyond the wave maximum.
template <int NB> __device__ inline int asc_col0(int lane, int b) { return 1024 * b + 16 * lane; }
// The key's tie-break part of column 1024 b + 16 l + t (bits 1..7).
__device__ inline int32_t asc_tie(int b, int t) { return 32 * (7 - b) + 2 * (15 - t); }

template <int NB>
__device__ void ascend_i8(const AscArgs &a, int64_t p, int lane)
{
    const int64_t c = a.idx[a.offset + p];
    if (c < 0 || c >= a.x_rows) {
        if (lane == 0) atomicOr(a.err, 2);
        return;
    }
    uint64_t *xr = a.X + c * a.W;
    // key_i = Delta_i * 256 + 32 (7 - b) + 2 (15 - t) + x_i: the largest key is the
    // largest Delta, then the lowest block, then the lowest t; bit 0 carries x_i.
    v16i kk[NB];
    // s_i = 1 - 2 x_i as signed bytes, four per register
    uint32_t ss[NB][4];
    // keys of this lane's columns from the matrix-core epilogue; columns past n_pad
    // (Delta = 0, x = 0) are synthesised
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int col0 = asc_col0<NB>(lane, b);
        const bool in = col0 < a.n_pad;
        const int32_t *yrow = a.Y + p * a.n_pad + col0;
#pragma unroll
        for (int t4 = 0; t4 < 4; t4++) {
            int4 v = {0, 0, 0, 0};
            if (in) v = ubqp_ldg16i(yrow + 4 * t4);
            const int32_t kv[4] = {v.x, v.y, v.z, v.w};
            uint32_t sw = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int t = 4 * t4 + k;
                const int32_t key = in ? kv[k] : asc_tie(b, t);
                kk[b][t] = key;
                sw |= ((key & 1) ? 0xFFu : 0x01u) << (8 * k);
            }
            ss[b][t4] = sw;
        }
    }

    const int8_t *qa = (const int8_t *)a.qa;
    // the gain is summed from zero and f read only after the loop: a load still in
    // flight at the loop's first use (f is read through a flat pointer) would put a
    // wait on all memory into every flip
    int64_t gain = 0;
    int32_t flips = 0;
    const int32_t cap = a.max_flips > 0 ? a.max_flips : a.safety_cap;
    int32_t V;
    __builtin_amdgcn_s_waitcnt(WAIT_VM_LGKM_0);
    for (;;) {
        const int32_t best = lane_max<NB>(kk);
        const int32_t ld = best >> 5;           // Delta * 8 + 7 - block
        V = wave_max_i32(ld);
        if ((V >> 3) <= 0 || flips >= cap) break;
        // among the lanes holding the largest Delta in the lowest block, the lowest
        // lane holds the lowest column
        const int lstar = __ffsll((unsigned long long)__ballot(ld == V)) - 1;
        const int32_t bk = __builtin_amdgcn_readlane(best, lstar);
        const int bs = 7 - ((bk >> 5) & 7), ts = 15 - ((bk >> 1) & 15);
        const int32_t xk = bk & 1;              // x_k before the flip
        const int K = asc_col0<NB>(lstar, bs) + ts;
        // row k is read first: its latency is the flip's critical path
        const int8_t *row = qa + (int64_t)K * a.ncol_a;
        uint4 w[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) w[b] = ubqp_ldg16(row + asc_col0<NB>(lane, b));
        const int32_t dk = V >> 3;              // Delta_k
        // the flipped variable: Delta_k -> -Delta_k, x_k and s_k toggle (lane lstar only)
        const bool own = lane == lstar;
        const int32_t knew = -dk * 256 + (bk & 0xFE) + (1 - xk);
        const uint32_t sflip = own ? 0xFEu << (8 * (ts & 3)) : 0u;  // +1 <-> -1 as a byte
#pragma unroll
        for (int b = 0; b < NB; b++) {
            if (b == bs) {
                const int32_t ko = kk[b][ts];
                kk[b][ts] = own ? knew : ko;
#pragma unroll
                for (int r = 0; r < 4; r++) ss[b][r] ^= (r == (ts >> 2)) ? sflip : 0u;
            }
        }
        gain += dk;
        flips++;
        // Delta_i += 2 d s_i q_ik for i != k, with d = 1 - 2 x_k: key_i += (q_ik s_i) * 512 d
        const int32_t step = xk ? -512 : 512;
        // the update is the VALU burst of a flip; with the wave's priority raised
        // while it runs, the SIMD's other wave fills the gaps its loads leave
        // rather than stretching it
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int b = 0; b < NB; b++) {
            int32_t k[16];
#pragma unroll
            for (int t = 0; t < 16; t++) k[t] = kk[b][t];
            update_keys8(k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7], w[b].x, w[b].y, ss[b][0], ss[b][1], step);
            update_keys8(k[8], k[9], k[10], k[11], k[12], k[13], k[14], k[15], w[b].z, w[b].w, ss[b][2], ss[b][3],
                         step);
#pragma unroll
            for (int t = 0; t < 16; t++) kk[b][t] = k[t];
        }
        __builtin_amdgcn_s_setprio(0);
    }
    if ((V >> 3) > 0 && a.max_flips == 0 && lane == 0) atomicOr(a.err, 1);  // safety cap reached

#pragma unroll
    for (int b = 0; b < NB; b++) {
        uint32_t bits = 0;
#pragma unroll
        for (int t = 0; t < 16; t++) bits |= ((uint32_t)kk[b][t] & 1u) << t;
        const int ci = asc_col0<NB>(lane, b) >> 4;
        if (ci < 4 * a.W) ((uint16_t *)xr)[ci] = (uint16_t)bits;
    }
    if (lane == 0) {
        a.f[c] += gain;
        a.flips[c] = flips;
    }
}

// Eight deltas (columns 8 h .. 8 h + 7 of a 16-column block): delta += (q * s) * step
// for q the signed words of {q0..q3} (two columns per word) and s the signed bytes
// of {u0, u1}; one asm statement, four products in flight.
__device__ inline void update_deltas8(int32_t &d0, int32_t &d1, int32_t &d2, int32_t &d3, int32_t &d4, int32_t &d5,
                                      int32_t &d6, int32_t &d7, uint32_t q0, uint32_t q1, uint32_t q2, uint32_t q3,
                                      uint32_t u0, uint32_t u1, int32_t step)
{
    int32_t t0, t1, t2, t3;
    asm("v_mul_i32_i24_sdwa %8, sext(%12), sext(%16) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:BYTE_0\n\t"
        "v_mul_i32_i24_sdwa %9, sext(%12), sext(%16) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:BYTE_1\n\t"
        "v_mul_i32_i24_sdwa %10, sext(%13), sext(%16) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:BYTE_2\n\t"
        "v_mul_i32_i24_sdwa %11, sext(%13), sext(%16) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:BYTE_3\n\t"
        "v_mad_i32_i24 %0, %8, %18, %0\n\t"
        "v_mad_i32_i24 %1, %9, %18, %1\n\t"
        "v_mad_i32_i24 %2, %10, %18, %2\n\t"
        "v_mad_i32_i24 %3, %11, %18, %3\n\t"
        "v_mul_i32_i24_sdwa %8, sext(%14), sext(%17) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:BYTE_0\n\t"
        "v_mul_i32_i24_sdwa %9, sext(%14), sext(%17) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:BYTE_1\n\t"
        "v_mul_i32_i24_sdwa %10, sext(%15), sext(%17) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:BYTE_2\n\t"
        "v_mul_i32_i24_sdwa %11, sext(%15), sext(%17) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:BYTE_3\n\t"
        "v_mad_i32_i24 %4, %8, %18, %4\n\t"
        "v_mad_i32_i24 %5, %9, %18, %5\n\t"
        "v_mad_i32_i24 %6, %10, %18, %6\n\t"
        "v_mad_i32_i24 %7, %11, %18, %7"
        : "+v"(d0), "+v"(d1), "+v"(d2), "+v"(d3), "+v"(d4), "+v"(d5), "+v"(d6), "+v"(d7), "=&v"(t0), "=&v"(t1),
          "=&v"(t2), "=&v"(t3)
        : "v"(q0), "v"(q1), "v"(q2), "v"(q3), "v"(u0), "v"(u1), "s"(step));
}


// int16 Q: |Delta| < 2^30, too wide to share 32 bits with a column index, so the
// lane keeps Delta_i itself (and s_i as a byte) for its contiguous columns
// [l PL, (l+1) PL).  Per flip: the maximum of each 16-column block, the lane's
// and the wave's maximum V; the lowest lane attaining V, then (in that lane) its
// lowest block and lowest column attaining V -- the lowest global column.  The
// update is one SDWA multiply (q word x s byte) and one mad by the uniform 2 d.
// T = UBQP_TEAM: the team layout of ascend_i8_team (four waves per passer, each
// flip's best of the waves combined through LDS); T = 1: one wave.
template <int NB, int T>
__device__ void ascend_i16(const AscArgs &a, int64_t p, int wv, int lane, int2 (*slots)[UBQP_TEAM], int S = 1,
                           int64_t prs = 0)
{
    constexpr int PL = 16 * NB;
    const int vl = wv * 64 + lane;  // virtual lane
    const int64_t c = a.idx[a.offset + p];
    if (c < 0 || c >= a.x_rows) {  // the same for every wave of a team
        if (vl == 0) atomicOr(a.err, 2);
        return;
    }
    uint64_t *xr = a.X + c * a.W;
    const int col_base = vl * PL;
    // popcount(x) for the constant part of the split planes
    int pc = 0;
    for (int w = lane; w < a.W; w += 64) pc += __popcll(xr[w]);
    for (int o = 32; o > 0; o >>= 1) pc += __shfl_xor(pc, o);
    v16i dl[NB];
    uint32_t ss[NB][4];
    const int64_t ystride = a.max_idx * a.n_pad;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int col0 = col_base + 16 * b;
        const bool in = col0 < a.n_pad;
        uint32_t bits = 0;
        if (in) {
            const int w = col0 >> 6;
            if (w < a.W) bits = (uint32_t)(xr[w] >> (col0 & 63)) & 0xFFFFu;
        }
#pragma unroll
        for (int t4 = 0; t4 < 4; t4++) {
            int4 v0 = {0, 0, 0, 0}, v1 = {0, 0, 0, 0}, dg = {0, 0, 0, 0};
            if (in) {
                // split K (team kernels only): the sum of the S partial rows of each plane
                for (int s = 0; s < S; s++) {
                    const int64_t r = (p + (int64_t)s * prs) * a.n_pad + col0 + 4 * t4;
                    const int4 u0 = ubqp_ldg16i(a.Y + r), u1 = ubqp_ldg16i(a.Y + ystride + r);
                    v0.x += u0.x; v0.y += u0.y; v0.z += u0.z; v0.w += u0.w;
                    v1.x += u1.x; v1.y += u1.y; v1.z += u1.z; v1.w += u1.w;
                }
                dg = ubqp_ldg16i(a.diag + col0 + 4 * t4);
            }
            const int32_t y0[4] = {v0.x, v0.y, v0.z, v0.w}, y1[4] = {v1.x, v1.y, v1.z, v1.w};
            const int32_t d[4] = {dg.x, dg.y, dg.z, dg.w};
            uint32_t sw = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int t = 4 * t4 + k;
                const bool xi = (bits >> t) & 1u;
                // y = (x Q)_j = 256 Y_hi + Y_lo + 128 popcount(x); g = 2 y + q_jj (1 - 2 x_j)
                const int32_t y = (int32_t)a.weight0 * y0[k] + y1[k] + (int32_t)a.bias * pc;
                const int32_t g = 2 * y + (xi ? -d[k] : d[k]);
                // padding columns (j >= n) keep Delta = 0, so they are never taken
                dl[b][t] = (in && col0 + t < a.n) ? (xi ? -g : g) : 0;
                sw |= (xi ? 0xFFu : 0x01u) << (8 * k);
            }
            ss[b][t4] = sw;
        }
    }

    const int16_t *qa = (const int16_t *)a.qa;
    // the gain is summed from zero and f read only after the loop: a load still in
    // flight at the loop's first use (f is read through a flat pointer) would put a
    // wait on all memory into every flip
    int64_t gain = 0;
    int32_t flips = 0;
    const int32_t cap = a.max_flips > 0 ? a.max_flips : a.safety_cap;
    int32_t V;
    int par = 0;
    __builtin_amdgcn_s_waitcnt(WAIT_VM_LGKM_0);
    for (;;) {
        int32_t bm[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) bm[b] = max16(dl[b]);
        int32_t best = bm[0];
#pragma unroll
        for (int b = 1; b < NB; b++) best = max(best, bm[b]);
        V = wave_max_i32(best);
        if (T == 1 && (V <= 0 || flips >= cap)) break;
        const int lstar = __ffsll((unsigned long long)__ballot(best == V)) - 1;
        int bsel = NB - 1;
#pragma unroll
        for (int b = NB - 2; b >= 0; b--) bsel = bm[b] == V ? b : bsel;
        const int bs = __builtin_amdgcn_readlane(bsel, lstar);
        int tsel = 15;
        uint32_t sword = 0;
#pragma unroll
        for (int b = 0; b < NB; b++) {
            if (b == bs) {
#pragma unroll
                for (int t = 14; t >= 0; t--) tsel = dl[b][t] == V ? t : tsel;
            }
        }
        const int ts = __builtin_amdgcn_readlane(tsel, lstar);
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                if (b == bs && r == (ts >> 2)) sword = ss[b][r];
        const uint32_t sk = (uint32_t)__builtin_amdgcn_readlane((int)sword, lstar);
        int32_t xk = ((sk >> (8 * (ts & 3))) & 0xFFu) == 0xFFu;   // x_k before the flip
        int K = (wv * 64 + lstar) * PL + 16 * bs + ts;
        bool own = lane == lstar;
        if constexpr (T > 1) {
            // the team's flip: the largest Delta of the waves, the lowest wave on ties
            if (lane == 0) slots[par][wv] = int2{V, K | (xk << 30)};
            __syncthreads();
            int2 win = slots[par][0];
#pragma unroll
            for (int u = 1; u < T; u++) {
                const int2 o = slots[par][u];
                win = o.x > win.x ? o : win;
            }
            par ^= 1;
            V = win.x;
            if (V <= 0 || flips >= cap) break;
            K = win.y & 0x3FFFFFFF;
            xk = (win.y >> 30) & 1;
            own = vl == K / PL;
        }
        // row k, read first (its latency is the flip's critical path) except by one
        // wave at NB >= 7, whose registers cannot hold the row across the flipped
        // column's update
        const int16_t *row = qa + (int64_t)K * a.ncol_a + col_base;
        uint4 w[NB][2];
        auto read_row = [&]() {
            // a team's virtual lanes can reach past the row's ncol_a columns
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const bool in = T == 1 || col_base + 16 * b < a.ncol_a;
                w[b][0] = in ? ubqp_ldg16(row + 16 * b) : uint4{0u, 0u, 0u, 0u};
                w[b][1] = in ? ubqp_ldg16(row + 16 * b + 8) : uint4{0u, 0u, 0u, 0u};
            }
        };
        constexpr bool EARLY = T > 1 || NB <= 6;
        if constexpr (EARLY) read_row();
        const int bs_k = (K % PL) >> 4, ts_k = K & 15;
        const uint32_t sflip = own ? 0xFEu << (8 * (ts_k & 3)) : 0u;
#pragma unroll
        for (int b = 0; b < NB; b++) {
            if (b == bs_k) {
                const int32_t ko = dl[b][ts_k];
                dl[b][ts_k] = own ? -V : ko;
#pragma unroll
                for (int r = 0; r < 4; r++) ss[b][r] ^= (r == (ts_k >> 2)) ? sflip : 0u;
            }
        }
        gain += V;
        flips++;
        // Delta_i += 2 d s_i q_ik for i != k, d = 1 - 2 x_k (the ascent matrix has q_kk = 0)
        const int32_t step = xk ? -2 : 2;
        if constexpr (!EARLY) read_row();
        __builtin_amdgcn_s_setprio(1);  // as in the int8 ascent
#pragma unroll
        for (int b = 0; b < NB; b++) {
            int32_t d[16];
#pragma unroll
            for (int t = 0; t < 16; t++) d[t] = dl[b][t];
            update_deltas8(d[0], d[1], d[2], d[3], d[4], d[5], d[6], d[7], w[b][0].x, w[b][0].y, w[b][0].z,
                           w[b][0].w, ss[b][0], ss[b][1], step);
            update_deltas8(d[8], d[9], d[10], d[11], d[12], d[13], d[14], d[15], w[b][1].x, w[b][1].y, w[b][1].z,
                           w[b][1].w, ss[b][2], ss[b][3], step);
#pragma unroll
            for (int t = 0; t < 16; t++) dl[b][t] = d[t];
        }
        __builtin_amdgcn_s_setprio(0);
    }
    if (V > 0 && a.max_flips == 0 && vl == 0) atomicOr(a.err, 1);  // flip limit reached

#pragma unroll
    for (int b = 0; b < NB; b++) {
        uint32_t bits = 0;
#pragma unroll
        for (int t = 0; t < 16; t++) bits |= (((ss[b][t >> 2] >> (8 * (t & 3))) & 0xFFu) == 0xFFu ? 1u : 0u) << t;
        const int ci = vl * NB + b;
        if (ci < 4 * a.W) ((uint16_t *)xr)[ci] = (uint16_t)bits;
    }
    if (vl == 0) {
        a.f[c] += gain;
        a.flips[c] = flips;
    }
    // the next passer's first flip writes slot set 0, which slower waves of the team
    // may still be reading in this passer's last flip
    if constexpr (T > 1) __syncthreads();
}

// One wave per workgroup: a wave whose candidate needs few flips retires at once
// and its slot is refilled, instead of idling until the slowest wave of a group.
// Registers hold the keys and signs of 16 NB columns per lane: NB <= 4 fits four
// waves per SIMD, NB <= 6 three, NB = 7, 8 two.  (Keeping the signs in LDS to fit
// a third wave at NB = 7 was measured 40% slower, and fitting NB = 7 into three
// waves' registers directly, with no spill inside the flip loop, 2.1 times slower:
// more waves do not get the rows delivered faster.)
template <int NB> struct AscOcc {
    static constexpr int waves = NB <= 4 ? 4 : NB <= 6 ? 3 : 2;
};

template <int NB>
__global__ __launch_bounds__(64, AscOcc<NB>::waves) void ascent_i8_kernel(AscArgs a)
{
    const int lane = threadIdx.x;
    int64_t P = *a.nidx_d - a.offset;
    P = P < a.max_idx ? P : a.max_idx;
    if (P <= a.team_max) return;  // the team kernel of the same launch takes these passers
    for (int64_t p = blockIdx.x; p < P; p += gridDim.x) ascend_i8<NB>(a, p, lane);
}

template <int NB>
__global__ __launch_bounds__(64, NB <= 4 ? 3 : 2) void ascent_i16_kernel(AscArgs a)
{
    int64_t P = *a.nidx_d - a.offset;
    P = P < a.max_idx ? P : a.max_idx;
    if (P <= a.team_max) return;  // the team kernel of the same launch takes these passers
    for (int64_t p = blockIdx.x; p < P; p += gridDim.x) ascend_i16<NB, 1>(a, p, 0, threadIdx.x, nullptr);
}

template <int NB>
__global__ __launch_bounds__(64, NB <= 4 ? 3 : 2) void ascent_i16_batched(const AscArgs *args, const int64_t *prefix, int count)
{
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const AscArgs a = args[i];
    const int64_t w0 = blockIdx.x - prefix[i], nw = prefix[i + 1] - prefix[i];
    int64_t P = *a.nidx_d - a.offset;
    P = P < a.max_idx ? P : a.max_idx;
    if (P <= a.team_max) return;  // the team kernel of the same launch takes these passers
    for (int64_t p = w0; p < P; p += nw) ascend_i16<NB, 1>(a, p, 0, threadIdx.x, nullptr);
}

template <int NB>
__global__ __launch_bounds__(64, AscOcc<NB>::waves) void ascent_i8_batched(const AscArgs *args, const int64_t *prefix, int count)
{
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const AscArgs a = args[i];
    const int64_t w0 = blockIdx.x - prefix[i], nw = prefix[i + 1] - prefix[i];
    int64_t P = *a.nidx_d - a.offset;
    P = P < a.max_idx ? P : a.max_idx;
    if (P <= a.team_max) return;  // the team kernel of the same launch takes these passers
    for (int64_t p = w0; p < P; p += nw) ascend_i8<NB>(a, p, threadIdx.x);
}

// ---- team ascent: few passers, four waves each ----------------------------------
// A launch with at most UBQP_TEAM_MAX_P passers (one per SIMD) leaves most wave
// slots idle, and each passer's flip chain (a row read, then the update and argmax of all its columns
// by one wave) is the launch's critical path.  There four waves share a passer:
// virtual lane v = 64 w + l of wave w owns the columns [v PLT, (v+1) PLT),
// PLT = 16 NBT, a quarter of the one-wave range, so each wave reads a quarter of
// the row and updates a quarter of the keys.  The waves combine their best
// (Delta, column) through LDS with one barrier per flip; since wave w's columns
// precede wave w+1's, the lowest wave attaining the largest Delta holds the
// lowest such column.  The keys and signs are those of the one-wave ascent, with
// the key's tie-break part rewritten for the shorter lane range.
template <int NBT>
__device__ void ascend_i8_team(const AscArgs &a, int64_t p, int w, int lane, int2 (*slots)[UBQP_TEAM], int S,
                               int64_t prs)
{
    constexpr int PLT = 16 * NBT;
    const int v = w * 64 + lane;
    const int64_t c = a.idx[a.offset + p];
    if (c < 0 || c >= a.x_rows) {
        if (w == 0 && lane == 0) atomicOr(a.err, 2);
        return;  // uniform over the team: every wave reads the same index
    }
    uint64_t *xr = a.X + c * a.W;
    v16i kk[NBT];
    uint32_t ss[NBT][4];
#pragma unroll
    for (int b = 0; b < NBT; b++) {
        const int col0 = v * PLT + 16 * b;
        const bool in = col0 < a.n_pad;
        const int32_t *yrow = a.Y + p * a.n_pad + col0;
        uint32_t bits = 0;  // split K: x of the 16 columns, for keys built here
        if (S > 1 && in && (col0 >> 6) < a.W) bits = (uint32_t)(xr[col0 >> 6] >> (col0 & 63)) & 0xFFFFu;
#pragma unroll
        for (int t4 = 0; t4 < 4; t4++) {
            int4 y = {0, 0, 0, 0};
            if (in && S == 1) {
                y = ubqp_ldg16i(yrow + 4 * t4);
            } else if (in) {
                // the S partial rows of x Q: Delta = q_jj + 2 (1 - 2 x_j) y_j, key = Delta 256 + x_j
                int4 ys = {0, 0, 0, 0};
                for (int s = 0; s < S; s++) {
                    const int4 u = ubqp_ldg16i(yrow + (int64_t)s * prs * a.n_pad + 4 * t4);
                    ys.x += u.x; ys.y += u.y; ys.z += u.z; ys.w += u.w;
                }
                const int4 dg = ubqp_ldg16i(a.diag + col0 + 4 * t4);
                const int32_t yv[4] = {ys.x, ys.y, ys.z, ys.w}, dv[4] = {dg.x, dg.y, dg.z, dg.w};
                int32_t kb[4];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int32_t xj = (bits >> (4 * t4 + k)) & 1u;
                    kb[k] = (dv[k] + (xj ? -2 * yv[k] : 2 * yv[k])) * 256 + xj;
                }
                y = int4{kb[0], kb[1], kb[2], kb[3]};
            }
            const int32_t kv[4] = {y.x, y.y, y.z, y.w};
            uint32_t sw = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int t = 4 * t4 + k;
                // Delta * 256 and x from the key, the tie-break part for this lane's range
                const int32_t key = (in ? (kv[k] & (int32_t)0xFFFFFF01) : 0) | (2 * (127 - (16 * b + t)));
                kk[b][t] = key;
                sw |= ((key & 1) ? 0xFFu : 0x01u) << (8 * k);
            }
            ss[b][t4] = sw;
        }
    }
    const int8_t *qa = (const int8_t *)a.qa;
    int64_t gain = 0;
    int32_t flips = 0;
    const int32_t cap = a.max_flips > 0 ? a.max_flips : a.safety_cap;
    int32_t V;
    int par = 0;
    __builtin_amdgcn_s_waitcnt(WAIT_VM_LGKM_0);
    for (;;) {
        const int32_t best = lane_max<NBT>(kk);
        const int32_t ld = best >> 8;
        const int32_t Vw = wave_max_i32(ld);
        const int lw = __ffsll((unsigned long long)__ballot(ld == Vw)) - 1;
        const int32_t bw = __builtin_amdgcn_readlane(best, lw);
        if (lane == 0) {
            const int localw = 127 - ((bw >> 1) & 127);
            slots[par][w] = int2{Vw, ((w * 64 + lw) * PLT + localw) | ((bw & 1) << 30)};
        }
        __syncthreads();
        int2 win = slots[par][0];
#pragma unroll
        for (int u = 1; u < UBQP_TEAM; u++) {
            const int2 o = slots[par][u];
            win = o.x > win.x ? o : win;  // strict: the lowest wave wins ties
        }
        par ^= 1;  // the other slot set next flip: no second barrier needed
        V = win.x;
        if (V <= 0 || flips >= cap) break;
        const int K = win.y & 0x3FFFFFFF;
        // row k is read first: its latency is the flip's critical path
        const int8_t *row = qa + (int64_t)K * a.ncol_a;
        uint4 wr[NBT];
#pragma unroll
        for (int b = 0; b < NBT; b++) {
            const int col0 = v * PLT + 16 * b;
            wr[b] = col0 < a.ncol_a ? ubqp_ldg16(row + col0) : uint4{0u, 0u, 0u, 0u};
        }
        const int32_t xk = (win.y >> 30) & 1;
        const int vk = K / PLT, local = K - vk * PLT;
        const int bs = local >> 4, ts = local & 15;
        const bool own = v == vk;
        const int32_t knew = -V * 256 + 2 * (127 - local) + (1 - xk);
        const uint32_t sflip = own ? 0xFEu << (8 * (ts & 3)) : 0u;
#pragma unroll
        for (int b = 0; b < NBT; b++) {
            if (b == bs) {
                const int32_t ko = kk[b][ts];
                kk[b][ts] = own ? knew : ko;
#pragma unroll
                for (int r = 0; r < 4; r++) ss[b][r] ^= (r == (ts >> 2)) ? sflip : 0u;
            }
        }
        gain += V;
        flips++;
        const int32_t step = xk ? -512 : 512;
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int b = 0; b < NBT; b++) {
            int32_t k[16];
#pragma unroll
            for (int t = 0; t < 16; t++) k[t] = kk[b][t];
            update_keys8(k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7], wr[b].x, wr[b].y, ss[b][0], ss[b][1], step);
            update_keys8(k[8], k[9], k[10], k[11], k[12], k[13], k[14], k[15], wr[b].z, wr[b].w, ss[b][2], ss[b][3],
                         step);
#pragma unroll
            for (int t = 0; t < 16; t++) kk[b][t] = k[t];
        }
        __builtin_amdgcn_s_setprio(0);
    }
    if (V > 0 && a.max_flips == 0 && w == 0 && lane == 0) atomicOr(a.err, 1);  // flip limit reached
#pragma unroll
    for (int b = 0; b < NBT; b++) {
        uint32_t bits = 0;
#pragma unroll
        for (int t = 0; t < 16; t++) bits |= ((uint32_t)kk[b][t] & 1u) << t;
        const int ci = (v * PLT + 16 * b) >> 4;
        if (ci < 4 * a.W) ((uint16_t *)xr)[ci] = (uint16_t)bits;
    }
    if (w == 0 && lane == 0) {
        a.f[c] += gain;
        a.flips[c] = flips;
    }
    // the next passer's first flip writes slot set 0, which slower waves of the team
    // may still be reading in this passer's last flip
    __syncthreads();
}

// Team kernels: one workgroup of UBQP_TEAM waves per passer.  They run only when
// the launch's passer count is at most UBQP_TEAM_MAX_P (the one-wave kernels take
// the other launches and return at once here, and the other way round).
template <int NBT, int PLANES>
__device__ inline void ascend_team(const AscArgs &a, int64_t p, int w, int lane, int2 (*slots)[UBQP_TEAM], int S,
                                   int64_t prs)
{
    if constexpr (PLANES == 1) ascend_i8_team<NBT>(a, p, w, lane, slots, S, prs);
    else ascend_i16<NBT, UBQP_TEAM>(a, p, w, lane, slots, S, prs);
}

template <int NBT, int PLANES>
__global__ __launch_bounds__(64 * UBQP_TEAM) void ascent_team_kernel(AscArgs a)
{
    __shared__ int2 slots[2][UBQP_TEAM];
    int64_t P = *a.nidx_d - a.offset;
    P = P < a.max_idx ? P : a.max_idx;
    if (P > a.team_max) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // split K of the Delta initialisation: S partial rows R 256 rows apart
    const int S = ubqp_dinit_split(P, a.max_idx, a.n_pad, a.planes, a.team_max, a.split_target);
    const int64_t prs = (P + 255) / 256 * 256;
    for (int64_t p = blockIdx.x; p < P; p += gridDim.x) ascend_team<NBT, PLANES>(a, p, w, lane, slots, S, prs);
}

template <int NBT, int PLANES>
__global__ __launch_bounds__(64 * UBQP_TEAM) void ascent_team_batched(const AscArgs *args, const int64_t *prefix,
                                                                       int count)
{
    __shared__ int2 slots[2][UBQP_TEAM];
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const AscArgs a = args[i];
    const int64_t b0 = blockIdx.x - prefix[i], nb = prefix[i + 1] - prefix[i];
    int64_t P = *a.nidx_d - a.offset;
    P = P < a.max_idx ? P : a.max_idx;
    if (P > a.team_max) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int S = ubqp_dinit_split(P, a.max_idx, a.n_pad, a.planes, a.team_max, a.split_target);
    const int64_t prs = (P + 255) / 256 * 256;
    for (int64_t p = b0; p < P; p += nb) ascend_team<NBT, PLANES>(a, p, w, lane, slots, S, prs);
}

// ---- greedy path relinking -------------------------------------------------
// From the initiating solution toward the guiding one: the free variables are
// those where the two differ; every step flips the free variable with the
// largest Delta (the lowest column on ties), improving or not, and retires it,
// for |D| - 1 steps; the intermediate of largest f (the first on ties) is kept.
// The lane layout and the int32 deltas are those of ascend_i16 for both
// coefficient widths (the keys of the one-plane layout supply Delta = key >> 8).
// Retired and fixed columns hold RL_GONE: each later flip moves them by at most
// 2 |q| <= 65534 and a path has fewer than 8192 flips, so they stay inside
// [-2.14e9, -1.06e9], below every real Delta (|Delta| < 5.4e8) and clear of
// int32 overflow.  The best intermediate is kept as a copy of the sign bytes.
// T = UBQP_TEAM walks a path with four waves (the team layout of the ascent: wave
// w's virtual lanes 64 w + l own consecutive ranges, the waves' best steps combined
// through LDS once per step); T = 1 with one wave.
constexpr int32_t RL_GONE = -1600000000;

template <int NB, int PLANES, int T>
__device__ void relink_path(const RelArgs &a, int64_t p, int wv, int lane, int2 (*slots)[UBQP_TEAM])
{
    constexpr int PL = 16 * NB;
    const int vl = wv * 64 + lane;  // virtual lane
    const int col_base = vl * PL;
    const int64_t ii = a.pairs[2 * p], gi = a.pairs[2 * p + 1];
    uint64_t *xr = a.X + p * a.W;
    if (ii < 0 || ii >= a.E || gi < 0 || gi >= a.E) {  // the same for every wave of a team
        if (vl == 0) {
            atomicOr(a.err, 2);
            a.f_mid[p] = INT64_MIN;
            a.f_out[p] = INT64_MIN;
            a.steps[p] = 0;
        }
        return;
    }
    const uint64_t *gr = a.elite + gi * a.W;
    int nd = 0, pc = 0;
    for (int w = lane; w < a.W; w += 64) {
        nd += __popcll(xr[w] ^ gr[w]);
        pc += __popcll(xr[w]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        nd += __shfl_xor(nd, o);
        pc += __shfl_xor(pc, o);
    }
    v16i dl[NB];
    uint32_t ss[NB][4];
    const int64_t ystride = a.P * a.n_pad;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int col0 = col_base + 16 * b;
        const bool in = col0 < a.n_pad;
        uint32_t bits = 0, free16 = 0;
        if (in) {
            const int w = col0 >> 6;
            if (w < a.W) {
                bits = (uint32_t)(xr[w] >> (col0 & 63)) & 0xFFFFu;
                free16 = (uint32_t)((xr[w] ^ gr[w]) >> (col0 & 63)) & 0xFFFFu;
            }
        }
#pragma unroll
        for (int t4 = 0; t4 < 4; t4++) {
            int32_t dv[4] = {0, 0, 0, 0};
            if (in) {
                if (PLANES == 1) {
                    const int4 k = ubqp_ldg16i(a.Y + p * a.n_pad + col0 + 4 * t4);
                    dv[0] = k.x >> 8; dv[1] = k.y >> 8; dv[2] = k.z >> 8; dv[3] = k.w >> 8;
                } else {
                    const int4 v0 = ubqp_ldg16i(a.Y + p * a.n_pad + col0 + 4 * t4);
                    const int4 v1 = ubqp_ldg16i(a.Y + ystride + p * a.n_pad + col0 + 4 * t4);
                    const int4 dg = ubqp_ldg16i(a.diag + col0 + 4 * t4);
                    const int32_t y0[4] = {v0.x, v0.y, v0.z, v0.w}, y1[4] = {v1.x, v1.y, v1.z, v1.w};
                    const int32_t d[4] = {dg.x, dg.y, dg.z, dg.w};
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const bool xi = (bits >> (4 * t4 + k)) & 1u;
                        const int32_t y = (int32_t)a.weight0 * y0[k] + y1[k] + (int32_t)a.bias * pc;
                        const int32_t g = 2 * y + (xi ? -d[k] : d[k]);
                        dv[k] = xi ? -g : g;
                    }
                }
            }
            uint32_t sw = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int t = 4 * t4 + k;
                const bool fr = in && col0 + t < a.n && ((free16 >> t) & 1u);
                dl[b][t] = fr ? dv[k] : RL_GONE;
                sw |= (((bits >> t) & 1u) ? 0xFFu : 0x01u) << (8 * k);
            }
            ss[b][t4] = sw;
        }
    }

    uint32_t sb[NB][4];
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int r = 0; r < 4; r++) sb[b][r] = ss[b][r];
    int64_t fv = a.f0[p], best = INT64_MIN;
    int32_t bstep = 0;
    int par = 0;
    __builtin_amdgcn_s_waitcnt(WAIT_VM_LGKM_0);
    for (int s = 1; s < nd; s++) {
        int32_t bm[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) bm[b] = max16(dl[b]);
        int32_t bl = bm[0];
#pragma unroll
        for (int b = 1; b < NB; b++) bl = max(bl, bm[b]);
        const int32_t V = wave_max_i32(bl);
        const int lstar = __ffsll((unsigned long long)__ballot(bl == V)) - 1;
        int bsel = NB - 1;
#pragma unroll
        for (int b = NB - 2; b >= 0; b--) bsel = bm[b] == V ? b : bsel;
        const int bs = __builtin_amdgcn_readlane(bsel, lstar);
        int tsel = 15;
        uint32_t sword = 0;
#pragma unroll
        for (int b = 0; b < NB; b++) {
            if (b == bs) {
#pragma unroll
                for (int t = 14; t >= 0; t--) tsel = dl[b][t] == V ? t : tsel;
            }
        }
        const int ts = __builtin_amdgcn_readlane(tsel, lstar);
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                if (b == bs && r == (ts >> 2)) sword = ss[b][r];
        const uint32_t sk = (uint32_t)__builtin_amdgcn_readlane((int)sword, lstar);
        int32_t xk = ((sk >> (8 * (ts & 3))) & 0xFFu) == 0xFFu;  // x_k before the flip
        int K = (wv * 64 + lstar) * PL + 16 * bs + ts;
        int32_t Vs = V;
        bool own = lane == lstar;
        if constexpr (T > 1) {
            // the team's step: the largest Delta of the waves, the lowest wave on ties
            if (lane == 0) slots[par][wv] = int2{V, K | (xk << 30)};
            __syncthreads();
            int2 win = slots[par][0];
#pragma unroll
            for (int u = 1; u < T; u++) {
                const int2 o = slots[par][u];
                win = o.x > win.x ? o : win;
            }
            par ^= 1;
            Vs = win.x;
            K = win.y & 0x3FFFFFFF;
            xk = (win.y >> 30) & 1;
            own = vl == K / PL;
        }
        // row k is read first: its latency is the step's critical path (a team's
        // virtual lanes can reach past the row's ncol_a columns)
        uint4 w1[PLANES == 1 ? NB : 1];
        uint4 w2[PLANES == 2 ? NB : 1][2];
        if constexpr (PLANES == 1) {
            const int8_t *row = (const int8_t *)a.qa + (int64_t)K * a.ncol_a + col_base;
#pragma unroll
            for (int b = 0; b < NB; b++)
                w1[b] = (T == 1 || col_base + 16 * b < a.ncol_a) ? ubqp_ldg16(row + 16 * b) : uint4{0u, 0u, 0u, 0u};
        } else {
            const int16_t *row = (const int16_t *)a.qa + (int64_t)K * a.ncol_a + col_base;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const bool in = T == 1 || col_base + 16 * b < a.ncol_a;
                w2[b][0] = in ? ubqp_ldg16(row + 16 * b) : uint4{0u, 0u, 0u, 0u};
                w2[b][1] = in ? ubqp_ldg16(row + 16 * b + 8) : uint4{0u, 0u, 0u, 0u};
            }
        }
        const int bs_k = (K % PL) >> 4, ts_k = K & 15;
        const uint32_t sflip = own ? 0xFEu << (8 * (ts_k & 3)) : 0u;
#pragma unroll
        for (int b = 0; b < NB; b++) {
            if (b == bs_k) {
                const int32_t ko = dl[b][ts_k];
                dl[b][ts_k] = own ? RL_GONE : ko;   // retired from the free set
#pragma unroll
                for (int r = 0; r < 4; r++) ss[b][r] ^= (r == (ts_k >> 2)) ? sflip : 0u;
            }
        }
        fv += Vs;
        if (fv > best) {
            best = fv;
            bstep = s;
#pragma unroll
            for (int b = 0; b < NB; b++)
#pragma unroll
                for (int r = 0; r < 4; r++) sb[b][r] = ss[b][r];
        }
        // Delta_i += 2 d s_i q_ik for i != k, d = 1 - 2 x_k (the ascent matrix has q_kk = 0)
        const int32_t step = xk ? -2 : 2;
        if constexpr (PLANES == 1) {
#pragma unroll
            for (int b = 0; b < NB; b++) {
                int32_t d[16];
#pragma unroll
                for (int t = 0; t < 16; t++) d[t] = dl[b][t];
                update_keys8(d[0], d[1], d[2], d[3], d[4], d[5], d[6], d[7], w1[b].x, w1[b].y, ss[b][0], ss[b][1],
                             step);
                update_keys8(d[8], d[9], d[10], d[11], d[12], d[13], d[14], d[15], w1[b].z, w1[b].w, ss[b][2],
                             ss[b][3], step);
#pragma unroll
                for (int t = 0; t < 16; t++) dl[b][t] = d[t];
            }
        } else {
#pragma unroll
            for (int b = 0; b < NB; b++) {
                int32_t d[16];
#pragma unroll
                for (int t = 0; t < 16; t++) d[t] = dl[b][t];
                update_deltas8(d[0], d[1], d[2], d[3], d[4], d[5], d[6], d[7], w2[b][0].x, w2[b][0].y, w2[b][0].z,
                               w2[b][0].w, ss[b][0], ss[b][1], step);
                update_deltas8(d[8], d[9], d[10], d[11], d[12], d[13], d[14], d[15], w2[b][1].x, w2[b][1].y,
                               w2[b][1].z, w2[b][1].w, ss[b][2], ss[b][3], step);
#pragma unroll
                for (int t = 0; t < 16; t++) dl[b][t] = d[t];
            }
        }
    }
    if (bstep > 0) {
#pragma unroll
        for (int b = 0; b < NB; b++) {
            uint32_t bits = 0;
#pragma unroll
            for (int t = 0; t < 16; t++) bits |= (((sb[b][t >> 2] >> (8 * (t & 3))) & 0xFFu) == 0xFFu ? 1u : 0u) << t;
            const int ci = vl * NB + b;
            if (ci < 4 * a.W) ((uint16_t *)xr)[ci] = (uint16_t)bits;
        }
    }
    if (vl == 0) {
        a.f_mid[p] = best;
        a.f_out[p] = best;
        a.steps[p] = bstep;
    }
    // the next path's first step writes slot set 0, which slower waves of the team may
    // still be reading in this path's last step
    if constexpr (T > 1) __syncthreads();
}

template <int NB, int PLANES>
__global__ __launch_bounds__(64, NB <= 4 ? 2 : 1) void relink_kernel(RelArgs a)
{
    for (int64_t p = blockIdx.x; p < a.P; p += gridDim.x) relink_path<NB, PLANES, 1>(a, p, 0, threadIdx.x, nullptr);
}

// Few paths (at most UBQP_RELINK_TEAM_MAX_P, n_pad > 3072): four waves per path.
template <int NBT, int PLANES>
__global__ __launch_bounds__(64 * UBQP_TEAM) void relink_team_kernel(RelArgs a)
{
    __shared__ int2 slots[2][UBQP_TEAM];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t p = blockIdx.x; p < a.P; p += gridDim.x) relink_path<NBT, PLANES, UBQP_TEAM>(a, p, wv, lane, slots);
}

#define UBQP_NB_SWITCH(nb, LAUNCH) \
    switch (nb) {                    \
    case 1: LAUNCH(1); break;        \
    case 2: LAUNCH(2); break;        \
    case 3: LAUNCH(3); break;        \
    case 4: LAUNCH(4); break;        \
    case 5: LAUNCH(5); break;        \
    case 6: LAUNCH(6); break;        \
    case 7: LAUNCH(7); break;        \
    default: LAUNCH(8); break;       \
    }

}  // namespace

AscArgs ubqp_ascent_args(const ubqp_problem *p, uint64_t *X, int64_t x_rows, const int32_t *idx, const int64_t *nidx_d,
                         int64_t offset, int64_t cap, const int32_t *Y, int64_t *f, int32_t max_flips, int32_t *flips,
                         int32_t *err_flag)
{
    AscArgs a{};
    a.qa = p->qa;
    a.ncol_a = p->ncol_a;
    a.diag = p->diag;
    a.n = p->n;
    a.n_pad = p->n_pad;
    a.W = p->W;
    a.planes = p->planes;
    a.weight0 = p->weight0;
    a.bias = p->bias;
    a.X = X;
    a.x_rows = x_rows;
    a.idx = idx;
    a.nidx_d = nidx_d;
    a.offset = offset;
    a.max_idx = cap;
    a.Y = Y;
    a.f = f;
    a.flips = flips;
    a.max_flips = max_flips;
    a.safety_cap = ubqp_problem_flip_limit(p);
    a.err = err_flag;
    // at least four 16-column blocks per one-wave lane: launches with few passers
    // ascend them in teams of waves (int16 rows: the team's extra exchange outweighs
    // its shorter flips earlier, 1.35 against 1.21 ms at 1023 passers, n = 5500)
    a.team_max = (p->n_pad + 1023) / 1024 >= UBQP_TEAM_MIN_NB ? (p->planes == 1 ? UBQP_TEAM_MAX_P : UBQP_TEAM_MAX_P_I16) : 0;
    return a;
}

void ubqp_split_dinit(EvalArgs &yr, AscArgs &as, int target)
{
    as.split_target = target > 0 ? target : 0;
    yr.split_target = as.split_target;
    yr.split_team_max = as.team_max;
}

void ubqp_ascent_share_team(AscArgs &a, int group, int instances)
{
    // With other instances on the chip, four waves per passer take wave slots from
    // their passers, and a group's team and one-wave launches run one after the
    // other (served requests: p50 55 ms with 1024 / c against 46 ms with 512 / c).
    if (a.team_max > 0 && instances > 1) {
        const int64_t b = a.team_max < UBQP_TEAM_MAX_P_GROUP ? a.team_max : UBQP_TEAM_MAX_P_GROUP;
        a.team_max = b / group > 1 ? b / group : 1;
    }
}

int64_t ubqp_ascent_team_blocks(const AscArgs &a)
{
    if (a.team_max <= 0) return 0;
    return a.max_idx < a.team_max ? (a.max_idx < 1 ? 1 : a.max_idx) : a.team_max;
}

static hipError_t launch_team(hipStream_t st, const AscArgs &a)
{
    const unsigned blocks = (unsigned)ubqp_ascent_team_blocks(a);
    if (blocks == 0) return hipSuccess;
    const bool two = (a.n_pad + 4095) / 4096 > 1;
#define LT(NBT, PL) hipLaunchKernelGGL((ascent_team_kernel<NBT, PL>), dim3(blocks), dim3(64 * UBQP_TEAM), 0, st, a)
    if (a.planes == 2) {
        if (two) LT(2, 2);
        else LT(1, 2);
    } else {
        if (two) LT(2, 1);
        else LT(1, 1);
    }
#undef LT
    return hipGetLastError();
}

int ubqp_ascent_nb(const AscArgs &a) { return (a.n_pad + 1023) / 1024; }
int64_t ubqp_ascent_waves(const AscArgs &a) { return a.max_idx < 8192 ? (a.max_idx < 1 ? 1 : a.max_idx) : 8192; }

hipError_t ubqp_launch_ascent(hipStream_t st, const AscArgs &a)
{
    hipError_t e = launch_team(st, a);
    if (e != hipSuccess) return e;
    const unsigned waves = (unsigned)ubqp_ascent_waves(a);
#define L16(NB) hipLaunchKernelGGL(ascent_i16_kernel<NB>, dim3(waves), dim3(64), 0, st, a)
#define L8(NB) hipLaunchKernelGGL(ascent_i8_kernel<NB>, dim3(waves), dim3(64), 0, st, a)
    if (a.planes == 2) {
        UBQP_NB_SWITCH(ubqp_ascent_nb(a), L16)
    } else {
        UBQP_NB_SWITCH(ubqp_ascent_nb(a), L8)
    }
#undef L16
#undef L8
    return hipGetLastError();
}

hipError_t ubqp_launch_ascent_team_batch(hipStream_t st, int planes, int n_pad_max, const AscArgs *args,
                                         const int64_t *prefix, int count, int64_t blocks)
{
    if (blocks <= 0) return hipSuccess;
    const bool two = (n_pad_max + 4095) / 4096 > 1;
#define LT(NBT, PL)                                                                                                   \
    hipLaunchKernelGGL((ascent_team_batched<NBT, PL>), dim3((unsigned)blocks), dim3(64 * UBQP_TEAM), 0, st, args, \
                       prefix, count)
    if (planes == 2) {
        if (two) LT(2, 2);
        else LT(1, 2);
    } else {
        if (two) LT(2, 1);
        else LT(1, 1);
    }
#undef LT
    return hipGetLastError();
}

hipError_t ubqp_launch_ascent_batch(hipStream_t st, int planes, int nb, const AscArgs *args, const int64_t *prefix,
                                    int count, int64_t waves)
{
    if (waves <= 0) return hipSuccess;
#define L16(NB) hipLaunchKernelGGL(ascent_i16_batched<NB>, dim3((unsigned)waves), dim3(64), 0, st, args, prefix, count)
#define L8(NB) hipLaunchKernelGGL(ascent_i8_batched<NB>, dim3((unsigned)waves), dim3(64), 0, st, args, prefix, count)
    if (planes == 2) {
        UBQP_NB_SWITCH(nb, L16)
    } else {
        UBQP_NB_SWITCH(nb, L8)
    }
#undef L16
#undef L8
    return hipGetLastError();
}

RelArgs ubqp_relink_args(const ubqp_problem *p, const uint64_t *elite, int64_t E, const int32_t *pairs, int64_t P,
                         uint64_t *X, const int32_t *Y, const int64_t *f0, int64_t *f_mid, int64_t *f_out,
                         int32_t *steps, int32_t *err)
{
    RelArgs a{};
    a.qa = p->qa;
    a.ncol_a = p->ncol_a;
    a.diag = p->diag;
    a.n = p->n;
    a.n_pad = p->n_pad;
    a.W = p->W;
    a.planes = p->planes;
    a.weight0 = p->weight0;
    a.bias = p->bias;
    a.elite = elite;
    a.E = E;
    a.pairs = pairs;
    a.P = P;
    a.X = X;
    a.Y = Y;
    a.f0 = f0;
    a.f_mid = f_mid;
    a.f_out = f_out;
    a.steps = steps;
    a.err = err;
    return a;
}

hipError_t ubqp_launch_relink(hipStream_t st, const RelArgs &a)
{
    if (a.P <= 0) return hipSuccess;
    if (a.P <= UBQP_RELINK_TEAM_MAX_P && (a.n_pad + 1023) / 1024 >= UBQP_TEAM_MIN_NB) {
        const unsigned blocks = (unsigned)a.P;
        const bool two = (a.n_pad + 4095) / 4096 > 1;
        if (a.planes == 2) {
            if (two) hipLaunchKernelGGL((relink_team_kernel<2, 2>), dim3(blocks), dim3(64 * UBQP_TEAM), 0, st, a);
            else hipLaunchKernelGGL((relink_team_kernel<1, 2>), dim3(blocks), dim3(64 * UBQP_TEAM), 0, st, a);
        } else {
            if (two) hipLaunchKernelGGL((relink_team_kernel<2, 1>), dim3(blocks), dim3(64 * UBQP_TEAM), 0, st, a);
            else hipLaunchKernelGGL((relink_team_kernel<1, 1>), dim3(blocks), dim3(64 * UBQP_TEAM), 0, st, a);
        }
        return hipGetLastError();
    }
    const unsigned waves = (unsigned)(a.P < 8192 ? a.P : 8192);
    const int nb = (a.n_pad + 1023) / 1024;
#define L1(NB) hipLaunchKernelGGL((relink_kernel<NB, 1>), dim3(waves), dim3(64), 0, st, a)
#define L2(NB) hipLaunchKernelGGL((relink_kernel<NB, 2>), dim3(waves), dim3(64), 0, st, a)
    if (a.planes == 2) {
        UBQP_NB_SWITCH(nb, L2)
    } else {
        UBQP_NB_SWITCH(nb, L1)
    }
#undef L1
#undef L2
    return hipGetLastError();
}
