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
// int8 Q (ascent_i8): lane l owns the contiguous columns [l PL, (l+1) PL),
// PL = 16 NB, and keeps for each of them the 32-bit key
//     key_i = Delta_i * 256 + 2 (127 - local_i) + x_i     (|Delta_i| < 2^21)
// and the sign s_i as a signed byte (four per VGPR).  A flip is
//     key_i += (q_ik * s_i) * 512 d  -- one SDWA v_mul_i32_i24 (byte x byte,
//                                       both sign-extended) and one v_mad_i32_i24
// with 512 d in an SGPR, so the lane's best key is a v_max3 tree, the wave's best
// Delta one DPP max, and the lowest column attaining it the lowest such lane
// (ballot + ffs) with its local index and old x_k read from the key.  The flipped
// variable's key and sign are rewritten through one uniform-indexed register
// access per block.
//
// int16 Q (ascent_general): lane l owns columns 1024 b + 16 l + t, keeps
// g_i = q_ii + 2 sum_{j != i} q_ij x_j (Delta_i = s_i g_i), and compares
// (Delta, column) pairs across the wave.
//
// The starting deltas come from Y = X Q on the passers (the matrix-core kernel):
//     y_i = w0 Y0_i + Y1_i + bias * popcount(x)   (bias / Y1 only when split)
//     g_i = 2 y_i + q_ii (1 - 2 x_i).
#include "ubqp_internal.h"

namespace {


template <typename QT> struct RowLoad;
template <> struct RowLoad<int8_t> {
    // 16 consecutive int8 entries
    __device__ static inline void load(const int8_t *p, int32_t (&q)[16])
    {
        const uint4 v = *(const uint4 *)p;
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int k = 0; k < 4; k++) q[i * 4 + k] = ((int32_t)(w[i] << (24 - 8 * k))) >> 24;
    }
};
template <> struct RowLoad<int16_t> {
    __device__ static inline void load(const int16_t *p, int32_t (&q)[16])
    {
        const uint4 v0 = *(const uint4 *)p, v1 = *(const uint4 *)(p + 8);
        const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
        for (int i = 0; i < 8; i++) {
            q[i * 2] = ((int32_t)(w[i] << 16)) >> 16;
            q[i * 2 + 1] = ((int32_t)w[i]) >> 16;
        }
    }
};

// Lane-local column index of register slot (b, t): local = 16 b + t (< 128);
// global column = 1024 b + 16 lane + t.
__device__ inline int32_t global_col(int32_t local, int lane) { return (local >> 4) * 1024 + lane * 16 + (local & 15); }

// Wave-wide max of (value, column) pairs: largest value, lowest column.
__device__ inline void wave_argmax(int32_t &v, int32_t &k)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t ov = __shfl_xor(v, o), ok = __shfl_xor(k, o);
        if (ov > v || (ov == v && ok < k)) { v = ov; k = ok; }
    }
}

template <int NB, typename QT>
__device__ void ascend_one(const AscArgs &a, int64_t p, int lane)
{
    // int8 Q: |g| < 2^21 for n <= 8192, so the argmax runs on packed 32-bit keys
    //   key = Delta * 128 + L,  L = 127 - local   (largest key: largest Delta,
    //                                              then lowest local index).
    // The register holds h = g * 128 + L, i.e. the key while x = 0; for x = 1 the
    // key is -g * 128 + L = -h + 2L = (h ^ m) + (m & (2L + 1)) with m = -x, one
    // v_xad.  The flip update adds 256 d q_ik to h and leaves L alone.
    // int16 Q keeps g and compares (Delta, column) pairs directly.
    constexpr bool KEYED = false;  // the int8 path is ascend_i8
    const int64_t c = a.idx[a.offset + p];
    if (c < 0 || c >= a.x_rows) {
        if (lane == 0) atomicOr(a.err, 2);
        return;
    }
    uint64_t *xr = a.X + c * a.W;
    const QT *qa = (const QT *)a.qa;

    uint32_t xb[NB];
    int32_t gv[NB][16];
    int pc = 0;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int col0 = b * 1024 + lane * 16;
        uint32_t bits = 0;
        if (col0 < a.n_pad) {
            const int w = col0 >> 6;
            if (w < a.W) bits = (uint32_t)(xr[w] >> (col0 & 63)) & 0xFFFFu;
        }
        xb[b] = bits;
        pc += __popc(bits);
    }
    if (a.planes == 2) {
        for (int o = 32; o > 0; o >>= 1) pc += __shfl_xor(pc, o);
    }
    const int64_t ystride = a.max_idx * a.n_pad;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int col0 = b * 1024 + lane * 16;
        if (col0 < a.n_pad) {
            const int32_t *y0 = a.Y + p * a.n_pad + col0;
#pragma unroll
            for (int t4 = 0; t4 < 4; t4++) {
                const int4 v = *(const int4 *)(y0 + t4 * 4);
                const int4 dg = *(const int4 *)(a.diag + col0 + t4 * 4);
                int32_t y[4] = {v.x, v.y, v.z, v.w};
                const int32_t d[4] = {dg.x, dg.y, dg.z, dg.w};
                if (a.planes == 2) {
                    const int4 u = *(const int4 *)(y0 + ystride + t4 * 4);
                    const int32_t y1[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int k = 0; k < 4; k++) y[k] = (int32_t)a.weight0 * y[k] + y1[k] + (int32_t)a.bias * pc;
                }
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int t = t4 * 4 + k;
                    // padding columns (j >= n) keep g = 0, so their Delta is 0 and never taken
                    const int32_t g = col0 + t < a.n ? 2 * y[k] + (((xb[b] >> t) & 1u) ? -d[k] : d[k]) : 0;
                    gv[b][t] = KEYED ? g * 128 + (127 - (b * 16 + t)) : g;
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < 16; t++) gv[b][t] = KEYED ? (127 - (b * 16 + t)) : 0;
        }
    }

    // (V, K): largest Delta and its lowest global column, identical in all lanes.
    auto argmax = [&](int32_t &V, int32_t &K) {
        if constexpr (KEYED) {
            int32_t best = INT32_MIN;
#pragma unroll
            for (int b = 0; b < NB; b++)
#pragma unroll
                for (int t = 0; t < 16; t += 2) {
                    const int32_t m0 = -(int32_t)((xb[b] >> t) & 1u), m1 = -(int32_t)((xb[b] >> (t + 1)) & 1u);
                    const int32_t k0 = (gv[b][t] ^ m0) + (m0 & (2 * (127 - (b * 16 + t)) + 1));
                    const int32_t k1 = (gv[b][t + 1] ^ m1) + (m1 & (2 * (127 - (b * 16 + t + 1)) + 1));
                    best = max(best, max(k0, k1));
                }
            int32_t v = best >> 7;
            int32_t k = global_col(127 - (best & 127), lane);
            wave_argmax(v, k);
            V = v;
            K = k;
        } else {
            int32_t bv = INT32_MIN, bk = 0x7FFFFFFF;
#pragma unroll
            for (int b = 0; b < NB; b++)
#pragma unroll
                for (int t = 0; t < 16; t++) {
                    const int32_t m = -(int32_t)((xb[b] >> t) & 1u);
                    const int32_t dl = (gv[b][t] ^ m) - m;
                    if (dl > bv) { bv = dl; bk = b * 16 + t; }
                }
            bk = global_col(bk, lane);
            wave_argmax(bv, bk);
            V = bv;
            K = bk;
        }
    };

    int64_t fv = a.f[c];
    int32_t flips = 0;
    const int32_t cap = a.max_flips > 0 ? a.max_flips : a.safety_cap;
    int32_t V, K;
    argmax(V, K);
    while (V > 0 && flips < cap) {
        const int kb = K >> 10, kl = (K >> 4) & 63, kt = K & 15;
        uint32_t xw = 0;
#pragma unroll
        for (int b = 0; b < NB; b++) xw = (b == kb) ? xb[b] : xw;
        const int xk = (__shfl((int)xw, kl) >> kt) & 1;
        if (lane == kl) {
#pragma unroll
            for (int b = 0; b < NB; b++) xb[b] ^= (b == kb) ? (1u << kt) : 0u;
        }
        // g_i += 2 d q_ik with d = +1 (x_k: 0 -> 1) or -1; scaled by 128 when keyed
        const int32_t step = (xk ? -2 : 2) * (KEYED ? 128 : 1);
        fv += V;
        flips++;
        const QT *row = qa + (int64_t)K * a.n_pad;
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int col0 = b * 1024 + lane * 16;
            if (col0 < a.n_pad) {
                int32_t q[16];
                RowLoad<QT>::load(row + col0, q);
#pragma unroll
                for (int t = 0; t < 16; t++) gv[b][t] += step * q[t];
            }
        }
        argmax(V, K);
    }
    if (V > 0 && a.max_flips == 0 && lane == 0) atomicOr(a.err, 1);  // safety cap reached

#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int col0 = b * 1024 + lane * 16;
        const uint64_t v0 = xb[b];
        const uint64_t v1 = (uint32_t)__shfl_down((int)xb[b], 1);
        const uint64_t v2 = (uint32_t)__shfl_down((int)xb[b], 2);
        const uint64_t v3 = (uint32_t)__shfl_down((int)xb[b], 3);
        if ((lane & 3) == 0 && col0 < a.n_pad) {
            const int w = col0 >> 6;
            if (w < a.W) xr[w] = v0 | (v1 << 16) | (v2 << 32) | (v3 << 48);
        }
    }
    if (lane == 0) {
        a.f[c] = fv;
        a.flips[c] = flips;
    }
}

// key += (q * s) * step, q = signed byte B of w, s = signed byte B of u, step
// wave-uniform: one SDWA multiply (both bytes sign-extended) and one 24-bit mad.
template <int B>
__device__ inline int32_t update_key(int32_t key, uint32_t w, uint32_t u, int32_t step)
{
    int32_t prod;
    asm("v_mul_i32_i24_sdwa %1, sext(%2), sext(%3) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_%5 "
        "src1_sel:BYTE_%5\n\t"
        "v_mad_i32_i24 %0, %1, %4, %0"
        : "+v"(key), "=&v"(prod)
        : "v"(w), "v"(u), "s"(step), "n"(B));
    return key;
}

// Largest value over the wave (DPP within rows of 16, then the four row leaders).
__device__ inline int32_t wave_max_i32(int32_t v)
{
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x124, 0xF, 0xF, false));  // row_ror:4
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x128, 0xF, 0xF, false));  // row_ror:8
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

typedef int32_t v16i __attribute__((ext_vector_type(16)));

template <int NB>
__device__ void ascend_i8(const AscArgs &a, int64_t p, int lane)
{
    constexpr int PL = 16 * NB;
    const int64_t c = a.idx[a.offset + p];
    if (c < 0 || c >= a.x_rows) {
        if (lane == 0) atomicOr(a.err, 2);
        return;
    }
    uint64_t *xr = a.X + c * a.W;
    const int col_base = lane * PL;
    // key_i = Delta_i * 256 + 2 L_i + x_i,  L_i = 127 - local_i: the largest key is
    // the largest Delta, then the lowest local index; bit 0 carries x_i.
    v16i kk[NB];
    // s_i = 1 - 2 x_i as signed bytes, four per register
    uint32_t ss[NB][4];
    // keys of this lane's columns from the matrix-core epilogue; columns past n_pad
    // (Delta = 0, x = 0) are synthesised
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int col0 = col_base + 16 * b;
        const bool in = col0 < a.n_pad;
        const int32_t *yrow = a.Y + p * a.n_pad + col0;
#pragma unroll
        for (int t4 = 0; t4 < 4; t4++) {
            int4 v = {0, 0, 0, 0};
            if (in) v = *(const int4 *)(yrow + 4 * t4);
            const int32_t kv[4] = {v.x, v.y, v.z, v.w};
            uint32_t sw = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int t = 4 * t4 + k;
                const int32_t key = in ? kv[k] : 2 * (127 - (16 * b + t));
                kk[b][t] = key;
                sw |= ((key & 1) ? 0xFFu : 0x01u) << (8 * k);
            }
            ss[b][t4] = sw;
        }
    }

    const int8_t *qa = (const int8_t *)a.qa;
    int64_t fv = a.f[c];
    int32_t flips = 0;
    const int32_t cap = a.max_flips > 0 ? a.max_flips : a.safety_cap;
    int32_t V;
    for (;;) {
        int32_t best = INT32_MIN;
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
            for (int t = 0; t < 16; t += 2) best = max(best, max(kk[b][t], kk[b][t + 1]));
        const int32_t ld = best >> 8;
        V = wave_max_i32(ld);
        if (V <= 0 || flips >= cap) break;
        const uint64_t bal = __ballot(ld == V);
        const int lstar = __ffsll((unsigned long long)bal) - 1;
        const int32_t bk = __builtin_amdgcn_readlane(best, lstar);
        const int local = 127 - ((bk >> 1) & 127);
        const int32_t xk = bk & 1;              // x_k before the flip
        const int K = lstar * PL + local;
        const int bs = local >> 4, ts = local & 15;
        // the flipped variable: Delta_k -> -V, x_k and s_k toggle (lane lstar only)
        const bool own = lane == lstar;
        const int32_t knew = -V * 256 + (bk & 0xFE) + (1 - xk);
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
        fv += V;
        flips++;
        // Delta_i += 2 d s_i q_ik for i != k, with d = 1 - 2 x_k: key_i += (q_ik s_i) * 512 d
        const int32_t step = xk ? -512 : 512;
        const int8_t *row = qa + (int64_t)K * a.ncol_a + col_base;
        uint4 w[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) w[b] = *(const uint4 *)(row + 16 * b);
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const uint32_t q4[4] = {w[b].x, w[b].y, w[b].z, w[b].w};
#pragma unroll
            for (int t = 0; t < 16; t++) {
                switch (t & 3) {
                case 0: kk[b][t] = update_key<0>(kk[b][t], q4[t >> 2], ss[b][t >> 2], step); break;
                case 1: kk[b][t] = update_key<1>(kk[b][t], q4[t >> 2], ss[b][t >> 2], step); break;
                case 2: kk[b][t] = update_key<2>(kk[b][t], q4[t >> 2], ss[b][t >> 2], step); break;
                default: kk[b][t] = update_key<3>(kk[b][t], q4[t >> 2], ss[b][t >> 2], step); break;
                }
            }
        }
    }
    if (V > 0 && a.max_flips == 0 && lane == 0) atomicOr(a.err, 1);  // safety cap reached

#pragma unroll
    for (int b = 0; b < NB; b++) {
        uint32_t bits = 0;
#pragma unroll
        for (int t = 0; t < 16; t++) bits |= ((uint32_t)kk[b][t] & 1u) << t;
        const int ci = lane * NB + b;
        if (ci < 4 * a.W) ((uint16_t *)xr)[ci] = (uint16_t)bits;
    }
    if (lane == 0) {
        a.f[c] = fv;
        a.flips[c] = flips;
    }
}

// One wave per workgroup: a wave whose candidate needs few flips retires at once
// and its slot is refilled, instead of idling until the slowest wave of a group.
template <int NB>
__global__ __launch_bounds__(64) void ascent_i8_kernel(AscArgs a)
{
    const int lane = threadIdx.x;
    int64_t P = *a.nidx_d - a.offset;
    P = P < a.max_idx ? P : a.max_idx;
    for (int64_t p = blockIdx.x; p < P; p += gridDim.x) ascend_i8<NB>(a, p, lane);
}

template <int NB, typename QT>
__global__ __launch_bounds__(64) void ascent_kernel(AscArgs a)
{
    int64_t P = *a.nidx_d - a.offset;
    P = P < a.max_idx ? P : a.max_idx;
    for (int64_t p = blockIdx.x; p < P; p += gridDim.x) ascend_one<NB, QT>(a, p, threadIdx.x);
}

template <int NB, typename QT>
__global__ __launch_bounds__(64) void ascent_batched(const AscArgs *args, const int64_t *prefix, int count)
{
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const AscArgs a = args[i];
    const int64_t w0 = blockIdx.x - prefix[i], nw = prefix[i + 1] - prefix[i];
    int64_t P = *a.nidx_d - a.offset;
    P = P < a.max_idx ? P : a.max_idx;
    for (int64_t p = w0; p < P; p += nw) ascend_one<NB, QT>(a, p, threadIdx.x);
}

template <int NB>
__global__ __launch_bounds__(64) void ascent_i8_batched(const AscArgs *args, const int64_t *prefix, int count)
{
    const int i = ubqp_find_inst(prefix, count, blockIdx.x);
    const AscArgs a = args[i];
    const int64_t w0 = blockIdx.x - prefix[i], nw = prefix[i + 1] - prefix[i];
    int64_t P = *a.nidx_d - a.offset;
    P = P < a.max_idx ? P : a.max_idx;
    for (int64_t p = w0; p < P; p += nw) ascend_i8<NB>(a, p, threadIdx.x);
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
    a.safety_cap = 64 * p->n_pad + 4096;
    a.err = err_flag;
    return a;
}

int ubqp_ascent_nb(const AscArgs &a) { return (a.n_pad + 1023) / 1024; }
int64_t ubqp_ascent_waves(const AscArgs &a) { return a.max_idx < 8192 ? (a.max_idx < 1 ? 1 : a.max_idx) : 8192; }

hipError_t ubqp_launch_ascent(hipStream_t st, const AscArgs &a)
{
    const unsigned waves = (unsigned)ubqp_ascent_waves(a);
#define L16(NB) hipLaunchKernelGGL((ascent_kernel<NB, int16_t>), dim3(waves), dim3(64), 0, st, a)
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

hipError_t ubqp_launch_ascent_batch(hipStream_t st, int planes, int nb, const AscArgs *args, const int64_t *prefix,
                                    int count, int64_t waves)
{
    if (waves <= 0) return hipSuccess;
#define L16(NB) hipLaunchKernelGGL((ascent_batched<NB, int16_t>), dim3((unsigned)waves), dim3(64), 0, st, args, prefix, count)
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
