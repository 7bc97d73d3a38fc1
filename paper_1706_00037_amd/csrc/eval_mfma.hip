// Batched exact objective on int8 matrix cores (the evaluation the paper moves
// to the GPU, Introduction and Pseudocode section):
//
//     Y = X Q  (int8 x int8 -> int32, v_mfma_i32_16x16x64_i8),
//     f_m = sum_j x_mj Y_mj  (int64)
//
// X is bit-packed (1 bit per variable, the A operand is expanded to int8 0/1 in
// registers), Q is a resident int8 plane [n_pad][n_pad].  Q is symmetric, so
// column j of Q is row j: both operands are K-contiguous and the B fragment of
// a lane is 16 consecutive bytes of one Q row.
//
// Exactness: |Y_mj| <= 128 n <= 2^20 for n <= 8192, inside int32; the row dot
// is summed per 64-column slab in int32 (<= 2^26) and accumulated across slabs
// and planes with int64 atomics (integer, so the order does not matter).
//
// Workgroup tile BM x BN = 256 x 128 (4 waves of 128 x 64), K staged through
// LDS KC = 128 at a time, double buffered.  A second epilogue stores Y rows
// instead (the Delta initialisation of the ascent, on gathered passer rows).
#include "ubqp_internal.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int BM = 256, BN = 128, KC = 128, THR = 256;
constexpr int BPITCH = KC + 16;  // bytes per staged Q row (pad against bank conflicts)
constexpr int WM = 128, WN = 64;  // wave tile
constexpr int FM = WM / 16, FN = WN / 16;

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

struct EvalArgs {
    const int8_t *q;        // plane 0; plane p at q + p * plane_stride
    int64_t plane_stride;
    int32_t n_pad;
    const uint64_t *X;
    int32_t W;
    int64_t M;              // rows (or capacity of the gather list)
    const int32_t *rows;    // gather list (STORE_Y) or null, already offset to the chunk
    int64_t x_rows;         // rows of X (gather targets outside [0, x_rows) read as zero)
    const int64_t *nrows_d; // device length of the whole list (STORE_Y)
    int64_t offset;         // first list entry of this chunk
    int64_t *f;             // row-dot output
    int32_t *Y;             // Y output [planes][M][n_pad]
    int64_t weight0;        // weight of plane 0 in the row dot
    int32_t m_tiles, n_tiles;
    const int32_t *diag;    // KEYS: q_jj
    int32_t keys_pl;        // KEYS: columns per lane of the ascent (16 NB)
};

// Epilogues of the contraction.
enum { EPI_ROWDOT = 0, EPI_Y = 1, EPI_KEYS = 2 };

template <int EPI>
__global__ __launch_bounds__(THR, 1) void eval_kernel(EvalArgs a)
{
    constexpr bool STORE_Y = EPI != EPI_ROWDOT;
    __shared__ __align__(16) int8_t Bs[2][BN * BPITCH];
    __shared__ __align__(16) uint64_t As[2][BM * 2];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // XCD-aware tile order: consecutive workgroups go round-robin to the 8 XCDs;
    // give each XCD a contiguous run of tiles, ordered n-tile-major so the
    // workgroups resident on one XCD share the same Q column block in its L2.
    const int64_t T = (int64_t)a.m_tiles * a.n_tiles;
    const int64_t b = blockIdx.x;
    const int64_t xcd = b % 8, j = b / 8, per = T / 8, rem = T % 8;
    // XCD x gets tiles [start_x, start_x + per + (x < rem)), a bijection on [0, T)
    const int64_t t = xcd * per + (xcd < rem ? xcd : rem) + j;
    if (b >= T) return;
    const int nt = (int)(t / a.m_tiles), mt = (int)(t % a.m_tiles);
    const int plane = blockIdx.y;

    int64_t Mrows = a.M;
    if (STORE_Y) { const int64_t k = *a.nrows_d - a.offset; Mrows = k < a.M ? k : a.M; }
    const int64_t m0 = (int64_t)mt * BM;
    if (m0 >= Mrows) return;
    const int n0 = nt * BN;
    const int8_t *qp = a.q + plane * a.plane_stride;

    // staging assignment: thread tid loads A row m0 + tid (2 words) and four
    // 16-byte chunks of the Q block
    const int64_t arow = m0 + tid;
    const uint64_t *xrow = nullptr;
    if (arow < Mrows) {
        const int64_t r = STORE_Y ? (int64_t)a.rows[arow] : arow;
        if (r >= 0 && r < a.x_rows) xrow = a.X + r * a.W;
    }

    uint64_t aw0 = 0, aw1 = 0;
    uint4 br0, br1, br2, br3;
    // global -> registers for stage kc (A: 2 words of row m0 + tid; B: four 16-byte chunks)
#define EVAL_LOAD_STAGE(kc)                                                                    \
    do {                                                                                       \
        const int w_ = (kc) * (KC / 64);                                                       \
        aw0 = (xrow && w_ < a.W) ? xrow[w_] : 0ull;                                            \
        aw1 = (xrow && w_ + 1 < a.W) ? xrow[w_ + 1] : 0ull;                                    \
        const int8_t *qb_ = qp + (int64_t)(n0 + (tid >> 3)) * a.n_pad + (kc) * KC + (tid & 7) * 16; \
        const int64_t rs_ = (int64_t)(THR / 8) * a.n_pad;                                      \
        br0 = *(const uint4 *)(qb_);                                                           \
        br1 = *(const uint4 *)(qb_ + rs_);                                                     \
        br2 = *(const uint4 *)(qb_ + 2 * rs_);                                                 \
        br3 = *(const uint4 *)(qb_ + 3 * rs_);                                                 \
    } while (0)
    // registers -> LDS buffer buf
#define EVAL_STORE_STAGE(buf)                                                                  \
    do {                                                                                       \
        As[buf][tid * 2] = aw0;                                                                \
        As[buf][tid * 2 + 1] = aw1;                                                            \
        int8_t *bs_ = &Bs[buf][(tid >> 3) * BPITCH + (tid & 7) * 16];                          \
        *(uint4 *)(bs_) = br0;                                                                 \
        *(uint4 *)(bs_ + (THR / 8) * BPITCH) = br1;                                            \
        *(uint4 *)(bs_ + 2 * (THR / 8) * BPITCH) = br2;                                        \
        *(uint4 *)(bs_ + 3 * (THR / 8) * BPITCH) = br3;                                        \
    } while (0)

    v4i acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
        for (int k = 0; k < FN; k++) acc[i][k] = v4i{0, 0, 0, 0};

    const int nk = a.n_pad / KC;
    EVAL_LOAD_STAGE(0);
    EVAL_STORE_STAGE(0);
    __syncthreads();
    const int g = lane >> 4, r16 = lane & 15;
    for (int kc = 0; kc < nk; kc++) {
        const int cur = kc & 1;
        if (kc + 1 < nk) EVAL_LOAD_STAGE(kc + 1);
#pragma unroll
        for (int ks = 0; ks < KC / 64; ks++) {
            v4i bf[FN];
#pragma unroll
            for (int ni = 0; ni < FN; ni++) {
                const int nrow = wn * WN + ni * 16 + r16;
                bf[ni] = *(const v4i *)(&Bs[cur][nrow * BPITCH + ks * 64 + g * 16]);
            }
#pragma unroll
            for (int mi = 0; mi < FM; mi++) {
                const int mrow = wm * WM + mi * 16 + r16;
                const uint64_t word = As[cur][mrow * 2 + ks];
                const v4i af = expand16((uint32_t)(word >> (g * 16)) & 0xFFFFu);
#pragma unroll
                for (int ni = 0; ni < FN; ni++)
                    acc[mi][ni] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf[ni], acc[mi][ni], 0, 0, 0);
            }
        }
        if (kc + 1 < nk) {
            EVAL_STORE_STAGE(cur ^ 1);
            __syncthreads();
        }
    }

    // D layout of a 16x16 block: lane holds rows 4*(lane/16) + r, column lane%16.
    if constexpr (!STORE_Y) {
        const int64_t wgt = plane == 0 ? a.weight0 : 1;
        const int word = (n0 + wn * WN) >> 6;  // the wave's 64 columns are one X word
#pragma unroll
        for (int mi = 0; mi < FM; mi++) {
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t row = m0 + wm * WM + mi * 16 + g * 4 + r;
                uint64_t xw = 0;
                if (row < Mrows && word < a.W) xw = a.X[row * a.W + word];
                int s = 0;
#pragma unroll
                for (int ni = 0; ni < FN; ni++) s += ((xw >> (ni * 16 + r16)) & 1ull) ? acc[mi][ni][r] : 0;
                s += __shfl_xor(s, 1);
                s += __shfl_xor(s, 2);
                s += __shfl_xor(s, 4);
                s += __shfl_xor(s, 8);
                if (r16 == 0 && row < Mrows && s != 0)
                    atomicAdd((unsigned long long *)&a.f[row], (unsigned long long)(wgt * (int64_t)s));
            }
        }
    } else if constexpr (EPI == EPI_Y) {
        int32_t *Yp = a.Y + (int64_t)plane * a.M * a.n_pad;
#pragma unroll
        for (int mi = 0; mi < FM; mi++) {
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t row = m0 + wm * WM + mi * 16 + g * 4 + r;
                if (row < Mrows) {
#pragma unroll
                    for (int ni = 0; ni < FN; ni++)
                        Yp[row * a.n_pad + n0 + wn * WN + ni * 16 + r16] = acc[mi][ni][r];
                }
            }
        }
    } else {
        // Ascent keys of the single-plane problem: with y = (x Q)_j and s = 1 - 2 x_j,
        // Delta_j = q_jj + 2 s y_j, key_j = Delta_j * 256 + 2 (127 - j mod PL) + x_j.
        const int word = (n0 + wn * WN) >> 6;
        int32_t dg[FN];
#pragma unroll
        for (int ni = 0; ni < FN; ni++) dg[ni] = a.diag[n0 + wn * WN + ni * 16 + r16];
#pragma unroll
        for (int mi = 0; mi < FM; mi++) {
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t row = m0 + wm * WM + mi * 16 + g * 4 + r;
                if (row < Mrows) {
                    const int64_t xr = a.rows[row];
                    const uint64_t xw = (xr >= 0 && xr < a.x_rows && word < a.W) ? a.X[xr * a.W + word] : 0ull;
#pragma unroll
                    for (int ni = 0; ni < FN; ni++) {
                        const int col = n0 + wn * WN + ni * 16 + r16;
                        const int32_t xj = (int32_t)((xw >> (ni * 16 + r16)) & 1ull);
                        const int32_t y2 = 2 * acc[mi][ni][r];
                        const int32_t delta = dg[ni] + (xj ? -y2 : y2);
                        a.Y[row * a.n_pad + col] = delta * 256 + 2 * (127 - col % a.keys_pl) + xj;
                    }
                }
            }
        }
    }
}

// f[c] = bias * popcount(X_c)^2 (the constant part of the split planes) or 0.
__global__ __launch_bounds__(256) void eval_init(const uint64_t *__restrict__ X, int32_t W, int64_t M, int64_t bias,
                                                 int64_t *__restrict__ f)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= M) return;
    int64_t v = 0;
    if (bias) {
        int64_t k = 0;
        for (int w = 0; w < W; w++) k += __popcll(X[c * W + w]);
        v = bias * k * k;
    }
    f[c] = v;
}

EvalArgs make_args(const ubqp_problem *p, const uint64_t *X, int64_t M)
{
    EvalArgs a{};
    a.q = p->q;
    a.plane_stride = (int64_t)p->n_pad * p->n_pad;
    a.n_pad = p->n_pad;
    a.X = X;
    a.W = p->W;
    a.M = M;
    a.weight0 = p->weight0;
    a.x_rows = M;
    a.m_tiles = (int32_t)((M + BM - 1) / BM);
    a.n_tiles = p->n_pad / BN;
    return a;
}

}  // namespace

hipError_t ubqp_launch_eval(hipStream_t st, const ubqp_problem *p, const uint64_t *X, int64_t M, int64_t *f)
{
    hipLaunchKernelGGL(eval_init, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, X, p->W, M, p->bias, f);
    EvalArgs a = make_args(p, X, M);
    a.f = f;
    const int64_t T = (int64_t)a.m_tiles * a.n_tiles;
    hipLaunchKernelGGL(eval_kernel<EPI_ROWDOT>, dim3((unsigned)T, p->planes), dim3(THR), 0, st, a);
    return hipGetLastError();
}

hipError_t ubqp_launch_yrows(hipStream_t st, const ubqp_problem *p, const uint64_t *X, int64_t x_rows,
                             const int32_t *rows, const int64_t *nrows_d, int64_t offset, int64_t cap, int32_t *Y)
{
    EvalArgs a = make_args(p, X, cap);
    a.x_rows = x_rows;
    a.rows = rows + offset;
    a.offset = offset;
    a.nrows_d = nrows_d;
    a.Y = Y;
    const int64_t T = (int64_t)a.m_tiles * a.n_tiles;
    if (p->planes == 1) {
        a.diag = p->diag;
        a.keys_pl = p->ncol_a / 64;
        hipLaunchKernelGGL(eval_kernel<EPI_KEYS>, dim3((unsigned)T, 1), dim3(THR), 0, st, a);
    } else {
        hipLaunchKernelGGL(eval_kernel<EPI_Y>, dim3((unsigned)T, p->planes), dim3(THR), 0, st, a);
    }
    return hipGetLastError();
}
