// Resident problems: Q is moved to the device once per solve and kept there
// (Pseudocode section).  The caller's coefficients (int8, int16 or int32,
// n x n row-major) are copied to a staging buffer and turned into the resident
// layout by kernels, so the host does no O(n^2) work:
//   check: symmetry, range [-32768, 32767], and whether every entry fits int8;
//   build: int8 planes [planes][n_pad][n_pad] (one plane, or hi = q >> 8 and
//          lo = (q & 255) - 128), the ascent matrix (Q with a zero diagonal,
//          int8 or int16 [n_pad][ncol_a], ncol_a = 1024 ceil(n_pad / 1024)),
//          zero padded;
//   rows:  q_ii and the first-derivative start x_i = [sum_j q_ij > 0].
// The pieces are queued on a caller's stream so that the request server can
// upload one problem while others compute.
#include <new>

#include "ubqp_internal.h"

namespace {

constexpr int THR = 256;

__device__ inline int32_t load_q(const void *q, int elem, int64_t k)
{
    if (elem == 1) return ((const int8_t *)q)[k];
    if (elem == 2) return ((const int16_t *)q)[k];
    return ((const int32_t *)q)[k];
}

__global__ __launch_bounds__(THR) void zero_words(uint32_t *p, int64_t words)
{
    const int64_t k = (int64_t)blockIdx.x * THR + threadIdx.x;
    if (k < words) p[k] = 0;
}

__global__ void check_init(ubqp_check_flags *fl)
{
    fl->bits = 0;
    fl->first[0] = fl->first[1] = ~0ull;
}

// 32 x 32 tiles (I, J), I <= J: tile (I, J) and its mirror (J, I) are read
// row-wise (coalesced), the mirror is transposed through LDS, and q_ij is compared
// with q_ji for j > i; every entry of both tiles is range-checked.
constexpr int CT = 32;
__global__ __launch_bounds__(CT * 8) void check_kernel(const void *q, int elem, int32_t n, ubqp_check_flags *fl)
{
    __shared__ int32_t mir[CT][CT + 1];
    const int I = blockIdx.y, J = blockIdx.x;
    if (I > J) return;
    const int tx = threadIdx.x & (CT - 1), ty = threadIdx.x / CT;
    uint32_t b = 0;
    unsigned long long first_asym = ~0ull, first_range = ~0ull;
    for (int r = ty; r < CT; r += 8) {
        const int64_t i = (int64_t)J * CT + r, j = (int64_t)I * CT + tx;  // mirror tile entry (i, j)
        if (i < n && j < n) {
            const int32_t v = load_q(q, elem, i * n + j);
            mir[tx][r] = v;
            if (v < -32768 || v > 32767) {
                b |= UBQP_CHECK_RANGE;
                first_range = min(first_range, (unsigned long long)(i * n + j));
            }
            if (v < -128 || v > 127) b |= UBQP_CHECK_WIDE;
        }
    }
    __syncthreads();
    for (int r = ty; r < CT; r += 8) {
        const int64_t i = (int64_t)I * CT + r, j = (int64_t)J * CT + tx;
        if (i < n && j < n) {
            const int32_t v = load_q(q, elem, i * n + j);
            if (v < -32768 || v > 32767) {
                b |= UBQP_CHECK_RANGE;
                first_range = min(first_range, (unsigned long long)(i * n + j));
            }
            if (v < -128 || v > 127) b |= UBQP_CHECK_WIDE;
            if (j > i && v != mir[r][tx]) {  // mir[r][tx] = q[J*CT + tx][I*CT + r] = q_ji
                b |= UBQP_CHECK_ASYM;
                first_asym = min(first_asym, (unsigned long long)(i * n + j));
            }
        }
    }
    if (b & UBQP_CHECK_ASYM) atomicMin(&fl->first[0], first_asym);
    if (b & UBQP_CHECK_RANGE) atomicMin(&fl->first[1], first_range);
    if (b) atomicOr(&fl->bits, b);
}

// One thread per entry of the larger of the plane and the ascent matrix.
__global__ __launch_bounds__(THR) void build_kernel(const void *q, int elem, int32_t n, int32_t n_pad, int32_t ncol_a,
                                                    int narrow, int8_t *planes, void *qa)
{
    const int64_t k = (int64_t)blockIdx.x * THR + threadIdx.x;
    const int64_t cols = ncol_a > n_pad ? ncol_a : n_pad;
    if (k >= (int64_t)n_pad * cols) return;
    const int64_t i = k / cols, j = k - i * cols;
    const bool in = i < n && j < n;
    const int32_t v = in ? load_q(q, elem, i * n + j) : 0;
    if (j < n_pad) {
        if (narrow) {
            planes[i * n_pad + j] = (int8_t)v;
        } else {
            planes[i * n_pad + j] = (int8_t)(v >> 8);
            planes[(int64_t)n_pad * n_pad + i * n_pad + j] = in ? (int8_t)((v & 255) - 128) : (int8_t)0;
        }
    }
    const int32_t a = (i == j) ? 0 : v;
    if (j < ncol_a) {
        if (narrow)
            ((int8_t *)qa)[i * ncol_a + j] = (int8_t)a;
        else
            ((int16_t *)qa)[i * ncol_a + j] = (int16_t)a;
    }
}

// One block per row: q_ii and the derivative-start bit of the row (deriv zeroed before).
__global__ __launch_bounds__(THR) void rows_kernel(const void *q, int elem, int32_t n, int32_t *diag,
                                                   unsigned long long *deriv)
{
    __shared__ int64_t part[THR / 64];
    const int64_t i = blockIdx.x;
    int64_t s = 0;
    if (i < n)
        for (int64_t j = threadIdx.x; j < n; j += THR) s += load_q(q, elem, i * n + j);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        s = 0;
        for (int w = 0; w < THR / 64; w++) s += part[w];
        diag[i] = i < n ? load_q(q, elem, i * n + i) : 0;
        if (i < n && s > 0) atomicOr(&deriv[i >> 6], 1ull << (i & 63));
    }
}

}  // namespace

void ubqp_problem_geometry(ubqp_problem *p, int32_t n, int32_t planes)
{
    p->n = n;
    p->n_pad = (n + UBQP_NPAD_ALIGN - 1) / UBQP_NPAD_ALIGN * UBQP_NPAD_ALIGN;
    p->W = (n + 63) / 64;
    p->planes = planes;
    p->weight0 = planes == 1 ? 1 : 256;
    p->bias = planes == 1 ? 0 : 128;
    const int64_t np = p->n_pad;
    p->ncol_a = (int32_t)((np + 1023) / 1024 * 1024);
}

size_t ubqp_problem_bytes(const ubqp_problem *p)
{
    const size_t np = (size_t)p->n_pad;
    const size_t qa = np * (size_t)p->ncol_a * (p->planes == 1 ? 1 : 2);
    return ((size_t)p->planes * np * np + 255) / 256 * 256 + (qa + 255) / 256 * 256 + (np * 4 + 255) / 256 * 256 +
           ((size_t)p->W * 8 + 255) / 256 * 256;
}

void ubqp_problem_bind(ubqp_problem *p, char *mem)
{
    const size_t np = (size_t)p->n_pad;
    const size_t qa = np * (size_t)p->ncol_a * (p->planes == 1 ? 1 : 2);
    size_t off = 0;
    p->q = (int8_t *)(mem + off);
    off += ((size_t)p->planes * np * np + 255) / 256 * 256;
    p->qa = mem + off;
    off += (qa + 255) / 256 * 256;
    p->diag = (int32_t *)(mem + off);
    off += (np * 4 + 255) / 256 * 256;
    p->deriv_x = (uint64_t *)(mem + off);
}

hipError_t ubqp_queue_problem_check(hipStream_t st, const void *stage, int elem, int32_t n, ubqp_check_flags *fl)
{
    const unsigned T = (unsigned)((n + CT - 1) / CT);
    hipLaunchKernelGGL(check_init, dim3(1), dim3(1), 0, st, fl);
    hipLaunchKernelGGL(check_kernel, dim3(T, T), dim3(CT * 8), 0, st, stage, elem, n, fl);
    return hipGetLastError();
}

hipError_t ubqp_queue_problem_build(hipStream_t st, const void *stage, int elem, const ubqp_problem *p)
{
    const int64_t np = p->n_pad, cols = p->ncol_a > np ? p->ncol_a : np;
    hipLaunchKernelGGL(zero_words, dim3((unsigned)((2 * p->W + THR - 1) / THR)), dim3(THR), 0, st,
                       (uint32_t *)p->deriv_x, (int64_t)2 * p->W);
    hipLaunchKernelGGL(build_kernel, dim3((unsigned)((np * cols + THR - 1) / THR)), dim3(THR), 0, st, stage, elem,
                       p->n, (int32_t)np, p->ncol_a, p->planes == 1 ? 1 : 0, p->q, p->qa);
    hipLaunchKernelGGL(rows_kernel, dim3((unsigned)np), dim3(THR), 0, st, stage, elem, p->n, p->diag,
                       (unsigned long long *)p->deriv_x);
    return hipGetLastError();
}

hipError_t ubqp_queue_zero(hipStream_t st, void *p, int64_t words)
{
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_words, dim3((unsigned)((words + THR - 1) / THR)), dim3(THR), 0, st, (uint32_t *)p, words);
    return hipGetLastError();
}

int ubqp_check_outcome(ubqp_ctx *ctx, const ubqp_check_flags &fl, int32_t n)
{
    if (fl.bits & UBQP_CHECK_RANGE) {
        const long long k = (long long)fl.first[1];
        return ubqp_fail(ctx, UBQP_ERANGE, "q[%lld][%lld] outside [-32768, 32767]", k / n, k % n);
    }
    if (fl.bits & UBQP_CHECK_ASYM) {
        const long long k = (long long)fl.first[0];
        return ubqp_fail(ctx, UBQP_EASYM, "q[%lld][%lld] != q[%lld][%lld]", k / n, k % n, k % n, k / n);
    }
    return UBQP_OK;
}

extern "C" {

int ubqp_problem_create_typed(ubqp_ctx *ctx, int32_t n, const void *q, int32_t elem_bytes, ubqp_problem **out)
{
    if (!ctx || !q || !out) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    *out = nullptr;
    if (n < 1 || n > UBQP_MAX_N) return ubqp_fail(ctx, UBQP_EINVAL, "n=%d outside [1, %d]", n, UBQP_MAX_N);
    if (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4)
        return ubqp_fail(ctx, UBQP_EINVAL, "element size %d not 1, 2 or 4", elem_bytes);
    UBQP_TRY(ubqp_set_device(ctx));
    hipStream_t st = ctx->stream;
    const size_t q_bytes = (size_t)n * n * elem_bytes;
    const size_t stage_bytes = (q_bytes + 255) / 256 * 256 + 256;
    void *stage_v = nullptr;
    UBQP_TRY(ubqp_ws_ensure(ctx, ubqp_ctx::WS_STAGE, stage_bytes, &stage_v));
    char *stage = (char *)stage_v;
    ubqp_check_flags *fl = (ubqp_check_flags *)(stage + (stage_bytes - 256));
    ubqp_check_flags hf{};
    UBQP_HIP_TRY(ctx, hipMemcpyAsync(stage, q, q_bytes, hipMemcpyHostToDevice, st));
    UBQP_HIP_TRY(ctx, ubqp_queue_problem_check(st, stage, elem_bytes, n, fl));
    UBQP_HIP_TRY(ctx, hipMemcpyAsync(&hf, fl, sizeof hf, hipMemcpyDeviceToHost, st));
    UBQP_HIP_TRY(ctx, hipStreamSynchronize(st));
    UBQP_TRY(ubqp_check_outcome(ctx, hf, n));
    ubqp_problem *p = new (std::nothrow) ubqp_problem();
    if (!p) return ubqp_fail(ctx, UBQP_ENOMEM, "host allocation");
    p->ctx = ctx;
    ubqp_ctx_hold(ctx);
    ubqp_problem_geometry(p, n, (hf.bits & UBQP_CHECK_WIDE) ? 2 : 1);
    hipError_t e = hipMalloc(&p->mem, ubqp_problem_bytes(p));
    if (e == hipSuccess) {
        ubqp_problem_bind(p, (char *)p->mem);
        e = ubqp_queue_problem_build(st, stage, elem_bytes, p);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        ubqp_problem_destroy(p);
        return ubqp_hip_fail(ctx, e, "problem upload");
    }
    *out = p;
    return UBQP_OK;
}

int ubqp_problem_create(ubqp_ctx *ctx, int32_t n, const int32_t *q_host, ubqp_problem **out)
{
    return ubqp_problem_create_typed(ctx, n, q_host, 4, out);
}

int ubqp_problem_destroy(ubqp_problem *p)
{
    if (!p) return UBQP_EINVAL;
    ubqp_ctx *ctx = p->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (p->mem) (void)hipFree(p->mem);
    delete p;
    ubqp_ctx_drop(ctx);
    return UBQP_OK;
}

int ubqp_problem_info(const ubqp_problem *p, int32_t *n, int32_t *n_pad, int32_t *planes)
{
    if (!p) return UBQP_EINVAL;
    if (n) *n = p->n;
    if (n_pad) *n_pad = p->n_pad;
    if (planes) *planes = p->planes;
    return UBQP_OK;
}

int ubqp_problem_set_flip_limit(ubqp_problem *p, int32_t limit)
{
    if (!p) return UBQP_EINVAL;
    if (limit < 0) return ubqp_fail(p->ctx, UBQP_EINVAL, "flip limit %d < 0", limit);
    p->flip_limit = limit;
    return UBQP_OK;
}

}  // extern "C"

int32_t ubqp_problem_flip_limit(const ubqp_problem *p)
{
    return p->flip_limit > 0 ? p->flip_limit : 64 * p->n_pad + 4096;
}
