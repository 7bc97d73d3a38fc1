// Measurements of the device's ceilings, the denominators of the kernels'
// rooflines:
//   ubqp_mfma_peak: the int8 matrix-core rate sustained on v_mfma_i32_32x32x32_i8
//     with operands in registers (no memory traffic), the instruction the
//     evaluation and the Delta initialisation are built on;
//   ubqp_read_peak: the read bandwidth a streaming kernel gets from a buffer of a
//     given size -- a few MB stays in each XCD's L2, about a hundred MB in the
//     Infinity Cache, GBs stream from HBM -- the levels the ascent's row reads
//     are served from.
#include "ubqp_internal.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int THR = 256;         // four waves per block
constexpr int CHAINS = 4;        // independent accumulators per wave
constexpr int64_t OPS_PER_MFMA = 2ll * 32 * 32 * 32;

__global__ __launch_bounds__(THR) void mfma_loop(int iters, int32_t *out)
{
    const int t = blockIdx.x * THR + threadIdx.x;
    v4i a = {t, t ^ 0x5a5a5a5a, t * 3, t + 7};
    v4i b = {t * 5, t ^ 0x3c3c3c3c, t + 11, t * 13};
    v16i acc[CHAINS];
    for (int k = 0; k < CHAINS; k++)
        for (int e = 0; e < 16; e++) acc[k][e] = k + e;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int k = 0; k < CHAINS; k++) acc[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[k], 0, 0, 0);
    }
    int32_t s = 0;
    for (int k = 0; k < CHAINS; k++)
        for (int e = 0; e < 16; e++) s += acc[k][e];
    out[t] = s;
}

}  // namespace

extern "C" int ubqp_mfma_peak(ubqp_ctx *ctx, double *tops)
{
    if (!ctx || !tops) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    UBQP_TRY(ubqp_set_device(ctx));
    int cus = 0;
    UBQP_HIP_TRY(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int blocks = 4 * (cus > 0 ? cus : 1);  // 16 waves per compute unit, four per SIMD
    const int iters = 4000;
    void *out = nullptr;
    UBQP_TRY(ubqp_ws_ensure(ctx, ubqp_ctx::WS_STAGE, (size_t)blocks * THR * 4, &out));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    UBQP_HIP_TRY(ctx, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    float best = 0.f;
    for (int rep = 0; e == hipSuccess && rep < 4; rep++) {
        e = hipEventRecord(e0, ctx->stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(mfma_loop, dim3(blocks), dim3(THR), 0, ctx->stream, iters, (int32_t *)out);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rep > 0 && (best == 0.f || ms < best)) best = ms;  // the first run warms up
    }
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    UBQP_HIP_TRY(ctx, e);
    const double ops = (double)blocks * (THR / 64) * iters * CHAINS * OPS_PER_MFMA;
    *tops = ops / (best * 1e-3) / 1e12;
    return UBQP_OK;
}

namespace {

constexpr int RTHR = 256;
constexpr int RUNROLL = 8;  // independent 16-byte loads in flight per thread

// Block b reads `per_block` bytes cycling through its window of `window` bytes,
// which starts at byte b * window of the buffer (modulo its size; the window
// divides the buffer, so it never wraps), as rows of RTHR * 16 contiguous bytes
// (one coalesced 4 KB access per wave-row).  The XOR of everything read is stored
// per thread so that no load is dead.
__global__ __launch_bounds__(RTHR) void read_loop(const uint4 *buf, int64_t nvec, int64_t win_vec,
                                                  int64_t per_block_vec, uint32_t *out)
{
    const int64_t start = ((int64_t)blockIdx.x * win_vec) % nvec;
    const int64_t rows = per_block_vec / RTHR;
    uint32_t acc = 0;
    int64_t off = threadIdx.x;  // offset inside the window, < win_vec
    for (int64_t r = 0; r < rows; r += RUNROLL) {
        uint4 v[RUNROLL];
#pragma unroll
        for (int u = 0; u < RUNROLL; u++) {
            v[u] = ubqp_ldg16(buf + start + off);
            off += RTHR;
            if (off >= win_vec) off -= win_vec;
        }
#pragma unroll
        for (int u = 0; u < RUNROLL; u++) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    out[(int64_t)blockIdx.x * RTHR + threadIdx.x] = acc;
}

__global__ void fill_words(uint32_t *p, int64_t words)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)(i * 2654435761u);
}

}  // namespace

extern "C" int ubqp_read_peak(ubqp_ctx *ctx, int64_t bytes, int64_t window, int64_t per_block, double *gbs)
{
    if (!ctx || !gbs) return ubqp_fail(ctx, UBQP_EINVAL, "null argument");
    const int64_t row = (int64_t)RTHR * 16 * RUNROLL;
    if (bytes < (1 << 20) || bytes > (1ll << 36) || bytes % 4096 != 0)
        return ubqp_fail(ctx, UBQP_EINVAL, "bytes=%lld outside [1 MiB, 64 GiB] or not a multiple of 4 KiB",
                         (long long)bytes);
    if (window < 4096 || window % 4096 != 0 || bytes % window != 0)
        return ubqp_fail(ctx, UBQP_EINVAL, "window=%lld not a multiple of 4 KiB dividing bytes", (long long)window);
    if (per_block < row || per_block % row != 0)
        return ubqp_fail(ctx, UBQP_EINVAL, "per_block=%lld not a positive multiple of %lld", (long long)per_block,
                         (long long)row);
    UBQP_TRY(ubqp_set_device(ctx));
    int cus = 0;
    UBQP_HIP_TRY(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int blocks = 8 * (cus > 0 ? cus : 1);
    void *buf = nullptr, *out = nullptr;
    UBQP_HIP_TRY(ctx, hipMalloc(&buf, (size_t)bytes));
    hipError_t e = hipMalloc(&out, (size_t)blocks * RTHR * 4);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fill_words, dim3(2048), dim3(256), 0, ctx->stream, (uint32_t *)buf, bytes / 4);
        e = hipGetLastError();
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 0.f;
    for (int rep = 0; e == hipSuccess && rep < 4; rep++) {
        e = hipEventRecord(e0, ctx->stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(read_loop, dim3(blocks), dim3(RTHR), 0, ctx->stream, (const uint4 *)buf, bytes / 16,
                               window / 16, per_block / 16, (uint32_t *)out);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rep > 0 && (best == 0.f || ms < best)) best = ms;  // the first run warms up
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    const hipError_t se = hipStreamSynchronize(ctx->stream);
    if (out) (void)hipFree(out);
    (void)hipFree(buf);
    UBQP_HIP_TRY(ctx, e);
    UBQP_HIP_TRY(ctx, se);
    *gbs = (double)blocks * per_block / (best * 1e-3) / 1e9;
    return UBQP_OK;
}
