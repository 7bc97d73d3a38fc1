// Measurement: the int8 matrix-core rate this device sustains on
// v_mfma_i32_32x32x32_i8 with operands in registers (no memory traffic), the
// instruction the evaluation and the Delta initialisation are built on.  The
// evaluation's MFMA fraction is reported against both this figure and the
// published dense int8 peak.
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
