// calib.hip -- device calibration for the roofline of the Metropolis sweep
// (gfx950): the rate at which the chip draws Philox4x32-10 words with the
// sweep's counter pattern and nothing else, and the rate of plain 32-bit
// integer VALU work.  The sweep's random numbers (one 32-bit word per
// attempted spin flip, Sec. III.A) are its largest cost, so the first rate
// is the practical ceiling of any sweep that draws them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "runner.h"
#include "step_common.h"

namespace pamc {

namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = 256 * 8;  // eight workgroups per compute unit
constexpr int kSweeps = 10;       // sweeps per replica, as in the workloads
constexpr int kReplicas = 512;    // replicas each thread draws for
constexpr int kValuIters = 1 << 14;
constexpr int kChains = 8;

// One thread stands for one Philox block (four sites) of one colour: for
// each of its replicas and each sweep it draws the block at counter
// (block, replica, step, TAG_SWEEP | sweep), as the sweep kernels do, and
// folds the four words into an accumulator so that nothing is dropped.
__global__ __launch_bounds__(kThreads) void k_philox_only(uint32_t key0, uint32_t key1, int k, uint32_t *out)
{
    const uint32_t g = blockIdx.x * kThreads + threadIdx.x;
    uint32_t acc = 0;
    for (int r = 0; r < kReplicas; ++r) {
#pragma unroll 2
        for (int t = 0; t < kSweeps; ++t) {
            const uint4 u = philox10(make_uint4(g, (uint32_t)r, (uint32_t)k, kTagSweep | (uint32_t)t), key0, key1);
            acc = xor3(acc, u.x, u.y);
            acc = xor3(acc, u.z, u.w);
        }
    }
    out[g] = acc;
}

// kChains independent chains of a three-input XOR and an add per step:
// two full-rate int32 VALU operations per chain and iteration.
__global__ __launch_bounds__(kThreads) void k_valu_only(uint32_t seed, uint32_t *out)
{
    uint32_t x[kChains], y[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        x[j] = seed + threadIdx.x + 977u * j;
        y[j] = blockIdx.x ^ (0x9E3779B9u * (j + 1));
    }
    for (int i = 0; i < kValuIters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            x[j] = xor3(x[j], y[j], (uint32_t)i);
            y[j] = y[j] + x[j];
        }
    }
    uint32_t a = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) a ^= x[j] ^ y[j];
    out[blockIdx.x * kThreads + threadIdx.x] = a;
}

}  // namespace

}  // namespace pamc

extern "C" int pamc_calibrate(int device, double *philox_words_per_ns, double *valu_ops_per_ns)
{
    using namespace pamc;
    if (device >= 0 && hipSetDevice(device) != hipSuccess) {
        set_error("pamc_calibrate: hipSetDevice failed");
        return PAMC_ERR_DEVICE;
    }
    uint32_t *out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int status = PAMC_OK;
    const size_t n = (size_t)kBlocks * kThreads;
    auto fail = [&](const char *what) {
        set_error(std::string("pamc_calibrate: ") + what);
        status = PAMC_ERR_DEVICE;
    };
    if (hipMalloc(&out, n * 4) != hipSuccess) {
        set_error("pamc_calibrate: device allocation failed");
        return PAMC_ERR_NOMEM;
    }
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&ev[0]) != hipSuccess ||
        hipEventCreate(&ev[1]) != hipSuccess) {
        fail("stream or event creation failed");
    }
    float best_p = 1e30f, best_v = 1e30f;
    for (int rep = 0; rep < 3 && status == PAMC_OK; ++rep) {
        float ms = 0.f;
        hipEventRecord(ev[0], st);
        k_philox_only<<<kBlocks, kThreads, 0, st>>>(0x12345678u, 0x9ABCDEF0u, 77, out);
        hipEventRecord(ev[1], st);
        if (hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
            fail("Philox kernel failed");
            break;
        }
        if (rep > 0) best_p = std::min(best_p, ms);
        hipEventRecord(ev[0], st);
        k_valu_only<<<kBlocks, kThreads, 0, st>>>((uint32_t)rep, out);
        hipEventRecord(ev[1], st);
        if (hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
            fail("VALU kernel failed");
            break;
        }
        if (rep > 0) best_v = std::min(best_v, ms);
    }
    if (status == PAMC_OK) {
        const double words = 4.0 * (double)n * kReplicas * kSweeps;
        const double ops = 2.0 * kChains * (double)kValuIters * (double)n;
        if (philox_words_per_ns) *philox_words_per_ns = words / (best_p * 1e6);
        if (valu_ops_per_ns) *valu_ops_per_ns = ops / (best_v * 1e6);
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(out);
    return status;
}
