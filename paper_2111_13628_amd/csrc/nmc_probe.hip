// Peak-rate probes for gfx950 (measurement helpers, not part of the method):
// what one launch of simple, fully occupied kernels reaches for the
// operations the sweep kernels are built from.
//
//   LDS_DISTINCT  byte reads from LDS, every lane of a wave on its own bank
//                 (address 4 * lane + a multiple of 256)
//   LDS_RANDOM    byte reads from LDS at uniformly random addresses inside a
//                 100 KB table (the spin tables' size at N = 50,000)
//   VALU_INT      32-bit integer adds: eight chains per lane, each step
//                 x_j += x_{j+1 mod 8} (one v_add_u32 per chain and step)
//
// Every workgroup has 1024 threads (16 waves) and, for the LDS probes, a
// 100 KB dynamic LDS block, so one workgroup runs per CU as in the k-SAT
// sweep.  Each lane keeps 16 read addresses in registers; the eight
// iterations of an unrolled group add offsets 0, 128, ..., 896 (immediates of
// the read instructions, which keep every lane's bank), and a compiler fence
// per iteration keeps the reads from being merged or hoisted.  The results feed a store guarded by a comparison with a value
// the host passes in (one no lane produces), so the compiler cannot drop the
// work as dead.
#include <cstdio>
#include <mutex>

#include "nmc.h"
#include "nmc_internal.h"

namespace nmc {

namespace {

constexpr int kProbeThreads = 1024;
constexpr int kProbeLdsBytes = 100 * 1024;
constexpr int kProbeAddrs = 16;
constexpr int kProbeChains = 8;

typedef __attribute__((address_space(3))) const uint8_t probe_lds_cu8;

__device__ __forceinline__ uint32_t probe_lds_u8(uint32_t a) { return *(probe_lds_cu8 *)(uintptr_t)a; }

__device__ __forceinline__ uint32_t xorshift(uint32_t h) {
    h ^= h << 13;
    h ^= h >> 17;
    h ^= h << 5;
    return h;
}

__global__ void __launch_bounds__(kProbeThreads) probe_lds_kernel(int groups, int random, uint32_t never,
                                                                  uint32_t *sink) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t *w = reinterpret_cast<uint32_t *>(lds);
    for (int i = tid; i < kProbeLdsBytes / 4; i += kProbeThreads)
        w[i] = (uint32_t)i * 2654435761u;
    // addresses stay below kProbeLdsBytes - 1024 so that the offset (at most
    // 7 * 128) keeps every read inside the block
    uint32_t a[kProbeAddrs];
    uint32_t h = ((uint32_t)blockIdx.x * kProbeThreads + (uint32_t)tid) * 2654435761u + 0x9E3779B9u;
#pragma unroll
    for (int j = 0; j < kProbeAddrs; ++j) {
        if (random) {
            h = xorshift(h);
            a[j] = h % (uint32_t)(kProbeLdsBytes - 1024);
        } else {
            a[j] = 4u * (uint32_t)lane + 256u * (uint32_t)((j * 37 + wave * 5) % 350);
        }
    }
    __syncthreads();
    uint32_t acc = 0;
    for (int it = 0; it < groups; ++it) {
#pragma unroll
        for (int o = 0; o < 8; ++o) {
#pragma unroll
            for (int j = 0; j < kProbeAddrs; ++j)
                acc |= probe_lds_u8(a[j] + 128u * o);
            __asm__ volatile("" ::: "memory");
        }
    }
    if (acc == never)
        sink[0] = acc;
}

__global__ void __launch_bounds__(kProbeThreads) probe_valu_kernel(int iters, uint32_t never, uint32_t *sink) {
    uint32_t x[kProbeChains];
#pragma unroll
    for (int j = 0; j < kProbeChains; ++j)
        x[j] = ((uint32_t)blockIdx.x * kProbeThreads + threadIdx.x) * (2u * j + 1u);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kProbeChains; ++j)
            x[j] += x[(j + 1) % kProbeChains];
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < kProbeChains; ++j)
        r ^= x[j];
    // r == never for some lane is possible but harmless: the store then only
    // writes the sink word
    if (r == never)
        sink[0] = r;
}

// one 256-byte word per device, allocated on the device's first probe and
// kept until the process ends
constexpr int kProbeMaxDevices = 64;

uint32_t *probe_sink() {
    static std::mutex mu;
    static uint32_t *sinks[kProbeMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kProbeMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!sinks[dev] && hipMalloc((void **)&sinks[dev], 256) != hipSuccess)
        sinks[dev] = nullptr;
    return sinks[dev];
}

}  // namespace

}  // namespace nmc

extern "C" int nmc_probe_peak(int32_t which, int32_t iters, int32_t blocks, double *ms_out, double *lane_ops_out,
                              void *stream) {
    using namespace nmc;
    char msg[160];
    if (!ms_out || !lane_ops_out)
        return set_last_error(NMC_ERR_INVALID, "NULL argument");
    if (which < NMC_PROBE_LDS_DISTINCT || which > NMC_PROBE_VALU_INT) {
        snprintf(msg, sizeof msg, "unknown probe %d", which);
        return set_last_error(NMC_ERR_INVALID, msg);
    }
    if (iters < 8 || iters > (1 << 24) || iters % 8 || blocks < 1 || blocks > (1 << 16)) {
        snprintf(msg, sizeof msg, "iters = %d must be a multiple of 8 in [8, 2^24] and blocks = %d in [1, 2^16]",
                 iters, blocks);
        return set_last_error(NMC_ERR_INVALID, msg);
    }
    uint32_t *sink = probe_sink();
    if (!sink)
        return set_last_error(NMC_ERR_DEVICE, "probe sink allocation failed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    static const hipError_t attr = hipFuncSetAttribute((const void *)probe_lds_kernel,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, kProbeLdsBytes);
    if (attr != hipSuccess)
        return set_last_error(NMC_ERR_DEVICE, hipGetErrorString(attr));
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return set_last_error(NMC_ERR_DEVICE, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_last_error(NMC_ERR_DEVICE, "hipEventCreate failed");
    }
    hipError_t err = hipEventRecord(e0, s);
    if (err == hipSuccess) {
        if (which == NMC_PROBE_VALU_INT)
            hipLaunchKernelGGL(probe_valu_kernel, dim3(blocks), dim3(kProbeThreads), 0, s, iters, 0xFFFFFFFFu, sink);
        else
            hipLaunchKernelGGL(probe_lds_kernel, dim3(blocks), dim3(kProbeThreads), kProbeLdsBytes, s, iters / 8,
                               which == NMC_PROBE_LDS_RANDOM ? 1 : 0, 0xFFFFFFFFu, sink);
        err = hipGetLastError();
    }
    if (err == hipSuccess)
        err = hipEventRecord(e1, s);
    if (err == hipSuccess)
        err = hipEventSynchronize(e1);
    float ms = 0;
    if (err == hipSuccess)
        err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess)
        return set_last_error(NMC_ERR_DEVICE, hipGetErrorString(err));
    const double per_lane = which == NMC_PROBE_VALU_INT ? (double)kProbeChains : (double)kProbeAddrs;
    *ms_out = ms;
    *lane_ops_out = (double)blocks * kProbeThreads * (double)iters * per_lane;
    return set_last_error(NMC_OK, "");
}
