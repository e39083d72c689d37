// Parallel-tempering kernels for gfx950 (appendix A, "Adaptive Parallel
// Tempering"; the replica-exchange step that opens algorithm 1).
//
// Replicas are laid out temperature-major: replica r = i * n_chains + c is
// ladder position i (inverse temperatures ascending in i) of chain c, so the
// replicas of one sweep workgroup (4 for k-SAT, 16 for QAP) share one
// temperature and the sweep kernels keep wave-uniform threshold tables.  An
// exchange moves configurations, not temperatures: neighbour positions i and
// i + 1 of a chain swap with probability
//   min{1, exp[(beta_i - beta_{i+1}) (E_i - E_{i+1})]},
// always when E_i <= E_{i+1}; otherwise word 0 of the Philox block at counter
// (c, t, i, PT_SWAP) is compared with the factored threshold of the gap.
// Pairs of one step are disjoint (i = parity, parity + 2, ...), so every
// pair is decided and moved by its own workgroup with no ordering between
// them.  The ladder's energy spread comes from exact 128-bit integer sums.
#include "nmc_internal.h"
#include "nmc_philox.h"

namespace nmc {

namespace {

// (A[d >> 10] * B[d & 1023]) >> 32 for pair position i; A is zero past len
__device__ __forceinline__ uint32_t pt_threshold(const PtCall &C, int i, unsigned long long d) {
    const unsigned long long h = d >> kQapLowBits;
    const int len = C.len[i];
    if (h >= (unsigned long long)len)
        return 0u;
    const uint32_t *A = C.tab + C.off[i];
    const unsigned long long a = A[h];
    const unsigned long long b = A[len + (int)(d & ((1u << kQapLowBits) - 1u))];
    return (uint32_t)((a * b) >> 32);
}

// true when the configurations at positions i (energy ea) and i + 1 (eb) of
// chain c exchange
__device__ __forceinline__ bool pt_decide(const PtCall &C, int i, int c, long long ea, long long eb) {
    const long long d = ea - eb;
    if (d <= 0)
        return true;
    const uint4 u = philox4x32_10((uint32_t)c, C.t, (uint32_t)i, kStreamPtSwap, C.key0, C.key1);
    return u.x < pt_threshold(C, i, (unsigned long long)d);
}

// swap the bits of mask m (replicated per byte in m4) between two spin rows
template <typename W>
__device__ __forceinline__ void swap_masked(W *a, W *b, int words, uint32_t m4, int tid, int nthr) {
    for (int k = tid; k < words; k += nthr) {
        const W va = a[k], vb = b[k];
        W na, nb;
        if constexpr (sizeof(W) == 16) {
            na.x = (va.x & ~m4) | (vb.x & m4);
            na.y = (va.y & ~m4) | (vb.y & m4);
            na.z = (va.z & ~m4) | (vb.z & m4);
            na.w = (va.w & ~m4) | (vb.w & m4);
            nb.x = (vb.x & ~m4) | (va.x & m4);
            nb.y = (vb.y & ~m4) | (va.y & m4);
            nb.z = (vb.z & ~m4) | (va.z & m4);
            nb.w = (vb.w & ~m4) | (va.w & m4);
        } else {
            na = (W)((va & ~(W)m4) | (vb & (W)m4));
            nb = (W)((vb & ~(W)m4) | (va & (W)m4));
        }
        a[k] = na;
        b[k] = nb;
    }
}

constexpr int kExchangeThreads = 256;

// k-SAT: one workgroup per (pair position, group column).  A group column
// holds chains 4gc..4gc+3, which are bits 0..3 of the spin bytes of group
// i * (n_chains / 4) + gc at position i and of the group n_chains / 4 further
// on at position i + 1: the four decisions form one byte mask.
__global__ void __launch_bounds__(kExchangeThreads) pt_exchange_ksat_kernel(KsatDev I, KsatRepDev R, PtCall C) {
    __shared__ uint32_t smask;
    const int i = C.parity + 2 * (int)blockIdx.x;
    const int gc = blockIdx.y;
    const int tid = threadIdx.x;
    const int cpg = C.n_chains / kGroup;
    if (tid < 64) {
        bool sw = false;
        if (tid < kGroup) {
            const int c = gc * kGroup + tid;
            const int a = i * C.n_chains + c, b = a + C.n_chains;
            const int ea = R.energy[a], eb = R.energy[b];
            sw = pt_decide(C, i, c, ea, eb);
            if (sw) {
                R.energy[a] = eb;
                R.energy[b] = ea;
            }
        }
        const unsigned long long bal = __ballot(sw);
        if (tid == 0) {
            smask = (uint32_t)bal;
            atomicAdd(&C.attempted[i], (unsigned long long)kGroup);
            if (bal)
                atomicAdd(&C.accepted[i], (unsigned long long)__popcll(bal));
        }
    }
    __syncthreads();
    const uint32_t m = smask;
    if (!m)
        return;
    const int n = I.n;
    const size_t ga = (size_t)i * cpg + gc, gb = ga + cpg;
    uint8_t *xa = R.xs + ga * n, *xb = R.xs + gb * n;
    const uint32_t m4 = m * 0x01010101u;
    if ((n & 15) == 0)
        swap_masked(reinterpret_cast<uint4 *>(xa), reinterpret_cast<uint4 *>(xb), n / 16, m4, tid, blockDim.x);
    else if ((n & 3) == 0)
        swap_masked(reinterpret_cast<uint32_t *>(xa), reinterpret_cast<uint32_t *>(xb), n / 4, m4, tid, blockDim.x);
    else
        swap_masked(xa, xb, n, m4, tid, blockDim.x);
}

// QAP: one wave per (pair position, chain); every lane takes the same
// decision from the same inputs, lane 0 moves the costs and counts.
__global__ void __launch_bounds__(64) pt_exchange_qap_kernel(QapDev I, QapRepDev R, PtCall C) {
    const int i = C.parity + 2 * (int)blockIdx.x;
    const int c = blockIdx.y;
    const int lane = threadIdx.x;
    const size_t a = (size_t)i * C.n_chains + c, b = a + C.n_chains;
    const long long ea = R.cost[a], eb = R.cost[b];
    const bool sw = pt_decide(C, i, c, ea, eb);
    if (lane == 0) {
        atomicAdd(&C.attempted[i], 1ull);
        if (sw) {
            atomicAdd(&C.accepted[i], 1ull);
            R.cost[a] = eb;
            R.cost[b] = ea;
        }
    }
    if (!sw)
        return;
    const int n = I.n;
    uint8_t *pa = R.perm + a * n, *pb = R.perm + b * n;
    for (int f = lane; f < n; f += 64) {
        const uint8_t va = pa[f], vb = pb[f];
        pa[f] = vb;
        pb[f] = va;
    }
}

// One workgroup sums count, E and E^2 over all replicas.  E < 2^32, so E^2
// fits 64 bits and the sums of squares are carried as (low, high) pairs.
constexpr int kMomentThreads = 1024;

__global__ void __launch_bounds__(kMomentThreads) pt_moments_kernel(const void *energy, int is64, int n,
                                                                    unsigned long long *acc) {
    __shared__ unsigned long long s_s1[kMomentThreads], s_lo[kMomentThreads], s_hi[kMomentThreads];
    const int tid = threadIdx.x;
    unsigned long long s1 = 0, lo = 0, hi = 0;
    for (int r = tid; r < n; r += kMomentThreads) {
        const unsigned long long e = is64 ? (unsigned long long)reinterpret_cast<const long long *>(energy)[r]
                                          : (unsigned long long)(unsigned)reinterpret_cast<const int *>(energy)[r];
        const unsigned long long sq = e * e;
        s1 += e;
        lo += sq;
        hi += lo < sq ? 1ull : 0ull;
    }
    s_s1[tid] = s1;
    s_lo[tid] = lo;
    s_hi[tid] = hi;
    __syncthreads();
    for (int w = kMomentThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            s_s1[tid] += s_s1[tid + w];
            const unsigned long long l = s_lo[tid] + s_lo[tid + w];
            s_hi[tid] += s_hi[tid + w] + (l < s_lo[tid] ? 1ull : 0ull);
            s_lo[tid] = l;
        }
        __syncthreads();
    }
    if (tid == 0) {
        acc[0] += (unsigned long long)n;
        acc[1] += s_s1[0];
        const unsigned long long l = acc[2] + s_lo[0];
        acc[3] += s_hi[0] + (l < acc[2] ? 1ull : 0ull);
        acc[2] = l;
    }
}

int pairs_of(const PtCall &C) { return (C.n_temps - C.parity) / 2; }

}  // namespace

hipError_t pt_launch_exchange_ksat(const KsatDev &I, const KsatRepDev &R, const PtCall &C, hipStream_t s) {
    const int np = pairs_of(C);
    if (np <= 0 || C.n_chains <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(pt_exchange_ksat_kernel, dim3(np, C.n_chains / kGroup), dim3(kExchangeThreads), 0, s, I, R,
                       C);
    return hipGetLastError();
}

hipError_t pt_launch_exchange_qap(const QapDev &I, const QapRepDev &R, const PtCall &C, hipStream_t s) {
    const int np = pairs_of(C);
    if (np <= 0 || C.n_chains <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(pt_exchange_qap_kernel, dim3(np, C.n_chains), dim3(64), 0, s, I, R, C);
    return hipGetLastError();
}

hipError_t pt_launch_moments(const void *energy, int energy_is_64, int n, unsigned long long *acc, hipStream_t s) {
    hipLaunchKernelGGL(pt_moments_kernel, dim3(1), dim3(kMomentThreads), 0, s, energy, energy_is_64, n, acc);
    return hipGetLastError();
}

}  // namespace nmc
