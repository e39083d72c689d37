// Collective flips of backbone clusters for gfx950 (the nonlocal move of the
// NMC scheme: a whole cluster of rigid variables flipped at once, accepted by
// the Metropolis rule; the section on annealed thresholds names it as the
// alternative to heating the backbone).
//
// One 1024-thread workgroup per group of 4 replicas holds the spin tables in
// LDS (x at v, not-x at N + v, always-false 2N, always-true 2N + 1, as in the
// sweep) and proposes the clusters in order.  For cluster k the workgroup
// walks the clauses that hold a variable of k, each with the 4-bit mask of
// its literal positions inside k: a clause is violated before when none of
// its literals is true, after when none is true once the masked literals
// toggle.  The energy changes of the 4 replicas are exact integer sums; the
// decisions use one Philox call (counter (k, sweep, group, CFLIP)) and a host
// table of thresholds; the accepted replicas' bits of the cluster's
// variables then toggle in both spin tables.
#include "nmc_internal.h"
#include "nmc_philox.h"

namespace nmc {

namespace {

__device__ __forceinline__ int wsum(int v) {
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

__global__ void __launch_bounds__(1024) ksat_cflip_kernel(KsatDev I, KsatRepDev R, CflipCall C) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ int red[4];
    __shared__ uint32_t take_mask;
    const int n = I.n, g = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int r0 = g * kGroup;
    const int nact = min(kGroup, R.n_rep - r0);
    const uint32_t amask = (1u << nact) - 1u;
    uint8_t *xt = smem;
    uint8_t *xg = R.xs + (size_t)g * n;
    for (int v = tid; v < n; v += blockDim.x) {
        const uint32_t b = xg[v] & amask;
        xt[v] = (uint8_t)b;
        xt[n + v] = (uint8_t)(~b & amask);
    }
    if (tid == 0) {
        xt[2 * n] = 0;
        xt[2 * n + 1] = (uint8_t)amask;
    }
    if (tid < 4)
        red[tid] = 0;
    int E = 0, best = 0, fh = -1, acc = 0;
    if (tid < nact) {
        E = R.energy[r0 + tid];
        best = R.best[r0 + tid];
        fh = R.first_hit[r0 + tid];
    }
    __syncthreads();

    for (int k = 0; k < C.n_clusters; ++k) {
        int d0 = 0, d1 = 0, d2 = 0, d3 = 0;
        for (int e = C.cl_ptr[k] + tid; e < C.cl_ptr[k + 1]; e += blockDim.x) {
            const uint32_t w = C.cl_list[e];
            const uint32_t a = w & 0x0FFFFFFFu, mask = w >> 28;
            uint32_t before = 0, after = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t t = xt[I.clause_addr[(size_t)a * 4 + j]];
                before |= t;
                after |= ((mask >> j) & 1u) ? (t ^ amask) : t;
            }
            const uint32_t vb = ~before & amask, va = ~after & amask;
            d0 += (int)(va & 1u) - (int)(vb & 1u);
            d1 += (int)((va >> 1) & 1u) - (int)((vb >> 1) & 1u);
            d2 += (int)((va >> 2) & 1u) - (int)((vb >> 2) & 1u);
            d3 += (int)((va >> 3) & 1u) - (int)((vb >> 3) & 1u);
        }
        d0 = wsum(d0);
        d1 = wsum(d1);
        d2 = wsum(d2);
        d3 = wsum(d3);
        if (lane == 0) {
            if (d0) atomicAdd(&red[0], d0);
            if (d1) atomicAdd(&red[1], d1);
            if (d2) atomicAdd(&red[2], d2);
            if (d3) atomicAdd(&red[3], d3);
        }
        __syncthreads();
        if (tid == 0) {
            const uint4 u = philox4x32_10((uint32_t)k, C.t, (uint32_t)g, kStreamCflip, C.key0, C.key1);
            const uint32_t uw[4] = {u.x, u.y, u.z, u.w};
            uint32_t m = 0;
            for (int j = 0; j < nact; ++j) {
                const int d = red[j];
                bool take = d <= 0;
                if (!take)
                    take = uw[j] < (d <= C.thr_len ? C.thr[d] : 0u);
                m |= take ? (1u << j) : 0u;
            }
            take_mask = m;
        }
        __syncthreads();
        const uint32_t m = take_mask;
        if (tid < nact && ((m >> tid) & 1u)) {
            E += red[tid];
            ++acc;
        }
        if (m) {
            for (int q = C.v_ptr[k] + tid; q < C.v_ptr[k + 1]; q += blockDim.x) {
                const int v = C.v_list[q];
                xt[v] = (uint8_t)(xt[v] ^ m);
                xt[n + v] = (uint8_t)(xt[n + v] ^ m);
            }
        }
        __syncthreads();
        if (tid < 4)
            red[tid] = 0;
        __syncthreads();
    }

    // the move counts as one sweep: best, snapshot, first hit
    __shared__ uint32_t imp;
    if (tid == 0)
        imp = 0;
    __syncthreads();
    if (tid < nact) {
        if (E < best) {
            best = E;
            atomicOr(&imp, 1u << tid);
        }
        if (fh < 0 && E <= C.target)
            fh = (int)(C.t + 1);
    }
    __syncthreads();
    const uint32_t im = imp;
    if (im) {
        uint8_t *bg = R.best_xs + (size_t)g * n;
        for (int v = tid; v < n; v += blockDim.x)
            bg[v] = (uint8_t)((bg[v] & ~im) | (xt[v] & im));
    }
    for (int v = tid; v < n; v += blockDim.x)
        xg[v] = xt[v];
    if (tid < nact) {
        R.energy[r0 + tid] = E;
        R.best[r0 + tid] = best;
        R.first_hit[r0 + tid] = fh;
        C.accepted[r0 + tid] = acc;
    }
}

}  // namespace

size_t ksat_cflip_lds_bytes(int n) { return align_up((size_t)2 * n + 2, 16); }

hipError_t ksat_launch_cflip(const KsatDev &I, const KsatRepDev &R, const CflipCall &C, hipStream_t s) {
    if (R.n_groups <= 0)
        return hipSuccess;
    static const hipError_t attr = hipFuncSetAttribute((const void *)ksat_cflip_kernel,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)kLdsBytes - 64);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL(ksat_cflip_kernel, dim3(R.n_groups), dim3(1024), ksat_cflip_lds_bytes(I.n), s, I, R, C);
    return hipGetLastError();
}

}  // namespace nmc
