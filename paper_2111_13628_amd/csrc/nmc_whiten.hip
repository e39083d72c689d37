// Whitening of low-energy k-SAT states for gfx950 (section "Whitening
// procedure for low energy states").
//
// A variable turns white ("star") unless some clause has the variable's
// literal as its only true literal and no other white variable; a violated
// clause pins nothing.  White sets only grow and the pin condition only
// weakens as they grow, so every inspection order that repeats until
// nothing changes reaches the same (least) fixed point: the whitening of one
// group of 4 replicas runs inside one workgroup, in place, pass after pass,
// with no global synchronization.
//
// LDS: one 16-bit word per variable, low byte the 4 replicas' spins, high
// byte their white bits.  The clause structure is the sweep's: per variable
// (a lane of a 64-variable chunk), one 8-byte record per clause slot holding
// the spin-table addresses of the clause's other literals (x_v at v, its
// negation at N + v, always-false 2N, always-true 2N + 1) and whether the
// variable's own literal is negated.  Padding slots (always-true first
// address) never pin.
#include <climits>

#include "nmc_internal.h"

namespace nmc {

namespace {

// spins and white bits of the literal at spin-table address a:
// returns (truth bits) | (white bits << 8) of the other literal
__device__ __forceinline__ uint32_t lit_state(const uint16_t *tbl, uint32_t a, uint32_t n, uint32_t amask) {
    if (a < 2u * n) {
        const uint32_t neg = a >= n ? 1u : 0u;
        const uint32_t e = tbl[a - neg * n];
        return ((e & 0xFFu) ^ (neg ? amask : 0u)) | (e & 0xFF00u);
    }
    return a == 2u * n + 1u ? amask : 0u;
}

__global__ void __launch_bounds__(1024) ksat_whiten_kernel(KsatDev I, const uint8_t *xs, int n_rep, uint8_t *white_out,
                                                           int32_t *frozen_out, int32_t *passes_out) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ int changed;
    __shared__ int cnt[4];
    uint16_t *tbl = reinterpret_cast<uint16_t *>(smem);
    const int n = I.n, g = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, nwaves = blockDim.x >> 6, wave = tid >> 6;
    const int r0 = g * kGroup;
    const int nact = min(kGroup, n_rep - r0);
    const uint32_t amask = (1u << nact) - 1u;
    const uint8_t *xg = xs + (size_t)g * n;
    for (int v = tid; v < n; v += blockDim.x)
        tbl[v] = (uint16_t)(xg[v] & amask);
    if (tid < 4)
        cnt[tid] = 0;
    const uint64_t *rec = I.rec;
    int passes = 0;
    for (;;) {
        if (tid == 0)
            changed = 0;
        __syncthreads();
        for (int h = wave; h < I.n_chunks; h += nwaves) {
            const int lw = I.chunk_var[(size_t)h * kChunk + lane];
            const int2 info = I.chunk_info[h];
            const int nslot = info.y & ((1 << kSplitShift) - 1);
            const int lg = info.y >> kSplitShift;  // a variable's records spread over 2^lg lanes
            const int i = lw & 0xFFFFF;
            const uint32_t own = lw < 0 ? 0u : tbl[i];
            const uint32_t xi = own & 0xFFu, si = own >> 8;
            // the lanes of one variable agree on skipping it
            const bool live = lw >= 0 && si != amask;
            uint32_t pinned = 0;
            for (int s = 0; live && s < nslot; ++s) {
                const uint64_t r = rec[((size_t)(info.x / 2 + s / 2) * kChunk + lane) * 2 + (s & 1)];
                const uint32_t a0 = (uint32_t)r & kAddrMask;
                const uint32_t a1 = (uint32_t)(r >> kAddrBits) & kAddrMask;
                const uint32_t a2 = (uint32_t)(r >> (2 * kAddrBits)) & kAddrMask;
                const uint32_t neg = (uint32_t)(r >> (3 * kAddrBits)) & 1u;
                const uint32_t own_true = neg ? (~xi & amask) : xi;
                const uint32_t o = lit_state(tbl, a0, n, amask) | lit_state(tbl, a1, n, amask) |
                                   lit_state(tbl, a2, n, amask);
                pinned |= own_true & ~(o & 0xFFu) & ~(o >> 8);
            }
            for (int off = 1; off < (1 << lg); off <<= 1)
                pinned |= (uint32_t)__shfl_xor((int)pinned, off, 64);
            const uint32_t ns = si | (~pinned & amask);
            if (live && (lane & ((1 << lg) - 1)) == 0 && ns != si) {
                tbl[i] = (uint16_t)((ns << 8) | xi);
                changed = 1;
            }
        }
        __syncthreads();
        ++passes;
        const int c = changed;
        __syncthreads();
        if (!c)
            break;
    }
    // white bits out, frozen counts per replica
    int f0 = 0, f1 = 0, f2 = 0, f3 = 0;
    uint8_t *wg = white_out + (size_t)g * n;
    for (int v = tid; v < n; v += blockDim.x) {
        const uint32_t w = tbl[v] >> 8;
        wg[v] = (uint8_t)w;
        const uint32_t fz = ~w & amask;
        f0 += fz & 1u;
        f1 += (fz >> 1) & 1u;
        f2 += (fz >> 2) & 1u;
        f3 += (fz >> 3) & 1u;
    }
    for (int off = 32; off > 0; off >>= 1) {
        f0 += __shfl_xor(f0, off, 64);
        f1 += __shfl_xor(f1, off, 64);
        f2 += __shfl_xor(f2, off, 64);
        f3 += __shfl_xor(f3, off, 64);
    }
    if (lane == 0) {
        atomicAdd(&cnt[0], f0);
        atomicAdd(&cnt[1], f1);
        atomicAdd(&cnt[2], f2);
        atomicAdd(&cnt[3], f3);
    }
    __syncthreads();
    if (tid < nact)
        frozen_out[r0 + tid] = cnt[tid];
    if (tid == 0)
        atomicMax(passes_out, passes);
}

}  // namespace

size_t ksat_whiten_lds_bytes(int n) { return align_up((size_t)n * 2, 16); }

hipError_t ksat_launch_whiten(const KsatDev &I, const uint8_t *xs, int n_groups, int n_rep, uint8_t *white_out,
                              int32_t *frozen_out, int32_t *passes_out, hipStream_t s) {
    if (n_groups <= 0)
        return hipSuccess;
    const size_t lds = ksat_whiten_lds_bytes(I.n);
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)ksat_whiten_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes - 64);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL(ksat_whiten_kernel, dim3(n_groups), dim3(1024), lds, s, I, xs, n_rep, white_out, frozen_out,
                       passes_out);
    return hipGetLastError();
}

}  // namespace nmc
