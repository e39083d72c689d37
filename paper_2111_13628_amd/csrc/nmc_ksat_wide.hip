// k-SAT sweeps for instances whose spin tables do not fit in LDS (the wide
// layout), for gfx950.
//
// The same single-variable Metropolis sweep as the LDS kernels (section
// "Nonequilibrium inhomogeneous sampling over subgraphs"; CNF energy as in
// subsection "4-SAT Problems Near Computational Phase Transitions"): the
// colour-major order, the closed form of dE from the OR of each clause's
// other literals, one generator call per (variable, group of 4 replicas) and
// the same threshold tables, so the results are bit-identical.  What changes
// is the mapping: the spins of a launch live in device memory, variable-major
// ([row][group], one byte per group of 4 replicas; rows 0..N hold x, rows
// N+1..2N+1 hold NOT x, row N is the absent literal), and a wave takes one
// variable for 64 groups, one lane per group.  A variable's clause records
// are then the same for the whole wave (scalar loads), and every literal read
// is one coalesced 64-byte row segment serving 256 replicas, a buffer load
// whose row offset is a scalar shift.  No two variables of a colour class share a
// clause, so one launch per class updates the class's variables
// concurrently; the launches of a sweep run in order on the stream.
#include <climits>

#include "nmc_internal.h"
#include "nmc_philox.h"

namespace nmc {

namespace {

__device__ __forceinline__ uint32_t wide_spread4(uint32_t f) { return (f * 0x00204081u) & 0x01010101u; }

// The GPL bytes of groups g .. g + GPL - 1 (GPL = 1 or 4; g a multiple of
// GPL) in table row `row`, byte k = group g + k.
template <int GPL>
__device__ __forceinline__ uint32_t row_groups(__amdgpu_buffer_rsrc_t tab, uint32_t row, int lg, int g) {
    if constexpr (GPL == 1)
        return __builtin_amdgcn_raw_buffer_load_b8(tab, g, (int)(row << lg), 0);
    else
        return __builtin_amdgcn_raw_buffer_load_b32(tab, g, (int)(row << lg), 0);
}

typedef const uint32_t __attribute__((address_space(4))) c_u32;

// Clause slots q .. q + K - 1 of a variable (those at or past q1 are
// skipped: their record reads stay on the last slot and add nothing) for the
// lane's GPL groups.  All K records are read first (scalar loads), then all
// 3K rows, then summed: acc[k] collects, for group g + k, spread(sat) xor
// (own literal negated ? all ones : 0), sat = OR of the clause's other
// literals (4 replica bits).
template <int K, int GPL>
__device__ __forceinline__ void wide_slots(const c_u32 *rw, __amdgpu_buffer_rsrc_t tab, int lg, int g, int q, int q1,
                                           uint32_t (&acc)[GPL], uint32_t &nneg) {
    uint4 r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int qk = min(q + k, q1 - 1);
        r[k] = make_uint4(rw[4 * qk], rw[4 * qk + 1], rw[4 * qk + 2], rw[4 * qk + 3]);
    }
    uint32_t b[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        b[k] = row_groups<GPL>(tab, r[k].x, lg, g) | row_groups<GPL>(tab, r[k].y, lg, g) |
               row_groups<GPL>(tab, r[k].z, lg, g);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (q + k < q1) {
            nneg += r[k].w;
#pragma unroll
            for (int j = 0; j < GPL; ++j)
                acc[j] = (wide_spread4((b[k] >> (8 * j)) & 0xFFu) ^ (0u - r[k].w)) + acc[j];
        }
    }
}

__device__ __forceinline__ uint32_t group_mask(const KsatRepDev &R, int g) {
    const int nact = g < R.n_groups ? min(kGroup, R.n_rep - g * kGroup) : 0;
    return (1u << nact) - 1u;
}

// [G][N] group-major spins (and best states) <-> [N + 1][wgp] variable-major,
// through 64 x 64 tiles in LDS so both sides move in rows.  Packing also
// writes the complement rows and the all-zero row N (the absent literal).
__global__ void __launch_bounds__(256) ksat_wide_pack_kernel(KsatDev I, KsatRepDev R, int unpack) {
    __shared__ uint8_t tx[64][65], tb[64][65];
    const int n = I.n, gp = R.wgp;
    const int v0 = blockIdx.x * 64, g0 = blockIdx.y * 64;
    if (!unpack) {
        for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
            const int gl = i >> 6, vl = i & 63;
            const int g = g0 + gl, v = v0 + vl;
            const bool in = g < R.n_groups && v < n;
            tx[gl][vl] = in ? R.xs[(size_t)g * n + v] : 0;
            tb[gl][vl] = in ? R.best_xs[(size_t)g * n + v] : 0;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
            const int vl = i >> 6, gl = i & 63;
            const int v = v0 + vl, g = g0 + gl;
            if (v > n)
                continue;
            const size_t o = (size_t)v * gp + g;
            if (v == n) {
                R.wx[o] = 0;
                R.wnx[o] = 0;
                continue;
            }
            const uint32_t am = group_mask(R, g);
            const uint32_t x = tx[gl][vl] & am;
            R.wx[o] = (uint8_t)x;
            R.wnx[o] = (uint8_t)(~x & am);
            R.wbx[o] = tb[gl][vl];
        }
    } else {
        for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
            const int vl = i >> 6, gl = i & 63;
            const int v = v0 + vl, g = g0 + gl;
            const bool in = v < n;
            tx[gl][vl] = in ? R.wx[(size_t)v * gp + g] : 0;
            tb[gl][vl] = in ? R.wbx[(size_t)v * gp + g] : 0;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
            const int gl = i >> 6, vl = i & 63;
            const int g = g0 + gl, v = v0 + vl;
            if (g < R.n_groups && v < n) {
                R.xs[(size_t)g * n + v] = tx[gl][vl];
                R.best_xs[(size_t)g * n + v] = tb[gl][vl];
            }
        }
    }
}

// Before the first sweep: a replica already at or below the target counts as
// hit at the call's first sweep index (as in the LDS kernels).
__global__ void ksat_wide_start_kernel(KsatRepDev R, SweepCall C) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R.n_rep && C.check_start && R.first_hit[r] < 0 && R.energy[r] <= C.target)
        R.first_hit[r] = (int)C.t0;
}

// One colour class c of sweep s.  Workgroup (slice, group block): waves take
// the class's variables i = stream, stream + kWideStreams, ...; a lane takes
// GPL adjacent groups (GPL = 4: one 4-byte row read serves 16 replicas, a
// quarter of the load instructions of one group per lane).
template <int GPL>
__global__ void __launch_bounds__(64 * kWideWaves) ksat_wide_class_kernel(KsatDev I, KsatRepDev R, SweepCall C,
                                                                          int c, int s) {
    extern __shared__ __align__(16) uint32_t tl[];  // the sweep's threshold rows
    const int tab_words = C.n_classes * C.stride;
    const uint32_t *tg = C.tab + (size_t)s * C.sweep_words;
    for (int i = threadIdx.x; i < tab_words; i += blockDim.x)
        tl[i] = tg[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = (blockIdx.y * 64 + lane) * GPL;  // the lane's first group
    const int gp = R.wgp;
    uint32_t amask[GPL];
#pragma unroll
    for (int k = 0; k < GPL; ++k)
        amask[k] = group_mask(R, g + k);
    const int stream = blockIdx.x * kWideWaves + wave;
    const int lg = R.wlg;
    // the spin and complement rows, [2 (N + 1)][wgp] bytes from wx
    const __amdgpu_buffer_rsrc_t tab = __builtin_amdgcn_make_buffer_rsrc(
        R.wx, 0, (int)(((size_t)2 * (I.n + 1)) << lg), kBufferWord3);
    // the records, read-only here: through the constant address space they
    // are scalar loads
    const c_u32 *rec = (const c_u32 *)I.wrec;
    const int c0 = I.wclass_ptr[c], c1 = I.wclass_ptr[c + 1];
    const uint32_t t = C.t0 + (uint32_t)s;
    int dsum[GPL][kGroup];
#pragma unroll
    for (int k = 0; k < GPL; ++k)
        dsum[k][0] = dsum[k][1] = dsum[k][2] = dsum[k][3] = 0;
    uint32_t n_acc = 0;
    for (int i = c0 + stream; i < c1; i += kWideStreams) {
        const int v = __builtin_amdgcn_readfirstlane(I.worder[i]);
        const int q0 = __builtin_amdgcn_readfirstlane(I.var_ptr[v]);
        const int q1 = __builtin_amdgcn_readfirstlane(I.var_ptr[v + 1]);
        const uint32_t xw = row_groups<GPL>(tab, (uint32_t)v, lg, g);
        // records 8 at a time (their 24 rows read together), then groups of 4
        uint32_t acc[GPL], nneg = 0;
#pragma unroll
        for (int k = 0; k < GPL; ++k)
            acc[k] = 0;
        int q = q0;
        for (; q + kWideGroup <= q1; q += kWideGroup)
            wide_slots<kWideGroup, GPL>(rec, tab, lg, g, q, q1, acc, nneg);
        for (; q < q1; q += 4)
            wide_slots<4, GPL>(rec, tab, lg, g, q, q1, acc, nneg);
        const uint32_t nslot = (uint32_t)(q1 - q0);
        const int cl = C.var_cls ? (int)C.var_cls[v] : 0;
        const uint32_t *T = tl + cl * C.stride;
        uint32_t nxw = xw;
#pragma unroll
        for (int k = 0; k < GPL; ++k) {
            // byte j of 0x80808080 + part = 128 + (clauses of this variable
            // whose other literals are all false, +1 where the variable's
            // own literal is positive, -1 where negated), for replica j of
            // group g + k
            const uint32_t a = 0x80808080u + ((nslot - 2u * nneg) * 0x01010101u - nneg - acc[k]);
            const uint32_t xi = (xw >> (8 * k)) & 0xFFu;
            int de[kGroup];
            uint32_t thr[kGroup];
            uint32_t flip = 0, need = 0;
#pragma unroll
            for (int j = 0; j < kGroup; ++j) {
                const int S = (int)((a >> (8 * j)) & 0xFFu) - 128;
                de[j] = ((xi >> j) & 1u) ? S : -S;
                thr[j] = T[max(de[j], 0)];
                const uint32_t on = (amask[k] >> j) & 1u;
                flip |= (on & (uint32_t)(de[j] <= 0)) << j;
                need |= (on & (uint32_t)(de[j] > 0) & (uint32_t)(thr[j] != 0)) << j;
            }
            if (need) {
                const uint4 u = philox4x32_10((uint32_t)v, t, (uint32_t)(g + k), kStreamKsatSweep, C.key0, C.key1);
                flip |= ((need & 1u) && u.x < thr[0]) ? 1u : 0u;
                flip |= ((need & 2u) && u.y < thr[1]) ? 2u : 0u;
                flip |= ((need & 4u) && u.z < thr[2]) ? 4u : 0u;
                flip |= ((need & 8u) && u.w < thr[3]) ? 8u : 0u;
            }
            n_acc += __builtin_popcount(flip);
            nxw ^= flip << (8 * k);
#pragma unroll
            for (int j = 0; j < kGroup; ++j)
                dsum[k][j] += ((flip >> j) & 1u) ? de[j] : 0;
        }
        if (nxw != xw) {
            uint32_t nnx = 0;
#pragma unroll
            for (int k = 0; k < GPL; ++k)
                nnx |= (~(nxw >> (8 * k)) & amask[k]) << (8 * k);
            const size_t own = (size_t)v * gp + g;
            if constexpr (GPL == 1) {
                R.wx[own] = (uint8_t)nxw;
                R.wnx[own] = (uint8_t)nnx;
            } else {
                *reinterpret_cast<uint32_t *>(R.wx + own) = nxw;
                *reinterpret_cast<uint32_t *>(R.wnx + own) = nnx;
            }
        }
    }
    // this stream's slots for the lane's groups: only this lane of this wave
    // touches them during a sweep, and the class launches run in order
#pragma unroll
    for (int k = 0; k < GPL; ++k) {
        if (dsum[k][0] | dsum[k][1] | dsum[k][2] | dsum[k][3]) {
            int4 *slot = reinterpret_cast<int4 *>(R.wdsum) + (size_t)(g + k) * kWideStreams + stream;
            int4 d = *slot;
            d.x += dsum[k][0];
            d.y += dsum[k][1];
            d.z += dsum[k][2];
            d.w += dsum[k][3];
            *slot = d;
        }
    }
    unsigned long long acc_w = n_acc;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        acc_w += __shfl_xor(acc_w, off, 64);
    if (lane == 0 && acc_w)
        atomicAdd(R.accepted, acc_w);
}

// Sweep end for group g (one workgroup): the streams' energy changes (then
// cleared), energies, best energies, first hits, and the mask of replicas
// whose best improved (their best state is copied by the snapshot kernel).
__global__ void __launch_bounds__(256) ksat_wide_sweep_end_kernel(KsatRepDev R, SweepCall C, uint32_t t) {
    __shared__ int red[kGroup][256 / 64];
    const int g = blockIdx.x;
    int d[kGroup] = {0, 0, 0, 0};
    for (int st = threadIdx.x; st < kWideStreams; st += blockDim.x) {
        int4 *slot = reinterpret_cast<int4 *>(R.wdsum) + (size_t)g * kWideStreams + st;
        const int4 v = *slot;
        if (v.x | v.y | v.z | v.w) {
            d[0] += v.x;
            d[1] += v.y;
            d[2] += v.z;
            d[3] += v.w;
            *slot = make_int4(0, 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < kGroup; ++j) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            d[j] += __shfl_xor(d[j], off, 64);
        if ((threadIdx.x & 63) == 0)
            red[j][threadIdx.x >> 6] = d[j];
    }
    __syncthreads();
    if (threadIdx.x < kGroup) {
        const int j = threadIdx.x, r = g * kGroup + j;
        bool imp = false;
        if (r < R.n_rep) {
            int sum = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
                sum += red[j][w];
            const int E = R.energy[r] + sum;
            R.energy[r] = E;
            if (E < R.best[r]) {
                R.best[r] = E;
                imp = true;
            }
            if (R.first_hit[r] < 0 && E <= C.target)
                R.first_hit[r] = (int)(t + 1);
        }
        // lanes 0..3 of wave 0: gather the 4 bits
        const uint64_t m = __ballot(imp);
        if (j == 0)
            R.wflag[g] = (uint8_t)(m & 0xFu);
    }
}

// Best-state snapshot after a sweep: replicas flagged by the sweep end copy
// their current spins, 16 groups per lane (rows are a multiple of 64 groups,
// so a 16-byte piece never crosses a row).
__global__ void ksat_wide_snapshot_kernel(KsatDev I, KsatRepDev R) {
    const size_t total = ((size_t)I.n * R.wgp) >> 4;
    const uint32_t row16 = (uint32_t)R.wgp >> 4;
    const uint4 *flag = reinterpret_cast<const uint4 *>(R.wflag);
    const uint4 *x = reinterpret_cast<const uint4 *>(R.wx);
    uint4 *best = reinterpret_cast<uint4 *>(R.wbx);
    for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < total; o += (size_t)gridDim.x * blockDim.x) {
        const uint4 m = flag[o & (row16 - 1)];
        if (m.x | m.y | m.z | m.w) {
            const uint4 b = best[o], c = x[o];
            best[o] = make_uint4((b.x & ~m.x) | (c.x & m.x), (b.y & ~m.y) | (c.y & m.y), (b.z & ~m.z) | (c.z & m.z),
                                 (b.w & ~m.w) | (c.w & m.w));
        }
    }
}

__global__ void ksat_wide_zero_kernel(int32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0;
}

// Energies of every replica from the variable-major tables (freshly packed
// from the group-major state): a wave takes a run of kRecountRun clauses for
// 64 groups, one lane per group, reads each clause's four addresses once
// (scalar loads) and the four literal rows (one coalesced row segment each),
// and counts the clauses with no true literal per replica.  The workgroup's
// four waves meet in LDS; workgroups add their counts with integer atomics,
// so the sums are exact in any order.
constexpr int kRecountRun = 1024;

__global__ void __launch_bounds__(256) ksat_wide_recount_kernel(KsatDev I, KsatRepDev R, int32_t *energy_out) {
    __shared__ uint32_t red[256 / 64][64][kGroup];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = blockIdx.y * 64 + lane;
    const int n = I.n, lg = R.wlg;
    const __amdgpu_buffer_rsrc_t tab = __builtin_amdgcn_make_buffer_rsrc(
        R.wx, 0, (int)(((size_t)2 * (n + 1)) << lg), kBufferWord3);
    const c_u32 *ca = (const c_u32 *)I.clause_addr;
    const int a0 = (blockIdx.x * 4 + wave) * kRecountRun, a1 = min(a0 + kRecountRun, I.m);
    // table row of a clause address: x_v at v, NOT x_v at N + 1 + v, the
    // absent literal at the all-zero row N
    auto row = [&](uint32_t ad) -> uint32_t {
        return ad < (uint32_t)n ? ad : ad < 2u * (uint32_t)n ? ad + 1u : (uint32_t)n;
    };
    uint32_t c[kGroup] = {0, 0, 0, 0};
    for (int a = a0; a < a1; a += 4) {
        uint32_t b[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int ak = min(a + k, a1 - 1);
            const uint32_t r0 = row(ca[4 * ak]), r1 = row(ca[4 * ak + 1]), r2 = row(ca[4 * ak + 2]),
                           r3 = row(ca[4 * ak + 3]);
            b[k] = __builtin_amdgcn_raw_buffer_load_b8(tab, g, (int)(r0 << lg), 0) |
                   __builtin_amdgcn_raw_buffer_load_b8(tab, g, (int)(r1 << lg), 0) |
                   __builtin_amdgcn_raw_buffer_load_b8(tab, g, (int)(r2 << lg), 0) |
                   __builtin_amdgcn_raw_buffer_load_b8(tab, g, (int)(r3 << lg), 0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (a + k < a1) {
#pragma unroll
                for (int j = 0; j < kGroup; ++j)
                    c[j] += ((b[k] >> j) & 1u) ^ 1u;
            }
    }
#pragma unroll
    for (int j = 0; j < kGroup; ++j)
        red[wave][lane][j] = c[j];
    __syncthreads();
    if (wave == 0 && g < R.n_groups) {
#pragma unroll
        for (int j = 0; j < kGroup; ++j) {
            const uint32_t sum = red[0][lane][j] + red[1][lane][j] + red[2][lane][j] + red[3][lane][j];
            const int r = g * kGroup + j;
            if (r < R.n_rep && sum)
                atomicAdd(&energy_out[r], (int32_t)sum);
        }
    }
}

}  // namespace

hipError_t ksat_launch_wide_pack(const KsatDev &I, const KsatRepDev &R, bool unpack, hipStream_t s) {
    // packing also covers row n (the absent literal)
    const int nv = I.n + (unpack ? 0 : 1);
    hipLaunchKernelGGL(ksat_wide_pack_kernel, dim3((nv + 63) / 64, R.wgp / 64), dim3(256), 0, s, I, R,
                       unpack ? 1 : 0);
    return hipGetLastError();
}

hipError_t ksat_launch_wide_recount(const KsatDev &I, const KsatRepDev &R, int32_t *energy_out, hipStream_t s) {
    const hipError_t e = ksat_launch_wide_pack(I, R, false, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(ksat_wide_zero_kernel, dim3((R.n_rep + 255) / 256), dim3(256), 0, s, energy_out, R.n_rep);
    const int runs = (I.m + kRecountRun - 1) / kRecountRun;
    if (runs > 0)
        hipLaunchKernelGGL(ksat_wide_recount_kernel, dim3((runs + 3) / 4, R.wgp / 64), dim3(256), 0, s, I, R,
                           energy_out);
    return hipGetLastError();
}

hipError_t ksat_launch_wide_sweeps(const KsatDev &I, const KsatRepDev &R, const SweepCall &C,
                                   const int32_t *class_size, hipStream_t s) {
    const size_t lds = (size_t)C.n_classes * C.stride * sizeof(uint32_t);
    // four groups per lane once a row holds at least 256 of them
    const bool quad = R.wgp >= 256;
    static const hipError_t attr1 = hipFuncSetAttribute((const void *)ksat_wide_class_kernel<1>,
                                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
    static const hipError_t attr4 = hipFuncSetAttribute((const void *)ksat_wide_class_kernel<4>,
                                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
    if (attr1 != hipSuccess || attr4 != hipSuccess)
        return attr1 != hipSuccess ? attr1 : attr4;
    hipLaunchKernelGGL(ksat_wide_start_kernel, dim3((R.n_rep + 255) / 256), dim3(256), 0, s, R, C);
    const size_t pieces = ((size_t)I.n * R.wgp) >> 4;
    const int snap_blocks = (int)std::min<size_t>((pieces + 255) / 256, 4096);
    for (int sw = 0; sw < C.n_sweeps; ++sw) {
        for (int c = 0; c < I.n_colors; ++c) {
            // no more workgroups than the class has variables for
            const int cs = class_size[c];
            const int slices = std::max(1, std::min(kWideSlices, (cs + kWideWaves - 1) / kWideWaves));
            if (quad)
                hipLaunchKernelGGL(ksat_wide_class_kernel<4>, dim3(slices, R.wgp / 256), dim3(64 * kWideWaves), lds, s,
                                   I, R, C, c, sw);
            else
                hipLaunchKernelGGL(ksat_wide_class_kernel<1>, dim3(slices, R.wgp / 64), dim3(64 * kWideWaves), lds, s,
                                   I, R, C, c, sw);
        }
        hipLaunchKernelGGL(ksat_wide_sweep_end_kernel, dim3(R.n_groups), dim3(256), 0, s, R, C, C.t0 + (uint32_t)sw);
        hipLaunchKernelGGL(ksat_wide_snapshot_kernel, dim3(snap_blocks), dim3(256), 0, s, I, R);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

}  // namespace nmc
