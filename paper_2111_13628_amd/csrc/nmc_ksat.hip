// k-SAT kernels for gfx950.
//
// Work decomposition.  One workgroup owns one group of 4 replicas for the
// whole launch.  Their spins live in LDS as a byte per variable (bit j =
// replica j of the group), next to the complement table, so "literal is
// true" is a single byte load whatever the literal's sign:
//   lds[v]       = x_v        (positive literal of v)
//   lds[N + v]   = NOT x_v    (negative literal of v)
//   lds[2N]      = 0          (absent literal: never true)
//   lds[2N + 1]  = all ones   (padding slot: clause counts as satisfied)
// The energy change of flipping x_i (section "Nonequilibrium inhomogeneous
// sampling over subgraphs" uses single-variable Metropolis moves; CNF energy
// as in subsection "4-SAT Problems Near Computational Phase Transitions") is
//   dE = sum over clauses a of i with every other literal false of
//        (+1 if i's literal in a is currently true, -1 otherwise),
// computed for the 4 replicas at once: the OR of the other literals' bytes
// is a 4-bit "satisfied by others" mask, spread into four byte lanes of a
// 32-bit accumulator (SIMD within a register).
// A wave handles 64 variables of one colour class (one lane per variable);
// classes are conflict-free, so all lanes update concurrently and the result
// equals the sequential colour-major order.  The instance (per-variable
// clause records) streams from L2/MALL, shared by every workgroup.
#include <climits>
#include <cstdlib>

#include "nmc_internal.h"
#include "nmc_philox.h"

namespace nmc {

namespace {

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over each group of 2^lg lanes (lg wave-uniform, at most 6), returned to
// every lane of the group: swaps within quads, the mirrors within half-rows
// and rows (register moves, no LDS crossbar), then shuffles across rows.
// Sums mod 2^32, so the order does not matter.
__device__ __forceinline__ uint32_t lane_group_sum(uint32_t x, int lg) {
    if (lg >= 1)
        x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    if (lg >= 2)
        x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    if (lg >= 3)
        x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    if (lg >= 4)
        x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false);  // row_mirror
    if (lg >= 5)
        x += (uint32_t)__shfl_xor((int)x, 16, 64);
    if (lg >= 6)
        x += (uint32_t)__shfl_xor((int)x, 32, 64);
    return x;
}

__device__ __forceinline__ uint32_t spread4(uint32_t f) {
    // bit j of f (j < 4) -> bit 8j; no carries for f < 16
    return (f * 0x00204081u) & 0x01010101u;
}

// Compiler-only barrier: memory operations are not moved across it, so
// prefetch loads stay where they are issued and their waits stay at first use.
__device__ __forceinline__ void issue_fence() { __asm__ volatile("" ::: "memory"); }

typedef __attribute__((address_space(3))) const uint8_t lds_cu8;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

// Byte at LDS address a.  The sweep kernel declares no static LDS, so its
// dynamic LDS block starts at address 0 and spin-table offsets are addresses.
__device__ __forceinline__ uint32_t lds_load_u8(uint32_t a) { return *(lds_cu8 *)(uintptr_t)a; }
__device__ __forceinline__ void lds_store_u8(uint32_t a, uint32_t v) { *(lds_u8 *)(uintptr_t)a = (uint8_t)v; }

// One clause slot: r.x bits 0..16 and r.y bits 0..1 / 2..18 hold the spin-table
// addresses of the clause's three other literals, r.y bit 19 whether the
// lane's own literal in the clause is negated.  Adds spread(sat) xor sign.
__device__ __forceinline__ uint32_t slot_step(uint32_t acc, uint2 r) {
    const uint32_t a0 = r.x & kAddrMask;
    const uint32_t a1 = __builtin_amdgcn_alignbit(r.y, r.x, kAddrBits) & kAddrMask;
    const uint32_t a2 = __builtin_amdgcn_ubfe(r.y, 2 * kAddrBits - 32, kAddrBits);
    const uint32_t sm = (uint32_t)__builtin_amdgcn_sbfe(r.y, 3 * kAddrBits - 32, 1);
    const uint32_t sat = lds_load_u8(a0) | lds_load_u8(a1) | lds_load_u8(a2);
    return (spread4(sat) ^ sm) + acc;
}

__global__ void ksat_init_kernel(KsatDev I, KsatRepDev R, uint32_t key0, uint32_t key1) {
    const size_t total = (size_t)R.n_groups * I.n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int g = (int)(idx / I.n);
        const int v = (int)(idx % I.n);
        const int nact = min(kGroup, R.n_rep - g * kGroup);
        const uint4 u = philox4x32_10((uint32_t)v, 0u, (uint32_t)g, kStreamKsatInit, key0, key1);
        uint32_t b = (u.x >> 31) | ((u.y >> 31) << 1) | ((u.z >> 31) << 2) | ((u.w >> 31) << 3);
        b &= (1u << nact) - 1u;
        R.xs[idx] = (uint8_t)b;
        R.best_xs[idx] = (uint8_t)b;
    }
}

// Full energy count of every replica of one group (one workgroup per group).
__global__ void ksat_recount_kernel(KsatDev I, const uint8_t *xs, int n_rep, int32_t *energy_out) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int n = I.n, g = blockIdx.x, tid = threadIdx.x;
    const int nact = min(kGroup, n_rep - g * kGroup);
    const uint32_t amask = (1u << nact) - 1u;
    uint8_t *xt = smem;
    int *red = (int *)(smem + align_up(2 * n + 2, 16));
    for (int v = tid; v < n; v += blockDim.x) {
        const uint32_t b = xs[(size_t)g * n + v] & amask;
        xt[v] = (uint8_t)b;
        xt[n + v] = (uint8_t)(~b & amask);
    }
    if (tid == 0) {
        xt[2 * n] = 0;
        xt[2 * n + 1] = (uint8_t)amask;
    }
    if (tid < kGroup)
        red[tid] = 0;
    __syncthreads();
    int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    for (int a = tid; a < I.m; a += blockDim.x) {
        const uint4 ad = reinterpret_cast<const uint4 *>(I.clause_addr)[a];
        const uint32_t sat = xt[ad.x] | xt[ad.y] | xt[ad.z] | xt[ad.w];
        const uint32_t f = ~sat & amask;
        c0 += f & 1;
        c1 += (f >> 1) & 1;
        c2 += (f >> 2) & 1;
        c3 += (f >> 3) & 1;
    }
    c0 = wave_sum(c0);
    c1 = wave_sum(c1);
    c2 = wave_sum(c2);
    c3 = wave_sum(c3);
    if ((tid & 63) == 0) {
        atomicAdd(&red[0], c0);
        atomicAdd(&red[1], c1);
        atomicAdd(&red[2], c2);
        atomicAdd(&red[3], c3);
    }
    __syncthreads();
    if (tid < nact)
        energy_out[g * kGroup + tid] = red[tid];
}

__global__ void ksat_reset_tallies_kernel(KsatRepDev R) {
    const int total = R.n_groups * kGroup;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < total; r += gridDim.x * blockDim.x) {
        R.best[r] = R.energy[r];
        R.first_hit[r] = -1;
    }
}

// One clause slot for the 8 replicas of two groups (spin bytes holding the
// first group in bits 0..3, the second in bits 4..7): the same record and
// gathers feed both accumulators.
__device__ __forceinline__ void slot_step2(uint32_t &a0, uint32_t &a1, uint2 r) {
    const uint32_t ad0 = r.x & kAddrMask;
    const uint32_t ad1 = __builtin_amdgcn_alignbit(r.y, r.x, kAddrBits) & kAddrMask;
    const uint32_t ad2 = __builtin_amdgcn_ubfe(r.y, 2 * kAddrBits - 32, kAddrBits);
    const uint32_t sm = (uint32_t)__builtin_amdgcn_sbfe(r.y, 3 * kAddrBits - 32, 1);
    const uint32_t sat = lds_load_u8(ad0) | lds_load_u8(ad1) | lds_load_u8(ad2);
    a0 = (spread4(sat & 0xFu) ^ sm) + a0;
    a1 = (spread4(sat >> 4) ^ sm) + a1;
}

// n_sweeps full sweeps of every colour class for the replicas of item g, by
// the whole workgroup, with smem = the workgroup's dynamic LDS block.
// GPW = 1: the 4 replicas of group g.  GPW = 2: the 8 replicas of groups 2g
// and 2g + 1, held in one spin byte per variable (first group in bits 0..3),
// so every clause record, address decode and LDS gather serves 8 replicas;
// the random words and every result are those of the groups run one by one.
// STAGED: the instance's records and chunk tables are copied into LDS at the
// start (instances small enough for them to fit beside the spin tables), so
// a colour class's loads are LDS reads instead of L2 round trips.
template <int GPW, bool STAGED = false>
__device__ __forceinline__ void sweep_group(const KsatDev &I, const KsatRepDev &R, const SweepCall &C, const int g,
                                            uint8_t *smem) {
    constexpr int NR = kGroup * GPW;  // replicas of the item
    const int n = I.n;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, nwaves = nthr >> 6;
    const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tab_words = C.n_classes * C.stride;

    uint8_t *xt = smem;
    uint32_t *tl = (uint32_t *)(smem + align_up(2 * n + 2, 16));
    int *red = (int *)(tl + align_up(tab_words, 4));  // [0..NR) dE sums, [NR] improved mask

    const int g0 = g * GPW;  // first group of the item
    const int r0 = g0 * kGroup;
    const int nact = min(NR, R.n_rep - r0);
    const uint32_t amask = (1u << nact) - 1u;
    const bool second = GPW == 2 && g0 + 1 < R.n_groups;  // the item's second group exists
    // per-temperature tables (tempering): the item's replicas share one row
    const uint32_t *tab = C.tab + (C.reps_per_row > 0 ? (size_t)(r0 / C.reps_per_row) * tab_words : 0);

    // spin tables x and not-x from the group rows; rows and tables are
    // 16-byte aligned when N is a multiple of 16, then moved 16 bytes a lane
    uint8_t *xg = R.xs + (size_t)g0 * n;
    const bool wide = (n & 15) == 0;
    if (wide) {
        const uint32_t m4 = amask * 0x01010101u;
        for (int w = tid; w < n / 16; w += nthr) {
            uint4 b = reinterpret_cast<const uint4 *>(xg)[w];
            if (GPW == 2 && second) {
                // the second group's nibbles (values below 16) move to bits 4..7 of each byte
                const uint4 h = reinterpret_cast<const uint4 *>(xg + n)[w];
                b.x |= h.x << 4;
                b.y |= h.y << 4;
                b.z |= h.z << 4;
                b.w |= h.w << 4;
            }
            b.x &= m4;
            b.y &= m4;
            b.z &= m4;
            b.w &= m4;
            reinterpret_cast<uint4 *>(xt)[w] = b;
            reinterpret_cast<uint4 *>(xt + n)[w] = make_uint4(~b.x & m4, ~b.y & m4, ~b.z & m4, ~b.w & m4);
        }
    } else {
        for (int v = tid; v < n; v += nthr) {
            uint32_t b = xg[v];
            if (GPW == 2 && second)
                b |= (uint32_t)xg[n + v] << 4;
            b &= amask;
            xt[v] = (uint8_t)b;
            xt[n + v] = (uint8_t)(~b & amask);
        }
    }
    if (tid == 0) {
        xt[2 * n] = 0;
        xt[2 * n + 1] = (uint8_t)amask;
    }
    if (tid < 16)
        red[tid] = 0;
    // staged instance: records, chunk descriptors, lane words, class ranges
    uint4 *s_rec = nullptr, *s_u = nullptr;
    int2 *s_info = nullptr;
    int *s_var = nullptr, *s_cc = nullptr;
    if constexpr (STAGED) {
        uint8_t *st = (uint8_t *)(red + 16);
        s_rec = (uint4 *)st;
        s_info = (int2 *)(st + align_up(I.rec_bytes, 16));
        s_var = (int *)((uint8_t *)s_info + align_up((size_t)I.n_chunks * 8, 16));
        s_cc = s_var + (size_t)I.n_chunks * kChunk;
        // each variable's random words of the current sweep
        s_u = (uint4 *)((uint8_t *)s_cc + align_up(((size_t)I.n_colors + 1) * 4, 16));
        for (int w = tid; w < (int)(I.rec_bytes / 16); w += nthr)
            s_rec[w] = reinterpret_cast<const uint4 *>(I.rec)[w];
        for (int w = tid; w < I.n_chunks; w += nthr)
            s_info[w] = I.chunk_info[w];
        for (int w = tid; w < I.n_chunks * kChunk / 4; w += nthr)
            reinterpret_cast<int4 *>(s_var)[w] = reinterpret_cast<const int4 *>(I.chunk_var)[w];
        for (int w = tid; w <= I.n_colors; w += nthr)
            s_cc[w] = I.color_chunk[w];
    }
    int E = 0, best = 0, fh = -1;
    if (tid < nact) {
        E = R.energy[r0 + tid];
        best = R.best[r0 + tid];
        fh = R.first_hit[r0 + tid];
        if (C.check_start && fh < 0 && E <= C.target)
            fh = (int)C.t0;
    }
    __syncthreads();

    uint32_t n_acc = 0;  // flips this lane accepted in this call
    // the instance's records (out-of-range offsets would read zeros)
    const __amdgpu_buffer_rsrc_t recs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint64_t *>(I.rec), 0, (int)I.rec_bytes, kBufferWord3);
    for (int s = 0; s < C.n_sweeps; ++s) {
        const uint32_t t = C.t0 + (uint32_t)s;
        const uint32_t *tg = tab + (size_t)s * C.sweep_words;
        for (int i = tid; i < tab_words; i += nthr)
            tl[i] = tg[i];
        if constexpr (STAGED) {
            // a staged (small, latency-bound) instance draws the sweep's
            // random words of every variable at once, spread over the whole
            // workgroup, instead of one dependent generator chain per colour
            // class (the words depend only on the variable, the sweep and the
            // group, so drawing them for every variable changes nothing)
            for (int w = tid; w < n; w += nthr)
                s_u[w] = philox4x32_10((uint32_t)w, t, (uint32_t)g0, kStreamKsatSweep, C.key0, C.key1);
        }
        __syncthreads();

        int dsum[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j)
            dsum[j] = 0;
        for (int c = 0; c < I.n_colors; ++c) {
            const int h0 = STAGED ? s_cc[c] : I.color_chunk[c], h1 = STAGED ? s_cc[c + 1] : I.color_chunk[c + 1];
            // chunks of a class are sorted by slot count (descending); rounds
            // alternate direction so heavy and light chunks pair up per wave
            const int nch = h1 - h0;
            for (int rnd = 0; rnd * nwaves < nch; ++rnd) {
                const int idx = rnd * nwaves + ((rnd & 1) ? nwaves - 1 - wave_u : wave_u);
                if (idx >= nch)
                    continue;
                const int h = h0 + idx;
                // after the class barrier every wave would start its gathers
                // at once; delaying waves by (index mod 4) x 128 cycles spreads
                // the workgroup's gathers on the shared LDS over time (measured
                // 2 % faster on N = 50,000, 1024 replicas)
                if (wave_u & 2)
                    __builtin_amdgcn_s_sleep(4);
                if (wave_u & 1)
                    __builtin_amdgcn_s_sleep(2);
                const int2 info = STAGED ? s_info[h] : I.chunk_info[h];
                const int nslot = __builtin_amdgcn_readfirstlane(info.y & ((1 << kSplitShift) - 1));
                const int lg = __builtin_amdgcn_readfirstlane(info.y >> kSplitShift);
                const int lw = STAGED ? s_var[h * kChunk + lane] : I.chunk_var[(size_t)h * kChunk + lane];
                // with lg > 0 a variable's clauses are spread over 2^lg lanes;
                // the first of them takes the decision
                const int v = (lw < 0 || (lane & ((1 << lg) - 1))) ? -1 : (lw & 0xFFFFF);
                // the variable's class is needed after the slot loop; load it now
                const int cl = (C.var_cls && v >= 0) ? (int)C.var_cls[v] : 0;
                // record row `row` of the chunk (16 bytes a lane) as a buffer
                // load: the row's byte offset is a scalar operand and the
                // lane's offset the same register for every row, so no vector
                // instruction computes a record address
                const int row0 = __builtin_amdgcn_readfirstlane(info.x) / 2;
                auto rp = [&](int row) -> uint4 {
                    if constexpr (STAGED)
                        return s_rec[(row0 + row) * kChunk + lane];
                    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                         recs, lane * 16, (row0 + row) * (kChunk * 16), 0));
                };
                // acc collects sum over slots of (spread(sat) xor signmask); the
                // closed form below turns it into 128 + dE-part per byte lane.
                // Slots come in 16-byte pairs; 8 slots of records are in flight
                // while 4 are consumed (nslot is a multiple of 4, at least 4; the
                // pair index is clamped so every load is in bounds).
                uint32_t acc[GPW];
#pragma unroll
                for (int k = 0; k < GPW; ++k)
                    acc[k] = 0;
                auto step = [&](uint32_t x, uint32_t y) {
                    if constexpr (GPW == 1)
                        acc[0] = slot_step(acc[0], make_uint2(x, y));
                    else
                        slot_step2(acc[0], acc[GPW - 1], make_uint2(x, y));
                };
                const int lastp = nslot / 2 - 1;
                uint4 q0 = rp(0), q1 = rp(min(1, lastp));
                uint4 q2 = rp(min(2, lastp)), q3 = rp(min(3, lastp));
                issue_fence();
                // whole groups of 8 slots with one exit, then a tail of 4
                int k = 0;
                for (; k + 2 * kSlotUnroll <= nslot; k += 2 * kSlotUnroll) {
                    step(q0.x, q0.y);
                    step(q0.z, q0.w);
                    step(q1.x, q1.y);
                    step(q1.z, q1.w);
                    q0 = rp(min(k / 2 + 4, lastp));
                    q1 = rp(min(k / 2 + 5, lastp));
                    issue_fence();
                    step(q2.x, q2.y);
                    step(q2.z, q2.w);
                    step(q3.x, q3.y);
                    step(q3.z, q3.w);
                    q2 = rp(min(k / 2 + 6, lastp));
                    q3 = rp(min(k / 2 + 7, lastp));
                    issue_fence();
                }
                if (k < nslot) {
                    step(q0.x, q0.y);
                    step(q0.z, q0.w);
                    step(q1.x, q1.y);
                    step(q1.z, q1.w);
                }
                const uint32_t nneg = lw < 0 ? 0u : ((uint32_t)lw >> 20) & 0xFFu;
                // the lane's share of the closed form (sums mod 2^32 add up
                // across lanes: an inert padding slot contributes 0)
#pragma unroll
                for (int k = 0; k < GPW; ++k) {
                    uint32_t part = ((uint32_t)nslot - 2u * nneg) * 0x01010101u - nneg - acc[k];
                    if constexpr (STAGED)
                        part = lane_group_sum(part, lg);
                    else
                        for (int off = 1; off < (1 << lg); off <<= 1)
                            part += (uint32_t)__shfl_xor((int)part, off, 64);
                    acc[k] = 0x80808080u + part;
                }
                if (v >= 0) {
                    const uint32_t xi = lds_load_u8((uint32_t)v);
                    const uint32_t *T = tl + cl * C.stride;
                    int de[NR];
                    uint32_t thr[NR];
                    uint32_t flip = 0, need = 0;
#pragma unroll
                    for (int j = 0; j < NR; ++j) {
                        const int S = (int)((acc[j >> 2] >> (8 * (j & 3))) & 0xFFu) - 128;
                        de[j] = ((xi >> j) & 1u) ? S : -S;
                        thr[j] = T[max(de[j], 0)];
                        const uint32_t on = (amask >> j) & 1u;
                        flip |= (on & (uint32_t)(de[j] <= 0)) << j;
                        need |= (on & (uint32_t)(de[j] > 0) & (uint32_t)(thr[j] != 0)) << j;
                    }
#pragma unroll
                    for (int k = 0; k < GPW; ++k) {
                        // one generator call per group gives its 4 replicas' words
                        if ((need >> (4 * k)) & 0xFu) {
                            const uint4 u = STAGED ? s_u[v]
                                                   : philox4x32_10((uint32_t)v, t, (uint32_t)(g0 + k),
                                                                   kStreamKsatSweep, C.key0, C.key1);
                            const int b = 4 * k;
                            flip |= (((need >> b) & 1u) && u.x < thr[b]) ? 1u << b : 0u;
                            flip |= (((need >> (b + 1)) & 1u) && u.y < thr[b + 1]) ? 2u << b : 0u;
                            flip |= (((need >> (b + 2)) & 1u) && u.z < thr[b + 2]) ? 4u << b : 0u;
                            flip |= (((need >> (b + 3)) & 1u) && u.w < thr[b + 3]) ? 8u << b : 0u;
                        }
                    }
                    if (flip) {
                        n_acc += __builtin_popcount(flip);
                        const uint32_t nx = xi ^ flip;
                        lds_store_u8((uint32_t)v, nx);
                        lds_store_u8((uint32_t)(n + v), ~nx & amask);
#pragma unroll
                        for (int j = 0; j < NR; ++j)
                            dsum[j] += ((flip >> j) & 1u) ? de[j] : 0;
                    }
                }
            }
            __syncthreads();
        }

        // sweep end: exact energies, best, first hit, snapshot
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const int dj = wave_sum(dsum[j]);
            if (lane == 0 && dj)
                atomicAdd(&red[j], dj);
        }
        __syncthreads();
        if (tid < nact) {
            E += red[tid];
            if (E < best) {
                best = E;
                atomicOr(&red[NR], 1 << tid);
            }
            if (fh < 0 && E <= C.target)
                fh = (int)(t + 1);
        }
        __syncthreads();
        const uint32_t imp = (uint32_t)red[NR];
        if (imp) {
#pragma unroll
            for (int k = 0; k < GPW; ++k) {
                const uint32_t ik = (imp >> (4 * k)) & 0xFu;
                if (!ik)
                    continue;
                uint8_t *bg = R.best_xs + (size_t)(g0 + k) * n;
                if (wide) {
                    const uint32_t i4 = ik * 0x01010101u;
                    for (int w = tid; w < n / 16; w += nthr) {
                        uint4 o = reinterpret_cast<const uint4 *>(bg)[w];
                        uint4 c = reinterpret_cast<const uint4 *>(xt)[w];
                        if (k) {
                            c.x >>= 4;
                            c.y >>= 4;
                            c.z >>= 4;
                            c.w >>= 4;
                        }
                        o.x = (o.x & ~i4) | (c.x & i4);
                        o.y = (o.y & ~i4) | (c.y & i4);
                        o.z = (o.z & ~i4) | (c.z & i4);
                        o.w = (o.w & ~i4) | (c.w & i4);
                        reinterpret_cast<uint4 *>(bg)[w] = o;
                    }
                } else {
                    for (int v = tid; v < n; v += nthr)
                        bg[v] = (uint8_t)((bg[v] & ~ik) | ((uint32_t)(xt[v] >> (4 * k)) & ik));
                }
            }
        }
        __syncthreads();
        if (tid < 16)
            red[tid] = 0;
    }

    __syncthreads();
#pragma unroll
    for (int k = 0; k < GPW; ++k) {
        if (k == 1 && !second)
            break;
        uint8_t *xk = xg + (size_t)k * n;
        if (wide) {
            for (int w = tid; w < n / 16; w += nthr) {
                uint4 b = reinterpret_cast<const uint4 *>(xt)[w];
                if (GPW == 2) {
                    const uint32_t sh = 4 * k;
                    b = make_uint4((b.x >> sh) & 0x0F0F0F0Fu, (b.y >> sh) & 0x0F0F0F0Fu, (b.z >> sh) & 0x0F0F0F0Fu,
                                   (b.w >> sh) & 0x0F0F0F0Fu);
                }
                reinterpret_cast<uint4 *>(xk)[w] = b;
            }
        } else {
            for (int v = tid; v < n; v += nthr)
                xk[v] = GPW == 2 ? (uint8_t)((xt[v] >> (4 * k)) & 0xFu) : xt[v];
        }
    }
    if (tid < nact) {
        R.energy[r0 + tid] = E;
        R.best[r0 + tid] = best;
        R.first_hit[r0 + tid] = fh;
    }
    unsigned long long acc_w = n_acc;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        acc_w += __shfl_xor(acc_w, off, 64);
    if (lane == 0 && acc_w)
        atomicAdd(R.accepted, acc_w);
}

// One item (GPW groups of 4 replicas) per workgroup (item = blockIdx.x).
template <int GPW>
__global__ void __launch_bounds__(1024) ksat_sweep_kernel(KsatDev I, KsatRepDev R, SweepCall C) {
    extern __shared__ __align__(16) uint8_t smem[];
    sweep_group<GPW>(I, R, C, blockIdx.x, smem);
}

// The same with the instance staged in LDS (one group of 4 replicas per
// workgroup).
__global__ void __launch_bounds__(1024) ksat_sweep_staged_kernel(KsatDev I, KsatRepDev R, SweepCall C) {
    extern __shared__ __align__(16) uint8_t smem[];
    sweep_group<1, true>(I, R, C, blockIdx.x, smem);
}

// Batched launch: many replica sets (jobs) of different instances in one
// grid.  items[] lists (job, group) pairs in decreasing cost; workgroup b
// runs items b, b + gridDim.x, ...  The dynamic LDS block is sized for the
// largest job.
__global__ void __launch_bounds__(1024) ksat_sweep_batch_kernel(const KsatJob *jobs, const int2 *items, int n_items) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const KsatJob &J = jobs[w.x];
        if (J.C.gpw == 2)
            sweep_group<2>(J.I, J.R, J.C, w.y, smem);
        else
            sweep_group<1>(J.I, J.R, J.C, w.y, smem);
        __syncthreads();
    }
}

// Backbone statistics for many jobs: items[] lists (job, first variable)
// blocks of 256 variables.
__global__ void ksat_magnetization_batch_kernel(const KsatJob *jobs, const int2 *items, int thr_num, int thr_den,
                                                int expand) {
    const int2 w = items[blockIdx.x];
    const KsatJob &J = jobs[w.x];
    const int v = w.y + threadIdx.x;
    if (v >= J.I.n)
        return;
    int c = 0;
    for (int g = 0; g < J.R.n_groups; ++g)
        c += __popc((uint32_t)J.R.xs[(size_t)g * J.I.n + v]);
    J.R.counts[v] = c;
    long long dev = 2ll * c - J.R.n_rep;
    if (dev < 0)
        dev = -dev;
    const uint8_t fz = (long long)thr_den * dev >= (long long)thr_num * J.R.n_rep;
    J.R.frozen[v] = fz;
    if (!expand)
        J.R.cls[v] = fz;
}

__global__ void ksat_expand_batch_kernel(const KsatJob *jobs, const int2 *items) {
    const int2 w = items[blockIdx.x];
    const KsatJob &J = jobs[w.x];
    const int v = w.y + threadIdx.x;
    if (v >= J.I.n)
        return;
    uint8_t hot = J.R.frozen[v];
    for (int q = J.I.var_ptr[v]; q < J.I.var_ptr[v + 1] && !hot; ++q) {
        const uint4 ad = reinterpret_cast<const uint4 *>(J.I.clause_addr)[J.I.var_cl[q]];
        const uint32_t a[4] = {ad.x, ad.y, ad.z, ad.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (a[j] < (uint32_t)(2 * J.I.n)) {
                const uint32_t u = a[j] < (uint32_t)J.I.n ? a[j] : a[j] - J.I.n;
                hot |= J.R.frozen[u];
            }
        }
    }
    J.R.cls[v] = hot;
}

// c_i = replicas with x_i = 1; frozen_i per the |magnetization| threshold.
__global__ void ksat_magnetization_kernel(KsatDev I, KsatRepDev R, int thr_num, int thr_den, int expand) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= I.n)
        return;
    int c = 0;
    for (int g = 0; g < R.n_groups; ++g)
        c += __popc((uint32_t)R.xs[(size_t)g * I.n + v]);
    R.counts[v] = c;
    long long dev = 2ll * c - R.n_rep;
    if (dev < 0)
        dev = -dev;
    const uint8_t fz = (long long)thr_den * dev >= (long long)thr_num * R.n_rep;
    R.frozen[v] = fz;
    if (!expand)
        R.cls[v] = fz;
}

// hot_i = frozen_i or some clause of i holds a frozen variable.
__global__ void ksat_expand_kernel(KsatDev I, KsatRepDev R) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= I.n)
        return;
    uint8_t hot = R.frozen[v];
    for (int q = I.var_ptr[v]; q < I.var_ptr[v + 1] && !hot; ++q) {
        const uint4 ad = reinterpret_cast<const uint4 *>(I.clause_addr)[I.var_cl[q]];
        const uint32_t a[4] = {ad.x, ad.y, ad.z, ad.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (a[j] < (uint32_t)(2 * I.n)) {
                const uint32_t w = a[j] < (uint32_t)I.n ? a[j] : a[j] - I.n;
                hot |= R.frozen[w];
            }
        }
    }
    R.cls[v] = hot;
}

// tally[0] = lowest best energy, tally[1] = replicas with best energy 0.
__global__ void ksat_tally_kernel(KsatRepDev R) {
    __shared__ int smin[16], scnt[16];
    int mn = INT_MAX, cnt = 0;
    for (int r = threadIdx.x; r < R.n_rep; r += blockDim.x) {
        const int b = R.best[r];
        mn = min(mn, b);
        cnt += b == 0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mn = min(mn, __shfl_xor(mn, off, 64));
        cnt += __shfl_xor(cnt, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smin[w] = mn;
        scnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
            mn = min(mn, smin[i]);
            cnt += scnt[i];
        }
        R.tally[0] = mn;
        R.tally[1] = cnt;
    }
}

__global__ void ksat_unpack_kernel(const uint8_t *xs, int n, int n_rep, uint8_t *rows) {
    const size_t total = (size_t)n_rep * n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(idx / n), v = (int)(idx % n);
        rows[idx] = (xs[(size_t)(r / kGroup) * n + v] >> (r % kGroup)) & 1u;
    }
}

__global__ void ksat_pack_kernel(const uint8_t *rows, int n, int n_groups, int n_rep, uint8_t *xs) {
    const size_t total = (size_t)n_groups * n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int g = (int)(idx / n), v = (int)(idx % n);
        uint32_t b = 0;
        for (int j = 0; j < kGroup; ++j) {
            const int r = g * kGroup + j;
            if (r < n_rep)
                b |= (rows[(size_t)r * n + v] & 1u) << j;
        }
        xs[idx] = (uint8_t)b;
    }
}

__global__ void set_status_kernel(const SetStatusSrc *src, SetStatus *out) {
    __shared__ long long smin[4];
    __shared__ int scnt[4], sfh[4];
    const SetStatusSrc S = src[blockIdx.x];
    long long mn = LLONG_MAX;
    int cnt = 0, fh = INT_MAX;
    for (int r = threadIdx.x; r < S.n_rep; r += blockDim.x) {
        const long long b = S.best_is_64 ? reinterpret_cast<const long long *>(S.best)[r]
                                         : (long long)reinterpret_cast<const int32_t *>(S.best)[r];
        mn = b < mn ? b : mn;
        cnt += b == 0;
        const int f = S.first_hit[r];
        if (f >= 0 && f < fh)
            fh = f;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const long long o = __shfl_xor(mn, off, 64);
        mn = o < mn ? o : mn;
        cnt += __shfl_xor(cnt, off, 64);
        fh = min(fh, __shfl_xor(fh, off, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smin[w] = mn;
        scnt[w] = cnt;
        sfh[w] = fh;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
            mn = smin[i] < mn ? smin[i] : mn;
            cnt += scnt[i];
            fh = min(fh, sfh[i]);
        }
        out[blockIdx.x].best = mn;
        out[blockIdx.x].n_zero = cnt;
        out[blockIdx.x].first_hit = fh == INT_MAX ? -1 : fh;
    }
}

int grid_for(size_t total, int block) {
    size_t g = (total + block - 1) / block;
    if (g > 65536)
        g = 65536;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

size_t ksat_sweep_lds_bytes(int n, int n_classes, int stride) {
    return align_up(2 * (size_t)n + 2, 16) + align_up((size_t)n_classes * stride, 4) * 4 + 16 * sizeof(int);
}

// LDS of the staged instance (records, chunk descriptors, lane words, class
// ranges, the sweep's random words per variable), placed after the block above
static size_t ksat_staged_bytes(const KsatDev &I) {
    return align_up(I.rec_bytes, 16) + align_up((size_t)I.n_chunks * 8, 16) + (size_t)I.n_chunks * kChunk * 4 +
           align_up(((size_t)I.n_colors + 1) * 4, 16) + (size_t)I.n * 16;
}

// small instances take the staged kernel unless NMC_KSAT_STAGE=0 (read at
// every launch, so a process can compare the two)
static bool ksat_stage_enabled() {
    const char *e = std::getenv("NMC_KSAT_STAGE");
    return !(e && e[0] == '0');
}

hipError_t launch_set_status(const SetStatusSrc *src, SetStatus *out, int n_sets, hipStream_t s) {
    hipLaunchKernelGGL(set_status_kernel, dim3(n_sets), dim3(256), 0, s, src, out);
    return hipGetLastError();
}

hipError_t ksat_launch_init(const KsatDev &I, const KsatRepDev &R, uint32_t key0, uint32_t key1, hipStream_t s) {
    const size_t total = (size_t)R.n_groups * I.n;
    hipLaunchKernelGGL(ksat_init_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, I, R, key0, key1);
    return hipGetLastError();
}

hipError_t ksat_launch_recount(const KsatDev &I, const uint8_t *xs, int n_groups, int n_rep, int32_t *energy_out,
                               hipStream_t s) {
    if (I.wide)
        return hipErrorNotSupported;  // wide instances count from their packed tables
    const size_t lds = align_up(2 * (size_t)I.n + 2, 16) + 16 * sizeof(int);
    // once per process (thread-safe initialization)
    static const hipError_t attr = hipFuncSetAttribute((const void *)ksat_recount_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)kLdsBytes);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL(ksat_recount_kernel, dim3(n_groups), dim3(1024), lds, s, I, xs, n_rep, energy_out);
    return hipGetLastError();
}

hipError_t ksat_launch_reset_tallies(const KsatRepDev &R, int n, hipStream_t s) {
    hipLaunchKernelGGL(ksat_reset_tallies_kernel, dim3(grid_for((size_t)R.n_groups * kGroup, 256)), dim3(256), 0, s,
                       R);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return hipMemcpyAsync(R.best_xs, R.xs, (size_t)R.n_groups * n, hipMemcpyDeviceToDevice, s);
}

hipError_t ksat_launch_sweep(const KsatDev &I, const KsatRepDev &R, const SweepCall &C, int block_threads,
                             hipStream_t s) {
    const size_t lds = ksat_sweep_lds_bytes(I.n, C.n_classes, C.stride);
    // once per process (thread-safe initialization)
    static const hipError_t attr = [] {
        hipError_t e = hipFuncSetAttribute((const void *)ksat_sweep_kernel<1>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)ksat_sweep_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kLdsBytes);
        return e;
    }();
    if (attr != hipSuccess)
        return attr;
    static const hipError_t attr_staged = hipFuncSetAttribute(
        (const void *)ksat_sweep_staged_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
    if (attr_staged != hipSuccess)
        return attr_staged;
    const size_t staged = lds + ksat_staged_bytes(I);
    if (C.gpw == 2)
        hipLaunchKernelGGL(ksat_sweep_kernel<2>, dim3((R.n_groups + 1) / 2), dim3(block_threads), lds, s, I, R, C);
    else if (staged <= kLdsBytes && ksat_stage_enabled())
        hipLaunchKernelGGL(ksat_sweep_staged_kernel, dim3(R.n_groups), dim3(block_threads), staged, s, I, R, C);
    else
        hipLaunchKernelGGL(ksat_sweep_kernel<1>, dim3(R.n_groups), dim3(block_threads), lds, s, I, R, C);
    return hipGetLastError();
}

hipError_t ksat_launch_sweep_batch(const KsatJob *jobs, const int2 *items, int n_items, size_t lds, int block_threads,
                                   int grid, hipStream_t s) {
    // once per process (thread-safe initialization)
    static const hipError_t attr = hipFuncSetAttribute((const void *)ksat_sweep_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)kLdsBytes);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL(ksat_sweep_batch_kernel, dim3(grid), dim3(block_threads), lds, s, jobs, items, n_items);
    return hipGetLastError();
}

int ksat_batch_occupancy(int block_threads, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)ksat_sweep_batch_kernel, block_threads, lds) !=
        hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

hipError_t ksat_launch_backbone_batch(const KsatJob *jobs, const int2 *items, int n_items, int thr_num, int thr_den,
                                      int expand, hipStream_t s) {
    hipLaunchKernelGGL(ksat_magnetization_batch_kernel, dim3(n_items), dim3(256), 0, s, jobs, items, thr_num, thr_den,
                       expand);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !expand)
        return e;
    hipLaunchKernelGGL(ksat_expand_batch_kernel, dim3(n_items), dim3(256), 0, s, jobs, items);
    return hipGetLastError();
}

hipError_t ksat_launch_backbone(const KsatDev &I, const KsatRepDev &R, int thr_num, int thr_den, int expand,
                                hipStream_t s) {
    hipLaunchKernelGGL(ksat_magnetization_kernel, dim3((I.n + 255) / 256), dim3(256), 0, s, I, R, thr_num, thr_den,
                       expand);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !expand)
        return e;
    hipLaunchKernelGGL(ksat_expand_kernel, dim3((I.n + 255) / 256), dim3(256), 0, s, I, R);
    return hipGetLastError();
}

hipError_t ksat_launch_tally(const KsatRepDev &R, hipStream_t s) {
    hipLaunchKernelGGL(ksat_tally_kernel, dim3(1), dim3(1024), 0, s, R);
    return hipGetLastError();
}

hipError_t ksat_launch_unpack(const uint8_t *xs, int n, int n_groups, int n_rep, uint8_t *rows, hipStream_t s) {
    (void)n_groups;
    hipLaunchKernelGGL(ksat_unpack_kernel, dim3(grid_for((size_t)n_rep * n, 256)), dim3(256), 0, s, xs, n, n_rep,
                       rows);
    return hipGetLastError();
}

hipError_t ksat_launch_pack(const uint8_t *rows, int n, int n_groups, int n_rep, uint8_t *xs, hipStream_t s) {
    hipLaunchKernelGGL(ksat_pack_kernel, dim3(grid_for((size_t)n_groups * n, 256)), dim3(256), 0, s, rows, n,
                       n_groups, n_rep, xs);
    return hipGetLastError();
}

}  // namespace nmc
