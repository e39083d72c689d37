// QAP kernels for gfx950.
//
// A workgroup of 16 waves owns 16 replicas, one per wave.  A wave evaluates
// four consecutive proposals of the lexicographic pair sequence at once, one
// per 16-lane row, each row splitting the sum over facilities k among its
// lanes; the decisions are then taken in sequence order: the first accepted
// proposal is applied and the ones after it (computed against the old
// assignment) are dropped and evaluated again in the next step.  A step thus
// commits 1 to 4 proposals with exactly the sequential result.  Flow F and
// distance D (bytes), the 16 permutations and the sweep's threshold tables sit
// in LDS.  Tempering launches (one table row per temperature) take the
// replicas in quads: a workgroup holds the quads blk, blk + B, blk + 2B and
// blk + 3B of its B-block grid, so under the temperature-major layout its four
// quads sit at four temperatures spread along the ladder and one workgroup's
// time no longer follows the hottest rows alone; every replica keeps its own
// counter block, so the mapping changes the speed, never the result.  For
// symmetric, zero-diagonal F and D (subsection "Quadratic
// Assignment Problems"; cost sum_ij F_ij D_{p_i p_j}) exchanging the locations
// of facilities a and b changes the cost by
//   dC = 2 * sum_{k != a,b} (F_ak - F_bk) * (D_{p_b p_k} - D_{p_a p_k}).
#include <climits>
#include <type_traits>

#include "nmc_internal.h"
#include "nmc_philox.h"

// The compiler's lane-write intrinsic (v_writelane_b32: src into lane
// `lane` of old; src and lane wave-uniform), which this toolchain's HIP
// headers do not name.
__device__ int nmc_amdgcn_writelane(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace nmc {

namespace {

constexpr int kRepPerBlock = kQapRepPerBlock;  // one replica per wave
constexpr int kBlockThreads = 64 * kRepPerBlock;

// Sum over the 16 lanes of each DPP row, returned to every lane of the row:
// rotations by 8, 4, 2, 1 within the row.
__device__ __forceinline__ int row_allreduce16(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);  // row_ror:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false);  // row_ror:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x122, 0xF, 0xF, false);  // row_ror:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x121, 0xF, 0xF, false);  // row_ror:1
    return x;
}

// Sum over each group of 8 lanes, returned to every lane of the group:
// swaps within quads (xor 1, xor 2), then the mirror within each half-row.
__device__ __forceinline__ int group_allreduce8(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    x += __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    x += __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    return x;
}

// Moves (a, b) `steps` places forward in the lexicographic pair order; past
// the last pair it parks on (n - 2, n - 1) so that every index stays in range.
// Row a holds the pairs (a, a + 1) .. (a, n - 1): steps that run past its end
// carry over to row a + 1, starting at (a + 1, a + 2).
__device__ __forceinline__ void pair_advance(int &a, int &b, int n, int steps) {
    b += steps;
    while (b >= n && a < n - 2) {
        const int over = b - n;  // steps left after reaching (a + 1, a + 2)
        ++a;
        b = a + 1 + over;
    }
    if (a >= n - 1 || b >= n) {
        a = n - 2;
        b = n - 1;
    }
}

__device__ __forceinline__ uint32_t sweep_word(uint32_t pair, uint32_t t, uint32_t group, int word, uint32_t key0,
                                               uint32_t key1) {
    const uint4 u4 = philox4x32_10(pair, t, group, kStreamQapSweep, key0, key1);
    return word == 0 ? u4.x : word == 1 ? u4.y : word == 2 ? u4.z : u4.w;
}

// Pair (a, b) at index q < n (n - 1) / 2 of the lexicographic order.  Counted
// from the last pair, m = n (n - 1) / 2 - 1 - q lies in row a = n - 2 - j,
// where j (j + 1) / 2 <= m < (j + 1) (j + 2) / 2; the float square root
// gives j up to one step, which the two checks settle.
__device__ __forceinline__ void pair_at(int q, int n, int &a, int &b) {
    const int m = n * (n - 1) / 2 - 1 - q;
    int j = (int)((sqrtf(8.0f * (float)m + 1.0f) - 1.0f) * 0.5f);
    j += (j + 1) * (j + 2) / 2 <= m;
    j -= j * (j + 1) / 2 > m;
    a = n - 2 - j;
    b = n - 1 - (m - j * (j + 1) / 2);
}

// x with lane l set to v (l and v wave-uniform).
__device__ __forceinline__ int lane_write(int x, int l, int v) { return nmc_amdgcn_writelane(v, l, x); }

// Threshold T(d) of a row in LDS (high digit A at [0, ha), low digit B at
// [ha, ha + 1024)): (A[d >> 10] B[d & 1023]) >> 32, and 0 from d = 1024 ha on.
__device__ __forceinline__ uint32_t qap_thr(const uint32_t *row, int ha, int d) {
    const int h = d >> kQapLowBits;
    return h < ha ? __umulhi(row[h], row[ha + (d & ((1 << kQapLowBits) - 1))]) : 0u;
}

// The acceptance bound of random word u: the smallest d >= 1 with T(d) <= u.
// For a row whose T never increases with d (the host checks every row), a
// proposal with cost change dC is accepted (dC <= 0, or u < T(dC)) exactly
// when dC < d*(u), so a step compares two integers instead of reading two
// table words.  The search starts at ceil(ln(2^32 / u) / beta), where
// 2^32 exp(-beta d) = u, checks that guess and the word before it, and
// otherwise moves outward in doubling steps and bisects: the result is exact
// whatever the guess; the guess only saves steps (for all but the smallest u
// it is right or one off).  1 / beta is the float after the row's B.
__device__ int qap_dstar(const uint32_t *row, int ha, uint32_t u) {
    const int dlim = ha << kQapLowBits;  // T(dlim) = 0 <= u
    const float inv_beta = __uint_as_float(row[ha + (1 << kQapLowBits)]);
    int e;
    const float m = frexpf((float)u, &e);  // u = m 2^e, m in [1/2, 1)
    const float x = ((float)(32 - e) - __log2f(m)) * 0.6931472f * inv_beta;
    const int g = x < (float)dlim ? max(1, (int)ceilf(x)) : dlim;
    const uint32_t tg = qap_thr(row, ha, g), tp = qap_thr(row, ha, max(g - 1, 1));
    int lo, hi;  // T(lo) > u (lo = 0: no d below hi), T(hi) <= u
    if (tg <= u) {
        if (g == 1 || tp > u)
            return g;
        hi = g - 1;
        for (int step = 1;; step <<= 1) {
            lo = max(0, hi - step);
            if (lo == 0 || qap_thr(row, ha, lo) > u)
                break;
            hi = lo;
        }
    } else {
        lo = g;
        for (int step = 1;; step <<= 1) {
            hi = min(dlim, lo + step);
            if (hi == dlim || qap_thr(row, ha, hi) <= u)
                break;
            lo = hi;
        }
    }
    while (hi - lo > 1) {
        const int mid = lo + ((hi - lo) >> 1);
        if (qap_thr(row, ha, mid) <= u)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

// Per lane, for pair index q (clamped to the sweep): with C.dstar the bound
// d* of the pair's random word u in the table row of the pair's class (HOT if
// either facility is), else u itself.
__device__ __forceinline__ uint32_t qap_lane_word(const QapDev &I, const QapCall &C, const uint32_t *tw,
                                                  const uint8_t *cls, bool one_class, uint32_t q, uint32_t t,
                                                  uint32_t group, int word) {
    const uint32_t u = sweep_word(q, t, group, word, C.key0, C.key1);
    if (!C.dstar)
        return u;
    const uint32_t *row = tw;
    if (!one_class) {
        int a, b;
        pair_at(min((int)q, I.n * (I.n - 1) / 2 - 1), I.n, a, b);
        row += max((int)cls[a], (int)cls[b]) * C.stride;
    }
    return (uint32_t)qap_dstar(row, I.ha, u);
}

__global__ void qap_init_kernel(QapDev I, QapRepDev R, uint32_t key0, uint32_t key1) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R.n_rep)
        return;
    const int n = I.n;
    uint8_t *p = R.perm + (size_t)r * n;
    for (int i = 0; i < n; ++i)
        p[i] = (uint8_t)i;
    for (int j = n - 1; j >= 1; --j) {
        const uint4 u4 = philox4x32_10((uint32_t)j, 0u, (uint32_t)(r >> 2), kStreamQapInit, key0, key1);
        const uint32_t w = (r & 3) == 0 ? u4.x : (r & 3) == 1 ? u4.y : (r & 3) == 2 ? u4.z : u4.w;
        const int k = (int)(((uint64_t)w * (uint64_t)(j + 1)) >> 32);
        const uint8_t tmp = p[j];
        p[j] = p[k];
        p[k] = tmp;
    }
    for (int i = 0; i < n; ++i)
        R.best_perm[(size_t)r * n + i] = p[i];
}

// Full cost of every replica: one workgroup per replica.
__global__ void qap_cost_kernel(QapDev I, const uint8_t *perm, int64_t *cost_out) {
    __shared__ uint8_t p[kQapMaxN + 1];
    __shared__ long long part[16];
    const int r = blockIdx.x, n = I.n, tid = threadIdx.x;
    for (int i = tid; i < n; i += blockDim.x)
        p[i] = perm[(size_t)r * n + i];
    __syncthreads();
    long long c = 0;
    for (int idx = tid; idx < n * n; idx += blockDim.x) {
        const int i = idx / n, j = idx % n;
        c += (long long)I.F[idx] * I.D[p[i] * n + p[j]];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        c += __shfl_xor(c, off, 64);
    if ((tid & 63) == 0)
        part[tid >> 6] = c;
    __syncthreads();
    if (tid == 0) {
        long long s = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            s += part[w];
        cost_out[r] = s;
    }
}

__global__ void qap_reset_tallies_kernel(QapRepDev R) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R.n_rep) {
        R.best[r] = R.cost[r];
        R.first_hit[r] = -1;
    }
}

// Flow matrix layout in LDS: row b holds F[b][k] at byte (k % 16) * KP + k / 16
// (zero for k >= n), so the KP bytes a lane of a 16-lane row needs
// (k = q, q + 16, ...) are contiguous and come in one wide read.  Fills
// f[i] = F[row][k_i] for the lane's k_i = q + (64 / ROWS) * i (the table-mode
// row sums).
template <int ROWS, int KPL, int KP>
__device__ __forceinline__ void flow_row(const uint8_t *row, int q, int (&f)[KPL]) {
    if constexpr (ROWS == 4) {
        uint32_t w[KP / 4];
        const uint32_t *src = reinterpret_cast<const uint32_t *>(row + q * KP);
#pragma unroll
        for (int j = 0; j < KP / 4; ++j)
            w[j] = src[j];
#pragma unroll
        for (int i = 0; i < KPL; ++i)
            f[i] = (int)((w[i >> 2] >> (8 * (i & 3))) & 0xFFu);
    } else {
#pragma unroll
        for (int i = 0; i < KPL; ++i) {
            const int k = q + (64 / ROWS) * i;
            f[i] = row[(k & 15) * KP + (k >> 4)];
        }
    }
}

// Second flow layout, for eight 8-lane rows: row b holds F[b][q + 8i] at byte
// q * 16 + i (zero past n), so a lane's 16 bytes come in one 16-byte read.
//
// Flow row b of a lane of the ROWS-row schemes as KW words, four facilities
// per word (byte j of word w: facility k_{4w+j} = q + (64 / ROWS)(4w + j)),
// straight from either layout: the lane's bytes are contiguous in both.
template <int ROWS, int KW, int KP>
__device__ __forceinline__ void flow_words(const uint8_t *F, const uint8_t *F8, int b, int q, uint32_t (&w)[KW]) {
    static_assert(ROWS == 8 ? KW <= 4 : 4 * KW <= KP, "flow layout");
    const uint32_t *src = reinterpret_cast<const uint32_t *>(ROWS == 8 ? F8 + b * 128 + q * 16 : F + b * 16 * KP + q * KP);
#pragma unroll
    for (int j = 0; j < KW; ++j)
        w[j] = src[j];
}

// Distance bytes drow[p_k] of the lane's facilities 4w .. 4w + 3, packed as
// one word (0 past the lane's KPL facilities).
template <int KPL>
__device__ __forceinline__ uint32_t gather_word(const uint8_t *drow, const int (&pk)[KPL], int w) {
    uint32_t g[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        g[j] = 4 * w + j < KPL ? (uint32_t)drow[pk[4 * w + j]] : 0u;
    return __builtin_amdgcn_perm(g[2] | (g[3] << 8), g[0] | (g[1] << 8), 0x05040100u);
}

// One sweep of one replica by one wave.  ROWS (4 or 8) proposals are
// evaluated per step, one per row of LANES = 64 / ROWS lanes; KPL = facilities per lane
// (k = q, q + LANES, ...), LANES * KPL <= 16 * KP, the flow row length (rows
// of F padded with zeros, so padding k contribute (0 - 0) * (...) = 0 and no
// lane needs a bound check).  Each lane keeps, for its k: the location p_k,
// and for its row's proposal (a, b): F[a][k] and D[p_a][p_k] in registers,
// refreshed when the row's a changes or a swap is applied; a proposal then
// needs F[b][k] and D[p_b][p_k] from LDS.  The sum runs over every k and is
// corrected by + 2 F_ab D_{p_a p_b}: with symmetric zero-diagonal matrices the
// k = a and k = b terms are -F_ab D_{p_b p_a} and -F_ab D_{p_a p_b}.
// The decisions are taken in pair order: the first accepted proposal is
// applied and the ones after it are evaluated again in the next step.
// Random words: lane l of a batch holds the word of pair base + l (64 pairs
// per generator call per lane); counter (pair, sweep, replica / 4, stream),
// word replica % 4.  Returns the number of accepted swaps.
template <int ROWS, int KPL, int KP>
__device__ __forceinline__ int qap_wave_sweep(const QapDev &I, const QapCall &C, const uint8_t *F, const uint8_t *F8,
                                              const uint8_t *D, const uint8_t *cls, const uint32_t *tl, uint8_t *pr,
                                              uint32_t t, uint32_t group, int word, long long &cost) {
    constexpr int LANES = 64 / ROWS;
    constexpr int RB = 16 * KP;  // bytes per flow row
    static_assert(ROWS == 8 || (ROWS == 4 && KPL <= KP), "flow layout");
    const int n = I.n;
    const int npairs = n * (n - 1) / 2;
    const int lane = threadIdx.x & 63;
    const int row = lane / LANES, q = lane % LANES;
    const bool one_class = C.n_classes == 1;
    // the lane's facilities four to a word: F[a][k] and D[p_a][p_k], and their
    // products' sum rw (all bytes, so every product is an exact 4-way dot)
    constexpr int KW = (KPL + 3) / 4;
    int pk[KPL];
    uint32_t faw[KW], daw[KW], rw = 0;
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = q + LANES * i;
        pk[i] = k < n ? pr[k] : 0;
    }
    // this row's proposal is pair p0 + row
    int p0 = 0, ar = 0, br = 1;
    pair_advance(ar, br, n, row);
    int cur_a = -1, pa = 0, n_acc = 0;
    bool refresh = false;  // a swap was applied: D[p_a][p_k] is stale
    uint32_t pbase = 0;
    // lane l: the word (or acceptance bound) of pair pbase + l and of pbase + 64 + l
    uint32_t uw = qap_lane_word(I, C, tl, cls, one_class, (uint32_t)lane, t, group, word);
    uint32_t uw2 = qap_lane_word(I, C, tl, cls, one_class, 64u + (uint32_t)lane, t, group, word);
    // locations of this step's b and a, read during the previous step
    // (valid because no swap happened since; re-read after a swap)
    int pb = pr[br], pa_ahead = pr[ar];
    while (p0 < npairs) {
        if (ar != cur_a) {
            cur_a = ar;
            pa = pa_ahead;
            flow_words<ROWS, KW, KP>(F, F8, ar, q, faw);
            refresh = true;
        }
        if (refresh) {
            rw = 0;
#pragma unroll
            for (int w = 0; w < KW; ++w) {
                daw[w] = gather_word<KPL>(D + pa * n, pk, w);
                rw = __builtin_amdgcn_udot4(faw[w], daw[w], rw, false);
            }
            refresh = false;
        }
        // the next step's pairs if no proposal of this step is accepted
        int an = ar, bn = br;
        pair_advance(an, bn, n, ROWS);
        const int pbn = pr[bn], pan = pr[an];
        uint32_t fbw[KW];
        flow_words<ROWS, KW, KP>(F, F8, br, q, fbw);
        const uint8_t *drow_b = D + pb * n;
        // sum_k (F_ak - F_bk)(D_{p_b p_k} - D_{p_a p_k}) over the lane's k as
        // F_a.D_b + F_b.D_a - F_b.D_b - F_a.D_a: four facilities per dot
        // instruction, in 32-bit words that hold each sum exactly
        uint32_t x = 0u - rw, y = 0u;
#pragma unroll
        for (int w = 0; w < KW; ++w) {
            const uint32_t dbw = gather_word<KPL>(drow_b, pk, w);
            x = __builtin_amdgcn_udot4(faw[w], dbw, x, false);
            x = __builtin_amdgcn_udot4(fbw[w], daw[w], x, false);
            y = __builtin_amdgcn_udot4(fbw[w], dbw, y, false);
        }
        int part = (int)(x - y);
        if (q == 0)
            part += 2 * (int)F[ar * RB + (br & 15) * KP + (br >> 4)] * (int)D[pa * n + pb];
        if constexpr (ROWS == 8)
            part = group_allreduce8(part);
        else
            part = row_allreduce16(part);
        const int dc = 2 * part;
        const int src = p0 + row - (int)pbase;  // 0 .. 63 + ROWS - 1
        const int sl = (src & 63) << 2;
        const uint32_t ua = (uint32_t)__builtin_amdgcn_ds_bpermute(sl, (int)uw);
        const uint32_t ub = (uint32_t)__builtin_amdgcn_ds_bpermute(sl, (int)uw2);
        const uint32_t u = src < 64 ? ua : ub;
        bool acc;
        if (C.dstar) {
            acc = dc < (int)u;
        } else {
            acc = dc <= 0;
            if (!acc) {
                const int cl = one_class ? 0 : max((int)cls[ar], (int)cls[br]);
                const uint32_t *T = tl + cl * C.stride;
                const int h = dc >> kQapLowBits, l = dc & ((1 << kQapLowBits) - 1);
                const uint32_t thr = h < I.ha ? (uint32_t)(((uint64_t)T[h] * (uint64_t)T[I.ha + l]) >> 32) : 0u;
                acc = u < thr;
            }
        }
        int adv = ROWS, j = -1;
        acc = acc && p0 + row < npairs;
        // every lane of a row holds its row's decision, so the first accepted
        // row starts at the ballot's lowest set bit
        const uint64_t m = __ballot(acc);
        if (m)
            j = (int)__builtin_ctzll(m) / LANES;
        if (j >= 0) {
            adv = j + 1;
            ++n_acc;
            const int jl = LANES * j;
            const int aj = __builtin_amdgcn_readlane(ar, jl);
            const int bj = __builtin_amdgcn_readlane(br, jl);
            const int paj = __builtin_amdgcn_readlane(pa, jl);
            const int pbj = __builtin_amdgcn_readlane(pb, jl);
            cost += __builtin_amdgcn_readlane(dc, jl);
            if (lane == 0) {
                pr[aj] = (uint8_t)pbj;
                pr[bj] = (uint8_t)paj;
            }
            // only the lanes holding k = aj and k = bj see new locations
            // (register index k / LANES is wave-uniform)
#pragma unroll
            for (int i = 0; i < KPL; ++i) {
                if (i == aj / LANES && q == aj % LANES)
                    pk[i] = pbj;
                if (i == bj / LANES && q == bj % LANES)
                    pk[i] = paj;
            }
            if (ar == aj)
                pa = pbj;
            else if (ar == bj)
                pa = paj;
            refresh = true;
        }
        p0 += adv;
        if (j >= 0) {
            pair_advance(ar, br, n, adv);
            pb = pr[br];
            pa_ahead = pr[ar];
        } else {
            ar = an;
            br = bn;
            pb = pbn;
            pa_ahead = pan;
        }
        if (p0 >= (int)pbase + 64) {
            pbase += 64;
            uw = uw2;
            uw2 = qap_lane_word(I, C, tl, cls, one_class, pbase + 64u + (uint32_t)lane, t, group, word);
        }
    }
    return n_acc;
}

// Sum over the wave, returned from lane 63: rotations within each 16-lane
// row, then row 1 takes row 0's sum and row 3 row 2's (row broadcast of lane
// 15), then rows 2 and 3 take lane 31's (row broadcast of lane 31).
__device__ __forceinline__ int wave_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);  // row_ror:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false);  // row_ror:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x122, 0xF, 0xF, false);  // row_ror:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x121, 0xF, 0xF, false);  // row_ror:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
    return __builtin_amdgcn_readlane(x, 63);
}


// One sweep of one replica by one wave, one proposal per step on all 64
// lanes (KPL facilities per lane, k = lane + 64 i), for sweeps where most
// proposals are accepted.  The permutation lives in the lanes while the sweep
// runs (p_k in the lane of facility k; a location is a readlane, a swap two
// lane selects) and goes back to LDS at the end.  Per row a of the pair order
// each lane keeps F[a][k] and D[p_a][p_k]; a proposal (a, b)
// reads F[b][k], gathers D[p_b][p_k], and sums (F_ak - F_bk)(D_{p_b p_k} -
// D_{p_a p_k}) over every k.  With symmetric zero-diagonal F and D the k = a
// and k = b terms are both -F_ab D_{p_a p_b}, so the definition's sum over the
// other k is that total plus 2 F_ab D_{p_a p_b}, whose factors b's lane holds.
// An accepted swap turns the cached row into the one just gathered, with 0 at
// k = a and the old D_{p_a p_b} at k = b.  A proposal is accepted when its
// change is below the acceptance bound d* of its random word (lane l holds
// the bound of pair pbase + l, from the wave's threshold rows tw in LDS;
// the call's rows must pass the host's check, C.dstar).  Same decisions,
// words and counters as qap_wave_sweep.  Returns the number of accepted swaps.
template <int KPL, int KP>
__device__ __forceinline__ int qap_wave_sweep1(const QapDev &I, const QapCall &C, const uint8_t *F, const uint8_t *D,
                                               const uint8_t *cls, const uint32_t *tw, uint8_t *pr, uint32_t t,
                                               uint32_t group, int word, long long &cost) {
    constexpr int RB = 16 * KP;
    const int n = I.n;
    const int lane = threadIdx.x & 63;
    const bool one_class = C.n_classes == 1;
    const int flo = (lane & 15) * KP + (lane >> 4);  // byte of k = lane in a flow row; k + 64 i at + 4 i
    int pk[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = lane + 64 * i;
        pk[i] = k < n ? pr[k] : 0;
    }
    int n_acc = 0, widx = 0;
    uint32_t pbase = 0;
    uint32_t dsv = qap_lane_word(I, C, tw, cls, one_class, (uint32_t)lane, t, group, word);
    // accepted changes since the last flush into cost: at most 64 proposals,
    // each |dC| <= 2 (n - 2) 255^2, so the sum fits 32 bits for n <= 255
    int csum = 0;
    // rows a in slot SA, pairs (a, b) with b in slot S >= SA: every slot index
    // is a compile-time constant, so the per-facility arrays stay in registers
#pragma unroll
    for (int SA = 0; SA < KPL; ++SA) {
        const int a_end = min(n - 1, 64 * SA + 64);
        for (int a = 64 * SA; a < a_end; ++a) {
            const int la = a - 64 * SA;
            int pa = __builtin_amdgcn_readlane(pk[SA], la);
            int fa[KPL], da[KPL];
#pragma unroll
            for (int i = 0; i < KPL; ++i) {
                fa[i] = F[a * RB + flo + 4 * i];
                da[i] = D[pa * n + pk[i]];
            }
            // the cached row's word at k = a: D[p_a][p_a] = 0 when gathered,
            // the accepted swap's D_{p_a p_b} after an accept (left in place
            // and taken out of the sum in closed form)
            int g = 0;
#pragma unroll
            for (int S = SA; S < KPL; ++S) {
                const int b_end = min(n, 64 * S + 64);
                for (int b = max(a + 1, 64 * S); b < b_end; ++b) {
                    const int lb = b - 64 * S;
                    const int pb = __builtin_amdgcn_readlane(pk[S], lb);
                    int db[KPL];
                    int part = 0;
#pragma unroll
                    for (int i = 0; i < KPL; ++i) {
                        const int fb = F[b * RB + flo + 4 * i];
                        db[i] = D[pb * n + pk[i]];
                        part += __mul24(fa[i] - fb, db[i] - da[i]);
                    }
                    // the k = b term is -F_ab D_ab and the k = a term, with g in
                    // place of D[p_a][p_a] = 0, -F_ab (D_ab - g)
                    const int fab = __builtin_amdgcn_readlane(fa[S], lb), dab = __builtin_amdgcn_readlane(da[S], lb);
                    const int dc = 2 * (wave_sum(part) + fab * (2 * dab - g));
                    const int ds = __builtin_amdgcn_readlane((int)dsv, widx);
                    if (dc < ds) {
                        ++n_acc;
                        csum += dc;
                        // p_a <-> p_b; the cached row becomes D[p_b][.]: the
                        // gathered row, with the old D_{p_a p_b} at k = b and
                        // (as g) at k = a
                        pk[SA] = lane_write(pk[SA], la, pb);
                        pk[S] = lane_write(pk[S], lb, pa);
#pragma unroll
                        for (int i = 0; i < KPL; ++i)
                            da[i] = db[i];
                        da[S] = lane_write(da[S], lb, dab);
                        g = dab;
                        pa = pb;
                    }
                    if (++widx == 64) {
                        widx = 0;
                        pbase += 64;
                        dsv = qap_lane_word(I, C, tw, cls, one_class, pbase + (uint32_t)lane, t, group, word);
                        cost += csum;
                        csum = 0;
                    }
                }
            }
        }
    }
    cost += csum;
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = lane + 64 * i;
        if (k < n)
            pr[k] = (uint8_t)pk[i];
    }
    return n_acc;
}

// ---- table mode -----------------------------------------------------------
//
// For sweeps where almost every proposal is rejected, each wave keeps its
// replica's change of cost dC(a, b) for every pair in a table in device
// memory (pair-index order), so a proposal costs one table read and 64
// consecutive proposals are judged at once; only an accepted swap (r, s)
// costs O(n^2) work (the Taillard-style delta update of subsection
// "Quadratic Assignment Problems"' move evaluation).  With symmetric,
// zero-diagonal F and D and
//   a_u = F_ur - F_us,  b_u = D_{p_u p_r} - D_{p_u p_s}   (before the swap),
// a pair (u, v) disjoint from {r, s} changes by 2 (a_u - a_v)(b_u - b_v):
// only its k = r, s terms move.  Pairs holding r or s are summed anew
// against the new assignment.  Decisions, words and counters are those of
// the other paths (the first accepted proposal of the 64 is applied, the
// ones after it are judged again), so the result is the sequential one.

__device__ __forceinline__ int pair_index(int a, int b, int n) { return a * (2 * n - a - 1) / 2 + (b - a - 1); }

// Table words are read and written at device scope (the accesses bypass the
// CU's vector L1 and meet at L2, where the no-return atomic adds of an
// update are performed), so a wave's reads after its own updates see them.
__device__ __forceinline__ int tab_ld(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void tab_st(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum over k of (F[x][k] - F[v][k]) (D[p_v][p_k] - D[p_x][p_k]) over every k
// except x and v, for this 16-lane row's v, with fx, dx, pk the lane's
// F[x][k], D[p_x][p_k], p_k (k = q + 16 i; zero flow past n).  Every lane of
// the row gets the sum.
template <int KPL, int KP>
__device__ __forceinline__ int tab_row_sum(const uint8_t *F, const uint8_t *D, int n, int q, int x, int px, int v,
                                           int pv, const int (&fx)[KPL], const int (&dx)[KPL],
                                           const int (&pk)[KPL]) {
    constexpr int RB = 16 * KP;
    int fv[KPL];
    flow_row<4, KPL, KP>(F + v * RB, q, fv);
    const uint8_t *drow = D + pv * n;
    int part = 0;
#pragma unroll
    for (int i = 0; i < KPL; ++i)
        part += (fx[i] - fv[i]) * ((int)drow[pk[i]] - dx[i]);
    // the k = x and k = v terms are each -F_xv D_{p_x p_v}
    if (q == 0)
        part += 2 * (int)F[x * RB + (v & 15) * KP + (v >> 4)] * (int)D[px * n + pv];
    return row_allreduce16(part);
}

template <int KPL, int KP>
__device__ __forceinline__ void tab_load_row(const uint8_t *F, const uint8_t *D, int n, int q, int x, int px,
                                             const int (&pk)[KPL], int (&fx)[KPL], int (&dx)[KPL]) {
    constexpr int RB = 16 * KP;
    flow_row<4, KPL, KP>(F + x * RB, q, fx);
#pragma unroll
    for (int i = 0; i < KPL; ++i)
        dx[i] = D[px * n + pk[i]];
}

// Fills the wave's table from its permutation: row a of pairs (a, b), four b
// per step, one per 16-lane row.
template <int KPL, int KP>
__device__ void tab_build(const QapDev &I, const uint8_t *F, const uint8_t *D, const uint8_t *pr, int32_t *dt) {
    const int n = I.n;
    const int lane = threadIdx.x & 63, row = lane >> 4, q = lane & 15;
    int pk[KPL], fa[KPL], da[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = q + 16 * i;
        pk[i] = k < n ? pr[k] : 0;
    }
    for (int a = 0; a < n - 1; ++a) {
        const int pa = pr[a];
        tab_load_row<KPL, KP>(F, D, n, q, a, pa, pk, fa, da);
        const int base = pair_index(a, a + 1, n) - (a + 1);
        for (int b0 = a + 1; b0 < n; b0 += 4) {
            const int b = b0 + row;
            const bool valid = b < n;
            const int bb = valid ? b : a + 1;
            const int sum = tab_row_sum<KPL, KP>(F, D, n, q, a, pa, bb, pr[bb], fa, da, pk);
            if (valid && q == 0)
                tab_st(dt + base + b, 2 * sum);
        }
    }
    __threadfence_block();
}

// The accepted swap (r, s), with pr still holding the old assignment:
// updates the table, then applies the swap to pr.
template <int KPL, int KP>
__device__ void tab_apply(const QapDev &I, const uint8_t *F, const uint8_t *D, uint8_t *pr, const uint16_t *PT,
                          int32_t *ab, int32_t *dt, int r, int s) {
    constexpr int RB = 16 * KP;
    const int n = I.n, npairs = n * (n - 1) / 2;
    const int lane = threadIdx.x & 63, row = lane >> 4, q = lane & 15;
    const int pr_r = pr[r], pr_s = pr[s];
    for (int u = lane; u < n; u += 64) {
        const int fo = (u & 15) * KP + (u >> 4);  // F[x][u] in the 16-lane flow layout
        const int au = (int)F[r * RB + fo] - (int)F[s * RB + fo];
        const int pu = pr[u];
        const int bu = (int)D[pu * n + pr_r] - (int)D[pu * n + pr_s];
        ab[u] = (int32_t)(((uint32_t)au & 0xFFFFu) | ((uint32_t)bu << 16));
    }
    __threadfence_block();
    // pairs disjoint from {r, s}: added in place (no-return atomic adds, so
    // the wave never waits on a table word here)
    for (int idx = lane; idx < npairs; idx += 64) {
        const uint32_t uv = PT[idx];
        const int u = uv & 0xFF, v = uv >> 8;
        if (u == r || u == s || v == r || v == s)
            continue;
        const int xu = ab[u], xv = ab[v];
        const int dau = __builtin_amdgcn_sbfe(xu, 0, 16) - __builtin_amdgcn_sbfe(xv, 0, 16);
        const int dbu = __builtin_amdgcn_sbfe(xu, 16, 16) - __builtin_amdgcn_sbfe(xv, 16, 16);
        const int inc = 2 * dau * dbu;
        if (inc)
            atomicAdd(dt + idx, inc);
    }
    if (lane == 0) {
        pr[r] = (uint8_t)pr_s;
        pr[s] = (uint8_t)pr_r;
    }
    __threadfence_block();
    // pairs holding r or s, summed against the new assignment
    int pk[KPL], fx[KPL], dx[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = q + 16 * i;
        pk[i] = k < n ? pr[k] : 0;
    }
#pragma unroll 1
    for (int w = 0; w < 2; ++w) {
        const int x = w == 0 ? r : s;
        const int px = pr[x];
        tab_load_row<KPL, KP>(F, D, n, q, x, px, pk, fx, dx);
        for (int v0 = 0; v0 < n; v0 += 4) {
            const int v = v0 + row;
            const bool valid = v < n && v != x;
            const int vv = valid ? v : (x == 0 ? 1 : 0);
            const int sum = tab_row_sum<KPL, KP>(F, D, n, q, x, px, vv, pr[vv], fx, dx, pk);
            if (valid && q == 0)
                tab_st(dt + (x < v ? pair_index(x, v, n) : pair_index(v, x, n)), 2 * sum);
        }
    }
    __threadfence_block();
}

// One sweep of one replica in table mode; `fresh` says whether the table
// already holds this permutation's changes (it does after a table-mode
// sweep of the same launch).  Returns the number of accepted swaps.
template <int KPL, int KP>
__device__ __forceinline__ int qap_wave_sweep_tab(const QapDev &I, const QapCall &C, const uint8_t *F,
                                                  const uint8_t *D, const uint8_t *cls, const uint32_t *tl,
                                                  uint8_t *pr, const uint16_t *PT, int32_t *ab, int32_t *dt,
                                                  uint32_t t, uint32_t group, int word, long long &cost,
                                                  bool &fresh) {
    const int n = I.n;
    const int npairs = n * (n - 1) / 2;
    const int lane = threadIdx.x & 63;
    const bool one_class = C.n_classes == 1;
    if (!fresh) {
        tab_build<KPL, KP>(I, F, D, pr, dt);
        fresh = true;
    }
    int n_acc = 0;
    uint32_t pbase = 0;
    uint32_t uw = sweep_word((uint32_t)lane, t, group, word, C.key0, C.key1);
    uint32_t uw2 = sweep_word(64u + (uint32_t)lane, t, group, word, C.key0, C.key1);
    // the table words of the next two 64-pair chunks are read ahead (valid
    // until a swap is applied; then read again from the restart)
    int p0 = 0;
    int d1 = lane < npairs ? tab_ld(dt + lane) : 0;
    int d2 = 64 + lane < npairs ? tab_ld(dt + 64 + lane) : 0;
    while (p0 < npairs) {
        const int idx = p0 + lane;
        const bool valid = idx < npairs;
        const int d = d1;
        d1 = d2;
        d2 = idx + 128 < npairs ? tab_ld(dt + idx + 128) : 0;
        const int src = idx - (int)pbase;  // 0 .. 126
        const int sl = (src & 63) << 2;
        const uint32_t ua = (uint32_t)__builtin_amdgcn_ds_bpermute(sl, (int)uw);
        const uint32_t ub = (uint32_t)__builtin_amdgcn_ds_bpermute(sl, (int)uw2);
        const uint32_t u = src < 64 ? ua : ub;
        bool acc = d <= 0;
        if (!acc) {
            int cl = 0;
            if (!one_class) {
                const uint32_t uv = PT[valid ? idx : 0];
                cl = max((int)cls[uv & 0xFF], (int)cls[uv >> 8]);
            }
            const uint32_t *T = tl + cl * C.stride;
            const int h = d >> kQapLowBits, l = d & ((1 << kQapLowBits) - 1);
            const uint32_t thr = h < I.ha ? (uint32_t)(((uint64_t)T[h] * (uint64_t)T[I.ha + l]) >> 32) : 0u;
            acc = u < thr;
        }
        const uint64_t m = __ballot(acc && valid);
        if (m == 0) {
            p0 += 64;
        } else {
            const int j = __builtin_ctzll(m);
            const int pj = p0 + j;
            cost += __builtin_amdgcn_readlane(d, j);
            ++n_acc;
            const uint32_t rs = PT[pj];
            tab_apply<KPL, KP>(I, F, D, pr, PT, ab, dt, (int)(rs & 0xFF), (int)(rs >> 8));
            p0 = pj + 1;
            d1 = p0 + lane < npairs ? tab_ld(dt + p0 + lane) : 0;
            d2 = p0 + 64 + lane < npairs ? tab_ld(dt + p0 + 64 + lane) : 0;
        }
        if (p0 >= (int)pbase + 64) {
            pbase += 64;
            uw = uw2;
            uw2 = sweep_word(pbase + 64u + (uint32_t)lane, t, group, word, C.key0, C.key1);
        }
    }
    return n_acc;
}

// ---- several replicas per wave --------------------------------------------
//
// For sweeps where many proposals are accepted, one wave runs RPW (2 or 4)
// replicas of one Philox group at once, one per row of 64 / RPW lanes: every
// replica proposes the same pair at the same step (the lexicographic order),
// so the walk over pairs, the flow rows and the class lookup are shared, and
// one generator call per lane gives a row the words of 64 / RPW pairs.  Each
// row sums its replica's change over k = q, q + 64 / RPW, ... (corrected by
// 2 F_ab D_{p_a p_b} for the k = a, b terms), decides, and applies its own
// swap under its own lane mask.  Decisions, words and counters are those of
// the one-replica paths.  costq / accq: the replicas' costs in and out and
// their accepted swaps, indexed by local replica.

// Sum over each row of 32 lanes, returned to every lane of the row.
__device__ __forceinline__ int row_allreduce32(int x) {
    x = row_allreduce16(x);
    const auto sw = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // rows 0 <-> 1, 2 <-> 3
    return (int)sw[0] + (int)sw[1];
}

// F[b][k] for k = q + LANES i (i < KPL) from the 16-lane flow layout (row b
// holds F[b][k] at byte (k % 16) * KP + k / 16): for LANES = 32 the lane's
// bytes are q / 16 + 2 i of its KP-byte segment.
template <int LANES, int KPL, int KP>
__device__ __forceinline__ void flow_row_lanes(const uint8_t *row, int q, int (&f)[KPL]) {
    if constexpr (LANES == 16) {
        flow_row<4, KPL, KP>(row, q, f);
    } else {
        static_assert(LANES == 32 && 2 * KPL <= KP, "flow layout");
        uint32_t w[KP / 4];
        const uint32_t *src = reinterpret_cast<const uint32_t *>(row + (q & 15) * KP);
#pragma unroll
        for (int j = 0; j < KP / 4; ++j)
            w[j] = src[j];
        const int h = q >> 4;
#pragma unroll
        for (int i = 0; i < KPL; ++i) {
            const uint32_t lo = (w[(2 * i) >> 2] >> (8 * ((2 * i) & 3))) & 0xFFu;
            const uint32_t hi = (w[(2 * i + 1) >> 2] >> (8 * ((2 * i + 1) & 3))) & 0xFFu;
            f[i] = (int)(h ? hi : lo);
        }
    }
}

template <int RPW, int KPL, int KP>
__device__ __forceinline__ void qap_multi_sweep(const QapDev &I, const QapCall &C, const uint8_t *F,
                                                const uint8_t *D, const uint8_t *cls, const uint32_t *tl, uint8_t *P,
                                                int npad, int w, uint32_t t, uint32_t group, int word0,
                                                long long *costq, int *accq) {
    constexpr int LANES = 64 / RPW;
    constexpr int RB = 16 * KP;
    const int n = I.n;
    const int npairs = n * (n - 1) / 2;
    const int lane = threadIdx.x & 63, row = lane / LANES, q = lane % LANES;
    const bool one_class = C.n_classes == 1;
    const int lr = w * RPW + row;  // local replica of this row
    uint8_t *pr = P + lr * npad;
    long long cost = costq[lr];
    int pk[KPL], fa[KPL], da[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = q + LANES * i;
        pk[i] = k < n ? pr[k] : 0;
    }
    int ar = 0, br = 1;
    int pa = pr[0], pb = pr[1];
    flow_row_lanes<LANES, KPL, KP>(F, q, fa);
#pragma unroll
    for (int i = 0; i < KPL; ++i)
        da[i] = D[pa * n + pk[i]];
    int n_acc = 0;
    uint32_t pbase = 0;
    // lane (row, q) holds its replica's word of pair pbase + q
    uint32_t uw = sweep_word(pbase + (uint32_t)q, t, group, word0 + row, C.key0, C.key1);
    for (int p0 = 0; p0 < npairs; ++p0) {
        int an = ar, bn = br;
        pair_advance(an, bn, n, 1);
        const bool new_a = an != ar;  // wave-uniform
        int pbn = pr[bn], pan = pa;
        int fan[KPL];
        if (new_a) {
            pan = pr[an];
            flow_row_lanes<LANES, KPL, KP>(F + an * RB, q, fan);
        }
        int fb[KPL], db[KPL];
        flow_row_lanes<LANES, KPL, KP>(F + br * RB, q, fb);
        const uint8_t *drow = D + pb * n;
        int part = 0;
#pragma unroll
        for (int i = 0; i < KPL; ++i) {
            db[i] = drow[pk[i]];
            part += (fa[i] - fb[i]) * (db[i] - da[i]);
        }
        if (q == 0)
            part += 2 * (int)F[ar * RB + (br & 15) * KP + (br >> 4)] * (int)D[pa * n + pb];
        const int dc = 2 * (LANES == 16 ? row_allreduce16(part) : row_allreduce32(part));
        const uint32_t u = (uint32_t)__builtin_amdgcn_ds_bpermute((row * LANES + (p0 - (int)pbase)) << 2, (int)uw);
        bool acc = dc <= 0;
        if (!acc) {
            const int cl = one_class ? 0 : max((int)cls[ar], (int)cls[br]);
            const uint32_t *T = tl + cl * C.stride;
            const int h = dc >> kQapLowBits, l = dc & ((1 << kQapLowBits) - 1);
            const uint32_t thr = h < I.ha ? (uint32_t)(((uint64_t)T[h] * (uint64_t)T[I.ha + l]) >> 32) : 0u;
            acc = u < thr;
        }
        if (acc) {
            ++n_acc;
            cost += dc;
            if (q == 0) {
                pr[ar] = (uint8_t)pb;
                pr[br] = (uint8_t)pa;
            }
            // the new row D[p_a][p_k] is the one just gathered, with 0 at k = a
            // and the old D[p_a][p_b] at k = b (register index k / LANES is
            // wave-uniform)
#pragma unroll
            for (int i = 0; i < KPL; ++i) {
                const int da_old = da[i];
                da[i] = db[i];
                if (i == ar / LANES && q == ar % LANES) {
                    da[i] = 0;
                    pk[i] = pb;
                }
                if (i == br / LANES && q == br % LANES) {
                    da[i] = da_old;
                    pk[i] = pa;
                }
            }
            // locations read ahead that this swap changed
            if (bn == ar)
                pbn = pb;
            else if (bn == br)
                pbn = pa;
            if (an == br)
                pan = pa;
            const int pa_old = pa;
            pa = pb;
            pb = pa_old;
        }
        if (new_a) {
            ar = an;
            pa = pan;
#pragma unroll
            for (int i = 0; i < KPL; ++i) {
                fa[i] = fan[i];
                da[i] = D[pa * n + pk[i]];
            }
        }
        br = bn;
        pb = pbn;
        if (p0 + 1 == (int)pbase + LANES) {
            pbase += LANES;
            uw = sweep_word(pbase + (uint32_t)q, t, group, word0 + row, C.key0, C.key1);
        }
    }
    if (q == 0) {
        costq[lr] = cost;
        accq[lr] = n_acc;
    }
}

// Sweeps a launch must still hold for a wave to enter the table mode with a
// table it has to build first (about a quarter of a sweep's work).
constexpr int kTabMinSweeps = 8;
// Acceptance below which the per-sweep choice takes the table mode: fewer
// than npairs / kTabAccDen swaps accepted in the previous sweep.
constexpr int kTabAccDen = 128;

// n_sweeps sweeps for the 16 replicas of block `blk`, by the whole
// 1024-thread workgroup, with smem = the workgroup's dynamic LDS block.  Each
// wave picks, per sweep, eight proposals per step (8 lanes each) when very few
// proposals were accepted in its previous sweep, four (16 lanes each) when
// few, else one (64 lanes): with
// many acceptances most of the four would be dropped.  The previous sweep may
// be the replica's last one in an earlier launch (a per-replica hint byte), so
// launches of one sweep each, as in tempering, still get the width that
// suits the replica.  The choice changes only the speed, never the result.  With `mix` (tempering, n_rep a multiple
// of 16) wave w runs replica 4 (blk + (w / 4) B) + w % 4 for B = n_rep / 16
// and reads the table row of its quad; otherwise replica 16 blk + w and the
// block's one row.
// MODE selects the optional sweep kinds compiled into the kernel (each adds
// registers that would otherwise slow the default paths): bit 0 the table
// mode, bit 1 four replicas per wave.
template <int KPL4, int KPL1, int KPL8, int MODE>
__device__ __forceinline__ void qap_sweep_block(const QapDev &I, const QapRepDev &R, const QapCall &C, const int blk,
                                                const bool mix, uint8_t *smem) {
    constexpr int KP = KPL4 <= 4 ? 4 : KPL4 <= 8 ? 8 : 16;  // flow bytes per lane of a 16-lane row
    constexpr int FS = 16 * KP;                            // flow row bytes
    static_assert(64 * KPL1 <= FS, "flow row too short for one proposal per step");
    static_assert(8 * KPL8 <= FS, "flow row too short for eight proposals per step");
    const int n = I.n, nn = n * n;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int npad = (int)align_up(n, 4);
    const int npairs = n * (n - 1) / 2;

    uint8_t *F = smem;  // [n][FS]
    uint8_t *F8 = F + align_up((size_t)n * FS, 16);  // [n][128], only with the 8-row scheme
    uint8_t *D = F8 + (KPL8 > 0 ? align_up((size_t)n * 128, 16) : 0);
    uint8_t *P = D + align_up(nn, 16);
    uint8_t *cls = P + kRepPerBlock * npad;
    uint32_t *tl = (uint32_t *)(cls + align_up(n, 16));
    const int tab_words = C.n_classes * C.stride;
    const int nslots = mix ? kRepPerBlock / 4 : 1;  // table rows held in LDS
    // table mode: pair list and per-wave update vectors after the thresholds
    // (present when they fit; the launch sizes LDS with the same rule)
    const bool tab_ok =
        (MODE & 1) && qap_tab_fits(n, nslots * C.n_classes, C.stride) && (C.tab_allow || C.rows == 2);
    uint8_t *QX = (uint8_t *)tl + align_up((size_t)nslots * tab_words * 4, 16);
    long long *qcost = (long long *)QX;               // [16]
    int *qacc = (int *)(QX + 16 * sizeof(long long)); // [16]
    int *qrows = qacc + 16;                           // [16]
    uint16_t *PT = (uint16_t *)(QX + kQapQuadBytes);
    int32_t *AB = (int32_t *)((uint8_t *)PT + align_up((size_t)n * (n - 1), 16));
    const int quad_stride = R.n_rep / 4 / 4;        // B quads between a block's slots (mix only)
    // replica of wave (or P row) w
    auto rep_of = [&](int w) { return mix ? 4 * (blk + (w >> 2) * quad_stride) + (w & 3) : blk * kRepPerBlock + w; };

    for (int i = tid; i < n * FS; i += blockDim.x) {
        const int r = i / FS, o = i % FS;
        const int k = (o % KP) * 16 + o / KP;  // inverse of (k % 16) * KP + k / 16
        F[i] = k < n ? I.F[r * n + k] : 0;
    }
    if constexpr (KPL8 > 0) {
        for (int i = tid; i < n * 128; i += blockDim.x) {
            const int r = i >> 7, k = ((i >> 4) & 7) + 8 * (i & 15);  // byte q * 16 + j holds k = q + 8j
            F8[i] = k < n ? I.F[r * n + k] : 0;
        }
    }
    for (int i = tid; i < nn; i += blockDim.x)
        D[i] = I.D[i];
    for (int i = tid; i < n; i += blockDim.x)
        cls[i] = C.fac_cls ? C.fac_cls[i] : 0;
    if ((MODE & 1) && tab_ok) {
        // pair list: entry pair_index(a, b) holds a | b << 8
        for (int a = tid; a < n - 1; a += blockDim.x) {
            const int base = pair_index(a, a + 1, n) - (a + 1);
            for (int b = a + 1; b < n; ++b)
                PT[base + b] = (uint16_t)(a | (b << 8));
        }
    }
    // per-temperature tables (tempering): the replicas of a quad (mix) or of
    // the block share one row
    auto row_of = [&](int slot) {
        return C.tab + (C.reps_per_row > 0 ? (size_t)(rep_of(4 * slot) / C.reps_per_row) * tab_words : 0);
    };
    for (int i = tid; i < kRepPerBlock * n; i += blockDim.x) {
        const int rl = i / n, f = i % n;
        const int rep = rep_of(rl);
        P[rl * npad + f] = rep < R.n_rep ? R.perm[(size_t)rep * n + f] : (uint8_t)f;
    }
    const int rep = rep_of(wave);
    const bool active = rep < R.n_rep;  // wave-uniform
    uint8_t *pr = P + wave * npad;
    const uint32_t *tw = tl + (mix ? (wave >> 2) * tab_words : 0);  // this wave's table
    const uint32_t group = (uint32_t)rep >> 2;
    const int word = rep & 3;

    long long cost = 0, best = 0;
    unsigned long long acc_total = 0;  // swaps this wave accepted in this call
    int fh = -1, hint = 0;
    if (active) {
        hint = R.rows_hint[rep];
        cost = R.cost[rep];
        best = R.best[rep];
        fh = R.first_hit[rep];
        if (C.check_start && fh < 0 && cost <= C.target)
            fh = (int)C.t0;
    }
    __syncthreads();

    // proposals per step: 8 (when the size allows), 4 or 1, or the table
    // mode (2); the first sweep of a launch takes what the replica's last
    // sweep chose (the table mode only when the launch is long enough to
    // repay building the table)
    int rows = C.rows == 3 ? 1 : C.rows != 0 ? C.rows : (hint == 1 || hint == 8 || hint == 2) ? hint : 4;
    if (rows == 2 && !(tab_ok && (C.rows == 2 || C.n_sweeps >= kTabMinSweeps)))
        rows = 8;
    if (rows == 8 && KPL8 == 0)
        rows = 4;
    bool fresh = false;  // this wave's table holds its permutation's changes
    int32_t *dt = R.dtab + (size_t)(active ? rep : 0) * npairs;
    int32_t *ab = AB + wave * (int)align_up((size_t)n, 4);
    // every wave's choice for the next sweep: when all 16 replicas take one
    // proposal per step (or C.rows pins 3), waves 0..3 run them four per wave
    if ((MODE & 2) && lane == 0)
        qrows[wave] = active ? rows : 0;
    for (int s = 0; s < C.n_sweeps; ++s) {
        const uint32_t t = C.t0 + (uint32_t)s;
        for (int q = 0; q < nslots; ++q) {
            const uint32_t *tg = row_of(q) + (size_t)s * C.sweep_words;
            for (int i = tid; i < tab_words; i += blockDim.x)
                tl[q * tab_words + i] = tg[i];
        }
        if ((MODE & 2) && lane == 0 && active)
            qcost[wave] = cost;
        __syncthreads();
        bool quad = (MODE & 2) != 0;
        if constexpr ((MODE & 2) != 0) {
#pragma unroll
            for (int w = 0; w < kRepPerBlock; ++w) {
                const int rw = qrows[w];
                quad = quad && (C.rows == 3 ? rw != 0 : C.rows == 0 && rw == 1);
            }
            if (quad) {
                // RPW replicas per wave in waves 0 .. 16 / RPW - 1
                constexpr int RPW = (MODE & 4) ? 4 : 2;
                constexpr int KPLR = RPW == 4 ? KPL4 : (KPL4 + 1) / 2;
                if (wave < kRepPerBlock / RPW)
                    qap_multi_sweep<RPW, KPLR, KP>(I, C, F, D, cls, tl + (mix ? (wave * RPW / 4) * tab_words : 0), P,
                                                   npad, wave, t, (uint32_t)rep_of(wave * RPW) >> 2,
                                                   rep_of(wave * RPW) & 3, qcost, qacc);
                fresh = false;
                __syncthreads();
            }
        }

        if (active) {
            int n_acc;
            if ((MODE & 2) && quad) {
                cost = qcost[wave];
                n_acc = qacc[wave];
            } else if ((MODE & 1) && rows == 2) {
                if constexpr ((MODE & 1) != 0)
                    n_acc = qap_wave_sweep_tab<KPL4, KP>(I, C, F, D, cls, tw, pr, PT, ab, dt, t, group, word, cost,
                                                         fresh);
            } else {
                fresh = false;  // the other paths do not keep the table
                if constexpr (KPL8 > 0) {
                    if (rows == 8)
                        n_acc = qap_wave_sweep<8, KPL8, KP>(I, C, F, F8, D, cls, tw, pr, t, group, word, cost);
                    else
                        n_acc = rows == 4 || !C.dstar
                                    ? qap_wave_sweep<4, KPL4, KP>(I, C, F, F8, D, cls, tw, pr, t, group, word, cost)
                                    : qap_wave_sweep1<KPL1, KP>(I, C, F, D, cls, tw, pr, t, group, word, cost);
                } else {
                    // (the one-proposal path needs the acceptance bounds)
                    n_acc = rows == 4 || !C.dstar
                                ? qap_wave_sweep<4, KPL4, KP>(I, C, F, F8, D, cls, tw, pr, t, group, word, cost)
                                : qap_wave_sweep1<KPL1, KP>(I, C, F, D, cls, tw, pr, t, group, word, cost);
                }
            }
            acc_total += (unsigned long long)n_acc;
            if (C.rows == 0) {
                // acceptance of this sweep: above 1/8 one proposal per step,
                // below 1/16 eight, else four; below 1/kTabAccDen the table
                // mode, when its table is current or the launch has sweeps
                // enough left to repay building it
                rows = 8 * n_acc > npairs ? 1 : (16 * n_acc < npairs && KPL8 > 0) ? 8 : 4;
                if (tab_ok && kTabAccDen * n_acc < npairs && (fresh || C.n_sweeps - s - 1 >= kTabMinSweeps))
                    rows = 2;
            }
            // sweep end
            bool imp = false;
            if (cost < best) {
                best = cost;
                imp = true;
            }
            if (fh < 0 && cost <= C.target)
                fh = (int)(t + 1);
            if (imp) {
                for (int f = lane; f < n; f += 64)
                    R.best_perm[(size_t)rep * n + f] = pr[f];
            }
        }
        if ((MODE & 2) && lane == 0)
            qrows[wave] = active ? (C.rows == 3 ? 3 : rows) : 0;
        __syncthreads();
    }

    if (active) {
        for (int f = lane; f < n; f += 64)
            R.perm[(size_t)rep * n + f] = pr[f];
        if (lane == 0) {
            R.cost[rep] = cost;
            R.best[rep] = best;
            R.first_hit[rep] = fh;
            if (C.rows == 0)
                R.rows_hint[rep] = (uint8_t)rows;
            if (acc_total)
                atomicAdd(R.accepted, acc_total);
        }
    }
}

// facilities per lane with 16, 64 and 8 lanes per proposal (0: no 8-lane mode)
template <typename Fn>
__device__ __forceinline__ void qap_dispatch_kpl(int n, Fn &&fn) {
    using std::integral_constant;
    if (n <= 32)
        fn(integral_constant<int, 2>{}, integral_constant<int, 1>{}, integral_constant<int, 4>{});
    else if (n <= 64)
        fn(integral_constant<int, 4>{}, integral_constant<int, 1>{}, integral_constant<int, 8>{});
    else if (n <= 112)
        fn(integral_constant<int, 7>{}, integral_constant<int, 2>{}, integral_constant<int, 14>{});
    else if (n <= 160)
        fn(integral_constant<int, 10>{}, integral_constant<int, 3>{}, integral_constant<int, 0>{});
    else
        fn(integral_constant<int, 16>{}, integral_constant<int, 4>{}, integral_constant<int, 0>{});
}

template <int MODE>
__global__ void __launch_bounds__(1024) qap_sweep_kernel(QapDev I, QapRepDev R, QapCall C, bool mix) {
    extern __shared__ __align__(16) uint8_t smem[];
    qap_dispatch_kpl(I.n, [&](auto k4, auto k1, auto k8) {
        qap_sweep_block<decltype(k4)::value, decltype(k1)::value, decltype(k8)::value, MODE>(I, R, C, blockIdx.x,
                                                                                            mix, smem);
    });
}

// Batched launch over (job, block of 16 replicas) items in decreasing cost.
__global__ void __launch_bounds__(1024) qap_sweep_batch_kernel(const QapJob *jobs, const int2 *items, int n_items) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 w = items[it];
        const QapJob &J = jobs[w.x];
        qap_dispatch_kpl(J.I.n, [&](auto k4, auto k1, auto k8) {
            qap_sweep_block<decltype(k4)::value, decltype(k1)::value, decltype(k8)::value, 0>(J.I, J.R, J.C, w.y,
                                                                                             false, smem);
        });
        __syncthreads();
    }
}

// Assignment frequencies and the per-facility frozen test: one workgroup per facility.
__device__ __forceinline__ void qap_backbone_facility(const QapDev &I, const QapRepDev &R, int thr_num, int thr_den,
                                                      const int f) {
    __shared__ int hist[kQapMaxN + 1];
    __shared__ int mx;
    const int n = I.n;
    for (int l = threadIdx.x; l < n; l += blockDim.x)
        hist[l] = 0;
    if (threadIdx.x == 0)
        mx = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < R.n_rep; r += blockDim.x)
        atomicAdd(&hist[R.perm[(size_t)r * n + f]], 1);
    __syncthreads();
    for (int l = threadIdx.x; l < n; l += blockDim.x) {
        R.freq[(size_t)f * n + l] = hist[l];
        atomicMax(&mx, hist[l]);
    }
    __syncthreads();
    if (threadIdx.x == 0)
        R.cls[f] = (long long)thr_den * mx >= (long long)thr_num * R.n_rep;
}

__global__ void qap_backbone_kernel(QapDev I, QapRepDev R, int thr_num, int thr_den) {
    qap_backbone_facility(I, R, thr_num, thr_den, blockIdx.x);
}

__global__ void qap_backbone_batch_kernel(const QapJob *jobs, const int2 *items, int thr_num, int thr_den) {
    const int2 w = items[blockIdx.x];
    qap_backbone_facility(jobs[w.x].I, jobs[w.x].R, thr_num, thr_den, w.y);
}

__global__ void qap_tally_kernel(QapRepDev R) {
    __shared__ long long smin[16];
    __shared__ int scnt[16];
    long long mn = LLONG_MAX;
    int cnt = 0;
    for (int r = threadIdx.x; r < R.n_rep; r += blockDim.x) {
        const long long b = R.best[r];
        mn = b < mn ? b : mn;
        cnt += b == 0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const long long o = __shfl_xor(mn, off, 64);
        mn = o < mn ? o : mn;
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
            mn = smin[i] < mn ? smin[i] : mn;
            cnt += scnt[i];
        }
        reinterpret_cast<long long *>(R.tally)[0] = mn;
        R.tally[2] = cnt;
    }
}

}  // namespace

size_t qap_sweep_lds_bytes(int n, int n_classes, int stride) {
    return qap_base_lds(n, n_classes, stride) + (qap_tab_fits(n, n_classes, stride) ? qap_tab_lds(n) : 0);
}

hipError_t qap_launch_init(const QapDev &I, const QapRepDev &R, uint32_t key0, uint32_t key1, hipStream_t s) {
    hipLaunchKernelGGL(qap_init_kernel, dim3((R.n_rep + 127) / 128), dim3(128), 0, s, I, R, key0, key1);
    return hipGetLastError();
}

hipError_t qap_launch_cost(const QapDev &I, const uint8_t *perm, int n_rep, int64_t *cost_out, hipStream_t s) {
    hipLaunchKernelGGL(qap_cost_kernel, dim3(n_rep), dim3(256), 0, s, I, perm, cost_out);
    return hipGetLastError();
}

hipError_t qap_launch_reset_tallies(const QapRepDev &R, int n, hipStream_t s) {
    hipLaunchKernelGGL(qap_reset_tallies_kernel, dim3((R.n_rep + 255) / 256), dim3(256), 0, s, R);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return hipMemcpyAsync(R.best_perm, R.perm, (size_t)R.n_rep * n, hipMemcpyDeviceToDevice, s);
}

hipError_t qap_launch_sweep(const QapDev &I, const QapRepDev &R, const QapCall &C, int block_threads, hipStream_t s) {
    (void)block_threads;
    // quads of four temperatures per workgroup when their four table rows fit
    const size_t lds_mix = qap_sweep_lds_bytes(I.n, 4 * C.n_classes, C.stride);
    const bool mix = C.reps_per_row > 0 && C.reps_per_row % 4 == 0 && R.n_rep % kRepPerBlock == 0 &&
                     lds_mix <= kLdsBytes;
    const size_t lds = mix ? lds_mix : qap_sweep_lds_bytes(I.n, C.n_classes, C.stride);
    // once per process (thread-safe initialization)
    static const hipError_t attr = [] {
        hipError_t e = hipSuccess;
        for (const void *f : {(const void *)qap_sweep_kernel<0>, (const void *)qap_sweep_kernel<1>,
                              (const void *)qap_sweep_kernel<2>, (const void *)qap_sweep_kernel<6>})
            if (e == hipSuccess)
                e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
        return e;
    }();
    if (attr != hipSuccess)
        return attr;
    const int blocks = (R.n_rep + kRepPerBlock - 1) / kRepPerBlock;
    // the table mode and four replicas per wave are kernels of their own
    if (C.rows == 2 || C.tab_allow)
        hipLaunchKernelGGL(qap_sweep_kernel<1>, dim3(blocks), dim3(kBlockThreads), lds, s, I, R, C, mix);
    else if ((C.rows == 3 || C.quad_allow) && C.quad_allow == 4)
        hipLaunchKernelGGL(qap_sweep_kernel<6>, dim3(blocks), dim3(kBlockThreads), lds, s, I, R, C, mix);
    else if (C.rows == 3 || C.quad_allow)
        hipLaunchKernelGGL(qap_sweep_kernel<2>, dim3(blocks), dim3(kBlockThreads), lds, s, I, R, C, mix);
    else
        hipLaunchKernelGGL(qap_sweep_kernel<0>, dim3(blocks), dim3(kBlockThreads), lds, s, I, R, C, mix);
    return hipGetLastError();
}

hipError_t qap_launch_sweep_batch(const QapJob *jobs, const int2 *items, int n_items, size_t lds, int grid,
                                  hipStream_t s) {
    // once per process (thread-safe initialization)
    static const hipError_t attr = hipFuncSetAttribute((const void *)qap_sweep_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)kLdsBytes);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL(qap_sweep_batch_kernel, dim3(grid), dim3(kBlockThreads), lds, s, jobs, items, n_items);
    return hipGetLastError();
}

int qap_batch_occupancy(size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)qap_sweep_batch_kernel, kBlockThreads, lds) !=
        hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

hipError_t qap_launch_backbone_batch(const QapJob *jobs, const int2 *items, int n_items, int thr_num, int thr_den,
                                     hipStream_t s) {
    hipLaunchKernelGGL(qap_backbone_batch_kernel, dim3(n_items), dim3(256), 0, s, jobs, items, thr_num, thr_den);
    return hipGetLastError();
}

hipError_t qap_launch_backbone(const QapDev &I, const QapRepDev &R, int thr_num, int thr_den, hipStream_t s) {
    hipLaunchKernelGGL(qap_backbone_kernel, dim3(I.n), dim3(256), 0, s, I, R, thr_num, thr_den);
    return hipGetLastError();
}

hipError_t qap_launch_tally(const QapRepDev &R, hipStream_t s) {
    hipLaunchKernelGGL(qap_tally_kernel, dim3(1), dim3(1024), 0, s, R);
    return hipGetLastError();
}

}  // namespace nmc
