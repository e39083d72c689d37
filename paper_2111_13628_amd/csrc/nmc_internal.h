// Internal definitions shared by the host side of the library (nmc_api.cpp)
// and the device kernels (nmc_ksat.hip, nmc_qap.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

struct nmc_replicas;

namespace nmc {

// Philox stream identifiers (fourth counter word).
constexpr uint32_t kStreamKsatSweep = 0;
constexpr uint32_t kStreamKsatInit = 1;
constexpr uint32_t kStreamQapSweep = 2;
constexpr uint32_t kStreamQapInit = 3;
constexpr uint32_t kStreamPtSwap = 4;
constexpr uint32_t kStreamCflip = 5;

// k-SAT: replicas are handled in groups of 4; group g holds replicas
// 4g..4g+3 as bits 0..3 of one byte per variable.
constexpr int kGroup = 4;
// Largest variable count: spin-table byte addresses use 17 bits and the
// "always false" / "always true" entries sit at 2N and 2N+1.
constexpr int kMaxVars = 65534;
// Instances above kMaxVars (or loaded with NMC_KSAT_WIDE=1) take the wide
// layout: spins in device memory, variable-major with one byte per group of
// 4 replicas and 64 groups per wave (one lane per group).  Literal rows are
// 31-bit indices, so the wide layout reaches 2^24 variables.
constexpr int kMaxWideVars = (1 << 24) - 2;
// Wide sweeps: variables of a colour class are dealt to kWideStreams
// (workgroup, wave) streams; each stream keeps its replicas' energy changes
// for the sweep in its own slots.
constexpr int kWideWaves = 4;
constexpr int kWideSlices = 1024;
constexpr int kWideStreams = kWideSlices * kWideWaves;
constexpr int kWideGroup = 8;  // clause slots whose records and rows a wide sweep reads at once
constexpr int kAddrBits = 17;
constexpr uint32_t kAddrMask = (1u << kAddrBits) - 1;
constexpr int kMaxClasses = 8;
constexpr int kChunk = 64;  // variables per sweep chunk = lanes of one wave
constexpr int kSlotUnroll = 4;  // clause slots per chunk are padded to a multiple of this
// A chunk's info word y holds its slot count in bits 0..15 and lg in bits
// 16..: each variable occupies 2^lg adjacent lanes (lg <= kMaxSplitLog), the
// first of which (lane % 2^lg == 0) takes the decision.
constexpr int kSplitShift = 16;
constexpr int kMaxSplitLog = 4;

// LDS available to one workgroup on gfx950.
constexpr size_t kLdsBytes = 160 * 1024;

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Device view of a bound k-SAT instance.
struct KsatDev {
    const uint64_t *rec;         // chunk records, [slot-row][64 lanes]
    const int32_t *chunk_var;    // [n_chunks][64] lane word: variable | negated-count << 20, -1 = empty
    const int2 *chunk_info;      // [n_chunks] (first slot-row, slot count | lg << kSplitShift)
    const int32_t *color_chunk;  // [n_colors + 1] chunk range of each colour class
    const uint32_t *clause_addr; // [M][4] spin-table addresses of the clause's literals
    const int32_t *var_ptr;      // [N + 1] variable -> clause incidence
    const int32_t *var_cl;       // [sum deg]
    const uint32_t *lbp_caddr;   // [M][4] clause_addr in the LBP clause order (clauses by smallest variable)
    const int32_t *lbp_pos;      // [M] position of each clause in the LBP clause order
    int32_t n, m, n_colors, n_chunks, dmax;
    uint32_t rec_bytes;          // size of rec in bytes (the bound of the sweep's buffer loads)
    // wide layout (wide != 0; rec and the chunk arrays are then empty)
    const uint4 *wrec;           // [sum deg] per incidence in var_ptr order: the clause's other three
                                 // literals as row | negated << 31 (row N: absent, never true), own sign
    const int32_t *worder;       // [N] sweep order (colour-major)
    const int32_t *wclass_ptr;   // [n_colors + 1] range of each colour class in worder
    int32_t wide;
};

// Buffer resource word 3 (format and type bits) for raw byte-addressed
// buffer loads on gfx9-family GPUs.
constexpr int kBufferWord3 = 0x00020000;

// Device view of a k-SAT replica set.
struct KsatRepDev {
    uint8_t *xs;       // [G][N] current spins, group-major nibbles
    uint8_t *best_xs;  // [G][N] best-state snapshot
    int32_t *energy;   // [4G]
    int32_t *best;     // [4G]
    int32_t *first_hit;// [4G]
    uint8_t *cls;      // [N] backbone classes (device profile)
    int32_t *counts;   // [N] replicas with x_i = 1
    uint8_t *frozen;   // [N]
    int32_t *tally;    // [4] scratch for per-set reductions
    unsigned long long *accepted;  // [1] moves accepted by the sweep kernels (reset by the host)
    int32_t n_rep, n_groups;
    // wide layout: variable-major spin bytes [2 (N + 1)][wgp] (rows 0..N the
    // spins, row N all zero; rows N+1..2N+1 their complements, wnx = wx +
    // (N + 1) wgp), the best states [N][wgp]; wgp = 2^wlg >= 64 bytes per row
    // (the groups, padded); per-stream energy changes [wgp][kWideStreams][4];
    // per-group masks of the replicas whose best improved in the last sweep
    uint8_t *wx, *wnx, *wbx;
    int32_t *wdsum;
    uint8_t *wflag;
    int32_t wgp, wlg;
};

struct SweepCall {
    const uint32_t *tab;    // [n_sweeps][n_classes][stride] thresholds
    const uint8_t *var_cls; // per-variable class or nullptr
    int32_t n_classes, stride, n_sweeps;
    int32_t sweep_words;    // words between consecutive sweeps' tables (0: one table for all)
    uint32_t t0;
    int32_t target;
    int32_t check_start;
    uint32_t key0, key1;
    int32_t reps_per_row;   // > 0: replica r reads table row r / reps_per_row (one [n_classes][stride] block per row)
    int32_t gpw;            // groups of 4 replicas per workgroup: 1, or 2 (8 replicas share each spin byte in LDS)
};

// QAP: permutations as bytes, pair ranks in lexicographic order.
constexpr int kQapMaxN = 255;
constexpr int kQapRepPerBlock = 16;   // one replica per wave, 16 waves per workgroup
constexpr int kQapLowBits = 10;       // low digit of the two-level threshold

// Per-replica costs, accepted swaps and width choices the 16 waves of a QAP
// sweep workgroup exchange (four-replicas-per-wave sweeps).
constexpr size_t kQapQuadBytes = 256;
// LDS of the QAP sweep workgroup: flow rows in the 16-lane layout (and the
// 8-lane layout for n <= 112), distances, 16 permutations, classes,
// n_slots * n_classes threshold rows of `stride` words and the exchange
// area of the four-replicas-per-wave sweeps; then, when it fits,
// the table mode's pair list (2 bytes per pair) and per-wave update vectors
// (4 bytes per facility).
__host__ __device__ inline int qap_flow_row(int n) { return n <= 64 ? 64 : n <= 112 ? 128 : 256; }
__host__ __device__ inline size_t qap_base_lds(int n, int rows, int stride) {
    const size_t nn = (size_t)n * n;
    return align_up((size_t)n * qap_flow_row(n), 16) + (n <= 112 ? align_up((size_t)n * 128, 16) : 0) +
           align_up(nn, 16) + kQapRepPerBlock * align_up(n, 4) + align_up(n, 16) +
           align_up((size_t)rows * stride * sizeof(uint32_t), 16) + kQapQuadBytes;
}
__host__ __device__ inline size_t qap_tab_lds(int n) {
    return align_up((size_t)n * (n - 1), 16) + kQapRepPerBlock * align_up((size_t)n * 4, 16);
}
__host__ __device__ inline bool qap_tab_fits(int n, int rows, int stride) {
    return qap_base_lds(n, rows, stride) + qap_tab_lds(n) <= kLdsBytes;
}

struct QapDev {
    const uint8_t *F;  // [n][n]
    const uint8_t *D;  // [n][n]
    int32_t n;
    int32_t ha;        // entries of the high-digit threshold table
};

struct QapRepDev {
    int32_t *dtab;      // [R][n(n-1)/2] swap cost changes of every pair (table mode; rebuilt per launch)
    uint8_t *perm;      // [R][n]
    uint8_t *best_perm; // [R][n]
    int64_t *cost;      // [R]
    int64_t *best;      // [R]
    int32_t *first_hit; // [R]
    uint8_t *cls;       // [n]
    int32_t *freq;      // [n][n]
    int32_t *tally;     // scratch
    unsigned long long *accepted;  // [1] swaps accepted by the sweep kernels (reset by the host)
    uint8_t *rows_hint; // [R] proposals per step the replica's last sweep chose (0: none yet)
    int32_t n_rep;
};

struct QapCall {
    const uint32_t *tab;   // [n_sweeps][n_classes][ha + 1024 + 1]: A, B, then 1 / beta as a float
    const uint8_t *fac_cls;// per-facility class or nullptr
    int32_t n_classes, stride, n_sweeps;
    int32_t sweep_words;   // words between consecutive sweeps' tables (0: one table for all)
    uint32_t t0;
    int64_t target;
    int32_t check_start;
    uint32_t key0, key1;
    int32_t rows;          // proposals per step: 0 = chosen per sweep, else 1, 4 or 8; 2 = table mode
    int32_t tab_allow;     // the per-sweep choice may use the table mode (when its LDS fits)
    int32_t quad_allow;    // the per-sweep choice may run several replicas per wave: 0 no, 2 or 4 per wave
    int32_t reps_per_row;  // > 0: replica r reads table row r / reps_per_row (one [n_classes][stride] block per row)
    int32_t dstar;         // every row's T(d) never increases: decide by the bound d*(u) (else read T per proposal)
};

// One replica set of a batched launch.
struct KsatJob {
    KsatDev I;
    KsatRepDev R;
    SweepCall C;
};

struct QapJob {
    QapDev I;
    QapRepDev R;
    QapCall C;
};

// Per-set status after a batched step: lowest best energy, replicas whose
// best is 0, earliest first-hit sweep (-1 if none).
struct SetStatusSrc {
    const void *best;       // int32 (k-SAT) or int64 (QAP) per replica
    const int32_t *first_hit;
    int32_t n_rep;
    int32_t best_is_64;
};
struct SetStatus {
    long long best;
    int32_t n_zero;
    int32_t first_hit;
};
hipError_t launch_set_status(const SetStatusSrc *src, SetStatus *out, int n_sets, hipStream_t s);

// ---- launchers (nmc_ksat.hip) ----
size_t ksat_sweep_lds_bytes(int n, int n_classes, int stride);
hipError_t ksat_launch_init(const KsatDev &I, const KsatRepDev &R, uint32_t key0, uint32_t key1, hipStream_t s);
hipError_t ksat_launch_wide_pack(const KsatDev &I, const KsatRepDev &R, bool unpack, hipStream_t s);
// energies of every replica of a wide instance from its group-major state
// (packs the variable-major tables first)
hipError_t ksat_launch_wide_recount(const KsatDev &I, const KsatRepDev &R, int32_t *energy_out, hipStream_t s);
hipError_t ksat_launch_wide_sweeps(const KsatDev &I, const KsatRepDev &R, const SweepCall &C,
                                   const int32_t *class_size /* host, per colour */, hipStream_t s);
hipError_t ksat_launch_recount(const KsatDev &I, const uint8_t *xs, int n_groups, int n_rep, int32_t *energy_out,
                               hipStream_t s);
hipError_t ksat_launch_reset_tallies(const KsatRepDev &R, int n, hipStream_t s);
hipError_t ksat_launch_sweep(const KsatDev &I, const KsatRepDev &R, const SweepCall &C, int block_threads,
                             hipStream_t s);
hipError_t ksat_launch_backbone(const KsatDev &I, const KsatRepDev &R, int thr_num, int thr_den, int expand,
                                hipStream_t s);
hipError_t ksat_launch_tally(const KsatRepDev &R, hipStream_t s);
hipError_t ksat_launch_sweep_batch(const KsatJob *jobs, const int2 *items, int n_items, size_t lds, int block_threads,
                                   int grid, hipStream_t s);
int ksat_batch_occupancy(int block_threads, size_t lds);
hipError_t ksat_launch_backbone_batch(const KsatJob *jobs, const int2 *items, int n_items, int thr_num, int thr_den,
                                      int expand, hipStream_t s);
hipError_t ksat_launch_unpack(const uint8_t *xs, int n, int n_groups, int n_rep, uint8_t *x_rows, hipStream_t s);
hipError_t ksat_launch_pack(const uint8_t *x_rows, int n, int n_groups, int n_rep, uint8_t *xs, hipStream_t s);

// ---- launchers (nmc_qap.hip) ----
size_t qap_sweep_lds_bytes(int n, int n_classes, int stride);
hipError_t qap_launch_init(const QapDev &I, const QapRepDev &R, uint32_t key0, uint32_t key1, hipStream_t s);
hipError_t qap_launch_cost(const QapDev &I, const uint8_t *perm, int n_rep, int64_t *cost_out, hipStream_t s);
hipError_t qap_launch_reset_tallies(const QapRepDev &R, int n, hipStream_t s);
hipError_t qap_launch_sweep(const QapDev &I, const QapRepDev &R, const QapCall &C, int block_threads, hipStream_t s);
hipError_t qap_launch_backbone(const QapDev &I, const QapRepDev &R, int thr_num, int thr_den, hipStream_t s);
hipError_t qap_launch_tally(const QapRepDev &R, hipStream_t s);
hipError_t qap_launch_sweep_batch(const QapJob *jobs, const int2 *items, int n_items, size_t lds, int grid,
                                  hipStream_t s);
int qap_batch_occupancy(size_t lds);
hipError_t qap_launch_backbone_batch(const QapJob *jobs, const int2 *items, int n_items, int thr_num, int thr_den,
                                     hipStream_t s);

// ---- parallel tempering (nmc_pt.hip) ----
// Replicas are temperature-major: replica r = i * n_chains + c is ladder
// position i of chain c.  Exchange thresholds of neighbour pair i are the
// factored form (A_i[d >> 10] * B_i[d & 1023]) >> 32 with A_i = tab + off[i]
// holding len[i] high-digit entries (entries past len[i] are zero) and B_i
// the 1024 words after them.
struct PtCall {
    const uint32_t *tab;
    const int64_t *off;     // [n_temps - 1] word offsets of A_i
    const int32_t *len;     // [n_temps - 1]
    unsigned long long *accepted, *attempted;  // [n_temps - 1]
    int32_t n_temps, n_chains, parity;
    uint32_t t;             // sweeps done when the exchange is taken
    uint32_t key0, key1;
};
hipError_t pt_launch_exchange_ksat(const KsatDev &I, const KsatRepDev &R, const PtCall &C, hipStream_t s);
hipError_t pt_launch_exchange_qap(const QapDev &I, const QapRepDev &R, const PtCall &C, hipStream_t s);
// acc[0..3] += (count, sum E, low and high words of sum E^2) over energies
// [n] (non-negative, below 2^32), exactly
hipError_t pt_launch_moments(const void *energy, int energy_is_64, int n, unsigned long long *acc, hipStream_t s);

// ---- surrogate-Hamiltonian LBP and backbone growth (nmc_lbp.hip) ----
// Edges e = 4a + j (literal j of clause a); padded edges are never read.
struct LbpWork {
    double *u;                   // [4M] clause-to-variable messages, clause-major (edge e = 4a + j)
    double *uv;                  // [sum deg] sigma_ia u_{a->i}, variable-major (incidence order); u + 4M
    double *T;                   // [N] field totals H_i + sum_a sigma_ia u_{a->i}
    double *mag, *corr;          // [N] <r_i>, [M] clause moments
    int32_t *epos;               // [4M] variable-major position of each edge (padding slots unused)
    int8_t *s;                   // [N] reference spins (+1 / -1)
    unsigned long long *scal;    // [2][64] bits of the largest |du| of an iteration, by parity and slot
    double *res;                 // [0] overlap p, [1] self-overlap q1, [2] last iteration's max |du|
    int32_t *ctl;                // [0] 0 running / 1 converged / 2 out of iterations, [1] iterations
    int32_t *label, *out_label, *size;  // [N]
    uint8_t *seeded;             // [N]
    int32_t *flag;               // [1] labels changed
    int32_t *counts;             // [5] backbone size, clusters, largest, rigid clauses, seed clauses
};
// one LBP run: its instance, workspace, seed row and class output
struct LbpJob {
    KsatDev I;
    LbpWork W;
    const uint8_t *xs_row;  // the seed replica's group row of spins
    int32_t bit;            // the seed replica's bit in it
    uint8_t *cls;           // [N] class output (1 = backbone)
};
struct LbpDims {
    int n_jobs, max_n, max_m;
};
constexpr int kLbpDeltaSlots = 64;
// convergence decision on iteration iters - 1 of a step, whose largest |du|
// is in slot set `judge` (-1: none); `clear` (-1: none) is the set the next
// clause pass fills
struct LbpJudge {
    int judge, clear, iters, max_iter;
    double tol;
};
hipError_t lbp_launch_setup(const LbpJob *jobs, const LbpDims &D, double lambda0, hipStream_t s);
hipError_t lbp_launch_var(const LbpJob *jobs, const LbpDims &D, double lambda, int final_pass, hipStream_t s);
hipError_t lbp_launch_clause(const LbpJob *jobs, const LbpDims &D, double w, int final_pass, hipStream_t s);
// gated iterations first .. first + count - 1 of one step (variable side with
// the previous iteration's control, clause side; control after the last)
hipError_t lbp_launch_iterations(const LbpJob *jobs, const LbpDims &D, double lambda, double w, double tol,
                                 int max_iter, int first, int count, hipStream_t s);
hipError_t lbp_launch_overlap(const LbpJob *jobs, const LbpDims &D, hipStream_t s);
hipError_t lbp_launch_label_init(const LbpJob *jobs, const LbpDims &D, hipStream_t s);
hipError_t lbp_launch_hook_jump(const LbpJob *jobs, const LbpDims &D, double cut, hipStream_t s);
hipError_t lbp_launch_finish(const LbpJob *jobs, const LbpDims &D, double seed_thr, double cut, hipStream_t s);

// ---- whitening (nmc_whiten.hip) ----
size_t ksat_whiten_lds_bytes(int n);
// white bits per (group, variable) into white_out [G][N], frozen count per
// replica into frozen_out [R], passes of the slowest group (atomic max) into
// *passes_out (zero it first)
hipError_t ksat_launch_whiten(const KsatDev &I, const uint8_t *xs, int n_groups, int n_rep, uint8_t *white_out,
                              int32_t *frozen_out, int32_t *passes_out, hipStream_t s);

// ---- collective cluster flips (nmc_cflip.hip) ----
struct CflipCall {
    const int32_t *cl_ptr;    // [n_clusters + 1] clause-list range of each cluster
    const uint32_t *cl_list;  // clause | (mask of its literal positions inside the cluster) << 28
    const int32_t *v_ptr;     // [n_clusters + 1] variable-list range of each cluster
    const int32_t *v_list;    // the cluster's variables
    const uint32_t *thr;      // [thr_len + 1] thresholds T(beta, d); zero for d > thr_len
    int32_t *accepted;        // [R] clusters flipped per replica
    int32_t n_clusters, thr_len;
    uint32_t t;               // sweep counter of the move
    int32_t target;
    uint32_t key0, key1;
};
size_t ksat_cflip_lds_bytes(int n);
hipError_t ksat_launch_cflip(const KsatDev &I, const KsatRepDev &R, const CflipCall &C, hipStream_t s);

// records msg as the calling thread's nmc_last_error text; returns code
int set_last_error(int code, const char *msg);

// nmc_anneal with the call's threshold tables (and host class array) uploaded
// to buf (device memory, cap bytes) instead of the replica set's own upload
// buffer: allocates nothing; NMC_ERR_CAPACITY when the call needs more than
// cap bytes (checked before any work is queued).  No timing events.
int anneal_into(nmc_replicas *P, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
                const uint8_t *class_of, int64_t target, void *stream, uint8_t *buf, size_t cap);

}  // namespace nmc
