/*
 * nmc.h -- C ABI of the MI355X (gfx950) Nonequilibrium Monte Carlo hot path.
 *
 * Paper: "Nonequilibrium Monte Carlo for unfreezing variables in hard
 * combinatorial optimization" (arXiv 2111.13628).  The library runs many
 * independent replicas of single-variable (k-SAT) or pairwise-swap (QAP)
 * Metropolis Markov chains on the GPU, with one inverse temperature per
 * variable class; estimates frozen ("backbone") variables from statistics
 * across replicas; turns them into a two-class temperature profile; and
 * re-anneals from the current states (Algorithm 1 "Nonequilibrium Monte
 * Carlo", section "Nonequilibrium inhomogeneous sampling over subgraphs",
 * appendix B "Sampling localized replicas by Monte Carlo").  The other steps
 * of Algorithm 1 are here as well: adaptive parallel tempering (appendix A),
 * the backbone estimate by loopy belief propagation on the localized
 * surrogate Hamiltonian with connected cluster growth (the sections on
 * surrogate Hamiltonians, LBP and backbones; appendix C), collective flips of
 * backbone clusters, and the whitening diagnostic of low-energy states.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an int status: NMC_OK (0) or a negative NMC_ERR_*
 *    code; nmc_last_error() then returns a message for the calling thread.
 *    No C++ exception crosses the ABI.
 *  - Host arrays passed in are read during the call only (the library copies
 *    what it keeps).  Host arrays passed out are written before the call
 *    returns; such calls synchronize the given stream.
 *  - Device memory for instances and replica sets is owned by the caller:
 *    nmc_footprint() gives the byte sizes, the caller allocates (e.g. torch
 *    tensors on cuda:0) and passes raw device pointers.  The library never
 *    frees caller memory.  The library owns only working buffers it sizes
 *    itself: per replica set, an upload buffer for threshold tables and
 *    tempering / cluster-flip lists, and (on first use) the tempering moment
 *    accumulators, the LBP workspace with a small pinned host buffer, and the
 *    whitening workspace, all released by nmc_replicas_free; a per-batch
 *    descriptor and table buffer (released by nmc_batch_free); and, for a
 *    server, the device memory of the requests it admits (released when a
 *    request retires or by nmc_server_free).  nmc_anneal_noalloc uses a fixed
 *    device array of the library instead (one per device, never freed).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it in call order; calls on one replica set must not overlap in time.
 *  - Energies are exact integers: the k-SAT energy is the number of violated
 *    clauses, the QAP cost is sum_ij F_ij D_{p_i p_j} (int64 at the ABI).
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = the
 *    replica set's 64-bit seed (low word first) and counter = (item, sweep,
 *    replica / 4, stream); replica r uses output word r mod 4.  Streams:
 *    0 k-SAT sweep (item = variable), 1 k-SAT init (item = variable, sweep 0),
 *    2 QAP sweep (item = pair rank), 3 QAP init (item = Fisher-Yates step),
 *    4 tempering exchange (counter (chain, sweep, ladder position, 4), word 0),
 *    5 cluster flip (item = cluster ordinal).
 *    Results are a deterministic function of (instance, seed, schedule,
 *    profile, call sequence): no result depends on tuning, launch shape or on
 *    other work sharing the GPU.
 */
#ifndef NMC_H
#define NMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum nmc_status {
    NMC_OK = 0,
    NMC_ERR_INVALID = -1,     /* malformed argument (bad literal, NULL pointer, bad range) */
    NMC_ERR_SIZE = -2,        /* a buffer is smaller than required */
    NMC_ERR_DEVICE = -3,      /* a HIP runtime call failed */
    NMC_ERR_STATE = -4,       /* call not valid in the object's current state */
    NMC_ERR_CAPACITY = -5,    /* does not fit (LDS or configured memory cap) */
    NMC_ERR_UNSUPPORTED = -6  /* valid input outside what the library supports */
};

enum nmc_kind { NMC_KIND_KSAT = 1, NMC_KIND_QAP = 2 };

/* Where nmc_anneal takes the class of each variable (k-SAT) or facility (QAP). */
enum nmc_profile {
    NMC_PROFILE_HOMOGENEOUS = 0, /* every item in class 0 (plain simulated annealing) */
    NMC_PROFILE_HOST = 1,        /* class_of[] host array, values < n_classes */
    NMC_PROFILE_BACKBONE = 2     /* the classes of the last nmc_estimate_backbone() */
};

/* Which state nmc_get_state() returns. */
enum nmc_which { NMC_STATE_CURRENT = 0, NMC_STATE_BEST = 1 };

typedef struct nmc_instance nmc_instance;
typedef struct nmc_replicas nmc_replicas;

typedef struct nmc_instance_info {
    int32_t kind;            /* NMC_KIND_* */
    int32_t n_items;         /* k-SAT: variables N; QAP: facilities n */
    int32_t n_clauses;       /* k-SAT: clauses M; QAP: 0 */
    int32_t max_clause_len;  /* k-SAT: k_max; QAP: 0 */
    int32_t max_degree;      /* k-SAT: most clauses on one variable; QAP: n-2 */
    int32_t n_colors;        /* k-SAT: sweep classes of the colouring; QAP: 1 */
    int64_t delta_bound;     /* largest |energy change| of one move */
    int32_t wide;            /* k-SAT: 1 = wide layout (see nmc_ksat_load), 0 = LDS layout; QAP: 0 */
} nmc_instance_info;

/* Message of the last failing call on this thread ("" if none). */
const char *nmc_last_error(void);
/* ABI version (major * 100 + minor). */
int32_t nmc_version(void);

/* ---------------------------------------------------------------------------
 * load_instance
 * ------------------------------------------------------------------------- */

/* Load a CNF formula (subsection "4-SAT Problems Near Computational Phase
 * Transitions": k-SAT as a conjunction of clauses, each a disjunction of
 * literals; energy = number of violated clauses).
 *   n_vars      1 <= N <= 2^24 - 2 variables.  Up to 65534 the sweeps keep
 *               each group of 4 replicas' spin tables in LDS; above that (or
 *               with the environment variable NMC_KSAT_WIDE=1 at load) the
 *               instance takes the wide layout: spins in device memory,
 *               variable-major, one lane per group of 4 replicas, one
 *               launch per colour class (same results bit for bit).  Wide
 *               instances support load, replicas, anneal / reanneal (also
 *               allocation-free), backbone, best energy, recount and state
 *               calls; tempering, LBP, whitening, cluster flips, batched
 *               launches and served requests return UNSUPPORTED for them.
 *   n_clauses   M >= 0
 *   clause_ptr  M+1 offsets into lits, non-decreasing, clause_ptr[0] = 0
 *   lits        DIMACS literals: +(v+1) means x_v, -(v+1) means NOT x_v;
 *               1 <= clause length <= 4, variables distinct within a clause
 *   class_cap   0 = plain greedy colouring; > 0 caps each colour class at
 *               that many variables.  The sweep order is the colour-major
 *               order of this colouring (see nmc_instance_order).
 * Errors: INVALID (literal 0 or out of range, repeated variable, empty
 * clause, bad offsets), UNSUPPORTED (clause longer than 4, N > 2^24 - 2,
 * a variable in more than 127 clauses). */
int nmc_ksat_load(int32_t n_vars, int32_t n_clauses, const int32_t *clause_ptr, const int32_t *lits,
                  int32_t class_cap, nmc_instance **out);

/* Load a QAP instance (subsection "Quadratic Assignment Problems"):
 * facilities f are assigned locations p_f, cost sum_ij F_ij D_{p_i p_j}.
 *   n           2 <= n <= 255
 *   flow, dist  n*n row-major int32, symmetric, zero diagonal, entries in
 *               [0, 255] (the device kernels use the symmetric swap formula
 *               and byte-packed matrices)
 * Errors: INVALID (asymmetric, nonzero diagonal), UNSUPPORTED (n or an entry
 * out of range). */
int nmc_qap_load(int32_t n, const int32_t *flow, const int32_t *dist, nmc_instance **out);

int nmc_instance_get_info(const nmc_instance *inst, nmc_instance_info *out);

/* The k-SAT sweep order: order[p] = variable visited at position p (N
 * entries); class_ptr[c]..class_ptr[c+1] delimit colour class c (n_colors+1
 * entries).  Either output may be NULL.  No two variables of one class share
 * a clause, so the device updates a class in parallel with results identical
 * to visiting it in this order.  QAP: UNSUPPORTED. */
int nmc_instance_order(const nmc_instance *inst, int32_t *order, int32_t *class_ptr, int32_t *n_colors);

/* Device bytes the instance needs (bind buffer) and that a replica set of
 * n_replicas needs (replicas_create buffer). */
int nmc_footprint(const nmc_instance *inst, int32_t n_replicas, size_t *instance_bytes, size_t *replica_bytes);

/* Upload the instance's device layout into caller memory dev_buf (>= the
 * footprint's instance_bytes, 256-byte aligned).  Must precede
 * nmc_replicas_create.  Errors: SIZE, INVALID (misaligned), DEVICE. */
int nmc_instance_bind(nmc_instance *inst, void *dev_buf, size_t bytes, void *stream);

/* Releases the caller's handle.  The host-side metadata is freed when the
 * handle and every replica set created from the instance have been released,
 * in any order (each replica set holds a reference; nmc_replicas_free drops
 * it).  The instance's device buffer (caller memory) must stay valid while
 * any of its replica sets runs work. */
void nmc_instance_free(nmc_instance *inst);

/* ---------------------------------------------------------------------------
 * replicas
 * ------------------------------------------------------------------------- */

/* Create n_replicas independent chains in dev_buf (>= replica_bytes, 256-byte
 * aligned).  k-SAT: x_i of replica r is the top bit of its init word for
 * item i; QAP: Fisher-Yates from the identity with its init words.  Energies
 * are counted in full; best = energy; first_hit = -1; sweeps_done = 0.
 * 1 <= n_replicas <= 2^20. */
int nmc_replicas_create(nmc_instance *inst, int32_t n_replicas, uint64_t seed, void *dev_buf, size_t bytes,
                        void *stream, nmc_replicas **out);
void nmc_replicas_free(nmc_replicas *rep);

/* ---------------------------------------------------------------------------
 * anneal / reanneal
 * ------------------------------------------------------------------------- */

/* Run n_sweeps Metropolis sweeps on every replica (section "Nonequilibrium
 * Nonlocal Monte Carlo": simulated annealing when the profile is
 * homogeneous; section "Nonequilibrium inhomogeneous sampling over
 * subgraphs" when classes differ).
 *   beta[c * n_sweeps + s]  inverse temperature of class c at sweep s of this
 *                           call (host doubles, finite, >= 0)
 *   n_classes               1..8 rows in beta
 *   profile, class_of       see nmc_profile; class_of is N (k-SAT) or n (QAP)
 *                           bytes, used only with NMC_PROFILE_HOST
 *   target                  first_hit[r] records the first sweep boundary
 *                           (number of sweeps done) at which replica r's
 *                           energy is <= target, checked at this call's start
 *                           and after each sweep; -1 until hit
 * One sweep: k-SAT visits the variables in nmc_instance_order; QAP proposes
 * every pair (a < b) in lexicographic order.  A move with energy change
 * d <= 0 is taken; otherwise the replica's sweep word u is compared with
 * T = min(2^32-1, floor(2^32 exp(-beta d))) (QAP: the two-level product
 * (A[d>>10] * B[d&1023]) >> 32 of such thresholds) and the move is taken iff
 * u < T.  The thresholds are computed on the host in IEEE double.  Energies
 * are tracked exactly; best energy and the best-state snapshot are updated at
 * sweep boundaries.  The sweep counter continues across calls, so splitting a
 * schedule over several calls gives identical results.
 * Errors: INVALID, STATE (unbound instance; BACKBONE profile without an
 * estimate), CAPACITY, DEVICE. */
int nmc_anneal(nmc_replicas *rep, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
               const uint8_t *class_of, int64_t target, void *stream);

/* The reanneal round of Algorithm 1 (inhomogeneous exploration followed by
 * homogeneous "unlearning"): identical to nmc_anneal, continuing from the
 * current states and sweep counter; kept as its own name for the API. */
int nmc_reanneal(nmc_replicas *rep, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
                 const uint8_t *class_of, int64_t target, void *stream);

/* Allocation-free nmc_anneal, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops that must not call the
 * allocator).  Arguments, results and errors are those of nmc_anneal, with
 * the same bits: the same kernels run, and only the place of the call's
 * threshold tables differs.  The tables (4 bytes per table word: sweeps x
 * classes x (max degree + 1) for k-SAT, x (high-digit entries + 1025) for
 * QAP, rounded up to 256 bytes, plus N or n bytes of class_of for
 * NMC_PROFILE_HOST, rounded up to 256) are uploaded into a fixed device array
 * of the library (nmc_anneal_noalloc_capacity() bytes, one per device, held
 * until the process ends) instead of the replica set's upload buffer; a call
 * that needs more fails with NMC_ERR_CAPACITY before anything runs (split the
 * schedule into shorter calls: the sweep counter continues).  The call makes
 * no hipMalloc or hipFree and creates no events (nmc_set_profiling does not
 * apply to it).  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other streams, other threads) race on it and
 * must be serialized by the caller; calls in order on one stream are safe.
 * Each call writes every byte of the array it reads, so no contents carry
 * over between calls.  The calling thread's current device must be the one
 * the replica set lives on. */
int nmc_anneal_noalloc(nmc_replicas *rep, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
                       const uint8_t *class_of, int64_t target, void *stream);
/* Bytes of the fixed device array nmc_anneal_noalloc uploads into. */
size_t nmc_anneal_noalloc_capacity(void);

/* ---------------------------------------------------------------------------
 * estimate_backbone
 * ------------------------------------------------------------------------- */

/* Backbone from the current states of all replicas (appendix B: empirical
 * averages over independent clones; section "Generating backbones of rigid
 * variables").
 * k-SAT: c_i = #{r : x_i = 1}; i is frozen iff thr_den * |2 c_i - R| >=
 *   thr_num * R (|magnetization| >= thr_num / thr_den, inclusive); with
 *   expand != 0 every variable sharing a clause with a frozen one is also hot.
 *   counts_out (optional) receives c_i (N int32).
 * QAP: freq[f][l] = #{r : p_f = l}; facility f is frozen (hot) iff
 *   thr_den * max_l freq[f][l] >= thr_num * R; expand is ignored.
 *   counts_out (optional) receives freq (n*n int32, row-major).
 * class_out (optional, N or n bytes) receives 1 = hot, 0 = cold.  The classes
 * stay on the device for NMC_PROFILE_BACKBONE.  0 < thr_num <= thr_den. */
int nmc_estimate_backbone(nmc_replicas *rep, int32_t thr_num, int32_t thr_den, int32_t expand, uint8_t *class_out,
                          int32_t *counts_out, void *stream);

/* ---------------------------------------------------------------------------
 * parallel tempering (appendix A, "Adaptive Parallel Tempering"; the
 * replica-exchange step that opens Algorithm 1)
 * ------------------------------------------------------------------------- */

/* n_rounds rounds of replica-exchange Monte Carlo.  The R replicas form
 * C = R / n_temps independent chains, laid out temperature-major: replica
 * r = i * C + c holds ladder position i of chain c and sweeps at beta[i].
 * C must be a multiple of 4 (k-SAT) or 16 (QAP), so that the replicas one
 * sweep workgroup owns share a temperature.
 *   beta[n_temps]     host doubles, finite, >= 0, strictly increasing (position
 *                     0 is the hottest)
 *   sweeps_per_round  >= 1 Metropolis sweeps of every replica at its own
 *                     temperature (the nmc_anneal rules, sweep counter
 *                     continuing), then one exchange step
 *   first_parity      the exchange step of round k offers the pairs
 *                     (i, i + 1), i = p, p + 2, ... with p = (first_parity + k)
 *                     mod 2, in every chain
 *   target            as nmc_anneal (first_hit of each replica slot)
 *   accepted, attempted  optional host arrays [n_temps - 1]: exchanges taken
 *                     and offered per pair position during this call
 * Exchange: the pair swaps its configurations (and their energies) with
 * probability min{1, exp[(beta_i - beta_{i+1})(E_i - E_{i+1})]}: always when
 * E_i <= E_{i+1}; otherwise iff u < T with u word 0 of the Philox block at
 * counter (c, sweeps done, i, 4) and T the two-level threshold of nmc_anneal
 * at beta_{i+1} - beta_i and gap E_i - E_{i+1}.  Best energies, best-state
 * snapshots and first-hit sweeps belong to replica slots (ladder positions)
 * and are updated at sweep boundaries only.  n_temps = 1 runs plain sweeps.
 * The exchange tables and counters live in the library-owned upload buffer.
 * Errors: INVALID (layout, ladder, counts), STATE (unbound), CAPACITY (LDS,
 * or a ladder step too fine for the energy range), DEVICE. */
int nmc_pt_run(nmc_replicas *rep, const double *beta, int32_t n_temps, int32_t n_rounds, int32_t sweeps_per_round,
               int32_t first_parity, int64_t target, int64_t *accepted, int64_t *attempted, void *stream);

/* Adaptive temperature ladder (appendix A).  Starting at beta_first, all
 * replicas run equil_sweeps sweeps at the current beta_i, then meas_sweeps
 * sweeps after each of which every replica's energy is sampled on the
 * device; sigma_i = sqrt(<E^2> - <E>^2) over those R * meas_sweeps samples,
 * evaluated as (n S2 - S1^2) / n^2 with exact integer sums and one rounding.
 * The next position is beta_i + alpha / sigma_i; the ladder ends at the first
 * sigma_i <= sigma_min, or after max_temps positions.  The replicas carry
 * their states from one temperature to the next (the sweep counter advances
 * by equil_sweeps + meas_sweeps per position).
 *   beta_out, sigma_out  host arrays of max_temps doubles; *n_temps receives
 *                        the positions written
 * alpha > 0 (about 1.1 per appendix A), sigma_min >= 0, meas_sweeps >= 1,
 * R * meas_sweeps <= 2^26.  Errors: INVALID, STATE, CAPACITY, DEVICE. */
int nmc_apt_ladder(nmc_replicas *rep, double beta_first, double alpha, double sigma_min, int32_t equil_sweeps,
                   int32_t meas_sweeps, int32_t max_temps, double *beta_out, double *sigma_out, int32_t *n_temps,
                   void *stream);

/* ---------------------------------------------------------------------------
 * surrogate-Hamiltonian backbone (section "Constructing localized surrogate
 * Hamiltonians"; section "Efficient sampling of localized surrogate
 * Hamiltonians via LBP" and its CNF form in subsection "4-SAT Problems Near
 * Computational Phase Transitions" and appendix C; section "Generating
 * backbones of rigid variables")
 * ------------------------------------------------------------------------- */

typedef struct nmc_lbp_config {
    double beta;          /* a violated clause weighs exp(-2 beta), a satisfied one 1 */
    double lambda0;       /* first (largest) localization strength, > 0 */
    double lambda_ratio;  /* lambda_{k+1} = lambda_k * ratio, in (0, 1) */
    double lambda_min;    /* no step below this lambda (the first step always runs) */
    int32_t max_iter;     /* message iterations per step, >= 1 */
    double tol;           /* a step has converged when max |du| of an iteration < tol */
    double p_min;         /* a step whose overlap p falls below this is discarded */
    double theta_seed;    /* seed clauses: |clause moment| >= theta_seed */
    double theta_cut;     /* rigid clauses: |clause moment| >= theta_cut (<= theta_seed) */
} nmc_lbp_config;

typedef struct nmc_lbp_result {
    double lambda;            /* lambda of the kept messages */
    int32_t steps;            /* lambda steps tried (the discarded one included) */
    int32_t iterations;       /* message iterations over all steps */
    int32_t converged;        /* 1 when the kept messages converged */
    double delta;             /* max |du| of the kept step's last iteration */
    double overlap;           /* p  = (1/N) sum_i s*_i <r_i> */
    double self_overlap;      /* q1 = (1/N) sum_i <r_i>^2 */
    int32_t backbone_size;    /* variables in the backbone (hot class) */
    int32_t n_clusters;
    int32_t largest_cluster;
    int32_t rigid_clauses;
    int32_t seed_clauses;
} nmc_lbp_result;

/* Backbone of rigid variables around the state s* of one replica (k-SAT
 * only): loopy belief propagation on the surrogate Hamiltonian
 * H(r) - lambda sum_i eps_i s*_i r_i over the CNF factor graph, then
 * connected clusters of strongly correlated clauses.
 *   replica, which    s*_i = 2 x_i - 1 of replica `replica`'s current or best
 *                     state (NMC_STATE_CURRENT / NMC_STATE_BEST)
 * Spins r_i = 2 x_i - 1; eps_i = number of clauses holding i; sigma_{ia} = +1
 * for a positive literal of i in clause a, -1 for a negated one.  Messages:
 *   h_{i->a} = sigma_{ia} lambda eps_i s*_i + sum_{b in di \ a} sigma_{ia} sigma_{ib} u_{b->i}
 *   u_{a->i} = -1/2 ln[1 - (1 - e^{-2 beta}) prod_{j in da \ i} (1 - tanh h_{j->a}) / 2]
 * updated all h, then all u, per iteration.  Adiabatic schedule: messages
 * start at h = sigma lambda0 eps s*, u from them; step k runs at
 * lambda0 * ratio^k (while >= lambda_min) until converged or max_iter; a step
 * that does not converge, or whose overlap p drops below p_min, is discarded
 * and the previous step's messages are kept.  From the kept messages:
 * <r_i> = tanh(lambda eps_i s*_i + sum_a sigma_{ia} u_{a->i}) and the clause
 * moment <prod_{i in a} r_i> under the clause measure
 * omega_a(r) prod_i (1 + sigma_{ia} r_i tanh h_{i->a}) / 2.  A clause is rigid
 * when |moment| >= theta_cut, a seed when |moment| >= theta_seed; the
 * backbone is every connected group of variables (joined by rigid clauses)
 * that holds a seed clause.  The backbone becomes the device class array
 * (1 = hot) used by NMC_PROFILE_BACKBONE, as after nmc_estimate_backbone.
 * Outputs (each optional, host): class_out [N] bytes, mag_out [N] doubles,
 * corr_out [M] doubles (signed clause moments), label_out [N] int32 (the
 * smallest variable index of the cluster, -1 outside the backbone).
 * Arithmetic is IEEE double.  The workspace (20 bytes per literal slot of
 * the padded 4-per-clause layout, 16 per literal, 8 per clause and about 35
 * per variable) is allocated on the first call and kept with the replica
 * set.
 * Errors: INVALID (arguments), STATE (unbound), UNSUPPORTED (QAP), DEVICE. */
int nmc_lbp_backbone(nmc_replicas *rep, int32_t replica, int32_t which, const nmc_lbp_config *cfg,
                     nmc_lbp_result *res, uint8_t *class_out, double *mag_out, double *corr_out, int32_t *label_out,
                     void *stream);

/* ---------------------------------------------------------------------------
 * whitening (section "Whitening procedure for low energy states")
 * ------------------------------------------------------------------------- */

/* Frozen variables of every replica's current or best state (k-SAT only).
 * A variable turns white unless some clause has the variable's literal as its
 * only true literal and no other white variable in it; a violated clause
 * pins nothing (the section's extension to states that are not solutions).
 * Repeated until nothing changes; the remaining variables are frozen (for a
 * solution, a lower bound on the variables frozen across its cluster).
 *   which       NMC_STATE_CURRENT or NMC_STATE_BEST
 *   frozen_out  host int32 [R]: frozen variables per replica
 *   white_out   optional host bytes [R][N]: 1 = white, 0 = frozen
 *   passes      optional: passes over the variables of the slowest group of
 *               4 replicas (the last pass changes nothing)
 * The result does not depend on the inspection order.  The device workspace
 * (N bytes per 4 replicas) is allocated on the first call and kept with the
 * replica set.  Errors: INVALID, STATE, UNSUPPORTED (QAP), DEVICE. */
int nmc_whiten(nmc_replicas *rep, int32_t which, int32_t *frozen_out, uint8_t *white_out, int32_t *passes,
               void *stream);

/* ---------------------------------------------------------------------------
 * collective cluster flips (the nonlocal move of the NMC scheme: a whole
 * backbone cluster flipped at once; the section on annealed thresholds names
 * it as the alternative to heating the backbone)
 * ------------------------------------------------------------------------- */

/* One collective-move sweep of every replica (k-SAT only).
 *   label    host int32 [N]: -1, or the cluster of variable i named by a
 *            variable that labels itself (label[label[i]] == label[i]); the
 *            label_out of nmc_lbp_backbone has this form
 *   beta     inverse temperature of the acceptance, finite, >= 0
 * The clusters are proposed in increasing label order; proposal k flips every
 * variable of the k-th cluster at once.  With dE the exact energy change, the
 * flip is taken when dE <= 0, else when the replica's word of the Philox
 * block at counter (k, sweeps done, replica / 4, 5) is below
 * T = min(2^32-1, floor(2^32 exp(-beta dE))).  The call counts as one sweep:
 * the sweep counter advances by 1, and best energies, best-state snapshots
 * and first hits (against target) are updated at its end.  accepted_out
 * (optional, host int32 [R]) receives the clusters flipped per replica.  The
 * cluster lists are built on the host and uploaded to the library-owned
 * buffer.  Errors: INVALID (labels, beta), STATE, UNSUPPORTED (QAP),
 * CAPACITY, DEVICE. */
int nmc_cluster_flip(nmc_replicas *rep, const int32_t *label, double beta, int64_t target, int32_t *accepted_out,
                     void *stream);

/* ---------------------------------------------------------------------------
 * best_energy and state access
 * ------------------------------------------------------------------------- */

/* best: lowest energy any replica has reached at a sweep boundary;
 * n_at_zero: replicas whose best energy is 0; per-replica arrays (R entries,
 * each optional): best energies, current energies, first-hit sweeps. */
int nmc_best_energy(nmc_replicas *rep, int64_t *best, int32_t *n_at_zero, int64_t *best_per_replica,
                    int64_t *energy_per_replica, int32_t *first_hit, void *stream);

/* Full recount of every replica's current energy on the device (R int64),
 * independent of the incrementally tracked energies. */
int nmc_recount(nmc_replicas *rep, int64_t *energy_out, void *stream);

/* Copy a state out as R rows: k-SAT x[r][i] in {0,1} (R*N bytes); QAP
 * p[r][f] (R*n bytes).  which = NMC_STATE_CURRENT or NMC_STATE_BEST. */
int nmc_get_state(nmc_replicas *rep, int32_t which, uint8_t *host_out, size_t bytes, void *stream);

/* Replace the current state (same layout as nmc_get_state) and the sweep
 * counter, for checkpoint/resume.  Energies are recounted; best energies and
 * snapshots restart from the restored state; first_hit resets to -1. */
int nmc_set_state(nmc_replicas *rep, const uint8_t *host_in, size_t bytes, uint32_t sweeps_done, void *stream);

int nmc_replicas_info(const nmc_replicas *rep, int32_t *n_replicas, uint64_t *seed, uint32_t *sweeps_done);

/* ---------------------------------------------------------------------------
 * tuning and timing (results never depend on these)
 * ------------------------------------------------------------------------- */

/* block_threads: threads per workgroup of the k-SAT sweep kernel (64..1024,
 * multiple of 64; 0 = default 1024).  QAP sweeps always run one replica per
 * wave, 16 per 1024-thread workgroup, and ignore it. */
int nmc_set_tuning(nmc_replicas *rep, int32_t block_threads);

/* k-SAT replicas per sweep workgroup: 4 (0 = default; one group, bits 0..3
 * of a spin byte in LDS) or 8 (two groups sharing each spin byte, so every
 * clause record read, address decode and LDS gather serves 8 replicas; half
 * as many workgroups).  Used by nmc_anneal / nmc_reanneal and batched calls
 * (not by tempering).  Results never depend on it.  QAP: UNSUPPORTED. */
int nmc_set_replicas_per_workgroup(nmc_replicas *rep, int32_t reps);

/* The set's current k-SAT sweep workgroup size and replicas per workgroup
 * (QAP: 0 replicas per workgroup); either output may be NULL. */
int nmc_get_tuning(const nmc_replicas *rep, int32_t *block_threads, int32_t *reps_per_workgroup);

/* Tunes one k-SAT replica set: times probe_sweeps sweeps on a copy of its
 * states (the set does not move) for every workgroup size (64 .. 1024) and
 * then 4 or 8 replicas per workgroup (nmc_batch_tune on a batch of this one
 * set), keeps the fastest and returns it (outputs optional).
 * Errors: INVALID, UNSUPPORTED (QAP), DEVICE. */
int nmc_tune(nmc_replicas *rep, int32_t probe_sweeps, int32_t *block_threads, int32_t *reps_per_workgroup,
             void *stream);

/* When enabled, every sweep-kernel launch is bracketed by HIP events on the
 * launch stream; nmc_kernel_time() then returns the summed kernel time (ms),
 * the number of sweep-kernel launches and the Metropolis attempts they made
 * since the last reset (nmc_pt_run counts its sweep launches, not its
 * exchange launches).  Enabling it adds a stream synchronization per call. */
int nmc_set_profiling(nmc_replicas *rep, int32_t enable);
int nmc_kernel_time(nmc_replicas *rep, double *ms, int64_t *launches, double *attempts, int32_t reset);

/* Moves the sweep kernels accepted on this replica set (k-SAT: single-variable
 * flips; QAP: swaps), summed over every sweep call since creation or the last
 * reset (reset != 0 zeroes it after the read).  With the attempts of those
 * calls (k-SAT: R x N per sweep; QAP: R x n(n-1)/2) it gives the mean
 * acceptance rate.  Each call adds its count at its end (one atomic add per
 * wave).  Synchronizes the stream. */
int nmc_accept_count(nmc_replicas *rep, uint64_t *accepted, int32_t reset, void *stream);

/* With profiling enabled, nmc_lbp_backbone brackets the two kernels of every
 * message iteration with HIP events; this returns their summed time (ms) and
 * the iterations timed since the last reset. */
int nmc_lbp_kernel_time(nmc_replicas *rep, double *ms, int64_t *iterations, int32_t reset);


/* ---------------------------------------------------------------------------
 * measurement helper (not part of the method)
 * ------------------------------------------------------------------------- */

enum {
    NMC_PROBE_LDS_DISTINCT = 0, /* LDS byte reads, every lane of a wave on its own bank */
    NMC_PROBE_LDS_RANDOM = 1,   /* LDS byte reads at uniformly random addresses in 100 KB */
    NMC_PROBE_VALU_INT = 2      /* 32-bit integer adds, 8 chains per lane */
};

/* Times one launch of a peak-rate probe kernel on `stream` with HIP events:
 * `blocks` workgroups of 1024 threads (one per CU at a time for the LDS
 * probes, which take 100 KB of LDS each), every lane doing `iters`
 * iterations of 16 reads (LDS probes) or 8 adds (VALU probe).  Writes the
 * kernel time (ms) and the lane operations done (blocks x 1024 x iters x 16
 * reads or x 8 adds), so the ratio is the measured rate to set beside a
 * published peak.  The library allocates one 256-byte word on the current
 * device at its first probe there (kept until the process ends).
 * Synchronizes the stream.  Errors: INVALID (unknown probe, iters not a
 * multiple of 8 in [8, 2^24], blocks outside [1, 2^16]), DEVICE. */
int nmc_probe_peak(int32_t which, int32_t iters, int32_t blocks, double *ms, double *lane_ops, void *stream);


/* ---------------------------------------------------------------------------
 * batched launches (many replica sets of different instances at once)
 * ------------------------------------------------------------------------- */

typedef struct nmc_batch nmc_batch;

/* One anneal -> [backbone -> reanneal] x rounds plan (Algorithm 1's loop of
 * inhomogeneous exploration and homogeneous unlearning, with the backbone
 * re-estimated before every round).
 *   anneal_beta[s]                 s < anneal_sweeps, one class
 *   reanneal_beta[c * S + s]       c = 0 cold, 1 hot; S = reanneal_sweeps
 *   thr_num / thr_den, expand      as nmc_estimate_backbone
 *   chunk_sweeps                   > 0: every phase runs as launches of at
 *                                  most this many sweeps, so all sets advance
 *                                  in lockstep; 0: one launch per phase */
typedef struct nmc_plan {
    const double *anneal_beta;
    int32_t anneal_sweeps;
    int32_t rounds;
    const double *reanneal_beta;
    int32_t reanneal_sweeps;
    int32_t thr_num, thr_den, expand;
    int32_t chunk_sweeps;
} nmc_plan;

/* Group n_sets distinct replica sets (k-SAT and QAP may be mixed) for batched
 * calls.  The handle keeps the pointers; the sets must outlive it.  Results of
 * every set are identical to running its calls alone (same seeds, same sweep
 * counters): nothing a set computes depends on the other sets. */
int nmc_batch_create(nmc_replicas *const *sets, int32_t n_sets, nmc_batch **out);
void nmc_batch_free(nmc_batch *batch);

/* Replace the batch's member sets (n_sets >= 0, distinct); keeps the handle's
 * device buffers, tuning and profiling state.  For continuous batching. */
int nmc_batch_set_members(nmc_batch *batch, nmc_replicas *const *sets, int32_t n_sets);

/* k-SAT sweep workgroup size for this batch's launches (64..1024, multiple of
 * 64; 0 = choose from the instances' colour-class sizes).  Results never
 * depend on it. */
int nmc_batch_set_tuning(nmc_batch *batch, int32_t block_threads);

/* The autotuner.  On copies of the sets' states (the sets themselves do not
 * move), probe_sweeps sweeps of every k-SAT set in one batched launch:
 * (1) for each candidate workgroup size (64, 128, 256, 512, 1024) with 4
 * replicas per workgroup; the fastest is kept for this batch and returned in
 * *chosen; (2) then per set, the replicas per workgroup (4, or 8 sharing each
 * spin byte; nmc_set_replicas_per_workgroup): the sets fall into up to four
 * classes by work (N x R), and each class in turn takes 8 when that makes the
 * batched probe at least 1 % faster (each configuration is timed twice and
 * the shorter time counts).  Each set keeps its choice for later
 * calls.  Results never depend on the tuning. */
int nmc_batch_tune(nmc_batch *batch, int32_t probe_sweeps, int32_t *chosen, void *stream);

/* nmc_anneal for every set of the batch in one launch per kernel kind: one
 * persistent grid walks all (set, replica group) items, largest first.
 * profile: NMC_PROFILE_HOMOGENEOUS or NMC_PROFILE_BACKBONE (HOST is
 * UNSUPPORTED here).  targets: n_sets entries or NULL (no target).
 * Synchronizes the stream before returning. */
int nmc_batch_anneal(nmc_batch *batch, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
                     const int64_t *targets, void *stream);

/* nmc_lbp_backbone for every set at once (k-SAT sets only): one run per set
 * around replica replicas[i] of set i (current or best state), all runs
 * sharing cfg and advancing through the lambda steps together (a run that
 * stops keeps its messages while the others go on), one grid per kernel for
 * all runs.  Each run's result equals the single-set call's; results
 * (optional) receives n_sets entries; each set's backbone becomes its device
 * class array.  The job descriptors (device) and a small pinned readback
 * buffer belong to the batch.  Errors: INVALID, STATE, UNSUPPORTED, DEVICE. */
int nmc_batch_lbp_backbone(nmc_batch *batch, const int32_t *replicas, int32_t which, const nmc_lbp_config *cfg,
                           nmc_lbp_result *results, void *stream);

/* nmc_estimate_backbone for every set (classes stay on the device). */
int nmc_batch_estimate_backbone(nmc_batch *batch, int32_t thr_num, int32_t thr_den, int32_t expand, void *stream);

/* The same plan for every set: nmc_batch_run with plans[i] = *plan. */
int nmc_batch_run_plan(nmc_batch *batch, const nmc_plan *plan, const int64_t *targets, int32_t use_graph,
                       void *stream);

/* Algorithm 1's loop for every set of the batch, each with its own plan
 * (plans[n_sets]: its own schedule, beta units, sweep counts, rounds,
 * backbone rule and chunk size), so k-SAT and QAP sets with different
 * schedules run together.  Set i runs exactly
 *   nmc_anneal(plans[i].anneal_beta, 1 class, anneal_sweeps, homogeneous,
 *              targets[i]);
 *   rounds x { nmc_estimate_backbone(thr_num, thr_den, expand);
 *              nmc_reanneal(reanneal_beta, 2 classes, reanneal_sweeps,
 *                           backbone, targets[i]) }
 * with identical results (targets NULL = no target).  The call's timeline
 * is cut at every phase and chunk boundary of every set; each cut is one
 * batched launch per kernel kind over the sets that have sweeps there (a set
 * whose plan is shorter is left out once it is done), with each set's
 * backbone estimates launched before its rounds.  With use_graph != 0 the
 * whole launch sequence is captured into one HIP graph; the executable graph
 * is kept with the batch and replayed by later calls whose launch sequence
 * has the same shape (same sets' sizes, plan lengths, chunks and rules; the
 * schedules' betas, targets and sweep counters are data uploaded before each
 * launch).  Synchronizes the stream before returning.
 * Errors: INVALID (a plan's fields, betas, thresholds; sweep counter
 * overflow), CAPACITY (LDS), DEVICE. */
int nmc_batch_run(nmc_batch *batch, const nmc_plan *plans, const int64_t *targets, int32_t use_graph, void *stream);

/* Graph bookkeeping of nmc_batch_run / nmc_batch_run_plan: graphs captured
 * and instantiated, and calls that replayed the kept graph. */
int nmc_batch_graph_info(const nmc_batch *batch, int64_t *captures, int64_t *replays);

/* One step of n_sweeps for every set, each running its own segment of its
 * own schedule (continuous batching: sets may be at different points of their
 * plans).  segs[i] for set i:
 *   beta[0], beta[1]   constant inverse temperatures of the cold / hot class
 *                      over this step (class 1 only with the backbone profile)
 *   profile            NMC_PROFILE_HOMOGENEOUS, NMC_PROFILE_BACKBONE, or < 0
 *                      to leave the set idle in this step
 *   backbone_before    != 0: estimate the set's backbone (thr_num / thr_den,
 *                      expand) before the step
 *   target             first-hit target, as nmc_anneal
 * status_out (optional, n_sets entries) receives every set's best energy,
 * replicas with best energy 0 and earliest first-hit sweep (-1 if none).
 * One launch per kernel kind.  Synchronizes the stream before returning. */
typedef struct nmc_segment {
    double beta[2];
    int32_t profile;
    int32_t backbone_before;
    int64_t target;
} nmc_segment;

typedef struct nmc_set_status {
    int64_t best;
    int32_t n_at_zero;
    int32_t first_hit;
} nmc_set_status;

int nmc_batch_step(nmc_batch *batch, const nmc_segment *segs, int32_t n_sweeps, int32_t thr_num, int32_t thr_den,
                   int32_t expand, nmc_set_status *status_out, void *stream);

/* Kernel timing of batched sweeps, as nmc_set_profiling / nmc_kernel_time. */
int nmc_batch_set_profiling(nmc_batch *batch, int32_t enable);
int nmc_batch_kernel_time(nmc_batch *batch, double *ms, int64_t *launches, double *attempts, int32_t reset);

/* ---------------------------------------------------------------------------
 * serving: continuous batching of solve requests
 * ------------------------------------------------------------------------- */

typedef struct nmc_server nmc_server;

typedef struct nmc_server_config {
    size_t hbm_cap_bytes;    /* admit while the admitted requests' device bytes fit (0 = 64 GiB) */
    int32_t chunk_sweeps;    /* sweeps per round; targets are checked at round ends (0 = 50) */
    int32_t max_active;      /* most requests on the GPU at once (0 = 512) */
    int32_t loader_threads;  /* host threads building instance layouts (0 = 4) */
    int32_t block_threads;   /* k-SAT sweep workgroup size (0 = chosen per round) */
    int32_t thr_num, thr_den, expand;  /* backbone rule for every request (0, 0 = 9/10, expand) */
} nmc_server_config;

/* A solve request.  The server copies every array during nmc_server_submit.
 * Schedule (piecewise constant over rounds of chunk_sweeps sweeps): anneal
 * rounds take beta0 .. beta1 linearly (both ends) on one class; then `rounds`
 * times: backbone estimate (the server's rule), reanneal rounds with the cold
 * class at beta1 and the hot class ramped beta_hot .. beta1.
 * anneal_sweeps and reanneal_sweeps must be multiples of chunk_sweeps.
 * QAP betas are in inverse cost units (already scaled by the caller). */
typedef struct nmc_request {
    int32_t kind;                                  /* NMC_KIND_KSAT or NMC_KIND_QAP */
    int32_t n_vars, n_clauses, class_cap;          /* k-SAT (as nmc_ksat_load) */
    const int32_t *clause_ptr, *lits;
    int32_t n;                                     /* QAP (as nmc_qap_load) */
    const int32_t *flow, *dist;
    int32_t n_replicas;
    uint64_t seed;
    double beta0, beta1, beta_hot;
    int32_t anneal_sweeps, rounds, reanneal_sweeps;
    int64_t target;                                /* stop at the first round end with a replica <= target */
    int32_t has_target;
    double budget_s;                               /* stop after this long since admission (0 = none) */
} nmc_request;

enum nmc_request_status {
    NMC_REQ_QUEUED = 0, NMC_REQ_LOADED = 1, NMC_REQ_RUNNING = 2,
    NMC_REQ_SOLVED = 3,     /* reached its target */
    NMC_REQ_EXHAUSTED = 4,  /* finished its schedule without reaching the target */
    NMC_REQ_TIMEOUT = 5,    /* budget spent */
    NMC_REQ_FAILED = 6      /* see message */
};

typedef struct nmc_result {
    int32_t status;          /* nmc_request_status */
    int32_t n_at_zero;
    int64_t best;            /* lowest energy any replica reached at a sweep end */
    int32_t first_hit_sweep; /* first sweep boundary at or below the target, -1 if none */
    uint32_t sweeps_done;
    double t_submit, t_admit, t_done;  /* seconds on the server clock */
    size_t device_bytes;
    char message[128];
} nmc_result;

typedef struct nmc_server_stats {
    int64_t rounds, submitted, completed;
    int32_t active, waiting;
    size_t device_bytes_in_use;
    double gpu_busy_s;       /* summed wall time of the rounds */
} nmc_server_stats;

/* Start a server: a worker thread that owns the GPU work on its own stream and
 * loader threads that build instance layouts.  Every round advances all
 * admitted requests by chunk_sweeps sweeps in one batched launch per kernel
 * kind; loaded requests are admitted in arrival order as device memory and
 * slots free up (a request larger than the cap runs alone), and retire at the
 * round end where they reach their target, spend their budget or finish their
 * schedule.  A request's results do not depend on what
 * else is on the GPU (its own seed, schedule and sweep counter). */
int nmc_server_create(const nmc_server_config *config, nmc_server **out);
/* Thread-safe; copies the request.  *id identifies it in nmc_server_poll. */
int nmc_server_submit(nmc_server *server, const nmc_request *req, uint64_t *id);
/* Thread-safe snapshot of a request's state and result. */
int nmc_server_poll(nmc_server *server, uint64_t id, nmc_result *out);
/* Block until every submitted request has completed or timeout_s passes
 * (returns NMC_ERR_STATE on timeout). */
int nmc_server_wait_idle(nmc_server *server, double timeout_s);
int nmc_server_get_stats(nmc_server *server, nmc_server_stats *out);
/* Seconds on the server clock (steady, since creation). */
double nmc_server_now(const nmc_server *server);
/* Stop the threads (requests still running are marked FAILED) and free. */
void nmc_server_free(nmc_server *server);

#ifdef __cplusplus
}
#endif

#endif /* NMC_H */
