/*
 * nmc_oracle.c -- plain sequential CPU oracle for the NMC hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file.  It is used by the tests, by the smoke check and by the
 * benchmark's CPU-baseline leg, and shares no code with the GPU path.
 *
 * What it computes (paper: "Nonequilibrium Monte Carlo for unfreezing
 * variables in hard combinatorial optimization"):
 *   - k-SAT energy = number of violated clauses of a CNF formula (subsection
 *     "4-SAT Problems Near Computational Phase Transitions"; a violated clause
 *     costs one unit here, see the clause weight of appendix C for the
 *     paper's two-unit convention).
 *   - single-variable Metropolis sweeps with a per-variable inverse
 *     temperature (section "Nonequilibrium inhomogeneous sampling over
 *     subgraphs": backbone variables run hotter than the rest), simulated
 *     annealing being the homogeneous special case (section "Nonequilibrium
 *     Nonlocal Monte Carlo").
 *   - backbone estimate from empirical averages over independent replicas
 *     (appendix B, "Sampling localized replicas by Monte Carlo": average the
 *     spins over R clones), thresholded on |magnetization|.
 *   - QAP cost (Koopmans-Beckmann form, subsection "Quadratic Assignment
 *     Problems") with pairwise-swap Metropolis moves and the per-facility
 *     assignment-frequency backbone.
 *   - replica exchange between neighbouring temperatures and the energy
 *     spread that sets the adaptive temperature ladder (appendix A,
 *     "Adaptive Parallel Tempering"; the first step of algorithm 1).
 *   - loopy belief propagation on the localized surrogate Hamiltonian of a
 *     CNF and connected backbone growth (sections on surrogate Hamiltonians,
 *     LBP and backbones; appendix C).
 *   - whitening of low-energy states (section "Whitening procedure for low
 *     energy states").
 *   - collective flips of backbone clusters (the NMC scheme's nonlocal
 *     move: a whole cluster flipped at once under the Metropolis rule).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), written here from that paper's
 * definition of the round function and key schedule.
 *
 * Every loop below runs in the order the method defines; nothing is blocked,
 * fused or reordered.  All energies are exact integers.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* RNG stream identifiers (fourth counter word) */
#define ORC_STREAM_SWEEP 0u
#define ORC_STREAM_INIT 1u
#define ORC_STREAM_QAP_SWEEP 2u
#define ORC_STREAM_QAP_INIT 3u
#define ORC_STREAM_PT_SWAP 4u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. SC'11, section 3.3 "Philox")                 */
/* ------------------------------------------------------------------------ */

/* One Philox S-box round on a 4-word block: the two multipliers act on
 * words 0 and 2; the high halves are xored with the other two words and the
 * round key; the low halves pass through.  The key is bumped by the Weyl
 * constants (golden ratio and sqrt(3)-1, scaled to 32 bits) between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The uniform 32-bit word a replica draws for item j at sweep t:
 * key = (low, high) halves of the seed; counter = (j, t, replica / 4, stream);
 * the replica takes output word (replica mod 4). */
uint32_t orc_uniform_u32(uint64_t seed, uint32_t stream, uint32_t j, uint32_t t, uint32_t replica)
{
    uint32_t ctr[4] = { j, t, replica >> 2, stream };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[replica & 3u];
}

/* ------------------------------------------------------------------------ */
/* Metropolis acceptance thresholds                                          */
/* ------------------------------------------------------------------------ */

/* Accepting a move that raises the energy by d > 0 with probability
 * exp(-beta d) is done as u < T with u uniform on [0, 2^32):
 * T = min(2^32 - 1, floor(2^32 exp(-beta d))), in IEEE double. */
uint32_t orc_threshold(double beta, int64_t d)
{
    double v = ldexp(exp(-(beta * (double)d)), 32);
    if (!(v < 4294967295.0))
        return 0xFFFFFFFFu;
    return (uint32_t)floor(v);
}

/* QAP energy changes reach millions, so the threshold is factored as
 * exp(-beta d) = exp(-beta h 2^b) * exp(-beta l) with d = h 2^b + l:
 * T = (A * B) >> 32 with A = orc_threshold(beta, h 2^b) (A = 2^32-1 at h=0)
 * and B = orc_threshold(beta, l) (B = 2^32-1 at l=0), b = 10. */
uint32_t orc_qap_threshold(double beta, int64_t d)
{
    int64_t h = d >> 10, l = d & 1023;
    uint64_t a = h == 0 ? 0xFFFFFFFFull : (uint64_t)orc_threshold(beta, h << 10);
    uint64_t b = l == 0 ? 0xFFFFFFFFull : (uint64_t)orc_threshold(beta, l);
    return (uint32_t)((a * b) >> 32);
}

/* ------------------------------------------------------------------------ */
/* k-SAT                                                                     */
/* ------------------------------------------------------------------------ */

/* literal +(v+1) is true iff x_v = 1; literal -(v+1) is true iff x_v = 0 */
static int lit_true(int32_t lit, const uint8_t *x)
{
    int32_t v = (lit > 0 ? lit : -lit) - 1;
    return lit > 0 ? (x[v] != 0) : (x[v] == 0);
}

static int clause_sat(const int32_t *cptr, const int32_t *lits, int32_t a, const uint8_t *x)
{
    for (int32_t p = cptr[a]; p < cptr[a + 1]; ++p)
        if (lit_true(lits[p], x))
            return 1;
    return 0;
}

/* E(x) = number of clauses with no true literal. */
int32_t orc_ksat_energy(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, const uint8_t *x)
{
    (void)n;
    int32_t e = 0;
    for (int32_t a = 0; a < m; ++a)
        e += !clause_sat(cptr, lits, a, x);
    return e;
}

/* variable -> clauses incidence, built by counting (each clause listed once
 * per literal of the variable; clauses hold distinct variables) */
typedef struct {
    int32_t *ptr; /* n+1 */
    int32_t *cl;  /* cptr[m] */
} orc_adj;

static int adj_build(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, orc_adj *g)
{
    int32_t nl = cptr[m];
    g->ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    g->cl = (int32_t *)malloc(((size_t)nl + 1) * sizeof(int32_t));
    int32_t *fill = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!g->ptr || !g->cl || !fill) {
        free(g->ptr); free(g->cl); free(fill);
        return -1;
    }
    for (int32_t p = 0; p < nl; ++p) {
        int32_t v = (lits[p] > 0 ? lits[p] : -lits[p]) - 1;
        g->ptr[v + 1]++;
    }
    for (int32_t v = 0; v < n; ++v)
        g->ptr[v + 1] += g->ptr[v];
    for (int32_t a = 0; a < m; ++a)
        for (int32_t p = cptr[a]; p < cptr[a + 1]; ++p) {
            int32_t v = (lits[p] > 0 ? lits[p] : -lits[p]) - 1;
            g->cl[g->ptr[v] + fill[v]++] = a;
        }
    free(fill);
    return 0;
}

static void adj_free(orc_adj *g)
{
    free(g->ptr);
    free(g->cl);
}

/* Energy change of flipping x_i: for every clause holding i, compare its
 * violation before and after the flip (the definition, literal by literal). */
static int32_t ksat_delta(const orc_adj *g, const int32_t *cptr, const int32_t *lits, int32_t i, uint8_t *x)
{
    int32_t d = 0;
    for (int32_t q = g->ptr[i]; q < g->ptr[i + 1]; ++q) {
        int32_t a = g->cl[q];
        int before = clause_sat(cptr, lits, a, x);
        x[i] ^= 1;
        int after = clause_sat(cptr, lits, a, x);
        x[i] ^= 1;
        d += (!after) - (!before);
    }
    return d;
}

int32_t orc_ksat_delta(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, int32_t i, uint8_t *x)
{
    orc_adj g;
    if (adj_build(n, m, cptr, lits, &g))
        return INT32_MIN;
    int32_t d = ksat_delta(&g, cptr, lits, i, x);
    adj_free(&g);
    return d;
}

/* Sweep order: greedy colouring of the variable interaction graph (two
 * variables interact when they share a clause).  Variables are visited in
 * index order; each takes the smallest colour that no already-coloured
 * neighbour holds and, when cap > 0, that holds fewer than cap variables.
 * The order lists colour 0's variables in index order, then colour 1's, ...
 * Returns the number of colours; class_ptr[c]..class_ptr[c+1] delimit them. */
int32_t orc_ksat_color(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, int32_t cap,
                       int32_t *color, int32_t *order, int32_t *class_ptr)
{
    orc_adj g;
    if (adj_build(n, m, cptr, lits, &g))
        return -1;
    int32_t *mark = (int32_t *)malloc(((size_t)n + 2) * sizeof(int32_t));
    int32_t *size = (int32_t *)calloc((size_t)n + 2, sizeof(int32_t));
    for (int32_t c = 0; c < n + 2; ++c)
        mark[c] = -1;
    int32_t ncol = 0;
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t q = g.ptr[v]; q < g.ptr[v + 1]; ++q) {
            int32_t a = g.cl[q];
            for (int32_t p = cptr[a]; p < cptr[a + 1]; ++p) {
                int32_t w = (lits[p] > 0 ? lits[p] : -lits[p]) - 1;
                if (w < v) /* already coloured */
                    mark[color[w]] = v;
            }
        }
        int32_t c = 0;
        while (mark[c] == v || (cap > 0 && size[c] >= cap))
            ++c;
        color[v] = c;
        size[c]++;
        if (c + 1 > ncol)
            ncol = c + 1;
    }
    class_ptr[0] = 0;
    for (int32_t c = 0; c < ncol; ++c)
        class_ptr[c + 1] = class_ptr[c] + size[c];
    int32_t *fill = (int32_t *)calloc((size_t)ncol + 1, sizeof(int32_t));
    for (int32_t v = 0; v < n; ++v) {
        int32_t c = color[v];
        order[class_ptr[c] + fill[c]++] = v;
    }
    free(fill);
    free(mark);
    free(size);
    adj_free(&g);
    return ncol;
}

/* Initial spins: x_i of replica r is the top bit of the INIT-stream word
 * drawn for item i at sweep 0.  x is [R][n]. */
void orc_ksat_init(int32_t n, int32_t r_begin, int32_t r_end, uint64_t seed, uint8_t *x)
{
    for (int32_t r = r_begin; r < r_end; ++r)
        for (int32_t i = 0; i < n; ++i)
            x[(size_t)r * n + i] = (uint8_t)(orc_uniform_u32(seed, ORC_STREAM_INIT, (uint32_t)i, 0u, (uint32_t)r) >> 31);
}

/* Metropolis sweeps for replicas r_begin..r_end-1.
 *   order[p]        : variable visited at position p of every sweep
 *   beta[c*S + s]   : inverse temperature of class c at sweep s of this call
 *   class_of[i]     : class of variable i (NULL = every variable in class 0)
 *   t0              : global index of the first sweep of this call
 * Per replica: energy[r] is the energy at entry and is set to the energy at
 * exit; best[r] is the lowest energy seen at a sweep boundary; first_hit[r] is
 * the first sweep boundary (number of sweeps done) with energy <= target, -1
 * while none; best_x (optional) receives the state of each strict improvement.
 * A move with dE <= 0 is always taken; otherwise the replica draws its SWEEP
 * word for (variable, sweep) and takes the move iff u < T(beta, dE). */
int orc_ksat_anneal(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, const int32_t *order,
                    int32_t r_begin, int32_t r_end, uint64_t seed, uint32_t t0, int32_t n_sweeps,
                    int32_t n_classes, const double *beta, const uint8_t *class_of, int64_t target,
                    uint8_t *x, int32_t *energy, int32_t *best, int32_t *first_hit, uint8_t *best_x)
{
    orc_adj g;
    if (adj_build(n, m, cptr, lits, &g))
        return -1;
    int32_t dmax = 0;
    for (int32_t v = 0; v < n; ++v)
        if (g.ptr[v + 1] - g.ptr[v] > dmax)
            dmax = g.ptr[v + 1] - g.ptr[v];
    /* thresholds of the current sweep, one row per class: tab[c][d] = T(beta, d) */
    uint32_t *tab = (uint32_t *)malloc(((size_t)n_classes * (dmax + 1) + 1) * sizeof(uint32_t));
    for (int32_t r = r_begin; r < r_end; ++r) {
        uint8_t *xr = x + (size_t)r * n;
        int32_t e = orc_ksat_energy(n, m, cptr, lits, xr);
        if (first_hit[r] < 0 && e <= target)
            first_hit[r] = (int32_t)t0;
        for (int32_t s = 0; s < n_sweeps; ++s) {
            uint32_t t = t0 + (uint32_t)s;
            for (int32_t c = 0; c < n_classes; ++c)
                for (int32_t d = 0; d <= dmax; ++d)
                    tab[(size_t)c * (dmax + 1) + d] = orc_threshold(beta[(size_t)c * n_sweeps + s], d);
            for (int32_t p = 0; p < n; ++p) {
                int32_t i = order[p];
                int32_t c = class_of ? class_of[i] : 0;
                int32_t d = ksat_delta(&g, cptr, lits, i, xr);
                int accept = d <= 0;
                if (!accept) {
                    uint32_t u = orc_uniform_u32(seed, ORC_STREAM_SWEEP, (uint32_t)i, t, (uint32_t)r);
                    accept = u < tab[(size_t)c * (dmax + 1) + d];
                }
                if (accept)
                    xr[i] ^= 1;
            }
            e = orc_ksat_energy(n, m, cptr, lits, xr);
            if (e < best[r]) {
                best[r] = e;
                if (best_x)
                    memcpy(best_x + (size_t)r * n, xr, (size_t)n);
            }
            if (first_hit[r] < 0 && e <= target)
                first_hit[r] = (int32_t)(t + 1);
        }
        energy[r] = e;
    }
    free(tab);
    adj_free(&g);
    return 0;
}

/* Backbone from replica averages: c_i = number of replicas with x_i = 1, so the
 * magnetization over replicas is m_i = (2 c_i - R) / R.  Variable i is frozen
 * iff |m_i| >= num/den, i.e. den |2 c_i - R| >= num R.  With expand != 0 the
 * hot class also takes every variable that shares a clause with a frozen one.
 * cls[i] = 1 (hot) or 0 (cold).  x is [R][n]. */
void orc_ksat_backbone(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, int32_t R,
                       const uint8_t *x, int32_t thr_num, int32_t thr_den, int32_t expand,
                       int32_t *counts, uint8_t *cls)
{
    uint8_t *frozen = (uint8_t *)calloc((size_t)n + 1, 1);
    for (int32_t i = 0; i < n; ++i) {
        int32_t c = 0;
        for (int32_t r = 0; r < R; ++r)
            c += x[(size_t)r * n + i] != 0;
        if (counts)
            counts[i] = c;
        int64_t dev = 2 * (int64_t)c - R;
        if (dev < 0)
            dev = -dev;
        frozen[i] = (int64_t)thr_den * dev >= (int64_t)thr_num * R;
        cls[i] = frozen[i];
    }
    if (expand) {
        for (int32_t a = 0; a < m; ++a) {
            int any = 0;
            for (int32_t p = cptr[a]; p < cptr[a + 1]; ++p)
                any |= frozen[(lits[p] > 0 ? lits[p] : -lits[p]) - 1];
            if (any)
                for (int32_t p = cptr[a]; p < cptr[a + 1]; ++p)
                    cls[(lits[p] > 0 ? lits[p] : -lits[p]) - 1] = 1;
        }
    }
    free(frozen);
}

/* ------------------------------------------------------------------------ */
/* QAP                                                                       */
/* ------------------------------------------------------------------------ */

/* perm[f] = location of facility f.  C = sum_i sum_j F_ij D_{perm_i perm_j}. */
int64_t orc_qap_cost(int32_t n, const int32_t *F, const int32_t *D, const uint8_t *perm)
{
    int64_t c = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j)
            c += (int64_t)F[(size_t)i * n + j] * D[(size_t)perm[i] * n + perm[j]];
    return c;
}

/* Cost change of exchanging the locations of facilities r != s, for general
 * (not necessarily symmetric) F and D: only the rows and columns r, s of the
 * double sum change; every other term is unchanged. */
int64_t orc_qap_delta(int32_t n, const int32_t *F, const int32_t *D, const uint8_t *perm, int32_t r, int32_t s)
{
#define FF(i, j) ((int64_t)F[(size_t)(i) * n + (j)])
#define DD(i, j) ((int64_t)D[(size_t)(i) * n + (j)])
    int32_t pr = perm[r], ps = perm[s];
    int64_t d = 0;
    for (int32_t k = 0; k < n; ++k) {
        if (k == r || k == s)
            continue;
        int32_t pk = perm[k];
        d += FF(r, k) * (DD(ps, pk) - DD(pr, pk));
        d += FF(s, k) * (DD(pr, pk) - DD(ps, pk));
        d += FF(k, r) * (DD(pk, ps) - DD(pk, pr));
        d += FF(k, s) * (DD(pk, pr) - DD(pk, ps));
    }
    d += FF(r, r) * (DD(ps, ps) - DD(pr, pr));
    d += FF(s, s) * (DD(pr, pr) - DD(ps, ps));
    d += FF(r, s) * (DD(ps, pr) - DD(pr, ps));
    d += FF(s, r) * (DD(pr, ps) - DD(ps, pr));
    return d;
#undef FF
#undef DD
}

/* Random initial assignment: Fisher-Yates from the identity, step j = n-1..1
 * takes k = floor(u (j+1) / 2^32) with u the QAP_INIT word for item j, and
 * exchanges positions j and k.  perm is [R][n]. */
void orc_qap_init(int32_t n, int32_t r_begin, int32_t r_end, uint64_t seed, uint8_t *perm)
{
    for (int32_t r = r_begin; r < r_end; ++r) {
        uint8_t *p = perm + (size_t)r * n;
        for (int32_t i = 0; i < n; ++i)
            p[i] = (uint8_t)i;
        for (int32_t j = n - 1; j >= 1; --j) {
            uint64_t u = orc_uniform_u32(seed, ORC_STREAM_QAP_INIT, (uint32_t)j, 0u, (uint32_t)r);
            int32_t k = (int32_t)((u * (uint64_t)(j + 1)) >> 32);
            uint8_t tmp = p[j];
            p[j] = p[k];
            p[k] = tmp;
        }
    }
}

/* Swap-move Metropolis sweeps: one sweep proposes every pair (a, b), a < b,
 * in lexicographic order; pair q (its rank in that order) draws the
 * QAP_SWEEP word for (q, sweep).  The pair's class is the larger of its two
 * facilities' classes.  Bookkeeping as orc_ksat_anneal, with int64 costs. */
int orc_qap_anneal(int32_t n, const int32_t *F, const int32_t *D, int32_t r_begin, int32_t r_end,
                   uint64_t seed, uint32_t t0, int32_t n_sweeps, int32_t n_classes, const double *beta,
                   const uint8_t *class_of, int64_t target, uint8_t *perm, int64_t *cost, int64_t *best,
                   int32_t *first_hit, uint8_t *best_perm)
{
    (void)n_classes;
    for (int32_t r = r_begin; r < r_end; ++r) {
        uint8_t *p = perm + (size_t)r * n;
        int64_t c = orc_qap_cost(n, F, D, p);
        if (first_hit[r] < 0 && c <= target)
            first_hit[r] = (int32_t)t0;
        for (int32_t s = 0; s < n_sweeps; ++s) {
            uint32_t t = t0 + (uint32_t)s;
            uint32_t q = 0;
            for (int32_t a = 0; a + 1 < n; ++a) {
                for (int32_t b = a + 1; b < n; ++b, ++q) {
                    int32_t ca = class_of ? class_of[a] : 0;
                    int32_t cb = class_of ? class_of[b] : 0;
                    int32_t cl = ca > cb ? ca : cb;
                    int64_t d = orc_qap_delta(n, F, D, p, a, b);
                    int accept = d <= 0;
                    if (!accept) {
                        uint32_t u = orc_uniform_u32(seed, ORC_STREAM_QAP_SWEEP, q, t, (uint32_t)r);
                        accept = u < orc_qap_threshold(beta[(size_t)cl * n_sweeps + s], d);
                    }
                    if (accept) {
                        uint8_t tmp = p[a];
                        p[a] = p[b];
                        p[b] = tmp;
                    }
                }
            }
            c = orc_qap_cost(n, F, D, p);
            if (c < best[r]) {
                best[r] = c;
                if (best_perm)
                    memcpy(best_perm + (size_t)r * n, p, (size_t)n);
            }
            if (first_hit[r] < 0 && c <= target)
                first_hit[r] = (int32_t)(t + 1);
        }
        cost[r] = c;
    }
    return 0;
}

/* Assignment-frequency backbone: freq[f][l] = #{r : perm_r[f] = l}; facility f
 * is frozen (hot) iff den * max_l freq[f][l] >= num * R. */
void orc_qap_backbone(int32_t n, int32_t R, const uint8_t *perm, int32_t thr_num, int32_t thr_den,
                      int32_t *freq, uint8_t *cls)
{
    int32_t *h = freq ? freq : (int32_t *)malloc((size_t)n * n * sizeof(int32_t));
    memset(h, 0, (size_t)n * n * sizeof(int32_t));
    for (int32_t r = 0; r < R; ++r)
        for (int32_t f = 0; f < n; ++f)
            h[(size_t)f * n + perm[(size_t)r * n + f]]++;
    for (int32_t f = 0; f < n; ++f) {
        int32_t mx = 0;
        for (int32_t l = 0; l < n; ++l)
            if (h[(size_t)f * n + l] > mx)
                mx = h[(size_t)f * n + l];
        cls[f] = (int64_t)thr_den * mx >= (int64_t)thr_num * R;
    }
    if (!freq)
        free(h);
}

/* ------------------------------------------------------------------------ */
/* Parallel tempering (appendix A, "Adaptive Parallel Tempering")            */
/* ------------------------------------------------------------------------ */

/* Replicas are laid out temperature-major: replica r = i * n_chains + c holds
 * ladder position i (inverse temperature beta[i], ascending in i) of chain c.
 * One exchange step offers, in every chain, the neighbour pairs (i, i + 1)
 * for i = parity, parity + 2, ... (disjoint pairs; the caller alternates the
 * parity).  The pair exchanges its two configurations with probability
 * p = min{1, exp[(beta_i - beta_{i+1}) (E_i - E_{i+1})]} (appendix A, the
 * replica-exchange rule), so p = 1 when E_i <= E_{i+1}.  Otherwise the pair
 * draws word 0 of the Philox block at counter (c, t, i, PT_SWAP) and swaps iff
 * u < orc_qap_threshold(beta_{i+1} - beta_i, E_i - E_{i+1}): the factored
 * threshold of the QAP moves, since energy gaps between replicas span the
 * whole energy range.  t is the number of sweeps done when the step is taken.
 * rows is [R][row_len] (spins or assignments) and energy [R]; both move with
 * the configuration.  Only chains c_begin..c_end-1 are stepped (chains are
 * independent, so a sample of them can be followed alone).  accepted /
 * attempted [n_temps - 1] count per pair position. */
void orc_pt_exchange(int32_t n_temps, int32_t n_chains, int32_t c_begin, int32_t c_end, const double *beta,
                     uint64_t seed, uint32_t t, int32_t parity, int32_t row_len, uint8_t *rows, int64_t *energy,
                     int64_t *accepted, int64_t *attempted)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (int32_t i = parity; i + 1 < n_temps; i += 2) {
        double dbeta = beta[i + 1] - beta[i];
        for (int32_t c = c_begin; c < c_end; ++c) {
            int64_t a = (int64_t)i * n_chains + c;
            int64_t b = a + n_chains;
            int64_t d = energy[a] - energy[b];
            int accept = d <= 0;
            if (!accept) {
                uint32_t ctr[4] = { (uint32_t)c, t, (uint32_t)i, ORC_STREAM_PT_SWAP };
                uint32_t out[4];
                orc_philox4x32_10(ctr, key, out);
                accept = out[0] < orc_qap_threshold(dbeta, d);
            }
            attempted[i]++;
            if (accept) {
                accepted[i]++;
                for (int32_t k = 0; k < row_len; ++k) {
                    uint8_t tmp = rows[(size_t)a * row_len + k];
                    rows[(size_t)a * row_len + k] = rows[(size_t)b * row_len + k];
                    rows[(size_t)b * row_len + k] = tmp;
                }
                int64_t te = energy[a];
                energy[a] = energy[b];
                energy[b] = te;
            }
        }
    }
}

/* Energy spread at one inverse temperature (appendix A):
 * sigma^2 = <E^2> - <E>^2 over the samples.  Energies are non-negative and
 * below 2^32, so with S1 = sum E and S2 = sum E^2 the numerator
 * count * S2 - S1^2 is an exact 128-bit integer; it is rounded to double once
 * and divided by count^2 (exact in double for count < 2^26). */
double orc_energy_sigma(const int64_t *e, int64_t count)
{
    unsigned __int128 s1 = 0, s2 = 0;
    for (int64_t k = 0; k < count; ++k) {
        unsigned __int128 v = (unsigned __int128)(uint64_t)e[k];
        s1 += v;
        s2 += v * v;
    }
    unsigned __int128 num = (unsigned __int128)(uint64_t)count * s2 - s1 * s1;
    double var = (double)num / ((double)count * (double)count);
    return sqrt(var);
}

/* ------------------------------------------------------------------------ */
/* Localized surrogate Hamiltonian and LBP on the CNF factor graph           */
/* (section "Constructing localized surrogate Hamiltonians", section         */
/* "Efficient sampling of localized surrogate Hamiltonians via LBP",         */
/* subsection "4-SAT Problems Near Computational Phase Transitions",         */
/* appendix C "Loopy Belief propagation for k-local Hamiltonians over        */
/* conjugate normal form")                                                   */
/* ------------------------------------------------------------------------ */

/* Spins r_i = +1 for x_i = 1, -1 for x_i = 0.  Edge p (a literal position of
 * the CSR) joins clause a and variable i = var(p); sigma_p = +1 if the literal
 * is positive (r_i = +1 satisfies it), -1 if negated.  A clause violated by
 * r carries the weight exp(-2 beta), a satisfied one 1.  The reference
 * configuration s* couples through the field H_i = lambda eps_i s*_i with
 * eps_i = the number of clauses holding i.
 *
 * Messages (in the frame of the clause: positive = leaning to satisfy it):
 *   h_{i->a} = sigma_{ia} H_i + sum_{b in di \ a} sigma_{ia} sigma_{ib} u_{b->i}
 *   u_{a->i} = -1/2 ln[1 - (1 - e^{-2 beta}) prod_{j in da \ i} (1 - tanh h_{j->a}) / 2]
 * Magnetization <r_i> = tanh(H_i + sum_{a in di} sigma_{ia} u_{a->i}).
 * Clause moment under mu_a(r) ~ omega_a(r) prod_j (1 + sigma_{ja} r_j t_j) / 2,
 * t_j = tanh h_{j->a}:
 *   <prod_j r_j>_a = [prod_j sigma_{ja} t_j - (1 - e^{-2 beta}) prod_j (-sigma_{ja}) (1 - t_j) / 2] / z_a,
 *   z_a = 1 - (1 - e^{-2 beta}) prod_j (1 - t_j) / 2. */

static int32_t lit_var(int32_t l) { return (l > 0 ? l : -l) - 1; }
static double lit_sign(int32_t l) { return l > 0 ? 1.0 : -1.0; }

/* every edge of variable i: edge list built by counting, in CSR order */
typedef struct {
    int32_t *ptr; /* n+1 */
    int32_t *edge; /* cptr[m] */
} orc_vedges;

static int vedges_build(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, orc_vedges *g)
{
    int32_t ne = cptr[m];
    g->ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    g->edge = (int32_t *)malloc(((size_t)ne + 1) * sizeof(int32_t));
    int32_t *fill = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!g->ptr || !g->edge || !fill) {
        free(g->ptr); free(g->edge); free(fill);
        return -1;
    }
    for (int32_t p = 0; p < ne; ++p)
        g->ptr[lit_var(lits[p]) + 1]++;
    for (int32_t v = 0; v < n; ++v)
        g->ptr[v + 1] += g->ptr[v];
    for (int32_t p = 0; p < ne; ++p) {
        int32_t v = lit_var(lits[p]);
        g->edge[g->ptr[v] + fill[v]++] = p;
    }
    free(fill);
    return 0;
}

/* one message iteration: every h from u, then every u from h (both
 * computed as their definitions state); returns max |u_new - u_old| */
static double lbp_iterate(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, const orc_vedges *g,
                          const double *H, double beta, double *h, double *u, double *u_new)
{
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = g->ptr[i]; e < g->ptr[i + 1]; ++e) {
            int32_t p = g->edge[e];
            double sp = lit_sign(lits[p]);
            double s = sp * H[i];
            for (int32_t f = g->ptr[i]; f < g->ptr[i + 1]; ++f) {
                int32_t q = g->edge[f];
                if (q != p)
                    s += sp * lit_sign(lits[q]) * u[q];
            }
            h[p] = s;
        }
    double w = 1.0 - exp(-2.0 * beta);
    double delta = 0.0;
    for (int32_t a = 0; a < m; ++a)
        for (int32_t p = cptr[a]; p < cptr[a + 1]; ++p) {
            double prod = 1.0;
            for (int32_t q = cptr[a]; q < cptr[a + 1]; ++q)
                if (q != p)
                    prod *= (1.0 - tanh(h[q])) / 2.0;
            u_new[p] = -0.5 * log(1.0 - w * prod);
            double d = fabs(u_new[p] - u[p]);
            if (d > delta)
                delta = d;
        }
    memcpy(u, u_new, (size_t)cptr[m] * sizeof(double));
    return delta;
}

/* Adiabatic LBP (section on LBP: start at a large lambda with messages
 * h_{i->a} = sigma_{ia} H_i and u from them, then lower lambda step by step
 * keeping the messages).  Step k uses lambda_k = lambda0 * ratio^k while
 * lambda_k >= lambda_min; at each step the messages are iterated until
 * max |du| < tol (at most max_iter iterations).  A step that does not
 * converge, or whose overlap p = (1/N) sum s*_i <r_i> falls below p_min, is
 * discarded and the previous step's messages are kept.
 * Outputs from the kept messages: u (final), mag[n], corr[m] (signed clause
 * moments) and stats = {lambda, steps tried, iterations, converged, delta, p,
 * q1 = (1/N) sum <r_i>^2}.  s_star[i] in {-1, +1}.  Returns 0, or -1 on
 * allocation failure. */
int orc_lbp_cnf(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, const int8_t *s_star, double beta,
                double lambda0, double ratio, double lambda_min, int32_t max_iter, double tol, double p_min,
                double *u, double *mag, double *corr, double *stats)
{
    orc_vedges g;
    if (vedges_build(n, m, cptr, lits, &g))
        return -1;
    int32_t ne = cptr[m];
    double *eps = (double *)malloc(((size_t)n + 1) * sizeof(double));
    double *H = (double *)malloc(((size_t)n + 1) * sizeof(double));
    double *h = (double *)malloc(((size_t)ne + 1) * sizeof(double));
    double *un = (double *)malloc(((size_t)ne + 1) * sizeof(double));
    double *keep = (double *)malloc(((size_t)ne + 1) * sizeof(double));
    for (int32_t i = 0; i < n; ++i)
        eps[i] = (double)(g.ptr[i + 1] - g.ptr[i]);
    double w = 1.0 - exp(-2.0 * beta);

    /* initial messages at lambda0 */
    for (int32_t i = 0; i < n; ++i)
        H[i] = lambda0 * eps[i] * s_star[i];
    for (int32_t p = 0; p < ne; ++p)
        h[p] = lit_sign(lits[p]) * H[lit_var(lits[p])];
    for (int32_t a = 0; a < m; ++a)
        for (int32_t p = cptr[a]; p < cptr[a + 1]; ++p) {
            double prod = 1.0;
            for (int32_t q = cptr[a]; q < cptr[a + 1]; ++q)
                if (q != p)
                    prod *= (1.0 - tanh(h[q])) / 2.0;
            u[p] = -0.5 * log(1.0 - w * prod);
        }

    double lambda = lambda0, kept_lambda = lambda0, kept_delta = 0.0;
    int32_t steps = 0, iters = 0, have = 0;
    for (;;) {
        for (int32_t i = 0; i < n; ++i)
            H[i] = lambda * eps[i] * s_star[i];
        memcpy(keep, u, (size_t)ne * sizeof(double));
        double delta = 0.0;
        int conv = 0;
        for (int32_t it = 0; it < max_iter; ++it) {
            delta = lbp_iterate(n, m, cptr, lits, &g, H, beta, h, u, un);
            ++iters;
            if (delta < tol) {
                conv = 1;
                break;
            }
        }
        ++steps;
        double pov = 0.0;
        if (conv) {
            for (int32_t i = 0; i < n; ++i) {
                double f = H[i];
                for (int32_t e = g.ptr[i]; e < g.ptr[i + 1]; ++e)
                    f += lit_sign(lits[g.edge[e]]) * u[g.edge[e]];
                pov += s_star[i] * tanh(f);
            }
            pov = n ? pov / n : 1.0;
        }
        if (!conv || (have && pov < p_min)) {
            if (have)
                memcpy(u, keep, (size_t)ne * sizeof(double));
            else
                kept_delta = delta;
            break;
        }
        have = 1;
        kept_lambda = lambda;
        kept_delta = delta;
        double next = lambda * ratio;
        if (!(next >= lambda_min))
            break;
        lambda = next;
    }

    /* marginals and clause moments from the kept messages */
    for (int32_t i = 0; i < n; ++i)
        H[i] = kept_lambda * eps[i] * s_star[i];
    double p_sum = 0.0, q_sum = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double f = H[i];
        for (int32_t e = g.ptr[i]; e < g.ptr[i + 1]; ++e)
            f += lit_sign(lits[g.edge[e]]) * u[g.edge[e]];
        mag[i] = tanh(f);
        p_sum += s_star[i] * mag[i];
        q_sum += mag[i] * mag[i];
    }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = g.ptr[i]; e < g.ptr[i + 1]; ++e) {
            int32_t p = g.edge[e];
            double sp = lit_sign(lits[p]);
            double s = sp * H[i];
            for (int32_t f = g.ptr[i]; f < g.ptr[i + 1]; ++f) {
                int32_t q = g.edge[f];
                if (q != p)
                    s += sp * lit_sign(lits[q]) * u[q];
            }
            h[p] = s;
        }
    for (int32_t a = 0; a < m; ++a) {
        double sat = 1.0, viol = 1.0, pv = 1.0;
        for (int32_t q = cptr[a]; q < cptr[a + 1]; ++q) {
            double t = tanh(h[q]), sg = lit_sign(lits[q]);
            sat *= sg * t;
            viol *= -sg * (1.0 - t) / 2.0;
            pv *= (1.0 - t) / 2.0;
        }
        corr[a] = (sat - w * viol) / (1.0 - w * pv);
    }
    stats[0] = kept_lambda;
    stats[1] = steps;
    stats[2] = iters;
    stats[3] = have;
    stats[4] = kept_delta;
    stats[5] = n ? p_sum / n : 1.0;
    stats[6] = n ? q_sum / n : 1.0;
    free(eps); free(H); free(h); free(un); free(keep);
    free(g.ptr); free(g.edge);
    return 0;
}

/* Connected backbone growth (section "Generating backbones of rigid
 * variables"): a clause is rigid when |corr_a| >= theta_cut and a seed when
 * |corr_a| >= theta_seed.  Rigid clauses join all their variables; a
 * connected group of variables that holds at least one seed clause is a
 * cluster of the backbone.  label[i] = smallest variable index of i's
 * cluster, -1 outside the backbone; cls[i] = 1 inside, 0 outside.  Returns
 * the number of clusters. */
int32_t orc_cnf_clusters(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, const double *corr,
                         double theta_seed, double theta_cut, int32_t *label, uint8_t *cls)
{
    orc_adj g;
    if (adj_build(n, m, cptr, lits, &g))
        return -1;
    int32_t *queue = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *comp = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i)
        comp[i] = -1;
    int32_t clusters = 0;
    for (int32_t s = 0; s < n; ++s) {
        if (comp[s] >= 0)
            continue;
        /* breadth-first search from s over rigid clauses */
        int32_t qh = 0, qt = 0, seeded = 0;
        queue[qt++] = s;
        comp[s] = s;
        while (qh < qt) {
            int32_t i = queue[qh++];
            for (int32_t e = g.ptr[i]; e < g.ptr[i + 1]; ++e) {
                int32_t a = g.cl[e];
                double c = fabs(corr[a]);
                if (!(c >= theta_cut))
                    continue;
                if (c >= theta_seed)
                    seeded = 1;
                for (int32_t p = cptr[a]; p < cptr[a + 1]; ++p) {
                    int32_t j = lit_var(lits[p]);
                    if (comp[j] < 0) {
                        comp[j] = s;
                        queue[qt++] = j;
                    }
                }
            }
        }
        for (int32_t k = 0; k < qt; ++k) {
            label[queue[k]] = seeded ? s : -1;
            cls[queue[k]] = (uint8_t)seeded;
        }
        clusters += seeded;
    }
    free(queue);
    free(comp);
    adj_free(&g);
    return clusters;
}

/* ------------------------------------------------------------------------ */
/* Whitening of a low-energy state (section "Whitening procedure for low    */
/* energy states")                                                           */
/* ------------------------------------------------------------------------ */

/* A variable is labelled white ("star") when none of its clauses pins it.
 * Clause a pins its variable i when i's literal is the only true literal of
 * a and no other variable of a is white; a clause with no true literal (a
 * violated clause of a low-energy state) pins nothing, which is the
 * section's extension to states that are not solutions.  Variables are
 * inspected one at a time in the given order (index order when order is
 * NULL), pass after pass, until a pass labels nothing new; the others are
 * frozen.  star[i] = 1 for white, 0 for frozen.  Returns the number of
 * frozen variables; *passes receives the passes made (the last one labels
 * nothing). */
int32_t orc_ksat_whiten(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, const uint8_t *x,
                        const int32_t *order, uint8_t *star, int32_t *passes)
{
    orc_adj g;
    if (adj_build(n, m, cptr, lits, &g))
        return -1;
    for (int32_t i = 0; i < n; ++i)
        star[i] = 0;
    int32_t npass = 0, changed = 1;
    while (changed) {
        changed = 0;
        ++npass;
        for (int32_t k = 0; k < n; ++k) {
            int32_t i = order ? order[k] : k;
            if (star[i])
                continue;
            int pinned = 0;
            for (int32_t e = g.ptr[i]; e < g.ptr[i + 1] && !pinned; ++e) {
                int32_t a = g.cl[e];
                int own_true = 0, other_true = 0, other_star = 0;
                for (int32_t p = cptr[a]; p < cptr[a + 1]; ++p) {
                    int32_t v = lit_var(lits[p]);
                    int t = lit_true(lits[p], x);
                    if (v == i)
                        own_true = t;
                    else {
                        other_true |= t;
                        other_star |= star[v];
                    }
                }
                pinned = own_true && !other_true && !other_star;
            }
            if (!pinned) {
                star[i] = 1;
                changed = 1;
            }
        }
    }
    int32_t frozen = 0;
    for (int32_t i = 0; i < n; ++i)
        frozen += !star[i];
    if (passes)
        *passes = npass;
    adj_free(&g);
    return frozen;
}

/* ------------------------------------------------------------------------ */
/* Collective flips of backbone clusters (figure of the NMC scheme, panel   */
/* (c): a nonlocal flip of a whole backbone cluster; the section on         */
/* annealed thresholds lists it as the alternative to heating the backbone) */
/* ------------------------------------------------------------------------ */

/* One collective-move sweep: for every replica, the clusters (label[i] >= 0
 * names variable i's cluster by its smallest variable; -1 = no cluster) are
 * proposed in increasing label order; proposal k flips every variable of the
 * k-th cluster at once and is taken when dE <= 0, else when the replica's
 * CFLIP word u for (k, t, replica / 4) satisfies u < T(beta, dE) (the k-SAT
 * threshold of orc_threshold).  dE is the exact energy difference (recounted
 * here in full).  The sweep counts as sweep t of the schedule for best,
 * first-hit and snapshot bookkeeping (as in orc_ksat_anneal).  accepted[r]
 * receives the clusters flipped in replica r. */
#define ORC_STREAM_CFLIP 5u
int orc_ksat_cluster_flip(int32_t n, int32_t m, const int32_t *cptr, const int32_t *lits, const int32_t *label,
                          int32_t r_begin, int32_t r_end, uint64_t seed, uint32_t t, double beta, int64_t target,
                          uint8_t *x, int32_t *energy, int32_t *best, int32_t *first_hit, uint8_t *best_x,
                          int32_t *accepted)
{
    /* the clusters in increasing label order */
    int32_t *roots = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i)
        if (label[i] == i)
            roots[nc++] = i;
    uint8_t *y = (uint8_t *)malloc((size_t)n + 1);
    for (int32_t r = r_begin; r < r_end; ++r) {
        uint8_t *xr = x + (size_t)r * n;
        int32_t e = orc_ksat_energy(n, m, cptr, lits, xr);
        int32_t acc = 0;
        for (int32_t k = 0; k < nc; ++k) {
            memcpy(y, xr, (size_t)n);
            for (int32_t i = 0; i < n; ++i)
                if (label[i] == roots[k])
                    y[i] ^= 1;
            int32_t d = orc_ksat_energy(n, m, cptr, lits, y) - e;
            int take = d <= 0;
            if (!take) {
                uint32_t u = orc_uniform_u32(seed, ORC_STREAM_CFLIP, (uint32_t)k, t, (uint32_t)r);
                take = u < orc_threshold(beta, d);
            }
            if (take) {
                memcpy(xr, y, (size_t)n);
                e += d;
                ++acc;
            }
        }
        energy[r] = e;
        if (e < best[r]) {
            best[r] = e;
            if (best_x)
                memcpy(best_x + (size_t)r * n, xr, (size_t)n);
        }
        if (first_hit[r] < 0 && e <= target)
            first_hit[r] = (int32_t)(t + 1);
        if (accepted)
            accepted[r] = acc;
    }
    free(y);
    free(roots);
    return nc;
}
