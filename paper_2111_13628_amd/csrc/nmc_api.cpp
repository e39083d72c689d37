// Host side of the NMC library: argument validation, the instance layouts
// the kernels read, acceptance-threshold tables, handles, and the C ABI
// declared in include/nmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/nmc.h"
#include "nmc_internal.h"

using namespace nmc;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return NMC_OK;
}

}  // namespace

// Proposals per step of the QAP sweep: 0 = chosen per sweep by the kernel;
// NMC_QAP_ROWS=1, 4 or 8 pins it, 2 pins the table mode, 3 the four
// replicas per wave (for measurements; results do not change).
static int32_t qap_rows_setting() {
    const char *e = std::getenv("NMC_QAP_ROWS");
    const int v = e ? std::atoi(e) : 0;
    return (int32_t)(((v >= 1 && v <= 4) || v == 8) ? v : 0);
}

// Whether the per-sweep choice of single-set QAP sweeps may take the table
// mode (NMC_QAP_TAB=1) or run hot sweeps with 2 or 4 replicas per wave
// (NMC_QAP_RPW=2 or 4).  For measurements; results do not change.
static int32_t qap_tab_setting() {
    const char *e = std::getenv("NMC_QAP_TAB");
    return (int32_t)(e && e[0] == '1');
}
// NMC_QAP_DSTAR=0 makes the QAP sweeps read both threshold words per
// proposal instead of comparing against the per-word bound (for measurements;
// results do not change).
static int32_t qap_dstar_setting() {
    const char *e = std::getenv("NMC_QAP_DSTAR");
    return (int32_t)!(e && e[0] == '0');
}
static int32_t qap_quad_setting() {
    const char *e = std::getenv("NMC_QAP_RPW");  // replicas per wave in hot sweeps: 2 or 4
    const int v = e ? std::atoi(e) : 0;
    return (int32_t)(v == 2 || v == 4 ? v : 0);
}

int nmc::set_last_error(int code, const char *msg) {
    g_err = msg ? msg : "";
    return code;
}

namespace {

#define HIP_OR_FAIL(expr)                                                                                  \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return fail(NMC_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));                  \
    } while (0)

namespace {

// HIP events owned by a scope: destroyed when it ends, early error returns
// included
struct ScopedEvents {
    std::vector<hipEvent_t> ev;
    ScopedEvents() = default;
    ScopedEvents(const ScopedEvents &) = delete;
    ScopedEvents &operator=(const ScopedEvents &) = delete;
    ~ScopedEvents() {
        for (hipEvent_t e : ev)
            (void)hipEventDestroy(e);
    }
    hipError_t create(hipEvent_t *out) {
        hipEvent_t e = nullptr;
        const hipError_t r = hipEventCreate(&e);
        if (r == hipSuccess) {
            ev.push_back(e);
            *out = e;
        }
        return r;
    }
};

}  // namespace

// Acceptance threshold for an energy rise d > 0 at inverse temperature beta:
// min(2^32 - 1, floor(2^32 exp(-beta d))) evaluated in IEEE double.
uint32_t threshold(double beta, int64_t d) {
    const double v = std::ldexp(std::exp(-(beta * static_cast<double>(d))), 32);
    if (!(v < 4294967295.0))
        return 0xFFFFFFFFu;
    return static_cast<uint32_t>(std::floor(v));
}

// Words of one QAP threshold row: the high digit A[0 .. ha), the low digit
// B[0 .. 1024) and 1 / beta as a float (where the kernels start their search
// for the acceptance bound of a random word).
int32_t qap_row_words(int32_t ha) { return ha + (1 << kQapLowBits) + 1; }

// Fills one QAP threshold row for inverse temperature beta: T(d) =
// (A[d >> 10] B[d & 1023]) >> 32, A[h] = threshold(beta, 1024 h) and B[l] =
// threshold(beta, l) with A[0] = B[0] = 2^32 - 1, and T = 0 from d = 1024 ha
// on.  Returns whether T never increases with d: then a random word u has a
// bound d*(u) with u < T(d) exactly when d < d*(u), which the kernels use in
// place of the two table reads per proposal.
bool qap_fill_row(uint32_t *row, double beta, int32_t ha) {
    constexpr int32_t lo_n = 1 << kQapLowBits;
    uint32_t *lo = row + ha;
    row[0] = 0xFFFFFFFFu;
    for (int32_t h = 1; h < ha; ++h)
        row[h] = threshold(beta, (int64_t)h << kQapLowBits);
    lo[0] = 0xFFFFFFFFu;
    for (int32_t l = 1; l < lo_n; ++l)
        lo[l] = threshold(beta, l);
    const float inv = (float)(1.0 / beta);  // beta = 0: +inf
    std::memcpy(lo + lo_n, &inv, sizeof inv);
    bool mono = true;
    for (int32_t l = 1; l < lo_n; ++l)
        mono = mono && lo[l] <= lo[l - 1];
    // within a block T follows B; across blocks the last word of block h - 1
    // must not be below the first of block h
    for (int32_t h = 1; h < ha; ++h) {
        const uint64_t last = ((uint64_t)row[h - 1] * lo[lo_n - 1]) >> 32;
        const uint64_t first = ((uint64_t)row[h] * lo[0]) >> 32;
        mono = mono && row[h] <= row[h - 1] && first <= last;
    }
    return mono;
}

struct Arena {
    size_t size = 0;
    size_t take(size_t bytes) {
        size = align_up(size, 256);
        const size_t off = size;
        size += bytes;
        return off;
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// instance
// ---------------------------------------------------------------------------

struct nmc_instance {
    int kind = 0;
    // k-SAT host data
    int32_t n = 0, m = 0, kmax = 0, dmax = 0, n_colors = 0, n_chunks = 0;
    std::vector<int32_t> order, color_ptr;
    // layout offsets into the device arena
    size_t off_rec = 0, off_chunk_var = 0, off_chunk_info = 0, off_color_chunk = 0, off_clause_addr = 0,
           off_var_ptr = 0, off_var_cl = 0;
    // LBP clause order (clauses sorted by their smallest variable): the
    // clauses' literal addresses in that order and each clause's position
    size_t off_lbp_caddr = 0, off_lbp_pos = 0;
    std::vector<int32_t> lbp_pos;
    uint32_t rec_bytes = 0;  // size of the record array
    // wide layout (spins in device memory; see nmc_ksat_wide.hip)
    bool wide = false;
    size_t off_wrec = 0, off_worder = 0, off_wclass = 0;
    // QAP host data
    int64_t delta_bound = 0;
    int32_t qap_ha = 0;
    // largest energy any state can have (k-SAT: M; QAP: sum F * max D)
    int64_t energy_bound = 0;
    int64_t n_lits = 0;  // k-SAT: literal occurrences (sum of clause lengths)
    size_t off_F = 0, off_D = 0;
    // packed host image of the device arena
    std::vector<uint8_t> image;
    size_t arena_bytes = 0;
    uint8_t *dev = nullptr;
    std::atomic<int> live_replicas{0};
    // references: the caller's handle plus one per live replica set; the
    // host object goes when the last is released, whatever the order
    std::atomic<int> refs{1};

    KsatDev ksat_dev() const {
        KsatDev d{};
        d.rec = reinterpret_cast<const uint64_t *>(dev + off_rec);
        d.rec_bytes = rec_bytes;
        d.chunk_var = reinterpret_cast<const int32_t *>(dev + off_chunk_var);
        d.chunk_info = reinterpret_cast<const int2 *>(dev + off_chunk_info);
        d.color_chunk = reinterpret_cast<const int32_t *>(dev + off_color_chunk);
        d.clause_addr = reinterpret_cast<const uint32_t *>(dev + off_clause_addr);
        d.var_ptr = reinterpret_cast<const int32_t *>(dev + off_var_ptr);
        d.var_cl = reinterpret_cast<const int32_t *>(dev + off_var_cl);
        d.lbp_caddr = reinterpret_cast<const uint32_t *>(dev + off_lbp_caddr);
        d.lbp_pos = reinterpret_cast<const int32_t *>(dev + off_lbp_pos);
        d.wrec = reinterpret_cast<const uint4 *>(dev + off_wrec);
        d.worder = reinterpret_cast<const int32_t *>(dev + off_worder);
        d.wclass_ptr = reinterpret_cast<const int32_t *>(dev + off_wclass);
        d.wide = wide ? 1 : 0;
        d.n = n;
        d.m = m;
        d.n_colors = n_colors;
        d.n_chunks = n_chunks;
        d.dmax = dmax;
        return d;
    }
    QapDev qap_dev() const {
        QapDev d{};
        d.F = dev + off_F;
        d.D = dev + off_D;
        d.n = n;
        d.ha = qap_ha;
        return d;
    }
};

namespace {

// Greedy colouring: variables in index order take the smallest colour that
// no already-coloured variable sharing a clause holds and (cap > 0) that is
// not full.  Returns the colour of every variable.
std::vector<int32_t> greedy_colors(int32_t n, const std::vector<int32_t> &vptr, const std::vector<int32_t> &vcl,
                                   const int32_t *cptr, const int32_t *lits, int32_t cap, int32_t *n_colors) {
    std::vector<int32_t> color(n, -1), seen(n + 1, -1), fill;
    int32_t ncol = 0;
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t q = vptr[v]; q < vptr[v + 1]; ++q) {
            const int32_t a = vcl[q];
            for (int32_t p = cptr[a]; p < cptr[a + 1]; ++p) {
                const int32_t w = std::abs(lits[p]) - 1;
                if (color[w] >= 0)
                    seen[color[w]] = v;
            }
        }
        int32_t c = 0;
        while (seen[c] == v || (cap > 0 && c < (int32_t)fill.size() && fill[c] >= cap))
            ++c;
        if (c >= (int32_t)fill.size())
            fill.resize(c + 1, 0);
        fill[c]++;
        color[v] = c;
        ncol = std::max(ncol, c + 1);
    }
    *n_colors = ncol;
    return color;
}


// LDS bank-aware placement of one chunk's clause records into slots.  In a
// slot, every lane issues three byte gathers (its record's three addresses)
// as three wave-wide LDS reads.  gfx950 serves such a read 32 lanes at a time
// over 32 four-byte banks, so two lanes of one half-wave that hit different
// dwords of one bank serialize.  A lane's records may be visited in any slot
// order and a record's three addresses may be issued in any order without
// changing any result (integer sums), so the records are placed greedily,
// slot by slot, to keep each half-wave's addresses on distinct banks.
struct ChunkRec {
    uint32_t a[3];
    uint32_t neg;
};

// Bank model of one byte gather on gfx950 LDS: 32 banks of 4 bytes, a wave's
// 64 addresses served in two half-waves of 32; lanes reading the same dword
// share one access, different dwords on one bank serialize.  Cost of a
// half-wave = the largest number of distinct dwords on one bank.
struct BankLoad {
    int32_t dw[32][8];
    int8_t cnt[32];
    int8_t mx;
    void clear() {
        std::memset(cnt, 0, sizeof cnt);
        mx = 0;
    }
    // distinct-dword count of the bank after adding dword d (no change)
    int after(int32_t d) const {
        const int b = d & 31;
        for (int i = 0; i < cnt[b] && i < 8; ++i)
            if (dw[b][i] == d)
                return cnt[b];
        return cnt[b] + 1;
    }
    void add(int32_t d) {
        const int b = d & 31;
        for (int i = 0; i < cnt[b] && i < 8; ++i)
            if (dw[b][i] == d)
                return;
        if (cnt[b] < 8)
            dw[b][(int)cnt[b]] = d;
        cnt[b]++;
        mx = std::max<int8_t>(mx, cnt[b]);
    }
};

// Places every lane's records into slots (and orders each record's three
// addresses) so that each slot's three gathers touch few distinct dwords per
// bank in each half-wave.  Greedy per slot: lanes take, in turn, the record
// and address order that raises the half-wave's worst bank least, then loads
// the fewest-used banks; the most loaded lanes go first.  Any placement gives
// the same results; only the gathers' bank conflicts change.
void schedule_chunk(std::vector<std::vector<ChunkRec>> &lanes, int32_t nslot, bool optimize,
                    std::vector<ChunkRec> &out /* [nslot][64] */, const ChunkRec &dummy) {
    static const int perms[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {1, 0, 2}, {2, 1, 0}};
    out.assign((size_t)nslot * kChunk, dummy);
    if (!optimize) {
        for (int l = 0; l < kChunk; ++l)
            for (size_t s = 0; s < lanes[l].size(); ++s)
                out[s * kChunk + l] = lanes[l][s];
        return;
    }
    std::vector<int> order(kChunk);
    BankLoad load[3][2];
    for (int32_t s = 0; s < nslot; ++s) {
        for (int j = 0; j < 3; ++j)
            for (int h = 0; h < 2; ++h)
                load[j][h].clear();
        // lanes without records read the inert dummy in this slot
        for (int l = 0; l < kChunk; ++l)
            if (lanes[l].empty())
                for (int j = 0; j < 3; ++j)
                    load[j][l / 32].add((int32_t)(dummy.a[j] >> 2));
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return lanes[x].size() > lanes[y].size(); });
        for (int l : order) {
            std::vector<ChunkRec> &rem = lanes[l];
            if (rem.empty())
                continue;
            const int h = l / 32;
            // cost: 64 per gather whose worst bank grows, plus the distinct
            // dwords already on the banks this record's addresses join
            int best_i = 0, best_p = 0, best_c = 1 << 30;
            for (size_t i = 0; i < rem.size() && best_c > 0; ++i)
                for (int p = 0; p < 6 && best_c > 0; ++p) {
                    int c = 0;
                    for (int j = 0; j < 3; ++j) {
                        const int a = load[j][h].after((int32_t)(rem[i].a[perms[p][j]] >> 2));
                        c += (a > load[j][h].mx ? 64 : 0) + (a - 1);
                    }
                    if (c < best_c) {
                        best_c = c;
                        best_i = (int)i;
                        best_p = p;
                    }
                }
            ChunkRec r = rem[best_i];
            ChunkRec placed = r;
            for (int j = 0; j < 3; ++j) {
                placed.a[j] = r.a[perms[best_p][j]];
                load[j][h].add((int32_t)(placed.a[j] >> 2));
            }
            out[(size_t)s * kChunk + l] = placed;
            rem[best_i] = rem.back();
            rem.pop_back();
        }
    }
}

// Modeled LDS cycles of a chunk's gathers (sum over slots, positions and
// half-waves of the worst bank's distinct dwords).
int64_t chunk_gather_cycles(const std::vector<ChunkRec> &placed, int32_t nslot) {
    int64_t cyc = 0;
    BankLoad bl;
    for (int32_t s = 0; s < nslot; ++s)
        for (int j = 0; j < 3; ++j)
            for (int h = 0; h < 2; ++h) {
                bl.clear();
                for (int l = h * 32; l < h * 32 + 32; ++l)
                    bl.add((int32_t)(placed[(size_t)s * kChunk + l].a[j] >> 2));
                cyc += bl.mx;
            }
    return cyc;
}

}  // namespace

extern "C" {

const char *nmc_last_error(void) { return g_err.c_str(); }

int32_t nmc_version(void) { return 101; }

int nmc_ksat_load(int32_t n_vars, int32_t n_clauses, const int32_t *clause_ptr, const int32_t *lits,
                  int32_t class_cap, nmc_instance **out) {
    try {
        if (!out)
            return fail(NMC_ERR_INVALID, "out is NULL");
        *out = nullptr;
        if (n_vars < 1)
            return fail(NMC_ERR_INVALID, "n_vars must be >= 1");
        if (n_vars > kMaxWideVars)
            return fail(NMC_ERR_UNSUPPORTED, "n_vars %d exceeds %d", n_vars, kMaxWideVars);
        if (n_clauses < 0)
            return fail(NMC_ERR_INVALID, "n_clauses must be >= 0");
        if (!clause_ptr || (n_clauses > 0 && !lits))
            return fail(NMC_ERR_INVALID, "clause_ptr/lits is NULL");
        if (class_cap < 0)
            return fail(NMC_ERR_INVALID, "class_cap must be >= 0");
        if (clause_ptr[0] != 0)
            return fail(NMC_ERR_INVALID, "clause_ptr[0] must be 0");
        // every offset first, so that no literal is read through a bad offset
        int32_t kmax = 0;
        for (int32_t a = 0; a < n_clauses; ++a) {
            const int64_t len = (int64_t)clause_ptr[a + 1] - clause_ptr[a];
            if (len < 1)
                return fail(NMC_ERR_INVALID, "clause %d is empty or offsets decrease", a);
            if (len > 4)
                return fail(NMC_ERR_UNSUPPORTED, "clause %d has %lld literals (at most 4 supported)", a,
                            (long long)len);
            kmax = std::max(kmax, (int32_t)len);
        }
        for (int32_t a = 0; a < n_clauses; ++a) {
            for (int32_t p = clause_ptr[a]; p < clause_ptr[a + 1]; ++p) {
                const int32_t l = lits[p];
                if (l == 0 || l > n_vars || l < -n_vars)
                    return fail(NMC_ERR_INVALID, "clause %d: literal %d out of range", a, l);
                for (int32_t p2 = clause_ptr[a]; p2 < p; ++p2)
                    if (std::abs(lits[p2]) == std::abs(l))
                        return fail(NMC_ERR_INVALID, "clause %d repeats variable %d", a, std::abs(l));
            }
        }
        std::unique_ptr<nmc_instance> I(new nmc_instance());
        I->kind = NMC_KIND_KSAT;
        I->n = n_vars;
        I->m = n_clauses;
        // spin tables of more than kMaxVars variables do not fit in LDS;
        // NMC_KSAT_WIDE=1 takes the wide layout for any size (tests, measurements)
        const char *wide_env = std::getenv("NMC_KSAT_WIDE");
        I->wide = n_vars > kMaxVars || (wide_env && wide_env[0] == '1');
        I->energy_bound = n_clauses;
        I->n_lits = clause_ptr[n_clauses];
        I->kmax = kmax;
        const int32_t n = n_vars, m = n_clauses;

        // variable -> clause incidence (clause ids ascending per variable)
        std::vector<int32_t> vptr(n + 1, 0), vcl, vpos;
        for (int32_t p = 0; p < clause_ptr[m]; ++p)
            vptr[std::abs(lits[p])]++;
        for (int32_t v = 0; v < n; ++v)
            vptr[v + 1] += vptr[v];
        vcl.resize(vptr[n]);
        vpos.resize(vptr[n]);
        {
            std::vector<int32_t> fill(vptr.begin(), vptr.end() - 1);
            for (int32_t a = 0; a < m; ++a)
                for (int32_t p = clause_ptr[a]; p < clause_ptr[a + 1]; ++p) {
                    const int32_t v = std::abs(lits[p]) - 1;
                    vcl[fill[v]] = a;
                    vpos[fill[v]] = p;
                    fill[v]++;
                }
        }
        int32_t dmax = 0;
        for (int32_t v = 0; v < n; ++v)
            dmax = std::max(dmax, vptr[v + 1] - vptr[v]);
        if (dmax > 127)
            return fail(NMC_ERR_UNSUPPORTED, "a variable occurs in %d clauses (at most 127 supported)", dmax);
        I->dmax = dmax;

        // colouring and colour-major order
        int32_t ncol = 0;
        std::vector<int32_t> color = greedy_colors(n, vptr, vcl, clause_ptr, lits, class_cap, &ncol);
        I->n_colors = ncol;
        I->color_ptr.assign(ncol + 1, 0);
        for (int32_t v = 0; v < n; ++v)
            I->color_ptr[color[v] + 1]++;
        for (int32_t c = 0; c < ncol; ++c)
            I->color_ptr[c + 1] += I->color_ptr[c];
        I->order.resize(n);
        {
            std::vector<int32_t> fill(I->color_ptr.begin(), I->color_ptr.end() - 1);
            for (int32_t v = 0; v < n; ++v)
                I->order[fill[color[v]]++] = v;
        }

        // chunks: within a class, variables by degree (descending) in groups of 64
        const uint32_t ZERO = 2u * n, ONES = 2u * n + 1;
        auto lit_addr = [&](int32_t l) -> uint32_t {
            return l > 0 ? (uint32_t)(l - 1) : (uint32_t)(n + (-l - 1));
        };
        const char *sched_env = std::getenv("NMC_KSAT_BANK_SCHEDULE");
        const bool bank_schedule = !(sched_env && sched_env[0] == '0');
        // lanes per variable in chunks of small colour classes (results never
        // depend on it; NMC_KSAT_SPLIT=0 keeps one lane per variable)
        const char *split_env = std::getenv("NMC_KSAT_SPLIT");
        const bool split = !(split_env && split_env[0] == '0');
        const bool debug_banks = std::getenv("NMC_DEBUG_BANKS") != nullptr;
        int64_t model_cycles = 0, model_gathers = 0;
        std::vector<int32_t> chunk_var, color_chunk(ncol + 1, 0);
        std::vector<int2> chunk_info;
        std::vector<uint64_t> rec;
        int32_t slot_rows = 0;
        if (!I->wide) {
        // (1) every chunk's lanes and records, (2) placement (chunks are
        // independent: spread over host threads for large instances), (3) the
        // packed record image in chunk order
        struct ChunkWork {
            std::vector<std::vector<ChunkRec>> lanes;
            int32_t nslot = 0;
            std::vector<ChunkRec> placed;
        };
        std::vector<ChunkWork> work;
        for (int32_t c = 0; c < ncol; ++c) {
            std::vector<int32_t> vs(I->order.begin() + I->color_ptr[c], I->order.begin() + I->color_ptr[c + 1]);
            std::stable_sort(vs.begin(), vs.end(), [&](int32_t x, int32_t y) {
                return (vptr[x + 1] - vptr[x]) > (vptr[y + 1] - vptr[y]);
            });
            for (size_t b = 0; b < vs.size(); b += kChunk) {
                const size_t e = std::min(vs.size(), b + kChunk);
                // a chunk of few variables gives each variable L = 2^lg
                // adjacent lanes (its clauses dealt round-robin over them), so
                // a lane walks about 1/L of the variable's slots; the lanes'
                // partial sums are added before the decision
                int32_t lg = 0;
                while (split && lg < kMaxSplitLog && (int32_t)(e - b) << (lg + 1) <= kChunk)
                    ++lg;
                const int32_t L = 1 << lg;
                int32_t nslot = 0;
                for (size_t i = b; i < e; ++i)
                    nslot = std::max(nslot, (vptr[vs[i] + 1] - vptr[vs[i]] + L - 1) / L);
                nslot = std::max<int32_t>(kSlotUnroll, (int32_t)align_up(nslot, kSlotUnroll));  // padding slots are inert
                chunk_info.push_back(make_int2(slot_rows, nslot | (lg << kSplitShift)));
                slot_rows += nslot;
                ChunkWork w;
                w.lanes.resize(kChunk);
                w.nslot = nslot;
                int32_t n1[kChunk] = {0};
                for (size_t i = b; i < e; ++i) {
                    const int lane0 = (int)(i - b) * L;
                    const int32_t v = vs[i];
                    for (int32_t q = vptr[v]; q < vptr[v + 1]; ++q) {
                        const int32_t a = vcl[q], own = vpos[q];
                        const int lane = lane0 + (q - vptr[v]) % L;
                        ChunkRec r{{ZERO, ZERO, ZERO}, lits[own] < 0 ? 1u : 0u};
                        int k = 0;
                        for (int32_t p = clause_ptr[a]; p < clause_ptr[a + 1]; ++p)
                            if (p != own)
                                r.a[k++] = lit_addr(lits[p]);
                        n1[lane] += (int32_t)r.neg;
                        w.lanes[lane].push_back(r);
                    }
                }
                work.push_back(std::move(w));
                // lane word: variable in bits 0..19 and the count of the lane's
                // records whose own literal is negated in bits 20..27; -1 =
                // empty lane
                for (int lane = 0; lane < kChunk; ++lane) {
                    const size_t i = b + (size_t)(lane / L);
                    chunk_var.push_back(i < e ? (vs[i] | (n1[lane] << 20)) : -1);
                }
            }
            color_chunk[c + 1] = (int32_t)chunk_info.size();
        }
        {
            const ChunkRec dummy{{ONES, ZERO, ZERO}, 0u};
            std::atomic<size_t> next{0};
            auto worker = [&] {
                for (size_t i; (i = next.fetch_add(1)) < work.size();)
                    schedule_chunk(work[i].lanes, work[i].nslot, bank_schedule, work[i].placed, dummy);
            };
            const size_t n_rec = vcl.size();
            const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
            const unsigned nt = bank_schedule && n_rec >= 200000 ? std::min(8u, hw) : 1u;
            std::vector<std::thread> pool;
            for (unsigned t = 1; t < nt; ++t)
                pool.emplace_back(worker);
            worker();
            for (auto &t : pool)
                t.join();
        }
        rec.resize((size_t)slot_rows * kChunk);
        for (size_t i = 0; i < work.size(); ++i) {
            const int32_t nslot = work[i].nslot;
            const std::vector<ChunkRec> &placed = work[i].placed;
            if (debug_banks) {
                model_cycles += chunk_gather_cycles(placed, nslot);
                model_gathers += 3 * (int64_t)nslot;
            }
            const size_t base = (size_t)chunk_info[i].x * kChunk;
            // slots are stored in pairs: [slot / 2][lane][slot % 2], so one
            // 16-byte load gives a lane two consecutive slots
            for (int32_t sl = 0; sl < nslot; ++sl)
                for (int lane = 0; lane < kChunk; ++lane) {
                    const ChunkRec &r = placed[(size_t)sl * kChunk + lane];
                    rec[base + (size_t)(sl / 2) * 2 * kChunk + (size_t)lane * 2 + (sl & 1)] =
                        (uint64_t)r.a[0] | ((uint64_t)r.a[1] << kAddrBits) | ((uint64_t)r.a[2] << (2 * kAddrBits)) |
                        ((uint64_t)r.neg << (3 * kAddrBits));
                }
        }
        I->n_chunks = (int32_t)chunk_info.size();
        if (debug_banks && model_gathers)
            std::fprintf(stderr, "nmc: %d chunks, %lld slot gathers, modeled %.3f LDS cycles per gather\n",
                         I->n_chunks, (long long)model_gathers, (double)model_cycles / (double)model_gathers);
        }  // !I->wide
        // wide layout: per incidence (var_ptr order) the clause's other
        // literals as spin-table rows (v for x_v, n + 1 + v for NOT x_v, row
        // n: absent, never true), and whether the variable's own literal is
        // negated
        std::vector<uint4> wrec;
        if (I->wide) {
            wrec.resize(vcl.size());
            for (int32_t v = 0; v < n; ++v)
                for (int32_t q = vptr[v]; q < vptr[v + 1]; ++q) {
                    const int32_t a = vcl[q], own = vpos[q];
                    uint32_t w[3] = {(uint32_t)n, (uint32_t)n, (uint32_t)n};
                    int k = 0;
                    for (int32_t p = clause_ptr[a]; p < clause_ptr[a + 1]; ++p)
                        if (p != own) {
                            const int32_t l = lits[p];
                            w[k++] = (uint32_t)(std::abs(l) - 1) + (l < 0 ? (uint32_t)n + 1u : 0u);
                        }
                    wrec[q] = make_uint4(w[0], w[1], w[2], lits[own] < 0 ? 1u : 0u);
                }
        }

        std::vector<uint32_t> clause_addr((size_t)m * 4, ZERO);
        for (int32_t a = 0; a < m; ++a) {
            int k = 0;
            for (int32_t p = clause_ptr[a]; p < clause_ptr[a + 1]; ++p)
                clause_addr[(size_t)a * 4 + k++] = lit_addr(lits[p]);
        }
        // LBP clause order: a stable counting sort by smallest variable, so
        // the clauses a workgroup of the clause pass takes share variables
        // (their field reads and message writes then fall in the same cache
        // lines); the literal order inside a clause is kept
        std::vector<uint32_t> lbp_caddr;
        if (!I->wide) {
            std::vector<int32_t> first(m), start((size_t)n + 1, 0);
            for (int32_t a = 0; a < m; ++a) {
                int32_t mv = n;
                for (int32_t p = clause_ptr[a]; p < clause_ptr[a + 1]; ++p)
                    mv = std::min(mv, std::abs(lits[p]) - 1);
                first[a] = mv;
                ++start[(size_t)mv + 1];
            }
            for (int32_t v = 0; v < n; ++v)
                start[(size_t)v + 1] += start[v];
            I->lbp_pos.assign(m, 0);
            lbp_caddr.assign((size_t)m * 4, ZERO);
            for (int32_t a = 0; a < m; ++a) {
                const int32_t t = start[first[a]]++;
                I->lbp_pos[a] = t;
                std::memcpy(&lbp_caddr[(size_t)t * 4], &clause_addr[(size_t)a * 4], 16);
            }
        }

        Arena ar;
        I->off_rec = ar.take(rec.size() * 8);
        I->rec_bytes = (uint32_t)(rec.size() * 8);  // below 2^31: N <= 65534 and degree <= 127
        I->off_chunk_var = ar.take(chunk_var.size() * 4);
        I->off_chunk_info = ar.take(chunk_info.size() * 8);
        I->off_color_chunk = ar.take(color_chunk.size() * 4);
        I->off_clause_addr = ar.take(std::max<size_t>(clause_addr.size() * 4, 16));
        I->off_var_ptr = ar.take(vptr.size() * 4);
        I->off_var_cl = ar.take(std::max<size_t>(vcl.size() * 4, 4));
        if (!I->wide) {
            I->off_lbp_caddr = ar.take(std::max<size_t>(lbp_caddr.size() * 4, 16));
            I->off_lbp_pos = ar.take(std::max<size_t>(I->lbp_pos.size() * 4, 4));
        }
        if (I->wide) {
            I->off_wrec = ar.take(std::max<size_t>(wrec.size() * sizeof(uint4), 16));
            I->off_worder = ar.take((size_t)n * 4);
            I->off_wclass = ar.take(I->color_ptr.size() * 4);
        }
        I->arena_bytes = align_up(ar.size, 256);
        I->image.assign(I->arena_bytes, 0);
        auto put = [&](size_t off, const void *src, size_t bytes) {
            if (bytes)
                std::memcpy(I->image.data() + off, src, bytes);
        };
        put(I->off_rec, rec.data(), rec.size() * 8);
        put(I->off_chunk_var, chunk_var.data(), chunk_var.size() * 4);
        put(I->off_chunk_info, chunk_info.data(), chunk_info.size() * 8);
        put(I->off_color_chunk, color_chunk.data(), color_chunk.size() * 4);
        put(I->off_clause_addr, clause_addr.data(), clause_addr.size() * 4);
        put(I->off_var_ptr, vptr.data(), vptr.size() * 4);
        put(I->off_var_cl, vcl.data(), vcl.size() * 4);
        if (!I->wide) {
            put(I->off_lbp_caddr, lbp_caddr.data(), lbp_caddr.size() * 4);
            put(I->off_lbp_pos, I->lbp_pos.data(), I->lbp_pos.size() * 4);
        }
        if (I->wide) {
            put(I->off_wrec, wrec.data(), wrec.size() * sizeof(uint4));
            put(I->off_worder, I->order.data(), (size_t)n * 4);
            put(I->off_wclass, I->color_ptr.data(), I->color_ptr.size() * 4);
        }
        *out = I.release();
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    } catch (...) {
        return fail(NMC_ERR_INVALID, "unexpected failure in nmc_ksat_load");
    }
}

int nmc_qap_load(int32_t n, const int32_t *flow, const int32_t *dist, nmc_instance **out) {
    try {
        if (!out)
            return fail(NMC_ERR_INVALID, "out is NULL");
        *out = nullptr;
        if (!flow || !dist)
            return fail(NMC_ERR_INVALID, "flow/dist is NULL");
        if (n < 2 || n > kQapMaxN)
            return fail(NMC_ERR_UNSUPPORTED, "n = %d outside [2, %d]", n, kQapMaxN);
        int32_t fmax = 0, dmax = 0;
        for (int32_t i = 0; i < n; ++i)
            for (int32_t j = 0; j < n; ++j) {
                const int32_t f = flow[(size_t)i * n + j], d = dist[(size_t)i * n + j];
                if (f < 0 || f > 255 || d < 0 || d > 255)
                    return fail(NMC_ERR_UNSUPPORTED, "entry (%d,%d) outside [0, 255]", i, j);
                if (f != flow[(size_t)j * n + i] || d != dist[(size_t)j * n + i])
                    return fail(NMC_ERR_INVALID, "flow/dist must be symmetric (entry %d,%d)", i, j);
                if (i == j && (f != 0 || d != 0))
                    return fail(NMC_ERR_INVALID, "flow/dist must have a zero diagonal");
                fmax = std::max(fmax, f);
                dmax = std::max(dmax, d);
            }
        std::unique_ptr<nmc_instance> I(new nmc_instance());
        I->kind = NMC_KIND_QAP;
        I->n = n;
        I->delta_bound = 2ll * (n - 2) * fmax * dmax;
        int64_t fsum = 0;
        for (size_t i = 0; i < (size_t)n * n; ++i)
            fsum += flow[i];
        I->energy_bound = fsum * dmax;
        I->qap_ha = (int32_t)(I->delta_bound >> kQapLowBits) + 1;
        Arena ar;
        I->off_F = ar.take((size_t)n * n);
        I->off_D = ar.take((size_t)n * n);
        I->arena_bytes = align_up(ar.size, 256);
        I->image.assign(I->arena_bytes, 0);
        for (size_t i = 0; i < (size_t)n * n; ++i) {
            I->image[I->off_F + i] = (uint8_t)flow[i];
            I->image[I->off_D + i] = (uint8_t)dist[i];
        }
        *out = I.release();
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    } catch (...) {
        return fail(NMC_ERR_INVALID, "unexpected failure in nmc_qap_load");
    }
}

int nmc_instance_get_info(const nmc_instance *I, nmc_instance_info *out) {
    if (!I || !out)
        return fail(NMC_ERR_INVALID, "NULL argument");
    out->kind = I->kind;
    out->n_items = I->n;
    if (I->kind == NMC_KIND_KSAT) {
        out->n_clauses = I->m;
        out->max_clause_len = I->kmax;
        out->max_degree = I->dmax;
        out->n_colors = I->n_colors;
        out->delta_bound = I->dmax;
        out->wide = I->wide ? 1 : 0;
    } else {
        out->wide = 0;
        out->n_clauses = 0;
        out->max_clause_len = 0;
        out->max_degree = I->n - 2;
        out->n_colors = 1;
        out->delta_bound = I->delta_bound;
    }
    return ok();
}

int nmc_instance_order(const nmc_instance *I, int32_t *order, int32_t *class_ptr, int32_t *n_colors) {
    if (!I)
        return fail(NMC_ERR_INVALID, "NULL instance");
    if (I->kind != NMC_KIND_KSAT)
        return fail(NMC_ERR_UNSUPPORTED, "sweep order exists for k-SAT instances only");
    if (order)
        std::memcpy(order, I->order.data(), I->order.size() * 4);
    if (class_ptr)
        std::memcpy(class_ptr, I->color_ptr.data(), I->color_ptr.size() * 4);
    if (n_colors)
        *n_colors = I->n_colors;
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// replicas
// ---------------------------------------------------------------------------

struct nmc_replicas {
    nmc_instance *inst = nullptr;
    int32_t R = 0, G = 0;
    uint64_t seed = 0;
    uint32_t sweeps_done = 0;
    uint8_t *dev = nullptr;
    size_t bytes = 0;
    KsatRepDev k{};
    QapRepDev q{};
    int32_t *scratch_energy = nullptr;  // [4G] or [R] (int64 for QAP)
    bool has_backbone = false;
    int32_t block_threads = 1024;
    int32_t gpw = 1;  // k-SAT sweep: groups of 4 replicas per workgroup (1 or 2)
    // library-owned threshold / class upload buffer
    uint8_t *tab_dev = nullptr;
    size_t tab_cap = 0;
    // energy-moment accumulators of the tempering ladder (library-owned)
    unsigned long long *pt_acc = nullptr;
    // LBP workspace (library-owned, sized for the instance on first use)
    uint8_t *lbp_dev = nullptr;
    int64_t *lbp_pin = nullptr;  // pinned host words for the per-batch readback
    // whitening workspace (library-owned): white bits, counts, passes
    uint8_t *wh_dev = nullptr;
    // LBP message-iteration kernel time (profiling)
    double lbp_ms = 0;
    int64_t lbp_iters = 0;
    // profiling
    bool profiling = false;
    double prof_ms = 0;
    int64_t prof_launches = 0;
    double prof_attempts = 0;
};

namespace {

struct ReplicaLayout {
    size_t off_xs, off_best_xs, off_energy, off_best, off_first_hit, off_cls, off_counts, off_frozen, off_tally,
        off_scratch, off_hint, off_dtab, total;
    // wide k-SAT layout
    size_t off_wx, off_wnx, off_wbx, off_wdsum, off_wflag;
    int32_t wgp, wlg;
};

ReplicaLayout replica_layout(const nmc_instance *I, int32_t R) {
    ReplicaLayout L{};
    Arena ar;
    if (I->kind == NMC_KIND_KSAT) {
        const size_t G = (size_t)(R + kGroup - 1) / kGroup;
        L.off_xs = ar.take(G * I->n);
        L.off_best_xs = ar.take(G * I->n);
        L.off_energy = ar.take(G * kGroup * 4);
        L.off_best = ar.take(G * kGroup * 4);
        L.off_first_hit = ar.take(G * kGroup * 4);
        L.off_cls = ar.take(I->n);
        L.off_counts = ar.take((size_t)I->n * 4);
        L.off_frozen = ar.take(I->n);
        L.off_tally = ar.take(64);
        L.off_scratch = ar.take(G * kGroup * 8);
        if (I->wide) {
            // rows of a power-of-two size (a row offset is a shift), at least 64
            int32_t lg = 6;
            while (((size_t)1 << lg) < G)
                ++lg;
            const size_t gp = (size_t)1 << lg, rows = (size_t)I->n + 1;
            L.wgp = (int32_t)gp;
            L.wlg = lg;
            L.off_wx = ar.take(2 * rows * gp);  // spins, then complements
            L.off_wnx = L.off_wx + rows * gp;
            L.off_wbx = ar.take(rows * gp);
            L.off_wdsum = ar.take((size_t)kWideStreams * gp * kGroup * 4);
            L.off_wflag = ar.take(gp);
        }
    } else {
        const size_t n = I->n;
        L.off_xs = ar.take((size_t)R * n);
        L.off_best_xs = ar.take((size_t)R * n);
        L.off_energy = ar.take((size_t)R * 8);
        L.off_best = ar.take((size_t)R * 8);
        L.off_first_hit = ar.take((size_t)R * 4);
        L.off_cls = ar.take(n);
        L.off_counts = ar.take(n * n * 4);
        L.off_frozen = ar.take(16);
        L.off_tally = ar.take(64);
        L.off_scratch = ar.take((size_t)R * 8);
        L.off_hint = ar.take((size_t)R);
        L.off_dtab = ar.take((size_t)R * (n * (n - 1) / 2) * 4);  // table-mode swap deltas
    }
    L.total = align_up(ar.size, 256);
    return L;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

int ensure_tab(nmc_replicas *P, size_t bytes) {
    if (bytes <= P->tab_cap)
        return NMC_OK;
    if (P->tab_dev) {
        HIP_OR_FAIL(hipDeviceSynchronize());
        HIP_OR_FAIL(hipFree(P->tab_dev));
        P->tab_dev = nullptr;
        P->tab_cap = 0;
    }
    size_t cap = std::max<size_t>(bytes, 1 << 20);
    HIP_OR_FAIL(hipMalloc(&P->tab_dev, cap));
    P->tab_cap = cap;
    return NMC_OK;
}

int reset_after_state(nmc_replicas *P, hipStream_t s) {
    nmc_instance *I = P->inst;
    if (I->kind == NMC_KIND_KSAT) {
        if (I->wide)
            HIP_OR_FAIL(ksat_launch_wide_recount(I->ksat_dev(), P->k, P->k.energy, s));
        else
            HIP_OR_FAIL(ksat_launch_recount(I->ksat_dev(), P->k.xs, P->G, P->R, P->k.energy, s));
        HIP_OR_FAIL(ksat_launch_reset_tallies(P->k, I->n, s));
    } else {
        HIP_OR_FAIL(qap_launch_cost(I->qap_dev(), P->q.perm, P->R, P->q.cost, s));
        HIP_OR_FAIL(qap_launch_reset_tallies(P->q, I->n, s));
    }
    return NMC_OK;
}

}  // namespace

extern "C" {

int nmc_footprint(const nmc_instance *I, int32_t n_replicas, size_t *instance_bytes, size_t *replica_bytes) {
    if (!I)
        return fail(NMC_ERR_INVALID, "NULL instance");
    if (n_replicas < 1 || n_replicas > (1 << 20))
        return fail(NMC_ERR_INVALID, "n_replicas %d outside [1, 2^20]", n_replicas);
    if (instance_bytes)
        *instance_bytes = I->arena_bytes;
    if (replica_bytes)
        *replica_bytes = replica_layout(I, n_replicas).total;
    return ok();
}

int nmc_instance_bind(nmc_instance *I, void *dev_buf, size_t bytes, void *stream) {
    if (!I || !dev_buf)
        return fail(NMC_ERR_INVALID, "NULL argument");
    if (bytes < I->arena_bytes)
        return fail(NMC_ERR_SIZE, "instance buffer has %zu bytes, needs %zu", bytes, I->arena_bytes);
    if (reinterpret_cast<uintptr_t>(dev_buf) % 256)
        return fail(NMC_ERR_INVALID, "instance buffer must be 256-byte aligned");
    if (I->live_replicas)
        return fail(NMC_ERR_STATE, "instance has live replica sets");
    hipStream_t s = as_stream(stream);
    HIP_OR_FAIL(hipMemcpyAsync(dev_buf, I->image.data(), I->arena_bytes, hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    I->dev = static_cast<uint8_t *>(dev_buf);
    return ok();
}

void nmc_instance_free(nmc_instance *I) {
    if (I && I->refs.fetch_sub(1) == 1)
        delete I;
}

int nmc_replicas_create(nmc_instance *I, int32_t n_replicas, uint64_t seed, void *dev_buf, size_t bytes,
                        void *stream, nmc_replicas **out) {
    try {
        if (!out)
            return fail(NMC_ERR_INVALID, "out is NULL");
        *out = nullptr;
        if (!I || !dev_buf)
            return fail(NMC_ERR_INVALID, "NULL argument");
        if (!I->dev)
            return fail(NMC_ERR_STATE, "instance is not bound to device memory");
        if (n_replicas < 1 || n_replicas > (1 << 20))
            return fail(NMC_ERR_INVALID, "n_replicas %d outside [1, 2^20]", n_replicas);
        if (reinterpret_cast<uintptr_t>(dev_buf) % 256)
            return fail(NMC_ERR_INVALID, "replica buffer must be 256-byte aligned");
        const ReplicaLayout L = replica_layout(I, n_replicas);
        if (bytes < L.total)
            return fail(NMC_ERR_SIZE, "replica buffer has %zu bytes, needs %zu", bytes, L.total);
        if (I->kind == NMC_KIND_KSAT && I->wide && 2 * ((size_t)I->n + 1) * (size_t)L.wgp >= ((size_t)1 << 31))
            return fail(NMC_ERR_CAPACITY,
                        "wide spin tables of %d variables x %d groups exceed 2 GiB (buffer offsets are 32-bit): use "
                        "fewer replicas per set", I->n, L.wgp);
        std::unique_ptr<nmc_replicas> P(new nmc_replicas());
        P->inst = I;
        P->R = n_replicas;
        P->G = (n_replicas + kGroup - 1) / kGroup;
        P->seed = seed;
        P->dev = static_cast<uint8_t *>(dev_buf);
        P->bytes = bytes;
        uint8_t *b = P->dev;
        hipStream_t s = as_stream(stream);
        const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
        if (I->kind == NMC_KIND_KSAT) {
            KsatRepDev &k = P->k;
            k.xs = b + L.off_xs;
            k.best_xs = b + L.off_best_xs;
            k.energy = reinterpret_cast<int32_t *>(b + L.off_energy);
            k.best = reinterpret_cast<int32_t *>(b + L.off_best);
            k.first_hit = reinterpret_cast<int32_t *>(b + L.off_first_hit);
            k.cls = b + L.off_cls;
            k.counts = reinterpret_cast<int32_t *>(b + L.off_counts);
            k.frozen = b + L.off_frozen;
            k.tally = reinterpret_cast<int32_t *>(b + L.off_tally);
            k.accepted = reinterpret_cast<unsigned long long *>(b + L.off_tally + 32);
            k.n_rep = n_replicas;
            k.n_groups = P->G;
            if (I->wide) {
                k.wx = b + L.off_wx;
                k.wnx = b + L.off_wnx;
                k.wbx = b + L.off_wbx;
                k.wdsum = reinterpret_cast<int32_t *>(b + L.off_wdsum);
                k.wflag = b + L.off_wflag;
                k.wgp = L.wgp;
                k.wlg = L.wlg;
                // the per-stream energy changes start (and end every sweep) at zero
                HIP_OR_FAIL(hipMemsetAsync(k.wdsum, 0, (size_t)kWideStreams * L.wgp * kGroup * 4, s));
                HIP_OR_FAIL(hipMemsetAsync(k.wflag, 0, (size_t)L.wgp, s));
            }
            P->scratch_energy = reinterpret_cast<int32_t *>(b + L.off_scratch);
            HIP_OR_FAIL(hipMemsetAsync(b + L.off_energy, 0, L.off_first_hit + (size_t)P->G * kGroup * 4 - L.off_energy, s));
            HIP_OR_FAIL(hipMemsetAsync(b + L.off_tally, 0, 64, s));
            HIP_OR_FAIL(ksat_launch_init(I->ksat_dev(), k, key0, key1, s));
        } else {
            QapRepDev &q = P->q;
            q.perm = b + L.off_xs;
            q.best_perm = b + L.off_best_xs;
            q.cost = reinterpret_cast<int64_t *>(b + L.off_energy);
            q.best = reinterpret_cast<int64_t *>(b + L.off_best);
            q.first_hit = reinterpret_cast<int32_t *>(b + L.off_first_hit);
            q.cls = b + L.off_cls;
            q.freq = reinterpret_cast<int32_t *>(b + L.off_counts);
            q.tally = reinterpret_cast<int32_t *>(b + L.off_tally);
            q.accepted = reinterpret_cast<unsigned long long *>(b + L.off_tally + 32);
            q.rows_hint = b + L.off_hint;
            q.dtab = reinterpret_cast<int32_t *>(b + L.off_dtab);
            q.n_rep = n_replicas;
            P->scratch_energy = reinterpret_cast<int32_t *>(b + L.off_scratch);
            HIP_OR_FAIL(hipMemsetAsync(q.rows_hint, 0, (size_t)n_replicas, s));
            HIP_OR_FAIL(hipMemsetAsync(b + L.off_tally, 0, 64, s));
            HIP_OR_FAIL(qap_launch_init(I->qap_dev(), q, key0, key1, s));
        }
        int rc = reset_after_state(P.get(), s);
        if (rc)
            return rc;
        HIP_OR_FAIL(hipStreamSynchronize(s));
        I->live_replicas++;
        I->refs++;
        *out = P.release();
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

void nmc_replicas_free(nmc_replicas *P) {
    if (!P)
        return;
    if (P->tab_dev || P->pt_acc || P->lbp_dev || P->wh_dev)
        (void)hipDeviceSynchronize();
    if (P->wh_dev)
        (void)hipFree(P->wh_dev);
    if (P->tab_dev)
        (void)hipFree(P->tab_dev);
    if (P->pt_acc)
        (void)hipFree(P->pt_acc);
    if (P->lbp_dev)
        (void)hipFree(P->lbp_dev);
    if (P->lbp_pin)
        (void)hipHostFree(P->lbp_pin);
    nmc_instance *I = P->inst;
    delete P;
    if (I) {
        I->live_replicas--;
        if (I->refs.fetch_sub(1) == 1)
            delete I;
    }
}

// ext_buf != nullptr: the thresholds (and a host class array) go to ext_buf
// (device, ext_cap bytes) and nothing is allocated; a call that needs more
// fails with NMC_ERR_CAPACITY before any work is queued.  Otherwise they go to
// the replica set's own upload buffer, allocated or grown as needed.
static int anneal_impl(nmc_replicas *P, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
                       const uint8_t *class_of, int64_t target, void *stream, uint8_t *ext_buf = nullptr,
                       size_t ext_cap = 0) {
    if (!P || !beta)
        return fail(NMC_ERR_INVALID, "NULL argument");
    nmc_instance *I = P->inst;
    if (!I->dev)
        return fail(NMC_ERR_STATE, "instance is not bound");
    if (n_classes < 1 || n_classes > kMaxClasses)
        return fail(NMC_ERR_INVALID, "n_classes %d outside [1, %d]", n_classes, kMaxClasses);
    if (n_sweeps < 0)
        return fail(NMC_ERR_INVALID, "n_sweeps must be >= 0");
    if ((uint64_t)P->sweeps_done + (uint64_t)n_sweeps > 0xFFFFFFFFull)
        return fail(NMC_ERR_INVALID, "sweep counter would pass 2^32 - 1");
    for (int64_t i = 0; i < (int64_t)n_classes * n_sweeps; ++i)
        if (!std::isfinite(beta[i]) || beta[i] < 0)
            return fail(NMC_ERR_INVALID, "beta[%lld] = %g is not finite and >= 0", (long long)i, beta[i]);
    const int32_t nitems = I->n;
    if (profile == NMC_PROFILE_HOST) {
        if (!class_of)
            return fail(NMC_ERR_INVALID, "class_of is NULL for NMC_PROFILE_HOST");
        for (int32_t i = 0; i < nitems; ++i)
            if (class_of[i] >= n_classes)
                return fail(NMC_ERR_INVALID, "class_of[%d] = %d >= n_classes", i, class_of[i]);
    } else if (profile == NMC_PROFILE_BACKBONE) {
        if (!P->has_backbone)
            return fail(NMC_ERR_STATE, "no backbone estimate yet");
        if (n_classes < 2)
            return fail(NMC_ERR_INVALID, "the backbone profile needs n_classes >= 2");
    } else if (profile != NMC_PROFILE_HOMOGENEOUS) {
        return fail(NMC_ERR_INVALID, "unknown profile %d", profile);
    }
    hipStream_t s = as_stream(stream);
    const bool ksat = I->kind == NMC_KIND_KSAT;
    const int32_t stride = ksat ? I->dmax + 1 : qap_row_words(I->qap_ha);
    // (wide k-SAT sweeps hold only the threshold rows in LDS)
    const size_t lds = ksat ? (I->wide ? (size_t)n_classes * stride * 4 : ksat_sweep_lds_bytes(I->n, n_classes, stride))
                            : qap_sweep_lds_bytes(I->n, n_classes, stride);
    if (lds > kLdsBytes)
        return fail(NMC_ERR_CAPACITY, "sweep needs %zu bytes of LDS (limit %zu)", lds, kLdsBytes);
    if (ksat && I->n > 0 && target > INT32_MAX)
        target = INT32_MAX;

    // thresholds for every (sweep, class) of this call
    const size_t words = (size_t)n_sweeps * n_classes * stride;
    const size_t tab_bytes = align_up(std::max<size_t>(words * 4, 4), 256);
    const size_t cls_bytes = profile == NMC_PROFILE_HOST ? align_up(nitems, 256) : 0;
    uint8_t *up = ext_buf;
    if (ext_buf) {
        if (tab_bytes + cls_bytes > ext_cap)
            return fail(NMC_ERR_CAPACITY,
                        "this call's thresholds need %zu bytes (%d sweeps x %d classes x %d words%s), the "
                        "allocation-free buffer holds %zu: split the schedule into shorter calls",
                        tab_bytes + cls_bytes, n_sweeps, n_classes, stride,
                        cls_bytes ? " + the class array" : "", ext_cap);
    } else {
        int rc = ensure_tab(P, tab_bytes + cls_bytes);
        if (rc)
            return rc;
        up = P->tab_dev;
    }
    std::vector<uint32_t> tab(std::max<size_t>(words, 1));
    bool mono = true;  // every QAP row's T never increases
    for (int32_t sw = 0; sw < n_sweeps; ++sw)
        for (int32_t c = 0; c < n_classes; ++c) {
            const double b = beta[(size_t)c * n_sweeps + sw];
            uint32_t *row = tab.data() + ((size_t)sw * n_classes + c) * stride;
            if (ksat) {
                row[0] = 0xFFFFFFFFu;
                for (int32_t d = 1; d < stride; ++d)
                    row[d] = threshold(b, d);
            } else {
                mono = qap_fill_row(row, b, I->qap_ha) && mono;
            }
        }
    // the upload waits for earlier work on the stream that still reads the
    // buffer: pageable host-to-device copies are ordered in the stream
    HIP_OR_FAIL(hipMemcpyAsync(up, tab.data(), words * 4, hipMemcpyHostToDevice, s));
    const uint8_t *cls_dev = nullptr;
    if (profile == NMC_PROFILE_HOST) {
        HIP_OR_FAIL(hipMemcpyAsync(up + tab_bytes, class_of, nitems, hipMemcpyHostToDevice, s));
        cls_dev = up + tab_bytes;
    } else if (profile == NMC_PROFILE_BACKBONE) {
        cls_dev = ksat ? P->k.cls : P->q.cls;
    }

    // the allocation-free variant creates no timing events
    const bool timed = P->profiling && !ext_buf;
    ScopedEvents evs;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        HIP_OR_FAIL(evs.create(&e0));
        HIP_OR_FAIL(evs.create(&e1));
        HIP_OR_FAIL(hipEventRecord(e0, s));
    }
    if (ksat) {
        SweepCall C{};
        C.tab = reinterpret_cast<const uint32_t *>(up);
        C.var_cls = cls_dev;
        C.n_classes = n_classes;
        C.stride = stride;
        C.n_sweeps = n_sweeps;
        C.sweep_words = n_classes * stride;
        C.t0 = P->sweeps_done;
        C.target = (int32_t)std::max<int64_t>(std::min<int64_t>(target, INT32_MAX), INT32_MIN);
        C.check_start = 1;
        C.key0 = (uint32_t)P->seed;
        C.key1 = (uint32_t)(P->seed >> 32);
        C.gpw = P->gpw;
        if (I->wide) {
            // variable-major spins for the call's sweeps, back to the
            // group-major state afterwards
            const KsatDev D = I->ksat_dev();
            HIP_OR_FAIL(ksat_launch_wide_pack(D, P->k, false, s));
            std::vector<int32_t> csize(I->n_colors);
            for (int32_t c = 0; c < I->n_colors; ++c)
                csize[c] = I->color_ptr[c + 1] - I->color_ptr[c];
            HIP_OR_FAIL(ksat_launch_wide_sweeps(D, P->k, C, csize.data(), s));
            HIP_OR_FAIL(ksat_launch_wide_pack(D, P->k, true, s));
        } else {
            HIP_OR_FAIL(ksat_launch_sweep(I->ksat_dev(), P->k, C, P->block_threads, s));
        }
    } else {
        QapCall C{};
        C.tab = reinterpret_cast<const uint32_t *>(up);
        C.fac_cls = cls_dev;
        C.n_classes = n_classes;
        C.stride = stride;
        C.n_sweeps = n_sweeps;
        C.sweep_words = n_classes * stride;
        C.t0 = P->sweeps_done;
        C.target = target;
        C.check_start = 1;
        C.rows = qap_rows_setting();
        C.tab_allow = qap_tab_setting();
        C.quad_allow = qap_quad_setting();
        C.dstar = mono && qap_dstar_setting();
        C.key0 = (uint32_t)P->seed;
        C.key1 = (uint32_t)(P->seed >> 32);
        HIP_OR_FAIL(qap_launch_sweep(I->qap_dev(), P->q, C, 256, s));
    }
    if (timed) {
        HIP_OR_FAIL(hipEventRecord(e1, s));
        HIP_OR_FAIL(hipEventSynchronize(e1));
        float ms = 0;
        HIP_OR_FAIL(hipEventElapsedTime(&ms, e0, e1));
        P->prof_ms += ms;
        P->prof_launches += 1;
        const double per_sweep = ksat ? (double)P->R * I->n : (double)P->R * I->n * (I->n - 1) / 2.0;
        P->prof_attempts += per_sweep * n_sweeps;
    }
    P->sweeps_done += (uint32_t)n_sweeps;
    return ok();
}

int nmc_anneal(nmc_replicas *P, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
               const uint8_t *class_of, int64_t target, void *stream) {
    try {
        return anneal_impl(P, beta, n_classes, n_sweeps, profile, class_of, target, stream);
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_reanneal(nmc_replicas *P, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
                 const uint8_t *class_of, int64_t target, void *stream) {
    return nmc_anneal(P, beta, n_classes, n_sweeps, profile, class_of, target, stream);
}

}  // extern "C"

int nmc::anneal_into(nmc_replicas *P, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
                     const uint8_t *class_of, int64_t target, void *stream, uint8_t *buf, size_t cap) {
    if (!buf)
        return fail(NMC_ERR_INVALID, "NULL upload buffer");
    try {
        return anneal_impl(P, beta, n_classes, n_sweeps, profile, class_of, target, stream, buf, cap);
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

extern "C" {

int nmc_estimate_backbone(nmc_replicas *P, int32_t thr_num, int32_t thr_den, int32_t expand, uint8_t *class_out,
                          int32_t *counts_out, void *stream) {
    if (!P)
        return fail(NMC_ERR_INVALID, "NULL replicas");
    if (thr_den <= 0 || thr_num <= 0 || thr_num > thr_den)
        return fail(NMC_ERR_INVALID, "need 0 < thr_num <= thr_den");
    nmc_instance *I = P->inst;
    hipStream_t s = as_stream(stream);
    if (I->kind == NMC_KIND_KSAT) {
        HIP_OR_FAIL(ksat_launch_backbone(I->ksat_dev(), P->k, thr_num, thr_den, expand ? 1 : 0, s));
        if (class_out)
            HIP_OR_FAIL(hipMemcpyAsync(class_out, P->k.cls, I->n, hipMemcpyDeviceToHost, s));
        if (counts_out)
            HIP_OR_FAIL(hipMemcpyAsync(counts_out, P->k.counts, (size_t)I->n * 4, hipMemcpyDeviceToHost, s));
    } else {
        HIP_OR_FAIL(qap_launch_backbone(I->qap_dev(), P->q, thr_num, thr_den, s));
        if (class_out)
            HIP_OR_FAIL(hipMemcpyAsync(class_out, P->q.cls, I->n, hipMemcpyDeviceToHost, s));
        if (counts_out)
            HIP_OR_FAIL(hipMemcpyAsync(counts_out, P->q.freq, (size_t)I->n * I->n * 4, hipMemcpyDeviceToHost, s));
    }
    if (class_out || counts_out)
        HIP_OR_FAIL(hipStreamSynchronize(s));
    P->has_backbone = true;
    return ok();
}

int nmc_best_energy(nmc_replicas *P, int64_t *best, int32_t *n_at_zero, int64_t *best_per_replica,
                    int64_t *energy_per_replica, int32_t *first_hit, void *stream) {
    if (!P)
        return fail(NMC_ERR_INVALID, "NULL replicas");
    try {
        nmc_instance *I = P->inst;
        hipStream_t s = as_stream(stream);
        const int32_t R = P->R;
        if (I->kind == NMC_KIND_KSAT) {
            HIP_OR_FAIL(ksat_launch_tally(P->k, s));
            int32_t t[2];
            std::vector<int32_t> b(R), e(R), f(R);
            HIP_OR_FAIL(hipMemcpyAsync(t, P->k.tally, 8, hipMemcpyDeviceToHost, s));
            if (best_per_replica)
                HIP_OR_FAIL(hipMemcpyAsync(b.data(), P->k.best, (size_t)R * 4, hipMemcpyDeviceToHost, s));
            if (energy_per_replica)
                HIP_OR_FAIL(hipMemcpyAsync(e.data(), P->k.energy, (size_t)R * 4, hipMemcpyDeviceToHost, s));
            if (first_hit)
                HIP_OR_FAIL(hipMemcpyAsync(f.data(), P->k.first_hit, (size_t)R * 4, hipMemcpyDeviceToHost, s));
            HIP_OR_FAIL(hipStreamSynchronize(s));
            if (best)
                *best = t[0];
            if (n_at_zero)
                *n_at_zero = t[1];
            for (int32_t r = 0; r < R; ++r) {
                if (best_per_replica)
                    best_per_replica[r] = b[r];
                if (energy_per_replica)
                    energy_per_replica[r] = e[r];
                if (first_hit)
                    first_hit[r] = f[r];
            }
        } else {
            HIP_OR_FAIL(qap_launch_tally(P->q, s));
            int32_t t[4];
            HIP_OR_FAIL(hipMemcpyAsync(t, P->q.tally, 16, hipMemcpyDeviceToHost, s));
            if (best_per_replica)
                HIP_OR_FAIL(hipMemcpyAsync(best_per_replica, P->q.best, (size_t)R * 8, hipMemcpyDeviceToHost, s));
            if (energy_per_replica)
                HIP_OR_FAIL(hipMemcpyAsync(energy_per_replica, P->q.cost, (size_t)R * 8, hipMemcpyDeviceToHost, s));
            if (first_hit)
                HIP_OR_FAIL(hipMemcpyAsync(first_hit, P->q.first_hit, (size_t)R * 4, hipMemcpyDeviceToHost, s));
            HIP_OR_FAIL(hipStreamSynchronize(s));
            int64_t mn;
            std::memcpy(&mn, t, 8);
            if (best)
                *best = mn;
            if (n_at_zero)
                *n_at_zero = t[2];
        }
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_recount(nmc_replicas *P, int64_t *energy_out, void *stream) {
    if (!P || !energy_out)
        return fail(NMC_ERR_INVALID, "NULL argument");
    try {
        nmc_instance *I = P->inst;
        hipStream_t s = as_stream(stream);
        if (I->kind == NMC_KIND_KSAT) {
            if (I->wide)
                HIP_OR_FAIL(ksat_launch_wide_recount(I->ksat_dev(), P->k, P->scratch_energy, s));
            else
                HIP_OR_FAIL(ksat_launch_recount(I->ksat_dev(), P->k.xs, P->G, P->R, P->scratch_energy, s));
            std::vector<int32_t> e(P->R);
            HIP_OR_FAIL(hipMemcpyAsync(e.data(), P->scratch_energy, (size_t)P->R * 4, hipMemcpyDeviceToHost, s));
            HIP_OR_FAIL(hipStreamSynchronize(s));
            for (int32_t r = 0; r < P->R; ++r)
                energy_out[r] = e[r];
        } else {
            int64_t *tmp = reinterpret_cast<int64_t *>(P->scratch_energy);
            HIP_OR_FAIL(qap_launch_cost(I->qap_dev(), P->q.perm, P->R, tmp, s));
            HIP_OR_FAIL(hipMemcpyAsync(energy_out, tmp, (size_t)P->R * 8, hipMemcpyDeviceToHost, s));
            HIP_OR_FAIL(hipStreamSynchronize(s));
        }
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_get_state(nmc_replicas *P, int32_t which, uint8_t *host_out, size_t bytes, void *stream) {
    if (!P || !host_out)
        return fail(NMC_ERR_INVALID, "NULL argument");
    if (which != NMC_STATE_CURRENT && which != NMC_STATE_BEST)
        return fail(NMC_ERR_INVALID, "which must be NMC_STATE_CURRENT or NMC_STATE_BEST");
    try {
        nmc_instance *I = P->inst;
        const size_t need = (size_t)P->R * I->n;
        if (bytes < need)
            return fail(NMC_ERR_SIZE, "state buffer has %zu bytes, needs %zu", bytes, need);
        hipStream_t s = as_stream(stream);
        if (I->kind == NMC_KIND_KSAT) {
            const uint8_t *src = which == NMC_STATE_BEST ? P->k.best_xs : P->k.xs;
            std::vector<uint8_t> packed((size_t)P->G * I->n);
            HIP_OR_FAIL(hipMemcpyAsync(packed.data(), src, packed.size(), hipMemcpyDeviceToHost, s));
            HIP_OR_FAIL(hipStreamSynchronize(s));
            for (int32_t r = 0; r < P->R; ++r) {
                const uint8_t *row = packed.data() + (size_t)(r / kGroup) * I->n;
                uint8_t *dst = host_out + (size_t)r * I->n;
                for (int32_t v = 0; v < I->n; ++v)
                    dst[v] = (row[v] >> (r % kGroup)) & 1u;
            }
        } else {
            const uint8_t *src = which == NMC_STATE_BEST ? P->q.best_perm : P->q.perm;
            HIP_OR_FAIL(hipMemcpyAsync(host_out, src, need, hipMemcpyDeviceToHost, s));
            HIP_OR_FAIL(hipStreamSynchronize(s));
        }
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_set_state(nmc_replicas *P, const uint8_t *host_in, size_t bytes, uint32_t sweeps_done, void *stream) {
    if (!P || !host_in)
        return fail(NMC_ERR_INVALID, "NULL argument");
    try {
        nmc_instance *I = P->inst;
        const size_t need = (size_t)P->R * I->n;
        if (bytes < need)
            return fail(NMC_ERR_SIZE, "state buffer has %zu bytes, needs %zu", bytes, need);
        hipStream_t s = as_stream(stream);
        if (I->kind == NMC_KIND_KSAT) {
            for (size_t i = 0; i < need; ++i)
                if (host_in[i] > 1)
                    return fail(NMC_ERR_INVALID, "k-SAT state entries must be 0 or 1");
            std::vector<uint8_t> packed((size_t)P->G * I->n, 0);
            for (int32_t r = 0; r < P->R; ++r) {
                uint8_t *row = packed.data() + (size_t)(r / kGroup) * I->n;
                const uint8_t *src = host_in + (size_t)r * I->n;
                for (int32_t v = 0; v < I->n; ++v)
                    row[v] |= (uint8_t)((src[v] & 1u) << (r % kGroup));
            }
            HIP_OR_FAIL(hipMemcpyAsync(P->k.xs, packed.data(), packed.size(), hipMemcpyHostToDevice, s));
        } else {
            std::vector<uint8_t> seen(I->n);
            for (int32_t r = 0; r < P->R; ++r) {
                std::fill(seen.begin(), seen.end(), 0);
                for (int32_t f = 0; f < I->n; ++f) {
                    const uint8_t l = host_in[(size_t)r * I->n + f];
                    if (l >= I->n || seen[l])
                        return fail(NMC_ERR_INVALID, "row %d is not a permutation", r);
                    seen[l] = 1;
                }
            }
            HIP_OR_FAIL(hipMemcpyAsync(P->q.perm, host_in, need, hipMemcpyHostToDevice, s));
        }
        int rc = reset_after_state(P, s);
        if (rc)
            return rc;
        HIP_OR_FAIL(hipStreamSynchronize(s));
        P->sweeps_done = sweeps_done;
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_replicas_info(const nmc_replicas *P, int32_t *n_replicas, uint64_t *seed, uint32_t *sweeps_done) {
    if (!P)
        return fail(NMC_ERR_INVALID, "NULL replicas");
    if (n_replicas)
        *n_replicas = P->R;
    if (seed)
        *seed = P->seed;
    if (sweeps_done)
        *sweeps_done = P->sweeps_done;
    return ok();
}

int nmc_set_tuning(nmc_replicas *P, int32_t block_threads) {
    if (!P)
        return fail(NMC_ERR_INVALID, "NULL replicas");
    if (block_threads == 0)
        block_threads = 1024;
    if (block_threads < 64 || block_threads > 1024 || block_threads % 64)
        return fail(NMC_ERR_INVALID, "block_threads must be a multiple of 64 in [64, 1024]");
    P->block_threads = block_threads;
    return ok();
}

int nmc_set_replicas_per_workgroup(nmc_replicas *P, int32_t reps) {
    if (!P)
        return fail(NMC_ERR_INVALID, "NULL replicas");
    if (P->inst->kind != NMC_KIND_KSAT)
        return fail(NMC_ERR_UNSUPPORTED, "replicas per workgroup is a k-SAT setting");
    if (reps == 0)
        reps = kGroup;
    if (reps != kGroup && reps != 2 * kGroup)
        return fail(NMC_ERR_INVALID, "replicas per workgroup must be 4 or 8");
    P->gpw = reps / kGroup;
    return ok();
}

int nmc_get_tuning(const nmc_replicas *P, int32_t *block_threads, int32_t *reps_per_workgroup) {
    if (!P)
        return fail(NMC_ERR_INVALID, "NULL replicas");
    if (block_threads)
        *block_threads = P->block_threads;
    if (reps_per_workgroup)
        *reps_per_workgroup = P->inst->kind == NMC_KIND_KSAT ? P->gpw * kGroup : 0;
    return ok();
}

int nmc_set_profiling(nmc_replicas *P, int32_t enable) {
    if (!P)
        return fail(NMC_ERR_INVALID, "NULL replicas");
    P->profiling = enable != 0;
    return ok();
}

// ---------------------------------------------------------------------------
// parallel tempering (appendix A)
// ---------------------------------------------------------------------------

static int pt_run_impl(nmc_replicas *P, const double *beta, int32_t n_temps, int32_t n_rounds,
                       int32_t sweeps_per_round, int32_t first_parity, int64_t target, int64_t *accepted,
                       int64_t *attempted, void *stream) {
    if (!P || !beta)
        return fail(NMC_ERR_INVALID, "NULL argument");
    nmc_instance *I = P->inst;
    if (!I->dev)
        return fail(NMC_ERR_STATE, "instance is not bound");
    if (I->kind == NMC_KIND_KSAT && I->wide)
        return fail(NMC_ERR_UNSUPPORTED, "%s is not available for wide k-SAT instances (more than %d variables)", "tempering", kMaxVars);
    const bool ksat = I->kind == NMC_KIND_KSAT;
    if (n_temps < 1 || P->R % n_temps)
        return fail(NMC_ERR_INVALID, "n_temps = %d must be >= 1 and divide the %d replicas", n_temps, P->R);
    const int32_t chains = P->R / n_temps;
    const int32_t unit = ksat ? kGroup : kQapRepPerBlock;
    if (chains % unit)
        return fail(NMC_ERR_INVALID, "replicas / n_temps = %d chains must be a multiple of %d", chains, unit);
    if (n_rounds < 0 || sweeps_per_round < 1)
        return fail(NMC_ERR_INVALID, "need n_rounds >= 0 and sweeps_per_round >= 1");
    if (first_parity != 0 && first_parity != 1)
        return fail(NMC_ERR_INVALID, "first_parity must be 0 or 1");
    if ((uint64_t)P->sweeps_done + (uint64_t)n_rounds * (uint64_t)sweeps_per_round > 0xFFFFFFFFull)
        return fail(NMC_ERR_INVALID, "sweep counter would pass 2^32 - 1");
    for (int32_t i = 0; i < n_temps; ++i) {
        if (!std::isfinite(beta[i]) || beta[i] < 0)
            return fail(NMC_ERR_INVALID, "beta[%d] = %g is not finite and >= 0", i, beta[i]);
        if (i > 0 && !(beta[i] > beta[i - 1]))
            return fail(NMC_ERR_INVALID, "the ladder must increase strictly (beta[%d] <= beta[%d])", i, i - 1);
    }
    hipStream_t s = as_stream(stream);
    const int32_t stride = ksat ? I->dmax + 1 : qap_row_words(I->qap_ha);
    const size_t lds = ksat ? ksat_sweep_lds_bytes(I->n, 1, stride) : qap_sweep_lds_bytes(I->n, 1, stride);
    if (lds > kLdsBytes)
        return fail(NMC_ERR_CAPACITY, "sweep needs %zu bytes of LDS (limit %zu)", lds, kLdsBytes);
    if (ksat && target > INT32_MAX)
        target = INT32_MAX;

    // sweep thresholds, one row per ladder position
    std::vector<uint32_t> tab((size_t)n_temps * stride);
    bool mono = true;  // every QAP row's T never increases
    for (int32_t i = 0; i < n_temps; ++i) {
        uint32_t *row = tab.data() + (size_t)i * stride;
        if (ksat) {
            row[0] = 0xFFFFFFFFu;
            for (int32_t d = 1; d < stride; ++d)
                row[d] = threshold(beta[i], d);
        } else {
            mono = qap_fill_row(row, beta[i], I->qap_ha) && mono;
        }
    }
    // exchange thresholds of every neighbour pair: the high digit runs until
    // it reaches zero (every larger gap then has threshold zero) or covers the
    // largest possible energy gap; the 1024 low-digit words follow it
    const int32_t npairs = n_temps - 1;
    std::vector<int64_t> off(std::max(npairs, 1));
    std::vector<int32_t> len(std::max(npairs, 1));
    const size_t xtab_at = tab.size();
    const int64_t hmax = I->energy_bound >> kQapLowBits;
    for (int32_t i = 0; i < npairs; ++i) {
        const double db = beta[i + 1] - beta[i];
        off[i] = (int64_t)(tab.size() - xtab_at);
        tab.push_back(0xFFFFFFFFu);
        for (int64_t h = 1; h <= hmax; ++h) {
            const uint32_t v = threshold(db, h << kQapLowBits);
            if (!v)
                break;
            tab.push_back(v);
            if (tab.size() - xtab_at > ((size_t)1 << 26))
                return fail(NMC_ERR_CAPACITY, "ladder step %d (%g) is too fine for the energy range", i, db);
        }
        len[i] = (int32_t)(tab.size() - xtab_at - off[i]);
        tab.push_back(0xFFFFFFFFu);
        for (int32_t l = 1; l < (1 << kQapLowBits); ++l)
            tab.push_back(threshold(db, l));
    }
    const size_t tab_bytes = align_up(tab.size() * 4, 256);
    const size_t off_bytes = align_up(off.size() * 8, 256), len_bytes = align_up(len.size() * 4, 256);
    const size_t cnt_bytes = align_up((size_t)std::max(npairs, 1) * 8, 256);
    int rc = ensure_tab(P, tab_bytes + off_bytes + len_bytes + 2 * cnt_bytes);
    if (rc)
        return rc;
    uint8_t *base = P->tab_dev;
    HIP_OR_FAIL(hipMemcpyAsync(base, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(hipMemcpyAsync(base + tab_bytes, off.data(), off.size() * 8, hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(hipMemcpyAsync(base + tab_bytes + off_bytes, len.data(), len.size() * 4, hipMemcpyHostToDevice, s));
    unsigned long long *acc_dev = reinterpret_cast<unsigned long long *>(base + tab_bytes + off_bytes + len_bytes);
    unsigned long long *att_dev = reinterpret_cast<unsigned long long *>(base + tab_bytes + off_bytes + len_bytes +
                                                                         cnt_bytes);
    HIP_OR_FAIL(hipMemsetAsync(acc_dev, 0, 2 * cnt_bytes, s));

    PtCall X{};
    X.tab = reinterpret_cast<const uint32_t *>(base) + xtab_at;
    X.off = reinterpret_cast<const int64_t *>(base + tab_bytes);
    X.len = reinterpret_cast<const int32_t *>(base + tab_bytes + off_bytes);
    X.accepted = acc_dev;
    X.attempted = att_dev;
    X.n_temps = n_temps;
    X.n_chains = chains;
    X.key0 = (uint32_t)P->seed;
    X.key1 = (uint32_t)(P->seed >> 32);

    ScopedEvents evs;  // (start, end) of every round's sweep launch when profiling
    std::vector<hipEvent_t> &ev = evs.ev;
    for (int32_t k = 0; k < n_rounds; ++k) {
        if (P->profiling) {
            hipEvent_t a = nullptr, b = nullptr;
            HIP_OR_FAIL(evs.create(&a));
            HIP_OR_FAIL(evs.create(&b));
            HIP_OR_FAIL(hipEventRecord(a, s));
        }
        if (ksat) {
            SweepCall C{};
            C.tab = reinterpret_cast<const uint32_t *>(base);
            C.var_cls = nullptr;
            C.n_classes = 1;
            C.stride = stride;
            C.n_sweeps = sweeps_per_round;
            C.sweep_words = 0;
            C.t0 = P->sweeps_done;
            C.target = (int32_t)std::max<int64_t>(std::min<int64_t>(target, INT32_MAX), INT32_MIN);
            C.check_start = 1;
            C.key0 = X.key0;
            C.key1 = X.key1;
            C.reps_per_row = chains;
            C.gpw = 1;  // each sweep workgroup at one temperature
            HIP_OR_FAIL(ksat_launch_sweep(I->ksat_dev(), P->k, C, P->block_threads, s));
        } else {
            QapCall C{};
            C.tab = reinterpret_cast<const uint32_t *>(base);
            C.fac_cls = nullptr;
            C.n_classes = 1;
            C.stride = stride;
            C.n_sweeps = sweeps_per_round;
            C.sweep_words = 0;
            C.t0 = P->sweeps_done;
            C.target = target;
            C.check_start = 1;
            C.rows = qap_rows_setting();
            C.tab_allow = qap_tab_setting();
            C.quad_allow = qap_quad_setting();
            C.dstar = mono && qap_dstar_setting();
            C.key0 = X.key0;
            C.key1 = X.key1;
            C.reps_per_row = chains;
            HIP_OR_FAIL(qap_launch_sweep(I->qap_dev(), P->q, C, 256, s));
        }
        if (P->profiling)
            HIP_OR_FAIL(hipEventRecord(ev.back(), s));
        P->sweeps_done += (uint32_t)sweeps_per_round;
        if (n_temps > 1) {
            X.parity = (first_parity + k) & 1;
            X.t = P->sweeps_done;
            HIP_OR_FAIL(ksat ? pt_launch_exchange_ksat(I->ksat_dev(), P->k, X, s)
                             : pt_launch_exchange_qap(I->qap_dev(), P->q, X, s));
        }
    }
    if (!ev.empty()) {
        HIP_OR_FAIL(hipEventSynchronize(ev.back()));
        for (size_t e = 0; e < ev.size(); e += 2) {
            float ms = 0;
            HIP_OR_FAIL(hipEventElapsedTime(&ms, ev[e], ev[e + 1]));
            P->prof_ms += ms;
        }
        P->prof_launches += n_rounds;
        const double per_sweep = ksat ? (double)P->R * I->n : (double)P->R * I->n * (I->n - 1) / 2.0;
        P->prof_attempts += per_sweep * sweeps_per_round * n_rounds;
    }
    if (npairs > 0 && (accepted || attempted)) {
        std::vector<int64_t> a(npairs), t(npairs);
        HIP_OR_FAIL(hipMemcpyAsync(a.data(), acc_dev, (size_t)npairs * 8, hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipMemcpyAsync(t.data(), att_dev, (size_t)npairs * 8, hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
        for (int32_t i = 0; i < npairs; ++i) {
            if (accepted)
                accepted[i] = a[i];
            if (attempted)
                attempted[i] = t[i];
        }
    }
    return ok();
}

int nmc_pt_run(nmc_replicas *P, const double *beta, int32_t n_temps, int32_t n_rounds, int32_t sweeps_per_round,
               int32_t first_parity, int64_t target, int64_t *accepted, int64_t *attempted, void *stream) {
    try {
        return pt_run_impl(P, beta, n_temps, n_rounds, sweeps_per_round, first_parity, target, accepted, attempted,
                           stream);
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

static int apt_ladder_impl(nmc_replicas *P, double beta_first, double alpha, double sigma_min, int32_t equil_sweeps,
                           int32_t meas_sweeps, int32_t max_temps, double *beta_out, double *sigma_out,
                           int32_t *n_temps, void *stream) {
    if (!P || !beta_out || !sigma_out || !n_temps)
        return fail(NMC_ERR_INVALID, "NULL argument");
    nmc_instance *I = P->inst;
    if (!I->dev)
        return fail(NMC_ERR_STATE, "instance is not bound");
    if (I->kind == NMC_KIND_KSAT && I->wide)
        return fail(NMC_ERR_UNSUPPORTED, "%s is not available for wide k-SAT instances (more than %d variables)", "the tempering ladder", kMaxVars);
    if (!std::isfinite(beta_first) || beta_first < 0)
        return fail(NMC_ERR_INVALID, "beta_first = %g is not finite and >= 0", beta_first);
    if (!std::isfinite(alpha) || !(alpha > 0))
        return fail(NMC_ERR_INVALID, "alpha = %g must be finite and > 0", alpha);
    if (!std::isfinite(sigma_min) || sigma_min < 0)
        return fail(NMC_ERR_INVALID, "sigma_min = %g must be finite and >= 0", sigma_min);
    if (equil_sweeps < 0 || meas_sweeps < 1 || max_temps < 1)
        return fail(NMC_ERR_INVALID, "need equil_sweeps >= 0, meas_sweeps >= 1 and max_temps >= 1");
    if ((uint64_t)P->R * (uint64_t)meas_sweeps > ((uint64_t)1 << 26))
        return fail(NMC_ERR_INVALID, "replicas x meas_sweeps = %lld samples exceeds 2^26",
                    (long long)P->R * meas_sweeps);
    if ((uint64_t)P->sweeps_done + (uint64_t)max_temps * (uint64_t)(equil_sweeps + meas_sweeps) > 0xFFFFFFFFull)
        return fail(NMC_ERR_INVALID, "sweep counter could pass 2^32 - 1");
    hipStream_t s = as_stream(stream);
    if (!P->pt_acc)
        HIP_OR_FAIL(hipMalloc(&P->pt_acc, 256));
    const bool ksat = I->kind == NMC_KIND_KSAT;
    const void *energy = ksat ? (const void *)P->k.energy : (const void *)P->q.cost;
    std::vector<double> row(std::max(equil_sweeps, 1));
    double b = beta_first;
    for (int32_t k = 0;; ++k) {
        if (equil_sweeps) {
            std::fill(row.begin(), row.end(), b);
            int rc = anneal_impl(P, row.data(), 1, equil_sweeps, NMC_PROFILE_HOMOGENEOUS, nullptr, -1, stream);
            if (rc)
                return rc;
        }
        HIP_OR_FAIL(hipMemsetAsync(P->pt_acc, 0, 32, s));
        for (int32_t m = 0; m < meas_sweeps; ++m) {
            int rc = anneal_impl(P, &b, 1, 1, NMC_PROFILE_HOMOGENEOUS, nullptr, -1, stream);
            if (rc)
                return rc;
            HIP_OR_FAIL(pt_launch_moments(energy, ksat ? 0 : 1, P->R, P->pt_acc, s));
        }
        unsigned long long acc[4];
        HIP_OR_FAIL(hipMemcpyAsync(acc, P->pt_acc, 32, hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
        // sigma^2 = (count S2 - S1^2) / count^2, the numerator exact in 128 bits
        const unsigned __int128 s2 = ((unsigned __int128)acc[3] << 64) | acc[2];
        const unsigned __int128 num = (unsigned __int128)acc[0] * s2 - (unsigned __int128)acc[1] * acc[1];
        const double sigma = std::sqrt((double)num / ((double)acc[0] * (double)acc[0]));
        beta_out[k] = b;
        sigma_out[k] = sigma;
        if (sigma <= sigma_min || k + 1 == max_temps) {
            *n_temps = k + 1;
            return ok();
        }
        b = b + alpha / sigma;
    }
}

int nmc_apt_ladder(nmc_replicas *P, double beta_first, double alpha, double sigma_min, int32_t equil_sweeps,
                   int32_t meas_sweeps, int32_t max_temps, double *beta_out, double *sigma_out, int32_t *n_temps,
                   void *stream) {
    try {
        return apt_ladder_impl(P, beta_first, alpha, sigma_min, equil_sweeps, meas_sweeps, max_temps, beta_out,
                               sigma_out, n_temps, stream);
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

// ---------------------------------------------------------------------------
// surrogate-Hamiltonian LBP and connected backbone growth
// ---------------------------------------------------------------------------

static int lbp_check_config(const nmc_lbp_config &c) {
    if (!std::isfinite(c.beta) || c.beta < 0)
        return fail(NMC_ERR_INVALID, "beta = %g must be finite and >= 0", c.beta);
    if (!std::isfinite(c.lambda0) || !(c.lambda0 > 0))
        return fail(NMC_ERR_INVALID, "lambda0 = %g must be finite and > 0", c.lambda0);
    if (!(c.lambda_ratio > 0 && c.lambda_ratio < 1))
        return fail(NMC_ERR_INVALID, "lambda_ratio = %g must lie in (0, 1)", c.lambda_ratio);
    if (!std::isfinite(c.lambda_min) || c.lambda_min < 0)
        return fail(NMC_ERR_INVALID, "lambda_min = %g must be finite and >= 0", c.lambda_min);
    if (c.max_iter < 1 || !(c.tol > 0) || !std::isfinite(c.tol))
        return fail(NMC_ERR_INVALID, "need max_iter >= 1 and a finite tol > 0");
    if (std::isnan(c.p_min) || !std::isfinite(c.theta_seed) || !std::isfinite(c.theta_cut) || c.theta_cut < 0 ||
        c.theta_seed < c.theta_cut)
        return fail(NMC_ERR_INVALID, "need 0 <= theta_cut <= theta_seed (finite) and a p_min that is not NaN");
    return NMC_OK;
}

// One LBP run of a batch: its replica set, seed and progress.
struct LbpRun {
    nmc_replicas *P = nullptr;
    int32_t replica = 0;
    LbpWork W{};
    double *keep = nullptr;
    size_t ubytes = 0;
    double kept_lambda = 0, kept_delta = 0, ov[2] = {0, 0};
    int32_t steps = 0, iters = 0, cnt[5] = {0, 0, 0, 0, 0};
    bool have = false, done = false;
};

// the replica set's workspace (allocated on first use) laid out for its instance
static int lbp_workspace(LbpRun &r, hipStream_t s) {
    nmc_replicas *P = r.P;
    nmc_instance *I = P->inst;
    const int32_t n = I->n, m = I->m;
    Arena ar;
    // messages clause-major then variable-major in one block (one copy or
    // clear covers both), and the block's saved copy
    const size_t ub = ((size_t)m * 4 + (size_t)I->n_lits) * 8;
    const size_t o_u = ar.take(ub), o_keep = ar.take(ub), o_T = ar.take((size_t)n * 8);
    const size_t o_mag = ar.take((size_t)n * 8), o_corr = ar.take((size_t)m * 8);
    const size_t o_ep = ar.take((size_t)m * 4 * 4), o_s = ar.take((size_t)n);
    const size_t o_scal = ar.take(2 * kLbpDeltaSlots * 8), o_res = ar.take(24), o_ctl = ar.take(8);
    const size_t o_lab = ar.take((size_t)n * 4), o_olab = ar.take((size_t)n * 4), o_size = ar.take((size_t)n * 4);
    const size_t o_seed = ar.take((size_t)n), o_flag = ar.take(4), o_cnt = ar.take(5 * 4);
    const size_t o_job = ar.take(sizeof(LbpJob));
    const size_t total = align_up(ar.size, 256);
    if (!P->lbp_dev) {
        HIP_OR_FAIL(hipMalloc(&P->lbp_dev, total));
        HIP_OR_FAIL(hipMemsetAsync(P->lbp_dev, 0, total, s));
    }
    if (!P->lbp_pin)
        HIP_OR_FAIL(hipHostMalloc(reinterpret_cast<void **>(&P->lbp_pin), 64, hipHostMallocDefault));
    uint8_t *b = P->lbp_dev;
    LbpWork &W = r.W;
    W.u = reinterpret_cast<double *>(b + o_u);
    r.keep = reinterpret_cast<double *>(b + o_keep);
    W.T = reinterpret_cast<double *>(b + o_T);
    W.mag = reinterpret_cast<double *>(b + o_mag);
    W.corr = reinterpret_cast<double *>(b + o_corr);
    W.uv = W.u + (size_t)m * 4;
    W.epos = reinterpret_cast<int32_t *>(b + o_ep);
    W.s = reinterpret_cast<int8_t *>(b + o_s);
    W.scal = reinterpret_cast<unsigned long long *>(b + o_scal);
    W.res = reinterpret_cast<double *>(b + o_res);
    W.ctl = reinterpret_cast<int32_t *>(b + o_ctl);
    W.label = reinterpret_cast<int32_t *>(b + o_lab);
    W.out_label = reinterpret_cast<int32_t *>(b + o_olab);
    W.size = reinterpret_cast<int32_t *>(b + o_size);
    W.seeded = b + o_seed;
    W.flag = reinterpret_cast<int32_t *>(b + o_flag);
    W.counts = reinterpret_cast<int32_t *>(b + o_cnt);
    r.ubytes = ub;
    (void)o_job;
    return NMC_OK;
}

static size_t lbp_job_offset(const nmc_instance *I) {
    // the last region of the workspace laid out by lbp_workspace
    Arena ar;
    const int32_t n = I->n, m = I->m;
    const size_t ub = ((size_t)m * 4 + (size_t)I->n_lits) * 8;
    ar.take(ub), ar.take(ub), ar.take((size_t)n * 8);
    ar.take((size_t)n * 8), ar.take((size_t)m * 8);
    ar.take((size_t)m * 4 * 4), ar.take((size_t)n);
    ar.take(2 * kLbpDeltaSlots * 8), ar.take(24), ar.take(8);
    ar.take((size_t)n * 4), ar.take((size_t)n * 4), ar.take((size_t)n * 4);
    ar.take((size_t)n), ar.take(4), ar.take(5 * 4);
    return ar.take(sizeof(LbpJob));
}

// Adiabatic LBP and cluster growth for every run, in lockstep over the
// lambda steps (all runs share the configuration, so the runs still going
// share lambda); jobs_dev holds the runs' job descriptors on the device.
static int lbp_run_all(std::vector<LbpRun> &runs, const LbpJob *jobs_dev, const LbpDims &D, const nmc_lbp_config &c,
                       int64_t *pin, hipStream_t s, bool profiling, double *prof_ms, int64_t *prof_iters) {
    const double w = 1.0 - std::exp(-2.0 * c.beta);
    const size_t nr = runs.size();
    hipEvent_t pe[2] = {nullptr, nullptr};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int k = 0; k < 2; ++k)
                if (e[k])
                    (void)hipEventDestroy(e[k]);
        }
    } ev_guard{pe};
    if (profiling) {
        HIP_OR_FAIL(hipEventCreate(&pe[0]));
        HIP_OR_FAIL(hipEventCreate(&pe[1]));
    }
    // initial messages at lambda0: u = 0 and T = H give h = sigma H, u from h
    for (auto &r : runs)
        if (r.ubytes)
            HIP_OR_FAIL(hipMemsetAsync(r.W.u, 0, r.ubytes, s));
    HIP_OR_FAIL(lbp_launch_setup(jobs_dev, D, c.lambda0, s));
    HIP_OR_FAIL(lbp_launch_clause(jobs_dev, D, w, 0, s));
    double lambda = c.lambda0;
    for (;;) {
        // one step for the runs still going: queued in batches of 8, then
        // 16 iterations; convergence is decided on the device after every
        // iteration and read back (pinned memory) once per batch
        for (auto &r : runs)
            if (!r.done) {
                if (r.ubytes)
                    HIP_OR_FAIL(hipMemcpyAsync(r.keep, r.W.u, r.ubytes, hipMemcpyDeviceToDevice, s));
                HIP_OR_FAIL(hipMemsetAsync(r.W.scal, 0, 2 * kLbpDeltaSlots * 8, s));
                HIP_OR_FAIL(hipMemsetAsync(r.W.ctl, 0, 8, s));
            }
        int32_t queued = 0;
        for (;;) {
            const int32_t cnt = std::min(queued ? 16 : 8, c.max_iter - queued);
            if (pe[0])
                HIP_OR_FAIL(hipEventRecord(pe[0], s));
            HIP_OR_FAIL(lbp_launch_iterations(jobs_dev, D, lambda, w, c.tol, c.max_iter, queued, cnt, s));
            if (pe[1])
                HIP_OR_FAIL(hipEventRecord(pe[1], s));
            queued += cnt;
            for (size_t k = 0; k < nr; ++k)
                if (!runs[k].done) {
                    HIP_OR_FAIL(hipMemcpyAsync(pin + 2 * k, runs[k].W.ctl, 8, hipMemcpyDeviceToHost, s));
                    HIP_OR_FAIL(hipMemcpyAsync(pin + 2 * k + 1, runs[k].W.res + 2, 8, hipMemcpyDeviceToHost, s));
                }
            HIP_OR_FAIL(hipStreamSynchronize(s));
            if (pe[0]) {
                float ms = 0;
                HIP_OR_FAIL(hipEventElapsedTime(&ms, pe[0], pe[1]));
                *prof_ms += ms;
            }
            bool all_stopped = true;
            for (size_t k = 0; k < nr; ++k)
                if (!runs[k].done && reinterpret_cast<const int32_t *>(pin + 2 * k)[0] == 0)
                    all_stopped = false;
            if (all_stopped || queued >= c.max_iter)
                break;
        }
        // overlaps at this lambda (every run; the ones that stopped earlier
        // only overwrite scratch that the final pass recomputes)
        HIP_OR_FAIL(lbp_launch_var(jobs_dev, D, lambda, 1, s));
        HIP_OR_FAIL(lbp_launch_overlap(jobs_dev, D, s));
        std::vector<double> pov(nr, 0.0);
        std::vector<int32_t> ctl0(nr, 0), ctl1(nr, 0);
        std::vector<double> delta(nr, 0.0);
        for (size_t k = 0; k < nr; ++k)
            if (!runs[k].done) {
                const int32_t *cw = reinterpret_cast<const int32_t *>(pin + 2 * k);
                ctl0[k] = cw[0];
                ctl1[k] = cw[1];
                std::memcpy(&delta[k], pin + 2 * k + 1, 8);
            }
        for (size_t k = 0; k < nr; ++k)
            if (!runs[k].done)
                HIP_OR_FAIL(hipMemcpyAsync(pin + 2 * k, runs[k].W.res, 8, hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
        for (size_t k = 0; k < nr; ++k)
            if (!runs[k].done)
                std::memcpy(&pov[k], pin + 2 * k, 8);
        bool any = false;
        for (size_t k = 0; k < nr; ++k) {
            LbpRun &r = runs[k];
            if (r.done)
                continue;
            r.iters += ctl1[k];
            *prof_iters += profiling ? ctl1[k] : 0;
            ++r.steps;
            const bool conv = ctl0[k] == 1;
            if (!conv || (r.have && pov[k] < c.p_min)) {
                if (r.have) {
                    if (r.ubytes)
                        HIP_OR_FAIL(hipMemcpyAsync(r.W.u, r.keep, r.ubytes, hipMemcpyDeviceToDevice, s));
                } else {
                    r.kept_delta = delta[k];
                }
                r.done = true;
                continue;
            }
            r.have = true;
            r.kept_lambda = lambda;
            r.kept_delta = delta[k];
            if (!(lambda * c.lambda_ratio >= c.lambda_min))
                r.done = true;
            else
                any = true;
        }
        if (!any)
            break;
        lambda *= c.lambda_ratio;
    }
    // marginals, moments and overlaps from each run's kept messages
    for (size_t k = 0; k < nr; ++k) {
        LbpDims one{1, runs[k].P->inst->n, runs[k].P->inst->m};
        HIP_OR_FAIL(lbp_launch_var(jobs_dev + k, one, runs[k].have ? runs[k].kept_lambda : c.lambda0, 1, s));
    }
    HIP_OR_FAIL(lbp_launch_overlap(jobs_dev, D, s));
    HIP_OR_FAIL(lbp_launch_clause(jobs_dev, D, w, 1, s));
    // connected components of the rigid clauses (one shared change flag)
    HIP_OR_FAIL(lbp_launch_label_init(jobs_dev, D, s));
    int32_t *flag = runs[0].W.flag;
    for (int32_t pass = 0;; ++pass) {
        if (pass > 4 * D.max_n + 64)
            return fail(NMC_ERR_DEVICE, "component labels did not settle");
        HIP_OR_FAIL(hipMemsetAsync(flag, 0, 4, s));
        HIP_OR_FAIL(lbp_launch_hook_jump(jobs_dev, D, c.theta_cut, s));
        HIP_OR_FAIL(hipMemcpyAsync(pin, flag, 4, hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
        if (!reinterpret_cast<const int32_t *>(pin)[0])
            break;
    }
    HIP_OR_FAIL(lbp_launch_finish(jobs_dev, D, c.theta_seed, c.theta_cut, s));
    for (size_t k = 0; k < nr; ++k) {
        HIP_OR_FAIL(hipMemcpyAsync(runs[k].cnt, runs[k].W.counts, 20, hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipMemcpyAsync(runs[k].ov, runs[k].W.res, 16, hipMemcpyDeviceToHost, s));
    }
    HIP_OR_FAIL(hipStreamSynchronize(s));
    for (auto &r : runs)
        r.P->has_backbone = true;
    return NMC_OK;
}

static void lbp_fill_result(const LbpRun &r, const nmc_lbp_config &c, nmc_lbp_result *res) {
    res->lambda = r.have ? r.kept_lambda : c.lambda0;
    res->steps = r.steps;
    res->iterations = r.iters;
    res->converged = r.have ? 1 : 0;
    res->delta = r.kept_delta;
    res->overlap = r.ov[0];
    res->self_overlap = r.ov[1];
    res->backbone_size = r.cnt[0];
    res->n_clusters = r.cnt[1];
    res->largest_cluster = r.cnt[2];
    res->rigid_clauses = r.cnt[3];
    res->seed_clauses = r.cnt[4];
}

static int lbp_impl(nmc_replicas *P, int32_t replica, int32_t which, const nmc_lbp_config *cfg, nmc_lbp_result *res,
                    uint8_t *class_out, double *mag_out, double *corr_out, int32_t *label_out, void *stream) {
    if (!P || !cfg)
        return fail(NMC_ERR_INVALID, "NULL argument");
    nmc_instance *I = P->inst;
    if (!I->dev)
        return fail(NMC_ERR_STATE, "instance is not bound");
    if (I->kind != NMC_KIND_KSAT)
        return fail(NMC_ERR_UNSUPPORTED, "LBP runs on k-SAT instances");
    if (I->kind == NMC_KIND_KSAT && I->wide)
        return fail(NMC_ERR_UNSUPPORTED, "%s is not available for wide k-SAT instances (more than %d variables)", "LBP", kMaxVars);
    if (replica < 0 || replica >= P->R)
        return fail(NMC_ERR_INVALID, "replica %d outside [0, %d)", replica, P->R);
    if (which != NMC_STATE_CURRENT && which != NMC_STATE_BEST)
        return fail(NMC_ERR_INVALID, "which must be NMC_STATE_CURRENT or NMC_STATE_BEST");
    if (int rc = lbp_check_config(*cfg))
        return rc;
    hipStream_t s = as_stream(stream);
    std::vector<LbpRun> runs(1);
    runs[0].P = P;
    runs[0].replica = replica;
    if (int rc = lbp_workspace(runs[0], s))
        return rc;
    LbpJob J{};
    J.I = I->ksat_dev();
    J.W = runs[0].W;
    J.xs_row = (which == NMC_STATE_BEST ? P->k.best_xs : P->k.xs) + (size_t)(replica / kGroup) * I->n;
    J.bit = replica % kGroup;
    J.cls = P->k.cls;
    LbpJob *jd = reinterpret_cast<LbpJob *>(P->lbp_dev + lbp_job_offset(I));
    HIP_OR_FAIL(hipMemcpyAsync(jd, &J, sizeof J, hipMemcpyHostToDevice, s));
    const LbpDims D{1, I->n, I->m};
    if (int rc = lbp_run_all(runs, jd, D, *cfg, P->lbp_pin, s, P->profiling, &P->lbp_ms, &P->lbp_iters))
        return rc;
    const int32_t n = I->n, m = I->m;
    if (class_out && n)
        HIP_OR_FAIL(hipMemcpyAsync(class_out, P->k.cls, n, hipMemcpyDeviceToHost, s));
    if (mag_out && n)
        HIP_OR_FAIL(hipMemcpyAsync(mag_out, runs[0].W.mag, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    // the moments are in the LBP clause order on the device
    std::vector<double> corr_lbp;
    if (corr_out && m) {
        corr_lbp.resize(m);
        HIP_OR_FAIL(hipMemcpyAsync(corr_lbp.data(), runs[0].W.corr, (size_t)m * 8, hipMemcpyDeviceToHost, s));
    }
    if (label_out && n)
        HIP_OR_FAIL(hipMemcpyAsync(label_out, runs[0].W.out_label, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    if (corr_out && m)
        for (int32_t a = 0; a < m; ++a)
            corr_out[a] = corr_lbp[I->lbp_pos[a]];
    if (res)
        lbp_fill_result(runs[0], *cfg, res);
    return ok();
}

int nmc_lbp_backbone(nmc_replicas *P, int32_t replica, int32_t which, const nmc_lbp_config *cfg,
                     nmc_lbp_result *res, uint8_t *class_out, double *mag_out, double *corr_out, int32_t *label_out,
                     void *stream) {
    try {
        return lbp_impl(P, replica, which, cfg, res, class_out, mag_out, corr_out, label_out, stream);
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_whiten(nmc_replicas *P, int32_t which, int32_t *frozen_out, uint8_t *white_out, int32_t *passes,
               void *stream) {
    if (!P || !frozen_out)
        return fail(NMC_ERR_INVALID, "NULL argument");
    nmc_instance *I = P->inst;
    if (!I->dev)
        return fail(NMC_ERR_STATE, "instance is not bound");
    if (I->kind != NMC_KIND_KSAT)
        return fail(NMC_ERR_UNSUPPORTED, "whitening applies to k-SAT states");
    if (I->kind == NMC_KIND_KSAT && I->wide)
        return fail(NMC_ERR_UNSUPPORTED, "%s is not available for wide k-SAT instances (more than %d variables)", "whitening", kMaxVars);
    if (which != NMC_STATE_CURRENT && which != NMC_STATE_BEST)
        return fail(NMC_ERR_INVALID, "which must be NMC_STATE_CURRENT or NMC_STATE_BEST");
    try {
        hipStream_t s = as_stream(stream);
        const int32_t n = I->n, G = P->G, R = P->R;
        const size_t rows = align_up((size_t)G * n, 256), cnt = align_up((size_t)G * kGroup * 4, 256);
        if (!P->wh_dev)
            HIP_OR_FAIL(hipMalloc(&P->wh_dev, rows + cnt + 256));
        uint8_t *white = P->wh_dev;
        int32_t *frozen = reinterpret_cast<int32_t *>(P->wh_dev + rows);
        int32_t *pass = reinterpret_cast<int32_t *>(P->wh_dev + rows + cnt);
        HIP_OR_FAIL(hipMemsetAsync(pass, 0, 4, s));
        const uint8_t *src = which == NMC_STATE_BEST ? P->k.best_xs : P->k.xs;
        HIP_OR_FAIL(ksat_launch_whiten(I->ksat_dev(), src, G, R, white, frozen, pass, s));
        HIP_OR_FAIL(hipMemcpyAsync(frozen_out, frozen, (size_t)R * 4, hipMemcpyDeviceToHost, s));
        int32_t np = 0;
        HIP_OR_FAIL(hipMemcpyAsync(&np, pass, 4, hipMemcpyDeviceToHost, s));
        std::vector<uint8_t> packed;
        if (white_out) {
            packed.resize((size_t)G * n);
            HIP_OR_FAIL(hipMemcpyAsync(packed.data(), white, packed.size(), hipMemcpyDeviceToHost, s));
        }
        HIP_OR_FAIL(hipStreamSynchronize(s));
        if (white_out)
            for (int32_t r = 0; r < R; ++r) {
                const uint8_t *row = packed.data() + (size_t)(r / kGroup) * n;
                uint8_t *dst = white_out + (size_t)r * n;
                for (int32_t v = 0; v < n; ++v)
                    dst[v] = (row[v] >> (r % kGroup)) & 1u;
            }
        if (passes)
            *passes = np;
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

static int cluster_flip_impl(nmc_replicas *P, const int32_t *label, double beta, int64_t target,
                             int32_t *accepted_out, void *stream) {
    if (!P || !label)
        return fail(NMC_ERR_INVALID, "NULL argument");
    nmc_instance *I = P->inst;
    if (!I->dev)
        return fail(NMC_ERR_STATE, "instance is not bound");
    if (I->kind != NMC_KIND_KSAT)
        return fail(NMC_ERR_UNSUPPORTED, "cluster flips apply to k-SAT states");
    if (I->kind == NMC_KIND_KSAT && I->wide)
        return fail(NMC_ERR_UNSUPPORTED, "%s is not available for wide k-SAT instances (more than %d variables)", "the cluster flip", kMaxVars);
    if (!std::isfinite(beta) || beta < 0)
        return fail(NMC_ERR_INVALID, "beta = %g is not finite and >= 0", beta);
    if ((uint64_t)P->sweeps_done + 1 > 0xFFFFFFFFull)
        return fail(NMC_ERR_INVALID, "sweep counter would pass 2^32 - 1");
    const int32_t n = I->n, m = I->m;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t l = label[i];
        if (l < -1 || l >= n || (l >= 0 && label[l] != l))
            return fail(NMC_ERR_INVALID, "label[%d] = %d is not -1 or a variable that labels itself", i, l);
    }
    // clusters in increasing label order; their variables and clauses
    std::vector<int32_t> ord(n, -1), v_ptr(1, 0), v_list, cl_ptr, cnt;
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i)
        if (label[i] == i)
            ord[i] = nc++;
    cnt.assign(nc + 1, 0);
    for (int32_t i = 0; i < n; ++i)
        if (label[i] >= 0)
            cnt[ord[label[i]] + 1]++;
    v_ptr.assign(nc + 1, 0);
    for (int32_t k = 0; k < nc; ++k)
        v_ptr[k + 1] = v_ptr[k] + cnt[k + 1];
    v_list.resize(v_ptr[nc]);
    {
        std::vector<int32_t> fill(v_ptr.begin(), v_ptr.end() - 1);
        for (int32_t i = 0; i < n; ++i)
            if (label[i] >= 0)
                v_list[fill[ord[label[i]]]++] = i;
    }
    // clause entries: one per (clause, cluster among its variables)
    const std::vector<uint8_t> &img = I->image;
    const uint32_t *caddr = reinterpret_cast<const uint32_t *>(img.data() + I->off_clause_addr);
    std::vector<std::pair<int32_t, uint32_t>> ent;  // (cluster, clause | mask << 28)
    for (int32_t a = 0; a < m; ++a) {
        int32_t ks[4];
        int nk = 0;
        uint32_t masks[4] = {0, 0, 0, 0};
        for (int j = 0; j < 4; ++j) {
            const uint32_t ad = caddr[(size_t)a * 4 + j];
            if (ad >= 2u * (uint32_t)n)
                continue;
            const int32_t v = (int32_t)(ad >= (uint32_t)n ? ad - n : ad);
            if (label[v] < 0)
                continue;
            const int32_t k = ord[label[v]];
            int q = 0;
            while (q < nk && ks[q] != k)
                ++q;
            if (q == nk)
                ks[nk++] = k;
            masks[q] |= 1u << j;
        }
        for (int q = 0; q < nk; ++q)
            ent.emplace_back(ks[q], (uint32_t)a | (masks[q] << 28));
    }
    std::stable_sort(ent.begin(), ent.end(),
                     [](const std::pair<int32_t, uint32_t> &x, const std::pair<int32_t, uint32_t> &y) {
                         return x.first < y.first;
                     });
    cl_ptr.assign(nc + 1, 0);
    int32_t longest = 0;
    for (const auto &e : ent)
        cl_ptr[e.first + 1]++;
    for (int32_t k = 0; k < nc; ++k) {
        longest = std::max(longest, cl_ptr[k + 1]);
        cl_ptr[k + 1] += cl_ptr[k];
    }
    // thresholds up to the largest possible rise (the longest clause list),
    // cut at the first zero (every larger rise then has threshold zero)
    std::vector<uint32_t> thr(1, 0xFFFFFFFFu);
    for (int32_t d = 1; d <= longest; ++d) {
        const uint32_t v = threshold(beta, d);
        if (!v)
            break;
        thr.push_back(v);
    }
    const size_t b_clp = align_up((nc + 1) * 4, 256), b_cl = align_up(std::max<size_t>(ent.size(), 1) * 4, 256);
    const size_t b_vp = align_up((nc + 1) * 4, 256), b_vl = align_up(std::max<size_t>(v_list.size(), 1) * 4, 256);
    const size_t b_thr = align_up(thr.size() * 4, 256), b_acc = align_up((size_t)P->G * kGroup * 4, 256);
    int rc = ensure_tab(P, b_clp + b_cl + b_vp + b_vl + b_thr + b_acc);
    if (rc)
        return rc;
    hipStream_t s = as_stream(stream);
    uint8_t *base = P->tab_dev;
    std::vector<uint32_t> cl_list(ent.size());
    for (size_t i = 0; i < ent.size(); ++i)
        cl_list[i] = ent[i].second;
    HIP_OR_FAIL(hipMemcpyAsync(base, cl_ptr.data(), (nc + 1) * 4, hipMemcpyHostToDevice, s));
    if (!cl_list.empty())
        HIP_OR_FAIL(hipMemcpyAsync(base + b_clp, cl_list.data(), cl_list.size() * 4, hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(hipMemcpyAsync(base + b_clp + b_cl, v_ptr.data(), (nc + 1) * 4, hipMemcpyHostToDevice, s));
    if (!v_list.empty())
        HIP_OR_FAIL(hipMemcpyAsync(base + b_clp + b_cl + b_vp, v_list.data(), v_list.size() * 4,
                                   hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(hipMemcpyAsync(base + b_clp + b_cl + b_vp + b_vl, thr.data(), thr.size() * 4, hipMemcpyHostToDevice,
                               s));
    CflipCall C{};
    C.cl_ptr = reinterpret_cast<const int32_t *>(base);
    C.cl_list = reinterpret_cast<const uint32_t *>(base + b_clp);
    C.v_ptr = reinterpret_cast<const int32_t *>(base + b_clp + b_cl);
    C.v_list = reinterpret_cast<const int32_t *>(base + b_clp + b_cl + b_vp);
    C.thr = reinterpret_cast<const uint32_t *>(base + b_clp + b_cl + b_vp + b_vl);
    C.accepted = reinterpret_cast<int32_t *>(base + b_clp + b_cl + b_vp + b_vl + b_thr);
    C.n_clusters = nc;
    C.thr_len = (int32_t)thr.size() - 1;
    C.t = P->sweeps_done;
    C.target = (int32_t)std::max<int64_t>(std::min<int64_t>(target, INT32_MAX), INT32_MIN);
    C.key0 = (uint32_t)P->seed;
    C.key1 = (uint32_t)(P->seed >> 32);
    const size_t lds = ksat_cflip_lds_bytes(n);
    if (lds > kLdsBytes - 64)
        return fail(NMC_ERR_CAPACITY, "cluster flips need %zu bytes of LDS", lds);
    HIP_OR_FAIL(ksat_launch_cflip(I->ksat_dev(), P->k, C, s));
    P->sweeps_done += 1;
    if (accepted_out) {
        HIP_OR_FAIL(hipMemcpyAsync(accepted_out, C.accepted, (size_t)P->R * 4, hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
    }
    return ok();
}

int nmc_cluster_flip(nmc_replicas *P, const int32_t *label, double beta, int64_t target, int32_t *accepted_out,
                     void *stream) {
    try {
        return cluster_flip_impl(P, label, beta, target, accepted_out, stream);
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_lbp_kernel_time(nmc_replicas *P, double *ms, int64_t *iterations, int32_t reset) {
    if (!P)
        return fail(NMC_ERR_INVALID, "NULL replicas");
    if (ms)
        *ms = P->lbp_ms;
    if (iterations)
        *iterations = P->lbp_iters;
    if (reset) {
        P->lbp_ms = 0;
        P->lbp_iters = 0;
    }
    return ok();
}

int nmc_accept_count(nmc_replicas *P, uint64_t *accepted, int32_t reset, void *stream) {
    if (!P || !accepted)
        return fail(NMC_ERR_INVALID, "NULL argument");
    const bool ksat = P->inst->kind == NMC_KIND_KSAT;
    unsigned long long *d = ksat ? P->k.accepted : P->q.accepted;
    hipStream_t s = as_stream(stream);
    unsigned long long v = 0;
    HIP_OR_FAIL(hipMemcpyAsync(&v, d, sizeof v, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    *accepted = v;
    if (reset) {
        HIP_OR_FAIL(hipMemsetAsync(d, 0, sizeof v, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
    }
    return ok();
}

int nmc_kernel_time(nmc_replicas *P, double *ms, int64_t *launches, double *attempts, int32_t reset) {
    if (!P)
        return fail(NMC_ERR_INVALID, "NULL replicas");
    if (ms)
        *ms = P->prof_ms;
    if (launches)
        *launches = P->prof_launches;
    if (attempts)
        *attempts = P->prof_attempts;
    if (reset) {
        P->prof_ms = 0;
        P->prof_launches = 0;
        P->prof_attempts = 0;
    }
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched launches (many replica sets, one grid per kernel kind)
// ---------------------------------------------------------------------------

// One launch of the plan's sequence, in the order it is enqueued.  Everything
// a launch takes besides the uploaded descriptor blob is here, so two calls
// whose launch lists (and blob address) are equal can replay one graph.
struct BatchLaunch {
    int32_t what = 0;  // 0 k-SAT sweep, 1 QAP sweep, 2 k-SAT backbone, 3 QAP backbone
    size_t off_jobs = 0, off_items = 0;
    int32_t n_items = 0, grid = 0, block = 0;
    size_t lds = 0;
    int32_t thr_num = 0, thr_den = 0, expand = 0;
    double attempts = 0;
    bool operator==(const BatchLaunch &o) const {
        return what == o.what && off_jobs == o.off_jobs && off_items == o.off_items && n_items == o.n_items &&
               grid == o.grid && block == o.block && lds == o.lds && thr_num == o.thr_num && thr_den == o.thr_den &&
               expand == o.expand;
    }
};

struct nmc_batch {
    std::vector<nmc_replicas *> sets;
    int32_t block_threads = 0;  // k-SAT sweep workgroup size; 0 = heuristic
    uint8_t *dev = nullptr;     // library-owned: job descriptors, items, tables
    size_t cap = 0;
    hipStream_t cap_stream = nullptr;  // stream used for graph capture
    bool profiling = false;
    double prof_ms = 0;
    int64_t prof_launches = 0;
    double prof_attempts = 0;
    // batched LBP: job descriptors (device) and control readback (pinned)
    LbpJob *lbp_jobs = nullptr;
    int64_t *lbp_pin = nullptr;
    size_t lbp_cap = 0;
    double lbp_ms = 0;
    int64_t lbp_iters = 0;
    // executable graph of the last per-set plan call, replayed while the
    // launch list and the descriptor buffer stay the same
    hipGraphExec_t exec = nullptr;
    uint8_t *exec_dev = nullptr;
    std::vector<BatchLaunch> exec_launches;
    int64_t graph_captures = 0, graph_replays = 0;
};

namespace {

int device_cus() {
    static const int cus = [] {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                    hipSuccess || c <= 0)
            c = 256;
        return c;
    }();
    return cus;
}

struct Blob {
    std::vector<uint8_t> host;
    size_t take(size_t bytes) {
        const size_t off = align_up(host.size(), 256);
        host.resize(off + bytes);
        return off;
    }
};

struct PhaseSpec {
    const double *beta;
    int32_t n_classes, n_sweeps, profile;
};

struct BuiltPhase {
    int32_t n_sweeps = 0;
    size_t off_kjobs = 0, off_kitems = 0, off_qjobs = 0, off_qitems = 0;
    int nk_items = 0, nq_items = 0;
    size_t lds_k = 0, lds_q = 0;
    int grid_k = 0, grid_q = 0, block_k = 0;
    double attempts = 0;
};

struct BuiltBackbone {
    size_t off_kjobs = 0, off_kitems = 0, off_qjobs = 0, off_qitems = 0;
    int nk_items = 0, nq_items = 0;
};

int heuristic_block(const std::vector<nmc_replicas *> &ks) {
    // enough waves for the typical chunk count of one colour class
    std::vector<double> chunks;
    for (auto *P : ks)
        chunks.push_back((double)P->inst->n_chunks / std::max(1, P->inst->n_colors));
    if (chunks.empty())
        return 256;
    std::nth_element(chunks.begin(), chunks.begin() + chunks.size() / 2, chunks.end());
    const double c = chunks[chunks.size() / 2];
    int b = 64;
    while (b < 1024 && b / 64 < c)
        b *= 2;
    return b;
}

// Lay out, in one host blob, everything the batched kernels of the given
// phases need (job descriptors whose device pointers point into the blob's
// future device copy at dev_base).  Returns NMC_OK or an error code.
int build_batch(nmc_batch *B, const std::vector<PhaseSpec> &phases, bool with_backbone, const int64_t *targets,
                uint8_t *dev_base, Blob &blob, std::vector<BuiltPhase> &built, BuiltBackbone &bb,
                std::vector<nmc_replicas *> *override_sets = nullptr) {
    const std::vector<nmc_replicas *> &sets = override_sets ? *override_sets : B->sets;
    std::vector<int> kidx, qidx;
    for (size_t i = 0; i < sets.size(); ++i)
        (sets[i]->inst->kind == NMC_KIND_KSAT ? kidx : qidx).push_back((int)i);
    int32_t stride_k = 1, ha = 1;
    for (int i : kidx)
        stride_k = std::max(stride_k, sets[i]->inst->dmax + 1);
    for (int i : qidx)
        ha = std::max(ha, sets[i]->inst->qap_ha);
    const int32_t stride_q = qap_row_words(ha);
    std::vector<nmc_replicas *> ks;
    for (int i : kidx)
        ks.push_back(sets[i]);
    const int block_k = B->block_threads > 0 ? B->block_threads : heuristic_block(ks);
    const int cus = device_cus();
    uint32_t offset_sweeps = 0;
    for (const PhaseSpec &ph : phases) {
        BuiltPhase bp;
        bp.n_sweeps = ph.n_sweeps;
        bp.block_k = block_k;
        // thresholds shared by the phase's jobs of one kind
        size_t off_ktab = 0, off_qtab = 0;
        bool qmono = true;  // every QAP row's T never increases
        if (!kidx.empty()) {
            off_ktab = blob.take(std::max<size_t>((size_t)ph.n_sweeps * ph.n_classes * stride_k * 4, 4));
            uint32_t *t = reinterpret_cast<uint32_t *>(blob.host.data() + off_ktab);
            for (int32_t sw = 0; sw < ph.n_sweeps; ++sw)
                for (int32_t c = 0; c < ph.n_classes; ++c) {
                    uint32_t *row = t + ((size_t)sw * ph.n_classes + c) * stride_k;
                    row[0] = 0xFFFFFFFFu;
                    for (int32_t d = 1; d < stride_k; ++d)
                        row[d] = threshold(ph.beta[(size_t)c * ph.n_sweeps + sw], d);
                }
        }
        if (!qidx.empty()) {
            off_qtab = blob.take(std::max<size_t>((size_t)ph.n_sweeps * ph.n_classes * stride_q * 4, 4));
            for (int32_t sw = 0; sw < ph.n_sweeps; ++sw)
                for (int32_t c = 0; c < ph.n_classes; ++c) {
                    uint32_t *row = reinterpret_cast<uint32_t *>(blob.host.data() + off_qtab) +
                                    ((size_t)sw * ph.n_classes + c) * stride_q;
                    qmono = qap_fill_row(row, ph.beta[(size_t)c * ph.n_sweeps + sw], ha) && qmono;
                }
        }
        // k-SAT jobs and items
        if (!kidx.empty()) {
            bp.off_kjobs = blob.take(kidx.size() * sizeof(KsatJob));
            std::vector<std::pair<double, int2>> items;
            for (size_t j = 0; j < kidx.size(); ++j) {
                nmc_replicas *P = sets[kidx[j]];
                KsatJob J{};
                J.I = P->inst->ksat_dev();
                J.R = P->k;
                J.C.tab = reinterpret_cast<const uint32_t *>(dev_base + off_ktab);
                J.C.var_cls = ph.profile == NMC_PROFILE_BACKBONE ? P->k.cls : nullptr;
                J.C.n_classes = ph.n_classes;
                J.C.stride = stride_k;
                J.C.n_sweeps = ph.n_sweeps;
                J.C.sweep_words = ph.n_classes * stride_k;
                J.C.t0 = P->sweeps_done + offset_sweeps;
                const int64_t tg = targets ? targets[kidx[j]] : -1;
                J.C.target = (int32_t)std::max<int64_t>(std::min<int64_t>(tg, INT32_MAX), INT32_MIN);
                J.C.check_start = 1;
                J.C.key0 = (uint32_t)P->seed;
                J.C.key1 = (uint32_t)(P->seed >> 32);
                J.C.gpw = P->gpw;
                std::memcpy(blob.host.data() + bp.off_kjobs + j * sizeof(KsatJob), &J, sizeof J);
                const double cost = (double)P->inst->n * (P->inst->dmax + 1) * P->gpw;
                for (int g = 0; g < (P->G + P->gpw - 1) / P->gpw; ++g)
                    items.push_back({cost, make_int2((int)j, g)});
                bp.lds_k = std::max(bp.lds_k, ksat_sweep_lds_bytes(P->inst->n, ph.n_classes, stride_k));
                bp.attempts += (double)P->R * P->inst->n * ph.n_sweeps;
            }
            std::stable_sort(items.begin(), items.end(),
                             [](const std::pair<double, int2> &a, const std::pair<double, int2> &b) { return a.first > b.first; });
            bp.nk_items = (int)items.size();
            bp.off_kitems = blob.take(items.size() * sizeof(int2));
            for (size_t t = 0; t < items.size(); ++t)
                std::memcpy(blob.host.data() + bp.off_kitems + t * sizeof(int2), &items[t].second, sizeof(int2));
            if (bp.lds_k > kLdsBytes)
                return fail(NMC_ERR_CAPACITY, "batched k-SAT sweep needs %zu bytes of LDS", bp.lds_k);
            bp.grid_k = std::min(bp.nk_items, ksat_batch_occupancy(block_k, bp.lds_k) * cus);
        }
        if (!qidx.empty()) {
            bp.off_qjobs = blob.take(qidx.size() * sizeof(QapJob));
            std::vector<std::pair<double, int2>> items;
            for (size_t j = 0; j < qidx.size(); ++j) {
                nmc_replicas *P = sets[qidx[j]];
                QapJob J{};
                J.I = P->inst->qap_dev();
                J.I.ha = ha;
                J.R = P->q;
                J.C.tab = reinterpret_cast<const uint32_t *>(dev_base + off_qtab);
                J.C.fac_cls = ph.profile == NMC_PROFILE_BACKBONE ? P->q.cls : nullptr;
                J.C.n_classes = ph.n_classes;
                J.C.stride = stride_q;
                J.C.n_sweeps = ph.n_sweeps;
                J.C.sweep_words = ph.n_classes * stride_q;
                J.C.t0 = P->sweeps_done + offset_sweeps;
                J.C.target = targets ? targets[qidx[j]] : -1;
                J.C.check_start = 1;
                J.C.rows = qap_rows_setting();
                J.C.tab_allow = qap_tab_setting();
                J.C.quad_allow = qap_quad_setting();
                J.C.dstar = qmono && qap_dstar_setting();
                J.C.key0 = (uint32_t)P->seed;
                J.C.key1 = (uint32_t)(P->seed >> 32);
                std::memcpy(blob.host.data() + bp.off_qjobs + j * sizeof(QapJob), &J, sizeof J);
                const double n = P->inst->n;
                const int blocks = (P->R + kQapRepPerBlock - 1) / kQapRepPerBlock;
                for (int b = 0; b < blocks; ++b)
                    items.push_back({n * n * n, make_int2((int)j, b)});
                bp.lds_q = std::max(bp.lds_q, qap_sweep_lds_bytes(P->inst->n, ph.n_classes, stride_q));
                bp.attempts += (double)P->R * n * (n - 1) / 2.0 * ph.n_sweeps;
            }
            std::stable_sort(items.begin(), items.end(),
                             [](const std::pair<double, int2> &a, const std::pair<double, int2> &b) { return a.first > b.first; });
            bp.nq_items = (int)items.size();
            bp.off_qitems = blob.take(items.size() * sizeof(int2));
            for (size_t t = 0; t < items.size(); ++t)
                std::memcpy(blob.host.data() + bp.off_qitems + t * sizeof(int2), &items[t].second, sizeof(int2));
            if (bp.lds_q > kLdsBytes)
                return fail(NMC_ERR_CAPACITY, "batched QAP sweep needs %zu bytes of LDS", bp.lds_q);
            bp.grid_q = std::min(bp.nq_items, qap_batch_occupancy(bp.lds_q) * cus);
        }
        built.push_back(bp);
        offset_sweeps += (uint32_t)ph.n_sweeps;
    }
    if (with_backbone) {
        // descriptors without schedule fields; reuse of KsatRepDev/QapRepDev only
        if (!kidx.empty()) {
            bb.off_kjobs = blob.take(kidx.size() * sizeof(KsatJob));
            std::vector<int2> items;
            for (size_t j = 0; j < kidx.size(); ++j) {
                nmc_replicas *P = sets[kidx[j]];
                KsatJob J{};
                J.I = P->inst->ksat_dev();
                J.R = P->k;
                std::memcpy(blob.host.data() + bb.off_kjobs + j * sizeof(KsatJob), &J, sizeof J);
                for (int v0 = 0; v0 < P->inst->n; v0 += 256)
                    items.push_back(make_int2((int)j, v0));
            }
            bb.nk_items = (int)items.size();
            bb.off_kitems = blob.take(items.size() * sizeof(int2));
            std::memcpy(blob.host.data() + bb.off_kitems, items.data(), items.size() * sizeof(int2));
        }
        if (!qidx.empty()) {
            bb.off_qjobs = blob.take(qidx.size() * sizeof(QapJob));
            std::vector<int2> items;
            for (size_t j = 0; j < qidx.size(); ++j) {
                nmc_replicas *P = sets[qidx[j]];
                QapJob J{};
                J.I = P->inst->qap_dev();
                J.R = P->q;
                std::memcpy(blob.host.data() + bb.off_qjobs + j * sizeof(QapJob), &J, sizeof J);
                for (int f = 0; f < P->inst->n; ++f)
                    items.push_back(make_int2((int)j, f));
            }
            bb.nq_items = (int)items.size();
            bb.off_qitems = blob.take(items.size() * sizeof(int2));
            std::memcpy(blob.host.data() + bb.off_qitems, items.data(), items.size() * sizeof(int2));
        }
    }
    return NMC_OK;
}

int ensure_batch_mem(nmc_batch *B, size_t bytes) {
    if (bytes <= B->cap)
        return NMC_OK;
    if (B->dev) {
        HIP_OR_FAIL(hipDeviceSynchronize());
        HIP_OR_FAIL(hipFree(B->dev));
        B->dev = nullptr;
        B->cap = 0;
    }
    const size_t cap = std::max<size_t>(align_up(bytes + bytes / 4, 1 << 20), 4 << 20);
    HIP_OR_FAIL(hipMalloc(&B->dev, cap));
    B->cap = cap;
    return NMC_OK;
}

int enqueue_phase(nmc_batch *B, const BuiltPhase &bp, hipStream_t s) {
    if (bp.nk_items)
        HIP_OR_FAIL(ksat_launch_sweep_batch(reinterpret_cast<const KsatJob *>(B->dev + bp.off_kjobs),
                                            reinterpret_cast<const int2 *>(B->dev + bp.off_kitems), bp.nk_items,
                                            bp.lds_k, bp.block_k, bp.grid_k, s));
    if (bp.nq_items)
        HIP_OR_FAIL(qap_launch_sweep_batch(reinterpret_cast<const QapJob *>(B->dev + bp.off_qjobs),
                                           reinterpret_cast<const int2 *>(B->dev + bp.off_qitems), bp.nq_items,
                                           bp.lds_q, bp.grid_q, s));
    return NMC_OK;
}

int enqueue_backbone(nmc_batch *B, const BuiltBackbone &bb, int thr_num, int thr_den, int expand, hipStream_t s) {
    if (bb.nk_items)
        HIP_OR_FAIL(ksat_launch_backbone_batch(reinterpret_cast<const KsatJob *>(B->dev + bb.off_kjobs),
                                               reinterpret_cast<const int2 *>(B->dev + bb.off_kitems), bb.nk_items,
                                               thr_num, thr_den, expand, s));
    if (bb.nq_items)
        HIP_OR_FAIL(qap_launch_backbone_batch(reinterpret_cast<const QapJob *>(B->dev + bb.off_qjobs),
                                              reinterpret_cast<const int2 *>(B->dev + bb.off_qitems), bb.nq_items,
                                              thr_num, thr_den, s));
    return NMC_OK;
}

int validate_phase(nmc_batch *B, const PhaseSpec &ph, bool backbone_available) {
    if (!ph.beta && ph.n_sweeps > 0)
        return fail(NMC_ERR_INVALID, "beta is NULL");
    if (ph.n_classes < 1 || ph.n_classes > kMaxClasses)
        return fail(NMC_ERR_INVALID, "n_classes %d outside [1, %d]", ph.n_classes, kMaxClasses);
    if (ph.n_sweeps < 0)
        return fail(NMC_ERR_INVALID, "n_sweeps must be >= 0");
    for (int64_t i = 0; i < (int64_t)ph.n_classes * ph.n_sweeps; ++i)
        if (!std::isfinite(ph.beta[i]) || ph.beta[i] < 0)
            return fail(NMC_ERR_INVALID, "beta[%lld] = %g is not finite and >= 0", (long long)i, ph.beta[i]);
    if (ph.profile == NMC_PROFILE_BACKBONE) {
        if (ph.n_classes < 2)
            return fail(NMC_ERR_INVALID, "the backbone profile needs n_classes >= 2");
        if (!backbone_available)
            for (auto *P : B->sets)
                if (!P->has_backbone)
                    return fail(NMC_ERR_STATE, "a replica set has no backbone estimate yet");
    } else if (ph.profile != NMC_PROFILE_HOMOGENEOUS) {
        return fail(NMC_ERR_UNSUPPORTED, "batched calls take the homogeneous or backbone profile");
    }
    return NMC_OK;
}

int run_batch(nmc_batch *B, const std::vector<PhaseSpec> &phases, const std::vector<char> &bb_before, int thr_num,
              int thr_den, int expand, const int64_t *targets, hipStream_t s) {
    // phases run in order; bb_before[p] != 0 puts a backbone estimate before phase p
    bool any_bb = false, seen_bb = false;
    for (size_t p = 0; p < phases.size(); ++p) {
        seen_bb = seen_bb || bb_before[p];
        any_bb = any_bb || bb_before[p];
        const int rc = validate_phase(B, phases[p], seen_bb);
        if (rc)
            return rc;
    }
    const int rounds_with_backbone_before = any_bb ? 1 : 0;
    uint64_t total = 0;
    for (const auto &ph : phases)
        total += (uint64_t)ph.n_sweeps;
    for (auto *P : B->sets)
        if ((uint64_t)P->sweeps_done + total > 0xFFFFFFFFull)
            return fail(NMC_ERR_INVALID, "sweep counter would pass 2^32 - 1");
    Blob blob;
    std::vector<BuiltPhase> built;
    BuiltBackbone bb;
    // two passes: sizes first (device base unknown), then the real layout
    int rc = build_batch(B, phases, rounds_with_backbone_before != 0, targets, nullptr, blob, built, bb);
    if (rc)
        return rc;
    rc = ensure_batch_mem(B, blob.host.size());
    if (rc)
        return rc;
    blob.host.clear();
    built.clear();
    bb = BuiltBackbone{};
    rc = build_batch(B, phases, rounds_with_backbone_before != 0, targets, B->dev, blob, built, bb);
    if (rc)
        return rc;
    HIP_OR_FAIL(hipMemcpyAsync(B->dev, blob.host.data(), blob.host.size(), hipMemcpyHostToDevice, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));

    for (size_t p = 0; p < built.size(); ++p) {
        if (bb_before[p]) {
            rc = enqueue_backbone(B, bb, thr_num, thr_den, expand, s);
            if (rc)
                return rc;
        }
        ScopedEvents evs;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (B->profiling) {
            HIP_OR_FAIL(evs.create(&e0));
            HIP_OR_FAIL(evs.create(&e1));
            HIP_OR_FAIL(hipEventRecord(e0, s));
        }
        rc = enqueue_phase(B, built[p], s);
        if (rc)
            return rc;
        if (B->profiling) {
            HIP_OR_FAIL(hipEventRecord(e1, s));
            HIP_OR_FAIL(hipEventSynchronize(e1));
            float ms = 0;
            HIP_OR_FAIL(hipEventElapsedTime(&ms, e0, e1));
            B->prof_ms += ms;
            B->prof_launches += 1;
            B->prof_attempts += built[p].attempts;
        }
    }
    // the descriptor blob must outlive the kernels that read it
    HIP_OR_FAIL(hipStreamSynchronize(s));
    for (auto *P : B->sets) {
        P->sweeps_done += (uint32_t)total;
        if (any_bb)
            P->has_backbone = true;
    }
    return ok();
}

// ---- per-set plans (nmc_batch_run) -----------------------------------------

// One phase of one set's plan, on the call's sweep timeline.
struct SetPhase {
    int64_t start = 0;      // sweeps from the call's start
    int32_t len = 0;        // sweeps
    int32_t nc = 1;         // classes: 1 (anneal) or 2 (reanneal)
    int32_t profile = NMC_PROFILE_HOMOGENEOUS;
    const double *beta = nullptr;  // [nc][len]
    int32_t chunk = 0;      // > 0: launches of at most this many sweeps
    bool backbone_before = false;
};

int validate_plan(const nmc_plan &p, size_t i) {
    if (p.rounds < 0 || p.anneal_sweeps < 0 || p.reanneal_sweeps < 0 || p.chunk_sweeps < 0)
        return fail(NMC_ERR_INVALID, "plan %zu: negative field", i);
    if (p.anneal_sweeps > 0 && !p.anneal_beta)
        return fail(NMC_ERR_INVALID, "plan %zu: anneal_beta is NULL", i);
    if (p.rounds > 0 && p.reanneal_sweeps > 0 && !p.reanneal_beta)
        return fail(NMC_ERR_INVALID, "plan %zu: reanneal_beta is NULL", i);
    if (p.rounds > 0 && (p.thr_den <= 0 || p.thr_num <= 0 || p.thr_num > p.thr_den))
        return fail(NMC_ERR_INVALID, "plan %zu: need 0 < thr_num <= thr_den", i);
    for (int64_t t = 0; t < p.anneal_sweeps; ++t)
        if (!std::isfinite(p.anneal_beta[t]) || p.anneal_beta[t] < 0)
            return fail(NMC_ERR_INVALID, "plan %zu: anneal_beta[%lld] is not finite and >= 0", i, (long long)t);
    if (p.rounds > 0)
        for (int64_t t = 0; t < 2 * (int64_t)p.reanneal_sweeps; ++t)
            if (!std::isfinite(p.reanneal_beta[t]) || p.reanneal_beta[t] < 0)
                return fail(NMC_ERR_INVALID, "plan %zu: reanneal_beta[%lld] is not finite and >= 0", i,
                            (long long)t);
    return NMC_OK;
}

std::vector<SetPhase> plan_phases(const nmc_plan &p) {
    std::vector<SetPhase> v;
    SetPhase a;
    a.len = p.anneal_sweeps;
    a.beta = p.anneal_beta;
    a.chunk = p.chunk_sweeps;
    v.push_back(a);
    int64_t t = a.len;
    for (int32_t r = 0; r < p.rounds; ++r) {
        SetPhase ph;
        ph.start = t;
        ph.len = p.reanneal_sweeps;
        ph.nc = 2;
        ph.profile = NMC_PROFILE_BACKBONE;
        ph.beta = p.reanneal_beta;
        ph.chunk = p.chunk_sweeps;
        ph.backbone_before = true;
        v.push_back(ph);
        t += ph.len;
    }
    return v;
}

// Lay out every launch of the per-set plans: the call's timeline is cut at
// every phase and chunk boundary of every set, so that in each stage a set
// runs sweeps of one phase only (or none: its plan is done); a set's backbone
// estimates run at the start of its reanneal rounds.  Thresholds are built per
// (kind, classes, sweeps, betas) and shared by the sets whose slices agree.
int build_plans(nmc_batch *B, const std::vector<std::vector<SetPhase>> &ph, const std::vector<nmc_plan> &plans,
                const int64_t *targets, uint8_t *dev_base, Blob &blob, std::vector<BatchLaunch> &launches) {
    const std::vector<nmc_replicas *> &sets = B->sets;
    const size_t ns = sets.size();
    int32_t stride_k = 1, ha = 1;
    std::vector<nmc_replicas *> ks;
    for (auto *P : sets) {
        if (P->inst->kind == NMC_KIND_KSAT) {
            stride_k = std::max(stride_k, P->inst->dmax + 1);
            ks.push_back(P);
        } else {
            ha = std::max(ha, P->inst->qap_ha);
        }
    }
    const int32_t stride_q = qap_row_words(ha);
    const int block_k = B->block_threads > 0 ? B->block_threads : heuristic_block(ks);
    const int cus = device_cus();
    // stage boundaries
    std::vector<int64_t> cut;
    for (size_t i = 0; i < ns; ++i)
        for (const SetPhase &p : ph[i]) {
            const int64_t K = p.chunk > 0 ? p.chunk : std::max<int64_t>(p.len, 1);
            for (int64_t s0 = 0; s0 < p.len; s0 += K)
                cut.push_back(p.start + s0);
            cut.push_back(p.start + p.len);
            cut.push_back(p.start);
        }
    std::sort(cut.begin(), cut.end());
    cut.erase(std::unique(cut.begin(), cut.end()), cut.end());
    std::map<std::string, size_t> tab_at;
    std::map<size_t, bool> tab_mono;  // per QAP table: every row's T never increases
    auto table = [&](bool ksat, const SetPhase &p, int64_t off, int32_t len) -> size_t {
        std::string key(1, ksat ? 'k' : 'q');
        key.push_back((char)p.nc);
        for (int32_t c = 0; c < p.nc; ++c)
            key.append(reinterpret_cast<const char *>(p.beta + (size_t)c * p.len + off), (size_t)len * sizeof(double));
        auto it = tab_at.find(key);
        if (it != tab_at.end())
            return it->second;
        const int32_t stride = ksat ? stride_k : stride_q;
        const size_t at = blob.take(std::max<size_t>((size_t)len * p.nc * stride * 4, 4));
        bool mono = true;
        for (int32_t sw = 0; sw < len; ++sw)
            for (int32_t c = 0; c < p.nc; ++c) {
                uint32_t *row = reinterpret_cast<uint32_t *>(blob.host.data() + at) + ((size_t)sw * p.nc + c) * stride;
                const double b = p.beta[(size_t)c * p.len + off + sw];
                if (ksat) {
                    row[0] = 0xFFFFFFFFu;
                    for (int32_t d = 1; d < stride_k; ++d)
                        row[d] = threshold(b, d);
                } else {
                    mono = qap_fill_row(row, b, ha) && mono;
                }
            }
        tab_mono[at] = mono;
        tab_at.emplace(std::move(key), at);
        return at;
    };
    auto by_cost = [](const std::pair<double, int2> &x, const std::pair<double, int2> &y) { return x.first > y.first; };
    for (size_t k = 0; k < cut.size(); ++k) {
        const int64_t T = cut[k];
        // backbone estimates due at T, one launch per kind and rule
        std::map<std::tuple<int, int, int, int>, std::vector<size_t>> bb_groups;
        for (size_t i = 0; i < ns; ++i)
            for (const SetPhase &p : ph[i])
                if (p.backbone_before && p.start == T) {
                    const bool kq = sets[i]->inst->kind == NMC_KIND_KSAT;
                    bb_groups[{kq ? 2 : 3, plans[i].thr_num, plans[i].thr_den, kq ? (plans[i].expand ? 1 : 0) : 0}]
                        .push_back(i);
                    break;  // several zero-length rounds at T estimate the same states
                }
        for (auto &g : bb_groups) {
            BatchLaunch L;
            L.what = std::get<0>(g.first);
            L.thr_num = std::get<1>(g.first);
            L.thr_den = std::get<2>(g.first);
            L.expand = std::get<3>(g.first);
            const bool kq = L.what == 2;
            std::vector<int2> items;
            L.off_jobs = blob.take(g.second.size() * (kq ? sizeof(KsatJob) : sizeof(QapJob)));
            for (size_t j = 0; j < g.second.size(); ++j) {
                nmc_replicas *P = sets[g.second[j]];
                if (kq) {
                    KsatJob J{};
                    J.I = P->inst->ksat_dev();
                    J.R = P->k;
                    std::memcpy(blob.host.data() + L.off_jobs + j * sizeof(KsatJob), &J, sizeof J);
                    for (int v0 = 0; v0 < P->inst->n; v0 += 256)
                        items.push_back(make_int2((int)j, v0));
                } else {
                    QapJob J{};
                    J.I = P->inst->qap_dev();
                    J.R = P->q;
                    std::memcpy(blob.host.data() + L.off_jobs + j * sizeof(QapJob), &J, sizeof J);
                    for (int f = 0; f < P->inst->n; ++f)
                        items.push_back(make_int2((int)j, f));
                }
            }
            L.n_items = (int32_t)items.size();
            L.off_items = blob.take(items.size() * sizeof(int2));
            std::memcpy(blob.host.data() + L.off_items, items.data(), items.size() * sizeof(int2));
            if (L.n_items)
                launches.push_back(L);
        }
        if (k + 1 == cut.size())
            break;
        const int64_t T1 = cut[k + 1];
        const int32_t len = (int32_t)(T1 - T);
        std::vector<KsatJob> kj;
        std::vector<QapJob> qj;
        std::vector<std::pair<double, int2>> kit, qit;
        size_t lds_k = 0, lds_q = 0;
        double att_k = 0, att_q = 0;
        for (size_t i = 0; i < ns; ++i) {
            const SetPhase *cur = nullptr;
            for (const SetPhase &p : ph[i])
                if (p.len > 0 && p.start <= T && T < p.start + p.len)
                    cur = &p;
            if (!cur)
                continue;  // this set's plan is done (or between zero-length phases)
            nmc_replicas *P = sets[i];
            const int64_t off = T - cur->start;
            const bool kq = P->inst->kind == NMC_KIND_KSAT;
            const size_t tab = table(kq, *cur, off, len);
            const int64_t tg = targets ? targets[i] : -1;
            if (kq) {
                KsatJob J{};
                J.I = P->inst->ksat_dev();
                J.R = P->k;
                J.C.tab = reinterpret_cast<const uint32_t *>(dev_base + tab);
                J.C.var_cls = cur->profile == NMC_PROFILE_BACKBONE ? P->k.cls : nullptr;
                J.C.n_classes = cur->nc;
                J.C.stride = stride_k;
                J.C.n_sweeps = len;
                J.C.sweep_words = cur->nc * stride_k;
                J.C.t0 = P->sweeps_done + (uint32_t)T;
                J.C.target = (int32_t)std::max<int64_t>(std::min<int64_t>(tg, INT32_MAX), INT32_MIN);
                J.C.check_start = 1;
                J.C.key0 = (uint32_t)P->seed;
                J.C.key1 = (uint32_t)(P->seed >> 32);
                J.C.gpw = P->gpw;
                const double cost = (double)P->inst->n * (P->inst->dmax + 1) * P->gpw;
                for (int gi = 0; gi < (P->G + P->gpw - 1) / P->gpw; ++gi)
                    kit.push_back({cost, make_int2((int)kj.size(), gi)});
                lds_k = std::max(lds_k, ksat_sweep_lds_bytes(P->inst->n, cur->nc, stride_k));
                att_k += (double)P->R * P->inst->n * len;
                kj.push_back(J);
            } else {
                QapJob J{};
                J.I = P->inst->qap_dev();
                J.I.ha = ha;
                J.R = P->q;
                J.C.tab = reinterpret_cast<const uint32_t *>(dev_base + tab);
                J.C.fac_cls = cur->profile == NMC_PROFILE_BACKBONE ? P->q.cls : nullptr;
                J.C.n_classes = cur->nc;
                J.C.stride = stride_q;
                J.C.n_sweeps = len;
                J.C.sweep_words = cur->nc * stride_q;
                J.C.t0 = P->sweeps_done + (uint32_t)T;
                J.C.target = tg;
                J.C.check_start = 1;
                J.C.rows = qap_rows_setting();
                J.C.tab_allow = qap_tab_setting();
                J.C.quad_allow = qap_quad_setting();
                J.C.dstar = tab_mono[tab] && qap_dstar_setting();
                J.C.key0 = (uint32_t)P->seed;
                J.C.key1 = (uint32_t)(P->seed >> 32);
                const double nd = P->inst->n;
                const int blocks = (P->R + kQapRepPerBlock - 1) / kQapRepPerBlock;
                for (int b = 0; b < blocks; ++b)
                    qit.push_back({nd * nd * nd, make_int2((int)qj.size(), b)});
                lds_q = std::max(lds_q, qap_sweep_lds_bytes(P->inst->n, cur->nc, stride_q));
                att_q += (double)P->R * nd * (nd - 1) / 2.0 * len;
                qj.push_back(J);
            }
        }
        std::stable_sort(kit.begin(), kit.end(), by_cost);
        std::stable_sort(qit.begin(), qit.end(), by_cost);
        if (!kj.empty()) {
            if (lds_k > kLdsBytes)
                return fail(NMC_ERR_CAPACITY, "batched k-SAT sweep needs %zu bytes of LDS", lds_k);
            BatchLaunch L;
            L.what = 0;
            L.off_jobs = blob.take(kj.size() * sizeof(KsatJob));
            std::memcpy(blob.host.data() + L.off_jobs, kj.data(), kj.size() * sizeof(KsatJob));
            L.off_items = blob.take(kit.size() * sizeof(int2));
            for (size_t t = 0; t < kit.size(); ++t)
                std::memcpy(blob.host.data() + L.off_items + t * sizeof(int2), &kit[t].second, sizeof(int2));
            L.n_items = (int32_t)kit.size();
            L.lds = lds_k;
            L.block = block_k;
            L.grid = std::min(L.n_items, ksat_batch_occupancy(block_k, lds_k) * cus);
            L.attempts = att_k;
            launches.push_back(L);
        }
        if (!qj.empty()) {
            if (lds_q > kLdsBytes)
                return fail(NMC_ERR_CAPACITY, "batched QAP sweep needs %zu bytes of LDS", lds_q);
            BatchLaunch L;
            L.what = 1;
            L.off_jobs = blob.take(qj.size() * sizeof(QapJob));
            std::memcpy(blob.host.data() + L.off_jobs, qj.data(), qj.size() * sizeof(QapJob));
            L.off_items = blob.take(qit.size() * sizeof(int2));
            for (size_t t = 0; t < qit.size(); ++t)
                std::memcpy(blob.host.data() + L.off_items + t * sizeof(int2), &qit[t].second, sizeof(int2));
            L.n_items = (int32_t)qit.size();
            L.lds = lds_q;
            L.grid = std::min(L.n_items, qap_batch_occupancy(lds_q) * cus);
            L.attempts = att_q;
            launches.push_back(L);
        }
    }
    return NMC_OK;
}

int enqueue_plan_launch(nmc_batch *B, const BatchLaunch &L, hipStream_t s) {
    const uint8_t *d = B->dev;
    switch (L.what) {
    case 0:
        HIP_OR_FAIL(ksat_launch_sweep_batch(reinterpret_cast<const KsatJob *>(d + L.off_jobs),
                                            reinterpret_cast<const int2 *>(d + L.off_items), L.n_items, L.lds,
                                            L.block, L.grid, s));
        break;
    case 1:
        HIP_OR_FAIL(qap_launch_sweep_batch(reinterpret_cast<const QapJob *>(d + L.off_jobs),
                                           reinterpret_cast<const int2 *>(d + L.off_items), L.n_items, L.lds, L.grid,
                                           s));
        break;
    case 2:
        HIP_OR_FAIL(ksat_launch_backbone_batch(reinterpret_cast<const KsatJob *>(d + L.off_jobs),
                                               reinterpret_cast<const int2 *>(d + L.off_items), L.n_items, L.thr_num,
                                               L.thr_den, L.expand, s));
        break;
    default:
        HIP_OR_FAIL(qap_launch_backbone_batch(reinterpret_cast<const QapJob *>(d + L.off_jobs),
                                              reinterpret_cast<const int2 *>(d + L.off_items), L.n_items, L.thr_num,
                                              L.thr_den, s));
        break;
    }
    return NMC_OK;
}

void drop_graph(nmc_batch *B) {
    if (B->exec) {
        (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
    }
    B->exec_launches.clear();
}

int run_plans(nmc_batch *B, const std::vector<nmc_plan> &plans, const int64_t *targets, bool use_graph,
              hipStream_t s) {
    const size_t ns = B->sets.size();
    std::vector<std::vector<SetPhase>> ph(ns);
    for (size_t i = 0; i < ns; ++i) {
        const int rc = validate_plan(plans[i], i);
        if (rc)
            return rc;
        ph[i] = plan_phases(plans[i]);
        const uint64_t total = (uint64_t)plans[i].anneal_sweeps + (uint64_t)plans[i].rounds * plans[i].reanneal_sweeps;
        if ((uint64_t)B->sets[i]->sweeps_done + total > 0xFFFFFFFFull)
            return fail(NMC_ERR_INVALID, "set %zu: sweep counter would pass 2^32 - 1", i);
    }
    // two passes: sizes first (device base unknown), then the real layout
    Blob blob;
    std::vector<BatchLaunch> launches;
    int rc = build_plans(B, ph, plans, targets, nullptr, blob, launches);
    if (rc)
        return rc;
    if (blob.host.size() > B->cap)
        drop_graph(B);  // the buffer moves: a captured graph would point at the old one
    rc = ensure_batch_mem(B, blob.host.size());
    if (rc)
        return rc;
    blob.host.clear();
    launches.clear();
    rc = build_plans(B, ph, plans, targets, B->dev, blob, launches);
    if (rc)
        return rc;
    // the descriptors are data: a graph captured for the same launch list
    // reads this call's upload (ordered before the launch on the stream)
    HIP_OR_FAIL(hipMemcpyAsync(B->dev, blob.host.data(), blob.host.size(), hipMemcpyHostToDevice, s));
    double attempts = 0;
    for (const BatchLaunch &L : launches)
        attempts += L.attempts;
    ScopedEvents evs;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (B->profiling) {
        HIP_OR_FAIL(evs.create(&e0));
        HIP_OR_FAIL(evs.create(&e1));
    }
    if (use_graph) {
        if (!(B->exec && B->exec_dev == B->dev && B->exec_launches == launches)) {
            drop_graph(B);
            if (!B->cap_stream)
                HIP_OR_FAIL(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
            HIP_OR_FAIL(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
            int erc = NMC_OK;
            for (size_t l = 0; l < launches.size() && !erc; ++l)
                erc = enqueue_plan_launch(B, launches[l], B->cap_stream);
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(B->cap_stream, &graph);
            if (erc) {
                if (graph)
                    (void)hipGraphDestroy(graph);
                return erc;
            }
            if (ee != hipSuccess)
                return fail(NMC_ERR_DEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(ee));
            hipGraphExec_t exec = nullptr;
            const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess)
                return fail(NMC_ERR_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
            B->exec = exec;
            B->exec_dev = B->dev;
            B->exec_launches = launches;
            B->graph_captures++;
        } else {
            B->graph_replays++;
        }
        if (B->profiling)
            HIP_OR_FAIL(hipEventRecord(e0, s));
        const hipError_t el = hipGraphLaunch(B->exec, s);
        if (B->profiling && el == hipSuccess)
            HIP_OR_FAIL(hipEventRecord(e1, s));
        const hipError_t es = hipStreamSynchronize(s);
        if (el != hipSuccess || es != hipSuccess) {
            drop_graph(B);
            return fail(NMC_ERR_DEVICE, "graph launch failed: %s", hipGetErrorString(el != hipSuccess ? el : es));
        }
    } else {
        if (B->profiling)
            HIP_OR_FAIL(hipEventRecord(e0, s));
        for (const BatchLaunch &L : launches) {
            rc = enqueue_plan_launch(B, L, s);
            if (rc)
                return rc;
        }
        if (B->profiling)
            HIP_OR_FAIL(hipEventRecord(e1, s));
        // the descriptor blob must outlive the kernels that read it
        HIP_OR_FAIL(hipStreamSynchronize(s));
    }
    if (B->profiling) {
        float ms = 0;
        HIP_OR_FAIL(hipEventElapsedTime(&ms, e0, e1));
        B->prof_ms += ms;
        B->prof_launches += 1;
        B->prof_attempts += attempts;
    }
    for (size_t i = 0; i < ns; ++i) {
        nmc_replicas *P = B->sets[i];
        P->sweeps_done += (uint32_t)(plans[i].anneal_sweeps + (int64_t)plans[i].rounds * plans[i].reanneal_sweeps);
        if (plans[i].rounds > 0)
            P->has_backbone = true;
    }
    return ok();
}

}  // namespace

extern "C" {

int nmc_batch_create(nmc_replicas *const *sets, int32_t n_sets, nmc_batch **out) {
    if (!out)
        return fail(NMC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!sets || n_sets < 1)
        return fail(NMC_ERR_INVALID, "need at least one replica set");
    try {
        std::unique_ptr<nmc_batch> B(new nmc_batch());
        for (int32_t i = 0; i < n_sets; ++i) {
            if (!sets[i])
                return fail(NMC_ERR_INVALID, "sets[%d] is NULL", i);
            for (int32_t j = 0; j < i; ++j)
                if (sets[j] == sets[i])
                    return fail(NMC_ERR_INVALID, "replica set %d appears twice", i);
            if (sets[i]->inst->kind == NMC_KIND_KSAT && sets[i]->inst->wide)
                return fail(NMC_ERR_UNSUPPORTED,
                            "replica set %d: batched launches are not available for wide k-SAT instances (more than %d "
                            "variables)", i, kMaxVars);
            B->sets.push_back(sets[i]);
        }
        *out = B.release();
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_batch_set_members(nmc_batch *B, nmc_replicas *const *sets, int32_t n_sets) {
    if (!B || (!sets && n_sets > 0) || n_sets < 0)
        return fail(NMC_ERR_INVALID, "bad argument");
    try {
        std::vector<nmc_replicas *> v;
        for (int32_t i = 0; i < n_sets; ++i) {
            if (!sets[i])
                return fail(NMC_ERR_INVALID, "sets[%d] is NULL", i);
            for (int32_t j = 0; j < i; ++j)
                if (sets[j] == sets[i])
                    return fail(NMC_ERR_INVALID, "replica set %d appears twice", i);
            if (sets[i]->inst->kind == NMC_KIND_KSAT && sets[i]->inst->wide)
                return fail(NMC_ERR_UNSUPPORTED,
                            "replica set %d: batched launches are not available for wide k-SAT instances (more than %d "
                            "variables)", i, kMaxVars);
            v.push_back(sets[i]);
        }
        B->sets.swap(v);
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

void nmc_batch_free(nmc_batch *B) {
    if (!B)
        return;
    if (B->dev || B->exec)
        (void)hipDeviceSynchronize();
    if (B->exec)
        (void)hipGraphExecDestroy(B->exec);
    if (B->dev)
        (void)hipFree(B->dev);
    if (B->cap_stream)
        (void)hipStreamDestroy(B->cap_stream);
    if (B->lbp_jobs) {
        (void)hipDeviceSynchronize();
        (void)hipFree(B->lbp_jobs);
    }
    if (B->lbp_pin)
        (void)hipHostFree(B->lbp_pin);
    delete B;
}

int nmc_batch_lbp_backbone(nmc_batch *B, const int32_t *replicas, int32_t which, const nmc_lbp_config *cfg,
                           nmc_lbp_result *results, void *stream) {
    if (!B || !replicas || !cfg)
        return fail(NMC_ERR_INVALID, "NULL argument");
    if (which != NMC_STATE_CURRENT && which != NMC_STATE_BEST)
        return fail(NMC_ERR_INVALID, "which must be NMC_STATE_CURRENT or NMC_STATE_BEST");
    if (int rc = lbp_check_config(*cfg))
        return rc;
    const size_t ns = B->sets.size();
    if (ns == 0)
        return ok();
    try {
        for (size_t k = 0; k < ns; ++k) {
            nmc_replicas *P = B->sets[k];
            if (!P->inst->dev)
                return fail(NMC_ERR_STATE, "set %zu: instance is not bound", k);
            if (P->inst->kind != NMC_KIND_KSAT)
                return fail(NMC_ERR_UNSUPPORTED, "set %zu: LBP runs on k-SAT instances", k);
            if (replicas[k] < 0 || replicas[k] >= P->R)
                return fail(NMC_ERR_INVALID, "set %zu: replica %d outside [0, %d)", k, replicas[k], P->R);
        }
        hipStream_t s = as_stream(stream);
        if (B->lbp_cap < ns) {
            if (B->lbp_jobs) {
                HIP_OR_FAIL(hipDeviceSynchronize());
                HIP_OR_FAIL(hipFree(B->lbp_jobs));
                B->lbp_jobs = nullptr;
            }
            if (B->lbp_pin) {
                HIP_OR_FAIL(hipHostFree(B->lbp_pin));
                B->lbp_pin = nullptr;
            }
            B->lbp_cap = 0;
            HIP_OR_FAIL(hipMalloc(reinterpret_cast<void **>(&B->lbp_jobs), ns * sizeof(LbpJob)));
            HIP_OR_FAIL(hipHostMalloc(reinterpret_cast<void **>(&B->lbp_pin), std::max<size_t>(2 * ns, 8) * 8,
                                      hipHostMallocDefault));
            B->lbp_cap = ns;
        }
        std::vector<LbpRun> runs(ns);
        std::vector<LbpJob> jobs(ns);
        LbpDims D{(int)ns, 0, 0};
        for (size_t k = 0; k < ns; ++k) {
            nmc_replicas *P = B->sets[k];
            runs[k].P = P;
            runs[k].replica = replicas[k];
            if (int rc = lbp_workspace(runs[k], s))
                return rc;
            LbpJob &J = jobs[k];
            J.I = P->inst->ksat_dev();
            J.W = runs[k].W;
            J.W.flag = runs[0].W.flag;  // one change flag for the whole batch
            J.xs_row = (which == NMC_STATE_BEST ? P->k.best_xs : P->k.xs) + (size_t)(replicas[k] / kGroup) * P->inst->n;
            J.bit = replicas[k] % kGroup;
            J.cls = P->k.cls;
            D.max_n = std::max(D.max_n, P->inst->n);
            D.max_m = std::max(D.max_m, P->inst->m);
        }
        HIP_OR_FAIL(hipMemcpyAsync(B->lbp_jobs, jobs.data(), ns * sizeof(LbpJob), hipMemcpyHostToDevice, s));
        if (int rc = lbp_run_all(runs, B->lbp_jobs, D, *cfg, B->lbp_pin, s, B->profiling, &B->lbp_ms, &B->lbp_iters))
            return rc;
        if (results)
            for (size_t k = 0; k < ns; ++k)
                lbp_fill_result(runs[k], *cfg, &results[k]);
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_batch_set_tuning(nmc_batch *B, int32_t block_threads) {
    if (!B)
        return fail(NMC_ERR_INVALID, "NULL batch");
    if (block_threads != 0 && (block_threads < 64 || block_threads > 1024 || block_threads % 64))
        return fail(NMC_ERR_INVALID, "block_threads must be 0 or a multiple of 64 in [64, 1024]");
    B->block_threads = block_threads;
    return ok();
}

int nmc_batch_anneal(nmc_batch *B, const double *beta, int32_t n_classes, int32_t n_sweeps, int32_t profile,
                     const int64_t *targets, void *stream) {
    if (!B)
        return fail(NMC_ERR_INVALID, "NULL batch");
    if (B->sets.empty())
        return ok();
    try {
        return run_batch(B, {PhaseSpec{beta, n_classes, n_sweeps, profile}}, {0}, 0, 0, 0, targets,
                         as_stream(stream));
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_batch_estimate_backbone(nmc_batch *B, int32_t thr_num, int32_t thr_den, int32_t expand, void *stream) {
    if (!B)
        return fail(NMC_ERR_INVALID, "NULL batch");
    if (thr_den <= 0 || thr_num <= 0 || thr_num > thr_den)
        return fail(NMC_ERR_INVALID, "need 0 < thr_num <= thr_den");
    if (B->sets.empty())
        return ok();
    try {
        Blob blob;
        std::vector<BuiltPhase> built;
        BuiltBackbone bb;
        int rc = build_batch(B, {}, true, nullptr, nullptr, blob, built, bb);
        if (rc)
            return rc;
        rc = ensure_batch_mem(B, blob.host.size());
        if (rc)
            return rc;
        blob.host.clear();
        bb = BuiltBackbone{};
        rc = build_batch(B, {}, true, nullptr, B->dev, blob, built, bb);
        if (rc)
            return rc;
        hipStream_t s = as_stream(stream);
        HIP_OR_FAIL(hipMemcpyAsync(B->dev, blob.host.data(), blob.host.size(), hipMemcpyHostToDevice, s));
        rc = enqueue_backbone(B, bb, thr_num, thr_den, expand ? 1 : 0, s);
        if (rc)
            return rc;
        HIP_OR_FAIL(hipStreamSynchronize(s));
        for (auto *P : B->sets)
            P->has_backbone = true;
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_batch_run_plan(nmc_batch *B, const nmc_plan *plan, const int64_t *targets, int32_t use_graph, void *stream) {
    if (!B || !plan)
        return fail(NMC_ERR_INVALID, "NULL argument");
    if (B->sets.empty())
        return ok();
    try {
        const std::vector<nmc_plan> plans(B->sets.size(), *plan);
        return run_plans(B, plans, targets, use_graph != 0, as_stream(stream));
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_batch_run(nmc_batch *B, const nmc_plan *plans, const int64_t *targets, int32_t use_graph, void *stream) {
    if (!B || (!plans && !B->sets.empty()))
        return fail(NMC_ERR_INVALID, "NULL argument");
    if (B->sets.empty())
        return ok();
    try {
        const std::vector<nmc_plan> v(plans, plans + B->sets.size());
        return run_plans(B, v, targets, use_graph != 0, as_stream(stream));
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_batch_graph_info(const nmc_batch *B, int64_t *captures, int64_t *replays) {
    if (!B)
        return fail(NMC_ERR_INVALID, "NULL batch");
    if (captures)
        *captures = B->graph_captures;
    if (replays)
        *replays = B->graph_replays;
    return ok();
}

int nmc_batch_set_profiling(nmc_batch *B, int32_t enable) {
    if (!B)
        return fail(NMC_ERR_INVALID, "NULL batch");
    B->profiling = enable != 0;
    return ok();
}

int nmc_batch_kernel_time(nmc_batch *B, double *ms, int64_t *launches, double *attempts, int32_t reset) {
    if (!B)
        return fail(NMC_ERR_INVALID, "NULL batch");
    if (ms)
        *ms = B->prof_ms;
    if (launches)
        *launches = B->prof_launches;
    if (attempts)
        *attempts = B->prof_attempts;
    if (reset) {
        B->prof_ms = 0;
        B->prof_launches = 0;
        B->prof_attempts = 0;
    }
    return ok();
}

}  // extern "C"

namespace {

// A copy of a replica set's handle whose device pointers point into another
// arena of the same layout (used to probe launch shapes without moving the
// set itself).
nmc_replicas rebased(const nmc_replicas *P, uint8_t *base) {
    nmc_replicas C = *P;
    auto mv = [&](auto *ptr) { return reinterpret_cast<decltype(ptr)>(base + (reinterpret_cast<uint8_t *>(ptr) - P->dev)); };
    C.dev = base;
    C.tab_dev = nullptr;
    C.tab_cap = 0;
    if (P->inst->kind == NMC_KIND_KSAT) {
        C.k.xs = mv(P->k.xs);
        C.k.best_xs = mv(P->k.best_xs);
        C.k.energy = mv(P->k.energy);
        C.k.best = mv(P->k.best);
        C.k.first_hit = mv(P->k.first_hit);
        C.k.cls = mv(P->k.cls);
        C.k.counts = mv(P->k.counts);
        C.k.frozen = mv(P->k.frozen);
        C.k.tally = mv(P->k.tally);
        C.k.accepted = mv(P->k.accepted);
    } else {
        C.q.perm = mv(P->q.perm);
        C.q.best_perm = mv(P->q.best_perm);
        C.q.cost = mv(P->q.cost);
        C.q.best = mv(P->q.best);
        C.q.first_hit = mv(P->q.first_hit);
        C.q.cls = mv(P->q.cls);
        C.q.freq = mv(P->q.freq);
        C.q.tally = mv(P->q.tally);
        C.q.accepted = mv(P->q.accepted);
        C.q.rows_hint = mv(P->q.rows_hint);
        C.q.dtab = mv(P->q.dtab);
    }
    C.scratch_energy = mv(P->scratch_energy);
    return C;
}

}  // namespace

extern "C" int nmc_batch_tune(nmc_batch *B, int32_t probe_sweeps, int32_t *chosen, void *stream) {
    if (!B)
        return fail(NMC_ERR_INVALID, "NULL batch");
    if (probe_sweeps < 1 || probe_sweeps > 1000)
        return fail(NMC_ERR_INVALID, "probe_sweeps must be in [1, 1000]");
    try {
        hipStream_t s = as_stream(stream);
        std::vector<nmc_replicas *> ks;
        for (auto *P : B->sets)
            if (P->inst->kind == NMC_KIND_KSAT)
                ks.push_back(P);
        if (ks.empty()) {
            if (chosen)
                *chosen = 256;
            return ok();
        }
        size_t total = 0;
        std::vector<size_t> offs;
        for (auto *P : ks) {
            offs.push_back(total);
            total += align_up(P->bytes, 256);
        }
        // releases the probe's resources and restores the setting on every exit
        struct Guard {
            nmc_batch *B;
            hipStream_t s;
            int saved;
            bool keep = false;
            uint8_t *scratch = nullptr;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            ~Guard() {
                if (e0)
                    (void)hipEventDestroy(e0);
                if (e1)
                    (void)hipEventDestroy(e1);
                if (scratch) {
                    (void)hipStreamSynchronize(s);
                    (void)hipFree(scratch);
                }
                if (!keep)
                    B->block_threads = saved;
            }
        } guard{B, s, B->block_threads};
        HIP_OR_FAIL(hipMalloc(&guard.scratch, total));
        uint8_t *scratch = guard.scratch;
        std::vector<nmc_replicas> clones;
        clones.reserve(ks.size());
        for (size_t i = 0; i < ks.size(); ++i) {
            HIP_OR_FAIL(hipMemcpyAsync(scratch + offs[i], ks[i]->dev, ks[i]->bytes, hipMemcpyDeviceToDevice, s));
            clones.push_back(rebased(ks[i], scratch + offs[i]));
        }
        std::vector<nmc_replicas *> cptr;
        for (auto &c : clones)
            cptr.push_back(&c);
        std::vector<double> beta((size_t)probe_sweeps, 1.0);
        int rc = NMC_OK;
        HIP_OR_FAIL(hipEventCreate(&guard.e0));
        HIP_OR_FAIL(hipEventCreate(&guard.e1));
        hipEvent_t e0 = guard.e0, e1 = guard.e1;
        // kernel time of probe_sweeps sweeps of every clone, in one batched
        // launch with the current settings
        auto time_config = [&](float *ms) -> int {
            Blob blob;
            std::vector<BuiltPhase> built;
            BuiltBackbone bb;
            const std::vector<PhaseSpec> ph{PhaseSpec{beta.data(), 1, probe_sweeps, NMC_PROFILE_HOMOGENEOUS}};
            int r = build_batch(B, ph, false, nullptr, nullptr, blob, built, bb, &cptr);
            if (!r)
                r = ensure_batch_mem(B, blob.host.size());
            if (r)
                return r;
            blob.host.clear();
            built.clear();
            r = build_batch(B, ph, false, nullptr, B->dev, blob, built, bb, &cptr);
            if (r)
                return r;
            HIP_OR_FAIL(hipMemcpyAsync(B->dev, blob.host.data(), blob.host.size(), hipMemcpyHostToDevice, s));
            // the shorter of two timed runs (the clones' states move on, so
            // the second run starts where the first ended)
            float best = 0;
            for (int rep = 0; rep < 2; ++rep) {
                HIP_OR_FAIL(hipEventRecord(e0, s));
                r = enqueue_phase(B, built[0], s);
                if (r)
                    return r;
                HIP_OR_FAIL(hipEventRecord(e1, s));
                HIP_OR_FAIL(hipEventSynchronize(e1));
                float t = 0;
                HIP_OR_FAIL(hipEventElapsedTime(&t, e0, e1));
                best = rep == 0 ? t : std::min(best, t);
            }
            *ms = best;
            return NMC_OK;
        };
        // (1) the workgroup size, with 4 replicas per workgroup everywhere
        for (auto &c : clones)
            c.gpw = 1;
        int best_b = 0;
        float best_ms = 0;
        for (int cand : {64, 128, 256, 512, 1024}) {
            B->block_threads = cand;
            float ms = 0;
            rc = time_config(&ms);
            if (rc)
                break;
            if (best_b == 0 || ms < best_ms) {
                best_b = cand;
                best_ms = ms;
            }
        }
        // (2) replicas per workgroup (4, or 8 sharing each spin byte), per
        // set: the sets fall into up to four classes by work (N x R), and each
        // class takes 8 when that makes the whole batch at least 1 % faster
        std::vector<int> gsel(ks.size(), 1);
        if (!rc) {
            B->block_threads = best_b;
            std::vector<size_t> ord(ks.size());
            std::iota(ord.begin(), ord.end(), 0);
            std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
                return (double)ks[a]->inst->n * ks[a]->R < (double)ks[b]->inst->n * ks[b]->R;
            });
            const size_t nb = std::min<size_t>(4, ks.size());
            for (size_t bkt = 0; bkt < nb && !rc; ++bkt) {
                const size_t lo = ord.size() * bkt / nb, hi = ord.size() * (bkt + 1) / nb;
                bool any = false;
                for (size_t i = lo; i < hi; ++i)
                    if (ks[ord[i]]->G > 1) {
                        clones[ord[i]].gpw = 2;
                        any = true;
                    }
                if (!any)
                    continue;
                float ms = 0;
                rc = time_config(&ms);
                if (!rc && ms < 0.99f * best_ms) {
                    best_ms = ms;
                    for (size_t i = lo; i < hi; ++i)
                        gsel[ord[i]] = clones[ord[i]].gpw;
                } else {
                    for (size_t i = lo; i < hi; ++i)
                        clones[ord[i]].gpw = 1;
                }
            }
        }
        if (rc)
            return rc;
        guard.keep = true;
        B->block_threads = best_b;
        for (size_t i = 0; i < ks.size(); ++i)
            ks[i]->gpw = gsel[i];
        if (chosen)
            *chosen = best_b;
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

extern "C" int nmc_tune(nmc_replicas *P, int32_t probe_sweeps, int32_t *block_threads, int32_t *reps_per_workgroup,
                        void *stream) {
    if (!P)
        return fail(NMC_ERR_INVALID, "NULL replicas");
    if (P->inst->kind != NMC_KIND_KSAT)
        return fail(NMC_ERR_UNSUPPORTED, "the tuner's settings are k-SAT settings");
    if (P->inst->wide) {
        // the wide sweeps have no workgroup-shape settings
        if (block_threads)
            *block_threads = 0;
        if (reps_per_workgroup)
            *reps_per_workgroup = 0;
        return ok();
    }
    nmc_batch *B = nullptr;
    int rc = nmc_batch_create(&P, 1, &B);
    if (rc)
        return rc;
    int32_t chosen = 0;
    rc = nmc_batch_tune(B, probe_sweeps, &chosen, stream);
    nmc_batch_free(B);
    if (rc)
        return rc;
    P->block_threads = chosen;
    if (block_threads)
        *block_threads = P->block_threads;
    if (reps_per_workgroup)
        *reps_per_workgroup = P->gpw * kGroup;
    return ok();
}

// ---------------------------------------------------------------------------
// one batched step where every set runs its own segment (serving)
// ---------------------------------------------------------------------------

extern "C" int nmc_batch_step(nmc_batch *B, const nmc_segment *segs, int32_t n_sweeps, int32_t thr_num,
                              int32_t thr_den, int32_t expand, nmc_set_status *status_out, void *stream) {
    if (!B || !segs)
        return fail(NMC_ERR_INVALID, "NULL argument");
    if (n_sweeps < 0)
        return fail(NMC_ERR_INVALID, "n_sweeps must be >= 0");
    if (B->sets.empty())
        return ok();
    try {
        const size_t ns = B->sets.size();
        bool any_bb = false;
        for (size_t i = 0; i < ns; ++i) {
            const nmc_segment &g = segs[i];
            if (g.profile < 0)
                continue;
            if (g.profile != NMC_PROFILE_HOMOGENEOUS && g.profile != NMC_PROFILE_BACKBONE)
                return fail(NMC_ERR_UNSUPPORTED, "segment %zu: profile must be homogeneous or backbone", i);
            for (int c = 0; c < 2; ++c)
                if (!std::isfinite(g.beta[c]) || g.beta[c] < 0)
                    return fail(NMC_ERR_INVALID, "segment %zu: beta not finite and >= 0", i);
            if (g.profile == NMC_PROFILE_BACKBONE && !g.backbone_before && !B->sets[i]->has_backbone)
                return fail(NMC_ERR_STATE, "segment %zu: no backbone estimate yet", i);
            if ((uint64_t)B->sets[i]->sweeps_done + (uint64_t)n_sweeps > 0xFFFFFFFFull)
                return fail(NMC_ERR_INVALID, "segment %zu: sweep counter would pass 2^32 - 1", i);
            any_bb = any_bb || g.backbone_before;
        }
        if (any_bb && (thr_den <= 0 || thr_num <= 0 || thr_num > thr_den))
            return fail(NMC_ERR_INVALID, "need 0 < thr_num <= thr_den");
        hipStream_t s = as_stream(stream);
        int32_t stride_k = 1, ha = 1;
        for (size_t i = 0; i < ns; ++i) {
            if (segs[i].profile < 0)
                continue;
            const nmc_instance *I = B->sets[i]->inst;
            if (I->kind == NMC_KIND_KSAT)
                stride_k = std::max(stride_k, I->dmax + 1);
            else
                ha = std::max(ha, I->qap_ha);
        }
        const int32_t stride_q = qap_row_words(ha);
        std::vector<nmc_replicas *> ks;
        for (size_t i = 0; i < ns; ++i)
            if (segs[i].profile >= 0 && B->sets[i]->inst->kind == NMC_KIND_KSAT)
                ks.push_back(B->sets[i]);
        const int block_k = B->block_threads > 0 ? B->block_threads : heuristic_block(ks);
        const int cus = device_cus();

        // two passes over the layout: sizes, then contents with device addresses
        Blob blob;
        size_t off_kjobs = 0, off_kitems = 0, off_qjobs = 0, off_qitems = 0, off_bbk = 0, off_bbki = 0, off_bbq = 0,
               off_bbqi = 0, off_src = 0, off_out = 0;
        int nk = 0, nq = 0, nbk = 0, nbq = 0;
        size_t lds_k = 0, lds_q = 0;
        for (int pass = 0; pass < 2; ++pass) {
            uint8_t *base = pass ? B->dev : nullptr;
            blob.host.clear();
            std::vector<KsatJob> kj;
            std::vector<QapJob> qj;
            std::vector<std::pair<double, int2>> kit, qit;
            std::vector<int2> bbk, bbq;
            std::vector<KsatJob> bbkj;
            std::vector<QapJob> bbqj;
            for (size_t i = 0; i < ns; ++i) {
                const nmc_segment &g = segs[i];
                if (g.profile < 0)
                    continue;
                nmc_replicas *P = B->sets[i];
                const int32_t nc = g.profile == NMC_PROFILE_BACKBONE ? 2 : 1;
                if (P->inst->kind == NMC_KIND_KSAT) {
                    const size_t off = blob.take((size_t)nc * stride_k * 4);
                    uint32_t *t = reinterpret_cast<uint32_t *>(blob.host.data() + off);
                    for (int32_t c = 0; c < nc; ++c) {
                        t[(size_t)c * stride_k] = 0xFFFFFFFFu;
                        for (int32_t d = 1; d < stride_k; ++d)
                            t[(size_t)c * stride_k + d] = threshold(g.beta[c], d);
                    }
                    KsatJob J{};
                    J.I = P->inst->ksat_dev();
                    J.R = P->k;
                    J.C.tab = reinterpret_cast<const uint32_t *>(base + off);
                    J.C.var_cls = nc == 2 ? P->k.cls : nullptr;
                    J.C.n_classes = nc;
                    J.C.stride = stride_k;
                    J.C.n_sweeps = n_sweeps;
                    J.C.sweep_words = 0;
                    J.C.t0 = P->sweeps_done;
                    J.C.target = (int32_t)std::max<int64_t>(std::min<int64_t>(g.target, INT32_MAX), INT32_MIN);
                    J.C.check_start = 1;
                    J.C.key0 = (uint32_t)P->seed;
                    J.C.key1 = (uint32_t)(P->seed >> 32);
                    J.C.gpw = P->gpw;
                    const double cost = (double)P->inst->n * (P->inst->dmax + 1) * P->gpw;
                    for (int gi = 0; gi < (P->G + P->gpw - 1) / P->gpw; ++gi)
                        kit.push_back({cost, make_int2((int)kj.size(), gi)});
                    lds_k = std::max(lds_k, ksat_sweep_lds_bytes(P->inst->n, nc, stride_k));
                    kj.push_back(J);
                    if (g.backbone_before) {
                        for (int v0 = 0; v0 < P->inst->n; v0 += 256)
                            bbk.push_back(make_int2((int)bbkj.size(), v0));
                        bbkj.push_back(J);
                    }
                } else {
                    const size_t off = blob.take((size_t)nc * stride_q * 4);
                    uint32_t *t = reinterpret_cast<uint32_t *>(blob.host.data() + off);
                    bool mono = true;
                    for (int32_t c = 0; c < nc; ++c)
                        mono = qap_fill_row(t + (size_t)c * stride_q, g.beta[c], ha) && mono;
                    QapJob J{};
                    J.I = P->inst->qap_dev();
                    J.I.ha = ha;
                    J.R = P->q;
                    J.C.tab = reinterpret_cast<const uint32_t *>(base + off);
                    J.C.fac_cls = nc == 2 ? P->q.cls : nullptr;
                    J.C.n_classes = nc;
                    J.C.stride = stride_q;
                    J.C.n_sweeps = n_sweeps;
                    J.C.sweep_words = 0;
                    J.C.t0 = P->sweeps_done;
                    J.C.target = g.target;
                    J.C.check_start = 1;
                    J.C.rows = qap_rows_setting();
                    J.C.tab_allow = qap_tab_setting();
                    J.C.quad_allow = qap_quad_setting();
                    J.C.dstar = mono && qap_dstar_setting();
                    J.C.key0 = (uint32_t)P->seed;
                    J.C.key1 = (uint32_t)(P->seed >> 32);
                    const double nd = P->inst->n;
                    const int blocks = (P->R + kQapRepPerBlock - 1) / kQapRepPerBlock;
                    for (int b = 0; b < blocks; ++b)
                        qit.push_back({nd * nd * nd, make_int2((int)qj.size(), b)});
                    lds_q = std::max(lds_q, qap_sweep_lds_bytes(P->inst->n, nc, stride_q));
                    qj.push_back(J);
                    if (g.backbone_before) {
                        for (int f = 0; f < P->inst->n; ++f)
                            bbq.push_back(make_int2((int)bbqj.size(), f));
                        bbqj.push_back(J);
                    }
                }
            }
            auto by_cost = [](const std::pair<double, int2> &x, const std::pair<double, int2> &y) {
                return x.first > y.first;
            };
            std::stable_sort(kit.begin(), kit.end(), by_cost);
            std::stable_sort(qit.begin(), qit.end(), by_cost);
            auto put = [&](size_t &off, const void *src, size_t bytes) {
                off = blob.take(std::max<size_t>(bytes, 16));
                if (bytes)
                    std::memcpy(blob.host.data() + off, src, bytes);
            };
            std::vector<int2> kitems, qitems;
            for (auto &p : kit)
                kitems.push_back(p.second);
            for (auto &p : qit)
                qitems.push_back(p.second);
            put(off_kjobs, kj.data(), kj.size() * sizeof(KsatJob));
            put(off_kitems, kitems.data(), kitems.size() * sizeof(int2));
            put(off_qjobs, qj.data(), qj.size() * sizeof(QapJob));
            put(off_qitems, qitems.data(), qitems.size() * sizeof(int2));
            put(off_bbk, bbkj.data(), bbkj.size() * sizeof(KsatJob));
            put(off_bbki, bbk.data(), bbk.size() * sizeof(int2));
            put(off_bbq, bbqj.data(), bbqj.size() * sizeof(QapJob));
            put(off_bbqi, bbq.data(), bbq.size() * sizeof(int2));
            std::vector<SetStatusSrc> src(ns);
            for (size_t i = 0; i < ns; ++i) {
                nmc_replicas *P = B->sets[i];
                const bool k = P->inst->kind == NMC_KIND_KSAT;
                src[i].best = k ? (const void *)P->k.best : (const void *)P->q.best;
                src[i].first_hit = k ? P->k.first_hit : P->q.first_hit;
                src[i].n_rep = P->R;
                src[i].best_is_64 = k ? 0 : 1;
            }
            put(off_src, src.data(), src.size() * sizeof(SetStatusSrc));
            off_out = blob.take(ns * sizeof(SetStatus));
            nk = (int)kitems.size();
            nq = (int)qitems.size();
            nbk = (int)bbk.size();
            nbq = (int)bbq.size();
            if (pass == 0) {
                if (lds_k > kLdsBytes || lds_q > kLdsBytes)
                    return fail(NMC_ERR_CAPACITY, "batched step needs more LDS than a workgroup has");
                const int rc = ensure_batch_mem(B, blob.host.size());
                if (rc)
                    return rc;
            }
        }
        HIP_OR_FAIL(hipMemcpyAsync(B->dev, blob.host.data(), blob.host.size(), hipMemcpyHostToDevice, s));
        if (nbk)
            HIP_OR_FAIL(ksat_launch_backbone_batch(reinterpret_cast<const KsatJob *>(B->dev + off_bbk),
                                                   reinterpret_cast<const int2 *>(B->dev + off_bbki), nbk, thr_num,
                                                   thr_den, expand ? 1 : 0, s));
        if (nbq)
            HIP_OR_FAIL(qap_launch_backbone_batch(reinterpret_cast<const QapJob *>(B->dev + off_bbq),
                                                  reinterpret_cast<const int2 *>(B->dev + off_bbqi), nbq, thr_num,
                                                  thr_den, s));
        if (nk) {
            const int grid = std::min(nk, ksat_batch_occupancy(block_k, lds_k) * cus);
            HIP_OR_FAIL(ksat_launch_sweep_batch(reinterpret_cast<const KsatJob *>(B->dev + off_kjobs),
                                                reinterpret_cast<const int2 *>(B->dev + off_kitems), nk, lds_k,
                                                block_k, grid, s));
        }
        if (nq) {
            const int grid = std::min(nq, qap_batch_occupancy(lds_q) * cus);
            HIP_OR_FAIL(qap_launch_sweep_batch(reinterpret_cast<const QapJob *>(B->dev + off_qjobs),
                                               reinterpret_cast<const int2 *>(B->dev + off_qitems), nq, lds_q, grid,
                                               s));
        }
        HIP_OR_FAIL(launch_set_status(reinterpret_cast<const SetStatusSrc *>(B->dev + off_src),
                                      reinterpret_cast<SetStatus *>(B->dev + off_out), (int)ns, s));
        std::vector<SetStatus> st(ns);
        HIP_OR_FAIL(hipMemcpyAsync(st.data(), B->dev + off_out, ns * sizeof(SetStatus), hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
        for (size_t i = 0; i < ns; ++i) {
            if (segs[i].profile >= 0) {
                B->sets[i]->sweeps_done += (uint32_t)n_sweeps;
                if (segs[i].backbone_before)
                    B->sets[i]->has_backbone = true;
            }
            if (status_out) {
                status_out[i].best = st[i].best;
                status_out[i].n_at_zero = st[i].n_zero;
                status_out[i].first_hit = st[i].first_hit;
            }
        }
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(NMC_ERR_CAPACITY, "host allocation failed");
    }
}
