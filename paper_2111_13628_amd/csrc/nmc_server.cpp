// Continuous-batching solve server built on the batched step of the C ABI.
//
// Threads: loader threads turn submitted requests into loaded instances
// (host-side layout work); two worker threads, one per request kind, make
// every HIP call, each on its own stream, so that their launches overlap on
// the GPU and a slow round of one kind does not hold up the other.  A worker
// admits loaded requests of its kind in arrival order while the device bytes
// of all admitted requests fit under the cap, runs one batched step of
// chunk_sweeps sweeps over its admitted requests (each at its own point of its
// own schedule), reads the per-request status, and retires requests at
// targets, budgets or schedule ends.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/nmc.h"
#include "nmc_internal.h"

namespace {

struct Req {
    uint64_t id = 0;
    nmc_request r{};
    std::vector<int32_t> cptr, lits, flow, dist;
    nmc_instance *inst = nullptr;
    nmc_replicas *rep = nullptr;
    void *dev_inst = nullptr, *dev_rep = nullptr;
    size_t inst_bytes = 0, rep_bytes = 0;
    int phase = 0;  // 0 = anneal, 1..rounds = reanneal round
    int chunk = 0;  // round within the phase
    nmc_result res{};
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void set_msg(nmc_result &res, const char *what) {
    std::snprintf(res.message, sizeof res.message, "%s: %s", what, nmc_last_error());
}

}  // namespace

struct nmc_server {
    nmc_server_config cfg{};
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> to_load, loaded;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> all;
    std::vector<Req *> active[2];  // per worker: [0] k-SAT, [1] QAP
    std::vector<std::thread> loaders;
    std::thread workers[2];
    bool stop = false;
    uint64_t next_id = 1;
    int64_t rounds = 0, submitted = 0, completed = 0;
    size_t bytes_in_use = 0;
    uint64_t release_gen = 0;  // bumped whenever device bytes or active slots are given back
    double busy_s = 0;
    int init_rc = NMC_OK;
    char init_msg[128] = {0};
};

namespace {

void loader_main(nmc_server *S) {
    for (;;) {
        Req *q = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->to_load.empty(); });
            if (S->stop)
                return;
            q = S->to_load.front();
            S->to_load.pop_front();
        }
        int rc;
        if (q->r.kind == NMC_KIND_KSAT)
            rc = nmc_ksat_load(q->r.n_vars, q->r.n_clauses, q->cptr.data(), q->lits.data(), q->r.class_cap,
                               &q->inst);
        else
            rc = nmc_qap_load(q->r.n, q->flow.data(), q->dist.data(), &q->inst);
        if (rc == NMC_OK) {
            // served requests run in batched launches, which take the LDS layout
            nmc_instance_info info{};
            rc = nmc_instance_get_info(q->inst, &info);
            if (rc == NMC_OK && info.wide)
                rc = nmc::set_last_error(NMC_ERR_UNSUPPORTED,
                                         "served k-SAT requests need the LDS layout (at most 65534 variables)");
        }
        if (rc == NMC_OK)
            rc = nmc_footprint(q->inst, q->r.n_replicas, &q->inst_bytes, &q->rep_bytes);
        // the instance holds its own layout from here on
        std::vector<int32_t>().swap(q->cptr);
        std::vector<int32_t>().swap(q->lits);
        std::vector<int32_t>().swap(q->flow);
        std::vector<int32_t>().swap(q->dist);
        std::lock_guard<std::mutex> lk(S->mu);
        if (rc != NMC_OK) {
            set_msg(q->res, "load");
            q->res.status = NMC_REQ_FAILED;
            q->res.t_done = seconds_since(S->t0);
            if (q->inst) {
                nmc_instance_free(q->inst);
                q->inst = nullptr;
            }
            S->completed++;
        } else {
            q->res.status = NMC_REQ_LOADED;
            q->res.device_bytes = q->inst_bytes + q->rep_bytes;
            // loaded requests wait in arrival order
            auto at = std::upper_bound(S->loaded.begin(), S->loaded.end(), q,
                                       [](const Req *a, const Req *b) { return a->id < b->id; });
            S->loaded.insert(at, q);
        }
        S->cv.notify_all();
    }
}

// Device memory of requests comes from a stream-ordered pool of the worker:
// a plain hipFree would wait for the whole device, including the other
// worker's launches.
struct DevMem {
    hipMemPool_t pool = nullptr;
    hipStream_t s = nullptr;
};

// device resources of a request (worker thread only)
void release(Req *q, const DevMem &m) {
    if (q->rep)
        nmc_replicas_free(q->rep);
    if (q->inst)
        nmc_instance_free(q->inst);
    if (q->dev_rep)
        (void)hipFreeAsync(q->dev_rep, m.s);
    if (q->dev_inst)
        (void)hipFreeAsync(q->dev_inst, m.s);
    q->rep = nullptr;
    q->inst = nullptr;
    q->dev_rep = q->dev_inst = nullptr;
}

// On failure the reason goes to msg (the caller publishes it under the lock).
bool admit(Req *q, const DevMem &m, char (&msg)[sizeof(nmc_result::message)]) {
    const char *what = "device allocation";
    hipStream_t s = m.s;
    if (hipMallocFromPoolAsync(&q->dev_inst, std::max<size_t>(q->inst_bytes, 256), m.pool, s) != hipSuccess ||
        hipMallocFromPoolAsync(&q->dev_rep, std::max<size_t>(q->rep_bytes, 256), m.pool, s) != hipSuccess) {
        (void)hipGetLastError();
        std::snprintf(msg, sizeof msg, "device allocation failed");
        return false;
    }
    what = "bind";
    if (nmc_instance_bind(q->inst, q->dev_inst, q->inst_bytes, s) == NMC_OK) {
        what = "create";
        if (nmc_replicas_create(q->inst, q->r.n_replicas, q->r.seed, q->dev_rep, q->rep_bytes, s, &q->rep) ==
            NMC_OK)
            return true;
    }
    std::snprintf(msg, sizeof msg, "%s: %s", what, nmc_last_error());
    return false;
}

// this round's segment of request q's plan
nmc_segment segment_of(const Req *q, int K) {
    nmc_segment g{};
    g.target = q->r.has_target ? q->r.target : INT64_MIN;
    const nmc_request &r = q->r;
    if (q->phase == 0) {
        const int nc = r.anneal_sweeps / K;
        const double f = nc > 1 ? (double)q->chunk / (double)(nc - 1) : 0.0;
        g.beta[0] = g.beta[1] = r.beta0 + (r.beta1 - r.beta0) * f;
        g.profile = NMC_PROFILE_HOMOGENEOUS;
        g.backbone_before = 0;
    } else {
        const int nc = r.reanneal_sweeps / K;
        const double f = nc > 1 ? (double)q->chunk / (double)(nc - 1) : 0.0;
        g.beta[0] = r.beta1;
        g.beta[1] = r.beta_hot + (r.beta1 - r.beta_hot) * f;
        g.profile = NMC_PROFILE_BACKBONE;
        g.backbone_before = q->chunk == 0;
    }
    return g;
}

// advance q's position after a round; true when its schedule is complete
bool advance(Req *q, int K) {
    const nmc_request &r = q->r;
    q->chunk++;
    const int nc = q->phase == 0 ? r.anneal_sweeps / K : r.reanneal_sweeps / K;
    if (q->chunk >= nc) {
        q->chunk = 0;
        q->phase++;
        while (q->phase >= 1 && q->phase <= r.rounds && r.reanneal_sweeps / K == 0)
            q->phase++;
    }
    return q->phase > r.rounds;
}

size_t n_active(const nmc_server *S) { return S->active[0].size() + S->active[1].size(); }

bool has_loaded(const nmc_server *S, int32_t kind) {
    for (const Req *q : S->loaded)
        if (q->r.kind == kind)
            return true;
    return false;
}

void worker_main(nmc_server *S, int w) {
    const int32_t kind = w == 0 ? NMC_KIND_KSAT : NMC_KIND_QAP;
    std::vector<Req *> &active = S->active[w];
    hipStream_t s = nullptr;
    nmc_batch *batch = nullptr;
    DevMem mem;
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = 0;
    const uint64_t keep_all = UINT64_MAX;
    if (hipSetDevice(0) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipMemPoolCreate(&mem.pool, &props) != hipSuccess ||
        hipMemPoolSetAttribute(mem.pool, hipMemPoolAttrReleaseThreshold, (void *)&keep_all) != hipSuccess) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->init_rc = NMC_ERR_DEVICE;
        std::snprintf(S->init_msg, sizeof S->init_msg, "no usable GPU for the server worker");
        S->cv.notify_all();
        if (mem.pool)
            (void)hipMemPoolDestroy(mem.pool);
        if (s)
            (void)hipStreamDestroy(s);
        return;
    }
    mem.s = s;
    const int K = S->cfg.chunk_sweeps;
    std::vector<nmc_replicas *> sets;
    std::vector<nmc_segment> segs;
    std::vector<nmc_set_status> st;
    // loaded requests left waiting by the last admission pass (for memory or
    // a slot): with nothing active, wait for a release rather than retry
    bool blocked = false;
    uint64_t seen_gen = 0;
    for (;;) {
        // admission, in arrival order, while device bytes and slots allow
        std::vector<Req *> to_admit;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] {
                return S->stop || !active.empty() ||
                       (has_loaded(S, kind) && (!blocked || S->release_gen != seen_gen));
            });
            if (S->stop)
                break;
            seen_gen = S->release_gen;
            size_t bytes = S->bytes_in_use;
            size_t slots = n_active(S);
            for (auto it = S->loaded.begin(); it != S->loaded.end() && slots < (size_t)S->cfg.max_active;) {
                Req *q = *it;
                if (q->r.kind != kind) {
                    ++it;
                    continue;
                }
                const size_t need = q->inst_bytes + q->rep_bytes;
                if (bytes + need > S->cfg.hbm_cap_bytes && slots > 0)
                    break;  // wait for memory to free up
                it = S->loaded.erase(it);
                bytes += need;
                slots++;
                to_admit.push_back(q);
            }
            // reserve the bytes now so that the other worker sees them
            for (Req *q : to_admit)
                S->bytes_in_use += q->inst_bytes + q->rep_bytes;
            blocked = has_loaded(S, kind);
        }
        for (Req *q : to_admit) {
            char msg[sizeof(nmc_result::message)] = {0};
            const bool okq = admit(q, mem, msg);
            if (!okq)
                release(q, mem);
            std::lock_guard<std::mutex> lk(S->mu);
            if (okq) {
                q->res.t_admit = seconds_since(S->t0);
                q->res.status = NMC_REQ_RUNNING;
                active.push_back(q);
            } else {
                S->bytes_in_use -= std::min(S->bytes_in_use, q->inst_bytes + q->rep_bytes);
                S->release_gen++;
                std::memcpy(q->res.message, msg, sizeof msg);
                q->res.t_done = seconds_since(S->t0);
                q->res.status = NMC_REQ_FAILED;
                S->completed++;
                S->cv.notify_all();
            }
        }
        std::vector<Req *> act;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            act = active;
        }
        if (act.empty())
            continue;
        // one round over every admitted request
        sets.clear();
        segs.clear();
        for (Req *q : act) {
            sets.push_back(q->rep);
            segs.push_back(segment_of(q, K));
        }
        st.assign(act.size(), nmc_set_status{});
        int rc = batch ? nmc_batch_set_members(batch, sets.data(), (int32_t)sets.size())
                       : nmc_batch_create(sets.data(), (int32_t)sets.size(), &batch);
        if (rc == NMC_OK && S->cfg.block_threads > 0)
            rc = nmc_batch_set_tuning(batch, S->cfg.block_threads);
        const auto t_round = std::chrono::steady_clock::now();
        if (rc == NMC_OK) {
            rc = nmc_batch_step(batch, segs.data(), K, S->cfg.thr_num, S->cfg.thr_den, S->cfg.expand, st.data(), s);
        }
        const double round_s = seconds_since(t_round);
        const double now = seconds_since(S->t0);
        // new results are formed in copies (only this worker writes an active
        // request's result, so reading it here races with nothing) and
        // published under the lock, together with status and t_done, so that a
        // poll never sees a terminal status without its completion time
        std::vector<Req *> done;
        std::vector<Req *> keep;
        std::vector<nmc_result> fresh(act.size());
        for (size_t i = 0; i < act.size(); ++i) {
            Req *q = act[i];
            nmc_result &nr = fresh[i];
            nr = q->res;
            if (rc != NMC_OK) {
                set_msg(nr, "step");
                nr.status = NMC_REQ_FAILED;
                done.push_back(q);
                continue;
            }
            nr.best = st[i].best;
            nr.n_at_zero = st[i].n_at_zero;
            nr.first_hit_sweep = st[i].first_hit;
            nr.sweeps_done += (uint32_t)K;
            const bool finished = advance(q, K);
            if (q->r.has_target && st[i].first_hit >= 0)
                nr.status = NMC_REQ_SOLVED;
            else if (finished)
                nr.status = NMC_REQ_EXHAUSTED;
            else if (q->r.budget_s > 0 && now - nr.t_admit >= q->r.budget_s)
                nr.status = NMC_REQ_TIMEOUT;
            if (nr.status == NMC_REQ_RUNNING)
                keep.push_back(q);
            else
                done.push_back(q);
        }
        size_t freed = 0;
        for (Req *q : done) {
            freed += q->dev_rep ? q->inst_bytes + q->rep_bytes : 0;
            release(q, mem);
        }
        std::lock_guard<std::mutex> lk(S->mu);
        S->rounds++;
        S->busy_s += round_s;
        for (size_t i = 0; i < act.size(); ++i) {
            if (fresh[i].status != NMC_REQ_RUNNING)
                fresh[i].t_done = now;
            act[i]->res = fresh[i];
        }
        for (size_t i = 0; i < done.size(); ++i)
            S->completed++;
        S->bytes_in_use -= std::min(S->bytes_in_use, freed);
        if (!done.empty())
            S->release_gen++;
        active.swap(keep);
        S->cv.notify_all();
    }
    // shutdown: release whatever is still on the GPU
    std::lock_guard<std::mutex> lk(S->mu);
    for (Req *q : active) {
        release(q, mem);
        if (q->res.status == NMC_REQ_RUNNING) {
            q->res.status = NMC_REQ_FAILED;
            std::snprintf(q->res.message, sizeof q->res.message, "server stopped");
        }
    }
    active.clear();
    if (batch)
        nmc_batch_free(batch);
    (void)hipStreamSynchronize(s);
    (void)hipMemPoolDestroy(mem.pool);
    (void)hipStreamDestroy(s);
}

}  // namespace

extern "C" {

int nmc_server_create(const nmc_server_config *config, nmc_server **out) {
    if (!out)
        return nmc::set_last_error(NMC_ERR_INVALID, "NULL argument");
    *out = nullptr;
    try {
        std::unique_ptr<nmc_server> S(new nmc_server());
        if (config)
            S->cfg = *config;
        if (S->cfg.hbm_cap_bytes == 0)
            S->cfg.hbm_cap_bytes = (size_t)64 << 30;
        if (S->cfg.chunk_sweeps <= 0)
            S->cfg.chunk_sweeps = 50;
        if (S->cfg.max_active <= 0)
            S->cfg.max_active = 512;
        if (S->cfg.loader_threads <= 0)
            S->cfg.loader_threads = 4;
        if (S->cfg.thr_num == 0 && S->cfg.thr_den == 0) {
            S->cfg.thr_num = 9;
            S->cfg.thr_den = 10;
            S->cfg.expand = 1;
        }
        if (S->cfg.thr_den <= 0 || S->cfg.thr_num <= 0 || S->cfg.thr_num > S->cfg.thr_den)
            return nmc::set_last_error(NMC_ERR_INVALID, "need 0 < thr_num <= thr_den");
        if (S->cfg.block_threads < 0 || S->cfg.block_threads > 1024 || S->cfg.block_threads % 64)
            return nmc::set_last_error(NMC_ERR_INVALID, "block_threads must be 0 or a multiple of 64 up to 1024");
        S->t0 = std::chrono::steady_clock::now();
        nmc_server *raw = S.get();
        for (int i = 0; i < S->cfg.loader_threads; ++i)
            S->loaders.emplace_back(loader_main, raw);
        for (int w = 0; w < 2; ++w)
            S->workers[w] = std::thread(worker_main, raw, w);
        *out = S.release();
        return NMC_OK;
    } catch (...) {
        return nmc::set_last_error(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_server_submit(nmc_server *S, const nmc_request *req, uint64_t *id) {
    if (!S || !req)
        return nmc::set_last_error(NMC_ERR_INVALID, "NULL argument");
    const int K = S->cfg.chunk_sweeps;
    if (req->kind != NMC_KIND_KSAT && req->kind != NMC_KIND_QAP)
        return nmc::set_last_error(NMC_ERR_INVALID, "kind must be NMC_KIND_KSAT or NMC_KIND_QAP");
    if (req->anneal_sweeps < K || req->anneal_sweeps % K || req->reanneal_sweeps < 0 || req->reanneal_sweeps % K ||
        req->rounds < 0 || req->n_replicas < 1)
        return nmc::set_last_error(NMC_ERR_INVALID, "anneal_sweeps must be a positive multiple of chunk_sweeps, reanneal_sweeps a multiple, rounds >= 0, n_replicas >= 1");
    try {
        std::unique_ptr<Req> q(new Req());
        q->r = *req;
        if (req->kind == NMC_KIND_KSAT) {
            if (!req->clause_ptr || req->n_clauses < 0 || req->n_vars < 1)
                return nmc::set_last_error(NMC_ERR_INVALID, "k-SAT request needs clause_ptr, n_clauses >= 0 and n_vars >= 1");
            q->cptr.assign(req->clause_ptr, req->clause_ptr + req->n_clauses + 1);
            const int32_t nl = q->cptr.back();
            if (nl < 0 || (nl > 0 && !req->lits))
                return nmc::set_last_error(NMC_ERR_INVALID, "clause_ptr ends below 0, or lits is NULL");
            q->lits.assign(req->lits, req->lits + nl);
            q->r.clause_ptr = nullptr;
            q->r.lits = nullptr;
        } else {
            if (!req->flow || !req->dist || req->n < 2 || req->n > 255)
                return nmc::set_last_error(NMC_ERR_INVALID, "QAP request needs flow, dist and 2 <= n <= 255");
            q->flow.assign(req->flow, req->flow + (size_t)req->n * req->n);
            q->dist.assign(req->dist, req->dist + (size_t)req->n * req->n);
            q->r.flow = nullptr;
            q->r.dist = nullptr;
        }
        q->res.status = NMC_REQ_QUEUED;
        q->res.first_hit_sweep = -1;
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->init_rc != NMC_OK)
            return nmc::set_last_error(S->init_rc, S->init_msg);
        q->id = S->next_id++;
        q->res.t_submit = seconds_since(S->t0);
        if (id)
            *id = q->id;
        S->to_load.push_back(q.get());
        S->all[q->id] = std::move(q);
        S->submitted++;
        S->cv.notify_all();
        return NMC_OK;
    } catch (...) {
        return nmc::set_last_error(NMC_ERR_CAPACITY, "host allocation failed");
    }
}

int nmc_server_poll(nmc_server *S, uint64_t id, nmc_result *out) {
    if (!S || !out)
        return nmc::set_last_error(NMC_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(id);
    if (it == S->all.end())
        return nmc::set_last_error(NMC_ERR_INVALID, "unknown request id");
    *out = it->second->res;
    return NMC_OK;
}

int nmc_server_wait_idle(nmc_server *S, double timeout_s) {
    if (!S)
        return nmc::set_last_error(NMC_ERR_INVALID, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    const bool done = S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                     [&] { return S->completed == S->submitted || S->init_rc != NMC_OK; });
    if (S->init_rc != NMC_OK)
        return nmc::set_last_error(S->init_rc, S->init_msg);
    return done ? NMC_OK : nmc::set_last_error(NMC_ERR_STATE, "timed out with requests still open");
}

int nmc_server_get_stats(nmc_server *S, nmc_server_stats *out) {
    if (!S || !out)
        return nmc::set_last_error(NMC_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    out->rounds = S->rounds;
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->active = (int32_t)n_active(S);
    out->waiting = (int32_t)(S->to_load.size() + S->loaded.size());
    out->device_bytes_in_use = S->bytes_in_use;
    out->gpu_busy_s = S->busy_s;
    return NMC_OK;
}

double nmc_server_now(const nmc_server *S) { return S ? seconds_since(S->t0) : 0.0; }

void nmc_server_free(nmc_server *S) {
    if (!S)
        return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    for (auto &t : S->loaders)
        t.join();
    for (auto &t : S->workers)
        if (t.joinable())
            t.join();
    for (auto &kv : S->all) {
        Req *q = kv.second.get();
        if (q->inst && !q->rep && !q->dev_inst)
            nmc_instance_free(q->inst);
    }
    delete S;
}

}  // extern "C"
