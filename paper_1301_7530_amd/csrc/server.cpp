// Serving loop: continuous batching of requests from many sequences.
//
// Each request is one system of one sequence.  A worker thread owns the
// context's stream; between blocks of iterations it admits queued requests
// (at most one in flight per sequence, in arrival order, while slots and
// the HBM budget for working sets allow), begins their solves and adds them
// to the fused launches of their type, and completes the members that
// finished (solution copied out, basis recycled, solve-time buffers
// released).  The host part of a recycle (Ritz analysis and selection) runs
// on a helper thread while the worker keeps launching the other members; its
// device part is enqueued by the worker once the helper is done, and only
// then is the request completed and its sequence free for its next request.  A member's iterations are gated by its own device status, so
// joining or leaving the launches does not change its arithmetic: every
// result equals the one of a solve alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "seq.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0, Clock::time_point t) {
    return std::chrono::duration<double, std::milli>(t - t0).count();
}

struct Request {
    krs_seq* seq = nullptr;
    krs::SeqBase* impl = nullptr;
    std::vector<double> values, b;
    double* x_out = nullptr;
    uint64_t tag = 0;
    Clock::time_point t_arrive, t_admit;
    int64_t bytes = 0;
};

}  // namespace

struct krs_server {
    krs_ctx* ctx = nullptr;
    size_t budget = 0;
    int max_slots = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::deque<krs_completion> done;
    std::set<krs::SeqBase*> busy;
    bool stop = false;
    std::thread worker;
    // statistics
    Clock::time_point t0;
    bool started = false;
    Clock::time_point t_last;
    int64_t enqueued = 0, completed = 0, failed = 0, blocks = 0, member_blocks = 0, peak_bytes = 0;
    std::vector<double> lat_ms;
    krs_status fatal = KRS_OK;
    std::string fatal_msg;

    // msg: the failure's message (null: this thread's last error)
    void post(Request& r, krs_status st, const krs_solve_info& info, int batch, const char* msg = nullptr) {
        krs_completion c;
        std::memset(&c, 0, sizeof c);
        const auto now = Clock::now();
        c.tag = r.tag;
        c.seq = r.seq;
        c.status = st;
        c.batch_size = batch;
        c.latency_ms = ms_since(r.t_arrive, now);
        c.queue_ms = ms_since(r.t_arrive, r.t_admit);
        c.info = info;
        if (st != KRS_OK) {
            const char* m = msg ? msg : krs_last_error();
            std::strncpy(c.message, m ? m : "", sizeof c.message - 1);
        }
        r.impl->in_server.fetch_sub(1);
        std::lock_guard<std::mutex> g(mu);
        busy.erase(r.impl);
        done.push_back(c);
        ++completed;
        if (st != KRS_OK && st != KRS_E_MAXIT) ++failed;
        lat_ms.push_back(c.latency_ms);
        t_last = now;
        cv_done.notify_all();
    }

    void run();
    void serve();
};

// The worker thread's body: nothing escapes it.  A host failure (an
// allocation, a thread that cannot start) inside the loop stops the server
// the way a device failure does.
void krs_server::run() {
    (void)hipSetDevice(ctx->device);
    serve();
}

void krs_server::serve() {
    struct Active {
        Request req;
        int64_t bytes;
    };
    std::map<int, std::vector<Active>> members;  // by type key
    std::map<int, std::unique_ptr<krs::RunnerBase>> runners;
    // finished members whose recycle is planned on a helper thread
    struct Pending {
        std::vector<Active> fin;
        std::vector<krs_solve_info> infos;
        std::vector<krs_status> sts;
        std::vector<krs::SeqBase*> rec;
        std::vector<size_t> rec_idx;
        std::vector<krs_status> pst;
        std::vector<std::string> msgs;  // end_solve failures
        int batch = 0;
        std::atomic<bool> planned{false};
        std::thread th;
    };
    std::deque<std::unique_ptr<Pending>> pending;
    int64_t used = 0;
    int nact = 0;
    std::vector<int32_t> stat;
    // requests of the current admission round, and how many of them have
    // been begun (or completed) so far
    std::vector<Request> admit;
    size_t admit_done = 0;
    // apply the planned recycles (in order), release and complete; with
    // `block`, wait for the oldest plan first; with `fail`, complete them
    // with that status and message instead
    auto finish_pending = [&](bool block, krs_status fail, const char* fail_msg = nullptr) {
        while (!pending.empty()) {
            Pending& p = *pending.front();
            if (!block && !p.planned.load()) break;
            block = false;
            if (p.th.joinable()) p.th.join();
            for (size_t j = 0; j < p.rec.size(); ++j) {
                const size_t i = p.rec_idx[j];
                krs_status a = p.pst[j];
                int32_t added = 0;
                if (fail != KRS_OK) {
                    a = fail;
                } else if (a == KRS_OK) {
                    a = p.rec[j]->recycle_apply(&added);
                    if (a != KRS_OK) p.msgs[i] = krs_last_error();
                } else {
                    p.msgs[i] = p.rec[j]->plan_msg;
                }
                p.infos[i].added = added;
                if (a != KRS_OK && p.sts[i] == KRS_OK) p.sts[i] = a;
            }
            for (size_t i = 0; i < p.fin.size(); ++i) {
                p.fin[i].req.impl->trim();
                used -= p.fin[i].bytes;
                post(p.fin[i].req, p.sts[i], p.infos[i], p.batch, fail != KRS_OK ? fail_msg : p.msgs[i].c_str());
            }
            pending.pop_front();
        }
    };
    // a failure of the device or the host: fail every request in flight and
    // stop serving
    auto fail_all = [&](krs_status st, const std::string& msg) {
        while (!pending.empty()) finish_pending(true, st, msg.c_str());
        for (auto& kv : members)
            for (auto& a : kv.second) {
                krs_solve_info none;
                std::memset(&none, 0, sizeof none);
                post(a.req, st, none, 0, msg.c_str());
            }
        for (size_t i = admit_done; i < admit.size(); ++i) {
            krs_solve_info none;
            std::memset(&none, 0, sizeof none);
            post(admit[i], st, none, 0, msg.c_str());
        }
        admit.clear();
        members.clear();
        runners.clear();
        std::lock_guard<std::mutex> g(mu);
        fatal = st;
        fatal_msg = msg;
        for (auto& r : queue) r.impl->in_server.fetch_sub(1);
        queue.clear();
        busy.clear();
        stop = true;
        cv_done.notify_all();
    };
    try {
        while (true) {
            finish_pending(false, KRS_OK);
            // ---- admission
            admit.clear();
            admit_done = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                if (nact == 0 && queue.empty() && pending.empty()) {
                    if (stop) break;
                    cv_work.wait_for(lk, std::chrono::milliseconds(20));
                    continue;
                }
                std::set<krs::SeqBase*> seen;  // a sequence's later requests wait for its earlier ones
                for (auto it = queue.begin(); it != queue.end();) {
                    if (nact + (int)admit.size() >= max_slots) break;
                    if (busy.count(it->impl) || seen.count(it->impl)) {
                        seen.insert(it->impl);
                        ++it;
                        continue;
                    }
                    const int64_t bytes = it->impl->working_bytes();
                    const bool fits = budget == 0 || used + bytes <= (int64_t)budget;
                    if (!fits && (nact + admit.size()) > 0) break;  // in order: wait for memory
                    it->bytes = bytes;
                    it->t_admit = Clock::now();
                    used += bytes;
                    busy.insert(it->impl);
                    admit.push_back(std::move(*it));
                    it = queue.erase(it);
                }
                peak_bytes = std::max(peak_bytes, used);
            }
            std::set<int> dirty;
            for (; admit_done < admit.size(); ++admit_done) {
                Request& r = admit[admit_done];
                krs_status st = r.impl->submit(r.values.data(), r.b.data(), false);
                if (st == KRS_OK) st = r.impl->begin_solve();
                if (st != KRS_OK) {
                    krs_solve_info none;
                    std::memset(&none, 0, sizeof none);
                    none.status = st;
                    used -= r.bytes;
                    r.impl->trim();
                    post(r, st, none, 0);
                    continue;
                }
                const int key = r.impl->type_key();
                auto& mk = members[key];
                mk.reserve(mk.size() + 1);  // the move below cannot fail half-way
                std::vector<double>().swap(r.values);
                std::vector<double>().swap(r.b);
                const int64_t bytes = r.bytes;
                mk.push_back(Active{std::move(r), bytes});
                dirty.insert(key);
                ++nact;
            }
            krs_status st = KRS_OK;
            for (int key : dirty) {
                auto& rp = runners[key];
                if (!rp) rp = krs::make_runner(ctx, key);
                std::vector<krs::SeqBase*> m;
                for (auto& a : members[key]) m.push_back(a.req.impl);
                st = rp->set_members(m);
                if (st != KRS_OK) break;
            }
            if (nact == 0 && st == KRS_OK) {
                // nothing to iterate: the queued requests wait for recycles
                finish_pending(true, KRS_OK);
                continue;
            }
            // ---- one block of iterations for every member, all types
            for (auto& kv : runners) {
                if (st != KRS_OK) break;
                if (kv.second->size() > 0) st = kv.second->launch(32, true);
            }
            if (st == KRS_OK) {
                ++blocks;
                member_blocks += nact;
            }
            // ---- completions
            for (auto& kv : runners) {
                if (st != KRS_OK) break;
                if (kv.second->size() == 0) continue;
                st = kv.second->read_status(stat);
                if (st != KRS_OK) break;
                auto& mem = members[kv.first];
                std::vector<Active> keep, fin;
                const int batch = (int)mem.size();
                std::vector<int> fin_iter;  // their final iteration counts
                for (size_t i = 0; i < mem.size(); ++i) {
                    if (krs::finished_status(stat[2 * i])) {
                        fin.push_back(std::move(mem[i]));
                        fin_iter.push_back(stat[2 * i + 1]);
                    } else {
                        keep.push_back(std::move(mem[i]));
                    }
                }
                const bool changed = !fin.empty();
                if (changed) {
                    // copy the solutions out; plan the recycles on a helper thread
                    auto p = std::make_unique<Pending>();
                    p->batch = batch;
                    p->fin = std::move(fin);
                    const size_t nf = p->fin.size();
                    p->infos.resize(nf);
                    p->sts.resize(nf);
                    p->msgs.resize(nf);
                    for (size_t i = 0; i < nf; ++i) {
                        std::memset(&p->infos[i], 0, sizeof p->infos[i]);
                        p->sts[i] =
                            p->fin[i].req.impl->end_solve(p->fin[i].req.x_out, false, &p->infos[i], fin_iter[i]);
                        if (p->sts[i] != KRS_OK) p->msgs[i] = krs_last_error();
                        if (p->sts[i] == KRS_OK || p->sts[i] == KRS_E_MAXIT) {
                            p->rec.push_back(p->fin[i].req.impl);
                            p->rec_idx.push_back(i);
                        }
                    }
                    nact -= (int)nf;
                    p->pst.assign(p->rec.size(), KRS_OK);
                    Pending* pp = p.get();
                    pending.push_back(std::move(p));
                    auto plan = [pp] {
                        krs::plan_all(pp->rec.data(), (int)pp->rec.size(), pp->pst.data());
                        pp->planned.store(true);
                    };
                    try {
                        pp->th = std::thread(plan);
                    } catch (...) {
                        plan();  // no helper thread: plan here
                    }
                }
                if (changed) {
                    mem = std::move(keep);
                    std::vector<krs::SeqBase*> m;
                    for (auto& a : mem) m.push_back(a.req.impl);
                    st = kv.second->set_members(m);
                }
            }
            if (st != KRS_OK) {
                fail_all(st, krs_last_error() ? krs_last_error() : "");
                break;
            }
        }
    } catch (const std::exception& e) {
        fail_all(KRS_E_OOM, std::string("server stopped on a host failure: ") + e.what());
    }
}

extern "C" {

krs_status krs_server_create(krs_ctx* ctx, size_t hbm_budget, int32_t max_slots, krs_server** out) {
    try {
        if (!ctx || !out || max_slots <= 0) {
            krs::set_error("ctx, out and max_slots > 0 are required");
            return KRS_E_INVALID;
        }
        *out = nullptr;
        std::unique_ptr<krs_server> s(new krs_server());
        int none = 0;
        if (!ctx->live_servers.compare_exchange_strong(none, 1)) {
            krs::set_error("the context already has a server");
            return KRS_E_STATE;
        }
        s->ctx = ctx;
        s->budget = hbm_budget;
        s->max_slots = max_slots;
        krs_server* sp = s.get();
        try {
            s->worker = std::thread([sp] { sp->run(); });
        } catch (...) {
            ctx->live_servers -= 1;
            throw;
        }
        *out = s.release();
        return KRS_OK;
    } catch (const std::exception& e) {
        krs::set_error(e.what());
        return KRS_E_OOM;
    }
}

krs_status krs_server_enqueue(krs_server* s, krs_seq* seq, const double* values, const double* b, double* x_out,
                              uint64_t tag) {
    try {
        if (!s || !seq || !values || !b) {
            krs::set_error("server, seq, values and b are required");
            return KRS_E_INVALID;
        }
        if (seq->impl->ctx != s->ctx) {
            krs::set_error("the sequence belongs to another context");
            return KRS_E_INVALID;
        }
        if (seq->impl->desc.kernel_flags & 4) {
            krs::set_error("full reorthogonalisation is not available in the server's fused batches");
            return KRS_E_INVALID;
        }
        Request r;
        r.seq = seq;
        r.impl = seq->impl.get();
        const krs_seq_desc& d = r.impl->desc;
        const size_t nv = (size_t)d.nnzb * d.block * d.block;
        r.values.assign(values, values + nv);
        r.b.assign(b, b + d.n);
        r.x_out = x_out;
        r.tag = tag;
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) {
            krs::set_error(s->fatal != KRS_OK ? "server stopped after a device error: " + s->fatal_msg
                                              : std::string("server is shutting down"));
            return KRS_E_STATE;
        }
        if (s->queue.size() >= 65536) {
            krs::set_error("server queue is full");
            return KRS_E_BUSY;
        }
        r.t_arrive = Clock::now();
        if (!s->started) {
            s->started = true;
            s->t0 = r.t_arrive;
        }
        r.impl->in_server.fetch_add(1);
        s->queue.push_back(std::move(r));
        ++s->enqueued;
        s->cv_work.notify_one();
        return KRS_OK;
    } catch (const std::bad_alloc&) {
        krs::set_error("host allocation failed");
        return KRS_E_OOM;
    }
}

krs_status krs_server_poll(krs_server* s, krs_completion* out, int32_t cap, int32_t* count, int32_t timeout_ms) {
    if (!s || !count || (cap > 0 && !out)) {
        krs::set_error("server, count (and out when cap > 0) are required");
        return KRS_E_INVALID;
    }
    *count = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_ms != 0) {
        auto pred = [s] { return !s->done.empty() || s->stop; };
        if (timeout_ms < 0) s->cv_done.wait(lk, pred);
        else s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
    }
    int k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *count = k;
    if (s->fatal != KRS_OK && k == 0) {
        krs::set_error("server stopped after a device error: " + s->fatal_msg);
        return s->fatal;
    }
    return KRS_OK;
}

krs_status krs_server_stats(krs_server* s, krs_server_report* out) {
    if (!s || !out) {
        krs::set_error("server and out are required");
        return KRS_E_INVALID;
    }
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(out, 0, sizeof *out);
    out->enqueued = s->enqueued;
    out->completed = s->completed;
    out->failed = s->failed;
    out->queued = (int64_t)s->queue.size();
    out->blocks = s->blocks;
    out->mean_batch = s->blocks ? (double)s->member_blocks / (double)s->blocks : 0.0;
    out->peak_bytes = s->peak_bytes;
    if (s->completed > 0 && s->started) {
        const double span = ms_since(s->t0, s->t_last);
        out->solves_per_s = span > 0 ? 1e3 * (double)s->completed / span : 0.0;
        std::vector<double> l;
        try {
            l = s->lat_ms;
        } catch (const std::bad_alloc&) {
            krs::set_error("host allocation failed");
            return KRS_E_OOM;
        }
        auto pct = [&l](double q) {
            const size_t i = std::min(l.size() - 1, (size_t)(q * (double)(l.size() - 1) + 0.5));
            std::nth_element(l.begin(), l.begin() + i, l.end());
            return l[i];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        double sum = 0.0;
        for (double v : s->lat_ms) sum += v;
        out->mean_ms = sum / (double)s->lat_ms.size();
    }
    return KRS_OK;
}

krs_status krs_server_destroy(krs_server* s) {
    if (!s) return KRS_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    s->ctx->live_servers -= 1;
    delete s;
    return KRS_OK;
}

}  // extern "C"
