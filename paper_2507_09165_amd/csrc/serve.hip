// Continuous-batching request loop for PSD projections (psdproj_serve_*).
//
// One scheduler thread owns `slots` HIP streams. Each request needs the
// workspace of one projection; each slot keeps its own workspace pool, grown
// to the largest request it has served. Admission (in arrival order) takes a
// free slot whose pool can host the request without the slots' total
// exceeding the HBM budget; a blocked head request may be passed by later
// ones at most max_bypass times. Work is enqueued on the slot's stream and a
// completion event is recorded; the scheduler polls the events, stamps the
// result and wakes waiters. Requests that arrive while others run are
// admitted as slots free up, so their kernels overlap on the device.
//
// Coalescing: when a request of order <= coalesce_max_n is admitted, queued
// requests of the same mode and no larger order join it (in arrival order, up
// to kMaxGroup and within the budget) and the group runs as one batched
// projection on the slot: one launch sequence covers every matrix, and each
// result is bitwise the one the request would get alone (tile shapes and
// reduction orders are per matrix).
//
// The fake executor (config.fake_executor) runs no GPU work: a request
// "completes" after a modelled time, so the admission and bookkeeping logic
// can be exercised on a machine without a GPU.
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/psdproj.h"
#include "runtime.hpp"

namespace {

int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

struct Req {
    psdproj_request r;
    int mode = 0;
    size_t ws = 0;
    int64_t submit_ns = 0, start_ns = 0, end_ns = 0;
    int status = PSDPROJ_ERR_PENDING;
    int slot = -1;
    int bypassed = 0;
    bool finished = false;
};

constexpr int kMaxGroup = 32;  // requests in one coalesced launch

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    // numerical status of the running requests: one device info record each,
    // copied to pinned host memory before `done`
    psdproj_info *info_dev = nullptr;   // kMaxGroup records
    psdproj_info *info_host = nullptr;  // kMaxGroup records (pinned)
    bool busy = false;
    std::vector<uint64_t> group;  // tickets running on this slot
    size_t held = 0;        // workspace bytes this slot's pool holds
    int64_t fake_end = 0;
};

}  // namespace

struct psdproj_server {
    psdproj_serve_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Req> reqs;
    std::vector<Slot> slots;
    std::thread th;
    bool stop = false;
    uint64_t next_ticket = 1;
    // statistics
    std::vector<double> lat_ms;
    uint64_t n_sub = 0, n_done = 0, n_rej = 0, n_cancel = 0;
    int64_t first_submit = 0, last_end = 0;
    size_t peak_held = 0;

    size_t held_total() const {
        size_t s = 0;
        for (const Slot &sl : slots) s += sl.held;
        return s;
    }
    int running() const {
        int c = 0;
        for (const Slot &sl : slots) c += sl.busy;
        return c;
    }
    void loop();
    int pick_slot(size_t ws);
    void launch(int si, const std::vector<uint64_t> &group, std::unique_lock<std::mutex> &lk);
    void poll_completions();
    // Queued requests that may run with pending[idx] in one batched call.
    std::vector<size_t> coalesce(size_t idx) const;
};

static int choose_mode(const psdproj_request &r) {
    if (r.mode >= 0) return r.mode;
    return r.target <= 1e-4 ? PSDPROJ_MODE_FP32_EMU : PSDPROJ_MODE_FP8_FP16_SPLIT;
}

std::vector<size_t> psdproj_server::coalesce(size_t idx) const {
    std::vector<size_t> pos{idx};
    const Req &h = reqs.at(pending[idx]);
    if (cfg.coalesce_max_n < 0 || h.r.n > cfg.coalesce_max_n || h.r.n == 0) return pos;
    for (size_t k = idx + 1; k < pending.size() && (int)pos.size() < kMaxGroup; ++k) {
        const Req &q = reqs.at(pending[k]);
        if (q.mode == h.mode && q.r.n > 0 && q.r.n <= cfg.coalesce_max_n) pos.push_back(k);
    }
    return pos;
}

// Pick a free slot for a request of `ws` bytes: prefer the smallest pool that
// already fits, else the largest pool whose growth keeps the budget. If no
// slot qualifies but idle slots hold pools, release idle pools (largest
// first) until one can grow. Returns -1 if the request must wait.
int psdproj_server::pick_slot(size_t ws) {
    const size_t total = held_total();
    int best = -1;
    for (int i = 0; i < (int)slots.size(); ++i) {
        const Slot &sl = slots[i];
        if (sl.busy) continue;
        if (sl.held >= ws) {
            if (best < 0 || slots[best].held < ws || sl.held < slots[best].held) best = i;
        } else if (total - sl.held + ws <= cfg.hbm_budget_bytes) {
            if (best < 0 || (slots[best].held < ws && sl.held > slots[best].held)) best = i;
        }
    }
    if (best >= 0) return best;
    std::vector<int> idle;
    for (int i = 0; i < (int)slots.size(); ++i)
        if (!slots[i].busy) idle.push_back(i);
    if (idle.empty()) return -1;
    std::sort(idle.begin(), idle.end(), [&](int a, int b) { return slots[a].held > slots[b].held; });
    const int cand = idle[0];
    size_t t = total;
    for (size_t k = 1; k < idle.size() && t - slots[cand].held + ws > cfg.hbm_budget_bytes; ++k) {
        Slot &sl = slots[idle[k]];
        if (!sl.held) continue;
        if (!cfg.fake_executor) psd::pool_release(sl.stream);  // stream is idle
        t -= sl.held;
        sl.held = 0;
    }
    return t - slots[cand].held + ws <= cfg.hbm_budget_bytes ? cand : -1;
}

void psdproj_server::launch(int si, const std::vector<uint64_t> &group, std::unique_lock<std::mutex> &lk) {
    Slot &sl = slots[si];
    sl.busy = true;
    sl.group = group;
    const int64_t t0 = now_ns();
    const int g = (int)group.size();
    std::vector<int64_t> ns(g), lds(g);
    std::vector<const float *> xs(g);
    std::vector<float *> outs(g);
    for (int k = 0; k < g; ++k) {
        Req &q = reqs[group[k]];
        q.slot = si;
        q.start_ns = t0;
        ns[k] = q.r.n;
        lds[k] = q.r.ld;
        xs[k] = q.r.X;
        outs[k] = q.r.out;
    }
    const int mode = reqs[group[0]].mode;
    size_t ws = 0;
    for (uint64_t tk : group) ws += reqs[tk].ws;
    if (cfg.fake_executor) {
        const psdproj_opts o = psd::default_opts(mode);
        double flops = 0.0;
        for (int k = 0; k < g; ++k) {
            const double n = (double)ns[k];
            flops += (double)psd::gemm_count_for(o) * n * n * (n + 1.0);
        }
        sl.fake_end = t0 + 30000 + (int64_t)(flops / (cfg.fake_tflops * 1e12) * 1e9);
        sl.held = std::max(sl.held, ws);
    } else {
        hipStream_t st = sl.stream;
        hipEvent_t ev = sl.done;
        psdproj_info *info = sl.info_dev;
        psdproj_info *host = sl.info_host;
        lk.unlock();  // enqueueing ~160 launches takes a while; let clients submit
        const psdproj_opts o = psd::default_opts(mode);
        memset(host, 0, sizeof(psdproj_info) * (size_t)g);
        int status = g == 1 ? psd::run_projection(o, ns[0], lds[0], xs[0], outs[0], st, info, false)
                            : psd::run_batched(o, g, ns.data(), lds.data(), xs.data(), outs.data(), st, info);
        if (status == PSDPROJ_OK &&
            (hipMemcpyAsync(host, info, sizeof(psdproj_info) * (size_t)g, hipMemcpyDeviceToHost, st) != hipSuccess ||
             hipEventRecord(ev, st) != hipSuccess))
            status = PSDPROJ_ERR_HIP;
        const size_t held = psd::pool_held(st);
        lk.lock();
        slots[si].held = held;
        if (status != PSDPROJ_OK) {  // nothing left in flight for these requests
            const int64_t t1 = now_ns();
            for (uint64_t tk : group) {
                Req &q2 = reqs[tk];
                q2.status = status;
                q2.end_ns = t1;
                q2.finished = true;
            }
            slots[si].busy = false;
            slots[si].group.clear();
            cv_done.notify_all();
        }
    }
    peak_held = std::max(peak_held, held_total());
}

void psdproj_server::poll_completions() {
    const int64_t t = now_ns();
    for (int i = 0; i < (int)slots.size(); ++i) {
        Slot &sl = slots[i];
        if (!sl.busy) continue;
        int status = PSDPROJ_OK;
        if (cfg.fake_executor) {
            if (t < sl.fake_end) continue;
        } else {
            const hipError_t e = hipEventQuery(sl.done);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) status = PSDPROJ_ERR_HIP;
        }
        const int64_t t1 = now_ns();
        for (size_t k = 0; k < sl.group.size(); ++k) {
            Req &q = reqs[sl.group[k]];
            q.end_ns = t1;
            // a non-finite input leaves NaN in its out (its own entry only)
            q.status = (status == PSDPROJ_OK && !cfg.fake_executor && sl.info_host[k].nonfinite)
                           ? PSDPROJ_ERR_NONFINITE : status;
            q.finished = true;
            if (q.status == PSDPROJ_OK) {
                ++n_done;
                lat_ms.push_back((q.end_ns - q.submit_ns) * 1e-6);
                last_end = std::max(last_end, q.end_ns);
            }
        }
        sl.busy = false;
        sl.group.clear();
        cv_done.notify_all();
    }
}

void psdproj_server::loop() {
    if (!cfg.fake_executor) (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        poll_completions();
        // Admissions in arrival order; a blocked head may be passed by later
        // requests at most max_bypass times. launch() drops the lock while it
        // enqueues, so the queue is rescanned after every admission.
        bool admitted = true;
        while (admitted && !pending.empty() && running() < (int)slots.size()) {
            admitted = false;
            for (size_t idx = 0; idx < pending.size(); ++idx) {
                const uint64_t tk = pending[idx];
                // the request with the queued ones it can run with, shrunk
                // from the back until the group's workspace finds a slot
                // (a group's workspace is taken as the sum of its requests'
                // single workspaces, which bounds the batched layout's: that
                // shares one set of tables and drops per-section padding)
                std::vector<size_t> pos = coalesce(idx);
                if (idx > 0) {  // every member passes the head: at most its remaining bypasses
                    const int left = cfg.max_bypass - reqs[pending.front()].bypassed;
                    if ((int)pos.size() > left) pos.resize(left > 1 ? left : 1);
                }
                int si = -1;
                while (!pos.empty()) {
                    size_t ws = 0;
                    for (size_t p : pos) ws += reqs[pending[p]].ws;
                    si = pick_slot(ws);
                    if (si >= 0 || pos.size() == 1) break;
                    pos.resize(pos.size() > 2 ? pos.size() / 2 : 1);
                }
                if (si >= 0) {
                    std::vector<uint64_t> group;
                    for (size_t p : pos) group.push_back(pending[p]);
                    for (size_t k = pos.size(); k-- > 0;) pending.erase(pending.begin() + (long)pos[k]);
                    if (idx > 0 && !pending.empty()) reqs[pending.front()].bypassed += (int)group.size();
                    launch(si, group, lk);
                    admitted = true;
                    break;
                }
                if (idx == 0 && reqs[tk].bypassed >= cfg.max_bypass) break;
            }
        }
        if (stop && pending.empty() && running() == 0) break;
        if (running() == 0 && (pending.empty() || stop)) {
            cv_work.wait(lk);
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

extern "C" {

int psdproj_serve_create(const psdproj_serve_config *cfg, psdproj_server **out) {
    if (!out) return PSDPROJ_ERR_INVALID_ARG;
    psdproj_server *s = new psdproj_server();
    if (cfg) s->cfg = *cfg;
    if (!s->cfg.hbm_budget_bytes) s->cfg.hbm_budget_bytes = (size_t)200 << 30;
    if (s->cfg.slots <= 0) s->cfg.slots = 4;
    if (s->cfg.slots > 64) { delete s; return PSDPROJ_ERR_INVALID_ARG; }
    if (s->cfg.max_bypass <= 0) s->cfg.max_bypass = 8;
    if (s->cfg.fake_tflops <= 0.0) s->cfg.fake_tflops = 500.0;
    if (s->cfg.coalesce_max_n == 0) s->cfg.coalesce_max_n = 1024;
    s->slots.resize(s->cfg.slots);
    if (!s->cfg.fake_executor) {
        if (hipGetDevice(&s->device) != hipSuccess) { delete s; return PSDPROJ_ERR_HIP; }
        for (Slot &sl : s->slots) {
            if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
                hipMalloc((void **)&sl.info_dev, sizeof(psdproj_info) * kMaxGroup) != hipSuccess ||
                hipHostMalloc((void **)&sl.info_host, sizeof(psdproj_info) * kMaxGroup, hipHostMallocDefault) !=
                    hipSuccess) {
                for (Slot &x : s->slots) {
                    if (x.done) (void)hipEventDestroy(x.done);
                    if (x.stream) (void)hipStreamDestroy(x.stream);
                    if (x.info_dev) (void)hipFree(x.info_dev);
                    if (x.info_host) (void)hipHostFree(x.info_host);
                }
                delete s;
                return PSDPROJ_ERR_HIP;
            }
        }
    }
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return PSDPROJ_OK;
}

int psdproj_serve_submit(psdproj_server *s, const psdproj_request *r, uint64_t *ticket) {
    if (!s || !r || !ticket) return PSDPROJ_ERR_INVALID_ARG;
    if (r->n < 0 || r->ld < (r->n > 1 ? r->n : 1) || (r->n > 0 && !s->cfg.fake_executor && (!r->X || !r->out)))
        return PSDPROJ_ERR_INVALID_ARG;
    const int mode = choose_mode(*r);
    const size_t ws = psd::workspace_bytes_for(r->n > 0 ? r->n : 1, mode);
    if (ws == 0) return PSDPROJ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return PSDPROJ_ERR_CANCELLED;
    ++s->n_sub;
    if (ws > s->cfg.hbm_budget_bytes) {
        ++s->n_rej;
        return PSDPROJ_ERR_REJECTED;
    }
    const uint64_t tk = s->next_ticket++;
    Req &q = s->reqs[tk];
    q.r = *r;
    q.mode = mode;
    q.ws = ws;
    q.submit_ns = now_ns();
    if (!s->first_submit) s->first_submit = q.submit_ns;
    s->pending.push_back(tk);
    *ticket = tk;
    s->cv_work.notify_one();
    return PSDPROJ_OK;
}

static void fill_result(const Req &q, psdproj_result *res) {
    if (!res) return;
    res->status = q.status;
    res->mode = q.mode;
    res->tag = q.r.tag;
    res->submit_ns = q.submit_ns;
    res->start_ns = q.start_ns;
    res->end_ns = q.end_ns;
    res->slot = q.slot;
}

int psdproj_serve_wait(psdproj_server *s, uint64_t ticket, int64_t timeout_ns, psdproj_result *res) {
    if (!s) return PSDPROJ_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PSDPROJ_ERR_NOT_FOUND;
    auto done = [&] { auto j = s->reqs.find(ticket); return j == s->reqs.end() || j->second.finished; };
    if (timeout_ns < 0) {
        s->cv_done.wait(lk, done);
    } else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done)) {
        return PSDPROJ_ERR_TIMEOUT;
    }
    it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PSDPROJ_ERR_NOT_FOUND;
    fill_result(it->second, res);
    s->reqs.erase(it);
    return PSDPROJ_OK;
}

int psdproj_serve_poll(psdproj_server *s, uint64_t ticket, psdproj_result *res) {
    if (!s) return PSDPROJ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PSDPROJ_ERR_NOT_FOUND;
    if (!it->second.finished) return PSDPROJ_ERR_PENDING;
    fill_result(it->second, res);
    s->reqs.erase(it);
    return PSDPROJ_OK;
}

int psdproj_serve_cancel(psdproj_server *s, uint64_t ticket) {
    if (!s) return PSDPROJ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PSDPROJ_ERR_NOT_FOUND;
    if (it->second.finished) return PSDPROJ_OK;
    auto pit = std::find(s->pending.begin(), s->pending.end(), ticket);
    if (pit == s->pending.end()) return PSDPROJ_ERR_PENDING;  // already running
    s->pending.erase(pit);
    it->second.status = PSDPROJ_ERR_CANCELLED;
    it->second.finished = true;
    it->second.end_ns = now_ns();
    ++s->n_cancel;
    s->cv_done.notify_all();
    return PSDPROJ_OK;
}

int psdproj_serve_stats(psdproj_server *s, psdproj_serve_statistics *st) {
    if (!s || !st) return PSDPROJ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *st = psdproj_serve_statistics{};
    st->submitted = s->n_sub;
    st->completed = s->n_done;
    st->rejected = s->n_rej;
    st->cancelled = s->n_cancel;
    st->pending = s->pending.size();
    st->running = (uint64_t)s->running();
    if (!s->lat_ms.empty()) {
        std::vector<double> v = s->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const double pos = p * (double)(v.size() - 1);
            const size_t i = (size_t)pos;
            const double f = pos - (double)i;
            return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
        };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        double sum = 0.0;
        for (double x : v) sum += x;
        st->mean_ms = sum / (double)v.size();
        st->max_ms = v.back();
        const double span = (double)(s->last_end - s->first_submit) * 1e-9;
        st->throughput_per_s = span > 0.0 ? (double)s->n_done / span : 0.0;
    }
    st->bytes_held = s->held_total();
    st->peak_bytes_held = s->peak_held;
    return PSDPROJ_OK;
}

int psdproj_serve_destroy(psdproj_server *s) {
    if (!s) return PSDPROJ_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (uint64_t tk : s->pending) {
            Req &q = s->reqs[tk];
            q.status = PSDPROJ_ERR_CANCELLED;
            q.finished = true;
            ++s->n_cancel;
        }
        s->pending.clear();
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    s->th.join();  // the loop exits once running work has completed
    if (!s->cfg.fake_executor) {
        for (Slot &sl : s->slots) {
            psd::pool_release(sl.stream);
            (void)hipEventDestroy(sl.done);
            (void)hipStreamDestroy(sl.stream);
            (void)hipFree(sl.info_dev);
            (void)hipHostFree(sl.info_host);
        }
    }
    delete s;
    return PSDPROJ_OK;
}

}  // extern "C"
