// ms_server.cpp — the serving runtime of libms: sessions (batches of envs) admitted against an
// HBM budget, and continuous batching of their step requests into fused ms_step_many launches.
//
// Two threads per server, each with its own HIP stream on the server's device:
//   * the admitter admits waiting sessions in arrival order while their workspace fits in the
//     arena (a session that does not fit blocks the ones behind it, so none starves): it carves
//     the block, then builds the batch (host planning and uploads, which synchronise the
//     admission stream) outside the server lock, so admission never stalls the launches;
//   * the worker keeps up to two fused launches in flight.  Each launch takes, for every admitted
//     session, its first request that still has steps to enqueue (a session's requests run in
//     order), as many sessions as the fused work list fits in the scratch reserve, and advances
//     them by the smallest such step count in one ms_step_many call.  While the GPU runs one
//     launch the worker plans and enqueues the next; it then waits on the older launch's event
//     and completes the requests that have no steps left.
// Launches on one stream run in order, so a session's steps and its work list uploads need no
// other synchronisation.  Requests that arrive while launches run join the next launch.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [base, base + size) with coalescing of freed blocks.
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
    size_t used = 0, peak = 0;
    void init(size_t off, size_t bytes) {
        free_.clear();
        if (bytes) free_[off] = bytes;
        size = bytes;
    }
    bool alloc(size_t bytes, size_t& off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used += bytes;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Session {
    int64_t id = 0;
    // host copies of the descriptors until admission
    ms_sim_params params{};
    ms_plan plan{};
    bool has_plan = false;
    std::vector<int32_t> body_off, joint_off;
    std::vector<ms_body_desc> bodies;
    std::vector<ms_joint_desc> joints;
    std::vector<ms_compound_desc> compounds;
    size_t ws_bytes = 0, bytes = 0, off = 0;
    int32_t n_envs = 0, n_joints = 0;
    ms_batch* b = nullptr;
    float* dev_targets = nullptr;
    bool admitted = false, closing = false;
    int inflight = 0;   // launches in flight that step this session
    ms_status admit_status = MS_OK;
    std::deque<int64_t> queue;
};

struct Request {
    int64_t id = 0, session = 0;
    int32_t n_steps = 0, remaining = 0, enqueued = 0;   // steps not yet completed / already launched
    std::vector<float> targets;
    bool has_targets = false, done = false;
    ms_status status = MS_OK;
    double t_submit = 0, t_start = 0, t_done = 0;
    int32_t fused = 0;
};

}  // namespace

namespace {
// One fused launch in flight: its completion event and the steps it advances each request by.
struct Flight {
    int slot = 0;
    double t0 = 0;
    ms_status st = MS_OK;
    std::string err;
    std::vector<std::pair<int64_t, int32_t>> items;   // (request, steps)
    std::vector<int64_t> sessions;
};
}  // namespace

struct ms_server {
    int device = 0;
    hipStream_t stream = nullptr, admit_stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};   // completion of the launch in each of the two slots
    char* arena = nullptr;
    size_t arena_bytes = 0, scratch_bytes = 0;
    Arena alloc;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_admit;
    bool stop = false;
    uint64_t gen = 0;        // bumped by every client action (open, submit, close, stop) and admission
    uint64_t admit_gen = 0;  // bumped when a session queues for admission or arena space is freed
    std::deque<Flight> flights;
    int next_slot = 0;
    double last_done = 0;    // end of the busy interval so far (for the busy-time counter)
    std::thread worker, admitter;
    int64_t next_id = 1;
    std::map<int64_t, Session> sessions;   // ordered by id = arrival order
    std::deque<int64_t> admit_queue;
    std::unordered_map<int64_t, Request> reqs;
    void* pinned[2] = {nullptr, nullptr};   // host staging of drive targets, one per launch slot
    size_t pinned_cap[2] = {0, 0};
    std::string last_error;
    // counters: launches, fused batches, env-steps, requests done, sessions admitted,
    // busy microseconds (GPU time with a launch in flight), peak arena bytes, sessions rejected
    int64_t stats[8] = {};
    void run();
    void admit_loop();
};

namespace {

// The first request of a session that still has steps to launch (-1: none).
int64_t next_request(ms_server* s, const Session& ss) {
    for (int64_t r : ss.queue) {
        const Request& rq = s->reqs.at(r);
        if (rq.enqueued < rq.n_steps) return r;
    }
    return -1;
}

bool worker_has_work(ms_server* s) {
    if (!s->flights.empty()) return true;
    if (s->stop) return true;
    for (auto& kv : s->sessions) {
        const Session& ss = kv.second;
        if (ss.closing && ss.queue.empty() && ss.inflight == 0 && (ss.admitted || ss.admit_status != MS_OK)) return true;
        if (ss.admitted && next_request(s, ss) >= 0) return true;
    }
    return false;
}

void retire(ms_server* s, Session& ss) {
    if (ss.b) ms_destroy_batch(ss.b);
    ss.b = nullptr;
    s->alloc.release(ss.off, ss.bytes);
}

void fail_queue(ms_server* s, Session& ss, ms_status st) {
    for (int64_t r : ss.queue) {
        Request& rq = s->reqs.at(r);
        rq.done = true;
        rq.status = st;
        rq.t_done = now_s();
    }
    ss.queue.clear();
}

}  // namespace

// Admission thread: sessions in arrival order, each as soon as its block fits.
void ms_server::admit_loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    uint64_t seen = ~uint64_t(0);
    for (;;) {
        cv_admit.wait(lk, [&] { return (stop && admit_queue.empty()) || (!admit_queue.empty() && admit_gen != seen); });
        if (admit_queue.empty()) break;   // stopping, nothing left to admit
        seen = admit_gen;
        Session& ss = sessions.at(admit_queue.front());
        size_t off = 0;
        if (!alloc.alloc(ss.bytes, off)) continue;   // wait until a retirement frees space
        ss.off = off;
        stats[6] = int64_t(alloc.peak);
        // build the batch outside the lock (its descriptors are not touched by other threads)
        ms_scene_desc sd{ss.n_envs, ss.body_off.data(), ss.bodies.data(), ss.joint_off.data(),
                         ss.joints.empty() ? nullptr : ss.joints.data(), int32_t(ss.compounds.size()),
                         ss.compounds.empty() ? nullptr : ss.compounds.data()};
        char* base = arena + off;
        ms_batch* b = nullptr;
        lk.unlock();
        ms_status st = ms_create_batch(&ss.params, &sd, ss.has_plan ? &ss.plan : nullptr, base, ss.ws_bytes, admit_stream, &b);
        std::string err = st != MS_OK ? std::string(ms_last_error()) : std::string();
        lk.lock();
        admit_queue.pop_front();
        if (st != MS_OK) {
            alloc.release(off, ss.bytes);
            ss.admit_status = st;
            last_error = err;
            fail_queue(this, ss, st);
            stats[7] += 1;
        } else {
            ss.b = b;
            ss.dev_targets = reinterpret_cast<float*>(base + align_up(ss.ws_bytes));
            ss.admitted = true;
            stats[4] += 1;
            // the descriptors are no longer needed on the host
            std::vector<ms_body_desc>().swap(ss.bodies);
            std::vector<ms_joint_desc>().swap(ss.joints);
        }
        seen = ~uint64_t(0);
        gen += 1;
        cv_work.notify_all();
        cv_done.notify_all();
    }
}

void ms_server::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    uint64_t idle_gen = ~uint64_t(0);   // generation at which the last iteration made no progress
    for (;;) {
        cv_work.wait(lk, [&] { return !flights.empty() || (worker_has_work(this) && gen != idle_gen); });
        idle_gen = ~uint64_t(0);
        // retire closed sessions with nothing queued and nothing in flight
        bool freed = false;
        for (auto it = sessions.begin(); it != sessions.end();) {
            Session& ss = it->second;
            if (ss.closing && ss.queue.empty() && ss.inflight == 0 && (ss.admitted || ss.admit_status != MS_OK)) {
                if (ss.admitted) { retire(this, ss); freed = true; }
                it = sessions.erase(it);
            } else {
                ++it;
            }
        }
        if (freed) { admit_gen += 1; cv_admit.notify_all(); }
        cv_done.notify_all();
        if (stop && admit_queue.empty() && flights.empty()) {
            bool idle = true;
            for (auto& kv : sessions) idle = idle && kv.second.queue.empty();
            if (idle) break;
        }
        // 1. plan and enqueue a launch while fewer than two are in flight
        if (flights.size() < 2) {
            std::vector<Session*> run;
            std::vector<int64_t> rids;
            std::vector<ms_batch*> bl;
            int32_t k = INT32_MAX;
            for (auto& kv : sessions) {
                Session& ss = kv.second;
                if (!ss.admitted) continue;
                const int64_t r = next_request(this, ss);
                if (r < 0) continue;
                bl.push_back(ss.b);
                size_t need = 0;
                if (ms_query_step_many_bytes(bl.data(), int32_t(bl.size()), &need) != MS_OK || need > scratch_bytes) {
                    bl.pop_back();
                    if (bl.empty() && ss.inflight == 0 && r == ss.queue.front()) {
                        // a single session whose work list exceeds the reserve
                        Request& rq = reqs.at(r);
                        rq.done = true;
                        rq.status = MS_E_BUDGET;
                        rq.t_done = now_s();
                        ss.queue.pop_front();
                        last_error = "fused work list exceeds the scratch reserve";
                        continue;
                    }
                    break;
                }
                run.push_back(&ss);
                rids.push_back(r);
                const Request& rq = reqs.at(r);
                k = std::min(k, rq.n_steps - rq.enqueued);
            }
            if (!run.empty()) {
                Flight f;
                f.slot = next_slot;
                next_slot ^= 1;
                // targets of requests starting now go through this slot's pinned buffer into the
                // session's device buffer (the slot's previous launch has completed: at most two
                // are in flight and the other one holds the other slot)
                size_t tbytes = 0;
                for (int64_t r : rids) {
                    const Request& rq = reqs.at(r);
                    if (rq.has_targets && rq.enqueued == 0) tbytes += rq.targets.size() * 4;
                }
                std::vector<const float*> tg(run.size(), nullptr);
                bool ok = true;
                if (tbytes) {
                    void*& pin = pinned[f.slot];
                    if (pinned_cap[f.slot] < tbytes) {
                        if (pin) (void)hipHostFree(pin);
                        pin = nullptr;
                        pinned_cap[f.slot] = 0;
                        ok = hipHostMalloc(&pin, tbytes, hipHostMallocDefault) == hipSuccess;
                        if (ok) pinned_cap[f.slot] = tbytes;
                    }
                    size_t o = 0;
                    for (size_t i = 0; ok && i < run.size(); ++i) {
                        const Request& rq = reqs.at(rids[i]);
                        if (!(rq.has_targets && rq.enqueued == 0)) continue;
                        const size_t nb = rq.targets.size() * 4;
                        std::memcpy(static_cast<char*>(pin) + o, rq.targets.data(), nb);
                        ok = hipMemcpyAsync(run[i]->dev_targets, static_cast<char*>(pin) + o, nb, hipMemcpyHostToDevice,
                                            stream) == hipSuccess;
                        tg[i] = run[i]->dev_targets;
                        o += nb;
                    }
                }
                const double t0 = now_s();
                for (size_t i = 0; i < run.size(); ++i) {
                    Request& rq = reqs.at(rids[i]);
                    if (rq.t_start == 0) rq.t_start = t0;
                    rq.enqueued += k;
                    run[i]->inflight += 1;
                    f.items.emplace_back(rids[i], k);
                    f.sessions.push_back(run[i]->id);
                }
                f.t0 = t0;
                lk.unlock();
                // the fused launch (outside the lock: clients keep submitting)
                ms_status st = ok ? ms_step_many(bl.data(), tg.data(), int32_t(bl.size()), k, arena, scratch_bytes, stream)
                                  : MS_E_DEVICE;
                std::string err = st != MS_OK ? std::string(ms_last_error()) : std::string();
                if (st == MS_OK && hipEventRecord(ev[f.slot], stream) != hipSuccess) {
                    st = MS_E_DEVICE;
                    err = "event record after the fused launch failed";
                }
                // a failed launch may still have queued copies from the pinned buffer: let the
                // stream drain before that buffer is written or freed again
                if (st != MS_OK) (void)hipStreamSynchronize(stream);
                lk.lock();
                f.st = st;
                f.err = err.empty() && st != MS_OK ? "target upload failed" : err;
                stats[0] += 1;
                stats[1] += int64_t(run.size());
                flights.push_back(std::move(f));
                continue;   // plan the next launch while this one runs
            }
        }
        // 2. wait for the older launch and complete its requests
        if (!flights.empty()) {
            Flight f = std::move(flights.front());
            flights.pop_front();
            lk.unlock();
            if (f.st == MS_OK && hipEventSynchronize(ev[f.slot]) != hipSuccess) {
                f.st = MS_E_DEVICE;
                f.err = "event wait after the fused launch failed";
            }
            const double t1 = now_s();
            lk.lock();
            stats[5] += int64_t((t1 - std::max(f.t0, last_done)) * 1e6);
            last_done = t1;
            if (f.st != MS_OK) last_error = f.err;
            for (size_t i = 0; i < f.items.size(); ++i) {
                Session& ss = sessions.at(f.sessions[i]);
                Request& rq = reqs.at(f.items[i].first);
                ss.inflight -= 1;
                rq.fused = int32_t(f.items.size());
                if (f.st != MS_OK) {
                    rq.status = f.st;
                    rq.remaining = 0;
                } else {
                    rq.remaining -= f.items[i].second;
                    stats[2] += int64_t(f.items[i].second) * ss.n_envs;
                }
                if (rq.remaining == 0 && !rq.done) {
                    rq.done = true;
                    rq.t_done = t1;
                    // requests complete in their session's order: this one is at the front
                    auto qi = std::find(ss.queue.begin(), ss.queue.end(), rq.id);
                    if (qi != ss.queue.end()) ss.queue.erase(qi);
                    stats[3] += 1;
                }
            }
            cv_done.notify_all();
            continue;
        }
        idle_gen = gen;   // nothing runnable: sleep until a client changes something
    }
}

extern "C" {

double ms_server_clock(void) { return now_s(); }

ms_status ms_server_create(void* dev_arena, size_t arena_bytes, size_t scratch_bytes, ms_server** out) {
    if (!out) return fail(MS_E_INVALID_ARG, "null out");
    *out = nullptr;
    if (!dev_arena || reinterpret_cast<uintptr_t>(dev_arena) % ALIGN)
        return fail(MS_E_INVALID_ARG, "arena must be a non-null, 256-byte aligned device pointer");
    if (scratch_bytes == 0) scratch_bytes = std::max<size_t>(ALIGN, std::min<size_t>(arena_bytes / 16, size_t(16) << 20));
    scratch_bytes = align_up(scratch_bytes);
    if (arena_bytes < scratch_bytes + ALIGN) return fail(MS_E_BUDGET, "arena of %zu bytes is smaller than the scratch reserve", arena_bytes);
    std::unique_ptr<ms_server> s(new ms_server());
    HIP_OK(hipGetDevice(&s->device));
    s->arena = static_cast<char*>(dev_arena);
    s->arena_bytes = arena_bytes;
    s->scratch_bytes = scratch_bytes;
    s->alloc.init(scratch_bytes, (arena_bytes - scratch_bytes) & ~(ALIGN - 1));
    HIP_OK(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    HIP_OK(hipStreamCreateWithFlags(&s->admit_stream, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&s->ev[0], hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&s->ev[1], hipEventDisableTiming));
    ms_server* raw = s.get();
    raw->worker = std::thread([raw] { raw->run(); });
    raw->admitter = std::thread([raw] { raw->admit_loop(); });
    *out = s.release();
    return MS_OK;
}

ms_status ms_server_open(ms_server* s, const ms_sim_params* params, const ms_scene_desc* scene, const ms_plan* plan,
                         int64_t* session) {
    if (!s || !session) return fail(MS_E_INVALID_ARG, "null server or session output");
    size_t ws = 0;
    if (ms_status st = ms_query_batch_bytes(params, scene, plan, &ws); st != MS_OK) return st;
    Session ss;
    ss.params = *params;
    if (plan) { ss.plan = *plan; ss.has_plan = true; }
    ss.n_envs = scene->n_envs;
    ss.body_off.assign(scene->env_body_off, scene->env_body_off + scene->n_envs + 1);
    ss.joint_off.assign(scene->env_joint_off, scene->env_joint_off + scene->n_envs + 1);
    ss.n_joints = ss.joint_off.back();
    ss.bodies.assign(scene->bodies, scene->bodies + ss.body_off.back());
    if (ss.n_joints) ss.joints.assign(scene->joints, scene->joints + ss.n_joints);
    if (scene->n_compounds > 0) ss.compounds.assign(scene->compounds, scene->compounds + scene->n_compounds);
    ss.ws_bytes = ws;
    ss.bytes = align_up(ws) + align_up(size_t(std::max(ss.n_joints, 1)) * 4);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(MS_E_STATE, "server is shutting down");
    if (ss.bytes > s->alloc.size)
        return fail(MS_E_BUDGET, "session needs %zu bytes, the arena holds %zu", ss.bytes, s->alloc.size);
    ss.id = s->next_id++;
    *session = ss.id;
    s->admit_queue.push_back(ss.id);
    s->gen += 1;
    s->admit_gen += 1;
    s->sessions.emplace(ss.id, std::move(ss));
    s->cv_work.notify_all();
    s->cv_admit.notify_all();
    return MS_OK;
}

ms_status ms_server_submit(ms_server* s, int64_t session, int32_t n_steps, const float* host_targets, int64_t* request) {
    if (!s || !request) return fail(MS_E_INVALID_ARG, "null server or request output");
    if (n_steps < 1) return fail(MS_E_INVALID_ARG, "n_steps must be >= 1 (got %d)", n_steps);
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->sessions.find(session);
    if (it == s->sessions.end() || it->second.closing) return fail(MS_E_INVALID_ARG, "unknown or closed session %lld", (long long)session);
    Session& ss = it->second;
    if (ss.admit_status != MS_OK) return fail(ss.admit_status, "session %lld failed admission", (long long)session);
    Request rq;
    rq.id = s->next_id++;
    rq.session = session;
    rq.n_steps = rq.remaining = n_steps;
    rq.t_submit = now_s();
    if (host_targets && ss.n_joints > 0) {
        rq.targets.assign(host_targets, host_targets + ss.n_joints);
        rq.has_targets = true;
    }
    *request = rq.id;
    ss.queue.push_back(rq.id);
    s->gen += 1;
    s->reqs.emplace(rq.id, std::move(rq));
    s->cv_work.notify_all();
    return MS_OK;
}

ms_status ms_server_wait(ms_server* s, int64_t request, ms_request_info* info) {
    if (!s) return fail(MS_E_INVALID_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request);
    if (it == s->reqs.end()) return fail(MS_E_INVALID_ARG, "unknown request %lld", (long long)request);
    s->cv_done.wait(lk, [&] { return it->second.done; });
    const Request& rq = it->second;
    if (info) {
        info->request = rq.id;
        info->session = rq.session;
        info->status = rq.status;
        info->n_steps = rq.n_steps;
        info->t_submit = rq.t_submit;
        info->t_start = rq.t_start;
        info->t_done = rq.t_done;
        info->fused_batches = rq.fused;
    }
    ms_status st = rq.status;
    if (st != MS_OK) fail(st, "request %lld failed: %s", (long long)request, s->last_error.c_str());
    s->reqs.erase(it);
    return st;
}

ms_status ms_server_close(ms_server* s, int64_t session) {
    if (!s) return fail(MS_E_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->sessions.find(session);
    if (it == s->sessions.end() || it->second.closing) return fail(MS_E_INVALID_ARG, "unknown or closed session %lld", (long long)session);
    it->second.closing = true;
    s->gen += 1;
    s->cv_work.notify_all();
    return MS_OK;
}

ms_status ms_server_get_state(ms_server* s, int64_t session, const ms_state_view* dst, void* hip_stream) {
    if (!s || !dst) return fail(MS_E_INVALID_ARG, "null server or destination");
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] {
        auto it = s->sessions.find(session);
        if (it == s->sessions.end()) return true;
        const Session& ss = it->second;
        return ss.admit_status != MS_OK || (ss.admitted && ss.queue.empty() && ss.inflight == 0);
    };
    s->cv_done.wait(lk, ready);
    auto it = s->sessions.find(session);
    if (it == s->sessions.end()) return fail(MS_E_INVALID_ARG, "unknown session %lld", (long long)session);
    if (it->second.admit_status != MS_OK) return fail(it->second.admit_status, "session %lld failed admission", (long long)session);
    // the session is idle and its last launch has completed: copy on the caller's stream
    return ms_get_state(it->second.b, dst, hip_stream);
}

ms_status ms_server_drain(ms_server* s) {
    if (!s) return fail(MS_E_INVALID_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] {
        if (!s->admit_queue.empty() || !s->flights.empty()) return false;
        for (auto& kv : s->sessions)
            if (!kv.second.queue.empty() || kv.second.closing) return false;
        return true;
    });
    return MS_OK;
}

ms_status ms_server_stats(ms_server* s, int64_t* host_stats) {
    if (!s || !host_stats) return fail(MS_E_INVALID_ARG, "null server or output");
    std::lock_guard<std::mutex> lk(s->mu);
    for (int k = 0; k < 8; ++k) host_stats[k] = s->stats[k];
    host_stats[6] = int64_t(s->alloc.peak);
    return MS_OK;
}

ms_status ms_server_destroy(ms_server* s) {
    if (!s) return MS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->gen += 1;
        for (auto& kv : s->sessions) kv.second.closing = true;
        s->cv_work.notify_all();
        s->cv_admit.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    if (s->admitter.joinable()) s->admitter.join();
    for (auto& kv : s->sessions)
        if (kv.second.admitted) retire(s, kv.second);
    s->sessions.clear();
    for (int k = 0; k < 2; ++k) {
        if (s->pinned[k]) (void)hipHostFree(s->pinned[k]);
        if (s->ev[k]) (void)hipEventDestroy(s->ev[k]);
    }
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->admit_stream) (void)hipStreamDestroy(s->admit_stream);
    delete s;
    return MS_OK;
}

}  // extern "C"
