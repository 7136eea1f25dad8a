// ms_server.cpp — the serving runtime of libms: sessions (batches of envs) admitted against an
// HBM budget, and continuous batching of their step requests into fused ms_step_many launches.
//
// One worker thread per server owns a HIP stream on the server's device.  Each iteration it
//   1. admits waiting sessions in arrival order while their workspace fits in the arena (a
//      session that does not fit blocks the ones behind it, so none starves);
//   2. takes the head request of every admitted session (a session's requests run in order),
//      as many as the fused work list fits in the scratch reserve;
//   3. advances all of them by the smallest remaining step count in one ms_step_many call,
//      waits for it, and completes the requests that have no steps left.
// Requests that arrive while a launch runs join the next iteration.
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
    size_t ws_bytes = 0, bytes = 0, off = 0;
    int32_t n_envs = 0, n_joints = 0;
    ms_batch* b = nullptr;
    float* dev_targets = nullptr;
    bool admitted = false, closing = false, busy = false;
    ms_status admit_status = MS_OK;
    std::deque<int64_t> queue;
};

struct Request {
    int64_t id = 0, session = 0;
    int32_t n_steps = 0, remaining = 0;
    std::vector<float> targets;
    bool has_targets = false, done = false;
    ms_status status = MS_OK;
    double t_submit = 0, t_start = 0, t_done = 0;
    int32_t fused = 0;
};

}  // namespace

struct ms_server {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    char* arena = nullptr;
    size_t arena_bytes = 0, scratch_bytes = 0;
    Arena alloc;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    bool in_flight = false;
    uint64_t gen = 0;   // bumped by every client action (open, submit, close, stop)
    std::thread worker;
    int64_t next_id = 1;
    std::map<int64_t, Session> sessions;   // ordered by id = arrival order
    std::deque<int64_t> admit_queue;
    std::unordered_map<int64_t, Request> reqs;
    void* pinned = nullptr;
    size_t pinned_cap = 0;
    std::string last_error;
    // counters: launches, fused batches, env-steps, requests done, sessions admitted,
    // busy microseconds, peak arena bytes, sessions rejected
    int64_t stats[8] = {};
    void run();
};

namespace {

bool has_work(ms_server* s) {
    if (s->stop) return true;
    if (!s->admit_queue.empty()) return true;
    for (auto& kv : s->sessions) {
        const Session& ss = kv.second;
        if (ss.admitted && (!ss.queue.empty() || ss.closing)) return true;
    }
    return false;
}

// Admission of one session (worker thread, lock held): carve its block, create its batch.
ms_status admit(ms_server* s, Session& ss, bool& fits) {
    fits = s->alloc.alloc(ss.bytes, ss.off);
    if (!fits) return MS_OK;
    ms_scene_desc sd{ss.n_envs, ss.body_off.data(), ss.bodies.data(), ss.joint_off.data(),
                     ss.joints.empty() ? nullptr : ss.joints.data()};
    char* base = s->arena + ss.off;
    ms_status st = ms_create_batch(&ss.params, &sd, ss.has_plan ? &ss.plan : nullptr, base, ss.ws_bytes, s->stream, &ss.b);
    if (st != MS_OK) {
        s->alloc.release(ss.off, ss.bytes);
        return st;
    }
    ss.dev_targets = reinterpret_cast<float*>(base + align_up(ss.ws_bytes));
    ss.admitted = true;
    s->stats[4] += 1;
    s->stats[6] = int64_t(s->alloc.peak);
    // the descriptors are no longer needed on the host
    std::vector<ms_body_desc>().swap(ss.bodies);
    std::vector<ms_joint_desc>().swap(ss.joints);
    return MS_OK;
}

void retire(ms_server* s, Session& ss) {
    if (ss.b) ms_destroy_batch(ss.b);
    ss.b = nullptr;
    s->alloc.release(ss.off, ss.bytes);
}

}  // namespace

void ms_server::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    uint64_t idle_gen = ~uint64_t(0);   // generation at which the last iteration made no progress
    for (;;) {
        cv_work.wait(lk, [&] { return has_work(this) && gen != idle_gen; });
        idle_gen = ~uint64_t(0);
        bool progressed = false;
        // 1. admission in arrival order
        while (!admit_queue.empty()) {
            Session& ss = sessions.at(admit_queue.front());
            bool fits = false;
            ms_status st = admit(this, ss, fits);
            if (st != MS_OK) {
                ss.admit_status = st;
                last_error = ms_last_error();
                for (int64_t r : ss.queue) {
                    Request& rq = reqs.at(r);
                    rq.done = true;
                    rq.status = st;
                    rq.t_done = now_s();
                }
                ss.queue.clear();
                admit_queue.pop_front();
                stats[7] += 1;
                progressed = true;
                continue;
            }
            if (!fits) break;
            admit_queue.pop_front();
            progressed = true;
        }
        // retire closed sessions with nothing left to run
        for (auto it = sessions.begin(); it != sessions.end();) {
            Session& ss = it->second;
            bool gone = ss.closing && ss.queue.empty() && (ss.admitted || ss.admit_status != MS_OK);
            if (gone) {
                if (ss.admitted) retire(this, ss);
                it = sessions.erase(it);
                progressed = true;
            } else {
                ++it;
            }
        }
        cv_done.notify_all();
        if (stop && admit_queue.empty()) {
            bool idle = true;
            for (auto& kv : sessions) idle = idle && kv.second.queue.empty();
            if (idle) break;
        }
        // 2. one head request per admitted session, while the fused work list fits
        std::vector<Session*> run;
        std::vector<ms_batch*> bl;
        int32_t k = INT32_MAX;
        for (auto& kv : sessions) {
            Session& ss = kv.second;
            if (!ss.admitted || ss.queue.empty()) continue;
            bl.push_back(ss.b);
            size_t need = 0;
            if (ms_query_step_many_bytes(bl.data(), int32_t(bl.size()), &need) != MS_OK || need > scratch_bytes) {
                bl.pop_back();
                if (bl.empty()) {   // a single session whose work list exceeds the reserve
                    Request& rq = reqs.at(ss.queue.front());
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
            Request& rq = reqs.at(ss.queue.front());
            if (rq.t_start == 0) rq.t_start = now_s();
            k = std::min(k, rq.remaining);
        }
        if (run.empty()) {   // nothing runnable: sleep until a client changes something
            if (!progressed) idle_gen = gen;
            continue;
        }
        // targets of requests starting now go through pinned memory into the session's buffer
        size_t tbytes = 0;
        for (Session* ss : run) {
            Request& rq = reqs.at(ss->queue.front());
            if (rq.has_targets && rq.remaining == rq.n_steps) tbytes += rq.targets.size() * 4;
        }
        std::vector<const float*> tg(run.size(), nullptr);
        bool ok = true;
        if (tbytes) {
            if (pinned_cap < tbytes) {
                if (pinned) (void)hipHostFree(pinned);
                pinned = nullptr;
                pinned_cap = 0;
                ok = hipHostMalloc(&pinned, tbytes, hipHostMallocDefault) == hipSuccess;
                if (ok) pinned_cap = tbytes;
            }
            size_t o = 0;
            for (size_t i = 0; ok && i < run.size(); ++i) {
                Request& rq = reqs.at(run[i]->queue.front());
                if (!(rq.has_targets && rq.remaining == rq.n_steps)) continue;
                const size_t nb = rq.targets.size() * 4;
                std::memcpy(static_cast<char*>(pinned) + o, rq.targets.data(), nb);
                ok = hipMemcpyAsync(run[i]->dev_targets, static_cast<char*>(pinned) + o, nb, hipMemcpyHostToDevice,
                                    stream) == hipSuccess;
                tg[i] = run[i]->dev_targets;
                o += nb;
            }
        }
        for (Session* ss : run) ss->busy = true;
        in_flight = true;
        lk.unlock();
        // 3. the fused launch (outside the lock: clients keep submitting)
        const double t0 = now_s();
        ms_status st = ok ? ms_step_many(bl.data(), tg.data(), int32_t(bl.size()), k, arena, scratch_bytes, stream)
                          : MS_E_DEVICE;
        std::string err = st != MS_OK ? std::string(ms_last_error()) : std::string();
        // a failed launch may still have queued the target copies from the pinned buffer: let
        // the stream drain before that buffer is written or freed again
        if (st != MS_OK) (void)hipStreamSynchronize(stream);
        if (st == MS_OK && (hipEventRecord(ev, stream) != hipSuccess || hipEventSynchronize(ev) != hipSuccess)) {
            st = MS_E_DEVICE;
            err = "event wait after the fused launch failed";
        }
        const double t1 = now_s();
        lk.lock();
        in_flight = false;
        if (st != MS_OK) last_error = err.empty() ? "target upload failed" : err;
        stats[0] += 1;
        stats[1] += int64_t(run.size());
        stats[5] += int64_t((t1 - t0) * 1e6);
        for (Session* ss : run) {
            ss->busy = false;
            Request& rq = reqs.at(ss->queue.front());
            rq.fused = int32_t(run.size());
            if (st != MS_OK) {
                rq.status = st;
                rq.remaining = 0;
            } else {
                rq.remaining -= k;
                stats[2] += int64_t(k) * ss->n_envs;
            }
            if (rq.remaining == 0) {
                rq.done = true;
                rq.t_done = t1;
                ss->queue.pop_front();
                stats[3] += 1;
            }
        }
        cv_done.notify_all();
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
    HIP_OK(hipEventCreateWithFlags(&s->ev, hipEventDisableTiming));
    ms_server* raw = s.get();
    raw->worker = std::thread([raw] { raw->run(); });
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
    s->sessions.emplace(ss.id, std::move(ss));
    s->cv_work.notify_all();
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
        return ss.admit_status != MS_OK || (ss.admitted && ss.queue.empty() && !ss.busy);
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
        if (!s->admit_queue.empty() || s->in_flight) return false;
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
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->sessions)
        if (kv.second.admitted) retire(s, kv.second);
    s->sessions.clear();
    if (s->pinned) (void)hipHostFree(s->pinned);
    if (s->ev) (void)hipEventDestroy(s->ev);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return MS_OK;
}

}  // extern "C"
