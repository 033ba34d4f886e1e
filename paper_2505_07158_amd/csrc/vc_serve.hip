// vc_serve.hip -- the serving core of libvcipher (include/vcipher.h,
// "Serving"): admission, per-stream ordering and continuous batching of
// per-frame encrypt / decrypt requests from many video streams, and a GPU
// backend that runs the batches through the cipher's calls on contexts and
// device streams of its own.
//
// The paper's monitoring system (Sec. V) encrypts every camera stream
// frame by frame in arrival order: a stream's key chain is serial (frame t+1
// starts from the iterates of frame t, Sec. II-A), frames of different
// streams are independent.  The scheduler therefore
//  - admits requests in arrival order while the device footprint of the
//    requests in flight (input, output and per-frame scratch) stays within a
//    budget (a request larger than the whole budget is admitted alone),
//  - launches a stream's frame t+1 only with or after frame t, and frames of
//    one stream in one batch in sequence order,
//  - forms a batch (one library call) from whatever has arrived, of one
//    class (the server uses the resolution, so small frames never wait for
//    the serial SHA-256 and key schedule of large ones), whenever fewer than
//    max_inflight batches of its kind and class are on the device,
//  - optionally hashes an encrypt request as soon as it arrives (the frame
//    hash does not depend on the stream's previous frame), in "hash"
//    batches that ignore stream order, and runs the ordered stage
//    (encrypt_frames_hashed) afterwards.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <iterator>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <tuple>
#include <vector>

#include "vc_internal.hpp"

namespace {

enum { KIND_ENC = 0, KIND_DEC = 1, KIND_HASH = 2 };

struct Req {
    vc_request r{};
    bool admitted = false;  // holds its footprint (from its first launch until done)
    bool hashed = false;    // encrypt request whose hash batch has completed
    double launched = NAN, done = NAN;
    int status = VC_OK;     // a failed launch's status, or VC_EORDER behind one
    std::list<std::unique_ptr<Req>>::iterator self;  // its entry in Scheduler::owned
};

struct Flight {
    int kind;
    uint64_t cls;
    int64_t handle;
    std::vector<Req *> reqs;
};

// What a batch runs on: the caller's callbacks (vc_sched) or the server's
// GPU backend (vc_server).
struct Backend {
    virtual ~Backend() = default;
    virtual int64_t launch(int kind, const std::vector<Req *> &reqs) = 0;  // handle >= 0, or a negative vc_status
    virtual int query(int64_t handle) = 0;                                // 1 done, 0 pending, < 0 error
    virtual void release(int64_t) {}
};

using Key = std::pair<int, uint32_t>;  // (request kind, stream)

class Scheduler {
public:
    explicit Scheduler(const vc_sched_config &c) : cfg(c) {
        if (cfg.max_inflight == 0) cfg.max_inflight = 1;
        if (cfg.max_inflight_hash == 0) cfg.max_inflight_hash = cfg.max_inflight;
        if (cfg.max_batch == 0) cfg.max_batch = 512;
    }

    // Batches of a kind allowed in flight per class.
    uint32_t limit(int kind) const { return kind == KIND_HASH ? cfg.max_inflight_hash : cfg.max_inflight; }

    void submit(std::unique_ptr<Req> q) {
        Req *r = q.get();
        owned.push_back(std::move(q));
        r->self = std::prev(owned.end());
        pending[cfg.hash_first && r->r.kind == KIND_ENC ? KIND_HASH : r->r.kind].push_back(r);
    }

    // Retire finished batches, then launch new ones while slots are free.
    // Returns the number of batches launched, or a negative vc_status.
    int pump(Backend &be, double now) {
        int rc = retire(be, now);
        if (rc < 0) return rc;
        int launched = 0;
        for (int kind : {KIND_ENC, KIND_DEC, KIND_HASH}) {
            drop_broken(kind, now);
            while (!pending[kind].empty()) {
                std::vector<Req *> batch = form_batch(kind);
                if (batch.empty()) break;
                for (Req *r : batch) {
                    const Key key{r->r.kind, r->r.stream};
                    if (!r->admitted) {
                        r->admitted = true;
                        r->launched = now;
                        inflight_bytes += r->r.nbytes;
                        stream_inflight[key] += 1;
                        next_admit[key] = r->r.seq + 1;
                    }
                    if (kind != KIND_HASH) next_seq[key] = r->r.seq + 1;
                }
                const int64_t h = be.launch(kind, batch);
                if (h < 0) {
                    fail(batch, now, static_cast<int>(h));
                    return static_cast<int>(h);
                }
                inflight.push_back(Flight{kind, batch[0]->r.cls, h, std::move(batch)});
                ++batches_launched;
                ++launched;
            }
        }
        return launched;
    }

    size_t poll(vc_completion *out, size_t max) {
        size_t k = 0;
        while (k < max && !completed.empty()) {
            Req *r = completed.front();
            completed.pop_front();
            out[k++] = vc_completion{r->r.tag, r->launched, r->done, r->hashed ? 1 : 0, r->status};
            forget(r);
        }
        return k;
    }

    bool idle() const {
        return inflight.empty() && pending[0].empty() && pending[1].empty() && pending[2].empty();
    }

    // Every stream starts again at frame 0 (its chain is back at the key).
    // Only when idle.
    void restart_streams() {
        next_seq.clear();
        next_admit.clear();
        stream_inflight.clear();
        broken.clear();
    }

    void stats(vc_sched_stats *s) const {
        s->inflight_batches = static_cast<uint32_t>(inflight.size());
        s->pending = static_cast<uint32_t>(pending[0].size() + pending[1].size() + pending[2].size());
        uint32_t mx = 0;
        for (const auto &kv : stream_inflight) mx = kv.second > mx ? kv.second : mx;
        s->max_stream_inflight = mx;
        s->completed_unpolled = static_cast<uint32_t>(completed.size());
        s->inflight_bytes = inflight_bytes;
        s->batches_launched = batches_launched;
    }

private:
    vc_sched_config cfg;
    std::list<std::unique_ptr<Req>> owned;
    std::deque<Req *> pending[3];
    std::vector<Flight> inflight;
    std::deque<Req *> completed;
    uint64_t inflight_bytes = 0, batches_launched = 0;
    std::map<Key, uint64_t> next_seq, next_admit;  // next frame to launch / to admit per (kind, stream)
    std::map<Key, uint32_t> stream_inflight;
    // Streams whose frame failed to launch: the library's chain did not
    // advance past it, so their later frames would fail its order check (and
    // take other streams' frames in the same batch with them); they complete
    // with VC_EORDER without launching until the streams are restarted.
    std::set<Key> broken;

    // Completes a request that will not run (or ran no further).
    void give_up(Req *r, double now, int status) {
        const Key key{r->r.kind, r->r.stream};
        if (r->admitted) {
            inflight_bytes -= r->r.nbytes;
            stream_inflight[key] -= 1;
            r->admitted = false;
        }
        r->done = now;
        r->status = status;
        completed.push_back(r);
    }

    void fail(const std::vector<Req *> &batch, double now, int status) {
        for (Req *r : batch) {
            broken.insert(Key{r->r.kind, r->r.stream});
            give_up(r, now, status);
        }
    }

    void drop_broken(int kind, double now) {
        if (broken.empty()) return;
        std::deque<Req *> keep;
        for (Req *r : pending[kind]) {
            if (broken.count(Key{r->r.kind, r->r.stream})) give_up(r, now, VC_EORDER);
            else keep.push_back(r);
        }
        pending[kind] = std::move(keep);
    }

    void forget(Req *r) { owned.erase(r->self); }

    uint32_t inflight_of(int kind, uint64_t cls) const {
        uint32_t n = 0;
        for (const Flight &f : inflight) n += (f.kind == kind && f.cls == cls) ? 1 : 0;
        return n;
    }

    int retire(Backend &be, double now) {
        std::vector<Flight> keep;
        int err = 0;
        for (Flight &f : inflight) {
            const int q = err ? 0 : be.query(f.handle);
            if (q < 0) err = q;
            if (q <= 0) {
                keep.push_back(std::move(f));
                continue;
            }
            be.release(f.handle);
            if (f.kind == KIND_HASH) {
                // on to the ordered stage; the footprint stays held
                for (Req *r : f.reqs) {
                    r->hashed = true;
                    pending[KIND_ENC].push_back(r);
                }
            } else {
                for (Req *r : f.reqs) {
                    r->done = now;
                    inflight_bytes -= r->r.nbytes;
                    stream_inflight[{r->r.kind, r->r.stream}] -= 1;
                    completed.push_back(r);
                }
            }
        }
        inflight = std::move(keep);
        return err;
    }

    // Requests to launch now, in arrival order: each the next frame of its
    // stream to admit and (except in hash batches) to launch, counting frames
    // taken earlier in this batch, within the memory budget (charged once,
    // at a request's first launch).  Passes over the queue repeat while they
    // take something, so a frame that arrived before its predecessor goes in
    // the same batch as it.
    std::vector<Req *> form_batch(int kind) {
        std::deque<Req *> &q = pending[kind];
        std::vector<Req *> batch;
        uint64_t cls = 0;
        std::map<Key, uint64_t> expect;
        std::map<Key, uint32_t> admitted_now;
        uint64_t budget = cfg.hbm_budget > inflight_bytes ? cfg.hbm_budget - inflight_bytes : 0;
        bool full = false, progress = true;
        std::deque<Req *> rest(q.begin(), q.end());
        const bool ordered = kind != KIND_HASH;  // a hash may run beside its predecessor's later stage
        while (progress && !full) {
            progress = false;
            std::deque<Req *> left;
            for (Req *r : rest) {
                const Key key{r->r.kind, r->r.stream};
                auto ex = expect.find(key);
                const uint64_t want = ex != expect.end() ? ex->second : next_seq[key];
                const uint32_t taken = admitted_now.count(key) ? admitted_now[key] : 0;
                const bool blocked =
                    full || (ordered && r->r.seq != want) || (!batch.empty() && r->r.cls != cls) ||
                    (!r->admitted && r->r.seq != next_admit[key] + taken) ||
                    (batch.empty() && inflight_of(kind, r->r.cls) >= limit(kind)) ||
                    (!r->admitted && cfg.max_stream_inflight &&
                     stream_inflight[key] + taken >= cfg.max_stream_inflight);
                if (blocked) {
                    left.push_back(r);
                    continue;
                }
                if (!r->admitted) {
                    const bool alone = batch.empty() && inflight_bytes == 0;
                    if (r->r.nbytes > budget && !alone) {
                        full = true;  // admission stops at the first request that does not fit
                        left.push_back(r);
                        continue;
                    }
                    budget = r->r.nbytes > budget ? 0 : budget - r->r.nbytes;
                    admitted_now[key] = taken + 1;
                }
                batch.push_back(r);
                cls = r->r.cls;
                if (ordered) expect[key] = want + 1;
                progress = true;
                if (batch.size() >= cfg.max_batch) full = true;
            }
            rest = std::move(left);
        }
        q = std::move(rest);
        return batch;
    }
};

// The caller's callbacks as a backend.
struct CallbackBackend : Backend {
    vc_launch_fn launch_fn;
    vc_query_fn query_fn;
    void *user;
    CallbackBackend(vc_launch_fn l, vc_query_fn q, void *u) : launch_fn(l), query_fn(q), user(u) {}
    int64_t launch(int kind, const std::vector<Req *> &reqs) override {
        std::vector<uint64_t> tags(reqs.size());
        for (size_t i = 0; i < reqs.size(); ++i) tags[i] = reqs[i]->r.tag;
        return launch_fn(user, kind, tags.size(), tags.data());
    }
    int query(int64_t h) override { return query_fn(user, h); }
};

// The server's GPU backend: per class (resolution) a sender and a receiver
// context (each stream's chain lives in one context), per (kind, class)
// max_inflight device streams used in rotation, and a completion event per
// batch in flight.
struct GpuBackend : Backend {
    int device = 0;
    uint32_t nclasses = 0;
    std::vector<std::pair<uint32_t, uint32_t>> classes;  // (w, h)
    std::vector<vc_cipher *> ctx;                        // [class][enc, dec]
    std::vector<hipStream_t> streams;                    // [class][enc slots, dec slots, hash slots]
    std::vector<uint32_t> turn;                          // [class][enc, dec, hash]
    uint32_t slots[3] = {1, 1, 1};                       // device streams per kind and class

    uint32_t per_class() const { return slots[0] + slots[1] + slots[2]; }
    std::vector<hipEvent_t> events;
    std::vector<int64_t> free_events;

    ~GpuBackend() override {
        (void)hipDeviceSynchronize();
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipStream_t s : streams)
            if (s) (void)hipStreamDestroy(s);
        for (vc_cipher *c : ctx) cipher_destroy(c);
    }

    int64_t launch(int kind, const std::vector<Req *> &reqs) override {
        const uint32_t ci = static_cast<uint32_t>(reqs[0]->r.cls);
        const size_t n = reqs.size();
        std::vector<const uint8_t *> frames(n);
        std::vector<uint8_t *> outs(n), hashes(n);
        std::vector<vc_shape> shapes(n);
        for (size_t i = 0; i < n; ++i) {
            const vc_request &r = reqs[i]->r;
            frames[i] = r.frame;
            outs[i] = r.out;
            hashes[i] = r.hash;
            shapes[i] = vc_shape{r.w, r.h, 3, r.stream, r.seq};
        }
        uint32_t &t = turn[3 * ci + kind];
        uint32_t first = ci * per_class();
        for (int k = 0; k < kind; ++k) first += slots[k];
        const hipStream_t st = streams[first + t];
        t = (t + 1) % slots[kind];
        vc_cipher *c = ctx[2 * ci + (kind == KIND_DEC ? 1 : 0)];
        const vc::CallKind ck = kind == KIND_HASH   ? vc::CallKind::Hash
                                : kind == KIND_DEC  ? vc::CallKind::Decrypt
                                : reqs[0]->hashed   ? vc::CallKind::EncryptHashed
                                                    : vc::CallKind::Encrypt;
        const int rc = vc::call_frames(c, ck, n, frames.data(), shapes.data(), hashes.data(), outs.data(), st);
        if (rc) return rc;
        if (free_events.empty()) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return VC_EDEVICE;
            events.push_back(e);
            free_events.push_back(static_cast<int64_t>(events.size() - 1));
        }
        const int64_t h = free_events.back();
        free_events.pop_back();
        if (hipEventRecord(events[h], st) != hipSuccess) return VC_EDEVICE;
        return h;
    }

    int query(int64_t h) override {
        const hipError_t e = hipEventQuery(events[h]);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        return VC_EDEVICE;
    }

    void release(int64_t h) override { free_events.push_back(h); }
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct vc_sched {
    Scheduler core;
    explicit vc_sched(const vc_sched_config &c) : core(c) {}
};

struct vc_server {
    Scheduler core;
    GpuBackend be;
    vc_key key{};
    uint32_t max_streams = 0;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::mutex mu;
    explicit vc_server(const vc_sched_config &c) : core(c) {}
};

extern "C" {

int vc_sched_create(const vc_sched_config *cfg, vc_sched **out) {
    if (out) *out = nullptr;
    if (!cfg || !out) return VC_EINVAL;
    vc_sched *s = new (std::nothrow) vc_sched(*cfg);
    if (!s) return VC_ENOMEM;
    *out = s;
    return VC_OK;
}

int vc_sched_submit(vc_sched *s, const vc_request *req) {
    if (!s || !req || (req->kind != KIND_ENC && req->kind != KIND_DEC)) return VC_EINVAL;
    std::unique_ptr<Req> r(new (std::nothrow) Req());
    if (!r) return VC_ENOMEM;
    r->r = *req;
    s->core.submit(std::move(r));
    return VC_OK;
}

int vc_sched_pump(vc_sched *s, double now, vc_launch_fn launch, vc_query_fn query, void *user) {
    if (!s || !launch || !query) return VC_EINVAL;
    CallbackBackend be(launch, query, user);
    return s->core.pump(be, now);
}

size_t vc_sched_poll(vc_sched *s, vc_completion *out, size_t max) {
    if (!s || !out) return 0;
    return s->core.poll(out, max);
}

int vc_sched_get_stats(const vc_sched *s, vc_sched_stats *st) {
    if (!s || !st) return VC_EINVAL;
    s->core.stats(st);
    return VC_OK;
}

int vc_sched_idle(const vc_sched *s) { return s && s->core.idle() ? 1 : 0; }

void vc_sched_destroy(vc_sched *s) { delete s; }

int vc_server_create(const vc_key *key, const uint32_t *classes, size_t nclasses, const vc_server_config *cfg,
                     vc_server **out) {
    if (out) *out = nullptr;
    if (!key || !classes || nclasses == 0 || nclasses > 64 || !cfg || !out || cfg->max_streams == 0)
        return VC_EINVAL;
    vc_server *srv = new (std::nothrow) vc_server(cfg->sched);
    if (!srv) return VC_ENOMEM;
    srv->key = *key;
    srv->max_streams = cfg->max_streams;
    GpuBackend &be = srv->be;
    if (hipGetDevice(&be.device) != hipSuccess) {
        delete srv;
        return VC_EDEVICE;
    }
    be.nclasses = static_cast<uint32_t>(nclasses);
    be.slots[KIND_ENC] = be.slots[KIND_DEC] = cfg->sched.max_inflight ? cfg->sched.max_inflight : 1;
    be.slots[KIND_HASH] = !cfg->sched.hash_first       ? 0  // no hash batches
                          : cfg->sched.max_inflight_hash ? cfg->sched.max_inflight_hash
                                                         : be.slots[KIND_ENC];
    const uint64_t scratch = cfg->scratch_bytes ? cfg->scratch_bytes
                                                : std::max<uint64_t>(cfg->sched.hbm_budget / nclasses, uint64_t(1) << 30);
    int rc = VC_OK;
    for (size_t c = 0; c < nclasses && rc == VC_OK; ++c) {
        be.classes.push_back({classes[2 * c], classes[2 * c + 1]});
        for (int k = 0; k < 2 && rc == VC_OK; ++k) {
            vc_cipher *cx = nullptr;
            rc = cipher_init(key, cfg->max_streams, scratch, &cx);
            if (rc == VC_OK) {
                be.ctx.push_back(cx);
                if (cfg->parts) rc = vc_set_overlap(cx, cfg->parts, cfg->side_streams, cfg->scratch_slots ? cfg->scratch_slots : 2);
            }
        }
        for (uint32_t k = 0; k < be.per_class() && rc == VC_OK; ++k) {
            hipStream_t st = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) rc = VC_EDEVICE;
            else be.streams.push_back(st);
        }
        for (int k = 0; k < 3; ++k) be.turn.push_back(0);
    }
    if (rc != VC_OK) {
        delete srv;
        return rc;
    }
    *out = srv;
    return VC_OK;
}

double vc_server_clock(const vc_server *srv) { return srv ? seconds_since(srv->t0) : 0.0; }

}  // extern "C"

namespace {

// The class (index of the resolution) of a request the server can take, or
// nclasses when it cannot: a kind other than encrypt / decrypt, a NULL
// buffer, a stream out of range, a hash buffer the device cannot reach or a
// shape that is not one of the classes.
uint32_t request_class(const vc_server *srv, const vc_request *req) {
    const uint32_t none = srv->be.nclasses;
    if ((req->kind != KIND_ENC && req->kind != KIND_DEC) || !req->frame || !req->out || !req->hash ||
        req->stream >= srv->max_streams || !vc::reachable(req->hash, 32))
        return none;
    for (uint32_t c = 0; c < srv->be.nclasses; ++c)
        if (srv->be.classes[c].first == req->w && srv->be.classes[c].second == req->h) return c;
    return none;
}

}  // namespace

extern "C" {

int vc_server_submit(vc_server *srv, const vc_request *req) {
    if (!srv || !req) return VC_EINVAL;
    const uint32_t ci = request_class(srv, req);
    if (ci == srv->be.nclasses) return VC_EINVAL;
    std::unique_ptr<Req> r(new (std::nothrow) Req());
    if (!r) return VC_ENOMEM;
    r->r = *req;
    r->r.cls = ci;
    if (!r->r.nbytes) r->r.nbytes = 6ull * req->w * req->h + vc_scratch_per_frame(req->w, req->h, srv->key.n);
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->core.submit(std::move(r));
    return VC_OK;
}

int vc_server_pump(vc_server *srv) {
    if (!srv) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    return srv->core.pump(srv->be, seconds_since(srv->t0));
}

size_t vc_server_poll(vc_server *srv, vc_completion *out, size_t max) {
    if (!srv || !out) return 0;
    std::lock_guard<std::mutex> lk(srv->mu);
    return srv->core.poll(out, max);
}

int vc_server_idle(vc_server *srv) {
    if (!srv) return 1;
    std::lock_guard<std::mutex> lk(srv->mu);
    return srv->core.idle() ? 1 : 0;
}

int vc_server_get_stats(vc_server *srv, vc_sched_stats *st) {
    if (!srv || !st) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->core.stats(st);
    return VC_OK;
}

int vc_server_run_trace(vc_server *srv, size_t count, const vc_request *reqs, vc_completion *done) {
    if (!srv || (count && (!reqs || !done))) return VC_EINVAL;
    // the whole trace is checked before anything is submitted
    for (size_t i = 0; i < count; ++i)
        if ((i && reqs[i].arrival < reqs[i - 1].arrival) || request_class(srv, &reqs[i]) == srv->be.nclasses)
            return VC_EINVAL;
    {
        // completions are matched to reqs by index: nothing else may be
        // pending, in flight or unpolled
        std::lock_guard<std::mutex> lk(srv->mu);
        vc_sched_stats st{};
        srv->core.stats(&st);
        if (!srv->core.idle() || st.completed_unpolled) return VC_EBUSY;
    }
    // completions are reported in the order of reqs: the internal tag is the index
    const double base = vc_server_clock(srv);
    size_t next = 0, finished = 0;
    std::vector<vc_completion> buf(256);
    while (finished < count) {
        const double now = vc_server_clock(srv) - base;
        size_t submitted = 0;
        while (next < count && reqs[next].arrival <= now) {
            vc_request r = reqs[next];
            r.tag = next;
            r.arrival = base + reqs[next].arrival;
            const int rc = vc_server_submit(srv, &r);
            if (rc) return rc;
            ++next;
            ++submitted;
        }
        const int launched = vc_server_pump(srv);
        if (launched < 0) return launched;
        size_t got;
        size_t polled = 0;
        while ((got = vc_server_poll(srv, buf.data(), buf.size())) > 0) {
            for (size_t k = 0; k < got; ++k) {
                vc_completion c = buf[k];
                const size_t i = static_cast<size_t>(c.tag);
                c.tag = reqs[i].tag;
                c.launched -= base;
                c.done -= base;
                done[i] = c;
            }
            finished += got;
            polled += got;
        }
        if (!launched && !submitted && !polled) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    return VC_OK;
}

int vc_server_reset(vc_server *srv) {
    if (!srv) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (!srv->core.idle()) return VC_EBUSY;
    if (hipDeviceSynchronize() != hipSuccess) return VC_EDEVICE;
    for (vc_cipher *c : srv->be.ctx)
        for (uint32_t s = 0; s < srv->max_streams; ++s) {
            const int rc = cipher_stream_reset(c, s);
            if (rc) return rc;
        }
    srv->core.restart_streams();
    return VC_OK;
}

int vc_server_status(vc_server *srv) {
    if (!srv) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    int worst = VC_OK;
    for (vc_cipher *c : srv->be.ctx) {
        const int rc = cipher_status(c, nullptr);
        if (rc) worst = rc;
    }
    return worst;
}

void vc_server_destroy(vc_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
    }
    delete srv;
}

}  // extern "C"
