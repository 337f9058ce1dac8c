// Serving: continuous batching of frames from many camera streams.
//
// The paper measures the latency of one frame from input image to detected
// lines (Sec. 5); a deployment feeds many cameras at once.  The server keeps
// every admitted stream's state resident in device memory (frame slot, edge
// map, edge list, accumulator, peak buffers, and for the pruned path the
// proposal logits and tile mask) and runs a few refill lanes, each a worker
// thread with its own batch plan over all slots, its own graphs and its own
// compute stream:
//
//   wait for requests -> take the oldest request of every stream not in a
//   running refill (one per stream) -> write the lane's per-slot flags ->
//   the set-up kernel (counters, queue, split accumulators) -> copy those
//   frames into their slots (or wait for their copies ahead) -> one graph
//   launch over all slots (proposal network and mask per size class when
//   pruned, then Sobel, vote, peaks; switched-off slots return at once;
//   the peak search writes each slot's peaks straight into page-locked
//   host memory) -> complete the requests.
//
// A slot belongs to one refill at a time, so the lanes never share a frame's
// buffers, and a stream's requests run in order.  Most kernels of a
// one-frame refill leave much of the GPU idle (the Sobel pass, key pass and
// peak search of one frame, the vote's last round of workgroups), so a
// request that arrives while another stream's refill runs starts beside it
// on a second lane rather than queueing behind it.  Streams with the same
// configuration form a class whose frame slots are contiguous, so the
// network runs over a class as one batch.  Admission: streams are taken in
// order while their device state fits the HBM budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string.h>
#include <thread>
#include <tuple>
#include <vector>

#include "lane_entry.h"

namespace {

// a pruned server with at most this many classes keeps one graph per
// non-empty subset of classes (2^n - 1 graphs)
constexpr int kSubsetClasses = 4;

int serve_lanes(const lane_server_cfg& cfg) { return cfg.lanes > 0 ? cfg.lanes : 2; }

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

int check_stream(const lane_stream_cfg& c, int pruned) {
    if (c.W < 1 || c.H < 1 || c.n_theta < 1 || c.k < 1 || c.threshold < 0 || c.threshold > 255)
        return LANE_E_ARG;
    if (c.W > LANE_MAX_DIM || c.H > LANE_MAX_DIM || c.n_theta > 8192) return LANE_E_SIZE;
    if (c.k > LANE_SERVE_MAX_K) return LANE_E_ARG;
    if (c.border_mode != LANE_BORDER_ZERO && c.border_mode != LANE_BORDER_ZERO_MASKRING)
        return LANE_E_UNSUPPORTED;
    if (pruned && (c.n_theta % 4) != 0) return LANE_E_UNSUPPORTED;
    return LANE_OK;
}

int check_cfg(const lane_server_cfg& c) {
    if (c.max_pending < 1) return LANE_E_ARG;
    if (c.vote_rows < 0 || (c.vote_rows & (c.vote_rows - 1)) != 0) return LANE_E_ARG;
    if (c.sobel_strip_rows < 0 || (c.sobel_strip_rows % 8) != 0) return LANE_E_ARG;
    if (c.vote_split < 0 || c.vote_split > 64) return LANE_E_ARG;
    if (c.pruned && (!c.cnn_params || !(c.conf > 0.5f && c.conf < 1.f))) return LANE_E_ARG;
    if (c.deadline_ns < 0) return LANE_E_ARG;
    if (c.lanes < 0 || c.lanes > LANE_SERVE_MAX_LANES) return LANE_E_ARG;
    if (c.spin_us < 0 || c.spin_us > 10000000) return LANE_E_ARG;
    return LANE_OK;
}

using ClassKey = std::tuple<int, int, int, int, int, int>;
ClassKey key_of(const lane_stream_cfg& c) {
    return ClassKey(c.W, c.H, c.n_theta, c.k, c.threshold, c.border_mode);
}

// Device bytes of one stream's buffers (the fused proposal network needs no
// activation workspace).
struct StreamSizes {
    size_t img, edges, list, acc, peaks_ws, counters, mask, logits, split;
    size_t total() const {
        return img + edges + list + acc + peaks_ws + counters + mask + logits + split;
    }
};

// The latency shape: 4 theta rows per workgroup and an 8-way edge split (a
// one-frame 4K vote in 170 us against 455 us for one row per workgroup,
// where 360 workgroups each read the whole edge list).
int serve_vote_rows(const lane_server_cfg& cfg) { return cfg.vote_rows > 0 ? cfg.vote_rows : 4; }
int serve_vote_split(const lane_server_cfg& cfg) { return cfg.vote_split > 0 ? cfg.vote_split : 8; }

// device bytes the lanes' plans hold for a stream's edge split: the parts
// add into the frame's accumulator, but a masked frame (pruned path) votes
// from a pruned copy of its edge list, which each plan allocates per frame
size_t split_bytes(const lane_stream_cfg& c, const lane_server_cfg& cfg) {
    if (!cfg.pruned || serve_vote_split(cfg) <= 1) return 0;
    size_t lb = 0;
    lane_edge_list_size(c.W, c.H, &lb);
    return al256(lb) * (size_t)serve_lanes(cfg);
}

StreamSizes stream_sizes(const lane_stream_cfg& c, const lane_server_cfg& cfg) {
    const int pruned = cfg.pruned;
    StreamSizes z;
    const int pitch = (c.W + 15) / 16 * 16;
    int32_t D = 0;
    lane_r_offset(c.W, c.H, &D);
    const size_t n_r = 2 * (size_t)D + 1;
    const size_t th = (c.H + 7) / 8, tw = (c.W + 7) / 8;
    z.img = al256((size_t)pitch * c.H);
    z.edges = al256((size_t)c.W * c.H);
    size_t lb = 0;
    lane_edge_list_size(c.W, c.H, &lb);
    z.list = al256(lb);
    z.acc = al256(sizeof(int32_t) * (size_t)c.n_theta * n_r);
    size_t ws = 0;
    lane_hough_peaks_workspace_size(c.n_theta, (int32_t)n_r, &ws);
    z.peaks_ws = al256(ws);
    z.counters = 256;
    z.mask = pruned ? al256(th * tw) : 0;
    z.logits = pruned ? al256(sizeof(float) * 9 * th * tw) : 0;
    z.split = split_bytes(c, cfg);
    return z;
}


// Admission in stream order; returns the device bytes of everything the
// server allocates for the admitted streams (tables and weights included).
size_t plan_admission(const lane_stream_cfg* s, int n, const lane_server_cfg& cfg,
                      uint8_t* admitted, size_t* stream_bytes) {
    std::map<ClassKey, int> count;
    std::map<int, int> thetas;
    size_t shared = 0;
    if (cfg.pruned) {
        size_t pk = 0;
        lane_cnn_sizes(16, 16, 1, &pk, nullptr, nullptr);
        shared += al256(pk) + al256(sizeof(float) * LANE_CNN_PARAMS);
    }
    size_t total = shared;
    for (int i = 0; i < n; ++i) {
        const StreamSizes z = stream_sizes(s[i], cfg);
        const ClassKey k = key_of(s[i]);
        const int c = count.count(k) ? count[k] : 0;
        size_t add = z.total();
        if (!thetas.count(s[i].n_theta)) add += al256(sizeof(int16_t) * 2 * (size_t)s[i].n_theta);
        if (stream_bytes) stream_bytes[i] = add;
        const bool ok = total + add <= cfg.hbm_budget;
        if (admitted) admitted[i] = ok ? 1 : 0;
        if (ok) {
            total += add;
            count[k] = c + 1;
            thetas[s[i].n_theta] = 1;
        }
    }
    return total;
}

struct Req {
    int stream;
    int pitch;
    const uint8_t* frame;
    uint64_t frame_id;
    int64_t t_submit;
    int64_t tag;    // >= 0: index in the running replay
    uint64_t id;    // unique per request (copy-ahead bookkeeping)
    bool ahead;     // (taken into a refill) its frame was copied ahead
    bool after_up;  // (taken) a copy ahead went to its slot: order after it
};

}  // namespace

struct lane_server {
    lane_server_cfg cfg;
    int dev = 0;
    std::vector<lane_stream_cfg> streams;  // admitted, in slot order
    std::vector<int> slot_of;              // caller's stream index -> slot (-1: not admitted)
    std::vector<int> stream_of;            // slot -> caller's stream index
    struct Class {
        lane_stream_cfg cfg;
        int first_slot, n;
        int pitch;
        uint8_t* img;
        uint8_t* mask;
        float* logits;
    };
    std::vector<Class> classes;
    std::vector<int> class_of;             // slot -> class
    std::vector<uint8_t*> slot_img;
    void* dmem = nullptr;
    size_t dbytes = 0;
    // page-locked, per slot (3k+1) at h_peak_off[slot]: the plan's peak
    // outputs (the peak search stores into it through its device address,
    // so no copy follows the refill)
    int32_t* h_peaks = nullptr;
    std::vector<size_t> h_peak_off;
    // a refill lane: its worker runs refills on its own stream with its own
    // plan (flags, work lists, queues) and graphs; h_flags: one per slot
    struct Lane {
        lane_batch* plan = nullptr;
        uint8_t* h_flags = nullptr;
        uint8_t* d_flags = nullptr;        // the plan's flags
        hipStream_t stream = nullptr;
        // graphs[m]: the refill whose active slots lie in the classes of bit
        // mask m (pruned, up to kSubsetClasses classes: only those classes
        // run their network and masks); otherwise graphs[0] serves every refill
        std::vector<hipGraph_t> graphs;
        std::vector<hipGraphExec_t> execs;
        std::thread worker;
    };
    std::vector<Lane> lanes;
    // copy-ahead: the frame of the request at the head of an idle slot's
    // queue is copied to the slot on its own stream as soon as it is
    // known, so the copy overlaps the refill running meanwhile; up_id[slot]
    // = the request whose copy up_ev[slot] marks (0: none); busy[slot]: 1
    // the slot is in a running refill (its buffers still in use), 2 a copy
    // ahead into it is being issued
    hipStream_t up_stream = nullptr;
    std::vector<hipEvent_t> up_ev;
    std::vector<uint64_t> up_id;
    std::vector<uint8_t> busy;
    uint64_t next_id = 1;
    bool per_subset = false;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    // bumped (under mu) whenever a lane may find new work: a submission, a
    // refill's slots freed, resume, stop; an idle lane that polls
    // (cfg.spin_us) watches it instead of sleeping on cv_work
    std::atomic<uint64_t> work_gen{0};
    std::vector<std::deque<Req>> pending;
    std::deque<lane_result> done;
    lane_result* replay_out = nullptr;
    int64_t replay_left = 0;
    bool stop = false;
    bool paused = false;
    int error = LANE_OK;
    lane_server_stats stats;
};

namespace {

void fill_result(lane_result& r, const Req& q, int status) {
    memset(&r, 0, sizeof(r));
    r.stream = q.stream;
    r.status = status;
    r.frame_id = q.frame_id;
    r.t_submit_ns = q.t_submit;
    r.count = 0;
}

// caller holds s->mu
void complete(lane_server* s, lane_result& r, int64_t tag) {
    if (tag >= 0 && s->replay_out) {
        s->replay_out[tag] = r;
        --s->replay_left;
    } else {
        s->done.push_back(r);
    }
    s->cv_done.notify_all();
}

// a request's frame into its slot's buffer on `st`
hipError_t copy_frame(lane_server* s, int slot, const Req& q, hipStream_t st) {
    const lane_server::Class& c = s->classes[s->class_of[slot]];
    if (q.pitch == c.cfg.W && c.pitch == c.cfg.W)  // one contiguous copy
        return hipMemcpyAsync(s->slot_img[slot], q.frame, (size_t)c.cfg.W * c.cfg.H, hipMemcpyHostToDevice, st);
    return hipMemcpy2DAsync(s->slot_img[slot], (size_t)c.pitch, q.frame, (size_t)q.pitch, (size_t)c.cfg.W,
                            (size_t)c.cfg.H, hipMemcpyHostToDevice, st);
}

// Copy ahead, in two steps so that the copy is issued without the lock (a
// pageable frame makes the copy call wait for the bytes, and the lanes
// need the lock to take and complete requests meanwhile).
// (caller holds s->mu) claim the request at the head of an idle slot's
// queue if its frame is not copied yet: the slot is marked copying (busy 2),
// so no lane takes it until the copy and its event are issued
bool copy_ahead_claim(lane_server* s, int slot, std::vector<std::pair<int, Req>>& claims) {
    if (!s->up_stream || s->busy[slot] || s->error != LANE_OK) return false;
    const auto& d = s->pending[slot];
    if (d.empty() || s->up_id[slot] == d.front().id) return false;
    s->busy[slot] = 2;
    claims.emplace_back(slot, d.front());
    return true;
}

// (lk holds s->mu) issue the claimed copies with the lock released, then
// release their slots and wake the lanes
void copy_ahead_issue(lane_server* s, std::unique_lock<std::mutex>& lk,
                      std::vector<std::pair<int, Req>>& claims) {
    if (claims.empty()) return;
    std::vector<uint8_t> ok(claims.size());
    lk.unlock();
    for (size_t i = 0; i < claims.size(); ++i) {
        const int slot = claims[i].first;
        hipError_t e = copy_frame(s, slot, claims[i].second, s->up_stream);
        if (e == hipSuccess) e = hipEventRecord(s->up_ev[slot], s->up_stream);
        ok[i] = e == hipSuccess;
    }
    lk.lock();
    for (size_t i = 0; i < claims.size(); ++i) {
        const int slot = claims[i].first;
        // the copy did not go out: the refill that takes the request copies it
        s->up_id[slot] = ok[i] ? claims[i].second.id : 0;
        s->busy[slot] = 0;
    }
    claims.clear();
    s->work_gen.fetch_add(1, std::memory_order_release);
    s->cv_work.notify_all();
}

// one refill on lane L (its slots marked busy by the caller, so no other
// lane touches their buffers meanwhile)
int run_batch(lane_server* s, lane_server::Lane& L, const std::vector<Req>& batch,
              std::vector<lane_result>& out) {
    const int n_slots = (int)s->streams.size();
    memset(L.h_flags, 0, (size_t)n_slots);
    for (const Req& q : batch) L.h_flags[s->slot_of[q.stream]] = 1;
    // switches and the work lists of exactly these slots, then the set-up
    // kernel (counters, the vote's queue and split accumulators), which does
    // not read the frames and so runs while their copies may still be going
    hipError_t e = lane_batch_select(L.plan, L.h_flags, L.stream) == LANE_OK ? hipSuccess
                                                                              : hipErrorUnknown;
    if (e == hipSuccess && lane_batch_enqueue_pass_stage(L.plan, 0, L.stream) != LANE_OK) e = hipErrorUnknown;
    for (size_t i = 0; i < batch.size() && e == hipSuccess; ++i) {
        const Req& q = batch[i];
        const int slot = s->slot_of[q.stream];
        if (q.after_up) e = hipStreamWaitEvent(L.stream, s->up_ev[slot], 0);
        if (e == hipSuccess && !q.ahead) e = copy_frame(s, slot, q, L.stream);
    }
    uint32_t cls_mask = 0;
    if (s->per_subset)
        for (const Req& q : batch) cls_mask |= 1u << s->class_of[s->slot_of[q.stream]];
    if (e == hipSuccess) e = hipGraphLaunch(L.execs[s->per_subset ? cls_mask : 0], L.stream);
    // (the peaks of these slots are in h_peaks once the graph has run)
    if (e == hipSuccess) e = hipStreamSynchronize(L.stream);
    const int64_t t_done = now_ns();
    const int status = e == hipSuccess ? LANE_OK : LANE_E_DEVICE;
    out.resize(batch.size());
    for (size_t i = 0; i < batch.size(); ++i) {
        const Req& q = batch[i];
        lane_result& r = out[i];
        fill_result(r, q, status);
        r.t_done_ns = t_done;
        r.batch_frames = (int32_t)batch.size();
        if (status != LANE_OK) continue;
        const int slot = s->slot_of[q.stream];
        const int k = s->streams[slot].k;
        const int32_t* p = s->h_peaks + s->h_peak_off[slot];
        r.count = p[3 * k];
        for (int j = 0; j < k; ++j) {
            r.theta_idx[j] = p[j];
            r.r_idx[j] = p[k + j];
            r.votes[j] = p[2 * k + j];
        }
    }
    return status;
}

void worker_main(lane_server* s, int li) {
    hipSetDevice(s->dev);
    lane_server::Lane& L = s->lanes[li];
    std::vector<Req> batch;
    std::vector<lane_result> out;
    std::vector<std::pair<int, Req>> claims;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // work for this lane: a request of a stream that is not in a running refill
        auto any = [&] {
            for (size_t slot = 0; slot < s->pending.size(); ++slot)
                if (!s->pending[slot].empty() && !s->busy[slot]) return true;
            return false;
        };
        auto ready = [&] { return s->stop || (!s->paused && any()); };
        if (!ready() && s->cfg.spin_us > 0) {
            // poll for up to spin_us before sleeping: a request then starts
            // without the wake-up of a sleeping thread
            const int64_t until = now_ns() + (int64_t)s->cfg.spin_us * 1000;
            while (!ready() && now_ns() < until) {
                const uint64_t g0 = s->work_gen.load(std::memory_order_acquire);
                lk.unlock();
                while (s->work_gen.load(std::memory_order_acquire) == g0 && now_ns() < until) {
                }
                lk.lock();
            }
        }
        s->cv_work.wait(lk, ready);
        if (s->stop) break;
        // the oldest request of every such stream; with a deadline, requests
        // that waited too long are completed unrun and the next one takes the place
        batch.clear();
        const int64_t t_take = now_ns();
        for (auto& d : s->pending) {
            const int slot = (int)(&d - &s->pending[0]);
            if (s->busy[slot]) continue;
            while (!d.empty() && s->cfg.deadline_ns > 0 && t_take - d.front().t_submit > s->cfg.deadline_ns) {
                lane_result r;
                fill_result(r, d.front(), LANE_E_TIMEOUT);
                r.t_start_ns = r.t_done_ns = t_take;
                s->stats.timed_out += 1;
                complete(s, r, d.front().tag);
                d.pop_front();
            }
            if (d.empty()) continue;
            // a copy ahead into this slot (this request's, or one of a
            // request that timed out) is ordered before the refill's use
            Req q = d.front();
            q.ahead = s->up_id[slot] == q.id;
            q.after_up = s->up_id[slot] != 0;
            s->up_id[slot] = 0;
            s->busy[slot] = 1;
            batch.push_back(q);
            d.pop_front();
        }
        if (batch.empty()) continue;
        const int64_t t_start = now_ns();
        const bool failed = s->error != LANE_OK;
        lk.unlock();
        int st = LANE_E_DEVICE;
        if (!failed) st = run_batch(s, L, batch, out);
        lk.lock();
        if (failed) {
            out.resize(batch.size());
            for (size_t i = 0; i < batch.size(); ++i) fill_result(out[i], batch[i], LANE_E_DEVICE);
        }
        if (st != LANE_OK) s->error = st;
        s->stats.batches += 1;
        s->stats.frames_in_batches += (int64_t)batch.size();
        for (size_t i = 0; i < batch.size(); ++i) {
            out[i].t_start_ns = t_start;
            s->stats.completed += 1;
            complete(s, out[i], batch[i].tag);
        }
        // the slots are free again: the next frames of their streams may go ahead
        for (const Req& q : batch) {
            const int slot = s->slot_of[q.stream];
            s->busy[slot] = 0;
            copy_ahead_claim(s, slot, claims);
        }
        s->work_gen.fetch_add(1, std::memory_order_release);
        copy_ahead_issue(s, lk, claims);
    }
}

// (lk holds s->mu) queue one request; a copy ahead of its frame is issued
// with the lock released
int submit_locked(lane_server* s, std::unique_lock<std::mutex>& lk, int stream, const uint8_t* frame,
                  int pitch, uint64_t frame_id, int64_t tag, std::vector<std::pair<int, Req>>& claims) {
    Req q;
    q.stream = stream;
    q.pitch = pitch;
    q.frame = frame;
    q.frame_id = frame_id;
    q.t_submit = now_ns();
    q.tag = tag;
    q.id = s->next_id++;
    q.ahead = q.after_up = false;
    s->stats.submitted += 1;
    const int slot = s->slot_of[stream];
    auto& d = s->pending[slot];
    if ((int)d.size() >= s->cfg.max_pending) {
        s->stats.dropped += 1;
        lane_result r;
        fill_result(r, q, LANE_E_BUSY);
        r.t_done_ns = q.t_submit;
        complete(s, r, tag);
        return LANE_E_BUSY;
    }
    d.push_back(q);
    if (d.size() == 1 && copy_ahead_claim(s, slot, claims)) {
        copy_ahead_issue(s, lk, claims);  // wakes the lanes
        return LANE_OK;
    }
    s->work_gen.fetch_add(1, std::memory_order_release);
    s->cv_work.notify_one();
    return LANE_OK;
}

int check_submit(lane_server* s, int32_t stream, const uint8_t* frame, int32_t pitch) {
    if (!s || !frame || stream < 0 || stream >= (int)s->slot_of.size()) return LANE_E_ARG;
    const int slot = s->slot_of[stream];
    if (slot < 0) return LANE_E_ARG;
    if (pitch < s->streams[slot].W) return LANE_E_ARG;
    return LANE_OK;
}

void free_server(lane_server* s) {
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->work_gen.fetch_add(1, std::memory_order_release);
    }
    s->cv_work.notify_all();
    for (auto& L : s->lanes)
        if (L.worker.joinable()) L.worker.join();
    for (auto& L : s->lanes)
        if (L.stream) hipStreamSynchronize(L.stream);
    if (s->up_stream) {
        hipStreamSynchronize(s->up_stream);
        hipStreamDestroy(s->up_stream);
    }
    for (auto ev : s->up_ev)
        if (ev) hipEventDestroy(ev);
    for (auto& L : s->lanes) {
        for (auto x : L.execs)
            if (x) hipGraphExecDestroy(x);
        for (auto g : L.graphs)
            if (g) hipGraphDestroy(g);
        if (L.plan) lane_batch_destroy(L.plan);
        if (L.stream) hipStreamDestroy(L.stream);
        if (L.h_flags) hipHostFree(L.h_flags);
    }
    if (s->dmem) hipFree(s->dmem);
    if (s->h_peaks) hipHostFree(s->h_peaks);
    delete s;
}

}  // namespace

extern "C" {

int lane_server_plan(const lane_stream_cfg* streams, int32_t n, const lane_server_cfg* cfg,
                     uint8_t* admitted, size_t* stream_bytes, size_t* total_bytes) {
    if (!streams || n < 1 || !cfg) return LANE_E_ARG;
    int st = check_cfg(*cfg);
    if (st != LANE_OK) return st;
    for (int i = 0; i < n; ++i)
        if ((st = check_stream(streams[i], cfg->pruned)) != LANE_OK) return st;
    const size_t t = plan_admission(streams, n, *cfg, admitted, stream_bytes);
    if (total_bytes) *total_bytes = t;
    return LANE_OK;
}

int lane_server_create(const lane_stream_cfg* streams, int32_t n, const lane_server_cfg* cfg,
                       lane_server** out, uint8_t* admitted_opt) {
    if (!streams || n < 1 || !cfg || !out) return LANE_E_ARG;
    *out = nullptr;
    int st = check_cfg(*cfg);
    if (st != LANE_OK) return st;
    for (int i = 0; i < n; ++i)
        if ((st = check_stream(streams[i], cfg->pruned)) != LANE_OK) return st;
    std::vector<uint8_t> adm(n, 0);
    plan_admission(streams, n, *cfg, adm.data(), nullptr);
    if (admitted_opt) memcpy(admitted_opt, adm.data(), (size_t)n);
    int n_adm = 0;
    for (int i = 0; i < n; ++i) n_adm += adm[i];
    if (n_adm == 0) return LANE_E_WS;

    lane_server* s = new (std::nothrow) lane_server();
    if (!s) return LANE_E_DEVICE;
    s->cfg = *cfg;
    memset(&s->stats, 0, sizeof(s->stats));
    if (hipGetDevice(&s->dev) != hipSuccess) {
        free_server(s);
        return LANE_E_DEVICE;
    }
    // classes in order of first appearance; slots grouped by class
    std::map<ClassKey, int> cidx;
    std::vector<std::vector<int>> members;
    for (int i = 0; i < n; ++i) {
        if (!adm[i]) continue;
        const ClassKey k = key_of(streams[i]);
        if (!cidx.count(k)) {
            cidx[k] = (int)members.size();
            members.emplace_back();
        }
        members[cidx[k]].push_back(i);
    }
    s->slot_of.assign(n, -1);
    for (size_t c = 0; c < members.size(); ++c) {
        lane_server::Class cl;
        memset(&cl, 0, sizeof(cl));
        cl.cfg = streams[members[c][0]];
        cl.first_slot = (int)s->streams.size();
        cl.n = (int)members[c].size();
        cl.pitch = (cl.cfg.W + 15) / 16 * 16;
        for (int i : members[c]) {
            s->slot_of[i] = (int)s->streams.size();
            s->stream_of.push_back(i);
            s->streams.push_back(streams[i]);
            s->class_of.push_back((int)c);
        }
        s->classes.push_back(cl);
    }
    const int n_slots = (int)s->streams.size();
    s->pending.resize(n_slots);

    // one device allocation: per class the frame slots (contiguous), masks,
    // logits and activations; per slot the path's buffers; shared tables
    std::vector<StreamSizes> sz(n_slots);
    for (int i = 0; i < n_slots; ++i) sz[i] = stream_sizes(s->streams[i], *cfg);
    std::map<int, size_t> trig_off;
    size_t off = 0;
    std::vector<size_t> o_img(s->classes.size()), o_mask(s->classes.size()), o_log(s->classes.size());
    for (size_t c = 0; c < s->classes.size(); ++c) {
        const auto& cl = s->classes[c];
        const StreamSizes& z = sz[cl.first_slot];
        o_img[c] = off;
        off += z.img * cl.n;
        o_mask[c] = off;
        off += z.mask * cl.n;
        o_log[c] = off;
        off += z.logits * cl.n;
    }
    std::vector<size_t> o_slot(n_slots);
    for (int i = 0; i < n_slots; ++i) {
        o_slot[i] = off;
        off += sz[i].total() - sz[i].img - sz[i].mask - sz[i].logits - sz[i].split;
        if (!trig_off.count(s->streams[i].n_theta)) {
            trig_off[s->streams[i].n_theta] = off;
            off += al256(sizeof(int16_t) * 2 * (size_t)s->streams[i].n_theta);
        }
    }
    size_t o_pk = off, o_par = off;
    if (cfg->pruned) {
        size_t pk = 0;
        lane_cnn_sizes(16, 16, 1, &pk, nullptr, nullptr);
        o_pk = off;
        off += al256(pk);
        o_par = off;
        off += al256(sizeof(float) * LANE_CNN_PARAMS);
    }
    s->dbytes = off;
    s->stats.device_bytes = (int64_t)off;
    s->stats.streams_admitted = n_slots;
    bool ok = hipMalloc(&s->dmem, off) == hipSuccess;
    s->lanes.resize((size_t)serve_lanes(*cfg));
    for (auto& L : s->lanes) {
        ok = ok && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&L.h_flags, (size_t)n_slots, hipHostMallocDefault) == hipSuccess;
    }
    ok = ok && hipStreamCreateWithFlags(&s->up_stream, hipStreamNonBlocking) == hipSuccess;
    s->up_ev.assign(n_slots, nullptr);
    s->up_id.assign(n_slots, 0);
    s->busy.assign(n_slots, 0);
    for (int i = 0; i < n_slots && ok; ++i)
        ok = hipEventCreateWithFlags(&s->up_ev[i], hipEventDisableTiming) == hipSuccess;
    // each slot's peaks on cache lines of their own (256 bytes): two lanes'
    // refills store into the buffer while the other's results are read
    size_t hp = 0;
    s->h_peak_off.resize(n_slots);
    for (int i = 0; i < n_slots; ++i) {
        s->h_peak_off[i] = hp;
        hp += (3 * (size_t)s->streams[i].k + 1 + 63) & ~(size_t)63;
    }
    ok = ok && hipHostMalloc((void**)&s->h_peaks, sizeof(int32_t) * hp, hipHostMallocDefault) == hipSuccess;
    int32_t* d_peaks = nullptr;  // h_peaks as the device addresses it
    ok = ok && hipHostGetDevicePointer((void**)&d_peaks, s->h_peaks, 0) == hipSuccess;
    if (!ok) {
        free_server(s);
        return LANE_E_DEVICE;
    }
    char* base = (char*)s->dmem;
    // zeroed state first: every slot starts with an empty frame
    hipStream_t st0 = s->lanes[0].stream;
    ok = ok && hipMemsetAsync(s->dmem, 0, off, st0) == hipSuccess;
    ok = ok && hipStreamSynchronize(st0) == hipSuccess;
    // trig tables (host helper, then one copy each)
    for (auto& t : trig_off) {
        std::vector<int16_t> cs(2 * (size_t)t.first);
        lane_make_trig_q14(t.first, cs.data(), cs.data() + t.first);
        ok = ok && hipMemcpy(base + t.second, cs.data(), sizeof(int16_t) * cs.size(),
                             hipMemcpyHostToDevice) == hipSuccess;
    }
    if (cfg->pruned) {
        ok = ok && hipMemcpy(base + o_par, cfg->cnn_params, sizeof(float) * LANE_CNN_PARAMS,
                             hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && lane_cnn_pack((const float*)(base + o_par), base + o_pk, st0) == LANE_OK;
    }
    ok = ok && hipStreamSynchronize(st0) == hipSuccess;
    std::vector<lane_frame> frames(n_slots);
    s->slot_img.resize(n_slots);
    for (size_t c = 0; c < s->classes.size() && ok; ++c) {
        auto& cl = s->classes[c];
        cl.img = (uint8_t*)(base + o_img[c]);
        cl.mask = (uint8_t*)(base + o_mask[c]);
        cl.logits = (float*)(base + o_log[c]);
        for (int j = 0; j < cl.n; ++j) {
            const int i = cl.first_slot + j;
            const lane_stream_cfg& sc = s->streams[i];
            const StreamSizes& z = sz[i];
            int32_t D = 0;
            lane_r_offset(sc.W, sc.H, &D);
            char* p = base + o_slot[i];
            lane_frame& f = frames[i];
            memset(&f, 0, sizeof(f));
            s->slot_img[i] = cl.img + z.img * j;
            f.img = s->slot_img[i];
            f.W = sc.W;
            f.H = sc.H;
            f.pitch = cl.pitch;
            f.threshold = sc.threshold;
            f.border_mode = sc.border_mode;
            f.edges = (uint8_t*)p;
            p += z.edges;
            f.list = (uint32_t*)p;
            p += z.list;
            f.cos_q14 = (const int16_t*)(base + trig_off[sc.n_theta]);
            f.sin_q14 = f.cos_q14 + sc.n_theta;
            f.n_theta = sc.n_theta;
            f.r_offset = D;
            f.n_r = 2 * D + 1;
            // the mask kernel writes a class's masks back to back, [n][th][tw]
            const size_t tiles = (size_t)((sc.H + 7) / 8) * (size_t)((sc.W + 7) / 8);
            f.tile_mask_opt = cfg->pruned ? cl.mask + tiles * j : nullptr;
            f.acc = (int32_t*)p;
            p += z.acc;
            f.k = sc.k;
            f.h_theta = std::max(1, (sc.n_theta + 99) / 100);
            f.h_r = std::max(1, (f.n_r + 99) / 100);
            f.min_votes = 1;
            f.peaks = d_peaks + s->h_peak_off[i];
            f.peaks_ws = p;
            f.peaks_ws_bytes = z.peaks_ws;
            p += z.peaks_ws;
            f.counters_opt = (uint32_t*)p;
        }
    }
    lane_tune tune = {serve_vote_rows(*cfg), 1, 0, cfg->sobel_strip_rows > 0 ? cfg->sobel_strip_rows : 8,
                      serve_vote_split(*cfg)};
    for (auto& L : s->lanes) {
        // a refill runs one or a few frames: the latency shape of the Sobel pass
        if (ok && lane_batch_create_shaped(frames.data(), n_slots, &tune, 1, &L.plan) != LANE_OK) ok = false;
        ok = ok && lane_batch_active_flags(L.plan, &L.d_flags) == LANE_OK;
    }
    if (!ok) {
        free_server(s);
        return LANE_E_DEVICE;
    }
    // the whole refill as one graph: proposal per class (pruned), then the path
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        free_server(s);
        return LANE_E_DEVICE;
    }
    // pruned: the network and the masks run first, in the same sequence as
    // the rest (a branch of their own beside the Sobel pass, forked and
    // joined inside the graph, measured the same at p50 and worse in the
    // tails, with a second lane's refill sharing the GPU)
    hipError_t e = hipSuccess;
    int cst = LANE_OK;
    // one capture for lane L: the classes of cls_mask run their network and masks
    auto capture = [&](lane_server::Lane& L, uint32_t cls_mask, hipGraph_t* gout, hipGraphExec_t* xout) {
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return;
        if (cfg->pruned) {
            for (size_t c = 0; c < s->classes.size() && e == hipSuccess; ++c) {
                if (c < 32 && !((cls_mask >> c) & 1u)) continue;
                auto& cl = s->classes[c];
                const uint8_t* fl = L.d_flags + cl.first_slot;
                // network and tile masks in one kernel
                cst = lane_cnn_infer_mask_active(cl.img, cl.cfg.W, cl.cfg.H, cl.pitch,
                                                 (int64_t)sz[cl.first_slot].img, cl.n, base + o_pk,
                                                 cl.logits, cfg->conf, cl.mask, fl, cs);
                if (cst != LANE_OK) break;
            }
        }
        // (stage 0, the set-up kernel, is launched by the refill ahead of the
        // wait for its frames' copies: it does not read the frames)
        for (int stg = 1; stg < 4 && e == hipSuccess && cst == LANE_OK; ++stg)
            cst = lane_batch_enqueue_pass_stage(L.plan, stg, cs);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess && cst == LANE_OK) {
            *gout = g;
            e = hipGraphInstantiate(xout, g, nullptr, nullptr, 0);
        } else if (g) {
            hipGraphDestroy(g);
        }
    };
    const size_t n_cls = s->classes.size();
    s->per_subset = cfg->pruned && n_cls > 1 && n_cls <= (size_t)kSubsetClasses;
    const size_t n_graphs = s->per_subset ? ((size_t)1 << n_cls) : 1;
    for (auto& L : s->lanes) {
        L.graphs.assign(n_graphs, nullptr);
        L.execs.assign(n_graphs, nullptr);
        if (s->per_subset) {
            for (size_t m = 1; m < n_graphs && e == hipSuccess && cst == LANE_OK; ++m)
                capture(L, (uint32_t)m, &L.graphs[m], &L.execs[m]);
        } else if (e == hipSuccess && cst == LANE_OK) {
            capture(L, 0xFFFFFFFFu, &L.graphs[0], &L.execs[0]);
        }
    }
    hipStreamDestroy(cs);
    if (e != hipSuccess || cst != LANE_OK) {
        free_server(s);
        return LANE_E_DEVICE;
    }
    for (size_t li = 0; li < s->lanes.size(); ++li) s->lanes[li].worker = std::thread(worker_main, s, (int)li);
    *out = s;
    return LANE_OK;
}

int lane_server_submit(lane_server* s, int32_t stream, const uint8_t* frame, int32_t pitch,
                       uint64_t frame_id) {
    const int st = check_submit(s, stream, frame, pitch);
    if (st != LANE_OK) return st;
    std::vector<std::pair<int, Req>> claims;
    std::unique_lock<std::mutex> lk(s->mu);
    return submit_locked(s, lk, stream, frame, pitch, frame_id, -1, claims);
}

int lane_server_poll(lane_server* s, lane_result* out, int32_t max, int32_t wait_ms, int32_t* n_out) {
    if (!s || !out || max < 1 || !n_out) return LANE_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_ms != 0) {
        auto ready = [&] { return !s->done.empty(); };
        if (wait_ms < 0) s->cv_done.wait(lk, ready);
        else s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
    }
    int n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = n;
    return LANE_OK;
}

int lane_server_replay(lane_server* s, const lane_request* reqs, int32_t n, lane_result* results) {
    if (!s || !reqs || n < 1 || !results) return LANE_E_ARG;
    for (int i = 0; i < n; ++i) {
        const int st = check_submit(s, reqs[i].stream, reqs[i].frame, reqs[i].pitch);
        if (st != LANE_OK) return st;
        if (reqs[i].t_offset_ns < 0 || (i > 0 && reqs[i].t_offset_ns < reqs[i - 1].t_offset_ns))
            return LANE_E_ARG;
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->replay_out) return LANE_E_BUSY;  // one replay at a time
        s->replay_out = results;
        s->replay_left = n;
    }
    std::vector<std::pair<int, Req>> claims;
    claims.reserve(1);
    const int64_t t0 = now_ns();
    for (int i = 0; i < n; ++i) {
        const int64_t target = t0 + reqs[i].t_offset_ns;
        // sleep to just before the arrival time, then spin the rest
        const int64_t early = target - now_ns() - 200000;
        if (early > 0) std::this_thread::sleep_for(std::chrono::nanoseconds(early));
        while (now_ns() < target) {
        }
        std::unique_lock<std::mutex> lk(s->mu);
        submit_locked(s, lk, reqs[i].stream, reqs[i].frame, reqs[i].pitch, reqs[i].frame_id, i, claims);
    }
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->replay_left == 0; });
    s->replay_out = nullptr;
    return LANE_OK;
}

int lane_server_stats_get(lane_server* s, lane_server_stats* out) {
    if (!s || !out) return LANE_E_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->error = s->error;
    return LANE_OK;
}

int lane_server_pause(lane_server* s, int32_t paused) {
    if (!s || (paused != 0 && paused != 1)) return LANE_E_ARG;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->paused = paused != 0;
        s->work_gen.fetch_add(1, std::memory_order_release);
    }
    s->cv_work.notify_all();
    return LANE_OK;
}

int lane_server_destroy(lane_server* s) {
    if (!s) return LANE_E_ARG;
    free_server(s);
    return LANE_OK;
}

}  // extern "C"
