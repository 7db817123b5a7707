// Request server (include/tdes_serve.h): admission by in-flight bytes and
// arena space, continuous batching over HIP streams, completion tracking.
#include <string.h>

#include <chrono>
#include <deque>
#include <iterator>
#include <map>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "tdes_serve.h"

namespace {

constexpr uint64_t kAlign = 256;  // arena granularity
constexpr int kPlainEvents = 4096;
// Batches of up to this many requests run as one plain launch per request:
// three small requests take ~10 us each back to back, before the copy, scan
// and batched kernel (~45 us) would finish.
constexpr size_t kPlainBatchMax = 3;
// Larger batches of at most this many requests and this many bytes in all
// run as one launch of the table kernel over the requests (one block per
// lane, each request's round keys built on the host), which finishes well
// before the batched bitsliced path, whose lanes run 32 blocks each.
constexpr size_t kTableBatchMax = tdes::kSpboxMultiMax;
// Its staging area: descriptors, then round keys (one pinned host buffer
// mirrored by one device buffer, so a batch needs a single copy).
constexpr size_t kTabKeysOff = kTableBatchMax * sizeof(tdes::SpboxMsg);
constexpr size_t kTabBytes = kTabKeysOff + kTableBatchMax * sizeof(tdes::SpboxKeys);
static_assert(kTabKeysOff % 16 == 0, "round keys 16-byte aligned");

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Arena {
  public:
    void reset(uint64_t size) {
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    bool alloc(uint64_t bytes, uint64_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const uint64_t rest = it->second - bytes;
            const uint64_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t used_ = 0;
};

struct Active {
    tdes_request req;
    uint64_t out_off, out_bytes;  // arena range (out_bytes rounded to kAlign)
    double t_submit, t_admit;
};

// A slot's staging area, one pinned host buffer mirrored by one device
// buffer so a batch needs a single copy: [first-slice table as the batched
// cipher's workspace | descriptors | key bundles].
struct Staging {
    size_t ws_off = 0, msgs_off = 0, keys_off = 0, bytes = 0;
    void layout(size_t n) {
        ws_off = 0;
        msgs_off = (tdes::batch_workspace_bytes(n) + 255) / 256 * 256;
        keys_off = msgs_off + (n * sizeof(tdes_msg) + 255) / 256 * 256;
        bytes = keys_off + n * 24;
    }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    uint32_t batch = 0;
    double t_launch = 0;
    uint32_t polls_left = 0;
    std::vector<Active> reqs;
    Staging lay;
    uint8_t *h_stage = nullptr, *d_stage = nullptr;
    uint32_t *d_sched = nullptr;
    uint8_t *h_tab = nullptr, *d_tab = nullptr;  // table-kernel batches
};

struct PlainEntry {
    Active a;
    hipEvent_t ev;
    uint32_t seq;
    double t_launch;
};

uint64_t round_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct tdes_server {
    tdes_server_config cfg{};
    uint64_t budget = 0;
    Arena arena;
    std::deque<std::pair<tdes_request, double>> queue;
    std::deque<tdes_completion> done;
    std::unordered_map<uint64_t, uint64_t> live;  // arena offset -> bytes of a completed result
    std::vector<Slot> slots;
    std::deque<PlainEntry> plain;                 // plain mode: launched, in order
    std::vector<hipEvent_t> plain_events;         // plain mode: free events
    hipStream_t plain_stream = nullptr;
    tdes_server_stats st{};
    uint32_t next_batch = 0;
    bool device = true;
};

namespace {

tdes_status fail(tdes_status s, const char *msg) { return tdes::set_last_error(s, msg); }

void complete(tdes_server *s, const Active &a, uint32_t batch, double t_launch, double t_done,
              int32_t status) {
    tdes_completion c{};
    c.tag = a.req.tag;
    c.d_out = static_cast<uint8_t *>(s->cfg.d_arena) + a.out_off;
    c.nbytes = a.req.nbytes;
    c.status = status;
    c.batch = batch;
    c.t_submit = a.t_submit;
    c.t_admit = a.t_admit;
    c.t_launch = t_launch;
    c.t_done = t_done;
    s->done.push_back(c);
    s->live[a.out_off] = a.out_bytes;
    s->st.in_flight_bytes -= a.req.nbytes;  // the input is the caller's again
    s->st.completed++;
}

// A request whose batch failed on the device: it completes with `status`
// and no result, and its budget and arena range are given back at once.
void complete_failed(tdes_server *s, const Active &a, uint32_t batch, double t_launch,
                     int32_t status) {
    tdes_completion c{};
    c.tag = a.req.tag;
    c.nbytes = a.req.nbytes;
    c.status = status;
    c.batch = batch;
    c.t_submit = a.t_submit;
    c.t_admit = a.t_admit;
    c.t_launch = t_launch;
    c.t_done = now_s();
    s->done.push_back(c);
    s->arena.release(a.out_off, a.out_bytes);
    s->st.in_flight_bytes -= a.req.nbytes + a.out_bytes;
    s->st.arena_used_bytes = s->arena.used();
    s->st.completed++;
    s->st.failed++;
}

void reject(tdes_server *s, const tdes_request &r, double t, int32_t status) {
    tdes_completion c{};
    c.tag = r.tag;
    c.nbytes = r.nbytes;
    c.status = status;
    c.t_submit = c.t_admit = c.t_launch = c.t_done = t;
    s->done.push_back(c);
    s->st.rejected++;
}

// Admit the head of the queue if it fits: reserve its output and budget.
bool admit_head(tdes_server *s, Active *a) {
    const tdes_request r = s->queue.front().first;  // a copy: the entry is popped below
    const uint64_t out_bytes = round_up(r.nbytes);
    if (s->st.in_flight_bytes + r.nbytes + out_bytes > s->budget) return false;
    uint64_t off;
    if (!s->arena.alloc(out_bytes, &off)) return false;
    a->req = r;
    a->out_off = off;
    a->out_bytes = out_bytes;
    a->t_submit = s->queue.front().second;
    a->t_admit = now_s();
    s->queue.pop_front();
    s->st.in_flight_bytes += r.nbytes + out_bytes;
    if (s->st.in_flight_bytes > s->st.peak_in_flight_bytes)
        s->st.peak_in_flight_bytes = s->st.in_flight_bytes;
    s->st.arena_used_bytes = s->arena.used();
    if (s->st.arena_used_bytes > s->st.peak_arena_used_bytes)
        s->st.peak_arena_used_bytes = s->st.arena_used_bytes;
    s->st.admitted++;
    s->st.queued = s->queue.size();
    return true;
}

tdes_status launch_slot(tdes_server *s, Slot &sl) {
    const size_t n = sl.reqs.size();
    sl.batch = s->next_batch++;
    sl.busy = true;
    sl.t_launch = now_s();
    s->st.batches++;
    s->st.batched_msgs += n;
    for (const Active &a : sl.reqs) s->st.batched_bytes += a.req.nbytes;
    if (!s->device) {
        sl.polls_left = s->cfg.test_polls > 1 ? s->cfg.test_polls - 1 : 1;
        return s->cfg.test_fail_batch == sl.batch + 1
                   ? fail(TDES_ERR_DEVICE, "injected launch failure (host test mode)")
                   : TDES_OK;
    }
    hipError_t e = hipSuccess;
    if (n <= kPlainBatchMax) {
        // a batch of a few requests: plain launches with host-built key
        // material (no copies, one launch each, the kernel tdes_ecb_crypt
        // picks for the size) finish sooner than the copy, the descriptor
        // scan and the batched kernel, whose lanes each run 32 blocks
        // through the rounds
        for (const Active &a : sl.reqs) {
            tdes_schedule ks;
            for (int b = 0; b < 3; b++) tdes::des_round_keys(a.req.key24 + 8 * b, ks.k[b]);
            e = tdes::launch_ecb_auto(ks, (int)a.req.dir, static_cast<const uint8_t *>(a.req.d_in),
                                      static_cast<uint8_t *>(s->cfg.d_arena) + a.out_off,
                                      a.req.nbytes, sl.stream);
            if (e != hipSuccess) break;
        }
        if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
        return e == hipSuccess ? TDES_OK : fail(TDES_ERR_DEVICE, hipGetErrorString(e));
    }
    uint64_t batch_bytes = 0;
    for (const Active &a : sl.reqs) batch_bytes += a.req.nbytes;
    if (n <= kTableBatchMax && batch_bytes <= tdes::spbox_one_pass_bytes()) {
        tdes::SpboxMsg *tm = reinterpret_cast<tdes::SpboxMsg *>(sl.h_tab);
        tdes::SpboxKeys *tk = reinterpret_cast<tdes::SpboxKeys *>(sl.h_tab + kTabKeysOff);
        uint64_t nb[kTableBatchMax];
        for (size_t i = 0; i < n; i++) nb[i] = sl.reqs[i].req.nbytes / 8;
        const uint32_t per = tdes::spbox_multi_lanes(nb, n);
        uint64_t wg = 0;
        for (size_t i = 0; i < n; i++) {
            const Active &a = sl.reqs[i];
            tdes_schedule ks;
            for (int b = 0; b < 3; b++) tdes::des_round_keys(a.req.key24 + 8 * b, ks.k[b]);
            tdes::RoundSequence seq;
            tdes::round_sequence(ks, (int)a.req.dir, &seq);
            tdes::spbox_keys(seq, &tk[i]);
            tm[i].in = static_cast<const uint8_t *>(a.req.d_in);
            tm[i].out = static_cast<uint8_t *>(s->cfg.d_arena) + a.out_off;
            tm[i].nblocks = nb[i];
            tm[i].first_wg = (uint32_t)wg;
            tm[i].pad = 0;
            wg += (nb[i] + per - 1) / per;
        }
        // (the tail of the descriptor area is copied too: it is small)
        e = hipMemcpyAsync(sl.d_tab, sl.h_tab, kTabKeysOff + n * sizeof(tdes::SpboxKeys),
                           hipMemcpyHostToDevice, sl.stream);
        if (e == hipSuccess)
            e = tdes::launch_spbox_multi(
                reinterpret_cast<const tdes::SpboxMsg *>(sl.d_tab), (uint32_t)n,
                reinterpret_cast<const tdes::SpboxKeys *>(sl.d_tab + kTabKeysOff), per,
                (uint32_t)wg, sl.stream);
        if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
        return e == hipSuccess ? TDES_OK : fail(TDES_ERR_DEVICE, hipGetErrorString(e));
    }
    // laid out for this batch's size (the buffers hold the largest batch), so
    // the copy carries only what the batch uses
    Staging lay;
    lay.layout(n);
    uint64_t *ws = reinterpret_cast<uint64_t *>(sl.h_stage + lay.ws_off);
    tdes_msg *msgs = reinterpret_cast<tdes_msg *>(sl.h_stage + lay.msgs_off);
    uint8_t *keys = sl.h_stage + lay.keys_off;
    uint64_t total = 0;
    for (size_t i = 0; i < n; i++) {
        const Active &a = sl.reqs[i];
        tdes_msg m;
        m.in_off = (uint64_t)(uintptr_t)a.req.d_in;  // against a zero input base
        m.out_off = a.out_off;
        m.nbytes = a.req.nbytes;
        m.sched_idx = (uint32_t)i;
        m.dir = a.req.dir;
        msgs[i] = m;
        memcpy(keys + 24 * i, a.req.key24, 24);
        ws[2 + i] = total;
        total += (a.req.nbytes + 255) / 256;  // 256-byte lane slices
    }
    ws[0] = total;
    ws[1] = 0;
    ws[2 + n] = total;
    e = hipMemcpyAsync(sl.d_stage, sl.h_stage, lay.bytes, hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess)
        e = tdes::launch_expand(sl.d_stage + lay.keys_off, n, sl.d_sched, sl.stream);
    if (e == hipSuccess)
        e = tdes::launch_batch_prefixed(
            reinterpret_cast<const tdes_msg *>(sl.d_stage + lay.msgs_off), n, sl.d_sched, n,
            nullptr, static_cast<uint8_t *>(s->cfg.d_arena),
            reinterpret_cast<const uint64_t *>(sl.d_stage + lay.ws_off), total, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    return e == hipSuccess ? TDES_OK : fail(TDES_ERR_DEVICE, hipGetErrorString(e));
}

// Every request of the slot's batch fails (launch or completion query
// error).  The slot's stream is drained first, so work already enqueued for
// the batch cannot touch the staging area or the arena after the slot and
// the requests' output ranges are reused.
void fail_slot(tdes_server *s, Slot &sl) {
    if (s->device && sl.stream) (void)hipStreamSynchronize(sl.stream);
    for (const Active &a : sl.reqs) complete_failed(s, a, sl.batch, sl.t_launch, TDES_ERR_DEVICE);
    sl.reqs.clear();
    sl.busy = false;
}

tdes_status progress_batched(tdes_server *s) {
    uint32_t busy = 0;
    for (Slot &sl : s->slots) {  // retire
        if (!sl.busy) continue;
        bool finished;
        if (s->device) {
            const hipError_t q = hipEventQuery(sl.done);
            if (q != hipSuccess && q != hipErrorNotReady) {
                fail(TDES_ERR_DEVICE, hipGetErrorString(q));
                fail_slot(s, sl);
                continue;
            }
            finished = q == hipSuccess;
        } else {
            finished = sl.polls_left <= 1;
            if (!finished) sl.polls_left--;
        }
        if (!finished) continue;
        const double t = now_s();
        for (const Active &a : sl.reqs) complete(s, a, sl.batch, sl.t_launch, t, TDES_OK);
        sl.reqs.clear();
        sl.busy = false;
    }
    for (Slot &sl : s->slots) {  // admit and launch
        if (sl.busy) {
            busy++;
            continue;
        }
        uint64_t bytes = 0;
        while (!s->queue.empty() && sl.reqs.size() < s->cfg.max_batch_msgs) {
            const uint64_t nb = s->queue.front().first.nbytes;
            if (s->cfg.max_batch_bytes && !sl.reqs.empty() && bytes + nb > s->cfg.max_batch_bytes)
                break;
            Active a;
            if (!admit_head(s, &a)) break;
            bytes += nb;
            sl.reqs.push_back(a);
        }
        if (sl.reqs.empty()) break;  // nothing admissible: later slots stay free too
        if (launch_slot(s, sl) != TDES_OK) {
            fail_slot(s, sl);
            continue;
        }
        busy++;
    }
    s->st.busy_slots = busy;
    if (busy > s->st.peak_busy_slots) s->st.peak_busy_slots = busy;
    return TDES_OK;
}

tdes_status progress_plain(tdes_server *s) {
    while (!s->plain.empty()) {  // retire in order
        PlainEntry &p = s->plain.front();
        const hipError_t q = hipEventQuery(p.ev);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
            fail(TDES_ERR_DEVICE, hipGetErrorString(q));
            (void)hipStreamSynchronize(s->plain_stream);
            complete_failed(s, p.a, p.seq, p.t_launch, TDES_ERR_DEVICE);
        } else {
            complete(s, p.a, p.seq, p.t_launch, now_s(), TDES_OK);
        }
        s->plain_events.push_back(p.ev);
        s->plain.pop_front();
    }
    while (!s->queue.empty() && !s->plain_events.empty()) {  // one launch per request
        Active a;
        if (!admit_head(s, &a)) break;
        tdes_schedule ks;
        for (int b = 0; b < 3; b++) tdes::des_round_keys(a.req.key24 + 8 * b, ks.k[b]);
        PlainEntry p{a, s->plain_events.back(), s->next_batch++, now_s()};
        s->plain_events.pop_back();
        hipError_t e = tdes::launch_ecb_auto(ks, (int)a.req.dir,
                                             static_cast<const uint8_t *>(a.req.d_in),
                                             static_cast<uint8_t *>(s->cfg.d_arena) + a.out_off,
                                             a.req.nbytes, s->plain_stream);
        if (e == hipSuccess) e = hipEventRecord(p.ev, s->plain_stream);
        if (e != hipSuccess) {  // the request fails; its event goes back to the pool
            fail(TDES_ERR_DEVICE, hipGetErrorString(e));
            (void)hipStreamSynchronize(s->plain_stream);
            complete_failed(s, a, p.seq, p.t_launch, TDES_ERR_DEVICE);
            s->plain_events.push_back(p.ev);
            continue;
        }
        s->plain.push_back(p);
        s->st.batches++;
        s->st.batched_msgs++;
        s->st.batched_bytes += a.req.nbytes;
    }
    s->st.busy_slots = s->plain.empty() ? 0 : 1;
    if (s->st.busy_slots > s->st.peak_busy_slots) s->st.peak_busy_slots = s->st.busy_slots;
    return TDES_OK;
}

void free_device(tdes_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.h_stage) (void)hipHostFree(sl.h_stage);
        if (sl.d_stage) (void)hipFree(sl.d_stage);
        if (sl.d_sched) (void)hipFree(sl.d_sched);
        if (sl.h_tab) (void)hipHostFree(sl.h_tab);
        if (sl.d_tab) (void)hipFree(sl.d_tab);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->plain_stream) (void)hipStreamSynchronize(s->plain_stream);
    for (PlainEntry &p : s->plain) (void)hipEventDestroy(p.ev);
    for (hipEvent_t e : s->plain_events) (void)hipEventDestroy(e);
    if (s->plain_stream) (void)hipStreamDestroy(s->plain_stream);
}

}  // namespace

extern "C" {

double tdes_server_now(void) { return now_s(); }

tdes_status tdes_server_create(const tdes_server_config *cfg, tdes_server **out) {
    if (cfg == nullptr || out == nullptr) return fail(TDES_ERR_ARG, "NULL config or result");
    *out = nullptr;
    if (cfg->mode > TDES_SERVE_HOST_TEST || cfg->slots < 1 || cfg->slots > 16 ||
        cfg->max_batch_msgs < 1 || cfg->max_batch_msgs > 65536 || cfg->arena_bytes == 0 ||
        cfg->d_arena == nullptr)
        return fail(TDES_ERR_ARG, "bad server configuration");
    if ((uintptr_t)cfg->d_arena % kAlign != 0) return fail(TDES_ERR_ALIGN, "arena must be 256-byte aligned");
    tdes_server *s = new tdes_server;
    s->cfg = *cfg;
    s->budget = cfg->budget_bytes ? cfg->budget_bytes : 2 * cfg->arena_bytes;
    s->arena.reset(cfg->arena_bytes / kAlign * kAlign);
    s->device = cfg->mode != TDES_SERVE_HOST_TEST;
    hipError_t e = hipSuccess;
    if (cfg->mode == TDES_SERVE_PLAIN) {
        e = hipStreamCreateWithFlags(&s->plain_stream, hipStreamNonBlocking);
        for (int i = 0; i < kPlainEvents && e == hipSuccess; i++) {
            hipEvent_t ev;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) s->plain_events.push_back(ev);
        }
    } else {
        s->slots.resize(cfg->slots);
        const size_t n = cfg->max_batch_msgs;
        for (Slot &sl : s->slots) {
            if (!s->device) continue;
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
            sl.lay.layout(n);
            if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_stage, sl.lay.bytes, 0);
            if (e == hipSuccess) e = hipMalloc((void **)&sl.d_stage, sl.lay.bytes);
            if (e == hipSuccess) e = hipMalloc((void **)&sl.d_sched, n * TDES_DEVICE_SCHEDULE_BYTES);
            if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_tab, kTabBytes, 0);
            if (e == hipSuccess) e = hipMalloc((void **)&sl.d_tab, kTabBytes);
        }
    }
    if (e != hipSuccess) {
        free_device(s);
        delete s;
        return fail(TDES_ERR_DEVICE, hipGetErrorString(e));
    }
    *out = s;
    return TDES_OK;
}

void tdes_server_destroy(tdes_server *s) {
    if (s == nullptr) return;
    if (s->device) free_device(s);
    delete s;
}

tdes_status tdes_server_submit(tdes_server *s, const tdes_request *reqs, size_t n) {
    if (s == nullptr || (reqs == nullptr && n > 0)) return fail(TDES_ERR_ARG, "NULL server or requests");
    const double t = now_s();
    for (size_t i = 0; i < n; i++) {
        const tdes_request &r = reqs[i];
        s->st.submitted++;
        if (r.nbytes == 0) {  // nothing to compute and no result to release
            reject(s, r, t, TDES_OK);
            s->st.rejected--;
            s->st.completed++;
        } else if (r.nbytes % 8 != 0) reject(s, r, t, TDES_ERR_LENGTH);
        else if ((uintptr_t)r.d_in % 8 != 0) reject(s, r, t, TDES_ERR_ALIGN);
        else if (r.dir > 1 || (r.d_in == nullptr && r.nbytes > 0)) reject(s, r, t, TDES_ERR_ARG);
        else if (r.nbytes + round_up(r.nbytes) > s->budget || round_up(r.nbytes) > s->cfg.arena_bytes)
            reject(s, r, t, TDES_ERR_NOMEM);
        else s->queue.emplace_back(r, t);
    }
    s->st.queued = s->queue.size();
    return TDES_OK;
}

tdes_status tdes_server_progress(tdes_server *s, tdes_completion *out, size_t cap, size_t *n_out) {
    if (s == nullptr || n_out == nullptr || (out == nullptr && cap > 0))
        return fail(TDES_ERR_ARG, "NULL argument");
    tdes_status r = s->cfg.mode == TDES_SERVE_PLAIN ? progress_plain(s) : progress_batched(s);
    size_t k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = k;
    s->st.queued = s->queue.size();
    return r;
}

tdes_status tdes_server_release(tdes_server *s, void *d_out) {
    if (s == nullptr) return fail(TDES_ERR_ARG, "NULL server");
    const uint64_t off = (uint64_t)((uint8_t *)d_out - (uint8_t *)s->cfg.d_arena);
    auto it = s->live.find(off);
    if (d_out == nullptr || it == s->live.end()) return fail(TDES_ERR_ARG, "not a live result");
    s->arena.release(off, it->second);
    s->st.in_flight_bytes -= it->second;
    s->st.arena_used_bytes = s->arena.used();
    s->live.erase(it);
    s->st.released++;
    return TDES_OK;
}

tdes_status tdes_server_release_many(tdes_server *s, void *const *d_outs, size_t n,
                                     size_t *n_released) {
    if (s == nullptr || (d_outs == nullptr && n > 0)) return fail(TDES_ERR_ARG, "NULL argument");
    size_t k = 0;
    tdes_status st = TDES_OK;
    for (size_t i = 0; i < n; i++) {
        if (tdes_server_release(s, d_outs[i]) == TDES_OK) {
            k++;
        } else if (st == TDES_OK) {
            char msg[96];
            snprintf(msg, sizeof msg, "entry %zu is not a live result", i);
            st = fail(TDES_ERR_ARG, msg);
        }
    }
    if (n_released != nullptr) *n_released = k;
    return st;
}

tdes_status tdes_server_get_stats(const tdes_server *s, tdes_server_stats *out) {
    if (s == nullptr || out == nullptr) return fail(TDES_ERR_ARG, "NULL argument");
    *out = s->st;
    return TDES_OK;
}

}  // extern "C"
