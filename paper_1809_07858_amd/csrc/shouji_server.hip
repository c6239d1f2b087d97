// Serving form of the Shouji filter: a request server with continuous batching.
//
// A request is a set of pairs held in host memory: reads (2-bit packed,
// pair-major), for each pair the offset of its reference segment in a packed
// reference pool that stays resident in device memory, its length and its
// edit threshold.  The device memory budget is cut into batch slots of a fixed
// pair capacity.  A scheduler thread fills a free slot with the parts of the
// queued requests, in arrival order, as soon as one is free (a large request
// spreads over several batches, small ones share a batch) and enqueues the
// batch on the slot's own stream: host-to-device copies, relayout of the
// reads, extraction of the reference segments from the pool, the batched
// filter, copies back.  A completion thread waits for the batches in launch
// order and hands the results to the requests.  Copies and filtering of
// different batches overlap, and requests that arrive meanwhile go into the
// next free slot.  Each pair is filtered exactly as alone (the batched form
// guarantees it), so a request's results never depend on its batch mates.
//
// All device and pinned host memory is allocated in shouji_server_create.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/shouji.h"
#include "shouji_internal.h"

namespace shouji {

// Reads of a batch, read p in words in[woff[p] .. woff[p+1]) (rows of nw
// words, or packed reads of their own length) -> word-major out[nw][ld];
// words past a read's own are written as 0.  One thread per pair: its reads
// walk one contiguous run, and each of its writes is coalesced with the
// neighbouring pairs' writes of the same word.
__global__ __launch_bounds__(256) void reads_to_word_major_kernel(const uint32_t *__restrict__ in,
                                                                  const int32_t *__restrict__ woff, int64_t n,
                                                                  uint32_t *__restrict__ out, int nw, int64_t ld) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t a = woff[p];
    const int cnt = woff[p + 1] - a;
    for (int w = 0; w < nw; w++) out[(int64_t)w * ld + p] = w < cnt ? in[a + w] : 0u;
}

// Reference segment of pair p = pool bases [off[p], off[p] + len[p]), written
// word-major to out[nw][ld]; pool base b sits in bits 2(b%16).. of word b/16;
// words past the segment's end are written as 0.  A segment that does not lie
// inside the pool makes the pair invalid (len[p] = -1, so the filter gives it
// the sentinels).  One thread per pair, as above.
__global__ __launch_bounds__(256) void pool_gather_kernel(const uint32_t *__restrict__ pool, int64_t pool_bases,
                                                          const int64_t *__restrict__ off, int32_t *__restrict__ len,
                                                          int64_t n, uint32_t *__restrict__ out, int nw, int64_t ld) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t o = off[p];
    const int32_t m = len[p];
    const bool ok = o >= 0 && o <= pool_bases && m >= 0 && (int64_t)m <= pool_bases - o;
    if (!ok) len[p] = -1;
    // words holding bases of the segment (none for an invalid pair)
    const int nseg = ok ? (int)min((int64_t)nw, ((int64_t)m + kHalf - 1) / kHalf) : 0;
    const int64_t pool_words = (pool_bases + kHalf - 1) / kHalf;
    const int sh = (int)(o & 15) * 2;
    int64_t q = o >> 4;                              // pool word of the segment's first base
    uint32_t lo = nseg > 0 && q < pool_words ? pool[q] : 0u;
    for (int w = 0; w < nw; w++) {
        uint32_t v = 0u;
        if (w < nseg) {
            const uint32_t hi = (sh != 0 && q + 1 < pool_words) ? pool[q + 1] : 0u;
            v = sh ? (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) : lo;
            lo = sh ? hi : (q + 1 < pool_words ? pool[q + 1] : 0u);
            q++;
        }
        out[(int64_t)w * ld + p] = v;
    }
}

}  // namespace shouji

namespace {

using clk = std::chrono::steady_clock;
constexpr int kDefaultHostThreads = 8;

struct Request {
    shouji_request req;
    clk::time_point submitted, finished;
    int64_t pairs_left = 0;   // pairs whose results are not delivered yet
    bool done = false;
    int status = SHOUJI_OK;
};

struct Part {
    Request *r;
    int64_t first;   // first pair of the request in this part
    int64_t count;
    int64_t word_first = 0;   // packed request: word of the request's reads where pair `first` begins
};

// Words a packed request gives the read of a pair of length m.
inline int64_t packed_words(int32_t m, int max_len) {
    return (m >= 1 && m <= max_len) ? (m + shouji::kHalf - 1) / shouji::kHalf : 0;
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint32_t *h_reads = nullptr;  // pinned staging
    int64_t *h_off = nullptr;
    int32_t *h_len = nullptr, *h_E = nullptr;
    int32_t *h_woff = nullptr;    // word offset of each read in the read buffers (+ end)
    uint8_t *h_acc = nullptr;
    int16_t *h_pc = nullptr;
    uint32_t *d_reads_in = nullptr, *d_reads = nullptr, *d_refs = nullptr;
    int32_t *d_woff = nullptr;
    int64_t *d_off = nullptr;
    int32_t *d_len = nullptr, *d_E = nullptr;
    uint8_t *d_acc = nullptr;
    int16_t *d_pc = nullptr;
    void *d_ws = nullptr;
    int64_t ws_bytes = 0;
    std::vector<Part> parts;
    int64_t pairs = 0;
    int status = SHOUJI_OK;
    bool busy = false;
};

int64_t slot_device_bytes(int64_t B, int nw, int max_len) {
    return 3 * B * nw * 4 + B * (8 + 4 + 4 + 1 + 2) + (B + 1) * 4 + shouji_batched_workspace_bytes(B, max_len);
}

// Release a slot's streams, events and buffers.  Teardown is best-effort: a
// failed release leaves nothing the server still uses, so its status is not
// reported.
void free_slot(Slot &s) {
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.done) (void)hipEventDestroy(s.done);
    (void)hipHostFree(s.h_reads);
    (void)hipHostFree(s.h_off);
    (void)hipHostFree(s.h_len);
    (void)hipHostFree(s.h_E);
    (void)hipHostFree(s.h_woff);
    (void)hipHostFree(s.h_acc);
    (void)hipHostFree(s.h_pc);
    (void)hipFree(s.d_reads_in);
    (void)hipFree(s.d_woff);
    (void)hipFree(s.d_reads);
    (void)hipFree(s.d_refs);
    (void)hipFree(s.d_off);
    (void)hipFree(s.d_len);
    (void)hipFree(s.d_E);
    (void)hipFree(s.d_acc);
    (void)hipFree(s.d_pc);
    (void)hipFree(s.d_ws);
}

bool alloc_slot(Slot &s, int64_t B, int nw, int max_len) {
    s.ws_bytes = shouji_batched_workspace_bytes(B, max_len);
    return s.ws_bytes > 0 &&
           hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess &&
           hipHostMalloc((void **)&s.h_reads, (size_t)B * nw * 4, 0) == hipSuccess &&
           hipHostMalloc((void **)&s.h_off, (size_t)B * 8, 0) == hipSuccess &&
           hipHostMalloc((void **)&s.h_len, (size_t)B * 4, 0) == hipSuccess &&
           hipHostMalloc((void **)&s.h_E, (size_t)B * 4, 0) == hipSuccess &&
           hipHostMalloc((void **)&s.h_woff, (size_t)(B + 1) * 4, 0) == hipSuccess &&
           hipHostMalloc((void **)&s.h_acc, (size_t)B, 0) == hipSuccess &&
           hipHostMalloc((void **)&s.h_pc, (size_t)B * 2, 0) == hipSuccess &&
           hipMalloc((void **)&s.d_reads_in, (size_t)B * nw * 4) == hipSuccess &&
           hipMalloc((void **)&s.d_woff, (size_t)(B + 1) * 4) == hipSuccess &&
           hipMalloc((void **)&s.d_reads, (size_t)B * nw * 4) == hipSuccess &&
           hipMalloc((void **)&s.d_refs, (size_t)B * nw * 4) == hipSuccess &&
           hipMalloc((void **)&s.d_off, (size_t)B * 8) == hipSuccess &&
           hipMalloc((void **)&s.d_len, (size_t)B * 4) == hipSuccess &&
           hipMalloc((void **)&s.d_E, (size_t)B * 4) == hipSuccess &&
           hipMalloc((void **)&s.d_acc, (size_t)B) == hipSuccess &&
           hipMalloc((void **)&s.d_pc, (size_t)B * 2) == hipSuccess &&
           hipMalloc(&s.d_ws, (size_t)s.ws_bytes) == hipSuccess;
}

}  // namespace

struct shouji_server {
    shouji_server_config cfg{};
    int nw = 0;
    int device = 0;
    std::vector<std::unique_ptr<Slot>> slots;
    std::mutex mu;
    std::condition_variable cv;       // new parts, a free slot, a launched batch
    std::condition_variable cv_done;  // a request finished
    std::deque<Part> queue;           // parts not yet in a batch, arrival order
    std::deque<Slot *> inflight;      // launched batches, launch order
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread sched, reaper;
    int64_t batches = 0, pairs_done = 0, requests_done = 0, requests_deferred = 0;
};

namespace {

struct CopyJob {
    void *dst;
    const void *src;
    size_t bytes;
};

// Run host copies on up to `threads` threads (large copies are cut into
// chunks; a single thread does small batches, where thread start-up would
// cost more than it saves).
void run_copies(const std::vector<CopyJob> &jobs, int threads) {
    constexpr size_t kChunk = size_t(1) << 20;
    size_t total = 0;
    for (const CopyJob &j : jobs) total += j.bytes;
    if (threads <= 1 || total < 4 * kChunk) {
        for (const CopyJob &j : jobs) memcpy(j.dst, j.src, j.bytes);
        return;
    }
    std::vector<CopyJob> chunks;
    for (const CopyJob &j : jobs)
        for (size_t o = 0; o < j.bytes; o += kChunk)
            chunks.push_back(CopyJob{(char *)j.dst + o, (const char *)j.src + o, std::min(kChunk, j.bytes - o)});
    std::atomic<size_t> next{0};
    auto work = [&] {
        for (size_t i; (i = next.fetch_add(1)) < chunks.size();) memcpy(chunks[i].dst, chunks[i].src, chunks[i].bytes);
    };
    const int nt = (int)std::min<size_t>((size_t)threads, chunks.size());
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; t++) pool.emplace_back(work);
    work();
    for (std::thread &t : pool) t.join();
}

// A part whose request buffers are pinned and whose reads are packed or in
// rows of the server's width moves by DMA straight between the request and
// the device, unless it is small: each direct part costs its own copies (four
// in, two out), while consecutive staged parts share theirs.
constexpr int64_t kDirectMinPairs = 2048;
bool direct_part(const Part &pt, int nw) {
    const shouji_request &r = pt.r->req;
    return pt.count >= kDirectMinPairs && (r.flags & SHOUJI_REQUEST_PINNED) &&
           ((r.flags & SHOUJI_REQUEST_PACKED) || r.words_per_read == nw);
}

// Enqueue one batch on the slot's stream: parts in pageable memory are first
// copied into the slot's pinned staging buffers (consecutive such parts then
// move in one copy), pinned parts are copied directly.  The batch's reads lie
// back to back in the slot's read buffers, each part's where the previous one
// ends: a packed part's reads take their own word counts, rows nw words each;
// the word offset of every read goes to the device with them.  Runs without
// the server lock: the slot is marked busy and its requests stay alive until
// all their pairs are delivered.
int enqueue_batch(shouji_server *S, Slot &s) {
    const int nw = S->nw;
    const int max_len = S->cfg.max_len;
    const size_t np = s.parts.size();
    std::vector<int64_t> wpos(np + 1);   // first word of each part in the read buffers
    int64_t at = 0, wcur = 0;
    for (size_t i = 0; i < np; i++) {
        const Part &pt = s.parts[i];
        const shouji_request &r = pt.r->req;
        wpos[i] = wcur;
        int32_t *wo = s.h_woff + at;
        if (r.flags & SHOUJI_REQUEST_PACKED) {
            const int32_t *len = r.lengths + pt.first;
            for (int64_t k = 0; k < pt.count; k++) {
                wo[k] = (int32_t)wcur;
                wcur += packed_words(len[k], max_len);
            }
        } else {
            for (int64_t k = 0; k < pt.count; k++) wo[k] = (int32_t)(wcur + k * nw);
            wcur += pt.count * nw;
        }
        at += pt.count;
    }
    wpos[np] = wcur;
    s.h_woff[at] = (int32_t)wcur;

    std::vector<CopyJob> jobs;
    at = 0;
    for (size_t i = 0; i < np; i++) {
        const Part &pt = s.parts[i];
        const shouji_request &r = pt.r->req;
        const int64_t c = pt.count, f = pt.first;
        if (!direct_part(pt, nw)) {
            uint32_t *dst = s.h_reads + wpos[i];
            if (r.flags & SHOUJI_REQUEST_PACKED) {
                jobs.push_back(CopyJob{dst, r.reads + pt.word_first, (size_t)(wpos[i + 1] - wpos[i]) * 4});
            } else if (r.words_per_read == nw) {
                jobs.push_back(CopyJob{dst, r.reads + f * nw, (size_t)c * nw * 4});
            } else {
                const int cw = std::min(nw, (int)r.words_per_read);
                for (int64_t k = 0; k < c; k++) {
                    uint32_t *row = dst + k * nw;
                    memcpy(row, r.reads + (f + k) * r.words_per_read, (size_t)cw * 4);
                    for (int w = cw; w < nw; w++) row[w] = 0u;
                }
            }
            jobs.push_back(CopyJob{s.h_off + at, r.ref_offsets + f, (size_t)c * 8});
            jobs.push_back(CopyJob{s.h_len + at, r.lengths + f, (size_t)c * 4});
            jobs.push_back(CopyJob{s.h_E + at, r.E + f, (size_t)c * 4});
        }
        at += c;
    }
    run_copies(jobs, S->cfg.host_threads > 0 ? S->cfg.host_threads : kDefaultHostThreads);

    const int64_t n = s.pairs;
    hipStream_t st = s.stream;
    bool good = true;
    auto copy = [&](void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
        if (good && bytes) good = hipMemcpyAsync(dst, src, bytes, kind, st) == hipSuccess;
    };
    // host -> device
    int64_t run = -1, wrun = 0;   // first pair and first word of the current run of staged parts
    auto flush_in = [&](int64_t e, int64_t we) {
        if (run < 0) return;
        const int64_t c = e - run;
        copy(s.d_reads_in + wrun, s.h_reads + wrun, (size_t)(we - wrun) * 4, hipMemcpyHostToDevice);
        copy(s.d_off + run, s.h_off + run, (size_t)c * 8, hipMemcpyHostToDevice);
        copy(s.d_len + run, s.h_len + run, (size_t)c * 4, hipMemcpyHostToDevice);
        copy(s.d_E + run, s.h_E + run, (size_t)c * 4, hipMemcpyHostToDevice);
        run = -1;
    };
    at = 0;
    for (size_t i = 0; i < np; i++) {
        const Part &pt = s.parts[i];
        const shouji_request &r = pt.r->req;
        const int64_t c = pt.count, f = pt.first;
        if (direct_part(pt, nw)) {
            flush_in(at, wpos[i]);
            const uint32_t *src = (r.flags & SHOUJI_REQUEST_PACKED) ? r.reads + pt.word_first : r.reads + f * nw;
            copy(s.d_reads_in + wpos[i], src, (size_t)(wpos[i + 1] - wpos[i]) * 4, hipMemcpyHostToDevice);
            copy(s.d_off + at, r.ref_offsets + f, (size_t)c * 8, hipMemcpyHostToDevice);
            copy(s.d_len + at, r.lengths + f, (size_t)c * 4, hipMemcpyHostToDevice);
            copy(s.d_E + at, r.E + f, (size_t)c * 4, hipMemcpyHostToDevice);
        } else if (run < 0) {
            run = at;
            wrun = wpos[i];
        }
        at += c;
    }
    flush_in(at, wcur);
    copy(s.d_woff, s.h_woff, (size_t)(n + 1) * 4, hipMemcpyHostToDevice);
    int rc = good ? SHOUJI_OK : SHOUJI_ERR_DEVICE;
    if (rc == SHOUJI_OK) {
        const unsigned blocks = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(shouji::reads_to_word_major_kernel, dim3(blocks), dim3(256), 0, st, s.d_reads_in,
                           s.d_woff, n, s.d_reads, nw, n);
        hipLaunchKernelGGL(shouji::pool_gather_kernel, dim3(blocks), dim3(256), 0, st, S->cfg.pool,
                           S->cfg.pool_bases, s.d_off, s.d_len, n, s.d_refs, nw, n);
        rc = hipGetLastError() == hipSuccess ? SHOUJI_OK : SHOUJI_ERR_DEVICE;
    }
    if (rc == SHOUJI_OK)
        rc = shouji_filter_batched(s.d_reads, s.d_refs, s.d_len, s.d_E, s.d_acc, s.d_pc, n, S->cfg.max_len, n,
                                   s.d_ws, s.ws_bytes, nullptr, st);
    if (rc == SHOUJI_OK) {
        // device -> host: staged runs into the slot, pinned parts in place
        auto flush_out = [&](int64_t e) {
            if (run < 0) return;
            copy(s.h_acc + run, s.d_acc + run, (size_t)(e - run), hipMemcpyDeviceToHost);
            copy(s.h_pc + run, s.d_pc + run, (size_t)(e - run) * 2, hipMemcpyDeviceToHost);
            run = -1;
        };
        at = 0;
        for (const Part &pt : s.parts) {
            const shouji_request &r = pt.r->req;
            const int64_t c = pt.count, f = pt.first;
            if (direct_part(pt, nw)) {
                flush_out(at);
                copy(r.out_accept + f, s.d_acc + at, (size_t)c, hipMemcpyDeviceToHost);
                if (r.out_popcount) copy(r.out_popcount + f, s.d_pc + at, (size_t)c * 2, hipMemcpyDeviceToHost);
            } else if (run < 0) {
                run = at;
            }
            at += c;
        }
        flush_out(at);
        if (!good) rc = SHOUJI_ERR_DEVICE;
    }
    if (hipEventRecord(s.done, st) != hipSuccess && rc == SHOUJI_OK) rc = SHOUJI_ERR_DEVICE;
    return rc;
}

void scheduler_loop(shouji_server *S) {
    // on the server's device, or every batch this thread would launch fails
    const bool on_device = hipSetDevice(S->device) == hipSuccess;
    const int64_t B = S->cfg.max_batch_pairs;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        if (S->stop) break;
        Slot *s = nullptr;
        for (auto &q : S->slots)
            if (!q->busy) { s = q.get(); break; }
        if (!s || S->queue.empty()) {
            S->cv.wait(lk);
            continue;
        }
        // with a batch in flight the device is busy anyway: a part-filled batch
        // may wait for more requests, until the oldest queued one is due
        if (S->cfg.fill_wait_us > 0 && !S->inflight.empty()) {
            int64_t queued = 0;
            for (const Part &q : S->queue)
                if ((queued += q.count) >= B) break;
            const clk::time_point due = S->queue.front().r->submitted + std::chrono::microseconds(S->cfg.fill_wait_us);
            if (queued < B && clk::now() < due) {
                S->cv.wait_until(lk, due);
                continue;
            }
        }
        // fill the slot with queued parts in arrival order
        s->parts.clear();
        s->pairs = 0;
        while (!S->queue.empty() && s->pairs < B) {
            Part &q = S->queue.front();
            const int64_t take = std::min(q.count, B - s->pairs);
            s->parts.push_back(Part{q.r, q.first, take, q.word_first});
            s->pairs += take;
            if (take < q.count && (q.r->req.flags & SHOUJI_REQUEST_PACKED)) {
                // the rest of a packed request begins after the words of these reads
                const int32_t *len = q.r->req.lengths + q.first;
                int64_t words = 0;
                for (int64_t k = 0; k < take; k++) words += packed_words(len[k], S->cfg.max_len);
                q.word_first += words;
            }
            q.first += take;
            q.count -= take;
            if (q.count == 0) S->queue.pop_front();
        }
        s->busy = true;
        S->batches++;
        lk.unlock();
        s->status = on_device ? enqueue_batch(S, *s) : SHOUJI_ERR_DEVICE;
        lk.lock();
        S->inflight.push_back(s);
        S->cv.notify_all();
    }
}

void reaper_loop(shouji_server *S) {
    const bool on_device = hipSetDevice(S->device) == hipSuccess;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        if (S->inflight.empty()) {
            if (S->stop) break;
            S->cv.wait(lk);
            continue;
        }
        Slot &s = *S->inflight.front();
        lk.unlock();
        if ((!on_device || hipEventSynchronize(s.done) != hipSuccess) && s.status == SHOUJI_OK)
            s.status = SHOUJI_ERR_DEVICE;
        int64_t at = 0;
        for (const Part &pt : s.parts) {
            shouji_request &r = pt.r->req;
            if (!direct_part(pt, S->nw)) {
                memcpy(r.out_accept + pt.first, s.h_acc + at, (size_t)pt.count);
                if (r.out_popcount) memcpy(r.out_popcount + pt.first, s.h_pc + at, (size_t)pt.count * 2);
            }
            at += pt.count;
        }
        const auto now = clk::now();
        lk.lock();
        for (const Part &pt : s.parts) {
            Request &R = *pt.r;
            if (s.status != SHOUJI_OK) R.status = s.status;
            R.pairs_left -= pt.count;
            if (R.pairs_left == 0) {
                R.done = true;
                R.finished = now;
                S->requests_done++;
            }
        }
        S->pairs_done += s.pairs;
        S->inflight.pop_front();
        s.parts.clear();
        s.busy = false;
        S->cv.notify_all();
        S->cv_done.notify_all();
    }
}

}  // namespace

extern "C" int64_t shouji_server_slot_bytes(int64_t max_batch_pairs, int32_t max_len) {
    using shouji::set_error;
    if (max_batch_pairs <= 0) return set_error(SHOUJI_ERR_ARG, "shouji_server_slot_bytes: max_batch_pairs must be positive");
    if (max_len <= 0 || max_len > SHOUJI_MAX_LEN)
        return set_error(SHOUJI_ERR_RANGE, "shouji_server_slot_bytes: max_len %d outside 1..%d", max_len, SHOUJI_MAX_LEN);
    shouji::clear_error();
    return slot_device_bytes(max_batch_pairs, (max_len + shouji::kHalf - 1) / shouji::kHalf, max_len);
}

extern "C" int shouji_server_create(const shouji_server_config *cfg, shouji_server **out) {
    using shouji::set_error;
    if (!cfg || !out) return set_error(SHOUJI_ERR_NULL, "shouji_server_create: config and out are required");
    *out = nullptr;
    if (!cfg->pool || cfg->pool_bases <= 0)
        return set_error(SHOUJI_ERR_ARG, "shouji_server_create: a non-empty reference pool is required");
    if (cfg->max_len <= 0 || cfg->max_len > SHOUJI_MAX_LEN)
        return set_error(SHOUJI_ERR_RANGE, "shouji_server_create: max_len %d outside 1..%d", cfg->max_len,
                         SHOUJI_MAX_LEN);
    if (cfg->max_batch_pairs <= 0 || cfg->slots <= 0 || cfg->memory_budget < 0)
        return set_error(SHOUJI_ERR_ARG, "shouji_server_create: max_batch_pairs and slots must be positive");
    if (cfg->fill_wait_us < 0 || cfg->fill_wait_us > 1000000)
        return set_error(SHOUJI_ERR_RANGE, "shouji_server_create: fill_wait_us %d outside 0..1000000",
                         cfg->fill_wait_us);
    std::unique_ptr<shouji_server> S(new shouji_server());
    S->cfg = *cfg;
    S->nw = (cfg->max_len + shouji::kHalf - 1) / shouji::kHalf;
    if (cfg->max_batch_pairs > INT32_MAX / S->nw)
        return set_error(SHOUJI_ERR_RANGE, "shouji_server_create: max_batch_pairs %lld too large (read words of a "
                         "batch are indexed in 32 bits)", (long long)cfg->max_batch_pairs);
    if (hipGetDevice(&S->device) != hipSuccess)
        return set_error(SHOUJI_ERR_DEVICE, "shouji_server_create: no current HIP device");
    const int64_t per = slot_device_bytes(cfg->max_batch_pairs, S->nw, cfg->max_len);
    int64_t nslots = cfg->slots;
    if (cfg->memory_budget > 0) nslots = std::min<int64_t>(nslots, cfg->memory_budget / per);
    if (nslots < 1)
        return set_error(SHOUJI_ERR_NOMEM, "shouji_server_create: memory budget %lld below one batch slot (%lld bytes)",
                         (long long)cfg->memory_budget, (long long)per);
    for (int64_t i = 0; i < nslots; i++) {
        std::unique_ptr<Slot> s(new Slot());
        if (!alloc_slot(*s, cfg->max_batch_pairs, S->nw, cfg->max_len)) {
            free_slot(*s);
            for (auto &q : S->slots) free_slot(*q);
            return set_error(SHOUJI_ERR_NOMEM, "shouji_server_create: cannot allocate batch slot %lld", (long long)i);
        }
        S->slots.push_back(std::move(s));
    }
    S->sched = std::thread(scheduler_loop, S.get());
    S->reaper = std::thread(reaper_loop, S.get());
    *out = S.release();
    return shouji::clear_error();
}

extern "C" int shouji_server_submit(shouji_server *S, const shouji_request *r, uint64_t *ticket) {
    using shouji::set_error;
    if (!S || !r || !ticket)
        return set_error(SHOUJI_ERR_NULL, "shouji_server_submit: server, request and ticket are required");
    if (r->n_pairs < 0) return set_error(SHOUJI_ERR_ARG, "shouji_server_submit: n_pairs < 0");
    if (r->flags & ~(SHOUJI_REQUEST_PINNED | SHOUJI_REQUEST_PACKED))
        return set_error(SHOUJI_ERR_ARG, "shouji_server_submit: unknown flags 0x%x", r->flags);
    if (r->n_pairs > 0) {
        if (!r->reads || !r->ref_offsets || !r->lengths || !r->E || !r->out_accept)
            return set_error(SHOUJI_ERR_NULL, "shouji_server_submit: request buffer missing");
        if (!(r->flags & SHOUJI_REQUEST_PACKED) && r->words_per_read <= 0)
            return set_error(SHOUJI_ERR_ARG, "shouji_server_submit: words_per_read must be positive");
        if (r->flags & SHOUJI_REQUEST_PACKED) {
            // the words the lengths say the buffer holds, before anything is queued
            const int ml = S->cfg.max_len;
            int64_t need = 0;
            for (int64_t p = 0; p < r->n_pairs; p++) {
                const int32_t m = r->lengths[p];
                if (m >= 1 && m <= ml) need += (m + SHOUJI_BASES_PER_WORD - 1) / SHOUJI_BASES_PER_WORD;
            }
            if (r->read_words < need)
                return set_error(SHOUJI_ERR_ARG,
                                 "shouji_server_submit: packed reads hold %lld words, the lengths need %lld",
                                 (long long)r->read_words, (long long)need);
        }
    }
    std::unique_ptr<Request> R(new Request());
    R->req = *r;
    const int64_t B = S->cfg.max_batch_pairs;
    std::lock_guard<std::mutex> g(S->mu);
    R->submitted = clk::now();
    const uint64_t t = S->next_ticket++;
    R->pairs_left = r->n_pairs;
    if (r->n_pairs == 0) {
        R->done = true;
        R->finished = R->submitted;
        S->requests_done++;
    }
    if (r->n_pairs > 0 && (!S->queue.empty() || std::all_of(S->slots.begin(), S->slots.end(),
                                                            [](const std::unique_ptr<Slot> &q) { return q->busy; })))
        S->requests_deferred++;
    if (r->flags & SHOUJI_REQUEST_PACKED) {
        // one part: the scheduler cuts it and follows the word offset of each cut
        if (r->n_pairs > 0) S->queue.push_back(Part{R.get(), 0, r->n_pairs, 0});
    } else {
        for (int64_t f = 0; f < r->n_pairs; f += B) S->queue.push_back(Part{R.get(), f, std::min(B, r->n_pairs - f)});
    }
    S->reqs[t] = std::move(R);
    *ticket = t;
    S->cv.notify_all();
    return shouji::clear_error();
}

extern "C" int shouji_server_poll(shouji_server *S, uint64_t ticket, int32_t *done) {
    using shouji::set_error;
    if (!S || !done) return set_error(SHOUJI_ERR_NULL, "shouji_server_poll: server and done are required");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end())
        return set_error(SHOUJI_ERR_ARG, "shouji_server_poll: unknown ticket %llu", (unsigned long long)ticket);
    *done = it->second->done ? 1 : 0;
    return shouji::clear_error();
}

extern "C" int shouji_server_wait(shouji_server *S, uint64_t ticket, double *latency_ms) {
    using shouji::set_error;
    if (!S) return set_error(SHOUJI_ERR_NULL, "shouji_server_wait: server is required");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end())
        return set_error(SHOUJI_ERR_ARG, "shouji_server_wait: unknown ticket %llu", (unsigned long long)ticket);
    Request *R = it->second.get();
    S->cv_done.wait(lk, [R] { return R->done; });
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(R->finished - R->submitted).count();
    const int st = R->status;
    S->reqs.erase(it);
    if (st != SHOUJI_OK)
        return set_error(st, "shouji_server_wait: a batch of request %llu failed", (unsigned long long)ticket);
    return shouji::clear_error();
}

extern "C" int shouji_server_get_stats(shouji_server *S, shouji_server_stats *st) {
    using shouji::set_error;
    if (!S || !st) return set_error(SHOUJI_ERR_NULL, "shouji_server_get_stats: server and stats are required");
    std::lock_guard<std::mutex> g(S->mu);
    st->slots = (int32_t)S->slots.size();
    st->batches = S->batches;
    st->pairs_done = S->pairs_done;
    st->requests_done = S->requests_done;
    st->requests_deferred = S->requests_deferred;
    int64_t q = 0;
    for (const Part &p : S->queue) q += p.count;
    st->queued_pairs = q;
    return shouji::clear_error();
}

extern "C" int shouji_server_destroy(shouji_server *S) {
    if (!S) return SHOUJI_OK;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [S] {
            return S->queue.empty() && S->inflight.empty() &&
                   std::none_of(S->slots.begin(), S->slots.end(),
                                [](const std::unique_ptr<Slot> &s) { return s->busy; });
        });
        S->stop = true;
        S->cv.notify_all();
    }
    S->sched.join();
    S->reaper.join();
    (void)hipSetDevice(S->device);   // best-effort: the slots' buffers belong to it
    for (auto &s : S->slots) free_slot(*s);
    delete S;
    return SHOUJI_OK;
}
