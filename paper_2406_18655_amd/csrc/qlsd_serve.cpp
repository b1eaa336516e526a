// Continuous-batching decode service (include/qlsd_serve.h): lanes of decoders on their own
// streams, a scheduler thread that forms batches from arrived requests whenever a lane is free,
// and per-request latency bookkeeping.  All decoding runs through qlsd_decode.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/qlsd_serve.h"
#include "qlsd_internal.h"

namespace {

struct Request {
    const uint8_t *syn;
    uint8_t *out;
    uint64_t tag;
    double arrival_us;
    bool dev;  // syn and out are device memory (no host staging)
};

struct Lane {
    qlsd_decoder dec = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint8_t *d_syn = nullptr, *d_corr = nullptr, *d_info = nullptr;
    uint8_t *h_syn = nullptr, *h_corr = nullptr, *h_info = nullptr;
    bool busy = false;
    bool dev_batch = false;   // the batch in flight holds device requests
    double idle_since = 0.0;  // server clock when the lane last finished a batch
    size_t bytes = 0;         // device memory charged to the budget
    std::vector<Request> batch;
};

struct Code {
    int m = 0, n = 0, batch_shots = 0, max_lanes = 1;
    qlsd_code code = nullptr;
    qlsd_params params{};
    std::vector<double> priors;
    qlsd_net net = nullptr;
    std::vector<std::unique_ptr<Lane>> lanes;
    std::deque<Request> pending;  // arrival order
    std::atomic<int> n_lanes{0}, created{0}, retired{0};  // read by qlsd_server_lanes
};

}  // namespace

struct qlsd_server_s {
    size_t budget = 0, used = 0;
    double retire_us = 20000.0;  // an extra lane idle this long is freed
    std::vector<Code *> codes;
    std::mutex mu;                      // pending queues and completions
    std::condition_variable cv;
    std::vector<qlsd_completion> done;  // not yet drained by the caller
    int64_t completed = 0;
    std::atomic<bool> stop{false}, started{false}, failed{false};
    std::thread worker;
    std::chrono::steady_clock::time_point epoch;
    char error[256] = "";  // first asynchronous (device or decode) failure; written under mu
};

namespace {

// Records the first failure (under the lock qlsd_server_wait reads it with), stops the
// scheduler and wakes waiters.
void fail_server(qlsd_server_s *s, const char *fmt, const char *detail) {
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (!s->error[0]) snprintf(s->error, sizeof(s->error), fmt, detail);
        s->failed = true;
    }
    s->stop = true;
    s->cv.notify_all();
}

double now_us(const qlsd_server_s *s) {
    if (!s->started.load()) return 0.0;
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - s->epoch).count();
}

void free_lane(Lane &l) {
    if (l.stream) hipStreamSynchronize(l.stream);
    if (l.dec) qlsd_decoder_destroy(l.dec);
    if (l.done) hipEventDestroy(l.done);
    if (l.stream) hipStreamDestroy(l.stream);
    hipFree(l.d_syn);
    hipFree(l.d_corr);
    hipFree(l.d_info);
    hipHostFree(l.h_syn);
    hipHostFree(l.h_corr);
    hipHostFree(l.h_info);
    l = Lane();
}

// A new lane of code c if its device memory fits the remaining budget (decoder workspace, the
// refinement workspace of an attached net, one batch of buffers); nullptr otherwise.  Runs at
// registration and in the scheduler thread, which admits lanes as memory frees.
std::unique_ptr<Lane> make_lane(qlsd_server_s *s, Code &c, qlsd_status *st_out) {
    auto l = std::unique_ptr<Lane>(new (std::nothrow) Lane());
    *st_out = QLSD_E_NOMEM;
    if (!l) return nullptr;
    qlsd_status st = qlsd_decoder_create(c.code, &c.params, c.priors.data(), c.batch_shots, &l->dec);
    if (st == QLSD_OK && c.net) st = qlsd_decoder_set_net(l->dec, c.net);
    if (st != QLSD_OK) {
        if (l->dec) qlsd_decoder_destroy(l->dec);
        *st_out = st;
        return nullptr;
    }
    const size_t bufs = (size_t)c.batch_shots * (c.m + c.n + sizeof(qlsd_shot_info));
    l->bytes = qlsd::decoder_device_bytes(l->dec) + bufs;
    if (s->used + l->bytes > s->budget) {
        qlsd_decoder_destroy(l->dec);
        qlsd::set_last_error("device budget too small for another lane of this code");
        return nullptr;
    }
    const int bs = c.batch_shots;
    const bool ok = hipStreamCreateWithFlags(&l->stream, hipStreamNonBlocking) == hipSuccess &&
                    hipEventCreateWithFlags(&l->done, hipEventDisableTiming) == hipSuccess &&
                    hipMalloc((void **)&l->d_syn, (size_t)bs * c.m) == hipSuccess &&
                    hipMalloc((void **)&l->d_corr, (size_t)bs * c.n) == hipSuccess &&
                    hipMalloc((void **)&l->d_info, (size_t)bs * sizeof(qlsd_shot_info)) == hipSuccess &&
                    hipHostMalloc((void **)&l->h_syn, (size_t)bs * c.m, 0) == hipSuccess &&
                    hipHostMalloc((void **)&l->h_corr, (size_t)bs * c.n, 0) == hipSuccess &&
                    hipHostMalloc((void **)&l->h_info, (size_t)bs * sizeof(qlsd_shot_info), 0) == hipSuccess;
    if (!ok) {
        free_lane(*l);
        qlsd::set_last_error("lane allocation failed");
        return nullptr;
    }
    l->batch.reserve(bs);
    l->idle_since = now_us(s);
    s->used += l->bytes;
    c.created++;
    *st_out = QLSD_OK;
    return l;
}

// Launches one batch on a free lane from the requests of code c that have arrived.  A lane
// starts while another lane of the same code is still running only if at least half a batch has
// arrived: at light load one batch per code is in flight (fewer small decodes contending for
// the device), under backlog every lane works.
// Requests arrived by time t (the pending queue is in arrival order).
size_t arrived(const Code &c, double t) {
    const auto end = std::upper_bound(c.pending.begin(), c.pending.end(), t,
                                      [](double v, const Request &r) { return v < r.arrival_us; });
    return (size_t)(end - c.pending.begin());
}

// Device requests: consecutive requests whose rows follow each other in the caller's arrays
// form one run, moved with one device-to-device copy (a batch that is a single run is decoded
// in place, with no copy at all).
template <class F>
void for_runs(const std::vector<Request> &batch, size_t row_in, size_t row_out, F &&f) {
    size_t b = 0;
    while (b < batch.size()) {
        size_t e = b + 1;
        while (e < batch.size() && batch[e].syn == batch[b].syn + (e - b) * row_in &&
               batch[e].out == batch[b].out + (e - b) * row_out)
            e++;
        f(b, e);
        b = e;
    }
}

bool launch_batch(qlsd_server_s *s, Code &c, Lane &l, double t, int busy_lanes) {
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (busy_lanes > 0 && arrived(c, t) * 2 < (size_t)c.batch_shots) return false;
        // one batch carries requests of one kind (host-staged or device-resident)
        const bool dev = !c.pending.empty() && c.pending.front().dev;
        while (!c.pending.empty() && (int)l.batch.size() < c.batch_shots && c.pending.front().arrival_us <= t &&
               c.pending.front().dev == dev) {
            l.batch.push_back(c.pending.front());
            c.pending.pop_front();
        }
        l.dev_batch = dev;
    }
    const int B = (int)l.batch.size();
    if (B == 0) return false;
    bool ok = true;
    if (l.dev_batch) {
        int runs = 0;
        for_runs(l.batch, c.m, c.n, [&](size_t, size_t) { runs++; });
        const uint8_t *syn = l.d_syn;
        uint8_t *out = l.d_corr;
        if (runs == 1) {
            syn = l.batch[0].syn;
            out = l.batch[0].out;
        } else {
            for_runs(l.batch, c.m, c.n, [&](size_t b, size_t e) {
                ok = ok && hipMemcpyAsync(l.d_syn + b * c.m, l.batch[b].syn, (e - b) * c.m, hipMemcpyDeviceToDevice,
                                          l.stream) == hipSuccess;
            });
        }
        if (ok && qlsd_decode(l.dec, syn, B, out, (qlsd_shot_info *)l.d_info, l.stream) != QLSD_OK) {
            fail_server(s, "decode failed: %s", qlsd_last_error());
            return false;
        }
        if (runs > 1)
            for_runs(l.batch, c.m, c.n, [&](size_t b, size_t e) {
                ok = ok && hipMemcpyAsync(l.batch[b].out, l.d_corr + b * c.n, (e - b) * c.n, hipMemcpyDeviceToDevice,
                                          l.stream) == hipSuccess;
            });
    } else {
        for (int b = 0; b < B; b++) memcpy(l.h_syn + (size_t)b * c.m, l.batch[b].syn, c.m);
        ok = hipMemcpyAsync(l.d_syn, l.h_syn, (size_t)B * c.m, hipMemcpyHostToDevice, l.stream) == hipSuccess;
        if (ok && qlsd_decode(l.dec, l.d_syn, B, l.d_corr, (qlsd_shot_info *)l.d_info, l.stream) != QLSD_OK) {
            fail_server(s, "decode failed: %s", qlsd_last_error());
            return false;  // the batch's requests are not completed; waiters see the error
        }
        ok = ok && hipMemcpyAsync(l.h_corr, l.d_corr, (size_t)B * c.n, hipMemcpyDeviceToHost, l.stream) == hipSuccess;
    }
    ok = ok &&
         hipMemcpyAsync(l.h_info, l.d_info, (size_t)B * sizeof(qlsd_shot_info), hipMemcpyDeviceToHost, l.stream) ==
             hipSuccess &&
         hipEventRecord(l.done, l.stream) == hipSuccess;
    if (!ok) {
        fail_server(s, "%s", "enqueueing a batch failed");
        return false;
    }
    l.busy = true;
    return true;
}

void finish_batch(qlsd_server_s *s, int code_id, Code &c, Lane &l) {
    const double t = now_us(s);
    const int B = (int)l.batch.size();
    std::vector<qlsd_completion> recs(B);
    for (int b = 0; b < B; b++) {
        if (!l.dev_batch) memcpy(l.batch[b].out, l.h_corr + (size_t)b * c.n, c.n);
        qlsd_completion &r = recs[b];
        memset(&r, 0, sizeof(r));
        r.tag = l.batch[b].tag;
        r.code_id = code_id;
        r.status = ((const qlsd_shot_info *)l.h_info)[b].status;
        r.arrival_us = l.batch[b].arrival_us;
        r.done_us = t;
        r.batch_size = B;
    }
    l.batch.clear();
    l.busy = false;
    l.idle_since = t;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->done.insert(s->done.end(), recs.begin(), recs.end());
        s->completed += B;
    }
    s->cv.notify_all();
}

void scheduler(qlsd_server_s *s) {
    while (true) {
        bool progress = false, any_busy = false;
        const double t = now_us(s);
        // retire extra lanes that have idled: their memory admits lanes of codes with a backlog
        for (Code *cp : s->codes) {
            Code &c = *cp;
            for (size_t k = c.lanes.size(); k-- > 1;) {
                Lane &l = *c.lanes[k];
                if (!l.busy && t - l.idle_since > s->retire_us) {
                    s->used -= l.bytes;
                    free_lane(l);
                    c.lanes.erase(c.lanes.begin() + (long)k);
                    c.retired++;
                    c.n_lanes = (int)c.lanes.size();
                    progress = true;
                }
            }
        }
        for (size_t ci = 0; ci < s->codes.size(); ci++) {
            Code &c = *s->codes[ci];
            int busy = 0;
            for (auto &lp : c.lanes) busy += lp->busy ? 1 : 0;
            for (auto &lp : c.lanes) {
                Lane &l = *lp;
                if (l.busy) {
                    const hipError_t q = hipEventQuery(l.done);
                    if (q == hipSuccess) {
                        finish_batch(s, (int)ci, c, l);
                        busy--;
                        progress = true;
                    } else if (q != hipErrorNotReady) {
                        fail_server(s, "device failure: %s", hipGetErrorString(q));
                        // let in-flight work drain before the thread ends
                        for (Code *cc : s->codes)
                            for (auto &ll : cc->lanes)
                                if (ll->busy) hipStreamSynchronize(ll->stream);
                        return;
                    }
                }
                if (!l.busy && !s->failed.load() && launch_batch(s, c, l, t, busy)) {
                    busy++;
                    progress = true;
                }
                any_busy |= l.busy;
            }
            // every lane busy and a backlog of at least half a batch: admit one more lane if the
            // budget has room for it now
            if (!s->failed.load() && busy == (int)c.lanes.size() && (int)c.lanes.size() < c.max_lanes) {
                size_t backlog;
                {
                    std::lock_guard<std::mutex> g(s->mu);
                    backlog = arrived(c, t);
                }
                if (backlog * 2 >= (size_t)c.batch_shots) {
                    qlsd_status st;
                    auto nl = make_lane(s, c, &st);
                    if (nl) {
                        c.lanes.push_back(std::move(nl));
                        c.n_lanes = (int)c.lanes.size();
                        progress = true;
                    }
                }
            }
        }
        if (s->stop.load() && !any_busy) return;
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(any_busy ? 5 : 20));
    }
}

// Synchronous errors of an API call: reported to that caller only (the server stays usable).
qlsd_status serr(qlsd_server_s *, qlsd_status st, const char *msg) {
    qlsd::set_last_error("%s", msg);
    return st;
}

}  // namespace

extern "C" {

qlsd_status qlsd_server_create(size_t device_budget_bytes, qlsd_server *out) {
    if (!out) return serr(nullptr, QLSD_E_INVALID, "out is NULL");
    qlsd_server s = new (std::nothrow) qlsd_server_s();
    if (!s) return serr(nullptr, QLSD_E_NOMEM, "host allocation failed");
    s->budget = device_budget_bytes;
    *out = s;
    return QLSD_OK;
}

qlsd_status qlsd_server_add_code(qlsd_server s, qlsd_code code, const qlsd_params *params, const double *priors,
                                 int32_t batch_shots, int32_t max_lanes, int32_t *code_id, int32_t *lanes_out) {
    if (!s || !code || !params || !priors || !code_id) return serr(s, QLSD_E_INVALID, "NULL argument");
    if (s->started.load()) return serr(s, QLSD_E_INVALID, "codes must be added before qlsd_server_start");
    if (batch_shots < 1 || max_lanes < 1) return serr(s, QLSD_E_BATCH, "batch_shots and max_lanes must be >= 1");
    Code *c = new (std::nothrow) Code();
    if (!c) return serr(s, QLSD_E_NOMEM, "host allocation failed");
    c->m = qlsd::code_rows(code);
    c->n = qlsd::code_cols(code);
    c->batch_shots = batch_shots;
    c->max_lanes = max_lanes;
    c->code = code;
    c->params = *params;
    c->priors.assign(priors, priors + c->n);
    qlsd_status st;
    auto l = make_lane(s, *c, &st);
    if (!l) {
        delete c;
        return st == QLSD_OK ? QLSD_E_NOMEM : st;
    }
    c->lanes.push_back(std::move(l));
    c->n_lanes = 1;
    *code_id = (int32_t)s->codes.size();
    if (lanes_out) *lanes_out = (int32_t)c->lanes.size();
    s->codes.push_back(c);
    return QLSD_OK;
}

qlsd_status qlsd_server_set_net(qlsd_server s, int32_t code_id, qlsd_net net) {
    if (!s || code_id < 0 || code_id >= (int32_t)s->codes.size()) return serr(s, QLSD_E_INVALID, "bad server or code id");
    if (s->started.load()) return serr(s, QLSD_E_INVALID, "nets must be attached before qlsd_server_start");
    Code &c = *s->codes[code_id];
    // a net on a large graph gives every lane's decoder a feature workspace: charge it to the budget
    for (auto &lp : c.lanes) {
        Lane &l = *lp;
        const size_t before = qlsd::decoder_device_bytes(l.dec);
        const qlsd_status st = qlsd_decoder_set_net(l.dec, net);
        if (st != QLSD_OK) return st;
        const size_t after = qlsd::decoder_device_bytes(l.dec);
        if (after > before && s->used + (after - before) > s->budget) {
            qlsd_decoder_set_net(l.dec, nullptr);
            return serr(s, QLSD_E_NOMEM, "device budget too small for the refinement workspace of every lane");
        }
        s->used = s->used + after - before;
        l.bytes = l.bytes + after - before;
    }
    c.net = net;  // lanes created later get it too
    return QLSD_OK;
}

qlsd_status qlsd_server_submit_many(qlsd_server s, int32_t code_id, int32_t count, const uint8_t *syndromes,
                                    uint8_t *corrections_out, const uint64_t *tags, const double *arrival_us) {
    if (!s || code_id < 0 || code_id >= (int32_t)s->codes.size()) return serr(s, QLSD_E_INVALID, "bad server or code id");
    if (count < 0 || (count > 0 && (!syndromes || !corrections_out || !tags)))
        return serr(s, QLSD_E_INVALID, "bad request arrays");
    Code &c = *s->codes[code_id];
    std::lock_guard<std::mutex> g(s->mu);
    double last = c.pending.empty() ? -1e300 : c.pending.back().arrival_us;
    for (int32_t k = 0; k < count; k++) {
        const double a = arrival_us ? arrival_us[k] : 0.0;
        if (a < last) return serr(s, QLSD_E_INVALID, "arrival times of a code must be non-decreasing");
        last = a;
        c.pending.push_back(Request{syndromes + (size_t)k * c.m, corrections_out + (size_t)k * c.n, tags[k], a, false});
    }
    return QLSD_OK;
}

qlsd_status qlsd_server_submit_many_device(qlsd_server s, int32_t code_id, int32_t count, const uint8_t *syndromes,
                                           uint8_t *corrections_out, const uint64_t *tags, const double *arrival_us) {
    if (!s || code_id < 0 || code_id >= (int32_t)s->codes.size()) return serr(s, QLSD_E_INVALID, "bad server or code id");
    if (count < 0 || (count > 0 && (!syndromes || !corrections_out || !tags)))
        return serr(s, QLSD_E_INVALID, "bad request arrays");
    Code &c = *s->codes[code_id];
    std::lock_guard<std::mutex> g(s->mu);
    double last = c.pending.empty() ? -1e300 : c.pending.back().arrival_us;
    for (int32_t k = 0; k < count; k++) {
        const double a = arrival_us ? arrival_us[k] : 0.0;
        if (a < last) return serr(s, QLSD_E_INVALID, "arrival times of a code must be non-decreasing");
        last = a;
        c.pending.push_back(Request{syndromes + (size_t)k * c.m, corrections_out + (size_t)k * c.n, tags[k], a, true});
    }
    return QLSD_OK;
}

qlsd_status qlsd_server_lanes(qlsd_server s, int32_t code_id, int32_t *now, int32_t *created, int32_t *retired) {
    if (!s || code_id < 0 || code_id >= (int32_t)s->codes.size()) return serr(s, QLSD_E_INVALID, "bad server or code id");
    const Code &c = *s->codes[code_id];
    if (now) *now = c.n_lanes.load();
    if (created) *created = c.created.load();
    if (retired) *retired = c.retired.load();
    return QLSD_OK;
}

qlsd_status qlsd_server_set_retire_us(qlsd_server s, double retire_us) {
    if (!s || !(retire_us >= 0.0)) return serr(s, QLSD_E_INVALID, "bad server or retire time");
    if (s->started.load()) return serr(s, QLSD_E_INVALID, "set before qlsd_server_start");
    s->retire_us = retire_us;
    return QLSD_OK;
}

qlsd_status qlsd_server_start(qlsd_server s) {
    if (!s) return serr(s, QLSD_E_INVALID, "server is NULL");
    if (s->started.load()) return serr(s, QLSD_E_INVALID, "already started");
    s->epoch = std::chrono::steady_clock::now();
    s->started = true;
    s->worker = std::thread(scheduler, s);
    return QLSD_OK;
}

qlsd_status qlsd_server_wait(qlsd_server s, int64_t count, double timeout_s) {
    if (!s) return serr(s, QLSD_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> g(s->mu);
    const bool ok = s->cv.wait_for(g, std::chrono::duration<double>(timeout_s),
                                   [&] { return s->completed >= count || s->failed.load(); });
    if (s->failed.load()) {
        qlsd::set_last_error("%s", s->error);
        return QLSD_E_DEVICE;
    }
    if (!ok) return serr(s, QLSD_E_DEVICE, "timed out waiting for completions");
    return QLSD_OK;
}

qlsd_status qlsd_server_completions(qlsd_server s, qlsd_completion *out, int32_t max, int32_t *n_out) {
    if (!s || !n_out || (max > 0 && !out)) return serr(s, QLSD_E_INVALID, "bad arguments");
    std::lock_guard<std::mutex> g(s->mu);
    const int32_t k = (int32_t)std::min<size_t>((size_t)std::max(max, 0), s->done.size());
    std::copy(s->done.begin(), s->done.begin() + k, out);
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n_out = k;
    return QLSD_OK;
}

double qlsd_server_now_us(qlsd_server s) { return s ? now_us(s) : 0.0; }

void qlsd_server_destroy(qlsd_server s) {
    if (!s) return;
    s->stop = true;
    if (s->worker.joinable()) s->worker.join();
    for (Code *c : s->codes) {
        for (auto &l : c->lanes) free_lane(*l);
        delete c;
    }
    delete s;
}

}  // extern "C"
