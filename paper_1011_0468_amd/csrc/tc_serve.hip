// Serving engine for streams of independent estimate requests.
//
// A request names a graph (host pairs to build into a CSR, or a resident
// graph handle) and an operating point (p, seed).  Requests are released at
// their arrival time on the server clock and admitted strictly in submission
// order when their memory bound fits the device arena, which is reserved once
// when the server is created: nothing is allocated from the device while
// serving.  A fixed set of lanes (one host worker thread and one stream each,
// default priority) run admitted requests concurrently; every allocation of a
// request's CSR build and count goes to that request's reservation.  Results
// are the same integers as the stand-alone calls produce, so a request's
// counts do not depend on what else is in flight.
#include "tc_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace tc {

namespace {

// First-fit allocator of byte ranges of the arena (offsets, 256-byte granules).
class RangeSet {
public:
    explicit RangeSet(int64_t size) : size_(size) {
        if (size > 0) free_[0] = size;
    }
    bool take(int64_t bytes, int64_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const int64_t rest = it->second - bytes;
                const int64_t at = it->first + bytes;
                free_.erase(it);
                if (rest > 0) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void give(int64_t off, int64_t bytes) {
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }

private:
    int64_t size_;
    int64_t used_ = 0, peak_ = 0;
    std::map<int64_t, int64_t> free_;
};

// One request's reservation: a stack of allocations; freeing the top block
// (and any freed blocks under it) lowers the top again.  Its size is the sum
// of every allocation the request makes, so the top never passes the end.
class Reservation : public AllocRegion {
public:
    Reservation(char* base, int64_t size) : base_(base), size_(size) {}
    void* try_alloc(size_t bytes) override {
        const int64_t b = region_bytes((int64_t)bytes);
        if (top_ + b > size_) return nullptr;
        void* p = base_ + top_;
        blocks_.push_back({top_, b, false});
        top_ += b;
        high_ = std::max(high_, top_);
        return p;
    }
    bool try_free(void* p) override {
        char* c = static_cast<char*>(p);
        if (c < base_ || c >= base_ + size_) return false;
        const int64_t off = c - base_;
        for (auto it = blocks_.rbegin(); it != blocks_.rend(); ++it)
            if (it->off == off && !it->freed) {
                it->freed = true;
                break;
            }
        while (!blocks_.empty() && blocks_.back().freed) {
            top_ = blocks_.back().off;
            blocks_.pop_back();
        }
        return true;
    }
    int64_t high() const { return high_; }

private:
    struct Block {
        int64_t off, len;
        bool freed;
    };
    char* base_;
    int64_t size_;
    int64_t top_ = 0, high_ = 0;
    std::vector<Block> blocks_;
};

struct Job {
    tc_request req;
    int64_t bytes = 0;        // reservation size
    double release_s = 0.0;   // max(arrival, submission)
};

}  // namespace

void check_request(const tc_request* r) {
    if (!r) fail(TC_ERR_INVALID, "request is NULL");
    if (!p_valid(r->p)) fail(TC_ERR_INVALID, "p must be finite and in (0, 1]");
    if (!std::isfinite(r->arrival_s)) fail(TC_ERR_INVALID, "arrival_s must be finite");
    if (r->graph) return;
    if (r->n < 0 || r->num_pairs < 0) fail(TC_ERR_INVALID, "n and num_pairs must be >= 0");
    if (r->num_pairs > 0 && (!r->src || !r->dst)) fail(TC_ERR_INVALID, "src/dst is NULL");
    if (r->n > 0x7fffffffLL) fail(TC_ERR_OVERFLOW, "n exceeds 2^31-1");
    if (2 * r->num_pairs > 0x7fffffffLL) fail(TC_ERR_OVERFLOW, "2*num_pairs exceeds 2^31-1 (int32 CSR)");
}

// Requests a fused group may hold, and its pairs as a multiple of the fusion threshold.
constexpr int kFuseMaxJobs = 64;
constexpr int64_t kFusePairsFactor = 8;

bool fusible(const tc_request& r, int32_t fuse_max_pairs) {
    return fuse_max_pairs > 0 && !r.graph && r.num_pairs <= fuse_max_pairs;
}

int64_t pad_vertices(int64_t n) { return (n + kUnionAlign - 1) / kUnionAlign * kUnionAlign; }

// Arena bytes of a fused group: an upper bound of the sum of the sizes of
// every allocation its union build, union sample and union count make.
int64_t group_bytes(const std::vector<const tc_request*>& rs) {
    auto rb = region_bytes;
    const CountConfig cfg;
    const int64_t K = (int64_t)rs.size();
    int64_t P = 0, nU = 0, hsum = 0, ubytes = 0, ntiles = 0;
    int32_t maxd = 0;
    for (const tc_request* r : rs) {
        P += r->num_pairs;
        nU += pad_vertices(r->n);
        maxd = std::max<int32_t>(maxd, (int32_t)std::max<int64_t>(0, std::min<int64_t>(r->n - 1, 2 * r->num_pairs)));
        const double hb = 2.0 * std::sqrt((double)r->num_pairs) + 2.0;  // h < 2 m'^(1/2) at c = 1, m' <= pairs
        const int64_t h = std::min<int64_t>(r->n, (int64_t)hb);
        if (h >= 3) {
            const int64_t p = (h + 127) / 128 * 128;
            hsum += h;
            ubytes += p * p;
            ntiles += (p / 128) * (p / 128 + 1) / 2;
        }
    }
    const int64_t E2 = 2 * P, NW = (E2 + 63) / 64;
    int64_t b = 2 * rb(4 * P) + build_csr_bytes(nU, P) + rb(4);          // staging, build, max degree
    b += rb(4 * nU) + rb(4 * (K + 1)) + 3 * rb(8 * K) + rb(8 * kCountSlots * K);  // comp, off, salts, thrs, m', results
    b += rb(4 * (nU + 1)) + rb(4 * nU) + rb(8 * NW) + rb(4 * (NW + 1)) + scan_scratch_bytes(NW) + 2 * rb(4 * E2);
    b += count_union_bytes(nU, P, maxd, (int32_t)K, hsum, ubytes, ntiles, cfg);
    return b;
}

int64_t request_bytes(const tc_request* r) {
    const int sampled = r->p < 1.0 ? 1 : 0;
    const CountConfig cfg;  // requests run with the library defaults
    if (r->graph) return count_bytes(r->graph->n, r->graph->m, r->graph->max_deg, sampled, cfg);
    const int64_t n = r->n, P = r->num_pairs;
    int64_t b = 2 * region_bytes(4 * P) + build_csr_bytes(n, P) + region_bytes(4);  // staging, build, max degree
    // the built graph has m <= P edges and degrees <= min(n - 1, 2P)
    const int32_t maxd = (int32_t)std::max<int64_t>(0, std::min<int64_t>(n - 1, 2 * P));
    return b + count_bytes(n, P, maxd, sampled, cfg);
}

}  // namespace tc

struct tc_server_s {
    tc_server_config cfg{};
    int device = -1;
    char* arena = nullptr;
    tc::RangeSet ranges{0};
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work;  // lanes: queue changed, space freed, stop
    std::condition_variable cv_done;  // pollers: a result is ready
    std::deque<tc::Job> queue;
    std::deque<tc_result> done;
    bool stop = false;
    int64_t submitted = 0, completed = 0, rejected = 0, running = 0, spilled = 0;
    std::vector<std::thread> lanes;
    std::vector<hipStream_t> streams;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
    int64_t ranges_size() const { return cfg.budget_bytes / 256 * 256; }
    void lane_main(int lane);
    void run(int lane, const tc::Job& job, char* base, tc_result* res);
    void run_fused(int lane, const std::vector<tc::Job>& jobs, char* base, int64_t bytes, std::vector<tc_result>& res);
};

namespace {

void set_msg(tc_result* r, const std::string& m) {
    std::snprintf(r->message, sizeof(r->message), "%s", m.c_str());
}

}  // namespace

void tc_server_s::run(int lane, const tc::Job& job, char* base, tc_result* res) {
    using namespace tc;
    hipStream_t s = streams[(size_t)lane];
    Reservation region(base, job.bytes);
    AllocRegion* prev = set_thread_region(&region);
    const tc_request& r = job.req;
    try {
        const int sampled = r.p < 1.0 ? 1 : 0;
        const CountConfig cfg;
        tc_graph_s* g = r.graph;
        tc_graph_s* built = nullptr;
        if (!g) g = built = graph_from_pairs(r.n, r.num_pairs, r.src, r.dst, 0, s);
        try {
            count_core(g, sampled, keep_threshold(r.p), sample_salt(r.seed), cfg, s, &res->counts);
        } catch (...) {
            (void)hipStreamSynchronize(s);
            graph_release(built);
            throw;
        }
        graph_release(built);
        res->estimate = rescale(res->counts.triangles, r.p);
        res->status = TC_OK;
    } catch (const Error& e) {
        res->status = e.status;
        set_msg(res, e.msg);
    } catch (const std::exception& e) {
        res->status = TC_ERR_DEVICE;
        set_msg(res, e.what());
    } catch (...) {
        res->status = TC_ERR_DEVICE;
        set_msg(res, "unknown error");
    }
    // the reservation is handed back only after the stream has drained
    if (hipStreamSynchronize(s) != hipSuccess && res->status == TC_OK) {
        res->status = TC_ERR_DEVICE;
        set_msg(res, "stream synchronisation failed");
    }
    set_thread_region(prev);
    res->peak_bytes = region.high();
    res->spilled_bytes = region.spilled;
}

// A fused group: the requests' pairs, ids shifted to disjoint ranges padded
// to kUnionAlign, built as one graph; component k sampled with request k's
// (p, seed) and counted into its own result slots by one pass of the count.
// A request with an id outside [0, n) fails alone and joins no union.
void tc_server_s::run_fused(int lane, const std::vector<tc::Job>& jobs, char* base, int64_t bytes,
                            std::vector<tc_result>& res) {
    using namespace tc;
    hipStream_t s = streams[(size_t)lane];
    Reservation region(base, bytes);
    AllocRegion* prev = set_thread_region(&region);
    std::vector<int> members;  // jobs in the union, in order
    for (size_t i = 0; i < jobs.size(); ++i) {
        const tc_request& r = jobs[i].req;
        bool ok = true;
        for (int64_t e = 0; e < r.num_pairs && ok; ++e)
            ok = r.src[e] >= 0 && r.src[e] < r.n && r.dst[e] >= 0 && r.dst[e] < r.n;
        if (ok) {
            members.push_back((int)i);
        } else {
            res[i].status = TC_ERR_INVALID;
            set_msg(&res[i], "vertex id outside [0, n)");
        }
    }
    const int32_t K = (int32_t)members.size();
    try {
        if (K > 0) {
            std::vector<int32_t> off((size_t)K + 1, 0);
            std::vector<uint64_t> salts((size_t)K), thrs((size_t)K);
            int64_t P = 0;
            for (int32_t k = 0; k < K; ++k) {
                const tc_request& r = jobs[(size_t)members[(size_t)k]].req;
                off[(size_t)k + 1] = (int32_t)(off[(size_t)k] + pad_vertices(r.n));
                salts[(size_t)k] = sample_salt(r.seed);
                thrs[(size_t)k] = keep_threshold(r.p);
                P += r.num_pairs;
            }
            const int64_t nU = off[(size_t)K];
            if (nU > 0x7fffffffLL || 2 * P > 0x7fffffffLL) fail(TC_ERR_OVERFLOW, "fused group exceeds int32 ids");
            std::vector<int32_t> hs((size_t)P), hd((size_t)P);
            int64_t at = 0;
            for (int32_t k = 0; k < K; ++k) {
                const tc_request& r = jobs[(size_t)members[(size_t)k]].req;
                const int32_t o = off[(size_t)k];
                for (int64_t e = 0; e < r.num_pairs; ++e) {
                    hs[(size_t)at] = r.src[e] + o;
                    hd[(size_t)at] = r.dst[e] + o;
                    ++at;
                }
            }
            const CountConfig cfg;
            tc_graph_s* gu = graph_from_pairs(nU, P, hs.data(), hd.data(), 0, s);
            tc_graph_s* gs = new tc_graph_s();
            try {
                DevBuf<int32_t> comp(nU, s), offd((size_t)K + 1, s);
                DevBuf<uint64_t> saltd(K, s), thrd(K, s);
                DevBuf<int64_t> mk(K, s), accs((size_t)K * kCountSlots, s);
                check_hip(hipMemcpyAsync(offd.get(), off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, s),
                          "offsets");
                check_hip(hipMemcpyAsync(saltd.get(), salts.data(), sizeof(uint64_t) * (size_t)K, hipMemcpyHostToDevice,
                                         s), "salts");
                check_hip(hipMemcpyAsync(thrd.get(), thrs.data(), sizeof(uint64_t) * (size_t)K, hipMemcpyHostToDevice, s),
                          "thresholds");
                comp_from_offsets(nU, K, offd.get(), comp.get(), s);
                sample_union_components(gu, K, comp.get(), offd.get(), saltd.get(), thrd.get(), s, gs, mk.get());
                CountUnion un;
                un.K = K;
                un.comp = comp.get();
                un.off = offd.get();
                un.mk = mk.get();
                count_union(gs, un, cfg, s, accs.get());
                std::vector<int64_t> h((size_t)K * kCountSlots);
                check_hip(hipMemcpyAsync(h.data(), accs.get(), sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost, s),
                          "results");
                check_hip(hipStreamSynchronize(s), "sync");
                for (int32_t k = 0; k < K; ++k) {
                    tc_result& x = res[(size_t)members[(size_t)k]];
                    counts_from_slots(h.data() + (size_t)k * kCountSlots, &x.counts);
                    x.estimate = rescale(x.counts.triangles, jobs[(size_t)members[(size_t)k]].req.p);
                    x.status = TC_OK;
                }
            } catch (...) {
                (void)hipStreamSynchronize(s);
                graph_release(gs);
                graph_release(gu);
                throw;
            }
            graph_release(gs);
            graph_release(gu);
        }
    } catch (const Error& e) {
        for (int m : members) {
            res[(size_t)m].status = e.status;
            set_msg(&res[(size_t)m], e.msg);
        }
    } catch (const std::exception& e) {
        for (int m : members) {
            res[(size_t)m].status = TC_ERR_DEVICE;
            set_msg(&res[(size_t)m], e.what());
        }
    } catch (...) {
        for (int m : members) {
            res[(size_t)m].status = TC_ERR_DEVICE;
            set_msg(&res[(size_t)m], "unknown error");
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess)
        for (int m : members)
            if (res[(size_t)m].status == TC_OK) {
                res[(size_t)m].status = TC_ERR_DEVICE;
                set_msg(&res[(size_t)m], "stream synchronisation failed");
            }
    set_thread_region(prev);
    for (auto& x : res) {
        x.peak_bytes = region.high();
        x.spilled_bytes = region.spilled;
    }
}

void tc_server_s::lane_main(int lane) {
    if (device >= 0) (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        if (queue.empty()) {
            if (stop) return;
            cv_work.wait(lk);
            continue;
        }
        tc::Job& head = queue.front();
        const double t = now();
        if (head.release_s > t) {
            cv_work.wait_for(lk, std::chrono::duration<double>(head.release_s - t));
            continue;
        }
        // a small request takes the released small requests right behind it
        if (tc::fusible(head.req, cfg.fuse_max_pairs)) {
            std::vector<const tc_request*> grp{&head.req};
            int64_t pairs = head.req.num_pairs;
            for (size_t j = 1; j < queue.size() && grp.size() < (size_t)tc::kFuseMaxJobs; ++j) {
                const tc::Job& q = queue[j];
                if (!tc::fusible(q.req, cfg.fuse_max_pairs) || q.release_s > t ||
                    pairs + q.req.num_pairs > tc::kFusePairsFactor * cfg.fuse_max_pairs)
                    break;
                grp.push_back(&q.req);
                pairs += q.req.num_pairs;
            }
            if (grp.size() >= 2) {
                const int64_t gbytes = tc::group_bytes(grp);
                int64_t goff = 0;
                if (gbytes <= ranges_size() && ranges.take(gbytes, &goff)) {
                    std::vector<tc::Job> jobs(queue.begin(), queue.begin() + (long)grp.size());
                    for (size_t j = 0; j < grp.size(); ++j) queue.pop_front();
                    running += (int64_t)jobs.size();
                    std::vector<tc_result> res(jobs.size());
                    const double st = now();
                    for (size_t j = 0; j < jobs.size(); ++j) {
                        res[j].id = jobs[j].req.id;
                        res[j].lane = lane;
                        res[j].arrival_s = jobs[j].release_s;
                        res[j].reserved_bytes = gbytes;
                        res[j].start_s = st;
                    }
                    cv_work.notify_all();
                    lk.unlock();
                    run_fused(lane, jobs, arena + goff, gbytes, res);
                    const double dn = now();
                    lk.lock();
                    ranges.give(goff, gbytes);
                    running -= (int64_t)jobs.size();
                    completed += (int64_t)jobs.size();
                    for (auto& x : res) {
                        x.done_s = dn;
                        spilled += x.spilled_bytes;
                        done.push_back(x);
                    }
                    cv_done.notify_all();
                    cv_work.notify_all();
                    continue;
                }
                // the group does not fit now: the head goes alone
            }
        }
        int64_t off = 0;
        if (!ranges.take(head.bytes, &off)) {
            cv_work.wait(lk);  // woken when a lane hands its reservation back
            continue;
        }
        tc::Job job = head;
        queue.pop_front();
        ++running;
        tc_result res{};
        res.id = job.req.id;
        res.lane = lane;
        res.arrival_s = job.release_s;
        res.reserved_bytes = job.bytes;
        res.start_s = now();
        cv_work.notify_all();  // the next head may fit as well
        lk.unlock();
        run(lane, job, arena + off, &res);
        res.done_s = now();
        lk.lock();
        ranges.give(off, job.bytes);
        --running;
        ++completed;
        spilled += res.spilled_bytes;
        done.push_back(res);
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

using namespace tc;

namespace {

template <typename F>
tc_status guarded_serve(F&& f) {
    try {
        set_last_error("");
        f();
        return TC_OK;
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return TC_ERR_DEVICE;
    } catch (...) {
        set_last_error("unknown error");
        return TC_ERR_DEVICE;
    }
}

}  // namespace

extern "C" {

tc_status tc_request_bytes(const tc_request* r, int64_t* bytes) {
    return guarded_serve([&] {
        if (!bytes) fail(TC_ERR_INVALID, "output is NULL");
        check_request(r);
        *bytes = request_bytes(r);
    });
}

tc_status tc_server_create(const tc_server_config* cfg, tc_server* out) {
    return guarded_serve([&] {
        if (!cfg || !out) fail(TC_ERR_INVALID, "config or output is NULL");
        if (cfg->budget_bytes < 0) fail(TC_ERR_INVALID, "budget_bytes must be >= 0");
        if (cfg->lanes < 1 || cfg->lanes > 16) fail(TC_ERR_INVALID, "lanes must be in [1, 16]");
        if (cfg->fuse_max_pairs < 0) fail(TC_ERR_INVALID, "fuse_max_pairs must be >= 0");
        tc_server_s* sv = new tc_server_s();
        sv->cfg = *cfg;
        try {
            const int64_t budget = cfg->budget_bytes / 256 * 256;
            if (budget > 0) {
                sv->arena = static_cast<char*>(dev_alloc((size_t)budget, nullptr));
                check_hip(hipGetDevice(&sv->device), "get device");
                for (int i = 0; i < cfg->lanes; ++i) {
                    hipStream_t st = nullptr;
                    check_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream create");
                    sv->streams.push_back(st);
                }
            } else {
                sv->streams.assign((size_t)cfg->lanes, nullptr);  // nothing can be admitted
            }
            sv->ranges = RangeSet(budget);
            sv->t0 = std::chrono::steady_clock::now();
            for (int i = 0; i < cfg->lanes; ++i) sv->lanes.emplace_back(&tc_server_s::lane_main, sv, i);
        } catch (...) {
            for (hipStream_t st : sv->streams)
                if (st) (void)hipStreamDestroy(st);
            if (sv->arena) dev_free(sv->arena, nullptr);
            delete sv;
            throw;
        }
        *out = sv;
    });
}

tc_status tc_server_clock(tc_server sv, double* now_s) {
    return guarded_serve([&] {
        if (!sv || !now_s) fail(TC_ERR_INVALID, "server or output is NULL");
        *now_s = sv->now();
    });
}

tc_status tc_server_submit(tc_server sv, const tc_request* r) {
    return guarded_serve([&] {
        if (!sv || !r) fail(TC_ERR_INVALID, "server or request is NULL");
        check_request(r);
        const int64_t bytes = request_bytes(r);
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) fail(TC_ERR_INVALID, "server is shutting down");
        if (bytes > sv->cfg.budget_bytes / 256 * 256) {
            ++sv->rejected;
            fail(TC_ERR_BUDGET, "request needs " + std::to_string(bytes) + " bytes, budget is " +
                                    std::to_string(sv->cfg.budget_bytes));
        }
        Job j;
        j.req = *r;
        j.bytes = bytes;
        j.release_s = std::max(r->arrival_s, sv->now());
        sv->queue.push_back(j);
        ++sv->submitted;
        sv->cv_work.notify_all();
    });
}

tc_status tc_server_poll(tc_server sv, tc_result* out, int32_t cap, double timeout_s, int32_t* got) {
    return guarded_serve([&] {
        if (!sv || !got || (cap > 0 && !out)) fail(TC_ERR_INVALID, "server or output is NULL");
        if (cap < 0) fail(TC_ERR_INVALID, "cap must be >= 0");
        std::unique_lock<std::mutex> lk(sv->mu);
        auto ready = [&] {
            return !sv->done.empty() || (sv->queue.empty() && sv->running == 0);
        };
        if (timeout_s < 0) sv->cv_done.wait(lk, ready);
        else if (timeout_s > 0) sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
        int32_t k = 0;
        while (k < cap && !sv->done.empty()) {
            out[k++] = sv->done.front();
            sv->done.pop_front();
        }
        *got = k;
    });
}

tc_status tc_server_stats(tc_server sv, tc_server_info* st) {
    return guarded_serve([&] {
        if (!sv || !st) fail(TC_ERR_INVALID, "server or output is NULL");
        std::lock_guard<std::mutex> lk(sv->mu);
        st->submitted = sv->submitted;
        st->completed = sv->completed;
        st->rejected = sv->rejected;
        st->queued = (int64_t)sv->queue.size();
        st->running = sv->running;
        st->arena_bytes = sv->cfg.budget_bytes / 256 * 256;
        st->arena_used = sv->ranges.used();
        st->arena_peak = sv->ranges.peak();
        st->spilled_bytes = sv->spilled;
    });
}

void tc_server_destroy(tc_server sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    for (auto& t : sv->lanes) t.join();
    for (hipStream_t st : sv->streams)
        if (st) (void)hipStreamDestroy(st);
    if (sv->arena) {
        try {
            dev_free(sv->arena, nullptr);
        } catch (...) {
        }
    }
    delete sv;
}

}  // extern "C"
