// Host runtime and the extern "C" boundary: argument checks, status codes,
// thread-local error text, the device allocator (callback or caching pool),
// launch profiling, and the estimate / median-of-means arithmetic.
#include "tc_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

namespace tc {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

void fail(tc_status st, const std::string& msg) { throw Error{st, msg}; }

void set_last_error(const std::string& msg) { g_last_error = msg; }

void check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(TC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// allocator
// ---------------------------------------------------------------------------

namespace {

std::mutex g_alloc_mu;
tc_alloc_fn g_alloc = nullptr;
tc_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;

// Caching pool: blocks are reused by later allocations on the same stream
// (stream order makes that safe); sizes are rounded to classes.
struct Pool {
    std::mutex mu;
    std::multimap<std::pair<hipStream_t, size_t>, void*> free_blocks;
    std::unordered_map<void*, size_t> live;
};
Pool& pool() {
    static Pool* p = new Pool();  // never destroyed: blocks live until process exit
    return *p;
}

size_t size_class(size_t b) {
    if (b <= 512) return 512;
    if (b <= (1u << 20)) {
        size_t c = 512;
        while (c < b) c <<= 1;
        return c;
    }
    const size_t g = (size_t)2 << 20;
    return (b + g - 1) / g * g;
}

void* pool_alloc(size_t bytes, hipStream_t s) {
    const size_t c = size_class(bytes);
    Pool& P = pool();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.free_blocks.find({s, c});
        if (it != P.free_blocks.end()) {
            void* p = it->second;
            P.free_blocks.erase(it);
            P.live[p] = c;
            return p;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, c) != hipSuccess || !p) {
        (void)hipGetLastError();
        // release cached blocks and retry once
        std::vector<void*> drop;
        {
            std::lock_guard<std::mutex> lk(P.mu);
            for (auto& kv : P.free_blocks) drop.push_back(kv.second);
            P.free_blocks.clear();
        }
        if (!drop.empty()) {
            (void)hipDeviceSynchronize();
            for (void* q : drop) (void)hipFree(q);
        }
        p = nullptr;
        if (hipMalloc(&p, c) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> lk(P.mu);
    P.live[p] = c;
    return p;
}

void pool_free(void* p, hipStream_t s) {
    Pool& P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.live.find(p);
    if (it == P.live.end()) return;
    P.free_blocks.insert({{s, it->second}, p});
    P.live.erase(it);
}

}  // namespace

static thread_local AllocRegion* t_region = nullptr;

AllocRegion* set_thread_region(AllocRegion* r) {
    AllocRegion* old = t_region;
    t_region = r;
    return old;
}

void* dev_alloc(size_t bytes, hipStream_t s) {
    if (t_region) {
        if (void* p = t_region->try_alloc(bytes ? bytes : 1)) return p;
        if (t_region->strict)
            fail(TC_ERR_BUDGET, "allocation of " + std::to_string(bytes) + " bytes does not fit the fixed region");
        t_region->spilled += (int64_t)bytes;
    }
    tc_alloc_fn a;
    void* ctx;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        a = g_alloc;
        ctx = g_alloc_ctx;
    }
    void* p = a ? a(bytes ? bytes : 1, (void*)s, ctx) : pool_alloc(bytes ? bytes : 1, s);
    if (!p) fail(TC_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
}

void dev_free(void* p, hipStream_t s) {
    if (!p) return;
    if (t_region && t_region->try_free(p)) return;
    tc_free_fn f;
    void* ctx;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        f = g_free;
        ctx = g_alloc_ctx;
    }
    if (f) f(p, (void*)s, ctx);
    else pool_free(p, s);
}

// ---------------------------------------------------------------------------
// launch profiling
// ---------------------------------------------------------------------------

namespace {

struct Pending {
    const char* name;
    const char* phase;
    hipEvent_t a, b;
};

std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_event_pool;
std::map<std::string, std::pair<double, int64_t>> g_prof;
std::vector<std::string> g_prof_names;  // empty: profile every kernel

bool selected(const char* name) {
    if (g_prof_names.empty()) return true;
    for (auto& s : g_prof_names)
        if (s == name) return true;
    return false;
}

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    check_hip(hipEventCreate(&e), "event create");
    return e;
}

}  // namespace

static thread_local bool t_no_profile = false;
static thread_local const char* t_phase = nullptr;

PhaseScope::PhaseScope(const char* ph) : prev(t_phase) { t_phase = ph; }
PhaseScope::~PhaseScope() { t_phase = prev; }

NoProfileScope::NoProfileScope() : prev(t_no_profile) { t_no_profile = true; }
NoProfileScope::~NoProfileScope() { t_no_profile = prev; }

LaunchScope::LaunchScope(const char* n, hipStream_t s) : name(n), phase(t_phase), stream(s) {
    if (t_no_profile) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || !selected(n)) return;
    hipEvent_t e = take_event();
    check_hip(hipEventRecord(e, s), "event record");
    ev0 = (void*)e;
}

LaunchScope::~LaunchScope() {
    if (!ev0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t e1 = nullptr;
    try {
        e1 = take_event();
    } catch (...) {
        return;
    }
    if (hipEventRecord(e1, stream) != hipSuccess) return;
    g_pending.push_back({name, phase, (hipEvent_t)ev0, e1});
}

void profile_collect() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::vector<Pending> keep;
    for (auto& p : g_pending) {
        if (hipEventQuery(p.b) != hipSuccess) {
            keep.push_back(p);
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto& slot = g_prof[p.name];
            slot.first += ms;
            slot.second += 1;
            if (p.phase) {
                auto& ph = g_prof[std::string("@") + p.phase];
                ph.first += ms;
                ph.second += 1;
            }
        }
        g_event_pool.push_back(p.a);
        g_event_pool.push_back(p.b);
    }
    g_pending.swap(keep);
}

}  // namespace tc

// ---------------------------------------------------------------------------
// extern "C" boundary
// ---------------------------------------------------------------------------

using namespace tc;

namespace {

template <typename F>
tc_status guarded(F&& f) {
    try {
        g_last_error.clear();
        f();
        profile_collect();
        return TC_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.status;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return TC_ERR_DEVICE;
    } catch (...) {
        g_last_error = "unknown error";
        return TC_ERR_DEVICE;
    }
}


}  // namespace

namespace tc {

bool p_valid(double p) { return std::isfinite(p) && p > 0.0 && p <= 1.0; }

int num_cus() {
    // compute units of the current device (256 on MI355X), read once
    static const int cus = [] {
        int dev = 0, c = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            c = prop.multiProcessorCount;
        (void)hipGetLastError();
        return c > 0 ? c : 256;
    }();
    return cus;
}

// The heavy multiplier c = heavy_num / heavy_den enters the integer test
// heavy_den^2 deg^2 > heavy_num^2 m, which the device evaluates exactly for
// both terms up to 2^15.
void check_heavy_multiplier(int32_t num, int32_t den) {
    if (den < 1 || num < 0) fail(TC_ERR_INVALID, "heavy_num must be >= 0 and heavy_den >= 1");
    if (num > kHeavyTermMax || den > kHeavyTermMax)
        fail(TC_ERR_INVALID, "heavy_num and heavy_den must be at most 32768");
}

CountConfig config_from(const tc_params* prm, const tc_graph_s* g, int sampled, double p) {
    CountConfig c;
    if (prm) {
        check_heavy_multiplier(prm->heavy_num, prm->heavy_den);
        c.heavy_num = prm->heavy_num;
        c.heavy_den = prm->heavy_den;
        if (prm->use_tuned) c = tuned_config(g, sampled, p, c);  // the table's entry replaces the split too
    }
    return c;
}

double rescale(int64_t T, double p) {
    volatile double p2 = p * p;
    volatile double p3 = p2 * p;
    return (double)T / p3;
}

void graph_release(tc_graph_s* g) {
    if (!g) return;
    dev_free(g->row_ptr, g->home);
    dev_free(g->col, g->home);
    dev_free(g->src, g->home);
    dev_free(g->deg, g->home);
    if (g->ncls) dev_free(g->ncls, g->home);
    delete g;
}

__global__ void k_max_i32(const int32_t* a, int64_t n, int32_t* out) {
    int32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = a[i] > m ? a[i] : m;
    for (int d = 32; d >= 1; d >>= 1) {
        int32_t o = __shfl_xor(m, d, 64);
        m = o > m ? o : m;
    }
    if (__lane_id() == 0) atomicMax(out, m);
}

int32_t max_degree(const tc_graph_s* g, hipStream_t s) {
    if (g->n == 0) return 0;
    DevBuf<int32_t> out(1, s);
    fill_i32(out.get(), 0, 1, s);
    unsigned blocks = ceil_div(g->n, 256);
    if (blocks > 4096) blocks = 4096;
    TC_LAUNCH("max_deg", k_max_i32, dim3(blocks), dim3(256), 0, s, (const int32_t*)g->deg, g->n, out.get());
    int32_t h = 0;
    check_hip(hipMemcpyAsync(&h, out.get(), sizeof(int32_t), hipMemcpyDeviceToHost, s), "max deg");
    check_hip(hipStreamSynchronize(s), "sync");
    return h;
}

tc_graph_s* graph_from_pairs(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst, int on_device,
                             hipStream_t s) {
    if (n < 0 || num_pairs < 0) fail(TC_ERR_INVALID, "n and num_pairs must be >= 0");
    if (num_pairs > 0 && (!src || !dst)) fail(TC_ERR_INVALID, "src/dst is NULL");
    if (n > 0x7fffffffLL) fail(TC_ERR_OVERFLOW, "n exceeds 2^31-1");
    if (2 * num_pairs > 0x7fffffffLL) fail(TC_ERR_OVERFLOW, "2*num_pairs exceeds 2^31-1 (int32 CSR)");
    DevBuf<int32_t> hs, hd;
    const int32_t* ds = src;
    const int32_t* dd = dst;
    if (!on_device && num_pairs > 0) {
        hs.reset(num_pairs, s);
        hd.reset(num_pairs, s);
        check_hip(hipMemcpyAsync(hs.get(), src, sizeof(int32_t) * num_pairs, hipMemcpyHostToDevice, s), "H2D src");
        check_hip(hipMemcpyAsync(hd.get(), dst, sizeof(int32_t) * num_pairs, hipMemcpyHostToDevice, s), "H2D dst");
        ds = hs.get();
        dd = hd.get();
    }
    tc_graph_s* g = new tc_graph_s();
    try {
        if (build_csr(n, num_pairs, ds, dd, s, g)) fail(TC_ERR_INVALID, "vertex id outside [0, n)");
        g->max_deg = max_degree(g, s);
    } catch (...) {
        (void)hipStreamSynchronize(s);
        graph_release(g);
        throw;
    }
    return g;
}

}  // namespace tc

extern "C" {

tc_status tc_set_allocator(tc_alloc_fn alloc, tc_free_fn free_, void* ctx) {
    return guarded([&] {
        if ((alloc == nullptr) != (free_ == nullptr)) fail(TC_ERR_INVALID, "alloc and free must both be set or both NULL");
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_alloc = alloc;
        g_free = free_;
        g_alloc_ctx = ctx;
    });
}

tc_status tc_build_csr(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst, int32_t on_device,
                       void* stream, tc_graph* out) {
    return guarded([&] {
        if (!out) fail(TC_ERR_INVALID, "out is NULL");
        *out = graph_from_pairs(n, num_pairs, src, dst, on_device, (hipStream_t)stream);
    });
}

tc_status tc_graph_info(tc_graph g, int64_t* n, int64_t* m, int32_t* max_deg) {
    return guarded([&] {
        if (!g) fail(TC_ERR_INVALID, "graph is NULL");
        if (n) *n = g->n;
        if (m) *m = g->m;
        if (max_deg) *max_deg = g->max_deg;
    });
}

tc_status tc_graph_csr(tc_graph g, const int32_t** row_ptr, const int32_t** col) {
    return guarded([&] {
        if (!g) fail(TC_ERR_INVALID, "graph is NULL");
        if (row_ptr) *row_ptr = g->row_ptr;
        if (col) *col = g->col;
    });
}

tc_status tc_graph_read(tc_graph g, int32_t* row_ptr, int32_t* col, int32_t* deg, int32_t on_device, void* stream) {
    return guarded([&] {
        if (!g) fail(TC_ERR_INVALID, "graph is NULL");
        hipStream_t s = (hipStream_t)stream;
        const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (row_ptr)
            check_hip(hipMemcpyAsync(row_ptr, g->row_ptr, sizeof(int32_t) * (size_t)(g->n + 1), kind, s), "row_ptr");
        if (col && g->m > 0)
            check_hip(hipMemcpyAsync(col, g->col, sizeof(int32_t) * (size_t)(2 * g->m), kind, s), "col");
        if (deg && g->n > 0)
            check_hip(hipMemcpyAsync(deg, g->deg, sizeof(int32_t) * (size_t)g->n, kind, s), "deg");
        check_hip(hipStreamSynchronize(s), "sync");
    });
}

tc_status tc_sample(tc_graph g, double p, uint64_t seed, void* stream, tc_graph* out_sampled) {
    return guarded([&] {
        if (!g || !out_sampled) fail(TC_ERR_INVALID, "graph or output is NULL");
        if (!p_valid(p)) fail(TC_ERR_INVALID, "p must be finite and in (0, 1]");
        hipStream_t s = (hipStream_t)stream;
        const int64_t n = g->n, E2 = 2 * g->m, NW = (E2 + 63) / 64;
        tc_graph_s* o = new tc_graph_s();
        try {
            o->n = n;
            o->home = s;
            o->row_ptr = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(n + 1), s);
            o->deg = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1), s);
            PhaseScope ph("sample");
            DevBuf<uint64_t> bits(NW, s);
            DevBuf<int32_t> wpre(NW + 1, s);
            fill_i32(wpre.get(), 0, 1, s);
            sample_keep_bits(g, sample_salt(seed), keep_threshold(p), bits.get(), wpre.get(), s);
            if (NW > 0) scan_exclusive_i32(wpre.get(), wpre.get(), NW, s);
            positions_at_rows(g->row_ptr, n, E2, bits.get(), wpre.get(), o->row_ptr, o->deg, s);
            int32_t total = 0;
            check_hip(hipMemcpyAsync(&total, wpre.get() + NW, sizeof(int32_t), hipMemcpyDeviceToHost, s), "total");
            check_hip(hipStreamSynchronize(s), "sync");
            o->m = total / 2;
            o->col = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s);
            o->src = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s);
            compact_kept(g->col, g->src, E2, bits.get(), wpre.get(), o->col, o->src, s);
            o->max_deg = max_degree(o, s);
        } catch (...) {
            (void)hipStreamSynchronize(s);
            graph_release(o);
            throw;
        }
        *out_sampled = o;
    });
}

tc_status tc_count_exact(tc_graph g, const tc_params* prm, void* stream, tc_counts* out) {
    return guarded([&] {
        if (!g || !out) fail(TC_ERR_INVALID, "graph or output is NULL");
        CountConfig cfg = config_from(prm, g, 0, 1.0);
        tc_counts r;
        count_core(g, 0, 0, 0, cfg, (hipStream_t)stream, &r);
        *out = r;
    });
}

// Counts of several independent sparsified copies of g.  The copies of a
// chunk of seeds are sampled into one union graph (copy k of the chunk is
// component k) and counted together: every kernel launch of the chunk covers
// all of its seeds, and each component's counts equal a count of that copy
// alone.  Chunks are sized so that the union stays within int32 ids and a
// memory budget.  Without sampling (p = 1) every seed counts g itself.
static void count_batch(const tc_graph_s* g, int sampled, uint64_t thr, const uint64_t* salts, int32_t S,
                        const CountConfig& cfg, hipStream_t s, std::vector<tc_counts>& res) {
    res.resize((size_t)S);
    if (S == 1 || !sampled) {
        count_core(g, sampled, thr, salts[0], cfg, s, &res[0]);
        for (int32_t i = 1; i < S; ++i) res[(size_t)i] = res[0];
        return;
    }
    const int64_t npad = (g->n + kUnionAlign - 1) / kUnionAlign * kUnionAlign;
    const double p = (double)thr / 9007199254740992.0;
    const double kept = p * (double)(2 * g->m) * 1.1 + 4096.0;  // expected entries per copy, with slack
    const double per_copy = 110.0 * (double)npad + 48.0 * kept;  // bytes the union count takes per copy
    int64_t kc = S;
    kc = std::min<int64_t>(kc, (int64_t)((double)(1 << 30) / kept));
    kc = std::min<int64_t>(kc, npad > 0 ? ((int64_t)1 << 31) / (npad + 1) - 1 : kc);
    kc = std::min<int64_t>(kc, (int64_t)(48.0 * (double)(1ull << 30) / per_copy));
    if (kc < 1) kc = 1;
    for (int32_t i0 = 0; i0 < S; i0 += (int32_t)kc) {
        const int32_t K = (int32_t)std::min<int64_t>(kc, S - i0);
        if (K == 1) {  // a union of one costs two synchronisations and saves nothing
            count_core(g, sampled, thr, salts[i0], cfg, s, &res[(size_t)i0]);
            continue;
        }
        DevBuf<uint64_t> sd(K, s);
        check_hip(hipMemcpyAsync(sd.get(), salts + i0, sizeof(uint64_t) * (size_t)K, hipMemcpyHostToDevice, s),
                  "salts");
        DevBuf<int32_t> comp((size_t)K * (size_t)npad, s), off((size_t)K + 1, s);
        DevBuf<int64_t> mk(K, s), accs((size_t)K * kCountSlots, s);
        tc_graph_s* gu = new tc_graph_s();
        std::vector<int64_t> h((size_t)K * kCountSlots);
        try {
            sample_union_replicas(g, K, sd.get(), thr, s, gu, comp.get(), off.get(), mk.get());
            CountUnion un;
            un.K = K;
            un.comp = comp.get();
            un.off = off.get();
            un.mk = mk.get();
            count_union(gu, un, cfg, s, accs.get());
            check_hip(hipMemcpyAsync(h.data(), accs.get(), sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost, s),
                      "acc");
            check_hip(hipStreamSynchronize(s), "sync");
        } catch (...) {
            (void)hipStreamSynchronize(s);
            graph_release(gu);
            throw;
        }
        graph_release(gu);
        for (int32_t k = 0; k < K; ++k)
            counts_from_slots(h.data() + (size_t)k * kCountSlots, &res[(size_t)(i0 + k)]);
    }
}

// Median of the group means of the counts (groups of consecutive seeds; for
// an even number of groups the two middle group sums are added and divided
// once), rescaled by 1/p^3 (section 3.1), in the order of operations the
// oracle follows.
static double median_of_means(const std::vector<tc_counts>& res, int32_t num_groups, double p) {
    const int32_t S = (int32_t)res.size();
    const int32_t per = S / num_groups;
    std::vector<int64_t> sums((size_t)num_groups, 0);
    for (int32_t gi = 0; gi < num_groups; ++gi)
        for (int32_t i = 0; i < per; ++i) sums[(size_t)gi] += res[(size_t)(gi * per + i)].triangles;
    std::sort(sums.begin(), sums.end());
    volatile double p2 = p * p;
    volatile double p3 = p2 * p;
    if (num_groups % 2 == 0) {
        const int64_t M = sums[(size_t)(num_groups / 2 - 1)] + sums[(size_t)(num_groups / 2)];
        volatile double den = 2.0 * (double)per;
        den = den * p3;
        return (double)M / den;
    }
    volatile double den = (double)per;
    den = den * p3;
    return (double)sums[(size_t)((num_groups - 1) / 2)] / den;
}

tc_status tc_estimate(tc_graph g, double p, const uint64_t* seeds, int32_t num_seeds, int32_t num_groups,
                      const tc_params* prm, void* stream, tc_counts* per_seed, double* per_seed_est,
                      double* mom_est) {
    return guarded([&] {
        if (!g) fail(TC_ERR_INVALID, "graph is NULL");
        if (!p_valid(p)) fail(TC_ERR_INVALID, "p must be finite and in (0, 1]");
        if (num_seeds < 1 || !seeds) fail(TC_ERR_INVALID, "need at least one seed");
        if (num_groups < 1 || num_groups > num_seeds || num_seeds % num_groups)
            fail(TC_ERR_INVALID, "num_groups must divide num_seeds");
        const int sampled = p < 1.0 ? 1 : 0;  // p = 1 keeps every edge: the exact count itself
        CountConfig cfg = config_from(prm, g, sampled, p);
        const uint64_t thr = keep_threshold(p);
        std::vector<uint64_t> salts((size_t)num_seeds);
        for (int32_t i = 0; i < num_seeds; ++i) salts[(size_t)i] = sample_salt(seeds[i]);
        std::vector<tc_counts> res;
        count_batch(g, sampled, thr, salts.data(), num_seeds, cfg, (hipStream_t)stream, res);
        if (per_seed)
            for (int32_t i = 0; i < num_seeds; ++i) per_seed[i] = res[(size_t)i];
        if (per_seed_est)
            for (int32_t i = 0; i < num_seeds; ++i) per_seed_est[i] = rescale(res[(size_t)i].triangles, p);
        if (mom_est) *mom_est = median_of_means(res, num_groups, p);
    });
}

tc_status tc_estimate_adaptive(tc_graph g, double p0, double tol, uint64_t seed0, int32_t num_seeds,
                               int32_t num_groups, int32_t max_stages, const tc_params* prm, void* stream,
                               tc_stage* stages, int32_t* num_stages, double* p_balance) {
    if (num_stages) *num_stages = 0;
    return guarded([&] {
        if (!g || !stages || !num_stages) fail(TC_ERR_INVALID, "graph, stages or num_stages is NULL");
        if (!p_valid(p0)) fail(TC_ERR_INVALID, "p0 must be finite and in (0, 1]");
        if (!(tol >= 0.0) || !std::isfinite(tol)) fail(TC_ERR_INVALID, "tol must be finite and >= 0");
        if (max_stages < 1) fail(TC_ERR_INVALID, "max_stages must be >= 1");
        if (num_seeds < 1) fail(TC_ERR_INVALID, "need at least one seed");
        if (num_groups < 1 || num_groups > num_seeds || num_seeds % num_groups)
            fail(TC_ERR_INVALID, "num_groups must divide num_seeds");
        std::vector<tc_counts> res;
        std::vector<uint64_t> salts((size_t)num_seeds);
        double prev = 0.0;
        for (int32_t k = 0; k < max_stages; ++k) {
            const double p = std::min(1.0, std::ldexp(p0, k));  // exact: a power-of-two scaling
            const int sampled = p < 1.0 ? 1 : 0;
            const CountConfig cfg = config_from(prm, g, sampled, p);
            for (int32_t i = 0; i < num_seeds; ++i)
                salts[(size_t)i] = sample_salt(seed0 + (uint64_t)k * (uint64_t)num_seeds + (uint64_t)i);
            count_batch(g, sampled, keep_threshold(p), salts.data(), num_seeds, cfg, (hipStream_t)stream, res);
            tc_stage st{};
            st.p = p;
            st.estimate = median_of_means(res, num_groups, p);
            for (const tc_counts& c : res) st.m_sum += c.m;
            stages[k] = st;
            *num_stages = k + 1;
            if (p >= 1.0 || (k >= 1 && st.estimate > 0.0 && std::fabs(st.estimate - prev) <= tol * st.estimate)) break;
            prev = st.estimate;
        }
        if (p_balance) {
            const double E = stages[*num_stages - 1].estimate;
            double pb = 1.0;
            if (E > 0.0 && tol > 0.0) {
                const double x = std::sqrt((double)g->m) * std::log((double)g->n) / (E * (tol * tol));
                pb = std::min(1.0, std::pow(x, 0.4));
            }
            *p_balance = pb;
        }
    });
}

tc_status tc_triple_estimate(tc_graph g, double p, uint64_t sample_seed, int32_t hybrid, int64_t num_samples,
                             uint64_t triple_seed, void* stream, tc_triple_result* out) {
    return guarded([&] {
        if (!g || !out) fail(TC_ERR_INVALID, "graph or output is NULL");
        if (!p_valid(p)) fail(TC_ERR_INVALID, "p must be finite and in (0, 1]");
        if (hybrid != 0 && hybrid != 1) fail(TC_ERR_INVALID, "hybrid must be 0 or 1");
        if (num_samples < 1) fail(TC_ERR_INVALID, "need at least one sample");
        hipStream_t s = (hipStream_t)stream;
        tc_graph gs = g;
        if (p < 1.0) {
            const tc_status st = tc_sample(g, p, sample_seed, stream, &gs);
            if (st != TC_OK) fail(st, tc_last_error());
        }
        tc_triple_result r{};
        try {
            triple_sample(gs, hybrid, num_samples, triple_seed, s, &r.size, &r.weight_sum, &r.closed);
        } catch (...) {
            if (gs != g) tc_graph_free(gs);
            throw;
        }
        r.m = gs->m;
        if (gs != g) tc_graph_free(gs);
        volatile double num = (double)r.size * (double)r.weight_sum;
        volatile double den = 60.0 * (double)num_samples;
        volatile double t = num / den;
        volatile double p2 = p * p;
        volatile double p3 = p2 * p;
        r.estimate = t / p3;
        *out = r;
    });
}

tc_status tc_rp_trace(tc_graph g, int32_t k, uint64_t seed, void* stream, int64_t* q, double* tri_est) {
    return guarded([&] {
        if (!g || !q) fail(TC_ERR_INVALID, "graph or q is NULL");
        if (k < 1) fail(TC_ERR_INVALID, "k must be >= 1");
        std::vector<int64_t> hq((size_t)k);
        rp_trace(g, k, seed, (hipStream_t)stream, hq.data());
        __int128 tot = 0;
        for (int32_t l = 0; l < k; ++l) tot += hq[(size_t)l];
        std::memcpy(q, hq.data(), sizeof(int64_t) * (size_t)k);
        if (tri_est) *tri_est = (double)tot / (6.0 * (double)k);
    });
}

static CountConfig from_tuning(const tc_tuning* t) {
    CountConfig c;
    check_heavy_multiplier(t->heavy_num, t->heavy_den);
    if (t->small_dmax < 1 || t->small_dmax > 128) fail(TC_ERR_INVALID, "small_dmax must be in [1, 128]");
    if (t->vmajor_cap < 0) fail(TC_ERR_INVALID, "vmajor_cap must be >= 0");
    if (t->blocks_per_cu < 1 || t->blocks_per_cu > 16) fail(TC_ERR_INVALID, "blocks_per_cu must be in [1, 16]");
    c.heavy_num = t->heavy_num;
    c.heavy_den = t->heavy_den;
    c.small_dmax = t->small_dmax;
    c.vmajor_cap = t->vmajor_cap;
    c.light_blocks_per_cu = t->blocks_per_cu;
    return c;
}

static void to_tuning(const CountConfig& c, tc_tuning* t) {
    t->heavy_num = c.heavy_num;
    t->heavy_den = c.heavy_den;
    t->small_dmax = c.small_dmax;
    t->vmajor_cap = c.vmajor_cap;
    t->blocks_per_cu = c.light_blocks_per_cu;
}

tc_status tc_tune_set(tc_graph g, double p, const tc_tuning* t) {
    return guarded([&] {
        if (!g || !t) fail(TC_ERR_INVALID, "graph or tuning is NULL");
        if (!p_valid(p)) fail(TC_ERR_INVALID, "p must be finite and in (0, 1]");
        tune_store(g, p < 1.0 ? 1 : 0, p, from_tuning(t));
    });
}

tc_status tc_tune_get(tc_graph g, double p, tc_tuning* t) {
    return guarded([&] {
        if (!g || !t) fail(TC_ERR_INVALID, "graph or tuning is NULL");
        if (!p_valid(p)) fail(TC_ERR_INVALID, "p must be finite and in (0, 1]");
        CountConfig c;
        tune_lookup(g, p < 1.0 ? 1 : 0, p, &c);
        to_tuning(c, t);
    });
}

tc_status tc_autotune(tc_graph g, double p, uint64_t seed, int32_t search_heavy, void* stream, tc_tuning* best) {
    return guarded([&] {
        if (!g) fail(TC_ERR_INVALID, "graph is NULL");
        if (!p_valid(p)) fail(TC_ERR_INVALID, "p must be finite and in (0, 1]");
        const int sampled = p < 1.0 ? 1 : 0;
        CountConfig c =
            autotune(g, sampled, p, keep_threshold(p), sample_salt(seed), search_heavy, (hipStream_t)stream);
        if (best) to_tuning(c, best);
    });
}

void tc_graph_free(tc_graph g) {
    if (!g) return;
    try {
        (void)hipStreamSynchronize(g->home);
        graph_release(g);
    } catch (...) {
    }
}

const char* tc_last_error(void) { return g_last_error.c_str(); }

tc_status tc_profile_enable(int32_t on) {
    return guarded([&] {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_on = on != 0;
    });
}

tc_status tc_profile_select(const char* names) {
    return guarded([&] {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_names.clear();
        if (!names) return;
        std::string cur;
        for (const char* c = names;; ++c) {
            if (*c == ',' || *c == 0) {
                if (!cur.empty()) g_prof_names.push_back(cur);
                cur.clear();
                if (*c == 0) break;
            } else {
                cur.push_back(*c);
            }
        }
    });
}

tc_status tc_profile_reset(void) {
    return guarded([&] {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof.clear();
    });
}

tc_status tc_profile_read(const char* kernel, double* total_ms, int64_t* launches) {
    return guarded([&] {
        if (!kernel) fail(TC_ERR_INVALID, "kernel name is NULL");
        std::lock_guard<std::mutex> lk(g_prof_mu);
        auto it = g_prof.find(kernel);
        if (total_ms) *total_ms = it == g_prof.end() ? 0.0 : it->second.first;
        if (launches) *launches = it == g_prof.end() ? 0 : it->second.second;
    });
}

}  // extern "C"
