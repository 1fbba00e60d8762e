// Internal declarations shared by the HIP translation units of libtc.
// Device code targets gfx950 only: wave64, 160 KB LDS per CU, int8 MFMA.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>

#include "../../include/tc.h"

namespace tc {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Host side: status plumbing
// ---------------------------------------------------------------------------

struct Error {
    tc_status status;
    std::string msg;
};

// Thrown inside the library only; every extern "C" entry point catches it.
[[noreturn]] void fail(tc_status st, const std::string& msg);
void check_hip(hipError_t e, const char* what);
// Text returned by tc_last_error() on the calling thread.
void set_last_error(const std::string& msg);

// A sub-allocator that the calling thread's device allocations go to first
// (a serving request's reservation).  try_alloc returns nullptr when full, and
// the allocation then falls back to the installed allocator (counted in
// spilled); try_free returns false for pointers it does not own.
struct AllocRegion {
    int64_t spilled = 0;
    bool strict = false;  // a failed try_alloc is an error instead of a spill
    virtual void* try_alloc(size_t bytes) = 0;
    virtual bool try_free(void* p) = 0;
    virtual ~AllocRegion() = default;
};
// Install r for the calling thread (nullptr: none); returns the previous one.
AllocRegion* set_thread_region(AllocRegion* r);

// Device allocation through the installed allocator (throws TC_ERR_OOM).
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);

// Bytes a single allocation of b bytes takes in a reservation (256-byte granules).
inline int64_t region_bytes(int64_t b) { return ((b > 0 ? b : 1) + 255) / 256 * 256; }

// RAII device buffer.
template <typename T>
struct DevBuf {
    T* ptr = nullptr;
    size_t count = 0;
    hipStream_t stream = nullptr;
    DevBuf() = default;
    DevBuf(size_t n, hipStream_t s) { reset(n, s); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), count(o.count), stream(o.stream) { o.ptr = nullptr; o.count = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); ptr = o.ptr; count = o.count; stream = o.stream; o.ptr = nullptr; o.count = 0; }
        return *this;
    }
    void reset(size_t n, hipStream_t s) {
        release();
        stream = s;
        count = n;
        ptr = static_cast<T*>(dev_alloc((n ? n : 1) * sizeof(T), s));
    }
    void release() {
        if (ptr) dev_free(ptr, stream);
        ptr = nullptr;
        count = 0;
    }
    T* get() const { return ptr; }
};

// ---------------------------------------------------------------------------
// Profiling of launches (events on the launch stream)
// ---------------------------------------------------------------------------

// While alive on a thread, launches of that thread record no profiling events.
struct NoProfileScope {
    bool prev;
    NoProfileScope();
    ~NoProfileScope();
};

// While alive on a thread, profiled launches of that thread are also
// accumulated under "@<phase>" (the step of the path they belong to).
struct PhaseScope {
    const char* prev;
    explicit PhaseScope(const char* phase);
    ~PhaseScope();
};

struct LaunchScope {
    const char* name;
    const char* phase;
    hipStream_t stream;
    void* ev0 = nullptr;
    LaunchScope(const char* n, hipStream_t s);
    ~LaunchScope();
};

// Resolve recorded events into per-kernel totals (call after the stream is synchronised).
void profile_collect();

#define TC_LAUNCH(name, kernel, grid, block, shmem, stream, ...)                           \
    do {                                                                                    \
        ::tc::LaunchScope _tc_scope((name), (stream));                                      \
        hipLaunchKernelGGL(kernel, (grid), (block), (shmem), (stream), __VA_ARGS__);        \
        ::tc::check_hip(hipGetLastError(), (name));                                         \
    } while (0)

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Graph handle
// ---------------------------------------------------------------------------

}  // namespace tc

struct tc_graph_s {
    int64_t n = 0;
    int64_t m = 0;            // undirected edges
    int32_t max_deg = 0;
    int32_t* row_ptr = nullptr;   // [n+1]
    int32_t* col = nullptr;       // [2m]
    int32_t* src = nullptr;       // [2m] row index of each CSR entry
    int32_t* deg = nullptr;       // [n]
    uint8_t* ncls = nullptr;      // [2m] degree class of each entry's neighbour (graphs built by build_csr)
    hipStream_t home = nullptr;   // stream the buffers were allocated on
};

namespace tc {

// ---------------------------------------------------------------------------
// Device-wide primitives (tc_scan.hip)
// ---------------------------------------------------------------------------

// Exclusive scan of in[0..N) into out[0..N], out[N] = total.  In-place allowed.
void scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t N, hipStream_t s);
// four arrays of one length with the launches of one scan
void scan_exclusive_i32_x4(const int32_t* const in[4], int32_t* const out[4], int64_t N, hipStream_t s);
// Bytes the scratch of one scan of N elements takes (sum of its allocations).
int64_t scan_scratch_bytes(int64_t N);
int64_t scan_x4_scratch_bytes(int64_t N);

// Triple sampling (tc_triple.hip): |U|, the weight sum and the closed
// samples of num_samples samples of g's candidate triples.
void triple_sample(const tc_graph_s* g, int hybrid, int64_t num_samples, uint64_t seed, hipStream_t s,
                   int64_t* size, int64_t* wsum, int64_t* closed);
// exclusive scan of int64 values: out[0..N), out[N] = total (tc_triple.hip)
void scan64(const int64_t* in, int64_t* out, int64_t N, hipStream_t s);
void fill_i32(int32_t* p, int32_t v, int64_t N, hipStream_t s);
void fill_i64(int64_t* p, int64_t v, int64_t N, hipStream_t s);
void fill_u8(uint8_t* p, uint8_t v, int64_t N, hipStream_t s);

// ---------------------------------------------------------------------------
// CSR build (tc_csr.hip)
// ---------------------------------------------------------------------------

// Build into g (allocations through dev_alloc).  Returns 0 or 1 if an id is out of range.
int build_csr(int64_t n, int64_t num_pairs, const int32_t* src_dev, const int32_t* dst_dev,
              hipStream_t s, tc_graph_s* g);
// Sum of the sizes of every allocation build_csr makes (region_bytes each).
int64_t build_csr_bytes(int64_t n, int64_t num_pairs);
// g->ncls of a built graph: the degree class of every entry's neighbour, so
// that the orientation of the graph itself reads it in order instead of
// gathering it per entry (tc_count.hip)
void neighbour_classes(tc_graph_s* g, hipStream_t s);

// ---------------------------------------------------------------------------
// Sampling (tc_sample.hip)
// ---------------------------------------------------------------------------

uint64_t keep_threshold(double p);
uint64_t sample_salt(uint64_t seed);

// keep bits (one uint64 per 64 CSR entries) and per-word popcounts
void sample_keep_bits(const tc_graph_s* g, uint64_t salt, uint64_t thr, uint64_t* bits, int32_t* wcnt,
                      hipStream_t s);
// the same with the kept entries staged per range of 512 entries (st_col,
// st_src: E2 entries each), then moved into place by move_staged once wcnt
// is scanned into wpre
void sample_keep_staged(const tc_graph_s* g, uint64_t salt, uint64_t thr, uint64_t* bits, int32_t* wcnt,
                        int32_t* st_col, int32_t* st_src, hipStream_t s);
void move_staged(int64_t E2, const int32_t* wpre, const int32_t* st_col, const int32_t* st_src, int32_t* col_out,
                 int32_t* src_out, hipStream_t s);
// rank of CSR position e among kept entries, for every row start: rp_out[x] (x in [0,n])
void positions_at_rows(const int32_t* row_ptr, int64_t n, int64_t E2, const uint64_t* bits,
                       const int32_t* wpre, int32_t* rp_out, int32_t* deg_out, hipStream_t s);
// compaction of kept entries (col and src, each optional on output); E2 bounds
// the buffers, E2_dev (if not null) the entries that can have bits set
void compact_kept(const int32_t* col, const int32_t* src, int64_t E2, const uint64_t* bits,
                  const int32_t* wpre, int32_t* col_out, int32_t* src_out, hipStream_t s,
                  const int32_t* E2_dev = nullptr);

// ---------------------------------------------------------------------------
// Counting core (tc_count.hip)
// ---------------------------------------------------------------------------

struct CountConfig {
    int32_t heavy_num = 1, heavy_den = 1;
    int32_t small_dmax = 128;        // anchors with d+ <= small_dmax use a wave each, others a block
    int32_t vmajor_cap = 1024;       // pairs with d+(u) <= d+(v) <= cap are closed from v's side (0: never)
    int32_t light_blocks_per_cu = 8; // persistent grid of the wave-per-item kernel
};

// Device result slots of one count (int64 each).
constexpr int kCountSlots = 16;

// Enqueue the exact count of the graph, or of its copy sampled with (thr, salt)
// if sampled != 0, on stream s without any host synchronisation; the result
// lands in acc[kCountSlots] (device).  Launch sizes come from host-side bounds.
void count_enqueue(const tc_graph_s* g, int sampled, uint64_t thr, uint64_t salt, const CountConfig& cfg,
                   hipStream_t s, int64_t* acc);

// A graph that is the disjoint union of K components (independent samples of
// one graph, or several requests' graphs): vertex x belongs to component
// comp[x], component k owns the vertices [off[k], off[k+1]) and every off[k]
// is a multiple of kUnionAlign, so that aligned vertex windows of the count
// kernels never straddle two components.  mk[k] = edges of component k.  All
// arrays are device arrays.
constexpr int kUnionAlign = 256;
struct CountUnion {
    int32_t K = 1;
    const int32_t* comp = nullptr;  // [n]
    const int32_t* off = nullptr;   // [K + 1]
    const int64_t* mk = nullptr;    // [K]
};

// The exact count of every component of the (unsampled) union graph g with
// one pass of the count's kernels: component k's results land in
// acc[k * kCountSlots ..] (device, K * kCountSlots slots), equal to a count of
// that component alone.  Synchronises s once (to size the heavy block).
void count_union(const tc_graph_s* g, const CountUnion& un, const CountConfig& cfg, hipStream_t s, int64_t* acc);
// An upper bound of the sum of the sizes of every allocation count_union
// makes for a union of K components, n vertices, m edges, maximum degree maxd,
// at most h heavy vertices in all, heavy blocks of at most ubytes bytes and at
// most ntiles macro tiles.
int64_t count_union_bytes(int64_t n, int64_t m, int32_t maxd, int32_t K, int64_t h, int64_t ubytes, int64_t ntiles,
                          const CountConfig& cfg);

// Union of K independent samples of g (keep probability thr, salts[k] device
// array): component k is g sampled with salts[k], its vertex x is union vertex
// k * n_pad + x (n_pad = n rounded up to kUnionAlign).  Builds the union's CSR
// into *out (allocations through dev_alloc, released by graph_release) and
// the comp / off / mk arrays (owned by the caller's buffers: comp[K * n_pad],
// off[K + 1], mk[K]).  Synchronises s once (to size the sampled CSR).
void sample_union_replicas(const tc_graph_s* g, int32_t K, const uint64_t* salts, uint64_t thr, hipStream_t s,
                           tc_graph_s* out, int32_t* comp, int32_t* off, int64_t* mk);
// Union of the components of the graph gU (vertex ranges off[k]..off[k+1]
// given in comp / off, device), component k sampled with (thrs[k], salts[k])
// on its local ids x - off[k]; writes the sampled CSR to *out and mk.
// Synchronises s once.
// comp[x] for x < n from the component starts off[K + 1] (device)
void comp_from_offsets(int64_t n, int32_t K, const int32_t* off, int32_t* comp, hipStream_t s);
void sample_union_components(const tc_graph_s* gU, int32_t K, const int32_t* comp, const int32_t* off,
                             const uint64_t* salts, const uint64_t* thrs, hipStream_t s, tc_graph_s* out,
                             int64_t* mk);
void counts_from_slots(const int64_t* hacc, tc_counts* out);
// Sum of the sizes of every allocation count_core makes (region_bytes each) on
// a graph of n vertices, m edges and maximum degree maxd.
int64_t count_bytes(int64_t n, int64_t m, int32_t maxd, int sampled, const CountConfig& cfg);
// count_enqueue + read-back (synchronises s).
void count_core(const tc_graph_s* g, int sampled, uint64_t thr, uint64_t salt, const CountConfig& cfg,
                hipStream_t s, tc_counts* out);

// ---------------------------------------------------------------------------
// Random projection (tc_rp.hip)
// ---------------------------------------------------------------------------

void rp_trace(const tc_graph_s* g, int32_t k, uint64_t seed, hipStream_t s, int64_t* q_host);

// ---------------------------------------------------------------------------
// Host helpers of the entry points (tc_api.hip)
// ---------------------------------------------------------------------------

bool p_valid(double p);
// largest heavy_num / heavy_den accepted (the heavy test is exact up to it)
constexpr int32_t kHeavyTermMax = 1 << 15;
void check_heavy_multiplier(int32_t num, int32_t den);
CountConfig config_from(const tc_params* prm, const tc_graph_s* g, int sampled, double p);
double rescale(int64_t T, double p);
int32_t max_degree(const tc_graph_s* g, hipStream_t s);
void graph_release(tc_graph_s* g);
// CSR of the pairs (host arrays copied in unless on_device); throws on error.
tc_graph_s* graph_from_pairs(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst, int on_device,
                             hipStream_t s);
int num_cus();

// Autotuned parameters for a graph signature (tc_tune.hip)
CountConfig tuned_config(const tc_graph_s* g, int sampled, double p, const CountConfig& base);
void tune_store(const tc_graph_s* g, int sampled, double p, const CountConfig& c);
bool tune_lookup(const tc_graph_s* g, int sampled, double p, CountConfig* c);
CountConfig autotune(const tc_graph_s* g, int sampled, double p, uint64_t thr, uint64_t salt, int search_heavy,
                     hipStream_t s);

}  // namespace tc
