// Semi-streaming variant (section 5.2): three passes over the edges, with the
// adjacency lists in order.
//
//   pass 1: s1 = ceil(d m^(1/2) ln n) edges drawn uniformly with replacement
//           (the Lemma of section 5.2); their endpoints are the heavy
//           candidates, and those above the degree split (deg^2 > m) form H;
//   pass 2: s draws with replacement from U = L followed by X, where L holds
//           the wedges at the vertices outside H (vertices ascending, pairs of
//           neighbour positions in colex order) and X the pairs (h; e) of a
//           vertex of H and an edge (h ascending, edges in (v, w) order,
//           v < w); a draw asks for its closing edges: one for a wedge, two
//           for a pair whose vertex is not in its edge (none otherwise: never
//           closed).  The asked-for edges go into a hash table;
//   pass 3: one pass over the edges marks every asked-for edge that exists;
//           a draw is closed iff all its edges are marked.
//
// Every triangle has exactly three closed elements in U, one per vertex, so
// |U| closed / (3 s) estimates t.  Draw i of pass 1 is upper edge
// floor(h m / 2^64), h = mix64(mix64(i) ^ mix64(seed ^ "TC_STRM1")); draw j of
// pass 2 is element floor(h' |U| / 2^64), h' = mix64(mix64(j) ^
// mix64(seed ^ "TC_STRM2")).
#include "tc_internal.h"
#include "tc_device.h"

#include <cmath>

namespace tc {

namespace {

uint64_t host_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

constexpr uint64_t kEmpty = ~0ull;        // an empty slot of the query table
constexpr uint64_t kFound = 1ull << 63;   // set on a slot whose edge exists (ids < 2^31 leave bit 63 free)

__device__ __forceinline__ int64_t hi_mul(uint64_t h, uint64_t size) { return (int64_t)__umul64hi(h, size); }

// Sum of v over the block (256 threads) added to *acc by one atomic.
__device__ __forceinline__ void block_add(int64_t v, unsigned long long* acc) {
    __shared__ int64_t red[4];
    v = wave_sum(v);
    __syncthreads();  // red may still be read by a previous call
    if (__lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t t = red[0] + red[1] + red[2] + red[3];
        if (t) atomicAdd(acc, (unsigned long long)t);
    }
}

// up[u] = neighbours of u above u (sorted list: the first position holding an id > u)
__global__ void k_up_deg(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                         int32_t* __restrict__ up) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = rp[u], hi = rp[u + 1];
        const int32_t end = hi;
        while (lo < hi) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if (col[mid] <= (int32_t)u) lo = mid + 1;
            else hi = mid;
        }
        up[u] = end - lo;
    }
}

// A non-decreasing prefix pre[0..n] (pre[0] = 0, pre[n] = total) with an
// index of 2^k buckets: bucket b starts at position floor(b total / 2^k), and
// idx[b] is the item u whose range [pre[u], pre[u+1]) holds that position.
// The item of a position r in bucket b lies between idx[b] and idx[b+1], so
// its search takes a few steps instead of log2 n dependent loads.
template <typename T>
struct PrefixIndex {
    const T* pre;         // n + 1 entries on the device; total = pre[n]
    const int32_t* idx;   // 2^k entries
    int64_t n;
    int k;
};

// Bucket starts floor(b total / 2^k) = b q + floor(b rem / 2^k) with
// q = total >> k and rem = total mod 2^k: b, rem < 2^26, so b rem < 2^52.
struct Buckets {
    uint64_t q, rem;
    int k;
    __device__ __forceinline__ Buckets(uint64_t total, int k_) : q(total >> k_), rem(total & ((1ull << k_) - 1)), k(k_) {}
    __device__ __forceinline__ uint64_t start(uint64_t b) const { return b * q + ((b * rem) >> k); }
};

// the last bucket starting at or before r (r < total)
__device__ __forceinline__ int64_t bucket_of(uint64_t r, uint64_t total, int k) {
    const Buckets bs(total, k);
    const int64_t B = (int64_t)1 << k;
    int64_t b = (int64_t)((double)r / (double)total * (double)B);  // then made exact
    b = b < 0 ? 0 : (b > B - 1 ? B - 1 : b);
    while (b > 0 && bs.start((uint64_t)b) > r) --b;
    while (b + 1 < B && bs.start((uint64_t)(b + 1)) <= r) ++b;
    return b;
}

// the first bucket starting at or after x (B if none)
__device__ __forceinline__ int64_t first_bucket_at(uint64_t x, uint64_t total, int k) {
    const Buckets bs(total, k);
    const int64_t B = (int64_t)1 << k;
    int64_t b = (int64_t)ceil((double)x / (double)total * (double)B);  // then made exact
    b = b < 0 ? 0 : (b > B ? B : b);
    while (b > 0 && bs.start((uint64_t)(b - 1)) >= x) --b;
    while (b < B && bs.start((uint64_t)b) < x) ++b;
    return b;
}

// the item u with pre[u] <= r < pre[u+1] (the last u with pre[u] <= r), 0 <= r < total
template <typename T>
__device__ __forceinline__ int64_t find_item(const PrefixIndex<T>& P, int64_t r) {
    const int64_t B = (int64_t)1 << P.k;
    const int64_t b = bucket_of((uint64_t)r, (uint64_t)P.pre[P.n], P.k);
    int64_t lo = P.idx[b], hi = b + 1 < B ? P.idx[b + 1] : P.n - 1;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo + 1) >> 1);
        if ((int64_t)P.pre[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// idx of a prefix: every bucket start lies in exactly one non-empty range, and
// the item of that range writes it.  Items with at most 8 buckets write their
// own; the wave writes those of longer ranges together, one item at a time.
template <typename T>
__global__ void __launch_bounds__(256) k_bucket_index(int64_t n, const T* __restrict__ pre, int k,
                                                      int32_t* __restrict__ idx) {
    const uint64_t total = (uint64_t)pre[n];
    if (total == 0) return;
    const Buckets bs(total, k);
    const int lane = __lane_id();
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); u0 < n; u0 += step) {
        // u0 is the wave's first item (wave-uniform), u this lane's
        const int64_t u = u0 + lane;
        int64_t b0 = 0, b1 = 0;
        if (u < n) {
            const uint64_t a = (uint64_t)pre[u], e = (uint64_t)pre[u + 1];
            if (a != e) {
                b0 = first_bucket_at(a, total, k);
                b1 = first_bucket_at(e, total, k);
            }
        }
        const bool mine = b1 - b0 <= 8;
        if (mine)
            for (int64_t b = b0; b < b1; ++b) idx[b] = (int32_t)u;
        uint64_t longs = ballot64(!mine);
        while (longs) {
            const int src = __ffsll((long long)longs) - 1;
            longs &= longs - 1;
            const int64_t lb0 = __shfl(b0, src, 64), lb1 = __shfl(b1, src, 64);
            for (int64_t b = lb0 + lane; b < lb1; b += 64) idx[b] = (int32_t)(u0 + src);
        }
    }
}

// (u, v) of upper edge r (P: the prefix of the neighbours above each vertex)
__device__ __forceinline__ void upper_edge(const PrefixIndex<int32_t>& P, const int32_t* __restrict__ rp,
                                           const int32_t* __restrict__ col, int64_t r, int32_t& u, int32_t& v) {
    const int64_t x = find_item(P, r);
    const int32_t deg = rp[x + 1] - rp[x];
    const int32_t upd = P.pre[x + 1] - P.pre[x];
    u = (int32_t)x;
    v = col[rp[x] + (deg - upd) + (int32_t)(r - P.pre[x])];
}

// pass 1: the endpoints of s1 drawn edges
__global__ void k_stream_draw_edges(int64_t s1, uint64_t salt, int64_t m, const int32_t* __restrict__ rp,
                                    const int32_t* __restrict__ col, PrefixIndex<int32_t> up,
                                    uint8_t* __restrict__ cand) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s1; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t u, v;
        upper_edge(up, rp, col, hi_mul(mix64(mix64((uint64_t)i) ^ salt), (uint64_t)m), u, v);
        cand[u] = 1;
        cand[v] = 1;
    }
}

// H flags (candidates above the split) and the wedge count of every vertex
// outside H; acc[0] += candidates
__global__ void k_stream_classify(int64_t n, int64_t m, const uint8_t* __restrict__ cand,
                                  const int32_t* __restrict__ deg, int32_t* __restrict__ hf,
                                  int64_t* __restrict__ lc, unsigned long long* __restrict__ acc) {
    int64_t nc = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = deg[x];
        const bool c = cand[x] != 0;
        const bool h = c && d * d > m;  // the degree split of section 3.2 (c = 1)
        nc += c;
        hf[x] = h;
        lc[x] = h ? 0 : d * (d - 1) / 2;
    }
    block_add(nc, &acc[0]);
}

__global__ void k_stream_hlist(int64_t n, const int32_t* __restrict__ hf, const int32_t* __restrict__ hpos,
                               int32_t* __restrict__ hlist) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        if (hf[x]) hlist[hpos[x]] = (int32_t)x;
}

__device__ __forceinline__ uint64_t edge_key(int32_t a, int32_t b) {
    const uint64_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
    return (lo << 32) | hi;
}

// The query table: open addressing over 2^lg slots of 64-bit keys, home slot
// mix64(key) mod 2^lg, at most half of the slots used.
struct QueryTable {
    unsigned long long* tab;
    int lg;
    __device__ __forceinline__ uint64_t mask() const { return (1ull << lg) - 1; }
};

// the slot of key in the query table (inserted if absent)
__device__ __forceinline__ int32_t table_insert(const QueryTable& T, uint64_t key) {
    uint64_t slot = mix64(key) & T.mask();
    while (true) {
        const unsigned long long prev = atomicCAS(&T.tab[slot], (unsigned long long)kEmpty, (unsigned long long)key);
        if (prev == kEmpty || prev == key) return (int32_t)slot;
        slot = (slot + 1) & T.mask();
    }
}

// pass 2: draw j's element of U and the slots of its closing edges (-1: none,
// -2: drawn but never closed)
__global__ void __launch_bounds__(256) k_stream_draw_triples(int64_t s, uint64_t salt, int64_t m,
                                                             const int32_t* __restrict__ rp,
                                                             const int32_t* __restrict__ col, PrefixIndex<int32_t> up,
                                                             PrefixIndex<int64_t> light,
                                                             const int32_t* __restrict__ hlist,
                                                             const int32_t* __restrict__ hcount, QueryTable T,
                                                             int2* __restrict__ q) {
    const int64_t L = light.pre[light.n];
    const int64_t size = L + (int64_t)hcount[0] * m;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < s; j += (int64_t)gridDim.x * blockDim.x) {
        int2 slots = make_int2(-1, -1);
        if (size > 0) {
            const int64_t r = hi_mul(mix64(mix64((uint64_t)j) ^ salt), (uint64_t)size);
            if (r < L) {  // wedge k of light vertex u: pair (a, b) of colex order
                const int64_t u = find_item(light, r);
                const int64_t k = r - light.pre[u];
                int64_t b = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)k)) * 0.5);  // then made exact
                while (b > 1 && b * (b - 1) / 2 > k) --b;
                while ((b + 1) * b / 2 <= k) ++b;
                const int64_t a = k - b * (b - 1) / 2;
                slots.x = table_insert(T, edge_key(col[rp[u] + a], col[rp[u] + b]));
            } else {  // the pair of heavy vertex h and upper edge (v, w)
                const int64_t qq = r - L;
                const int32_t h = hlist[qq / m];
                int32_t v, w;
                upper_edge(up, rp, col, qq % m, v, w);
                if (h != v && h != w) {
                    slots.x = table_insert(T, edge_key(h, v));
                    slots.y = table_insert(T, edge_key(h, w));
                } else {
                    slots = make_int2(-2, -2);  // drawn, never closed, no query
                }
            }
        }
        q[j] = slots;
    }
}

// pass 3: every edge of the stream (upper entries) marks its slot if asked for
__global__ void __launch_bounds__(256) k_stream_mark(int64_t E2, const int32_t* __restrict__ src,
                                                     const int32_t* __restrict__ col, QueryTable T) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E2; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = src[e], v = col[e];
        if (u >= v) continue;  // each undirected edge once
        const uint64_t key = edge_key(u, v);
        uint64_t slot = mix64(key) & T.mask();
        while (true) {
            const uint64_t t = T.tab[slot];
            if (t == kEmpty) break;
            if ((t & ~kFound) == key) {
                if (!(t & kFound)) T.tab[slot] = key | kFound;  // only this edge's lookups write this slot
                break;
            }
            slot = (slot + 1) & T.mask();
        }
    }
}

// acc[1] += closed draws, acc[2] += closing-edge lookups
__global__ void k_stream_count(int64_t s, const int2* __restrict__ q, const unsigned long long* __restrict__ tab,
                               unsigned long long* __restrict__ acc) {
    int64_t closed = 0, queries = 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < s; j += (int64_t)gridDim.x * blockDim.x) {
        const int2 sl = q[j];
        if (sl.x == -2 || sl.x == -1) continue;  // never closed / no element
        const bool f0 = (tab[sl.x] & kFound) != 0;
        if (sl.y < 0) {
            queries += 1;
            closed += f0;
        } else {
            queries += 2;
            closed += f0 && (tab[sl.y] & kFound) != 0;
        }
    }
    block_add(closed, &acc[1]);
    block_add(queries, &acc[2]);
}

unsigned grid(int64_t N, int64_t cap = 65536) {
    int64_t b = (N + 255) / 256;
    if (b > cap) b = cap;
    return (unsigned)(b > 0 ? b : 1);
}

// kernels that reduce into one counter: a few resident rounds of blocks, so
// that the counter takes about a thousand atomics
constexpr int64_t kReduceBlocks = 1024;

}  // namespace

int64_t stream_draws(int64_t n, int64_t m, double d) {
    if (n < 2 || m < 1) return 0;
    return (int64_t)std::ceil(d * std::sqrt((double)m) * std::log((double)n));
}

void stream_estimate(const tc_graph_s* g, double d, int64_t s, uint64_t seed, hipStream_t st, tc_stream_result* out) {
    const int64_t n = g->n, m = g->m, E2 = 2 * m;
    tc_stream_result r{};
    r.m = m;
    r.draws1 = stream_draws(n, m, d);
    if (n < 2 || m < 1) {
        *out = r;
        return;
    }
    PhaseScope ph("stream");
    // the upper entries' prefix: edge r of the stream
    DevBuf<int32_t> upre(n + 1, st);
    TC_LAUNCH("stream_up", k_up_deg, dim3(grid(n)), dim3(256), 0, st, n, (const int32_t*)g->row_ptr,
              (const int32_t*)g->col, upre.get());
    scan_exclusive_i32(upre.get(), upre.get(), n, st);
    // bucket indexes of the two prefixes that draws are searched in
    int k = 10;
    while (k < 26 && ((int64_t)1 << k) < n) ++k;
    const int64_t B = (int64_t)1 << k;
    DevBuf<int32_t> up_idx(B, st), light_idx(B, st);
    TC_LAUNCH("stream_index", k_bucket_index<int32_t>, dim3(grid(n)), dim3(256), 0, st, n,
              (const int32_t*)upre.get(), k, up_idx.get());
    const PrefixIndex<int32_t> up{upre.get(), up_idx.get(), n, k};
    // pass 1
    DevBuf<uint8_t> cand(n, st);
    fill_u8(cand.get(), 0, n, st);
    const uint64_t salt1 = host_mix(seed ^ 0x54435F5354524D31ULL);  // "TC_STRM1"
    if (r.draws1 > 0)
        TC_LAUNCH("stream_pass1", k_stream_draw_edges, dim3(grid(r.draws1)), dim3(256), 0, st, r.draws1, salt1, m,
                  (const int32_t*)g->row_ptr, (const int32_t*)g->col, up, cand.get());
    DevBuf<int32_t> hf(n + 1, st), hpos(n + 1, st);
    DevBuf<int64_t> lc(n + 1, st), lpre(n + 1, st);
    DevBuf<unsigned long long> acc(3, st);
    fill_i64(reinterpret_cast<int64_t*>(acc.get()), 0, 3, st);
    TC_LAUNCH("stream_classify", k_stream_classify, dim3(grid(n, kReduceBlocks)), dim3(256), 0, st, n, m,
              (const uint8_t*)cand.get(), (const int32_t*)g->deg, hf.get(), lc.get(), acc.get());
    scan_exclusive_i32(hf.get(), hpos.get(), n, st);
    scan64(lc.get(), lpre.get(), n, st);
    DevBuf<int32_t> hlist(n, st);
    TC_LAUNCH("stream_hlist", k_stream_hlist, dim3(grid(n)), dim3(256), 0, st, n, (const int32_t*)hf.get(),
              (const int32_t*)hpos.get(), hlist.get());
    TC_LAUNCH("stream_index", k_bucket_index<int64_t>, dim3(grid(n)), dim3(256), 0, st, n,
              (const int64_t*)lpre.get(), k, light_idx.get());
    const PrefixIndex<int64_t> light{lpre.get(), light_idx.get(), n, k};
    // passes 2 and 3: a table of at least twice as many slots as lookups
    int lg = 10;
    while (((int64_t)1 << lg) < 4 * s) ++lg;
    const int64_t cap = (int64_t)1 << lg;
    DevBuf<unsigned long long> tab(cap, st);
    fill_i64(reinterpret_cast<int64_t*>(tab.get()), -1, cap, st);
    const QueryTable T{tab.get(), lg};
    DevBuf<int2> q(s > 0 ? s : 1, st);
    const uint64_t salt2 = host_mix(seed ^ 0x54435F5354524D32ULL);  // "TC_STRM2"
    if (s > 0) {
        TC_LAUNCH("stream_pass2", k_stream_draw_triples, dim3(grid(s)), dim3(256), 0, st, s, salt2, m,
                  (const int32_t*)g->row_ptr, (const int32_t*)g->col, up, light, (const int32_t*)hlist.get(),
                  (const int32_t*)hpos.get() + n, T, q.get());
        TC_LAUNCH("stream_pass3", k_stream_mark, dim3(grid(E2)), dim3(256), 0, st, E2, (const int32_t*)g->src,
                  (const int32_t*)g->col, T);
        TC_LAUNCH("stream_count", k_stream_count, dim3(grid(s, kReduceBlocks)), dim3(256), 0, st, s, (const int2*)q.get(),
                  (const unsigned long long*)tab.get(), acc.get());
    }
    int64_t h3[3], L = 0;
    int32_t H = 0;
    check_hip(hipMemcpyAsync(h3, acc.get(), sizeof(h3), hipMemcpyDeviceToHost, st), "stream counts");
    check_hip(hipMemcpyAsync(&H, hpos.get() + n, sizeof(int32_t), hipMemcpyDeviceToHost, st), "heavy count");
    check_hip(hipMemcpyAsync(&L, lpre.get() + n, sizeof(int64_t), hipMemcpyDeviceToHost, st), "light size");
    check_hip(hipStreamSynchronize(st), "sync");
    r.candidates = h3[0];
    r.heavy = H;
    r.light_size = L;
    r.size = L + (int64_t)H * m;
    r.closed = h3[1];
    r.queries = h3[2];
    if (s > 0) {
        volatile double num = (double)r.size * (double)r.closed;
        volatile double den = 3.0 * (double)s;
        r.estimate = num / den;
    }
    *out = r;
}

}  // namespace tc

using namespace tc;

extern "C" tc_status tc_stream_estimate(tc_graph g, double d, int64_t num_samples, uint64_t seed, void* stream,
                                        tc_stream_result* out) {
    try {
        set_last_error("");
        if (!g || !out) fail(TC_ERR_INVALID, "graph or output is NULL");
        if (!std::isfinite(d) || d <= 0.0) fail(TC_ERR_INVALID, "d must be finite and > 0");
        if (num_samples < 0) fail(TC_ERR_INVALID, "num_samples must be >= 0");
        if (num_samples > ((int64_t)1 << 28)) fail(TC_ERR_OVERFLOW, "num_samples exceeds 2^28");
        const int64_t s1 = stream_draws(g->n, g->m, d);
        if (s1 > ((int64_t)1 << 40)) fail(TC_ERR_OVERFLOW, "pass-1 draws exceed 2^40");
        tc_stream_result r;
        stream_estimate(g, d, num_samples, seed, (hipStream_t)stream, &r);
        *out = r;
        profile_collect();
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
