// Triple sampling (section 3.2, "Triple Sampling"; the Simple and Hybrid
// columns of Table 2) on the device.
//
// The candidate set U, in a fixed order: vertices u ascending; a vertex of
// the wedge kind contributes its pairs of neighbour positions (a, b), a < b,
// in colex order, the triple (N(u)[a], u, N(u)[b]); a vertex of the extension
// kind contributes, for each neighbour position a (v = N(u)[a]), each
// neighbour position j of v (w = N(v)[j]), the triple (u, v, w).  Simple:
// every vertex is of the wedge kind; hybrid: the extension kind iff
// deg^2 > m (the degree split of section 3.2).  A triangle appears once per
// wedge-kind and twice per extension-kind vertex, so a closed sample weighs
// 60 / (3 + its extension-kind vertices) and the weights of each triangle's
// appearances sum to 60: |U| * (sum of weights) / (60 s) estimates t.
//
//   1. per vertex, its number of triples: C(d, 2) (thread per vertex), or
//      the sum of its neighbours' degrees with, per list entry, the exclusive
//      prefix of that sum along the list (one wave per list);
//   2. their exclusive prefix (int64);
//   3. one thread per sample: index r = high half of h * |U| (h a 64-bit
//      counter hash of the sample number), its vertex by binary search over
//      the prefix, the pair by colex unranking or the list entry by binary
//      search over the entry prefix, and the closing edge by binary search in
//      the shorter sorted list.
#include "tc_internal.h"
#include "tc_device.h"

namespace tc {

namespace {

// SplitMix64's output function on the host (the device form is mix64)
uint64_t host_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ bool ext_kind(int hybrid, int64_t deg, int64_t m) { return hybrid && deg * deg > m; }

// per vertex of the wedge kind: C(d, 2); extension kind: 0 (k_tri_ext fills it)
__global__ void k_tri_counts(int64_t n, const int32_t* __restrict__ deg, int64_t m, int hybrid,
                             int64_t* __restrict__ cnt) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = deg[x];
        cnt[x] = ext_kind(hybrid, d, m) ? 0 : d * (d - 1) / 2;
    }
}

// extension-kind lists, one wave per list (64 consecutive vertices per step):
// EP[e] = sum of deg(N(u)[i]) over the entries i before e in u's list, and
// cnt[u] = the whole sum
__global__ void __launch_bounds__(256) k_tri_ext(int64_t n, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, const int32_t* __restrict__ deg,
                                                  int64_t m, int hybrid, int64_t* __restrict__ cnt,
                                                  int64_t* __restrict__ EP) {
    const int lane = __lane_id();
    const int64_t gw = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t x0 = gw * 64; x0 < n; x0 += nw * 64) {
        const int64_t x = x0 + lane;
        const int64_t d = x < n ? deg[x] : 0;
        uint64_t todo = ballot64(x < n && ext_kind(hybrid, d, m));
        while (todo) {
            const int l = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int32_t rs = rp[x0 + l], re = rp[x0 + l + 1];  // wave-uniform
            int64_t carry = 0;
            for (int32_t e0 = rs; e0 < re; e0 += 64) {
                const int32_t e = e0 + lane;
                const int64_t v = e < re ? (int64_t)deg[col[e]] : 0;
                const int64_t inc = wave_inclusive_sum(v);
                if (e < re) EP[e] = carry + inc - v;
                carry += __shfl(inc, 63, 64);
            }
            if (lane == 0) cnt[x0 + l] = carry;
        }
    }
}

// exclusive scan of int64 values: tiles of 2048 per block, then the tile sums
constexpr int kT64 = 256, kI64 = 8, kTile64 = kT64 * kI64;

__global__ void __launch_bounds__(kT64) k_scan64_tile(const int64_t* in, int64_t N, int64_t* out,
                                                       int64_t* __restrict__ bsum) {
    __shared__ int64_t tmp[kT64 / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kTile64 + (int64_t)threadIdx.x * kI64;
    int64_t v[kI64];
    int64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kI64; ++i) {
        v[i] = base + i < N ? in[base + i] : 0;
        acc += v[i];
    }
    int64_t total;
    int64_t pre = block_exclusive_sum<kT64>(acc, tmp, &total);
#pragma unroll
    for (int i = 0; i < kI64; ++i) {
        if (base + i < N) out[base + i] = pre;
        pre += v[i];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// adds each tile's offset (boff[tile], nb > 1) and writes the total to out[N]
__global__ void k_scan64_fin(int64_t* out, int64_t N, const int64_t* __restrict__ boff, int64_t nb) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= N; i += (int64_t)gridDim.x * blockDim.x) {
        if (i == N) out[N] = nb > 1 ? boff[nb] : boff[0];
        else if (nb > 1) out[i] += boff[i / kTile64];
    }
}

}  // namespace

void scan64(const int64_t* in, int64_t* out, int64_t N, hipStream_t s) {
    const int64_t nb = N > 0 ? (N + kTile64 - 1) / kTile64 : 1;
    DevBuf<int64_t> bs(nb + 1, s);
    TC_LAUNCH("tri_scan", k_scan64_tile, dim3((unsigned)nb), dim3(kT64), 0, s, in, N, out, bs.get());
    if (nb > 1) scan64(bs.get(), bs.get(), nb, s);
    const int64_t g = std::min<int64_t>((N + 256) / 256, 65536);
    TC_LAUNCH("tri_scan", k_scan64_fin, dim3((unsigned)g), dim3(256), 0, s, out, N, (const int64_t*)bs.get(), nb);
}

namespace {

// y in the sorted list of x
__device__ __forceinline__ bool in_list(const int32_t* __restrict__ rp, const int32_t* __restrict__ col, int32_t x,
                                        int32_t y) {
    int32_t lo = rp[x];
    const int32_t end = rp[x + 1];
    int32_t hi = end;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (col[mid] < y) lo = mid + 1;
        else hi = mid;
    }
    return lo < end && col[lo] == y;
}

__device__ __forceinline__ bool adjacent(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                         const int32_t* __restrict__ deg, int32_t x, int32_t y) {
    return deg[x] <= deg[y] ? in_list(rp, col, x, y) : in_list(rp, col, y, x);
}

// acc[0] += sum of the closed samples' weights, acc[1] += closed samples
__global__ void __launch_bounds__(256) k_tri_sample(int64_t s, uint64_t salt, int64_t n,
                                                     const int64_t* __restrict__ CU, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ deg, const int64_t* __restrict__ EP,
                                                     int64_t m, int hybrid, unsigned long long* __restrict__ acc) {
    const int64_t size = CU[n];
    int64_t wsum = 0, closed = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; size > 0 && i < s;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t h = mix64(mix64((uint64_t)i) ^ salt);
        const int64_t r = (int64_t)__umul64hi(h, (uint64_t)size);
        int64_t lo = 0, hi = n - 1;  // the largest u with CU[u] <= r
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo + 1) >> 1);
            if (CU[mid] <= r) lo = mid;
            else hi = mid - 1;
        }
        const int32_t u = (int32_t)lo;
        const int64_t k = r - CU[u];
        const int32_t du = deg[u];
        int32_t x, y, z;
        bool cl;
        if (!ext_kind(hybrid, du, m)) {
            int64_t b = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)k)) * 0.5);  // then made exact
            while (b > 1 && b * (b - 1) / 2 > k) --b;
            while ((b + 1) * b / 2 <= k) ++b;
            const int64_t a = k - b * (b - 1) / 2;
            x = col[rp[u] + a];
            y = u;
            z = col[rp[u] + b];
            cl = adjacent(rp, col, deg, x, z);
        } else {
            int32_t elo = rp[u], ehi = rp[u + 1] - 1;  // the largest entry e of u's list with EP[e] <= k
            while (elo < ehi) {
                const int32_t mid = elo + ((ehi - elo + 1) >> 1);
                if (EP[mid] <= k) elo = mid;
                else ehi = mid - 1;
            }
            const int32_t v = col[elo];
            x = u;
            y = v;
            z = col[rp[v] + (k - EP[elo])];
            cl = z != u && adjacent(rp, col, deg, u, z);
        }
        if (cl) {
            const int ne = (int)ext_kind(hybrid, deg[x], m) + (int)ext_kind(hybrid, deg[y], m) +
                           (int)ext_kind(hybrid, deg[z], m);
            wsum += 60 / (3 + ne);
            closed += 1;
        }
    }
    wsum = wave_sum(wsum);
    closed = wave_sum(closed);
    if (__lane_id() == 0 && (wsum || closed)) {
        atomicAdd(&acc[0], (unsigned long long)wsum);
        atomicAdd(&acc[1], (unsigned long long)closed);
    }
}

}  // namespace

void triple_sample(const tc_graph_s* g, int hybrid, int64_t num_samples, uint64_t seed, hipStream_t s,
                   int64_t* size, int64_t* wsum, int64_t* closed) {
    const int64_t n = g->n, m = g->m;
    *size = *wsum = *closed = 0;
    if (n == 0) return;
    DevBuf<int64_t> cnt(n + 1, s), CU(n + 1, s), EP(2 * m > 0 ? 2 * m : 1, s);
    DevBuf<unsigned long long> acc(2, s);
    fill_i64(reinterpret_cast<int64_t*>(acc.get()), 0, 2, s);
    const unsigned vg = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    TC_LAUNCH("tri_counts", k_tri_counts, dim3(vg), dim3(256), 0, s, n, (const int32_t*)g->deg, m, hybrid, cnt.get());
    if (hybrid)
        TC_LAUNCH("tri_ext", k_tri_ext, dim3(vg), dim3(256), 0, s, n, (const int32_t*)g->row_ptr,
                  (const int32_t*)g->col, (const int32_t*)g->deg, m, hybrid, cnt.get(), EP.get());
    scan64(cnt.get(), CU.get(), n, s);
    const uint64_t salt = host_mix64(seed ^ 0x54435F545249504CULL);  // "TC_TRIPL"
    const unsigned sg = (unsigned)std::min<int64_t>((num_samples + 255) / 256, (int64_t)num_cus() * 32);
    TC_LAUNCH("tri_sample", k_tri_sample, dim3(sg > 0 ? sg : 1), dim3(256), 0, s, num_samples, salt, n,
              (const int64_t*)CU.get(), (const int32_t*)g->row_ptr, (const int32_t*)g->col, (const int32_t*)g->deg,
              (const int64_t*)EP.get(), m, hybrid, acc.get());
    int64_t h[3];
    check_hip(hipMemcpyAsync(h, CU.get() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s), "size");
    check_hip(hipMemcpyAsync(h + 1, acc.get(), 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s), "acc");
    check_hip(hipStreamSynchronize(s), "sync");
    *size = h[0];
    *wsum = h[1];
    *closed = h[2];
}

}  // namespace tc
