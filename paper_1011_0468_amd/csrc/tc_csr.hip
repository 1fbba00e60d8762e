// CSR construction: symmetrise, drop self-loops, LSD radix sort of packed
// (u, v) keys, drop duplicates, degrees by aggregated atomics, row offsets by
// scan.  The result is the simple undirected graph with each neighbour list
// sorted ascending (section 4.1 and the sorted neighbour-list format of
// section 4.2).
#include "tc_internal.h"
#include "tc_device.h"

#include <algorithm>

namespace tc {

namespace {

constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
static_assert(kRadix == kRsThreads, "one thread per digit in the scatter's scan");

// Emit (u,v) and (v,u) packed as u << nb | v; self-loops become the sentinel
// (all 2nb bits set), which sorts after every valid key.
template <typename K>
__global__ void k_emit_keys(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, int64_t P,
                            int64_t n, int nb, K* __restrict__ keys, int32_t* __restrict__ bad) {
    const K sentinel = (K)((nb * 2 >= (int)(8 * sizeof(K))) ? ~(K)0 : (((K)1 << (2 * nb)) - 1));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = src[i], v = dst[i];
        const bool ok = u >= 0 && v >= 0 && (int64_t)u < n && (int64_t)v < n;
        if (!ok) atomicOr(bad, 1);
        K a = sentinel, b = sentinel;
        if (ok && u != v) {
            a = ((K)(uint32_t)u << nb) | (K)(uint32_t)v;
            b = ((K)(uint32_t)v << nb) | (K)(uint32_t)u;
        }
        keys[2 * i] = a;
        keys[2 * i + 1] = b;
    }
}

// Per-tile digit histogram, digit-major: hist[d * nblocks + block].
template <typename K>
__global__ void __launch_bounds__(kRsThreads) k_rs_hist(const K* __restrict__ keys, int64_t N, int shift,
                                                         int32_t* __restrict__ hist) {
    __shared__ int32_t cnt[kRadix];
    for (int d = threadIdx.x; d < kRadix; d += kRsThreads) cnt[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
    for (int i = 0; i < kRsItems; ++i) {
        const int64_t idx = base + (int64_t)i * kRsThreads + threadIdx.x;
        if (idx < N) atomicAdd(&cnt[(int)((keys[idx] >> shift) & (kRadix - 1))], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kRsThreads) hist[(int64_t)d * gridDim.x + blockIdx.x] = cnt[d];
}

// Stable scatter of one tile of kRsTile keys.  All 16 keys of a thread are
// loaded first; within each wave and iteration, peers with the same digit are
// found by 8 ballots; the per-(iteration, wave) digit counts go to LDS and one
// scan per digit over the 64 (iteration, wave) groups, in index order, gives
// every group its output base: two block barriers per tile.
template <typename K>
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const K* __restrict__ in, K* __restrict__ out,
                                                            int64_t N, int shift,
                                                            const int32_t* __restrict__ offs) {
    constexpr int NW = kRsThreads / 64;
    constexpr int NG = kRsItems * NW;  // (iteration, wave) groups in index order
    __shared__ int32_t cnt[NG][kRadix];
    const int t = threadIdx.x;
    const int w = t >> 6;
    for (int g = 0; g < NG; ++g) cnt[g][t] = 0;  // kRadix == kRsThreads
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    K key[kRsItems];
    int32_t dg[kRsItems], rk[kRsItems];
#pragma unroll
    for (int i = 0; i < kRsItems; ++i) {
        const int64_t idx = base + (int64_t)i * kRsThreads + t;
        key[i] = idx < N ? in[idx] : (K)0;
    }
    __syncthreads();  // counters zeroed
#pragma unroll
    for (int i = 0; i < kRsItems; ++i) {
        const bool valid = base + (int64_t)i * kRsThreads + t < N;
        const int d = (int)((key[i] >> shift) & (kRadix - 1));
        uint64_t peers = ballot64(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const int bit = (d >> b) & 1;
            const uint64_t bal = ballot64(valid && bit);
            peers &= bit ? bal : ~bal;
        }
        const int r = __popcll(peers & lanes_below());
        if (valid && r == 0) cnt[i * NW + w][d] = __popcll(peers);
        dg[i] = d;
        rk[i] = valid ? r : -1;
    }
    __syncthreads();
    {
        int32_t run = offs[(int64_t)t * gridDim.x + blockIdx.x];  // digit t of this tile
        for (int g = 0; g < NG; ++g) {
            const int32_t c = cnt[g][t];
            cnt[g][t] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRsItems; ++i)
        if (rk[i] >= 0) out[cnt[i * NW + w][dg[i]] + rk[i]] = key[i];
}

template <typename K>
__global__ void k_unique_flags(const K* __restrict__ keys, int64_t N, K sentinel, int32_t* __restrict__ flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const K k = keys[i];
        flag[i] = (k != sentinel && (i == 0 || keys[i - 1] != k)) ? 1 : 0;
    }
}

// Write unique keys to col/src and count degrees: unique keys of one wave form
// runs of equal rows (keys are sorted); each run adds its length with one atomic.
// Each wave takes 4 chunks of 64 keys per step with all their loads (keys, the
// key before each, positions) issued before the first use.
template <typename K>
__global__ void __launch_bounds__(256) k_unique_scatter(const K* __restrict__ keys, int64_t N, K sentinel, int nb,
                                                         const int32_t* __restrict__ pos, int32_t* __restrict__ col,
                                                         int32_t* __restrict__ srcrow, int32_t* __restrict__ deg) {
    const K vmask = ((K)1 << nb) - 1;
    const int lane = __lane_id();
    const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t c0 = wave * 256; c0 < N; c0 += nwaves * 256) {
        K k[4], kp[4];
        int32_t ps[4];
        bool in[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = c0 + 64 * q + lane;
            in[q] = i < N;
            const int64_t ic = in[q] ? i : N - 1;
            k[q] = keys[ic];
            kp[q] = ic > 0 ? keys[ic - 1] : sentinel;
            ps[q] = pos[ic];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = c0 + 64 * q + lane;
            const bool uniq = in[q] && k[q] != sentinel && (i == 0 || kp[q] != k[q]);
            int32_t u = -1;
            if (uniq) {
                u = (int32_t)(k[q] >> nb);
                col[ps[q]] = (int32_t)(k[q] & vmask);
                srcrow[ps[q]] = u;
            }
            const uint64_t active = ballot64(uniq);
            const int32_t up = __shfl_up(u, 1, 64);
            const bool prev_same = lane > 0 && ((active >> (lane - 1)) & 1ull) && up == u;
            const bool head = uniq && !prev_same;
            const uint64_t heads = ballot64(head);
            if (head) {
                const uint64_t breaks = (heads | ~active) & (lane == 63 ? 0ull : (~0ull << (lane + 1)));
                const int next = breaks ? __builtin_ctzll(breaks) : 64;
                atomicAdd(&deg[u], next - lane);
            }
        }
    }
}

template <typename K>
int build_csr_t(int64_t n, int64_t P, const int32_t* src, const int32_t* dst, int nb, hipStream_t s,
                tc_graph_s* g) {
    const int64_t N = 2 * P;
    const K sentinel = (K)((nb * 2 >= (int)(8 * sizeof(K))) ? ~(K)0 : (((K)1 << (2 * nb)) - 1));
    DevBuf<K> ka(N, s), kb(N, s);
    DevBuf<int32_t> bad(1, s);
    fill_i32(bad.get(), 0, 1, s);
    {
        unsigned blocks = ceil_div(P, 256);
        if (blocks > 65536) blocks = 65536;
        if (blocks == 0) blocks = 1;
        TC_LAUNCH("csr_emit", k_emit_keys<K>, dim3(blocks), dim3(256), 0, s, src, dst, P, n, nb, ka.get(), bad.get());
    }
    int32_t h_bad = 0;
    check_hip(hipMemcpyAsync(&h_bad, bad.get(), sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy flag");
    check_hip(hipStreamSynchronize(s), "sync");
    if (h_bad) return 1;

    const int key_bits = 2 * nb;
    const int64_t nblk = (N + kRsTile - 1) / kRsTile;
    if (N > 0) {
        DevBuf<int32_t> hist((size_t)kRadix * nblk + 1, s);
        for (int shift = 0; shift < key_bits; shift += kRadixBits) {
            TC_LAUNCH("csr_radix_hist", k_rs_hist<K>, dim3((unsigned)nblk), dim3(kRsThreads), 0, s, ka.get(), N, shift,
                      hist.get());
            scan_exclusive_i32(hist.get(), hist.get(), (int64_t)kRadix * nblk, s);
            TC_LAUNCH("csr_radix_scatter", k_rs_scatter<K>, dim3((unsigned)nblk), dim3(kRsThreads), 0, s, ka.get(),
                      kb.get(), N, shift, (const int32_t*)hist.get());
            std::swap(ka.ptr, kb.ptr);
        }
    }
    DevBuf<int32_t> pos(N + 1, s);
    unsigned blocks = ceil_div(N, 256);
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) blocks = 1;
    TC_LAUNCH("csr_unique_flags", k_unique_flags<K>, dim3(blocks), dim3(256), 0, s, ka.get(), N, sentinel, pos.get());
    scan_exclusive_i32(pos.get(), pos.get(), N, s);
    int32_t total = 0;
    check_hip(hipMemcpyAsync(&total, pos.get() + N, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy total");
    check_hip(hipStreamSynchronize(s), "sync");

    g->n = n;
    g->m = total / 2;
    g->row_ptr = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(n + 1), s);
    g->col = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s);
    g->src = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s);
    g->deg = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1), s);
    g->home = s;
    fill_i32(g->deg, 0, n, s);
    TC_LAUNCH("csr_unique_scatter", k_unique_scatter<K>, dim3(std::max<unsigned>(1, (unsigned)std::min<int64_t>(
                                                                 (N + 1023) / 1024, 65536))),
              dim3(256), 0, s, ka.get(), N, sentinel, nb, (const int32_t*)pos.get(), g->col, g->src, g->deg);
    scan_exclusive_i32(g->deg, g->row_ptr, n, s);
    return 0;
}

}  // namespace

static int key_bits_half(int64_t n) {
    int nb = 1;
    while (nb < 31 && ((int64_t)1 << nb) < n) ++nb;
    return nb;
}

int64_t build_csr_bytes(int64_t n, int64_t num_pairs) {
    auto rb = region_bytes;
    const int nb = key_bits_half(n);
    const int64_t K = 2 * nb <= 32 ? 4 : 8;
    const int64_t N = 2 * num_pairs;
    int64_t b = 2 * rb(K * N) + rb(4);  // key ping-pong, flag
    if (N > 0) {
        const int64_t nblk = (N + kRsTile - 1) / kRsTile;
        b += rb(4 * (kRadix * nblk + 1)) + scan_scratch_bytes(kRadix * nblk);
    }
    b += rb(4 * (N + 1)) + scan_scratch_bytes(N);                              // unique positions
    b += rb(4 * (n + 1)) + 2 * rb(4 * N) + rb(4 * n) + scan_scratch_bytes(n);  // the CSR (2m <= N)
    b += rb(N) + rb(n);                                                         // neighbour classes
    return b;
}

int build_csr(int64_t n, int64_t num_pairs, const int32_t* src, const int32_t* dst, hipStream_t s, tc_graph_s* g) {
    PhaseScope ph("csr");
    const int nb = key_bits_half(n);
    const int bad = 2 * nb <= 32 ? build_csr_t<uint32_t>(n, num_pairs, src, dst, nb, s, g)
                                 : build_csr_t<uint64_t>(n, num_pairs, src, dst, nb, s, g);
    if (!bad) neighbour_classes(g, s);
    return bad;
}

}  // namespace tc
