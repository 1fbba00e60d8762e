// Edge sparsification (section 3.1): every undirected edge is kept
// independently with probability p.  The coin is a counter-based hash of the
// edge's (min, max) ids and the seed, so both CSR directions of an edge, and
// any other implementation of the same hash, take the same decision.
//
// Layout: one keep bit per CSR entry, packed 64 to a word (a wave's ballot),
// plus the popcount of each word; an exclusive scan of the popcounts gives the
// compacted position of every kept entry and of every row start.
#include "tc_internal.h"
#include "tc_device.h"

namespace tc {

uint64_t keep_threshold(double p) { return (uint64_t)(p * 9007199254740992.0); }

uint64_t sample_salt(uint64_t seed) {
    uint64_t z = seed ^ 0x54435F53414D504Cull;  // "TC_SAMPL"
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

namespace {

__global__ void __launch_bounds__(256) k_keep_bits(const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                                                    int64_t E2, uint64_t salt, uint64_t thr,
                                                    uint64_t* __restrict__ bits, int32_t* __restrict__ wcnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x; e0 < E2; e0 += stride) {
        const int64_t e = e0 + threadIdx.x;
        bool keep = false;
        if (e < E2) keep = edge_kept((uint32_t)src[e], (uint32_t)col[e], salt, thr);
        const uint64_t b = ballot64(keep);
        if (__lane_id() == 0 && e < E2) {
            bits[e >> 6] = b;
            wcnt[e >> 6] = __popcll(b);
        }
    }
}

__device__ __forceinline__ int32_t kept_before(int64_t e, int64_t E2, const uint64_t* bits, const int32_t* wpre) {
    if (e >= E2) return wpre[(E2 + 63) >> 6];
    const uint64_t w = bits[e >> 6];
    const int r = (int)(e & 63);
    const uint64_t below = r == 0 ? 0ull : (w & (~0ull >> (64 - r)));
    return wpre[e >> 6] + __popcll(below);
}

__global__ void k_rows_at(const int32_t* __restrict__ row_ptr, int64_t n, int64_t E2, const uint64_t* __restrict__ bits,
                          const int32_t* __restrict__ wpre, int32_t* __restrict__ rp_out, int32_t* __restrict__ deg_out) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= n; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = kept_before(row_ptr[x], E2, bits, wpre);
        if (rp_out) rp_out[x] = a;
        if (deg_out && x < n) deg_out[x] = kept_before(row_ptr[x + 1], E2, bits, wpre) - a;
    }
}

// Each wave takes 4 words of keep bits (256 entries) per step: the words and
// their prefixes first, then the kept entries' loads, then the stores, so the
// latencies of the 4 words overlap.
__global__ void __launch_bounds__(256) k_compact(const int32_t* __restrict__ col, const int32_t* __restrict__ src,
                                                  int64_t E2, const int32_t* __restrict__ E2_dev,
                                                  const uint64_t* __restrict__ bits, const int32_t* __restrict__ wpre,
                                                  int32_t* __restrict__ col_out, int32_t* __restrict__ src_out,
                                                  int2* __restrict__ zero_out) {
    const int lane = __lane_id();
    const int64_t valid = E2_dev ? (int64_t)E2_dev[0] : E2;  // entries past it have no bits set
    const int64_t NW = (valid + 63) / 64;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t w0 = wave * 4; w0 < NW; w0 += nwaves * 4) {
        uint64_t bw[4];
        int32_t pre[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool ok = w0 + k < NW;
            bw[k] = ok ? bits[w0 + k] : 0ull;
            pre[k] = ok ? wpre[w0 + k] : 0;
        }
        int32_t cv[4], sv[4];
        bool on[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            on[k] = (bw[k] >> lane) & 1ull;  // set bits lie below valid <= E2
            const int64_t e = (w0 + k) * 64 + lane;
            cv[k] = on[k] ? col[e] : 0;
            sv[k] = (on[k] && src_out) ? src[e] : 0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (on[k]) {
                const int32_t p = pre[k] + __popcll(bw[k] & below);
                col_out[p] = cv[k];
                if (src_out) src_out[p] = sv[k];
                if (zero_out) zero_out[p] = make_int2(0, 0);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// unions of samples (batched seeds, fused requests)
// ---------------------------------------------------------------------------

// Copy k of the replicated entry space holds g's entries at union positions
// k * 64 NWp + e (e < E2; the rest of its words are never kept), so that no
// word of keep bits straddles two copies.  One wave per word of g, for every
// copy: the entries are read once and the seed-independent first mix of each
// edge's key is computed once (the coin is mix64(mix64(key) ^ salt) >> 11 <
// thr, section 3.1's coin as the single-sample kernels compute it).
__global__ void __launch_bounds__(256) k_keep_rep(const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                                                   int64_t E2, int64_t NWp, int32_t K,
                                                   const uint64_t* __restrict__ salts, uint64_t thr,
                                                   uint64_t* __restrict__ bits, int32_t* __restrict__ wcnt) {
    const int lane = __lane_id();
    const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t w = wave; w < NWp; w += nwaves) {
        const int64_t e = w * 64 + lane;
        const bool in = e < E2;
        uint64_t base = 0;
        if (in) {
            const uint32_t u = (uint32_t)src[e], v = (uint32_t)col[e];
            const uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
            base = mix64((lo << 32) | hi);
        }
        for (int32_t k = 0; k < K; ++k) {
            const uint64_t b = ballot64(in && (mix64(base ^ salts[k]) >> 11) < thr);
            if (lane == 0) {
                bits[(int64_t)k * NWp + w] = b;
                wcnt[(int64_t)k * NWp + w] = __popcll(b);
            }
        }
    }
}

// Row offsets and degrees of the union of samples: union vertex k * npad + x
// is vertex x of copy k (x >= n: isolated padding).
__global__ void k_rows_rep(const int32_t* __restrict__ row_ptr, int64_t n, int64_t npad, int64_t E2, int64_t NWp,
                           int32_t K, const uint64_t* __restrict__ bits, const int32_t* __restrict__ wpre,
                           int32_t* __restrict__ rp_out, int32_t* __restrict__ deg_out) {
    const int64_t nU = (int64_t)K * npad;
    const int64_t E2U = (int64_t)K * NWp * 64;
    for (int64_t xu = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; xu <= nU; xu += (int64_t)gridDim.x * blockDim.x) {
        if (xu == nU) {
            rp_out[nU] = wpre[K * NWp];
            continue;
        }
        const int64_t k = xu / npad;
        const int64_t x = xu - k * npad;
        const int64_t base = k * NWp * 64;
        const int64_t e0 = base + (x < n ? row_ptr[x] : E2);
        const int64_t e1 = base + (x < n ? row_ptr[x + 1] : E2);
        const int32_t a = kept_before(e0, E2U, bits, wpre);
        rp_out[xu] = a;
        deg_out[xu] = kept_before(e1, E2U, bits, wpre) - a;
    }
}

// Kept entries of the replicated space, relabelled to union vertex ids.
__global__ void __launch_bounds__(256) k_compact_rep(const int32_t* __restrict__ col, const int32_t* __restrict__ src,
                                                      int64_t E2, int64_t NWp, int32_t K, int64_t npad,
                                                      const uint64_t* __restrict__ bits,
                                                      const int32_t* __restrict__ wpre, int32_t* __restrict__ col_out,
                                                      int32_t* __restrict__ src_out) {
    const int lane = __lane_id();
    const int64_t nw = (int64_t)K * NWp;
    const uint64_t below = lanes_below();
    const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t w = wave; w < nw; w += nwaves) {
        const uint64_t bw = bits[w];
        if (!bw) continue;  // wave-uniform
        const int64_t k = w / NWp;
        const int64_t e = (w - k * NWp) * 64 + lane;
        if ((bw >> lane) & 1ull) {  // set bits lie below E2
            const int32_t p = wpre[w] + __popcll(bw & below);
            col_out[p] = (int32_t)(k * npad + col[e]);
            src_out[p] = (int32_t)(k * npad + src[e]);
        }
    }
}

// Keep bits of a union graph whose component k is sampled with (thrs[k],
// salts[k]) on its local ids (x - off[k]).
__global__ void __launch_bounds__(256) k_keep_comp(const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                                                    int64_t E2, const int32_t* __restrict__ comp,
                                                    const int32_t* __restrict__ off,
                                                    const uint64_t* __restrict__ salts,
                                                    const uint64_t* __restrict__ thrs, uint64_t* __restrict__ bits,
                                                    int32_t* __restrict__ wcnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x; e0 < E2; e0 += stride) {
        const int64_t e = e0 + threadIdx.x;
        bool keep = false;
        if (e < E2) {
            const int32_t u = src[e], v = col[e];
            const int32_t k = comp[u];
            const int32_t o = off[k];
            keep = edge_kept((uint32_t)(u - o), (uint32_t)(v - o), salts[k], thrs[k]);
        }
        const uint64_t b = ballot64(keep);
        if (__lane_id() == 0 && e < E2) {
            bits[e >> 6] = b;
            wcnt[e >> 6] = __popcll(b);
        }
    }
}

// comp[x] = x / npad, off[k] = k * npad
__global__ void k_comp_rep(int64_t npad, int32_t K, int32_t* __restrict__ comp, int32_t* __restrict__ off) {
    const int64_t nU = (int64_t)K * npad;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < nU; x += (int64_t)gridDim.x * blockDim.x)
        comp[x] = (int32_t)(x / npad);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= K) off[t] = (int32_t)(t * npad);
}

// mk[k] = edges of component k = (rp[off[k+1]] - rp[off[k]]) / 2
__global__ void k_comp_edges(int32_t K, const int32_t* __restrict__ off, const int32_t* __restrict__ rp,
                             int64_t* __restrict__ mk) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x)
        mk[k] = ((int64_t)rp[off[k + 1]] - (int64_t)rp[off[k]]) / 2;
}

unsigned grid_for(int64_t N, int threads) {
    unsigned b = ceil_div(N, threads);
    if (b > 65536) b = 65536;
    return b ? b : 1;
}

}  // namespace

void sample_keep_bits(const tc_graph_s* g, uint64_t salt, uint64_t thr, uint64_t* bits, int32_t* wcnt, hipStream_t s) {
    const int64_t E2 = 2 * g->m;
    if (E2 == 0) return;
    TC_LAUNCH("sample_keep", k_keep_bits, dim3(grid_for(E2, 256)), dim3(256), 0, s, g->src, g->col, E2, salt, thr, bits,
              wcnt);
}

void positions_at_rows(const int32_t* row_ptr, int64_t n, int64_t E2, const uint64_t* bits, const int32_t* wpre,
                       int32_t* rp_out, int32_t* deg_out, hipStream_t s) {
    TC_LAUNCH("rows_at", k_rows_at, dim3(grid_for(n + 1, 256)), dim3(256), 0, s, row_ptr, n, E2, bits, wpre, rp_out,
              deg_out);
}

void compact_kept(const int32_t* col, const int32_t* src, int64_t E2, const uint64_t* bits, const int32_t* wpre,
                  int32_t* col_out, int32_t* src_out, hipStream_t s, const int32_t* E2_dev, int2* zero_out) {
    if (E2 == 0) return;
    TC_LAUNCH("compact", k_compact, dim3(grid_for((E2 + 63) / 64, 16)), dim3(256), 0, s, col, src, E2, E2_dev, bits,
              wpre, col_out, src_out, zero_out);
}

}  // namespace tc

namespace tc {

static int32_t read_total(const int32_t* p, hipStream_t s) {
    int32_t t = 0;
    check_hip(hipMemcpyAsync(&t, p, sizeof(int32_t), hipMemcpyDeviceToHost, s), "sample total");
    check_hip(hipStreamSynchronize(s), "sync");
    return t;
}

void sample_union_replicas(const tc_graph_s* g, int32_t K, const uint64_t* salts, uint64_t thr, hipStream_t s,
                           tc_graph_s* out, int32_t* comp, int32_t* off, int64_t* mk) {
    const int64_t n = g->n, E2 = 2 * g->m;
    const int64_t npad = (n + kUnionAlign - 1) / kUnionAlign * kUnionAlign;
    const int64_t nU = (int64_t)K * npad;
    const int64_t NWp = (E2 + 63) / 64;
    const int64_t NW = (int64_t)K * NWp;
    if (nU > 0x7fffffffLL || NW * 64 > 0x7fffffffLL) fail(TC_ERR_OVERFLOW, "the union of the samples exceeds int32 ids");
    PhaseScope ph("sample");
    out->n = nU;
    out->home = s;
    out->max_deg = g->max_deg;  // sampled degrees never exceed the graph's
    out->row_ptr = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(nU + 1), s);
    out->deg = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(nU > 0 ? nU : 1), s);
    TC_LAUNCH("comp_rep", k_comp_rep, dim3(grid_for(nU > K + 1 ? nU : K + 1, 256)), dim3(256), 0, s, npad, K, comp, off);
    int32_t total = 0;
    if (NW > 0) {
        DevBuf<uint64_t> bits(NW, s);
        DevBuf<int32_t> wpre(NW + 1, s);
        TC_LAUNCH("keep_rep", k_keep_rep, dim3(grid_for(NWp, 4)), dim3(256), 0, s, (const int32_t*)g->src,
                  (const int32_t*)g->col, E2, NWp, K, salts, thr, bits.get(), wpre.get());
        scan_exclusive_i32(wpre.get(), wpre.get(), NW, s);
        TC_LAUNCH("rows_rep", k_rows_rep, dim3(grid_for(nU + 1, 256)), dim3(256), 0, s, (const int32_t*)g->row_ptr, n,
                  npad, E2, NWp, K, (const uint64_t*)bits.get(), (const int32_t*)wpre.get(), out->row_ptr, out->deg);
        total = read_total(wpre.get() + NW, s);
        out->m = total / 2;
        out->col = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s);
        out->src = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s);
        TC_LAUNCH("compact_rep", k_compact_rep, dim3(grid_for(NW, 4)), dim3(256), 0, s, (const int32_t*)g->col,
                  (const int32_t*)g->src, E2, NWp, K, npad, (const uint64_t*)bits.get(), (const int32_t*)wpre.get(),
                  out->col, out->src);
    } else {
        fill_i32(out->row_ptr, 0, nU + 1, s);
        if (nU > 0) fill_i32(out->deg, 0, nU, s);
        out->m = 0;
        out->col = (int32_t*)dev_alloc(sizeof(int32_t), s);
        out->src = (int32_t*)dev_alloc(sizeof(int32_t), s);
    }
    TC_LAUNCH("comp_edges", k_comp_edges, dim3(ceil_div(K, 256)), dim3(256), 0, s, K, (const int32_t*)off,
              (const int32_t*)out->row_ptr, mk);
}

void sample_union_components(const tc_graph_s* gU, int32_t K, const int32_t* comp, const int32_t* off,
                             const uint64_t* salts, const uint64_t* thrs, hipStream_t s, tc_graph_s* out,
                             int64_t* mk) {
    const int64_t n = gU->n, E2 = 2 * gU->m, NW = (E2 + 63) / 64;
    PhaseScope ph("sample");
    out->n = n;
    out->home = s;
    out->max_deg = gU->max_deg;
    out->row_ptr = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(n + 1), s);
    out->deg = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1), s);
    int32_t total = 0;
    if (E2 > 0) {
        DevBuf<uint64_t> bits(NW, s);
        DevBuf<int32_t> wpre(NW + 1, s);
        TC_LAUNCH("keep_comp", k_keep_comp, dim3(grid_for(E2, 256)), dim3(256), 0, s, (const int32_t*)gU->src,
                  (const int32_t*)gU->col, E2, comp, off, salts, thrs, bits.get(), wpre.get());
        scan_exclusive_i32(wpre.get(), wpre.get(), NW, s);
        positions_at_rows(gU->row_ptr, n, E2, bits.get(), wpre.get(), out->row_ptr, out->deg, s);
        total = read_total(wpre.get() + NW, s);
        out->m = total / 2;
        out->col = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s);
        out->src = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s);
        compact_kept(gU->col, gU->src, E2, bits.get(), wpre.get(), out->col, out->src, s);
    } else {
        fill_i32(out->row_ptr, 0, n + 1, s);
        if (n > 0) fill_i32(out->deg, 0, n, s);
        out->m = 0;
        out->col = (int32_t*)dev_alloc(sizeof(int32_t), s);
        out->src = (int32_t*)dev_alloc(sizeof(int32_t), s);
    }
    TC_LAUNCH("comp_edges", k_comp_edges, dim3(ceil_div(K, 256)), dim3(256), 0, s, K, off,
              (const int32_t*)out->row_ptr, mk);
}

}  // namespace tc
