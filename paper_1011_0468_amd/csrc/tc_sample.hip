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
