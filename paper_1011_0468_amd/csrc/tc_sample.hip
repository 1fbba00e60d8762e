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
                                                  int32_t* __restrict__ col_out, int32_t* __restrict__ src_out) {
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
            }
        }
    }
}

// Keep bits with the kept entries staged: one wave per range of kStageWords
// words (64 entries each).  The wave writes the range's keep words and their
// popcounts, and packs the range's kept entries, in order, at the start of
// the range's region of the staging arrays (entries [64 w0, 64 w0 + kept)),
// with full-width stores.  Once the word counts are scanned, k_move_staged
// copies each range's packed entries to their place, so no entry of the
// graph is read twice and no store is one lane wide.
constexpr int kStageWords = 8;

__device__ __forceinline__ void wave_lds_order_s() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(256) k_keep_stage(const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                                                     int64_t E2, uint64_t salt, uint64_t thr,
                                                     uint64_t* __restrict__ bits, int32_t* __restrict__ wcnt,
                                                     int32_t* __restrict__ st_col, int32_t* __restrict__ st_src) {
    constexpr int RW = kStageWords;
    __shared__ int32_t pack[4][2][RW * 64];
    const int lane = __lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int32_t* pc = pack[wv][0];
    int32_t* ps = pack[wv][1];
    const uint64_t below = lanes_below();
    const int64_t NW = (E2 + 63) / 64;
    const int64_t nR = (NW + RW - 1) / RW;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t r = (int64_t)blockIdx.x * 4 + wv; r < nR; r += nwaves) {
        const int64_t w0 = r * RW;
        int32_t uu[RW], vv[RW];
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int64_t e = (w0 + i) * 64 + lane;
            const bool in = e < E2;
            uu[i] = in ? src[e] : 0;
            vv[i] = in ? col[e] : 0;
        }
        int32_t cnt = 0;
        uint64_t mine = 0;  // lane i < RW: word w0 + i
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int64_t e = (w0 + i) * 64 + lane;
            const bool keep = e < E2 && edge_kept((uint32_t)uu[i], (uint32_t)vv[i], salt, thr);
            const uint64_t b = ballot64(keep);
            if (lane == i) mine = b;
            if (keep) {
                const int32_t q = cnt + (int32_t)__popcll(b & below);
                pc[q] = vv[i];
                ps[q] = uu[i];
            }
            cnt += (int32_t)__popcll(b);
        }
        if (lane < RW && w0 + lane < NW) {
            bits[w0 + lane] = mine;
            wcnt[w0 + lane] = (int32_t)__popcll(mine);
        }
        wave_lds_order_s();
        for (int32_t q = lane; q < cnt; q += 64) {
            st_col[w0 * 64 + q] = pc[q];
            st_src[w0 * 64 + q] = ps[q];
        }
        wave_lds_order_s();  // read before the next range packs
    }
}

// Each range's staged entries to positions wpre[w0] .. (wpre: exclusive scan
// of the word counts, NW + 1 entries).
__global__ void __launch_bounds__(256) k_move_staged(int64_t E2, const int32_t* __restrict__ wpre,
                                                      const int32_t* __restrict__ st_col,
                                                      const int32_t* __restrict__ st_src, int32_t* __restrict__ col_out,
                                                      int32_t* __restrict__ src_out) {
    constexpr int RW = kStageWords;
    const int lane = __lane_id();
    const int64_t NW = (E2 + 63) / 64;
    const int64_t nR = (NW + RW - 1) / RW;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t r = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); r < nR; r += nwaves) {
        const int64_t w0 = r * RW;
        const int64_t w1 = w0 + RW < NW ? w0 + RW : NW;
        const int32_t a = wpre[w0];
        const int32_t cnt = wpre[w1] - a;
        for (int32_t q = lane; q < cnt; q += 64) {
            col_out[a + q] = st_col[w0 * 64 + q];
            src_out[a + q] = st_src[w0 * 64 + q];
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

// The id of union vertex x after dropping the isolated ones:
// nzt[x / 64].z + (the kept vertices below x in its 64-vertex word), from one
// 16-byte gather (see k_nz_table).
__device__ __forceinline__ int32_t nz_id(const int4* __restrict__ nzt, int64_t x) {
    const int4 t = nzt[x >> 6];
    const uint64_t b = ((uint64_t)(uint32_t)t.y << 32) | (uint32_t)t.x;
    const int r = (int)(x & 63);
    return t.z + __popcll(r == 0 ? 0ull : (b & (~0ull >> (64 - r))));
}

// Orders one wave's LDS accesses (a wave's LDS operations complete in issue
// order; only the compiler must not move accesses across).
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Words of g per range of k_compact_rep
constexpr int kRepWords = 8;

// Kept entries of the replicated space, written with the union's final ids
// (nz_id of the padded layout's id).  One wave per range of kRepWords words
// of g: the range's entries are read once and held in registers, and for
// every copy the kept entries of the whole range, which are consecutive in
// that copy's output, are packed in LDS, relabelled by full-width table
// gathers and written with full-width stores (one store per 64 kept entries
// instead of one per word and copy).  The copies' keep words and prefixes
// are loaded 64 at a time (8 copies x 8 words, one per lane) and taken with
// readlane.
__global__ void __launch_bounds__(256) k_compact_rep(const int32_t* __restrict__ col, const int32_t* __restrict__ src,
                                                      int64_t E2, int64_t NWp, int32_t K, int64_t npad,
                                                      const uint64_t* __restrict__ bits,
                                                      const int32_t* __restrict__ wpre, const int4* __restrict__ nzt,
                                                      int32_t* __restrict__ col_out, int32_t* __restrict__ src_out) {
    constexpr int RW = kRepWords, CPL = 64 / RW;  // words per range, copies per load
    __shared__ int32_t pack[4][2][RW * 64];
    const int lane = __lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int32_t* pc = pack[wv][0];
    int32_t* ps = pack[wv][1];
    const uint64_t below = lanes_below();
    const int64_t wave = (int64_t)blockIdx.x * 4 + wv;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int64_t nR = (NWp + RW - 1) / RW;
    for (int64_t r = wave; r < nR; r += nwaves) {
        const int64_t w0 = r * RW;
        int32_t vv[RW], uu[RW];
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int64_t e = (w0 + i) * 64 + lane;
            const bool in = w0 + i < NWp && e < E2;
            vv[i] = in ? col[e] : 0;
            uu[i] = in ? src[e] : 0;
        }
        for (int32_t k0 = 0; k0 < K; k0 += CPL) {
            const int32_t kl = k0 + lane / RW;
            const int64_t wl = w0 + lane % RW;
            const bool ok = kl < K && wl < NWp;  // words past NWp belong to no copy of this range
            const uint64_t myb = ok ? bits[(int64_t)kl * NWp + wl] : 0ull;
            const int32_t myp = ok ? wpre[(int64_t)kl * NWp + wl] : 0;
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                const int64_t k = k0 + j;
                if (k >= K) break;
                const int32_t base = __builtin_amdgcn_readlane(myp, j * RW);  // the copy's first kept entry here
                int32_t cnt = 0;
#pragma unroll
                for (int i = 0; i < RW; ++i) {
                    const int src_lane = j * RW + i;
                    const uint64_t bw =
                        ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(myb >> 32), src_lane) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)myb, src_lane);
                    if ((bw >> lane) & 1ull) {  // set bits lie below E2
                        const int32_t q = cnt + (int32_t)__popcll(bw & below);
                        pc[q] = (int32_t)(k * npad + vv[i]);
                        ps[q] = (int32_t)(k * npad + uu[i]);
                    }
                    cnt += (int32_t)__popcll(bw);
                }
                if (cnt == 0) continue;
                wave_lds_order();
                for (int32_t q = lane; q < cnt; q += 64) {
                    col_out[base + q] = nz_id(nzt, pc[q]);
                    src_out[base + q] = nz_id(nzt, ps[q]);
                }
                wave_lds_order();  // read before the next copy packs
            }
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

// ---- dropping the isolated vertices of a union of samples -----------------
// A vertex without kept edges takes part in no triangle and in no statistic
// of the count, and an order-preserving relabelling keeps the (deg, id)
// order, so the union keeps only the vertices of degree > 0: component k's
// nz[k] of them take new ids off'[k] .. off'[k] + nz[k] - 1 in their old
// order, and off'[k + 1] = off'[k] + nz[k] rounded up to kUnionAlign.

// one bit per union vertex (degree > 0), per-word counts
__global__ void __launch_bounds__(256) k_nz_bits(int64_t nU, const int32_t* __restrict__ deg, uint64_t* __restrict__ nzb,
                                                  int32_t* __restrict__ nzc) {
    const int lane = __lane_id();
    const int64_t nw = (nU + 63) / 64;
    const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t w = wave; w < nw; w += nwaves) {
        const int64_t x = w * 64 + lane;
        const uint64_t b = ballot64(x < nU && deg[x] > 0);
        if (lane == 0) {
            nzb[w] = b;
            nzc[w] = __popcll(b);
        }
    }
}

// new component offsets (one thread; K is small): off2[k], off2[K] = new n
__global__ void k_nz_offsets(int32_t K, int64_t npad, const int32_t* __restrict__ nzpre, int32_t* __restrict__ off2) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t o = 0;
    const int64_t wpc = npad / 64;  // words per component
    for (int32_t k = 0; k < K; ++k) {
        off2[k] = (int32_t)o;
        const int64_t nz = (int64_t)nzpre[(k + 1) * wpc] - (int64_t)nzpre[k * wpc];
        o += (nz + kUnionAlign - 1) / kUnionAlign * kUnionAlign;
    }
    off2[K] = (int32_t)o;
}

// new id of union vertex x (degree > 0)
__device__ __forceinline__ int32_t nz_newid(int64_t x, int64_t npad, const uint64_t* __restrict__ nzb,
                                            const int32_t* __restrict__ nzpre, const int32_t* __restrict__ off2) {
    const int64_t k = x / npad;
    const int64_t w = x >> 6;
    const int r = (int)(x & 63);
    const uint64_t below = r == 0 ? 0ull : (nzb[w] & (~0ull >> (64 - r)));
    return off2[k] + (nzpre[w] - nzpre[k * (npad / 64)]) + __popcll(below);
}

// row offsets, degrees and components of the kept vertices at their new ids;
// the padding slots after each component's vertices get its end offset
__global__ void k_nz_place(int64_t nU, int64_t npad, int32_t K, const int32_t* __restrict__ rp,
                           const int32_t* __restrict__ deg, const uint64_t* __restrict__ nzb,
                           const int32_t* __restrict__ nzpre, const int32_t* __restrict__ off2,
                           int32_t* __restrict__ rp2, int32_t* __restrict__ deg2, int32_t* __restrict__ comp2) {
    const int64_t nU2 = off2[K];
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < nU; x += (int64_t)gridDim.x * blockDim.x) {
        if (deg[x] > 0) {
            const int32_t y = nz_newid(x, npad, nzb, nzpre, off2);
            rp2[y] = rp[x];
            deg2[y] = deg[x];
            comp2[y] = (int32_t)(x / npad);
        }
    }
    // padding slots: from each component's last kept vertex to the next component
    for (int64_t k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t wpc = npad / 64;
        const int64_t nz = (int64_t)nzpre[(k + 1) * wpc] - (int64_t)nzpre[k * wpc];
        const int32_t end = rp[(k + 1) * npad];
        for (int64_t y = off2[k] + nz; y < off2[k + 1]; ++y) {
            rp2[y] = end;
            deg2[y] = 0;
            comp2[y] = (int32_t)k;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) rp2[nU2] = rp[nU];
}

// nzt[w] = (keep-vertex bits of union vertices 64 w .. 64 w + 63, new id of
// the first kept vertex at or after 64 w), for the relabelling gathers
__global__ void k_nz_table(int64_t NV, int64_t npad, const uint64_t* __restrict__ nzb,
                           const int32_t* __restrict__ nzpre, const int32_t* __restrict__ off2, int4* __restrict__ nzt) {
    const int64_t wpc = npad / 64;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < NV; w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = w / wpc;
        const uint64_t b = nzb[w];
        nzt[w] = make_int4((int32_t)(uint32_t)b, (int32_t)(uint32_t)(b >> 32),
                           (int32_t)(off2[k] + nzpre[w] - nzpre[k * wpc]), 0);
    }
}

// comp[x] = the k with off[k] <= x < off[k + 1] (largest such k)
__global__ void k_comp_from_off(int64_t n, int32_t K, const int32_t* __restrict__ off, int32_t* __restrict__ comp) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = K - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (off[mid] <= x) lo = mid; else hi = mid - 1;
        }
        comp[x] = lo;
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

void sample_keep_staged(const tc_graph_s* g, uint64_t salt, uint64_t thr, uint64_t* bits, int32_t* wcnt,
                        int32_t* st_col, int32_t* st_src, hipStream_t s) {
    const int64_t E2 = 2 * g->m;
    if (E2 == 0) return;
    const int64_t nR = ((E2 + 63) / 64 + kStageWords - 1) / kStageWords;
    TC_LAUNCH("sample_keep", k_keep_stage, dim3(grid_for(nR, 4)), dim3(256), 0, s, g->src, g->col, E2, salt, thr,
              bits, wcnt, st_col, st_src);
}

void move_staged(int64_t E2, const int32_t* wpre, const int32_t* st_col, const int32_t* st_src, int32_t* col_out,
                 int32_t* src_out, hipStream_t s) {
    if (E2 == 0) return;
    const int64_t nR = ((E2 + 63) / 64 + kStageWords - 1) / kStageWords;
    TC_LAUNCH("compact", k_move_staged, dim3(grid_for(nR, 4)), dim3(256), 0, s, E2, wpre, st_col, st_src, col_out,
              src_out);
}

void positions_at_rows(const int32_t* row_ptr, int64_t n, int64_t E2, const uint64_t* bits, const int32_t* wpre,
                       int32_t* rp_out, int32_t* deg_out, hipStream_t s) {
    TC_LAUNCH("rows_at", k_rows_at, dim3(grid_for(n + 1, 256)), dim3(256), 0, s, row_ptr, n, E2, bits, wpre, rp_out,
              deg_out);
}

void compact_kept(const int32_t* col, const int32_t* src, int64_t E2, const uint64_t* bits, const int32_t* wpre,
                  int32_t* col_out, int32_t* src_out, hipStream_t s, const int32_t* E2_dev) {
    if (E2 == 0) return;
    TC_LAUNCH("compact", k_compact, dim3(grid_for((E2 + 63) / 64, 16)), dim3(256), 0, s, col, src, E2, E2_dev, bits,
              wpre, col_out, src_out);
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
    out->home = s;
    out->max_deg = g->max_deg;  // sampled degrees never exceed the graph's
    if (NW == 0 || nU == 0) {  // no entries: every component is empty
        TC_LAUNCH("comp_rep", k_comp_rep, dim3(grid_for(nU > K + 1 ? nU : K + 1, 256)), dim3(256), 0, s, npad, K, comp,
                  off);
        out->n = nU;
        out->row_ptr = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(nU + 1), s);
        out->deg = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(nU > 0 ? nU : 1), s);
        fill_i32(out->row_ptr, 0, nU + 1, s);
        if (nU > 0) fill_i32(out->deg, 0, nU, s);
        out->m = 0;
        out->col = (int32_t*)dev_alloc(sizeof(int32_t), s);
        out->src = (int32_t*)dev_alloc(sizeof(int32_t), s);
        TC_LAUNCH("comp_edges", k_comp_edges, dim3(ceil_div(K, 256)), dim3(256), 0, s, K, (const int32_t*)off,
                  (const int32_t*)out->row_ptr, mk);
        return;
    }
    // 1. keep bits of every copy, their scan, the union's rows in the padded layout
    DevBuf<uint64_t> bits(NW, s);
    DevBuf<int32_t> wpre(NW + 1, s);
    TC_LAUNCH("keep_rep", k_keep_rep, dim3(grid_for(NWp, 4)), dim3(256), 0, s, (const int32_t*)g->src,
              (const int32_t*)g->col, E2, NWp, K, salts, thr, bits.get(), wpre.get());
    scan_exclusive_i32(wpre.get(), wpre.get(), NW, s);
    DevBuf<int32_t> rp(nU + 1, s), deg(nU, s);
    TC_LAUNCH("rows_rep", k_rows_rep, dim3(grid_for(nU + 1, 256)), dim3(256), 0, s, (const int32_t*)g->row_ptr, n, npad,
              E2, NWp, K, (const uint64_t*)bits.get(), (const int32_t*)wpre.get(), rp.get(), deg.get());
    // 2. the vertices of degree > 0 and the components' new offsets
    const int64_t NV = nU / 64;  // nU is a multiple of kUnionAlign
    DevBuf<uint64_t> nzb(NV, s);
    DevBuf<int32_t> nzpre(NV + 1, s);
    TC_LAUNCH("nz_bits", k_nz_bits, dim3(grid_for(NV, 4)), dim3(256), 0, s, nU, (const int32_t*)deg.get(), nzb.get(),
              nzpre.get());
    scan_exclusive_i32(nzpre.get(), nzpre.get(), NV, s);
    TC_LAUNCH("nz_offsets", k_nz_offsets, dim3(1), dim3(64), 0, s, K, npad, (const int32_t*)nzpre.get(), off);
    int32_t sizes[2] = {0, 0};  // 2m' of the union, new vertex count
    check_hip(hipMemcpyAsync(&sizes[0], wpre.get() + NW, sizeof(int32_t), hipMemcpyDeviceToHost, s), "sample total");
    check_hip(hipMemcpyAsync(&sizes[1], off + K, sizeof(int32_t), hipMemcpyDeviceToHost, s), "union vertices");
    check_hip(hipStreamSynchronize(s), "sync");
    const int64_t total = sizes[0], nU2 = sizes[1];
    // 3. the compacted union: rows at the new ids, kept entries relabelled
    out->n = nU2;
    out->m = total / 2;
    out->row_ptr = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(nU2 + 1), s);
    out->deg = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(nU2 > 0 ? nU2 : 1), s);
    out->col = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s);
    out->src = (int32_t*)dev_alloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s);
    TC_LAUNCH("nz_place", k_nz_place, dim3(grid_for(nU, 256)), dim3(256), 0, s, nU, npad, K, (const int32_t*)rp.get(),
              (const int32_t*)deg.get(), (const uint64_t*)nzb.get(), (const int32_t*)nzpre.get(), (const int32_t*)off,
              out->row_ptr, out->deg, comp);
    DevBuf<int4> nzt(NV, s);
    TC_LAUNCH("nz_table", k_nz_table, dim3(grid_for(NV, 256)), dim3(256), 0, s, NV, npad, (const uint64_t*)nzb.get(),
              (const int32_t*)nzpre.get(), (const int32_t*)off, nzt.get());
    TC_LAUNCH("compact_rep", k_compact_rep, dim3(grid_for((NWp + kRepWords - 1) / kRepWords, 4)), dim3(256), 0, s,
              (const int32_t*)g->col,
              (const int32_t*)g->src, E2, NWp, K, npad, (const uint64_t*)bits.get(), (const int32_t*)wpre.get(),
              (const int4*)nzt.get(), out->col, out->src);
    TC_LAUNCH("comp_edges", k_comp_edges, dim3(ceil_div(K, 256)), dim3(256), 0, s, K, (const int32_t*)off,
              (const int32_t*)out->row_ptr, mk);
}

void comp_from_offsets(int64_t n, int32_t K, const int32_t* off, int32_t* comp, hipStream_t s) {
    if (n > 0 && K > 0)
        TC_LAUNCH("comp_from_off", k_comp_from_off, dim3(grid_for(n, 256)), dim3(256), 0, s, n, K, off, comp);
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
