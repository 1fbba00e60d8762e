// Exact triangle count of a (possibly sparsified) graph with the light/heavy
// vertex partition of section 3.2.
//
//   1. the counted graph: the input CSR, or the entries kept by the section
//      3.1 coin compacted into a CSR of their own, and its degrees;
//   2. orientation u -> v iff (deg u, u) < (deg v, v); every triangle is
//      charged to its lowest-ranked vertex.  Heavy vertices (deg > c m^(1/2))
//      rank above every light vertex, so a triangle whose lowest vertex is
//      heavy has three heavy vertices;
//   3. light phase: for every light u, the wedges of section 3.2 (pairs of
//      out-neighbours) are closed by counting, for each v in N+(u), the
//      common members of N+(u) and N+(v).  Only the third edge of a wedge
//      needs a test (section 4.2).  N+(u) is first sorted into rank order,
//      so that only its members ranked above v can close (u, v); the test
//      streams that part of N+(u), or N+(v), whichever is shorter, through an
//      LDS hash set of the other list: pairs of the first kind are grouped by
//      v (N+(v) staged once, the parts of its light in-neighbours' lists
//      streamed), the others by u;
//   4. heavy phase: the < 2 m^(1/2) / c heavy vertices, in rank order, form a
//      strictly upper-triangular 0/1 matrix U; sum((U U) .* U) counts each
//      all-heavy triangle once (the matrix-multiplication route of Alon,
//      Yuster and Zwick that section 2.1 and section 3 build on) and runs on
//      int8 MFMA with int32 accumulation.
#include "tc_internal.h"
#include "tc_device.h"

#include <atomic>

#include <algorithm>
#include <cmath>
#include <vector>

namespace tc {

namespace {

enum Acc {
    kTL = 0, kTH, kLightSources, kLightOut, kWedges, kGather, kProbes, kDmaxLarge, kBytesSmall, kBytesLarge,
    kItemsSmall, kItemsLarge, kMp, kH, kHeavyOverflow, kAccN
};
static_assert(kAccN <= kCountSlots, "count result slots");

unsigned grid_for(int64_t N, int threads) {
    unsigned b = ceil_div(N, threads);
    if (b > 65536) b = 65536;
    return b ? b : 1;
}

// Blocks of the classification pass (one partial of its statistics each).
constexpr unsigned kClassifyBlocks = 2048;

// Entries of an iterated list processed by one work item.
constexpr int kJL = 256;
// Tiny items (k_light_tiny): at most kTinyKeys anchor keys and iterated
// descriptors and kTinyPositions streamed positions, kTinyLanes lanes each
constexpr int kTinyLanes = 8;
constexpr int kTinyKeys = 8;
constexpr int kTinyPositions = 64;
// Largest anchor out-degree whose table the block kernel keeps in LDS.
constexpr int kLdsDcap = 1024;
// Strips of 64 positions per super-strip of the closure loop.
constexpr int kU = 4;

// ---------------------------------------------------------------------------
// orientation
// ---------------------------------------------------------------------------

// A byte that orders degrees: the degree itself below 16, above it 8 steps
// per octave (exponent and the three bits after the leading one), so
// class(d) < class(d') implies d < d', and equal classes below 16 mean equal
// degrees.  At most 16 + 8 * 26 + 7 = 231.
__device__ __forceinline__ uint32_t deg_class(int32_t d) {
    if (d < 16) return d > 0 ? (uint32_t)d : 0u;
    const int e = 31 - __builtin_clz((uint32_t)d);  // >= 4
    return 16u + 8u * (uint32_t)(e - 4) + (((uint32_t)d >> (e - 3)) & 7u);
}

__global__ void k_deg_class(int64_t n, const int32_t* __restrict__ degp, uint8_t* __restrict__ cls) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        cls[x] = (uint8_t)deg_class(degp[x]);
}

// the degree class of every entry's neighbour, gathered from the class array
// (one byte per vertex: a quarter of the degrees' footprint)
__global__ void k_neighbour_class(int64_t E2, const int32_t* __restrict__ col, const uint8_t* __restrict__ cls,
                                  uint8_t* __restrict__ ncls) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E2; e += (int64_t)gridDim.x * blockDim.x)
        ncls[e] = cls[col[e]];
}

// Per CSR entry (u, v) of a kept edge: "up" if (deg u, u) < (deg v, v).  Each
// kept undirected edge has exactly one up entry, in the row of its
// lower-ranked end.  The neighbour's degree class comes from ncls (one byte
// per entry, in order) when the graph itself is counted, else from a random
// lookup of the class array (one byte per vertex); only ties of classes above
// 15 (about 7% of R-MAT's entries) read the exact degrees; the entry streams
// bypass the cache.  E2 bounds the buffers; E2_dev (if not null) holds the
// number of valid entries, which may be smaller (a compacted sample in buffers
// sized for the full graph): words past it get zero bits.  Each wave takes 4
// words (256 entries) per step and issues all their loads before the first
// use, the class gathers likewise.
__global__ void __launch_bounds__(256) k_orient_bits(const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                                                      int64_t E2, const int32_t* __restrict__ E2_dev,
                                                      const uint8_t* __restrict__ cls,
                                                      const uint8_t* __restrict__ ncls,
                                                      const int32_t* __restrict__ degp, uint64_t* __restrict__ ubits,
                                                      int32_t* __restrict__ ucnt) {
    const int lane = __lane_id();
    const int64_t NW = (E2 + 63) / 64;
    const int64_t valid = E2_dev ? (int64_t)E2_dev[0] : E2;
    const int64_t NWv = (valid + 63) / 64;  // words holding valid entries
    const int64_t last = valid > 0 ? valid - 1 : 0;
    const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    // words past the valid entries only need a zero count (the scan runs over
    // all NW words; their bits are never read)
    for (int64_t w = NWv + (wave * 64 + lane); w < NW; w += nwaves * 64) ucnt[w] = 0;
    for (int64_t w0 = wave * 4; w0 < NWv; w0 += nwaves * 4) {
        int32_t u[4], v[4];
        uint32_t nc[4];
        bool in[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t e = (w0 + k) * 64 + lane;
            const int64_t ec = e < last ? e : last;  // loads stay inside the buffers
            in[k] = e < valid;
            const int32_t a = __builtin_nontemporal_load(src + ec), c = __builtin_nontemporal_load(col + ec);
            u[k] = in[k] ? a : 0;  // vertex 0 exists whenever a count runs
            v[k] = in[k] ? c : 0;
            nc[k] = ncls ? (uint32_t)__builtin_nontemporal_load(ncls + ec) : 0u;
        }
        uint32_t cu[4], cv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            cu[k] = cls[u[k]];
            cv[k] = ncls ? (in[k] ? nc[k] : cls[0]) : cls[v[k]];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            bool below = cu[k] < cv[k];
            if (cu[k] == cv[k]) {
                if (cu[k] < 16) below = u[k] < v[k];  // equal degrees
                else below = rank_below(degp[u[k]], u[k], degp[v[k]], v[k]);
            }
            const bool up = in[k] && below;
            const uint64_t bu = ballot64(up);
            if (lane == k && w0 + k < NWv) {
                ubits[w0 + k] = bu;
                ucnt[w0 + k] = __popcll(bu);
            }
        }
    }
}

// int32 words of one 4-wave block's table, list staging and flags (one byte
// per position, 64 kU per wave; 16-byte multiple).  With the largest table
// (dcap = 1024) a block takes 19.5 KB, so 8 blocks fit a CU's LDS.
__host__ __device__ inline int64_t large_block_words(int32_t dcap) {
    return (4 * (int64_t)dcap + 2 * kJL + 1 + 64 * kU + 3) / 4 * 4;
}

// Heavy block: U is stored padded to a multiple of the MFMA macro tile edge.
constexpr int kHT = 128;
__host__ __device__ inline int64_t heavy_pad(int64_t h) { return (h + kHT - 1) / kHT * kHT; }

// ---------------------------------------------------------------------------
// classification and light work
// ---------------------------------------------------------------------------

// b^2 deg^2 > a^2 m without overflow: the entry points cap a and b at 2^15 and
// m < 2^30 (2m fits int32), so a^2 m < 2^60; x = b deg < 2^46, and x >= 2^31
// already gives x^2 >= 2^62 > a^2 m.
__device__ __forceinline__ bool is_heavy(int64_t deg, int64_t m, int32_t a, int32_t b) {
    const uint64_t x = (uint64_t)(uint32_t)b * (uint64_t)deg;
    const uint64_t y = (uint64_t)(uint32_t)a * (uint64_t)(uint32_t)a * (uint64_t)m;
    if (x >> 31) return true;
    return x * x > y;
}

// The device's heavy count, clamped to the host bound every heavy buffer is
// sized for (it always holds: h < 2 m'^(1/2) / c; k_heavy_list flags a
// violation, which the read-back turns into TC_ERR_OVERFLOW).
__device__ __forceinline__ int32_t heavy_count(const int32_t* h_dev, int32_t hmax) {
    const int32_t h = h_dev[0];
    return h < hmax ? h : hmax;
}

// Orders one wave's shared-table writes before its later reads.  LDS
// operations of a wave are executed and complete in issue order, so for
// tables in LDS only the compiler must be kept from moving accesses across
// (fences and the wave barrier); no wait is needed, and global loads stay in
// flight.  Tables in global scratch (GLOBAL) need every outstanding access
// drained.
template <bool GLOBAL>
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (GLOBAL) __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void wave_lds_sync() { wave_sync<false>(); }

// Pair (u, v), u a light source, whose test streams len entries of N+(u)
// (the members of N+(u) ranked above v, or all of N+(u)) or the d+(v) entries
// of N+(v): closed from v's side ("v-major": stage N+(v), stream the part of
// N+(u)) when that part is the shorter list and N+(v) fits the staging cap;
// else from u's side (stage N+(u), stream N+(v)).
__device__ __forceinline__ bool vmajor(int32_t len, int32_t dv, int32_t vcap) {
    return len <= dv && dv <= vcap;
}

// Up entries before CSR position e of the counted graph: the word prefix of
// the orientation bits plus the set bits below e in its word (E2 bounds the
// buffers; positions at or past the valid entries have no bits below them).
__device__ __forceinline__ int32_t up_before(int64_t e, int64_t E2, const uint64_t* __restrict__ ubits,
                                             const int32_t* __restrict__ upre) {
    if (e >= E2) return upre[(E2 + 63) >> 6];
    const int r = (int)(e & 63);
    const uint64_t below = r == 0 ? 0ull : (ubits[e >> 6] & (~0ull >> (64 - r)));
    return upre[e >> 6] + __popcll(below);
}

// Per vertex, everything the light phase needs of it: the start of its up
// list, rpO[x] (x <= n), and d+(x), from the orientation bits at its row
// start; the heavy flag; code = d+(x) if x is a light source (light,
// d+ >= 2), else 0 (in a union of components, m' is that of x's component:
// mk[comp[x]]); rowQ[x] = (start of
// N+(x), code ? d+ : ~d+, deg, 0), what the anchor work gathers of a vertex in
// one 16-byte load; rpD[x], the first slot of x's v-major descriptors: the
// in-degrees d- = deg - d+ of the vertices before x, that is x's row start in
// the counted graph (row) minus its start in the up lists (rpO); and
// cw[x] = rpD[x] << 32 (see claim_vmajor).  Also clears the counts of the
// three wide-list classes, wide[c * (n + 1)], and stores the up lists'
// sentinel (-2, past the last possible up entry).
__global__ void k_vertex_prep(int64_t n, int64_t E2, const uint64_t* __restrict__ ubits,
                              const int32_t* __restrict__ upre, const int32_t* __restrict__ degp,
                              const int32_t* __restrict__ mp_dev, const int32_t* __restrict__ comp,
                              const int64_t* __restrict__ mk, int32_t ha, int32_t hb, const int32_t* __restrict__ row,
                              int32_t* __restrict__ rpO, int32_t* __restrict__ dplus, int32_t* __restrict__ heavy,
                              int32_t* __restrict__ code, int32_t* __restrict__ rpD, int4* __restrict__ rowQ,
                              unsigned long long* __restrict__ cw, int32_t* __restrict__ wide,
                              int32_t* __restrict__ sentinel) {
    const int64_t mp = comp ? 0 : mp_dev[0];
    if (blockIdx.x == 0 && threadIdx.x < 3) wide[threadIdx.x * (n + 1)] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *sentinel = -2;  // read by the closure past a range's positions
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= n; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t rx = row[x];
        const int32_t r = up_before(rx, E2, ubits, upre);
        rpO[x] = r;
        const int32_t dslot = rx - r;
        rpD[x] = dslot;
        if (x == n) break;
        const int32_t dp = up_before(row[x + 1], E2, ubits, upre) - r;
        dplus[x] = dp;
        const int32_t dg = degp[x];
        const bool hv = dg > 0 && is_heavy(dg, comp ? mk[comp[x]] : mp, ha, hb);
        heavy[x] = hv ? 1 : 0;
        const int32_t c = !hv && dp >= 2 ? dp : 0;
        code[x] = c;
        rowQ[x] = make_int4(r, c ? c : ~dp, dg, 0);
        cw[x] = (unsigned long long)(uint32_t)dslot << 32;
    }
}

// Longest out-list that the anchor work sorts into rank order (one wave, in
// registers).  A longer list keeps CSR order and each of its pairs streams all
// of it.
constexpr int kSortCap = 1024;

// The rank (deg, id) as one unsigned integer: rank_below(du, u, dv, v) iff
// rank_key(du, u) < rank_key(dv, v).
__device__ __forceinline__ uint64_t rank_key(int32_t deg, int32_t w) {
    return ((uint64_t)(uint32_t)deg << 32) | (uint32_t)w;
}

// The descriptor of pair (u, v) of the anchor work, for packU[rs + k]: v is
// entry k of N+(u) (rs = start of N+(u), d = d+(u)), qv = rowQ[v].  If N+(u)
// is in rank order, only its entries after k can close (u, v) (a common
// out-neighbour w of u and v ranks above v), and a pair with none gets (0, 0).
// u-major: (start of N+(v), d+(v)).  v-major: (start of the streamed part of
// N+(u), minus its length), placed by the caller through claim_vmajor.
__device__ __forceinline__ int2 pair_desc(int32_t rs, int32_t d, int32_t k, int4 qv, bool sorted, int32_t vcap,
                                          int64_t& wu, int64_t& gsum) {
    const int32_t dv = qv.y >= 0 ? qv.y : ~qv.y;
    gsum += dv;
    const int32_t len = sorted ? d - 1 - k : d;
    if (len <= 0) return make_int2(0, 0);
    if (vmajor(len, dv, vcap)) return make_int2(sorted ? rs + k + 1 : rs, -len);
    wu += dv;
    return make_int2(qv.x, dv);
}

// Claim the next slot of v's v-major descriptors: one atomic on cw[v], which
// starts at rpD[v] << 32 and gains (1 << 32) + length per descriptor (the
// lengths of one vertex sum to at most m' < 2^31); returns the slot.
__device__ __forceinline__ int64_t claim_vmajor(unsigned long long* cw, int32_t v, int32_t len) {
    return (int64_t)(atomicAdd(&cw[v], (1ull << 32) | (uint32_t)len) >> 32);
}

// lane ^ J exchange (J a power of two below 64)
template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
    if constexpr (J < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (J << 10) | 0x1F);
    else return (uint32_t)__shfl_xor((int)v, J, 64);
}

template <int J>
__device__ __forceinline__ uint64_t lane_xor64(uint64_t v) {
    return ((uint64_t)lane_xor<J>((uint32_t)(v >> 32)) << 32) | lane_xor<J>((uint32_t)v);
}

// c ? a : b as two 32-bit selects (keeps the sorting networks free of branches)
__device__ __forceinline__ uint64_t sel64(bool c, uint64_t a, uint64_t b) {
    const uint32_t lo = c ? (uint32_t)a : (uint32_t)b;
    const uint32_t hi = c ? (uint32_t)(a >> 32) : (uint32_t)(b >> 32);
    return ((uint64_t)hi << 32) | lo;
}

// Merge steps J, J/2, .., 1 of stage K of a bitonic network over each aligned
// group of G lanes (key, idx pairs): runs of K lanes alternate ascending and
// descending, and the last stage (K = G) sorts every group ascending.
template <int G, int K, int J>
__device__ __forceinline__ void bitonic_steps(uint64_t& key, int32_t& idx, int lane) {
    if constexpr (J > 0) {
        const uint64_t ok = lane_xor64<J>(key);
        const int32_t oi = (int32_t)lane_xor<J>((uint32_t)idx);
        const bool asc = K == G || (lane & K) == 0;
        const bool keep_min = asc == ((lane & J) == 0);
        const bool take = (ok < key) == keep_min;  // equal keys are interchangeable padding
        key = sel64(take, ok, key);
        idx = take ? oi : idx;
        bitonic_steps<G, K, J / 2>(key, idx, lane);
    }
}

// Ascending sort of the keys within each aligned group of G lanes (G a power
// of two <= 64), each key carrying idx along.
template <int G, int K = 2>
__device__ __forceinline__ void bitonic_lanes(uint64_t& key, int32_t& idx, int lane) {
    bitonic_steps<G, K, K / 2>(key, idx, lane);
    if constexpr (K < G) bitonic_lanes<G, 2 * K>(key, idx, lane);
}

// Merge steps J, .., 1 of stage K of a bitonic network over the 64 R keys of
// a wave held as position i = lane + 64 r (r < R): partners 64 apart or more
// sit in the same lane (a register swap), closer ones in the same register
// (a lane exchange).
template <int R, int K, int J>
__device__ __forceinline__ void wide_steps(uint64_t (&key)[R], int lane) {
    if constexpr (J > 0) {
        if constexpr (J >= 64) {
            constexpr int D = J / 64;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if ((r & D) == 0) {
                    const bool asc = ((64 * r) & K) == 0;
                    const uint64_t a = key[r], b = key[r | D];
                    const bool sw = (b < a) == asc;
                    key[r] = sel64(sw, b, a);
                    key[r | D] = sel64(sw, a, b);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t ok = lane_xor64<J>(key[r]);
                const bool asc = ((lane + 64 * r) & K) == 0;
                const bool keep_min = asc == ((lane & J) == 0);
                key[r] = sel64((ok < key[r]) == keep_min, ok, key[r]);
            }
        }
        wide_steps<R, K, J / 2>(key, lane);
    }
}

// Ascending sort of 64 R keys, position i = lane + 64 r.
template <int R, int K = 2>
__device__ __forceinline__ void bitonic_wide(uint64_t (&key)[R], int lane) {
    wide_steps<R, K, K / 2>(key, lane);
    if constexpr (K < 64 * R) bitonic_wide<R, 2 * K>(key, lane);
}

// Block reduction of the gather statistic into acc (256 threads).
__device__ __forceinline__ void add_gather(int64_t gsum, int64_t* acc) {
    gsum = wave_sum(gsum);
    __shared__ int64_t red[4];
    if (__lane_id() == 0) red[threadIdx.x >> 6] = gsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t t = red[0] + red[1] + red[2] + red[3];
        if (t) atomicAdd((unsigned long long*)&acc[kGather], (unsigned long long)t);
    }
}

// The lists of one 64-vertex window (q = rowQ of this lane's vertex) in mask
// whose lengths fit G lanes: 64 / G lists at a time, one per aligned group of
// G lanes, each sorted into rank order and written back, with the
// descriptors of its pairs and its Wu.
template <int G>
__device__ __forceinline__ void work_groups(uint64_t mask, const int4& q, int64_t x0, int lane,
                                            const int4* __restrict__ rowQ, int32_t* __restrict__ colO, int32_t vcap,
                                            int2* __restrict__ packU, int2* __restrict__ packD,
                                            unsigned long long* __restrict__ cw, int64_t* __restrict__ Wu,
                                            int64_t* __restrict__ Gx, int64_t& gsum) {
    constexpr int P = 64 / G;
    const int grp = lane / G;
    const int pos = lane & (G - 1);
    while (mask) {
        int mine = -1;  // window lane of this group's list
#pragma unroll
        for (int j = 0; j < P; ++j) {
            if (mask) {
                const int l = __builtin_ctzll(mask);
                mask &= mask - 1;
                if (grp == j) mine = l;
            }
        }
        // both shuffles run in every lane: a lane reads a list's length from
        // the window lane that holds it, which need not own a list itself
        const int sl = mine < 0 ? 0 : mine;
        const int32_t rs = __shfl(q.x, sl, 64);
        const int32_t dl = __shfl(q.y, sl, 64);
        const int32_t d = mine < 0 ? 0 : dl;
        const bool in = pos < d;
        const int32_t w = in ? colO[rs + pos] : 0;
        const int4 qw = in ? rowQ[w] : make_int4(0, 0, 0, 0);
        uint64_t key = in ? rank_key(qw.z, w) : ~0ull;
        int32_t idx = lane;
        bitonic_lanes<G>(key, idx, lane);
        // rowQ of the vertex that lands on this lane, from the lane that loaded it
        const int4 qv = make_int4(__shfl(qw.x, idx, 64), __shfl(qw.y, idx, 64), 0, 0);  // (start, code) are what pair_desc reads
        int64_t wu = 0, gl = 0;
        if (in) {
            const int32_t v = (int32_t)(uint32_t)key;
            colO[rs + pos] = v;
            int2 pk = pair_desc(rs, d, pos, qv, true, vcap, wu, gl);
            if (pk.y < 0) {
                packD[claim_vmajor(cw, v, -pk.y)] = make_int2(pk.x, -pk.y);
                pk = make_int2(0, 0);
            }
            packU[rs + pos] = pk;
        }
        gsum += gl;
#pragma unroll
        for (int J = G / 2; J >= 1; J >>= 1) wu += __shfl_xor(wu, J, 64);
        if (pos == 0 && mine >= 0) Wu[x0 + mine] = wu;
        if (Gx) {  // per-list gather statistic (unions of components)
#pragma unroll
            for (int J = G / 2; J >= 1; J >>= 1) gl += __shfl_xor(gl, J, 64);
            if (pos == 0 && mine >= 0) Gx[x0 + mine] = gl;
        }
    }
}

// Descriptors of up to B strips of 64 pairs of one list (v in the low half
// of vk[b], at position k0 + 64 b + lane): all rowQ gathers first, then all
// atomics, then the stores, so that a list waits for one round of each.
template <int B>
__device__ __forceinline__ void strip_work(const uint64_t (&vk)[B], int32_t k0, int32_t rs, int32_t d, bool sorted,
                                           int lane, const int4* __restrict__ rowQ, int32_t* __restrict__ colO,
                                           int32_t vcap, int2* __restrict__ packU, int2* __restrict__ packD,
                                           unsigned long long* __restrict__ cw, int64_t& wu, int64_t& gsum) {
    int4 qv[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int32_t k = k0 + 64 * b + lane;
        qv[b] = k < d ? rowQ[(int32_t)(uint32_t)vk[b]] : make_int4(0, 0, 0, 0);
    }
    int2 pk[B];
    int64_t slot[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int32_t k = k0 + 64 * b + lane;
        pk[b] = k < d ? pair_desc(rs, d, k, qv[b], sorted, vcap, wu, gsum) : make_int2(0, 0);
        slot[b] = pk[b].y < 0 ? claim_vmajor(cw, (int32_t)(uint32_t)vk[b], -pk[b].y) : 0;
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int32_t k = k0 + 64 * b + lane;
        if (k < d) {
            if (pk[b].y < 0) {
                packD[slot[b]] = make_int2(pk[b].x, -pk[b].y);
                pk[b] = make_int2(0, 0);
            }
            packU[rs + k] = pk[b];
            if (sorted) colO[rs + k] = (int32_t)(uint32_t)vk[b];
        }
    }
}

// One list of 64 (R - 1) < d <= 64 R entries: loaded into registers
// (position lane + 64 r), sorted into rank order, written back with the
// descriptors of its pairs.  The rank keys come from rowQ, so that the
// descriptors' rowQ gathers after the sort find their lines in the cache.
template <int R>
__device__ __forceinline__ void work_wide_list(int32_t rs, int32_t d, int lane, const int4* __restrict__ rowQ,
                                               int32_t* __restrict__ colO, int32_t vcap, int2* __restrict__ packU,
                                               int2* __restrict__ packD, unsigned long long* __restrict__ cw,
                                               int64_t& wu, int64_t& gsum) {
    int32_t w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lane + 64 * r;
        w[r] = i < d ? colO[rs + i] : 0;
    }
    uint64_t key[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lane + 64 * r;
        key[r] = i < d ? rank_key(rowQ[w[r]].z, w[r]) : ~0ull;
    }
    bitonic_wide<R>(key, lane);
    constexpr int B = R < 4 ? R : 4;
#pragma unroll
    for (int r0 = 0; r0 < R; r0 += B) {
        uint64_t vk[B];
#pragma unroll
        for (int b = 0; b < B; ++b) vk[b] = key[r0 + b];
        strip_work<B>(vk, 64 * r0, rs, d, true, lane, rowQ, colO, vcap, packU, packD, cw, wu, gsum);
    }
}

// The lists of one window in mask, one wave per list, with 32 R < d <= 64 R
// (R = 16 also takes the lists longer than kSortCap, which keep their order
// and whose pairs stream all of N+(u)); writes their Wu.
template <int R>
__device__ __forceinline__ void work_wide_lists(uint64_t mask, const int4& q, int64_t x0, int lane,
                                                const int4* __restrict__ rowQ, int32_t* __restrict__ colO,
                                                int32_t vcap, int2* __restrict__ packU, int2* __restrict__ packD,
                                                unsigned long long* __restrict__ cw, int64_t* __restrict__ Wu,
                                                int64_t* __restrict__ Gx, int64_t& gsum) {
    while (mask) {
        const int l = __builtin_ctzll(mask);
        mask &= mask - 1;
        const int32_t rs = __builtin_amdgcn_readlane(q.x, l);
        const int32_t d = __builtin_amdgcn_readlane(q.y, l);
        int64_t wu = 0, gl = 0;
        if (d <= 64 * R) {
            work_wide_list<R>(rs, d, lane, rowQ, colO, vcap, packU, packD, cw, wu, gl);
        } else {
            for (int32_t k0 = 0; k0 < d; k0 += 256) {
                uint64_t vk[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int32_t k = k0 + 64 * b + lane;
                    vk[b] = k < d ? (uint32_t)colO[rs + k] : 0;
                }
                strip_work<4>(vk, k0, rs, d, false, lane, rowQ, colO, vcap, packU, packD, cw, wu, gl);
            }
        }
        gsum += gl;
        wu = wave_sum(wu);
        if (lane == 0) Wu[x0 + l] = wu;
        if (Gx) {  // per-list gather statistic (unions of components)
            gl = wave_sum(gl);
            if (lane == 0) Gx[x0 + l] = gl;
        }
    }
}

// Appends the vertices of mask (window x0) to list L (count at L[-1]):
// one atomic per wave.
__device__ __forceinline__ void append_rows(uint64_t mask, int64_t x0, int lane, int32_t* __restrict__ L) {
    if (!mask) return;
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(&L[-1], (int32_t)__popcll(mask));
    base = __shfl(base, 0, 64);
    if ((mask >> lane) & 1ull) L[base + (int32_t)__popcll(mask & lanes_below())] = (int32_t)(x0 + lane);
}

// Anchor work of the light sources with d+ <= 128: each wave takes 64
// consecutive vertices per step, sorts their lists of up to 64 entries in lane
// groups of 4 to 64 and those of 65 to 128 entries in two registers per lane,
// and writes Wu (the length u-major pairs stream) of all of them, 0 for the
// longer lists, which it appends to the lists of k_work_wide's classes
// (wide[c * (n + 1)] holds the count of class c, its vertices follow).
__global__ void __launch_bounds__(256) k_work_lanes(int64_t n, const int4* __restrict__ rowQ,
                                                     int32_t* __restrict__ colO, int32_t vcap,
                                                     int2* __restrict__ packU, int2* __restrict__ packD,
                                                     unsigned long long* __restrict__ cw, int64_t* __restrict__ Wu,
                                                     int64_t* __restrict__ Gx, int32_t* __restrict__ wide,
                                                     int64_t* __restrict__ acc) {
    const int lane = __lane_id();
    const int64_t gw = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * 4;
    int64_t gsum = 0;
    for (int64_t x0 = gw * 64; x0 < n; x0 += nw * 64) {
        const int64_t x = x0 + lane;
        const int4 q = x < n ? rowQ[x] : make_int4(0, 0, 0, 0);
        const int32_t d = q.y;
        if (x < n && !(d >= 2 && d <= 128)) Wu[x] = 0;
        work_groups<4>(ballot64(d >= 2 && d <= 4), q, x0, lane, rowQ, colO, vcap, packU, packD, cw, Wu, Gx, gsum);
        work_groups<8>(ballot64(d > 4 && d <= 8), q, x0, lane, rowQ, colO, vcap, packU, packD, cw, Wu, Gx, gsum);
        work_groups<16>(ballot64(d > 8 && d <= 16), q, x0, lane, rowQ, colO, vcap, packU, packD, cw, Wu, Gx, gsum);
        work_groups<32>(ballot64(d > 16 && d <= 32), q, x0, lane, rowQ, colO, vcap, packU, packD, cw, Wu, Gx, gsum);
        work_groups<64>(ballot64(d > 32 && d <= 64), q, x0, lane, rowQ, colO, vcap, packU, packD, cw, Wu, Gx, gsum);
        work_wide_lists<2>(ballot64(d > 64 && d <= 128), q, x0, lane, rowQ, colO, vcap, packU, packD, cw, Wu, Gx, gsum);
        append_rows(ballot64(d > 128 && d <= 256), x0, lane, wide + 1);
        append_rows(ballot64(d > 256 && d <= 512), x0, lane, wide + (n + 1) + 1);
        append_rows(ballot64(d > 512), x0, lane, wide + 2 * (n + 1) + 1);
    }
    if (!Gx) add_gather(gsum, acc);
}

// Anchor work of the light sources with 32 R < d+ <= 64 R (R = 16: every
// d+ > 512), one wave per list, over the vertex list L (count at L[-1]) that
// k_work_lanes appended; one instantiation per register class, so that the
// shorter classes keep their occupancy.  Writes Wu of its lists.
template <int R>
__global__ void __launch_bounds__(256) k_work_wide(const int32_t* __restrict__ L, const int4* __restrict__ rowQ,
                                                    int32_t* __restrict__ colO, int32_t vcap,
                                                    int2* __restrict__ packU, int2* __restrict__ packD,
                                                    unsigned long long* __restrict__ cw, int64_t* __restrict__ Wu,
                                                    int64_t* __restrict__ Gx, int64_t* __restrict__ acc) {
    static_assert(kSortCap == 64 * 16, "list classes of k_work_wide");
    const int lane = __lane_id();
    const int32_t cnt = L[-1];
    int64_t gsum = 0;
    for (int32_t i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); i < cnt;
         i += gridDim.x * 4) {
        const int32_t x = L[i];
        const int4 q = rowQ[x];  // wave-uniform
        work_wide_lists<R>(1ull, q, x, lane, rowQ, colO, vcap, packU, packD, cw, Wu, Gx, gsum);
    }
    if (!Gx) add_gather(gsum, acc);
}

__device__ __forceinline__ int32_t items_of(int64_t w, int32_t len) {
    return w > 0 ? (len + kJL - 1) / kJL : 0;
}

// Length total of x's v-major descriptors, and one past their last slot.
__device__ __forceinline__ int64_t cw_len(unsigned long long c) { return (int64_t)(c & 0xFFFFFFFFull); }
__device__ __forceinline__ int32_t cw_end(unsigned long long c) { return (int32_t)(c >> 32); }

// per vertex: item counts of the two bins (wave / block anchors), statistics
// and the model bytes of each light kernel:
//   per item: anchor row offsets (8 B) + staging N+(anchor) (4 B per entry);
//   per iterated descriptor (d+ of them for u-major, the v-major count): 8 B;
//   per probe: the streamed entry (4 B).
// Per-vertex part of the classification: the item counts of x's bin, and
// x's contribution to the statistics st (sources, out, wedges, probes,
// bytes_s, bytes_l, items_s, items_l) and to the largest block-bin d+.
__device__ __forceinline__ void classify_vertex(int64_t x, const int32_t* __restrict__ code,
                                                const int32_t* __restrict__ dplus, const int64_t* __restrict__ Wu,
                                                const unsigned long long* __restrict__ cw,
                                                const int32_t* __restrict__ rpD, int32_t small_dmax,
                                                int32_t* __restrict__ ntn, int32_t* __restrict__ nsm,
                                                int32_t* __restrict__ nlg, int32_t* __restrict__ nhg,
                                                int64_t (&st)[8], int64_t& dmax) {
    const int32_t c = code[x];
    const int32_t dp = dplus[x];
    if (c > 0) { st[0] += 1; st[1] += c; st[2] += (int64_t)c * (c - 1) / 2; }
    const unsigned long long c2 = cw[x];
    const int64_t wu = Wu[x], wv = cw_len(c2);
    const int32_t nv = cw_end(c2) - rpD[x];
    const int32_t cu = items_of(wu, dp);
    const int32_t cv = items_of(wv, nv);
    const int64_t bytes = (int64_t)(cu + cv) * (8 + 4 * (int64_t)dp) + (wu > 0 ? 8 * (int64_t)dp : 0) +
                          8 * (int64_t)(cv > 0 ? nv : 0) + 4 * (wu + wv);
    st[3] += wu + wv;
    const bool small = dp <= small_dmax;
    const bool huge = dp > kLdsDcap;
    // tiny: at most kTinyKeys keys and descriptors and kTinyPositions
    // positions per item, so one item per group of kTinyLanes lanes
    const bool tiny = small && dp <= kTinyKeys && (cv == 0 || nv <= kTinyKeys) && wu <= kTinyPositions &&
                      wv <= kTinyPositions;
    ntn[x] = tiny ? cu + cv : 0;
    nsm[x] = small && !tiny ? cu + cv : 0;
    nlg[x] = (!small && !huge) ? cu + cv : 0;
    nhg[x] = huge ? cu + cv : 0;
    if (small) { st[4] += bytes; st[6] += cu + cv; }
    else {
        st[5] += bytes;
        st[7] += cu + cv;
        if (cu + cv > 0) dmax = dp > dmax ? dp : dmax;
    }
}

__global__ void __launch_bounds__(256) k_classify(int64_t n, const int32_t* __restrict__ code,
                                                   const int32_t* __restrict__ dplus, const int64_t* __restrict__ Wu,
                                                   const unsigned long long* __restrict__ cw,
                                                   const int32_t* __restrict__ rpD, int32_t small_dmax,
                                                   int32_t* __restrict__ ntn, int32_t* __restrict__ nsm,
                                                   int32_t* __restrict__ nlg, int32_t* __restrict__ nhg,
                                                   int64_t* __restrict__ part) {
    int64_t st[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // sources, out, wedges, probes, bytes_s, bytes_l, items_s, items_l
    int64_t dmax = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        classify_vertex(x, code, dplus, Wu, cw, rpD, small_dmax, ntn, nsm, nlg, nhg, st, dmax);
    __shared__ int64_t red[4][9];
    const int wv_ = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 8; ++q) st[q] = wave_sum(st[q]);
    dmax = wave_max(dmax);
    if (__lane_id() == 0) {
        for (int q = 0; q < 8; ++q) red[wv_][q] = st[q];
        red[wv_][8] = dmax;
    }
    __syncthreads();
    // one partial per block (no contended atomics); k_finish folds them
    if (threadIdx.x < 9) {
        int64_t v = red[0][threadIdx.x];
        for (int w = 1; w < 4; ++w) {
            const int64_t o = red[w][threadIdx.x];
            v = threadIdx.x == 8 ? (o > v ? o : v) : v + o;
        }
        part[(int64_t)blockIdx.x * 9 + threadIdx.x] = v;
    }
}

// The classification of a union of components: every block takes a
// contiguous range of whole 256-vertex windows (one component each, the
// component starts being multiples of kUnionAlign), and adds its statistics,
// the per-list gather statistic Gx of the light sources included, into the
// result slots of each component it covers.
__device__ __forceinline__ void flush_comp_stats(int32_t c, int64_t (&st)[8], int64_t& gth, int64_t& dmax,
                                                 int64_t* __restrict__ acc) {
    __shared__ int64_t red[4][10];
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 8; ++q) st[q] = wave_sum(st[q]);
    gth = wave_sum(gth);
    dmax = wave_max(dmax);
    if (__lane_id() == 0) {
        for (int q = 0; q < 8; ++q) red[w][q] = st[q];
        red[w][8] = gth;
        red[w][9] = dmax;
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        const int q = threadIdx.x;
        int64_t v = red[0][q];
        for (int i = 1; i < 4; ++i) v = q == 9 ? (red[i][q] > v ? red[i][q] : v) : v + red[i][q];
        const int slot[10] = {kLightSources, kLightOut, kWedges, kProbes, kBytesSmall, kBytesLarge, kItemsSmall,
                              kItemsLarge, kGather, kDmaxLarge};
        int64_t* a = acc + (int64_t)c * kCountSlots + slot[q];
        if (q == 9) atomicMax((unsigned long long*)a, (unsigned long long)v);
        else if (v) atomicAdd((unsigned long long*)a, (unsigned long long)v);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) st[q] = 0;
    gth = 0;
    dmax = 0;
}

__global__ void __launch_bounds__(256) k_classify_union(int64_t n, const int32_t* __restrict__ comp,
                                                         const int32_t* __restrict__ code,
                                                         const int32_t* __restrict__ dplus,
                                                         const int64_t* __restrict__ Wu,
                                                         const int64_t* __restrict__ Gx,
                                                         const unsigned long long* __restrict__ cw,
                                                         const int32_t* __restrict__ rpD, int32_t small_dmax,
                                                         int32_t* __restrict__ ntn, int32_t* __restrict__ nsm,
                                                         int32_t* __restrict__ nlg, int32_t* __restrict__ nhg,
                                                         int64_t* __restrict__ acc) {
    const int64_t windows = (n + 255) / 256;
    const int64_t per = (windows + gridDim.x - 1) / gridDim.x;
    const int64_t w0 = (int64_t)blockIdx.x * per;
    const int64_t w1 = min(windows, w0 + per);
    int64_t st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t gth = 0, dmax = 0;
    int32_t cur = -1;
    for (int64_t wi = w0; wi < w1; ++wi) {
        const int64_t xs = wi * 256;
        const int32_t c = comp[xs];  // block-uniform: one component per window
        if (c != cur) {
            if (cur >= 0) flush_comp_stats(cur, st, gth, dmax, acc);
            cur = c;
        }
        const int64_t x = xs + threadIdx.x;
        if (x < n) {
            classify_vertex(x, code, dplus, Wu, cw, rpD, small_dmax, ntn, nsm, nlg, nhg, st, dmax);
            if (code[x] > 0) gth += Gx[x];
        }
    }
    if (cur >= 0) flush_comp_stats(cur, st, gth, dmax, acc);
}

// items of anchor x: (x, r) for the u-major ranges r of N+(x), then (~x, r)
// for the ranges r of x's v-major descriptors
// The item lists of all four bins in one pass: an anchor's items go to the
// list of its bin (tiny, small, large or huge, exclusive) at its bin's prefix.
__global__ void k_items(int64_t n, const int32_t* __restrict__ ntn, const int32_t* __restrict__ nsm,
                        const int32_t* __restrict__ nlg, const int32_t* __restrict__ nhg,
                        const int32_t* __restrict__ tbase, const int32_t* __restrict__ sbase,
                        const int32_t* __restrict__ lbase, const int32_t* __restrict__ hbase,
                        const int32_t* __restrict__ dplus, const int64_t* __restrict__ Wu,
                        const unsigned long long* __restrict__ cw, const int32_t* __restrict__ rpD,
                        int2* __restrict__ items_t, int2* __restrict__ items_s, int2* __restrict__ items_l,
                        int2* __restrict__ items_h) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        int2* items;
        int32_t b;
        if (ntn[x]) { items = items_t; b = tbase[x]; }
        else if (nsm[x]) { items = items_s; b = sbase[x]; }
        else if (nlg[x]) { items = items_l; b = lbase[x]; }
        else if (nhg[x]) { items = items_h; b = hbase[x]; }
        else continue;
        const int32_t cu = items_of(Wu[x], dplus[x]);
        const unsigned long long c2 = cw[x];
        const int32_t cv = items_of(cw_len(c2), cw_end(c2) - rpD[x]);
        for (int32_t r = 0; r < cu; ++r) items[b++] = make_int2((int32_t)x, r);
        for (int32_t r = 0; r < cv; ++r) items[b++] = make_int2(~(int32_t)x, r);
    }
}

__global__ void k_heavy_list(int64_t n, const int32_t* __restrict__ heavy, const int32_t* __restrict__ hpos,
                             int32_t hmax, int32_t* __restrict__ hlist, int64_t* __restrict__ acc) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && hpos[n] > hmax) acc[kHeavyOverflow] = 1;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        if (heavy[x] && hpos[x] < hmax) hlist[hpos[x]] = (int32_t)x;
}

// zero the first heavy_pad(h)^2 bytes of U and UT (h from device)

// m', h and the classification statistics (sums of the per-block partials;
// the last one is a maximum).  One block of 576 threads.
__global__ void __launch_bounds__(576) k_finish(const int32_t* mp, const int32_t* hp,
                                                const int64_t* __restrict__ part, int32_t nparts, int64_t* acc) {
    // thread t folds statistic q = t % 9 of the blocks t / 9, t / 9 + 64, ..
    // (neighbouring threads read neighbouring words); then 64 values per q
    __shared__ int64_t red[64][9];
    const int t = threadIdx.x;
    const int q = t % 9, c = t / 9;
    // 8 independent loads in flight per thread and round (0 is neutral for
    // both the sums and the maximum of non-negative degrees)
    int64_t v = 0;
    for (int32_t b0 = c; b0 < nparts; b0 += 64 * 8) {
        int64_t x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t b = b0 + 64 * k;
            x[k] = b < nparts ? part[(int64_t)b * 9 + q] : 0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) v = q == 8 ? (x[k] > v ? x[k] : v) : v + x[k];
    }
    red[c][q] = v;
    __syncthreads();
    if (t < 9) {
        const int slot[9] = {kLightSources, kLightOut, kWedges, kProbes, kBytesSmall, kBytesLarge, kItemsSmall,
                             kItemsLarge, kDmaxLarge};
        int64_t r = red[0][t];
        for (int i = 1; i < 64; ++i) r = t == 8 ? (red[i][t] > r ? red[i][t] : r) : r + red[i][t];
        acc[slot[t]] = r;
    }
    if (t == 0) {
        acc[kMp] = mp[0];
        acc[kH] = hp[0];
    }
}

// m' and h of every component of a union: mk[k], and the heavy flags' prefix
// hpos at the component's bounds
__global__ void k_finish_union(int32_t K, const int32_t* __restrict__ off, const int64_t* __restrict__ mk,
                               const int32_t* __restrict__ hpos, int64_t* __restrict__ acc) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        acc[(int64_t)k * kCountSlots + kMp] = mk[k];
        acc[(int64_t)k * kCountSlots + kH] = hpos[off[k + 1]] - hpos[off[k]];
    }
}

// ---------------------------------------------------------------------------
// light closure
// ---------------------------------------------------------------------------

// multiplicative hash on the 24-bit multiplier (full-rate v_mul_u32_u24), with
// the high id bits folded in first.  HIP's __umul24 returns a signed int: the
// product is taken as unsigned before the shift, so the slot is its top lg bits.
__device__ __forceinline__ uint32_t hslot(int32_t w, int lg) {
    const uint32_t x = (uint32_t)w;
    const uint32_t prod = (x & 0xFFFFFFu) * 0x9E3779u + (x >> 24);  // v_mad_u32_u24
    return prod >> (32 - lg);
}

// The anchor's out-list is kept in a bucketed open-addressing table: 2^lg
// buckets of 4 slots (one 16-byte LDS read each), sized so that at most a
// quarter of the slots are used.  A key goes to the first bucket with a free
// slot along its probe sequence (home bucket, then the next ones).  An insert
// that finds all four slots of a bucket taken marks that bucket as passed
// over (the sign bit of its last slot; vertex ids are below 2^31 - 1, so a
// marked slot never reads as empty, -1) before it moves on.  Slots only ever
// change from empty to a key and from a key to the marked key, so after the
// inserts a key sits in its home bucket or further along a run of marked
// buckets, and a lookup stops at the first bucket that holds it or is not
// marked.
constexpr int32_t kPassed = (int32_t)0x80000000;  // mark on the last slot of a passed-over bucket
constexpr int32_t kKeyBits = 0x7FFFFFFF;

__device__ __forceinline__ void hash_insert(int32_t* tab, int lg, int32_t v) {
    const uint32_t mask = (1u << lg) - 1;
    uint32_t bk = hslot(v, lg) & mask;
    while (true) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int32_t prev = atomicCAS(&tab[4 * bk + s], -1, v);
            if (prev == -1 || (prev & kKeyBits) == v) return;
        }
        atomicOr(&tab[4 * bk + 3], kPassed);
        bk = (bk + 1) & mask;
    }
}

// Buckets for a table that holds d keys at load <= 1/4: 2^lg >= d, at least 16.
__device__ __forceinline__ int bucket_bits(int32_t d) {
    int lg = 4;
    while ((1 << lg) < d) ++lg;
    return lg;
}

// Buckets for d keys in a region of 2^lgmax buckets (lgmax >= bucket_bits(d)):
// 2^lg >= 2 d where the region allows it.  A lookup that misses in a
// passed-over home bucket walks on, one LDS read per bucket; at one key per
// bucket on average about one bucket in 300 is passed over, so a good share
// of the waves of 256 probes take that walk, and at half a key per bucket
// almost none.
__device__ __forceinline__ int table_bits(int32_t d, int lgmax) {
    const int lg = bucket_bits(2 * d);
    return lg < lgmax ? lg : lgmax;
}

// largest j in [0, d-1] with P[j] <= g  (P non-decreasing, P[0] = 0 <= g)
__device__ __forceinline__ int find_list(const int32_t* P, int d, int32_t g) {
    int lo = 0, hi = d - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}


// Membership tests of the keys x[k] against the bucketed table; returns the
// number of hits in the whole wave
// (wave-uniform).  One 16-byte read per key resolves it unless its home
// bucket was passed over by an insert and does not hold it (about one bucket
// in 300 at one key per bucket on average, one in 5000 at 0.6).  Every x[k]
// is a vertex id (>= 0) or, in lanes past the end of the positions, the
// sentinel -2, which matches no slot (slots hold ids, -1 or a marked id,
// whose low 31 bits are an id); such a lane can at most walk a marked run.
template <int U>
__device__ __forceinline__ int32_t probe_many(const int32_t* tab, int lg, const int32_t (&x)[U]) {
    const uint32_t mask = (1u << lg) - 1;
    const int4* t4 = reinterpret_cast<const int4*>(tab);
    uint32_t bk[U];
    int32_t found = 0;
    uint64_t live[U];
#pragma unroll
    for (int k = 0; k < U; ++k) bk[k] = hslot(x[k], lg);  // < 2^lg
    int4 e[U];
#pragma unroll
    for (int k = 0; k < U; ++k) e[k] = t4[bk[k]];
    uint64_t any = 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int32_t v = x[k];
        // one compare per slot straight into a wave mask (no per-lane booleans)
        const uint64_t hit = (ballot64(e[k].x == v) | ballot64(e[k].y == v) | ballot64(e[k].z == v) |
                              ballot64((e[k].w & kKeyBits) == v));
        const uint64_t passed = ballot64(e[k].w < -1);  // marked last slot
        found += (int32_t)__popcll(hit);
        live[k] = passed & ~hit;
        any |= live[k];
    }
    if (any) {  // rare: home bucket passed over and without the key
        const int lane = __lane_id();
#pragma unroll
        for (int k = 0; k < U; ++k) {
            bool on = (live[k] >> lane) & 1ull;
            while (ballot64(on)) {
                int32_t hitl = 0;
                if (on) {
                    bk[k] = (bk[k] + 1) & mask;
                    const int4 f = t4[bk[k]];
                    const int32_t v = x[k];
                    if (f.x == v || f.y == v || f.z == v || (f.w & kKeyBits) == v) { hitl = 1; on = false; }
                    else if (f.w >= -1) on = false;  // not passed over: the key is not further on
                }
                found += (int32_t)__popcll(ballot64(hitl != 0));
            }
        }
    }
    return found;
}

// Owners and gathers of one super-strip of 64 * U positions starting at g0
// (< b): position g lies in list j (P[j] <= g < P[j+1]) and reads
// colO[D[j] + g], D[j] being the list's start in colO minus P[j]; nl lists,
// none empty, so P is strictly increasing.  On entry jlo owns position g0 - 1
// (or g0), on exit position g0 + 64U - 1.  When no list starts inside the
// super-strip every lane owns jlo.  Otherwise the lists starting inside it (at
// most 64U, those after jlo) flag their start offsets in `mark` (64U bytes of
// per-wave memory, all zero between calls), and the owner of position
// g0 + 64k + lane is jlo plus the number of flags at offsets <= 64k + lane:
// one ballot and one mbcnt per strip of 64.  Whole wave.
template <int U, bool GLOBAL>
__device__ __forceinline__ void gather_strips(const int32_t* P, const int32_t* D, int nl, int32_t g0, int32_t b,
                                              const int32_t* __restrict__ colO, uint32_t sent, uint8_t* mark,
                                              int lane, int& jlo, int32_t (&x)[U]) {
    // every lane loads (lanes past b read colO[sent], which holds the sentinel
    // -2) and nothing consumes the loaded values before the probe, so these
    // loads stay in flight across the caller's other work
    const int32_t nxt = __builtin_amdgcn_readfirstlane(jlo + 1 < nl ? P[jlo + 1] : INT32_MAX);
    if (nxt >= g0 + 64 * U) {  // wave-uniform: one list covers the super-strip
        const int32_t d0 = D[jlo];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int32_t g = g0 + lane + 64 * k;
            x[k] = *(const int32_t*)((const char*)colO + ((uint32_t)(g < b ? d0 + g : sent) << 2));
        }
    } else {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int jf = jlo + 1 + 64 * k;  // first list of this group of 64 (wave-uniform)
            if (jf >= nl) break;
            if (k > 0 && __builtin_amdgcn_readfirstlane(P[jf]) >= g0 + 64 * U) break;  // group starts past it
            const int j = jf + lane;
            if (j < nl) {
                const int32_t off = P[j] - g0;  // >= 0: list jlo + 1 starts at g0 or later
                if (off < 64 * U) mark[off] = 1;
            }
        }
        wave_sync<GLOBAL>();
        int32_t base = jlo;
        int32_t dk[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int32_t f = mark[lane + 64 * k];
            const uint64_t M = ballot64(f != 0);
            const int32_t below = (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(M >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)M, 0u));
            dk[k] = D[base + below + f];  // the owner's offset (owner index < nl)
            base += (int32_t)__popcll(M);
            mark[lane + 64 * k] = 0;
        }
        jlo = base;
        wave_sync<GLOBAL>();  // flags cleared before the next super-strip sets any
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int32_t g = g0 + lane + 64 * k;
            x[k] = *(const int32_t*)((const char*)colO + ((uint32_t)(g < b ? dk[k] + g : sent) << 2));
        }
    }
}

// Closure tests for positions [a, b) of the concatenated streamed lists
// (layout as in gather_strips); returns the wave's number of hits.  Software-pipelined with two register sets:
// the gathers of the next super-strip are issued, unconditionally, before the
// hash probes of the current one, and no register copy waits on them.  SHORT
// adds unpipelined paths for ranges of at most one super-strip (worth it where
// most ranges are that short; elsewhere the extra code costs occupancy).
template <int U, bool GLOBAL, bool SHORT>
__device__ __forceinline__ int32_t close_flat(const int32_t* P, const int32_t* D, int nl, int32_t a, int32_t b,
                                              const int32_t* __restrict__ colO, uint32_t sent, const int32_t* tab,
                                              int lg, uint8_t* mark, int lane) {
    // a, b and nl are wave-uniform; saying so makes every exit of the
    // pipelined loop below a scalar branch.  Otherwise the loop is compiled
    // as a divergent one whose early exit reaches the loop head with the
    // other register set's gathers still in flight, and the compiler then
    // waits for all outstanding loads (vmcnt(0)) on every trip.
    a = __builtin_amdgcn_readfirstlane(a);
    b = __builtin_amdgcn_readfirstlane(b);
    nl = __builtin_amdgcn_readfirstlane(nl);
    int32_t cnt = 0;
    if (a >= b) return 0;
    int jlo = a == 0 ? 0 : __builtin_amdgcn_readfirstlane(find_list(P, nl, a));  // P[0] = 0 owns position 0
    if (SHORT && b - a <= 64) {  // one strip
        int32_t x1[1];
        gather_strips<1, GLOBAL>(P, D, nl, a, b, colO, sent, mark, lane, jlo, x1);
        return probe_many<1>(tab, lg, x1);
    }
    if (SHORT && b - a <= 64 * U) {  // one super-strip
        int32_t x1[U];
        gather_strips<U, GLOBAL>(P, D, nl, a, b, colO, sent, mark, lane, jlo, x1);
        return probe_many<U>(tab, lg, x1);
    }
    // super-strips i = 0 .. ns-1 start at a + i 64U.  The loop runs whole
    // pairs and has one exit, where only set a is in flight; the last one or
    // two super-strips follow it.
    constexpr int32_t S = 64 * U;
    const int32_t ns = (b - a + S - 1) / S;
    int32_t xa[U], xb[U];
    gather_strips<U, GLOBAL>(P, D, nl, a, b, colO, sent, mark, lane, jlo, xa);
    int32_t i = 0;
    for (; i + 2 < ns; i += 2) {
        gather_strips<U, GLOBAL>(P, D, nl, a + (i + 1) * S, b, colO, sent, mark, lane, jlo, xb);
        cnt += probe_many<U>(tab, lg, xa);
        gather_strips<U, GLOBAL>(P, D, nl, a + (i + 2) * S, b, colO, sent, mark, lane, jlo, xa);
        cnt += probe_many<U>(tab, lg, xb);
    }
    if (i + 1 < ns) {
        gather_strips<U, GLOBAL>(P, D, nl, a + (i + 1) * S, b, colO, sent, mark, lane, jlo, xb);
        cnt += probe_many<U>(tab, lg, xa);
        cnt += probe_many<U>(tab, lg, xb);
    } else {
        cnt += probe_many<U>(tab, lg, xa);
    }
    return cnt;
}

// Insert N+(x) (d entries at colO[rs..]) into the hash set; NT threads, thread t.
template <int NT>
__device__ __forceinline__ void build_hash(int32_t rs, int32_t d, const int32_t* __restrict__ colO, int32_t* tab,
                                           int lg, int t) {
    constexpr int R = 4;
    for (int j0 = 0; j0 < d; j0 += NT * R) {
        int32_t v[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int j = j0 + t + NT * k;
            v[k] = j < d ? colO[rs + j] : -1;
        }
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (v[k] >= 0) hash_insert(tab, lg, v[k]);
    }
}

// Stage the packed entries L[0..cnt) (cnt <= kJL) of an anchor's iterated
// list: (start in colO, length) of the list streamed for each entry, length 0
// when the pair is closed from the other side.  Non-empty lists are compacted
// in entry order into P (exclusive prefix of lengths, P[nl] = total) and D
// (start in colO minus P, so position g of list j reads colO[D[j] + g]).
// Returns nl; *total receives the number of positions.
template <int NT>
__device__ __forceinline__ void load_lists(const int2* __restrict__ L, int32_t cnt, int t,
                                           int32_t (&st)[(kJL + NT - 1) / NT], int32_t (&ln)[(kJL + NT - 1) / NT]) {
    constexpr int R = (kJL + NT - 1) / NT;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int j = t * R + k;  // consecutive entries per thread
        const int2 e = j < cnt ? L[j] : make_int2(0, 0);
        st[k] = e.x;
        ln[k] = e.y;
    }
}

template <int NT>
__device__ __forceinline__ int32_t stage_loaded(const int32_t (&st)[(kJL + NT - 1) / NT],
                                                const int32_t (&ln)[(kJL + NT - 1) / NT], int32_t* P, int32_t* D,
                                                int32_t* red, int t, int32_t* total) {
    constexpr int R = (kJL + NT - 1) / NT;
    int32_t loc = 0, nloc = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        loc += ln[k];
        nloc += ln[k] > 0 ? 1 : 0;
    }
    // two exclusive scans: positions and list slots
    int32_t ex, tot, nex, ntot;
    if (NT == 64) {
        const int32_t inc = wave_inclusive_sum(loc);
        ex = inc - loc;
        tot = __shfl(inc, 63, 64);
        const int32_t ninc = wave_inclusive_sum(nloc);
        nex = ninc - nloc;
        ntot = __shfl(ninc, 63, 64);
    } else {
        ex = block_exclusive_sum<NT>(loc, red, &tot);
        nex = block_exclusive_sum<NT>(nloc, red, &ntot);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (ln[k] > 0) {
            D[nex] = st[k] - ex;
            P[nex] = ex;
            ex += ln[k];
            ++nex;
        }
    }
    if (t == 0) P[ntot] = tot;
    *total = tot;
    return ntot;
}

template <int NT>
__device__ __forceinline__ int32_t stage_lists(const int2* __restrict__ L, int32_t cnt, int32_t* P, int32_t* D,
                                               int32_t* red, int t, int32_t* total) {
    constexpr int R = (kJL + NT - 1) / NT;
    int32_t st[R], ln[R];
    load_lists<NT>(L, cnt, t, st, ln);
    return stage_loaded<NT>(st, ln, P, D, red, t, total);
}

// One wave per item, persistent over items with a static stride.  Item
// (x, r): anchor x, kind u (x >= 0) or v (encoded ~x), entries r*kJL.. of the
// iterated list.  LDS per wave: hash (4*DS slots), P (kJL+1), D (kJL), flags
// (64 kU).  Items are short, so the chain of dependent loads that opens an
// item (item, row offsets, keys and list descriptors) is issued for the next
// item while the current one closes.
// Adds a wave's closure count of one component into that component's T_L.
__device__ __forceinline__ void flush_tl(int64_t* acc, int32_t c, int64_t total, int lane) {
    if (lane == 0 && total) atomicAdd((unsigned long long*)&acc[(int64_t)c * kCountSlots + kTL], (unsigned long long)total);
}

// UNION: the graph is a union of components (comp[x] of every vertex), and
// each item's closures count towards its anchor's component.  That variant
// is held to 7 waves per SIMD (72 VGPRs, as the other one compiles to), so
// that 7 blocks per CU (17.5 KB of LDS each) stay resident; left alone it
// takes 76 VGPRs and fits only 6.
template <int DS, bool UNION>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(UNION ? 7 : 1)))
k_light_small(const int2* __restrict__ items, const int32_t* __restrict__ n_items_dev, const int32_t* __restrict__ rpO,
              const int32_t* __restrict__ colO, const int32_t* __restrict__ rpD,
              const unsigned long long* __restrict__ cw, const int2* __restrict__ packU,
              const int2* __restrict__ packD, uint32_t sent, const int32_t* __restrict__ comp,
              int64_t* __restrict__ acc) {
    constexpr int HS_MAX = 4 * DS;                                     // buckets of 4 slots, load <= 1/4
    static_assert((DS & (DS - 1)) == 0 && DS >= 16, "DS: a power of two");
    constexpr int kLgDS = __builtin_ctz(DS);                           // the table region holds 2^kLgDS buckets
    constexpr int ROW = (HS_MAX + 2 * kJL + 1 + 16 * kU + 3) / 4 * 4;  // keeps every row 16-byte aligned
    constexpr int KR = (DS + 63) / 64;                                 // keys per lane
    constexpr int LR = (kJL + 63) / 64;                                // list descriptors per lane
    __shared__ __attribute__((aligned(16))) int32_t lds[4][ROW];
    const int w = threadIdx.x >> 6;
    const int lane = __lane_id();
    int32_t* tab = lds[w];
    int32_t* P = tab + HS_MAX;
    int32_t* D = P + kJL + 1;
    uint8_t* mark = reinterpret_cast<uint8_t*>(D + kJL);  // 64 kU bytes
    for (int i = lane; i < 16 * kU; i += 64) reinterpret_cast<int32_t*>(mark)[i] = 0;  // flags stay zero between super-strips
    const int64_t gw = (int64_t)blockIdx.x * 4 + w;
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int64_t n_items = n_items_dev[0];
    // the opening of item `it`: anchor x, its row (rs, d) and its iterated list (L, cnt)
    auto header = [&](int64_t it, int32_t& x, int32_t& rs, int32_t& d, const int2*& L, int32_t& cnt) {
        const int2 item = items[it];
        const bool kind_u = item.x >= 0;
        x = kind_u ? item.x : ~item.x;
        rs = rpO[x];
        d = rpO[x + 1] - rs;
        int32_t llen;
        if (kind_u) { L = packU + rs; llen = d; }
        else { const int32_t ds = rpD[x]; L = packD + ds; llen = cw_end(cw[x]) - ds; }
        const int32_t j0 = item.y * kJL;
        L += j0;
        cnt = min(kJL, llen - j0);
    };
    auto body = [&](int32_t rs, int32_t d, const int2* L, int32_t cnt, int32_t (&kv)[KR], int32_t (&st)[LR],
                    int32_t (&ln)[LR]) {
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int j = lane + 64 * k;
            kv[k] = j < d ? colO[rs + j] : -1;
        }
        load_lists<64>(L, cnt, lane, st, ln);
    };
    int64_t total = 0;
    int32_t cur = 0;  // component of the closures in total
    if (gw < n_items) {
        int32_t xa, rs, d, cnt;
        const int2* L;
        int32_t kv[KR], st[LR], ln[LR];
        header(gw, xa, rs, d, L, cnt);
        body(rs, d, L, cnt, kv, st, ln);
        if (UNION) cur = comp[xa];
        for (int64_t it = gw; it < n_items; it += nw) {
            const bool more = it + nw < n_items;  // wave-uniform
            int32_t xa2 = 0, rs2 = 0, d2 = 0, cnt2 = 0;
            const int2* L2 = L;
            if (more) header(it + nw, xa2, rs2, d2, L2, cnt2);
            if (UNION) {
                const int32_t c = comp[xa];
                if (c != cur) {
                    flush_tl(acc, cur, total, lane);
                    total = 0;
                    cur = c;
                }
            }
            const int lg = table_bits(d, kLgDS);
            const int hs = 4 << lg;
            for (int i = lane; i < hs / 4; i += 64) reinterpret_cast<int4*>(tab)[i] = make_int4(-1, -1, -1, -1);
            if (lane == 0) P[0] = 0;
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < KR; ++k)
                if (kv[k] >= 0) hash_insert(tab, lg, kv[k]);
            int32_t W;
            const int32_t nl = stage_loaded<64>(st, ln, P, D, nullptr, lane, &W);
            wave_lds_sync();
            if (more) body(rs2, d2, L2, cnt2, kv, st, ln);  // in flight during the closure
            total += close_flat<kU, false, true>(P, D, nl, 0, W, colO, sent, tab, lg, mark, lane);  // wave-uniform
            wave_lds_sync();
            xa = xa2;
            rs = rs2;
            d = d2;
            L = L2;
            cnt = cnt2;
        }
    }
    flush_tl(acc, cur, total, lane);
}

// One block (4 waves) per item for anchors with large out-lists.  The hash
// set and the list tables live in dynamic LDS (GLOBAL = false: the compiler
// sees the LDS address space and emits ds_* instructions), or in a global
// scratch slice per block when they do not fit (GLOBAL = true).  After
// staging, each wave closes a quarter of the item's positions.
// Broadcast of lane K of each group of 8 lanes, and the exchange with the
// lane X apart, inside the group (ds_swizzle bit mode on 32-lane halves).
template <int K>
__device__ __forceinline__ int32_t grp_lane(int32_t v) {
    return __builtin_amdgcn_ds_swizzle(v, 0x18 | (K << 5));
}
template <int X>
__device__ __forceinline__ int32_t grp_xor(int32_t v) {
    return __builtin_amdgcn_ds_swizzle(v, 0x1F | (X << 10));
}
template <int K = 0>
__device__ __forceinline__ void grp_all(int32_t v, int32_t (&out)[kTinyLanes]) {
    out[K] = grp_lane<K>(v);
    if constexpr (K + 1 < kTinyLanes) grp_all<K + 1>(v, out);
}

// Tiny items (at most 8 keys, 8 iterated descriptors and 64 positions): one
// group of 8 lanes per item, 8 items per wave and step, no tables.  Lane k of
// a group loads key k of the anchor's out-list and descriptor k (start and
// length of a streamed list); the group shares them through lane swizzles, and
// then each lane takes one position per round, finds its list among the 8 by
// comparing with the lists' ends, reads the streamed entry and compares it
// with the 8 keys.  Wave-per-item work costs some 180 instructions per item,
// mostly its LDS table and staging; here a round of 8 items costs about as
// much as one.
template <bool UNION>
__global__ void __launch_bounds__(256) k_light_tiny(const int2* __restrict__ items,
                                                     const int32_t* __restrict__ n_items_dev,
                                                     const int32_t* __restrict__ rpO, const int32_t* __restrict__ colO,
                                                     const int32_t* __restrict__ rpD,
                                                     const unsigned long long* __restrict__ cw,
                                                     const int2* __restrict__ packU, const int2* __restrict__ packD,
                                                     const int32_t* __restrict__ comp, int64_t* __restrict__ acc) {
    constexpr int G = kTinyLanes;
    static_assert(G == 8 && kTinyKeys <= G, "one key and one descriptor per lane of a group");
    const int lane = __lane_id();
    const int pos = lane & (G - 1);
    const int64_t gw = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int64_t n_items = n_items_dev[0];
    int64_t total = 0;
    for (int64_t it0 = gw * (64 / G); it0 < n_items; it0 += nw * (64 / G)) {
        const int64_t it = it0 + lane / G;
        const bool has = it < n_items;
        // the item: anchor x, its keys N+(x) and the iterated descriptors
        const int2 item = has ? items[it] : make_int2(0, 0);
        const bool kind_u = item.x >= 0;
        const int32_t x = kind_u ? item.x : ~item.x;
        const int32_t rs = has ? rpO[x] : 0;
        const int32_t d = has ? rpO[x + 1] - rs : 0;
        int32_t llen = d;
        const int2* L = packU + rs;
        if (has && !kind_u) {
            const int32_t ds = rpD[x];
            L = packD + ds;
            llen = cw_end(cw[x]) - ds;
        }
        const int32_t key = pos < d ? colO[rs + pos] : -1;
        const int2 e = pos < llen ? L[pos] : make_int2(0, 0);
        const int32_t ln = e.y > 0 ? e.y : 0;  // 0: the pair is closed from the other side
        int32_t kk[G], lk[G], sk[G];
        grp_all(key, kk);
        grp_all(ln, lk);
        grp_all(e.x, sk);
        int32_t ek[G];  // end of list k among the item's positions
        int32_t run = 0;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            run += lk[k];
            ek[k] = run;
        }
        const int32_t W = has ? run : 0;
        int32_t cnt = 0;
        for (int32_t c0 = 0; ballot64(c0 < W); c0 += G) {
            const int32_t g = c0 + pos;
            const bool on = g < W;
            // the first list whose end lies past g (empty lists end where the one before does)
            int32_t at = 0;
            bool found = false;
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const bool here = !found && ek[k] > g;
                at = here ? sk[k] + (g - (ek[k] - lk[k])) : at;
                found = found || here;
            }
            const int32_t v = on ? colO[at] : -1;
            bool hit = false;
#pragma unroll
            for (int k = 0; k < G; ++k) hit = hit || (v == kk[k]);
            cnt += on && hit ? 1 : 0;
        }
        if (UNION) {
            cnt += grp_xor<1>(cnt);
            cnt += grp_xor<2>(cnt);
            cnt += grp_xor<4>(cnt);
            if (pos == 0 && has && cnt)
                atomicAdd((unsigned long long*)&acc[(int64_t)comp[x] * kCountSlots + kTL], (unsigned long long)cnt);
        } else {
            total += cnt;
        }
    }
    if (!UNION) {
        total = wave_sum(total);
        if (lane == 0 && total) atomicAdd((unsigned long long*)&acc[kTL], (unsigned long long)total);
    }
}

template <bool GLOBAL, bool UNION>
__global__ void __launch_bounds__(256) k_light_large(const int2* __restrict__ items,
                                                      const int32_t* __restrict__ n_items_dev,
                                                      const int32_t* __restrict__ rpO, const int32_t* __restrict__ colO,
                                                      const int32_t* __restrict__ rpD,
                                                      const unsigned long long* __restrict__ cw,
                                                      const int2* __restrict__ packU, const int2* __restrict__ packD,
                                                      int32_t dcap, int32_t* __restrict__ gscratch, uint32_t sent,
                                                      const int32_t* __restrict__ comp, int64_t* __restrict__ acc) {
    extern __shared__ __attribute__((aligned(16))) int32_t dyn[];
    __shared__ int32_t red[5];
    // layout: hash table (4 x 2^lg <= 4 dcap slots), P (kJL + 1), D (kJL), flags (4 x 64 kU bytes)
    const int64_t per_block = large_block_words(dcap);
    const int lgcap = __builtin_ctz((uint32_t)dcap);  // dcap: a power of two, the table region's buckets
    int32_t* base = GLOBAL ? gscratch + (int64_t)blockIdx.x * per_block : dyn;
    int32_t* tab = base;
    int32_t* P = base + 4 * dcap;
    int32_t* D = P + kJL + 1;
    const int t = threadIdx.x;
    const int w = t >> 6;
    const int lane = __lane_id();
    uint8_t* mark = reinterpret_cast<uint8_t*>(D + kJL) + 64 * kU * w;  // 64 kU bytes per wave
    for (int i = lane; i < 16 * kU; i += 64) reinterpret_cast<int32_t*>(mark)[i] = 0;  // flags stay zero between super-strips
    const int64_t n_items = n_items_dev[0];
    int64_t total = 0;
    int32_t cur = 0;  // component of the closures in total
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = items[it];
        const bool kind_u = item.x >= 0;
        const int32_t x = kind_u ? item.x : ~item.x;
        if (UNION) {
            const int32_t c = comp[x];  // block-uniform
            if (c != cur) {
                flush_tl(acc, cur, total, lane);
                total = 0;
                cur = c;
            }
        }
        const int32_t rs = rpO[x];
        const int32_t d = rpO[x + 1] - rs;
        const int2* L;
        int32_t llen;
        if (kind_u) { L = packU + rs; llen = d; }
        else { const int32_t ds = rpD[x]; L = packD + ds; llen = cw_end(cw[x]) - ds; }
        const int32_t j0 = item.y * kJL;
        const int32_t cnt = min(kJL, llen - j0);
        const int lg = table_bits(d, lgcap);
        const int hs = 4 << lg;
        for (int i = t; i < hs / 4; i += 256) reinterpret_cast<int4*>(tab)[i] = make_int4(-1, -1, -1, -1);
        if (t == 0) P[0] = 0;
        __syncthreads();
        build_hash<256>(rs, d, colO, tab, lg, t);
        int32_t W;
        const int32_t nl = stage_lists<256>(L + j0, cnt, P, D, red, t, &W);
        __syncthreads();
        const int32_t q = (W + 3) / 4;
        const int32_t a = min(w * q, W);
        const int32_t b = min(a + q, W);
        total += close_flat<kU, GLOBAL, false>(P, D, nl, a, b, colO, sent, tab, lg, mark, lane);  // wave-uniform
        __syncthreads();
    }
    flush_tl(acc, cur, total, lane);
}

// ---------------------------------------------------------------------------
// heavy block
// ---------------------------------------------------------------------------

// rank of each heavy vertex in (deg, id) order, by counting smaller keys: tile
// (bx, by) compares heavy vertices bx*256.. with the `chunk` keys by*chunk..
// (a multiple of 256) and adds its counts into rank[] (zeroed beforehand)

// In a union of components (comp != nullptr) the order is (component, deg,
// id): each component's heavy vertices take a contiguous range of ranks, in
// their own (deg, id) order, so U is block diagonal.
__global__ void __launch_bounds__(256) k_heavy_rank(const int32_t* __restrict__ hlist, const int32_t* __restrict__ h_dev,
                                                     int32_t hmax, int32_t chunk, const int32_t* __restrict__ degp,
                                                     const int32_t* __restrict__ comp, int32_t* __restrict__ rank) {
    __shared__ uint64_t kk[256];  // rank keys (deg, id) of the staged heavy vertices
    __shared__ int32_t kc[256];   // and their components (unions)
    const int32_t h = heavy_count(h_dev, hmax);
    // tiles (256 heavy vertices) x (chunk keys), taken with a static
    // stride by a persistent grid sized for the device's h
    const int64_t tx = (h + 255) / 256, ty = (h + chunk - 1) / chunk;
    for (int64_t tile = blockIdx.x; tile < tx * ty; tile += gridDim.x) {  // block-uniform
        const int64_t i = (tile % tx) * 256 + threadIdx.x;
        const int64_t j0 = (tile / tx) * chunk;
        int32_t cx = 0;
        uint64_t key = 0;
        if (i < h) {
            const int32_t x = hlist[i];
            key = rank_key(degp[x], x);
            cx = comp ? comp[x] : 0;
        }
        const int64_t j1 = min((int64_t)h, j0 + chunk);
        int32_t r = 0;
        for (int64_t jb = j0; jb < j1; jb += 256) {
            const int64_t j = jb + threadIdx.x;
            if (j < j1) {
                const int32_t y = hlist[j];
                kk[threadIdx.x] = rank_key(degp[y], y);
                if (comp) kc[threadIdx.x] = comp[y];
            }
            __syncthreads();
            const int lim = (int)min((int64_t)256, j1 - jb);
            if (i < h) {
                if (!comp) {
                    for (int q = 0; q < lim; ++q) r += kk[q] < key ? 1 : 0;
                } else {
                    for (int q = 0; q < lim; ++q) r += (kc[q] < cx || (kc[q] == cx && kk[q] < key)) ? 1 : 0;
                }
            }
            __syncthreads();
        }
        if (i < h && r) atomicAdd(&rank[i], r);
    }
}

__global__ void k_heavy_place(const int32_t* __restrict__ hlist, const int32_t* __restrict__ h_dev, int32_t hmax,
                              const int32_t* __restrict__ rank, int32_t* __restrict__ hidx,
                              int32_t* __restrict__ horder) {
    const int32_t h = heavy_count(h_dev, hmax);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < h; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = hlist[i];
        hidx[x] = rank[i];
        horder[rank[i]] = x;
    }
}

// hs[k] = heavy vertices before component k (the heavy flags' prefix at its start)
__global__ void k_heavy_starts(int32_t K, const int32_t* __restrict__ off, const int32_t* __restrict__ hpos,
                               int32_t* __restrict__ hs) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k <= K; k += gridDim.x * blockDim.x) hs[k] = hpos[off[k]];
}

// U[i][j] = 1 and UT[j][i] = 1 for every oriented edge between heavy ranks i < j
// Rows of U: row i holds 1 at the ranks j > i of the heavy out-neighbours of
// the vertex of rank i (its N+ list: every vertex above a heavy one is heavy),
// rows h..hp-1 are zero.  Persistent blocks take rows with a static stride;
// a row is built in LDS 16 KB of columns at a time and written whole, so U
// needs no separate clearing.
constexpr int kRowChunk = 16384;
__global__ void __launch_bounds__(256) k_heavy_rows(const int32_t* __restrict__ horder,
                                                     const int32_t* __restrict__ h_dev, int32_t hmax,
                                                     const int32_t* __restrict__ rpO, const int32_t* __restrict__ colO,
                                                     const int32_t* __restrict__ hidx, uint8_t* __restrict__ U) {
    __shared__ __attribute__((aligned(16))) uint8_t row[kRowChunk];
    const int32_t h = heavy_count(h_dev, hmax);
    const int64_t hp = heavy_pad(h);
    for (int64_t i = blockIdx.x; i < hp; i += gridDim.x) {
        const int32_t b = i < h ? rpO[horder[i]] : 0;
        const int32_t e = i < h ? rpO[horder[i] + 1] : 0;
        for (int64_t c0 = 0; c0 < hp; c0 += kRowChunk) {
            const int32_t w = (int32_t)min<int64_t>(kRowChunk, hp - c0);  // a multiple of 128
            for (int32_t k = threadIdx.x; k < w / 16; k += 256) reinterpret_cast<int4*>(row)[k] = make_int4(0, 0, 0, 0);
            __syncthreads();
            for (int32_t q = b + threadIdx.x; q < e; q += 256) {
                const int64_t j = hidx[colO[q]] - c0;
                if (j >= 0 && j < w) row[j] = 1;
            }
            __syncthreads();
            int4* out = reinterpret_cast<int4*>(U + i * hp + c0);
            for (int32_t k = threadIdx.x; k < w / 16; k += 256) out[k] = reinterpret_cast<const int4*>(row)[k];
            __syncthreads();
        }
    }
}

// UT = U transposed, by 64 x 64 byte tiles through LDS (hp is a multiple of
// 128, so the tiles cover both matrices exactly).
__global__ void __launch_bounds__(256) k_heavy_transpose(const int32_t* __restrict__ h_dev, int32_t hmax,
                                                          const uint8_t* __restrict__ U, uint8_t* __restrict__ UT) {
    __shared__ uint8_t tile[64][64 + 4];
    const int64_t hp = heavy_pad(heavy_count(h_dev, hmax));
    const int64_t T = hp / 64;
    const int t = threadIdx.x;
    const int r = t >> 2, cc = (t & 3) * 16;  // row of the tile and first of 16 columns
    for (int64_t q = blockIdx.x; q < T * T; q += gridDim.x) {
        const int64_t ti = q / T, tj = q % T;
        const int4 v = *reinterpret_cast<const int4*>(U + (ti * 64 + r) * hp + tj * 64 + cc);
        const uint32_t wv[4] = {(uint32_t)v.x, (uint32_t)v.y, (uint32_t)v.z, (uint32_t)v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) tile[r][cc + k] = (uint8_t)(wv[k >> 2] >> (8 * (k & 3)));
        __syncthreads();
        uint32_t o[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 16; ++k) o[k >> 2] |= (uint32_t)tile[cc + k][r] << (8 * (k & 3));
        *reinterpret_cast<int4*>(UT + (tj * 64 + r) * hp + ti * 64 + cc) =
            make_int4((int)o[0], (int)o[1], (int)o[2], (int)o[3]);
        __syncthreads();
    }
}

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef int32_t v16i __attribute__((ext_vector_type(16)));

constexpr int kHK = 128;         // k-bytes staged per step
constexpr int kHRow = kHK + 16;  // LDS row stride: 16-lane groups of 16-byte reads hit 64 distinct banks

// T_H = sum over i < j of (U U)[i][j] U[i][j] with U the strictly upper
// triangular adjacency of the heavy vertices in rank order (each heavy
// triangle i < k < j once).  One block per 128 x 128 macro tile (I, J), I <= J,
// of C = U U; because U is strictly upper triangular, only k in
// [128 I, 128 J + 128) can contribute, and the k-loop covers exactly those
// k-blocks.  Per step the block stages 128 rows x 128 k-bytes of U (rows of
// the tile) and of U^T (columns of the tile) in LDS while the next step's
// global loads are in flight in registers; each wave owns a 64 x 64 quarter as
// 2 x 2 tiles of v_mfma_i32_32x32x32_i8.  Operand fragments: lane l supplies
// row (l mod 32) of the A tile and column (l mod 32) of the B tile, 16
// consecutive k-bytes starting at 16 (l / 32); A and B use the same
// k-permutation.  The epilogue masks C with U and adds into T_H.  Macro tiles
// are enumerated column by column (t = J (J + 1) / 2 + I) and dealt to the 8
// XCDs in contiguous ranges of equal work, so blocks of one XCD share the U^T
// panels of their columns in that XCD's L2.
// Masked sum of one 128 x 128 macro tile (I, J), I <= J, of C = U U over the
// k-blocks [128 I, 128 J + 128) (U strictly upper triangular, hp x hp):
// this thread's share.  As / Bs: the block's LDS staging.
__device__ __forceinline__ int64_t mfma_tile(const uint8_t* __restrict__ U, const uint8_t* __restrict__ UT,
                                             int64_t hp, int64_t I, int64_t J, uint8_t* As, uint8_t* Bs) {
    const int t = threadIdx.x;
    const int w = t >> 6;
    const int lane = __lane_id();
    const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
    const int fr = lane & 31, fk = 16 * (lane >> 5);
    const int lr = t >> 1, lc = (t & 1) * (kHK / 2);  // staging: row and byte offset of this thread
    const int64_t row0 = I * kHT, col0 = J * kHT;
    const uint8_t* ga = U + (row0 + lr) * hp + lc;
    const uint8_t* gb = UT + (col0 + lr) * hp + lc;
    v16i c[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) c[i][j] = (v16i){0};
    const int64_t kend = col0 + kHT;
    v4i ra[4], rb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        ra[q] = *(const v4i*)(ga + row0 + 16 * q);
        rb[q] = *(const v4i*)(gb + row0 + 16 * q);
    }
    for (int64_t k0 = row0; k0 < kend; k0 += kHK) {
        __syncthreads();  // the previous step's fragment reads are done
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            *(v4i*)(As + lr * kHRow + lc + 16 * q) = ra[q];
            *(v4i*)(Bs + lr * kHRow + lc + 16 * q) = rb[q];
        }
        __syncthreads();
        if (k0 + kHK < kend) {  // block-uniform: the next step's loads fly during these MFMAs
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ra[q] = *(const v4i*)(ga + k0 + kHK + 16 * q);
                rb[q] = *(const v4i*)(gb + k0 + kHK + 16 * q);
            }
        }
#pragma unroll
        for (int ks = 0; ks < kHK; ks += 32) {
            v4i af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = *(const v4i*)(As + (wr + 32 * i + fr) * kHRow + ks + fk);
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = *(const v4i*)(Bs + (wc + 32 * j + fr) * kHRow + ks + fk);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    c[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[i], bf[j], c[i][j], 0, 0, 0);
        }
    }
    int64_t total = 0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint8_t* ucol = U + col0 + wc + 32 * j + fr;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int64_t row = row0 + wr + 32 * i + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                total += (int64_t)c[i][j][q] * (int64_t)ucol[row * hp];
            }
        }
    return total;
}

// T_H = sum over i < j of (U U)[i][j] U[i][j] with U the strictly upper
// triangular adjacency of the heavy vertices in rank order (each heavy
// triangle i < k < j once).  One block per 128 x 128 macro tile (I, J), I <= J,
// of C = U U; because U is strictly upper triangular, only k in
// [128 I, 128 J + 128) can contribute, and the k-loop covers exactly those
// k-blocks.  Per step the block stages 128 rows x 128 k-bytes of U (rows of
// the tile) and of U^T (columns of the tile) in LDS while the next step's
// global loads are in flight in registers; each wave owns a 64 x 64 quarter as
// 2 x 2 tiles of v_mfma_i32_32x32x32_i8.  Operand fragments: lane l supplies
// row (l mod 32) of the A tile and column (l mod 32) of the B tile, 16
// consecutive k-bytes starting at 16 (l / 32); A and B use the same
// k-permutation.  The epilogue masks C with U and adds into T_H.  Macro tiles
// are enumerated column by column (t = J (J + 1) / 2 + I) and dealt to the 8
// XCDs in contiguous ranges of equal work, so blocks of one XCD share the U^T
// panels of their columns in that XCD's L2.
// Work of the macro tiles before tile t in column-major order (t = J (J + 1) /
// 2 + I): tile (I, J) takes J - I + 1 k-steps, so the columns before J take
// J (J + 1) (J + 2) / 6 and the tiles (0..I-1, J) I (J + 1) - I (I - 1) / 2.
// Returns the first tile whose preceding work reaches B (0 <= B <= the total
// work of nm columns); nm columns hold nm (nm + 1) / 2 tiles.
__device__ __forceinline__ int64_t tile_at_work(int64_t B, int64_t nm) {
    auto cols = [](int64_t J) { return J * (J + 1) * (J + 2) / 6; };
    int64_t J = (int64_t)cbrt(6.0 * (double)B);
    if (J > nm) J = nm;
    while (J > 0 && cols(J) > B) --J;
    while (J < nm && cols(J + 1) <= B) ++J;
    if (J >= nm) return nm * (nm + 1) / 2;
    const int64_t r = B - cols(J);  // work still to pass inside column J (< its J (J + 1) / 2 + J + 1)
    int64_t I = 0, w = 0;
    while (I <= J && w < r) { w += J - I + 1; ++I; }
    return J * (J + 1) / 2 + I;  // I = J + 1 is the next column's first tile
}

__global__ void __launch_bounds__(256) k_heavy_mfma(const uint8_t* __restrict__ U, const uint8_t* __restrict__ UT,
                                                     const int32_t* __restrict__ h_dev, int32_t hmax,
                                                     int64_t* __restrict__ acc) {
    __shared__ __attribute__((aligned(16))) uint8_t As[kHT * kHRow];
    __shared__ __attribute__((aligned(16))) uint8_t Bs[kHT * kHRow];
    const int32_t h = heavy_count(h_dev, hmax);
    if (h < 3) return;  // block-uniform
    const int64_t hp = heavy_pad(h);
    const int64_t nm = hp / kHT;
    const int64_t ntiles = nm * (nm + 1) / 2;
    const int lane = __lane_id();
    const int64_t xcd = blockIdx.x & 7;
    const int64_t per_xcd = gridDim.x >> 3;
    // each XCD takes a contiguous range of equal work (the later columns
    // hold longer tiles: an equal count of tiles gave the last XCD 1.5 times
    // its share)
    const int64_t work = nm * (nm + 1) * (nm + 2) / 6;
    const int64_t t_begin = tile_at_work(xcd * work / 8, nm);
    const int64_t t_end = xcd == 7 ? ntiles : tile_at_work((xcd + 1) * work / 8, nm);
    int64_t total = 0;
    for (int64_t tt = t_begin + (blockIdx.x >> 3); tt < t_end; tt += per_xcd) {
        int64_t J = (int64_t)((sqrt(8.0 * (double)tt + 1.0) - 1.0) * 0.5);
        while (J * (J + 1) / 2 > tt) --J;
        while ((J + 1) * (J + 2) / 2 <= tt) ++J;
        const int64_t I = tt - J * (J + 1) / 2;
        total += mfma_tile(U, UT, hp, I, J, As, Bs);
    }
    total = wave_sum(total);
    if (lane == 0 && total) atomicAdd((unsigned long long*)&acc[kTH], (unsigned long long)total);
}

// ---- heavy blocks of a union of components --------------------------------
// Component c's heavy vertices hold ranks [hs[c], hs[c+1]) and get their own
// strictly upper-triangular block U_c of pc[c] x pc[c] bytes (pc = the count
// rounded up to 128) at byte offset boff[c] of U (and of UT).  Row slot q of
// the rows of all blocks belongs to component c with prow[c] <= q < prow[c+1].

__device__ __forceinline__ int32_t comp_of_slot(const int64_t* __restrict__ pre, int32_t K, int64_t q) {
    int32_t lo = 0, hi = K - 1;  // largest c with pre[c] <= q
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) k_heavy_rows_u(int32_t K, const int32_t* __restrict__ hs,
                                                       const int32_t* __restrict__ pc,
                                                       const int64_t* __restrict__ prow,
                                                       const int64_t* __restrict__ boff,
                                                       const int32_t* __restrict__ horder,
                                                       const int32_t* __restrict__ rpO, const int32_t* __restrict__ colO,
                                                       const int32_t* __restrict__ hidx, uint8_t* __restrict__ U) {
    __shared__ __attribute__((aligned(16))) uint8_t row[kRowChunk];
    const int64_t R = prow[K];
    for (int64_t q = blockIdx.x; q < R; q += gridDim.x) {  // block-uniform
        const int32_t c = comp_of_slot(prow, K, q);
        const int64_t i = q - prow[c];
        const int32_t h = hs[c + 1] - hs[c];
        const int64_t p = pc[c];
        const int32_t x = i < h ? horder[hs[c] + i] : 0;
        const int32_t b = i < h ? rpO[x] : 0;
        const int32_t e = i < h ? rpO[x + 1] : 0;
        uint8_t* Uc = U + boff[c];
        for (int64_t c0 = 0; c0 < p; c0 += kRowChunk) {
            const int32_t w = (int32_t)min<int64_t>(kRowChunk, p - c0);  // a multiple of 128
            for (int32_t k = threadIdx.x; k < w / 16; k += 256) reinterpret_cast<int4*>(row)[k] = make_int4(0, 0, 0, 0);
            __syncthreads();
            for (int32_t t = b + threadIdx.x; t < e; t += 256) {
                const int64_t j = (int64_t)(hidx[colO[t]] - hs[c]) - c0;
                if (j >= 0 && j < w) row[j] = 1;
            }
            __syncthreads();
            int4* out = reinterpret_cast<int4*>(Uc + i * p + c0);
            for (int32_t k = threadIdx.x; k < w / 16; k += 256) out[k] = reinterpret_cast<const int4*>(row)[k];
            __syncthreads();
        }
    }
}

// UT_c = U_c transposed, by 64 x 64 byte tiles; tile slot q of all blocks
// belongs to component c with ptt[c] <= q < ptt[c+1] ((pc/64)^2 per block).
__global__ void __launch_bounds__(256) k_heavy_transpose_u(int32_t K, const int32_t* __restrict__ pc,
                                                            const int64_t* __restrict__ ptt,
                                                            const int64_t* __restrict__ boff,
                                                            const uint8_t* __restrict__ U, uint8_t* __restrict__ UT) {
    __shared__ uint8_t tile[64][64 + 4];
    const int t = threadIdx.x;
    const int r = t >> 2, cc = (t & 3) * 16;
    const int64_t Q = ptt[K];
    for (int64_t q = blockIdx.x; q < Q; q += gridDim.x) {
        const int32_t c = comp_of_slot(ptt, K, q);
        const int64_t hp = pc[c];
        const int64_t T = hp / 64;
        const int64_t l = q - ptt[c];
        const int64_t ti = l / T, tj = l % T;
        const uint8_t* Uc = U + boff[c];
        uint8_t* UTc = UT + boff[c];
        const int4 v = *reinterpret_cast<const int4*>(Uc + (ti * 64 + r) * hp + tj * 64 + cc);
        const uint32_t wv[4] = {(uint32_t)v.x, (uint32_t)v.y, (uint32_t)v.z, (uint32_t)v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) tile[r][cc + k] = (uint8_t)(wv[k >> 2] >> (8 * (k & 3)));
        __syncthreads();
        uint32_t o[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 16; ++k) o[k >> 2] |= (uint32_t)tile[cc + k][r] << (8 * (k & 3));
        *reinterpret_cast<int4*>(UTc + (tj * 64 + r) * hp + ti * 64 + cc) =
            make_int4((int)o[0], (int)o[1], (int)o[2], (int)o[3]);
        __syncthreads();
    }
}

// T_H of every component: the macro tiles (c, I, J) of the blocks with at
// least three heavy vertices, from a tile list; each tile adds into its
// component's T_H.
__global__ void __launch_bounds__(256) k_heavy_mfma_u(int32_t ntiles, const int4* __restrict__ tiles,
                                                       const int32_t* __restrict__ pc,
                                                       const int64_t* __restrict__ boff,
                                                       const uint8_t* __restrict__ U, const uint8_t* __restrict__ UT,
                                                       int64_t* __restrict__ acc) {
    __shared__ __attribute__((aligned(16))) uint8_t As[kHT * kHRow];
    __shared__ __attribute__((aligned(16))) uint8_t Bs[kHT * kHRow];
    const int lane = __lane_id();
    int64_t total = 0;
    int32_t cur = -1;
    for (int32_t q = blockIdx.x; q < ntiles; q += gridDim.x) {
        const int4 tl = tiles[q];  // (component, I, J)
        if (tl.x != cur) {
            const int64_t tsum = wave_sum(total);
            if (cur >= 0 && lane == 0 && tsum)
                atomicAdd((unsigned long long*)&acc[(int64_t)cur * kCountSlots + kTH], (unsigned long long)tsum);
            total = 0;
            cur = tl.x;
        }
        total += mfma_tile(U + boff[tl.x], UT + boff[tl.x], pc[tl.x], tl.y, tl.z, As, Bs);
    }
    const int64_t tsum = wave_sum(total);
    if (cur >= 0 && lane == 0 && tsum)
        atomicAdd((unsigned long long*)&acc[(int64_t)cur * kCountSlots + kTH], (unsigned long long)tsum);
}

}  // namespace

// Heavy-vertex bound: heavy vertices have deg > c m'^(1/2) with c = a/b and the
// degrees sum to 2m', so h < 2 m'^(1/2) / c <= 2 b m^(1/2) / a (all n if a = 0).
static int64_t heavy_bound(int64_t n, int64_t m, int32_t a, int32_t b) {
    if (a == 0) return n;
    const double hb = 2.0 * (double)b * std::sqrt((double)m) / (double)a + 2.0;
    return hb < (double)n ? (int64_t)hb : n;
}

// Which block-per-item bins a count launches, and the table capacity of each
// (0: not launched).  maxd bounds the out-degree of every anchor.
struct LightPlan {
    int32_t dcap_lds = 0;     // anchors with small_dmax < d+ <= kLdsDcap: table in LDS
    int32_t dcap_global = 0;  // anchors with d+ > kLdsDcap: table in global scratch
};

static LightPlan light_plan(int64_t m, int32_t maxd, const CountConfig& cfg) {
    LightPlan pl;
    if (maxd > cfg.small_dmax) {
        int32_t dcap = 64;
        while (dcap < std::min<int32_t>(maxd, kLdsDcap)) dcap <<= 1;
        pl.dcap_lds = dcap;
    }
    if (maxd > kLdsDcap) {
        // anchors of this bin: light sources (d+ <= deg <= c m'^(1/2) <= c m^(1/2)) or
        // v-side anchors (d+ <= vmajor_cap)
        const double light_cap = cfg.heavy_num == 0 ? 0.0
                                 : (double)cfg.heavy_num * std::sqrt((double)m) / (double)cfg.heavy_den + 1.0;
        int64_t dbound = std::max<int64_t>((int64_t)cfg.vmajor_cap, (int64_t)std::min(light_cap, (double)maxd));
        dbound = std::min<int64_t>(dbound, maxd);
        int32_t dcap = 64;
        while (dcap < dbound) dcap <<= 1;
        if (dbound > kLdsDcap) pl.dcap_global = dcap;
    }
    return pl;
}

// Keys per rank tile for h heavy vertices: the largest of 1024, 512 and 256
// that still gives every CU a tile (longer chunks take fewer rank atomics,
// shorter ones more tiles when h is small).
static int32_t rank_chunk(int64_t h) {
    for (int32_t c = 1024; c > 256; c /= 2)
        if ((int64_t)ceil_div(h, 256) * (int64_t)ceil_div(h, c) >= num_cus()) return c;
    return 256;
}

// Blocks of 256 threads of `kernel` that stay resident on one CU with
// `lds_bytes` of dynamic LDS (at least 1).  Persistent launches take at most
// this many per CU, queried for the very variant they launch: the variants
// of one kernel need not compile to the same register count.
template <typename K>
static int resident_blocks(K kernel, size_t lds_bytes) {
    int r = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, kernel, 256, lds_bytes) != hipSuccess || r < 1) r = 1;
    (void)hipGetLastError();
    return r;
}

// Heavy phase of a union of components: the heavy counts at the component
// starts are read back (one synchronisation), and each component with at
// least three heavy vertices gets its own block, ranked (component, deg, id).
static void count_union_heavy(const tc_graph_s* g, const CountUnion& un, const CountConfig& cfg, hipStream_t s,
                              int64_t* acc, const DevBuf<int32_t>& heavy, const DevBuf<int32_t>& hpos,
                              const int32_t* degp, const DevBuf<int32_t>& rpO, const DevBuf<int32_t>& colO) {
    (void)cfg;
    const int64_t n = g->n;
    const int32_t K = un.K;
    DevBuf<int32_t> hsd((size_t)K + 1, s);
    TC_LAUNCH("heavy_starts", k_heavy_starts, dim3(ceil_div((int64_t)K + 1, 256)), dim3(256), 0, s, K, un.off,
              (const int32_t*)hpos.get(), hsd.get());
    std::vector<int32_t> hs((size_t)K + 1);
    check_hip(hipMemcpyAsync(hs.data(), hsd.get(), sizeof(int32_t) * hs.size(), hipMemcpyDeviceToHost, s), "heavy starts");
    check_hip(hipStreamSynchronize(s), "sync");
    const int64_t H = hs[(size_t)K];
    std::vector<int32_t> pc((size_t)K);
    std::vector<int64_t> prow((size_t)K + 1, 0), ptt((size_t)K + 1, 0), boff((size_t)K, 0);
    std::vector<int4> tiles;
    int64_t ubytes = 0;
    for (int32_t k = 0; k < K; ++k) {
        const int64_t h = hs[(size_t)k + 1] - hs[(size_t)k];
        const int64_t p = h >= 3 ? heavy_pad(h) : 0;  // blocks of fewer than 3 vertices hold no triangle
        pc[(size_t)k] = (int32_t)p;
        boff[(size_t)k] = ubytes;
        ubytes += p * p;
        prow[(size_t)k + 1] = prow[(size_t)k] + p;
        ptt[(size_t)k + 1] = ptt[(size_t)k] + (p / 64) * (p / 64);
        for (int32_t J = 0; J < p / kHT; ++J)
            for (int32_t I = 0; I <= J; ++I) tiles.push_back(make_int4(k, I, J, 0));
    }
    if (tiles.empty()) return;
    if (ubytes > ((int64_t)16 << 30)) fail(TC_ERR_OVERFLOW, "heavy blocks of the union exceed 16 GiB: raise the heavy threshold");
    if (tiles.size() > (size_t)0x7fffffff) fail(TC_ERR_OVERFLOW, "too many heavy tiles");
    PhaseScope ph("heavy");
    DevBuf<int32_t> pcd(K, s);
    DevBuf<int64_t> prowd((size_t)K + 1, s), pttd((size_t)K + 1, s), boffd(K, s);
    DevBuf<int4> tilesd(tiles.size(), s);
    check_hip(hipMemcpyAsync(pcd.get(), pc.data(), sizeof(int32_t) * pc.size(), hipMemcpyHostToDevice, s), "pc");
    check_hip(hipMemcpyAsync(prowd.get(), prow.data(), sizeof(int64_t) * prow.size(), hipMemcpyHostToDevice, s), "prow");
    check_hip(hipMemcpyAsync(pttd.get(), ptt.data(), sizeof(int64_t) * ptt.size(), hipMemcpyHostToDevice, s), "ptt");
    check_hip(hipMemcpyAsync(boffd.get(), boff.data(), sizeof(int64_t) * boff.size(), hipMemcpyHostToDevice, s), "boff");
    check_hip(hipMemcpyAsync(tilesd.get(), tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, s),
              "tiles");
    DevBuf<int32_t> hlist(H, s), hidx(n, s), horder(H, s), hrank(H, s);
    const int32_t hm = (int32_t)H;
    const int32_t* h_dev = hpos.get() + n;
    TC_LAUNCH("heavy_list", k_heavy_list, dim3(grid_for(n, 256)), dim3(256), 0, s, n, (const int32_t*)heavy.get(),
              (const int32_t*)hpos.get(), hm, hlist.get(), acc);
    fill_i32(hrank.get(), 0, H, s);
    const int32_t chunk = rank_chunk(H);
    TC_LAUNCH("heavy_rank", k_heavy_rank, dim3((unsigned)std::min<int64_t>(
                                              (int64_t)ceil_div(H, 256) * (int64_t)ceil_div(H, chunk),
                                              (int64_t)num_cus() * 4)),
              dim3(256), 0, s, (const int32_t*)hlist.get(), h_dev, hm, chunk, degp, un.comp, hrank.get());
    TC_LAUNCH("heavy_place", k_heavy_place, dim3(ceil_div(H, 256)), dim3(256), 0, s, (const int32_t*)hlist.get(),
              h_dev, hm, (const int32_t*)hrank.get(), hidx.get(), horder.get());
    DevBuf<uint8_t> U((size_t)ubytes, s), UT((size_t)ubytes, s);
    TC_LAUNCH("heavy_pack", k_heavy_rows_u, dim3((unsigned)std::min<int64_t>(prow[(size_t)K], (int64_t)num_cus() * 8)),
              dim3(256), 0, s, K, (const int32_t*)hsd.get(), (const int32_t*)pcd.get(), (const int64_t*)prowd.get(),
              (const int64_t*)boffd.get(), (const int32_t*)horder.get(), (const int32_t*)rpO.get(),
              (const int32_t*)colO.get(), (const int32_t*)hidx.get(), U.get());
    TC_LAUNCH("heavy_transpose", k_heavy_transpose_u,
              dim3((unsigned)std::min<int64_t>(ptt[(size_t)K], (int64_t)num_cus() * 8)), dim3(256), 0, s, K,
              (const int32_t*)pcd.get(), (const int64_t*)pttd.get(), (const int64_t*)boffd.get(),
              (const uint8_t*)U.get(), UT.get());
    TC_LAUNCH("heavy_mfma", k_heavy_mfma_u,
              dim3((unsigned)std::min<int64_t>((int64_t)tiles.size(), (int64_t)num_cus() * 8)), dim3(256), 0, s,
              (int32_t)tiles.size(), (const int4*)tilesd.get(), (const int32_t*)pcd.get(), (const int64_t*)boffd.get(),
              (const uint8_t*)U.get(), (const uint8_t*)UT.get(), acc);
}

// The count of g (un == nullptr), or of every component of the union graph g
// (un != nullptr; g unsampled): see count_enqueue and count_union.
static void count_impl(const tc_graph_s* g, int sampled, uint64_t thr, uint64_t salt, const CountConfig& cfg,
                       hipStream_t s, int64_t* acc, const CountUnion* un) {
    const int64_t n = g->n;
    const int64_t E2 = 2 * g->m;
    if (cfg.small_dmax > 128 || cfg.small_dmax < 1) fail(TC_ERR_INVALID, "small_dmax must be in [1, 128]");
    const int32_t K = un ? un->K : 1;
    const int32_t* comp = un ? un->comp : nullptr;
    fill_i64(acc, 0, (int64_t)K * kCountSlots, s);
    if (n == 0 || E2 == 0) {
        if (un && K > 0 && n > 0) {  // m' = 0 and h = 0 for every component
            DevBuf<int32_t> zero(n + 1, s);
            fill_i32(zero.get(), 0, n + 1, s);
            TC_LAUNCH("finish_union", k_finish_union, dim3(ceil_div(K, 256)), dim3(256), 0, s, K, un->off, un->mk,
                      (const int32_t*)zero.get(), acc);
        }
        return;
    }
    const int64_t NW = (E2 + 63) / 64;

    // host-side bounds for every launch (no read-back inside a count; a union
    // reads its heavy count back before the heavy phase instead)
    int64_t hmax = heavy_bound(n, g->m, cfg.heavy_num, cfg.heavy_den);
    int64_t hp_max = heavy_pad(hmax);
    if (!un && hp_max * hp_max > ((int64_t)16 << 30))
        fail(TC_ERR_OVERFLOW, "heavy block bound exceeds 16 GiB: raise the heavy threshold");
    const int64_t items_max = 2 * n + E2 / kJL + 2;

    // 1. the counted graph: the input CSR, or its sample compacted into buffers
    //    sized for the full graph (section 3.1 coin), so that every later pass
    //    touches m' entries instead of m
    const int32_t* v_row = g->row_ptr;
    const int32_t* v_col = g->col;
    const int32_t* v_src = g->src;
    const int32_t* degp = g->deg;
    const int32_t* E2_dev = nullptr;
    DevBuf<uint64_t> keep;
    DevBuf<int32_t> kpre, rps, degs, cols, srcs;
    if (sampled) {
        PhaseScope ph("sample");
        keep.reset(NW, s);
        kpre.reset(NW + 1, s);
        rps.reset(n + 1, s);
        degs.reset(n, s);
        cols.reset(E2, s);
        srcs.reset(E2, s);
        {
            // staging freed before any later allocation (last in, first out)
            DevBuf<int32_t> st_col(E2, s), st_src(E2, s);
            sample_keep_staged(g, salt, thr, keep.get(), kpre.get(), st_col.get(), st_src.get(), s);
            scan_exclusive_i32(kpre.get(), kpre.get(), NW, s);
            positions_at_rows(g->row_ptr, n, E2, keep.get(), kpre.get(), rps.get(), degs.get(), s);
            move_staged(E2, kpre.get(), st_col.get(), st_src.get(), cols.get(), srcs.get(), s);
        }
        v_row = rps.get();
        v_col = cols.get();
        v_src = srcs.get();
        degp = degs.get();
        E2_dev = kpre.get() + NW;  // 2 m'
    }

    // 2. orientation by (deg, id): compacted up lists N+(x), in CSR order
    PhaseScope ph_orient("orient");
    DevBuf<uint64_t> ubits(NW, s);
    DevBuf<int32_t> upre(NW + 1, s);
    DevBuf<uint8_t> cls(n, s);
    TC_LAUNCH("deg_class", k_deg_class, dim3(grid_for(n, 256)), dim3(256), 0, s, n, degp, cls.get());
    // the counted graph's own neighbour classes when it is the built graph
    const uint8_t* ncls = !sampled && !un ? g->ncls : nullptr;
    TC_LAUNCH("orient_bits", k_orient_bits, dim3(grid_for(NW, 16)), dim3(256), 0, s, v_src, v_col, E2, E2_dev,
              (const uint8_t*)cls.get(), ncls, degp, ubits.get(), upre.get());
    scan_exclusive_i32(upre.get(), upre.get(), NW, s);
    const int32_t* mp_dev = upre.get() + NW;  // number of up entries = m'
    // up-list starts and d+ at every row start, and the per-vertex fields of
    // the light phase (classification of each vertex, its rowQ and v-major
    // slot counter), in one pass
    DevBuf<int32_t> rpO(n + 1, s), dplus(n, s);
    // up lists: m' <= m entries, then the sentinel -2 at index m, which the
    // closure's gathers read for positions past a range
    DevBuf<int32_t> colO(g->m + 1, s);
    const uint32_t sent = (uint32_t)g->m;
    DevBuf<int32_t> heavy(n + 1, s), code(n, s), rpD(n + 1, s);
    DevBuf<int4> rowQ(n, s);
    DevBuf<int64_t> Wu(n, s), cw(n, s);
    DevBuf<int32_t> wide(3 * (n + 1), s);  // vertices with d+ in (128, 256], (256, 512], > 512; counts first
    unsigned long long* cwp = reinterpret_cast<unsigned long long*>(cw.get());
    TC_LAUNCH("vertex_prep", k_vertex_prep, dim3(grid_for(n + 1, 256)), dim3(256), 0, s, n, E2,
              (const uint64_t*)ubits.get(), (const int32_t*)upre.get(), degp, mp_dev, comp,
              un ? un->mk : (const int64_t*)nullptr, cfg.heavy_num, cfg.heavy_den, v_row, rpO.get(), dplus.get(),
              heavy.get(), code.get(), rpD.get(), rowQ.get(), cwp, wide.get(), colO.get() + sent);

    // one descriptor per up entry: the anchor work writes every entry of every
    // light source's list, and only those lists are read
    DevBuf<int2> packU(g->m, s);
    compact_kept(v_col, v_src, E2, ubits.get(), upre.get(), colO.get(), nullptr, s, E2_dev);

    // 3. classification; anchor work (each light source's N+(u) in rank
    //    order, one descriptor per pair); item lists
    const int32_t vcap = cfg.vmajor_cap;
    PhaseScope ph_light("light");
    DevBuf<int64_t> Gx(un ? n : 0, s);  // per-list gather statistic (unions)
    int64_t* gxp = un ? Gx.get() : nullptr;
    DevBuf<int2> packD(vcap > 0 ? g->m : 1, s);  // v-major descriptors, rpD[v].. for vertex v
    TC_LAUNCH("work", k_work_lanes, dim3(grid_for(n, 256)), dim3(256), 0, s, n, (const int4*)rowQ.get(),
              colO.get(), vcap, packU.get(), packD.get(), cwp, Wu.get(), gxp, wide.get(), acc);
    // longer lists by register class, persistent grids of one round of
    // resident blocks; max_deg bounds every d+
    auto launch_wide = [&](auto kernel, int c, int32_t lo, const char* name, std::atomic<int>& resident) {
        if (g->max_deg <= lo) return;
        int r = resident.load(std::memory_order_relaxed);
        if (!r) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, kernel, 256, 0) != hipSuccess || r < 1) r = 1;
            (void)hipGetLastError();
            resident.store(r, std::memory_order_relaxed);
        }
        TC_LAUNCH(name, kernel, dim3((unsigned)(num_cus() * r)), dim3(256), 0, s,
                  (const int32_t*)wide.get() + c * (n + 1) + 1, (const int4*)rowQ.get(), colO.get(), vcap,
                  packU.get(), packD.get(), cwp, Wu.get(), gxp, acc);
    };
    static std::atomic<int> res_w[3];
    launch_wide(k_work_wide<4>, 0, 128, "work_w4", res_w[0]);
    launch_wide(k_work_wide<8>, 1, 256, "work_w8", res_w[1]);
    launch_wide(k_work_wide<16>, 2, 512, "work_w16", res_w[2]);
    DevBuf<int32_t> ntn(n + 1, s), nsm(n + 1, s), nlg(n + 1, s), nhg(n + 1, s);
    const unsigned cgrid = std::min<unsigned>(grid_for(n, 256), kClassifyBlocks);
    DevBuf<int64_t> cpart((size_t)cgrid * 9, s);
    if (!un)
        TC_LAUNCH("classify", k_classify, dim3(cgrid), dim3(256), 0, s, n, (const int32_t*)code.get(),
                  (const int32_t*)dplus.get(), (const int64_t*)Wu.get(), (const unsigned long long*)cwp,
                  (const int32_t*)rpD.get(), cfg.small_dmax, ntn.get(), nsm.get(), nlg.get(), nhg.get(),
                  cpart.get());
    else
        TC_LAUNCH("classify", k_classify_union, dim3(cgrid), dim3(256), 0, s, n, comp, (const int32_t*)code.get(),
                  (const int32_t*)dplus.get(), (const int64_t*)Wu.get(), (const int64_t*)gxp,
                  (const unsigned long long*)cwp, (const int32_t*)rpD.get(), cfg.small_dmax, ntn.get(), nsm.get(),
                  nlg.get(), nhg.get(), acc);
    DevBuf<int32_t> sbase(n + 1, s), lbase(n + 1, s), hbase(n + 1, s), hpos(n + 1, s), tbase(n + 1, s);
    {
        const int32_t* in[4] = {nsm.get(), nlg.get(), nhg.get(), heavy.get()};
        int32_t* out[4] = {sbase.get(), lbase.get(), hbase.get(), hpos.get()};
        scan_exclusive_i32_x4(in, out, n, s);
        scan_exclusive_i32(ntn.get(), tbase.get(), n, s);
    }

    // 4. light phase: three bins by anchor out-degree; each kernel is a
    //    persistent grid that reads its item count from device memory
    const int32_t maxd = g->max_deg;  // bounds every d+ of every sample
    const LightPlan plan = light_plan(g->m, maxd, cfg);
    // the item lists of the launched bins (a bin that is not launched has no items)
    DevBuf<int2> items_t(items_max, s), items_s(items_max, s), items_l(plan.dcap_lds ? items_max : 0, s),
        items_h(plan.dcap_global ? items_max : 0, s);
    TC_LAUNCH("items", k_items, dim3(grid_for(n, 256)), dim3(256), 0, s, n, (const int32_t*)ntn.get(),
              (const int32_t*)nsm.get(), (const int32_t*)nlg.get(), (const int32_t*)nhg.get(),
              (const int32_t*)tbase.get(), (const int32_t*)sbase.get(), (const int32_t*)lbase.get(),
              (const int32_t*)hbase.get(), (const int32_t*)dplus.get(), (const int64_t*)Wu.get(),
              (const unsigned long long*)cwp, (const int32_t*)rpD.get(), items_t.get(), items_s.get(), items_l.get(),
              items_h.get());
    {
        static const int resident[2] = {resident_blocks(k_light_tiny<false>, 0), resident_blocks(k_light_tiny<true>, 0)};
        const int64_t blocks = (int64_t)num_cus() * std::min<int32_t>(cfg.light_blocks_per_cu, resident[un ? 1 : 0]);
        auto kernel = un ? k_light_tiny<true> : k_light_tiny<false>;
        TC_LAUNCH("light_tiny", kernel, dim3((unsigned)blocks), dim3(256), 0, s, (const int2*)items_t.get(),
                  (const int32_t*)tbase.get() + n, (const int32_t*)rpO.get(), (const int32_t*)colO.get(),
                  (const int32_t*)rpD.get(), (const unsigned long long*)cwp, (const int2*)packU.get(),
                  (const int2*)packD.get(), comp, acc);
    }
    {
        const DevBuf<int2>& items = items_s;
        // a persistent grid larger than what stays resident would run its last
        // blocks in a second round: cap the blocks per CU at the resident count
        // of the variant launched
        static const int resident[2] = {resident_blocks(k_light_small<128, false>, 0),
                                        resident_blocks(k_light_small<128, true>, 0)};
        const int64_t blocks = (int64_t)num_cus() * std::min<int32_t>(cfg.light_blocks_per_cu, resident[un ? 1 : 0]);
        auto kernel = un ? k_light_small<128, true> : k_light_small<128, false>;
        TC_LAUNCH("light_small", kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                  (const int2*)items.get(), (const int32_t*)sbase.get() + n, (const int32_t*)rpO.get(),
                  (const int32_t*)colO.get(), (const int32_t*)rpD.get(), (const unsigned long long*)cwp,
                  (const int2*)packU.get(), (const int2*)packD.get(), sent, comp, acc);
    }
    auto launch_large = [&](const DevBuf<int2>& items, const DevBuf<int32_t>& base, int32_t dcap, bool global) {
        // tab: 4 * next_pow2(d) <= 4 * dcap slots, P: kJL+1, D: kJL, flags: 4*64*kU (16-byte multiple)
        const size_t per_block = (size_t)large_block_words(dcap);
        const size_t lds_bytes = sizeof(int32_t) * per_block;
        if (!global) {
            // one round of resident blocks (LDS and registers permitting, at most 8 per CU)
            // by variant and log2(dcap); every thread computes the same value
            static std::atomic<int> resident[2][16];
            int lgc = 0;
            while ((1 << lgc) < dcap) ++lgc;
            auto kernel = un ? k_light_large<false, true> : k_light_large<false, false>;
            int r = resident[un ? 1 : 0][lgc].load(std::memory_order_relaxed);
            if (!r) {
                r = resident_blocks(kernel, lds_bytes);
                resident[un ? 1 : 0][lgc].store(r, std::memory_order_relaxed);
            }
            const int64_t per_cu = std::min(r, 8);
            const int64_t blocks = (int64_t)num_cus() * per_cu;
            TC_LAUNCH("light_large", kernel, dim3((unsigned)blocks), dim3(256), lds_bytes, s,
                      (const int2*)items.get(), (const int32_t*)base.get() + n, (const int32_t*)rpO.get(),
                      (const int32_t*)colO.get(), (const int32_t*)rpD.get(), (const unsigned long long*)cwp,
                      (const int2*)packU.get(), (const int2*)packD.get(), dcap, (int32_t*)nullptr, sent, comp,
                      acc);
        } else {
            const int64_t blocks = (int64_t)num_cus();
            DevBuf<int32_t> gscr((size_t)blocks * per_block, s);
            auto kernel = un ? k_light_large<true, true> : k_light_large<true, false>;
            TC_LAUNCH("light_huge", kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                      (const int2*)items.get(), (const int32_t*)base.get() + n, (const int32_t*)rpO.get(),
                      (const int32_t*)colO.get(), (const int32_t*)rpD.get(), (const unsigned long long*)cwp,
                      (const int2*)packU.get(), (const int2*)packD.get(), dcap, gscr.get(), sent, comp, acc);
        }
    };
    if (plan.dcap_lds) launch_large(items_l, lbase, plan.dcap_lds, false);
    if (plan.dcap_global) launch_large(items_h, hbase, plan.dcap_global, true);

    // 5. heavy phase: sized by the bound, trimmed to the device's h inside the
    //    kernels (a union: one block per component, sized from the heavy
    //    counts read back here)
    if (un) {
        count_union_heavy(g, *un, cfg, s, acc, heavy, hpos, degp, rpO, colO);
    } else if (hmax >= 3) {
        PhaseScope ph("heavy");
        DevBuf<int32_t> hlist(hmax, s), hidx(n, s), horder(hmax, s);
        const int32_t* h_dev = hpos.get() + n;
        const int32_t hm = (int32_t)hmax;
        TC_LAUNCH("heavy_list", k_heavy_list, dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                  (const int32_t*)heavy.get(), (const int32_t*)hpos.get(), hm, hlist.get(), acc);
        DevBuf<int32_t> hrank(hmax, s);
        fill_i32(hrank.get(), 0, hmax, s);
        const int32_t chunk = rank_chunk(hmax);
        TC_LAUNCH("heavy_rank", k_heavy_rank, dim3((unsigned)std::min<int64_t>(
                                                  (int64_t)ceil_div(hmax, 256) * (int64_t)ceil_div(hmax, chunk),
                                                  (int64_t)num_cus() * 4)),
                  dim3(256), 0, s,
                  (const int32_t*)hlist.get(), h_dev, hm, chunk, degp, (const int32_t*)nullptr, hrank.get());
        TC_LAUNCH("heavy_place", k_heavy_place, dim3(ceil_div(hmax, 256)), dim3(256), 0, s,
                  (const int32_t*)hlist.get(), h_dev, hm, (const int32_t*)hrank.get(), hidx.get(), horder.get());
        DevBuf<uint8_t> U((size_t)hp_max * hp_max, s), UT((size_t)hp_max * hp_max, s);
        TC_LAUNCH("heavy_pack", k_heavy_rows, dim3((unsigned)std::min<int64_t>(hp_max, (int64_t)num_cus() * 8)),
                  dim3(256), 0, s, (const int32_t*)horder.get(),
                  h_dev, hm, (const int32_t*)rpO.get(), (const int32_t*)colO.get(), (const int32_t*)hidx.get(), U.get());
        TC_LAUNCH("heavy_transpose", k_heavy_transpose, dim3((unsigned)std::min<int64_t>(
                                                            (hp_max / 64) * (hp_max / 64), (int64_t)num_cus() * 8)),
                  dim3(256), 0, s, h_dev, hm, (const uint8_t*)U.get(), UT.get());
        // one block per macro tile up to 16 per CU (blocks beyond the resident ones
        // start as others finish), a multiple of 8 (one share per XCD)
        const int64_t nm_max = hp_max / kHT;
        const int64_t tiles_max = nm_max * (nm_max + 1) / 2;
        const int64_t mblocks = std::min<int64_t>((int64_t)num_cus() * 16, (tiles_max + 7) / 8 * 8);
        TC_LAUNCH("heavy_mfma", k_heavy_mfma, dim3((unsigned)mblocks), dim3(256), 0, s, (const uint8_t*)U.get(),
                  (const uint8_t*)UT.get(), h_dev, hm, acc);
    }
    PhaseScope ph_finish("finish");
    if (!un)
        TC_LAUNCH("finish", k_finish, dim3(1), dim3(576), 0, s, mp_dev, (const int32_t*)hpos.get() + n,
                  (const int64_t*)cpart.get(), (int32_t)cgrid, acc);
    else
        TC_LAUNCH("finish_union", k_finish_union, dim3(ceil_div(K, 256)), dim3(256), 0, s, K, un->off, un->mk,
                  (const int32_t*)hpos.get(), acc);
}

void count_enqueue(const tc_graph_s* g, int sampled, uint64_t thr, uint64_t salt, const CountConfig& cfg,
                   hipStream_t s, int64_t* acc) {
    count_impl(g, sampled, thr, salt, cfg, s, acc, nullptr);
}

void count_union(const tc_graph_s* g, const CountUnion& un, const CountConfig& cfg, hipStream_t s, int64_t* acc) {
    if (un.K < 1 || !un.comp || !un.off || !un.mk) fail(TC_ERR_INVALID, "union descriptor incomplete");
    count_impl(g, 0, 0, 0, cfg, s, acc, &un);
}

void counts_from_slots(const int64_t* hacc, tc_counts* out) {
    if (hacc[kHeavyOverflow])
        fail(TC_ERR_OVERFLOW, "heavy vertex count exceeds its bound (the heavy threshold test overflowed)");
    tc_counts res{};
    res.light = hacc[kTL];
    res.heavy = hacc[kTH];
    res.triangles = res.light + res.heavy;
    res.m = hacc[kMp];
    res.n_heavy = hacc[kH];
    res.light_sources = hacc[kLightSources];
    res.light_out_edges = hacc[kLightOut];
    res.wedges = hacc[kWedges];
    res.gather = hacc[kGather];
    res.probes = hacc[kProbes];
    res.items_small = hacc[kItemsSmall];
    res.items_large = hacc[kItemsLarge];
    res.model_bytes_small = hacc[kBytesSmall];
    res.model_bytes_large = hacc[kBytesLarge];
    *out = res;
}

void neighbour_classes(tc_graph_s* g, hipStream_t s) {
    const int64_t E2 = 2 * g->m;
    if (E2 == 0) return;
    DevBuf<uint8_t> cls(g->n, s);
    TC_LAUNCH("deg_class", k_deg_class, dim3(grid_for(g->n, 256)), dim3(256), 0, s, g->n, (const int32_t*)g->deg,
              cls.get());
    g->ncls = (uint8_t*)dev_alloc((size_t)E2, s);
    TC_LAUNCH("neighbour_class", k_neighbour_class, dim3(grid_for(E2, 256)), dim3(256), 0, s, E2,
              (const int32_t*)g->col, (const uint8_t*)cls.get(), g->ncls);
}

int64_t count_bytes(int64_t n, int64_t m, int32_t maxd, int sampled, const CountConfig& cfg) {
    auto rb = region_bytes;
    int64_t b = rb(8 * kCountSlots);  // acc of count_core
    const int64_t E2 = 2 * m;
    if (n == 0 || E2 == 0) return b;
    const int64_t NW = (E2 + 63) / 64;
    if (sampled)  // keep bits and prefix, rows, degrees, entries, staged entries
        b += rb(8 * NW) + rb(4 * (NW + 1)) + rb(4 * (n + 1)) + rb(4 * n) + 4 * rb(4 * E2) + scan_scratch_bytes(NW);
    b += rb(n) + rb(8 * NW) + rb(4 * (NW + 1)) + scan_scratch_bytes(NW);  // degree classes, orientation bits
    b += rb(4 * (n + 1)) + rb(4 * n) + rb(4 * (m + 1));            // rpO, d+, up lists and their sentinel
    b += 2 * rb(4 * (n + 1)) + rb(4 * n);                          // heavy, code, descriptor slots
    b += rb(16 * n) + 2 * rb(8 * n) + rb(12 * (n + 1));            // rowQ, Wu, cw, wide-list vertices
    b += rb(8 * m) + rb(8 * (cfg.vmajor_cap > 0 ? m : 1));         // packed descriptors
    b += 9 * rb(4 * (n + 1)) + scan_x4_scratch_bytes(n) + scan_scratch_bytes(n);  // item counts and bases
    b += rb(8 * (2 * n + E2 / kJL + 2));                                           // tiny item list
    b += rb(8 * 9 * (int64_t)std::min<int64_t>((n + 255) / 256, kClassifyBlocks));  // classification partials
    const int64_t items_max = 2 * n + E2 / kJL + 2;
    b += rb(8 * items_max);
    const LightPlan plan = light_plan(m, maxd, cfg);
    b += plan.dcap_lds ? rb(8 * items_max) : rb(8);
    b += plan.dcap_global ? rb(8 * items_max) + rb(4 * (int64_t)num_cus() * large_block_words(plan.dcap_global)) : rb(8);
    const int64_t hmax = heavy_bound(n, m, cfg.heavy_num, cfg.heavy_den);
    if (hmax >= 3) {
        const int64_t hp = heavy_pad(hmax);
        b += 3 * rb(4 * hmax) + rb(4 * n) + 2 * rb(hp * hp);  // list, order, rank, index, U, UT
    }
    return b;
}

int64_t count_union_bytes(int64_t n, int64_t m, int32_t maxd, int32_t K, int64_t h, int64_t ubytes, int64_t ntiles,
                          const CountConfig& cfg) {
    auto rb = region_bytes;
    // the single count's allocations without its heavy phase
    int64_t b = count_bytes(n, m, maxd, 0, cfg) - rb(8 * kCountSlots);
    const int64_t hb = heavy_bound(n, m, cfg.heavy_num, cfg.heavy_den);
    if (n > 0 && m > 0 && hb >= 3) {
        const int64_t hp = heavy_pad(hb);
        b -= 3 * rb(4 * hb) + rb(4 * n) + 2 * rb(hp * hp);
    }
    b += rb(8 * n) + rb(4 * (n + 1));  // per-list gather statistic; the zero row of an edgeless union
    // heavy blocks: starts, block sizes and offsets, tile list, ranks, two matrices
    b += rb(4 * ((int64_t)K + 1)) + rb(4 * (int64_t)K) + 2 * rb(8 * ((int64_t)K + 1)) + rb(8 * (int64_t)K) +
         rb(16 * ntiles) + 3 * rb(4 * h) + rb(4 * n) + 2 * rb(ubytes);
    return b;
}

void count_core(const tc_graph_s* g, int sampled, uint64_t thr, uint64_t salt, const CountConfig& cfg,
                hipStream_t s, tc_counts* out) {
    DevBuf<int64_t> acc(kCountSlots, s);
    count_enqueue(g, sampled, thr, salt, cfg, s, acc.get());
    int64_t hacc[kCountSlots];
    check_hip(hipMemcpyAsync(hacc, acc.get(), sizeof(hacc), hipMemcpyDeviceToHost, s), "acc");
    check_hip(hipStreamSynchronize(s), "sync");
    counts_from_slots(hacc, out);
}

}  // namespace tc
