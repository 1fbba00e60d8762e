// Exact triangle count of a (possibly sparsified) graph with the light/heavy
// vertex partition of section 3.2.
//
//   1. degrees of the counted graph (after the section 3.1 coin, if sampled);
//   2. orientation u -> v iff (deg u, u) < (deg v, v); every triangle is
//      charged to its lowest-ranked vertex.  Heavy vertices (deg > c m^(1/2))
//      rank above every light vertex, so a triangle whose lowest vertex is
//      heavy has three heavy vertices;
//   3. light phase: for every light u, the wedges of section 3.2 (pairs of
//      out-neighbours) are closed by testing, for each v in N+(u), which
//      members of N+(v) lie in N+(u).  N+(u) is staged once in an LDS hash
//      set; the concatenation of the N+(v) lists is split into fixed-size
//      chunks so that every work item has a bounded cost;
//   4. heavy phase: the <= 2 m^(1/2) heavy vertices, in rank order, form a
//      strictly upper-triangular 0/1 matrix U; sum((U U) .* U) counts each
//      all-heavy triangle once (the matrix-multiplication route of Alon,
//      Yuster and Zwick that section 2.1 and section 3 build on) and runs on
//      int8 MFMA with int32 accumulation.
#include "tc_internal.h"
#include "tc_device.h"

#include <algorithm>
#include <vector>

namespace tc {

namespace {

enum Acc {
    kTL = 0, kTH, kLightSources, kLightOut, kWedges, kGather, kDmaxLarge, kSrcLarge, kOutLarge, kGatherLarge, kAccN
};

unsigned grid_for(int64_t N, int threads) {
    unsigned b = ceil_div(N, threads);
    if (b > 65536) b = 65536;
    return b ? b : 1;
}

int num_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

// ---------------------------------------------------------------------------
// orientation
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_orient_bits(const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                                                      int64_t E2, const uint64_t* __restrict__ keep,
                                                      const int32_t* __restrict__ degp, uint64_t* __restrict__ obits,
                                                      int32_t* __restrict__ ocnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x; e0 < E2; e0 += stride) {
        const int64_t e = e0 + threadIdx.x;
        bool o = false;
        if (e < E2) {
            const bool k = keep ? ((keep[e >> 6] >> (e & 63)) & 1ull) : true;
            if (k) {
                const int32_t u = src[e], v = col[e];
                o = rank_below(degp[u], u, degp[v], v);
            }
        }
        const uint64_t b = ballot64(o);
        if (__lane_id() == 0 && e < E2) {
            obits[e >> 6] = b;
            ocnt[e >> 6] = __popcll(b);
        }
    }
}

// ---------------------------------------------------------------------------
// classification and light work
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool is_heavy(int64_t deg, int64_t m, int32_t a, int32_t b) {
    return (int64_t)b * b * deg * deg > (int64_t)a * a * m;
}

// Sum of `val` over the run of equal `key` that ends at this lane; true on the
// run's last lane.  All lanes of the wave must call it; invalid lanes pass val 0.
__device__ __forceinline__ bool run_tail_sum(int32_t key, bool valid, int64_t val, int64_t* sum) {
    const int lane = __lane_id();
    const int64_t incl = wave_inclusive_sum(val);
    const int32_t pk = __shfl_up(key, 1, 64);
    const int32_t nk = __shfl_down(key, 1, 64);
    const uint64_t active = ballot64(valid);
    const bool head = valid && !(lane > 0 && ((active >> (lane - 1)) & 1ull) && pk == key);
    const bool tail = valid && !(lane < 63 && ((active >> (lane + 1)) & 1ull) && nk == key);
    const uint64_t heads = ballot64(head);
    const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    const uint64_t hm = heads & le;
    const int my_head = hm ? 63 - __builtin_clzll(hm) : 0;
    const int src_lane = my_head > 0 ? my_head - 1 : 0;
    const int64_t before = __shfl(incl, src_lane, 64);
    *sum = incl - (my_head > 0 ? before : 0);
    return tail;
}

// W[u] += d+(v) for oriented u -> v with u light and d+(u) >= 2
__global__ void __launch_bounds__(256) k_work(const int32_t* __restrict__ srcO, const int32_t* __restrict__ colO,
                                               const int32_t* __restrict__ degp,
                                               const int32_t* __restrict__ dplus, const int32_t* __restrict__ mp_dev,
                                               int32_t ha, int32_t hb, int64_t* __restrict__ W) {
    const int64_t mp = mp_dev[0];  // oriented edges = m'; entries beyond it are unused
    const int64_t mo = mp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x; e0 < mo; e0 += stride) {
        const int64_t e = e0 + threadIdx.x;
        bool valid = false;
        int32_t u = -1;
        int64_t val = 0;
        if (e < mo) {
            u = srcO[e];
            if (dplus[u] >= 2 && !is_heavy(degp[u], mp, ha, hb)) {
                valid = true;
                val = dplus[colO[e]];
            }
        }
        int64_t sum;
        const bool tail = run_tail_sum(valid ? u : -1, valid, val, &sum);
        if (tail) atomicAdd((unsigned long long*)&W[u], (unsigned long long)sum);
    }
}

// per-vertex: heavy flag, item counts of the two light bins, statistics
__global__ void __launch_bounds__(256) k_classify(int64_t n, const int32_t* __restrict__ degp,
                                                   const int32_t* __restrict__ dplus, const int64_t* __restrict__ W,
                                                   const int32_t* __restrict__ mp_dev, int32_t ha, int32_t hb,
                                                   int32_t small_dmax, int32_t chunk_s, int32_t chunk_l,
                                                   int32_t* __restrict__ heavy, int32_t* __restrict__ nsm,
                                                   int32_t* __restrict__ nlg, int64_t* __restrict__ acc) {
    const int64_t mp = mp_dev[0];
    int64_t ls = 0, lo = 0, wd = 0, ga = 0, dmax = 0, lsL = 0, loL = 0, gaL = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t dg = degp[x];
        const int32_t dp = dplus[x];
        const bool hv = dg > 0 && is_heavy(dg, mp, ha, hb);
        heavy[x] = hv ? 1 : 0;
        int32_t cs = 0, cl = 0;
        if (!hv && dp >= 2) {
            const int64_t w = W[x];
            ls += 1;
            lo += dp;
            wd += (int64_t)dp * (dp - 1) / 2;
            ga += w;
            if (w > 0) {
                if (dp <= small_dmax) cs = (int32_t)((w + chunk_s - 1) / chunk_s);
                else {
                    cl = (int32_t)((w + chunk_l - 1) / chunk_l);
                    dmax = dp > dmax ? dp : dmax;
                    lsL += 1;
                    loL += dp;
                    gaL += w;
                }
            }
        }
        nsm[x] = cs;
        nlg[x] = cl;
    }
    ls = wave_sum(ls); lo = wave_sum(lo); wd = wave_sum(wd); ga = wave_sum(ga); dmax = wave_max(dmax);
    lsL = wave_sum(lsL); loL = wave_sum(loL); gaL = wave_sum(gaL);
    if (__lane_id() == 0) {
        if (ls) atomicAdd((unsigned long long*)&acc[kLightSources], (unsigned long long)ls);
        if (lo) atomicAdd((unsigned long long*)&acc[kLightOut], (unsigned long long)lo);
        if (wd) atomicAdd((unsigned long long*)&acc[kWedges], (unsigned long long)wd);
        if (ga) atomicAdd((unsigned long long*)&acc[kGather], (unsigned long long)ga);
        if (dmax) atomicMax((unsigned long long*)&acc[kDmaxLarge], (unsigned long long)dmax);
        if (lsL) atomicAdd((unsigned long long*)&acc[kSrcLarge], (unsigned long long)lsL);
        if (loL) atomicAdd((unsigned long long*)&acc[kOutLarge], (unsigned long long)loL);
        if (gaL) atomicAdd((unsigned long long*)&acc[kGatherLarge], (unsigned long long)gaL);
    }
}

__global__ void k_items(int64_t n, const int32_t* __restrict__ cnt, const int32_t* __restrict__ base,
                        int2* __restrict__ items) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = cnt[x];
        const int32_t b = base[x];
        for (int32_t i = 0; i < c; ++i) items[b + i] = make_int2((int32_t)x, i);
    }
}

__global__ void k_heavy_list(int64_t n, const int32_t* __restrict__ heavy, const int32_t* __restrict__ hpos,
                             int32_t* __restrict__ hlist) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        if (heavy[x]) hlist[hpos[x]] = (int32_t)x;
}

__global__ void k_info(const int32_t* mp, const int32_t* sb, const int32_t* lb, const int32_t* hp, const int64_t* acc,
                       int64_t* info) {
    if (threadIdx.x == 0) {
        info[0] = mp[0];
        info[1] = sb[0];
        info[2] = lb[0];
        info[3] = hp[0];
        info[4] = acc[kDmaxLarge];
    }
}

// ---------------------------------------------------------------------------
// light closure
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t hslot(int32_t w, int lg) {
    return ((uint32_t)w * 0x9E3779B1u) >> (32 - lg);
}

__device__ __forceinline__ void hash_insert(int32_t* tab, int lg, int32_t v) {
    const uint32_t mask = (1u << lg) - 1;
    uint32_t s = hslot(v, lg);
    while (true) {
        const int32_t prev = atomicCAS(&tab[s], -1, v);
        if (prev == -1 || prev == v) break;
        s = (s + 1) & mask;
    }
}

__device__ __forceinline__ int hash_contains(const int32_t* tab, int lg, int32_t w) {
    const uint32_t mask = (1u << lg) - 1;
    uint32_t s = hslot(w, lg);
    while (true) {
        const int32_t k = tab[s];
        if (k == w) return 1;
        if (k == -1) return 0;
        s = (s + 1) & mask;
    }
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

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per item (u, chunk), persistent over items with a static stride.
// LDS per wave: hash (2*DS slots), P (DS+1), S (DS).
template <int DS>
__global__ void __launch_bounds__(256) k_light_small(const int2* __restrict__ items, int64_t n_items,
                                                      const int32_t* __restrict__ rpO,
                                                      const int32_t* __restrict__ colO, int32_t chunk,
                                                      int64_t* __restrict__ acc) {
    constexpr int HS_MAX = 2 * DS;
    __shared__ int32_t lds[4][HS_MAX + 2 * DS + 1];
    const int w = threadIdx.x >> 6;
    const int lane = __lane_id();
    int32_t* tab = lds[w];
    int32_t* P = tab + HS_MAX;
    int32_t* S = P + DS + 1;
    const int64_t gw = (int64_t)blockIdx.x * 4 + w;
    const int64_t nw = (int64_t)gridDim.x * 4;
    int64_t total = 0;
    for (int64_t it = gw; it < n_items; it += nw) {
        const int2 item = items[it];
        const int32_t u = item.x;
        const int32_t rs = rpO[u];
        const int32_t d = rpO[u + 1] - rs;
        int lg = 6;
        while ((1 << lg) < 2 * d) ++lg;
        const int hs = 1 << lg;
        for (int i = lane; i < hs; i += 64) tab[i] = -1;
        if (lane == 0) P[0] = 0;
        wave_lds_sync();
        int32_t carry = 0;
        for (int j0 = 0; j0 < d; j0 += 64) {
            const int j = j0 + lane;
            int32_t len = 0;
            if (j < d) {
                const int32_t v = colO[rs + j];
                const int32_t st = rpO[v];
                len = rpO[v + 1] - st;
                S[j] = st;
                hash_insert(tab, lg, v);
            }
            const int32_t inc = wave_inclusive_sum(len);
            if (j < d) P[j + 1] = carry + inc;
            carry += __shfl(inc, 63, 64);
        }
        wave_lds_sync();
        const int32_t g0 = item.y * chunk;
        const int32_t g1 = min(g0 + chunk, carry);
        int32_t cnt = 0;
        for (int32_t gb = g0; gb < g1; gb += 64) {
            const int32_t g = gb + lane;
            if (g < g1) {
                const int j = find_list(P, d, g);
                const int32_t x = colO[S[j] + (g - P[j])];
                cnt += hash_contains(tab, lg, x);
            }
        }
        total += cnt;
        wave_lds_sync();
    }
    total = wave_sum(total);
    if (lane == 0 && total) atomicAdd((unsigned long long*)&acc[kTL], (unsigned long long)total);
}

// One block (256 threads) per item; N+(u) of any light size.  The hash set and
// the list tables live in dynamic LDS, or in a global scratch slice per block
// when they do not fit (out-degrees beyond the LDS capacity).
__global__ void __launch_bounds__(256) k_light_large(const int2* __restrict__ items, int64_t n_items,
                                                      const int32_t* __restrict__ rpO,
                                                      const int32_t* __restrict__ colO, int32_t chunk, int32_t dcap,
                                                      int32_t* __restrict__ gscratch, int64_t* __restrict__ acc) {
    extern __shared__ int32_t dyn[];
    __shared__ int32_t red[5];
    // layout: hash table (up to 2 * dcap slots, 4 * dcap reserved), P (dcap + 1), S (dcap)
    int32_t* base = gscratch ? gscratch + (int64_t)blockIdx.x * (int64_t)(4 * dcap + 2 * dcap + 2) : dyn;
    int32_t* tab = base;
    int32_t* P = base + 4 * dcap;
    int32_t* S = P + dcap + 1;
    const int t = threadIdx.x;
    int64_t total = 0;
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = items[it];
        const int32_t u = item.x;
        const int32_t rs = rpO[u];
        const int32_t d = rpO[u + 1] - rs;
        int lg = 6;
        while ((1 << lg) < 2 * d) ++lg;
        const int hs = 1 << lg;
        for (int i = t; i < hs; i += 256) tab[i] = -1;
        if (t == 0) P[0] = 0;
        __syncthreads();
        int32_t carry = 0;
        for (int j0 = 0; j0 < d; j0 += 256) {
            const int j = j0 + t;
            int32_t len = 0;
            if (j < d) {
                const int32_t v = colO[rs + j];
                const int32_t st = rpO[v];
                len = rpO[v + 1] - st;
                S[j] = st;
                hash_insert(tab, lg, v);
            }
            int32_t tot;
            const int32_t ex = block_exclusive_sum<256>(len, red, &tot);
            if (j < d) P[j + 1] = carry + ex + len;
            carry += tot;
        }
        __syncthreads();
        const int32_t g0 = item.y * chunk;
        const int32_t g1 = min(g0 + chunk, carry);
        int32_t cnt = 0;
        for (int32_t g = g0 + t; g < g1; g += 256) {
            const int j = find_list(P, d, g);
            const int32_t x = colO[S[j] + (g - P[j])];
            cnt += hash_contains(tab, lg, x);
        }
        total += cnt;
        __syncthreads();
    }
    total = wave_sum(total);
    if (__lane_id() == 0 && total) atomicAdd((unsigned long long*)&acc[kTL], (unsigned long long)total);
}

// ---------------------------------------------------------------------------
// heavy block
// ---------------------------------------------------------------------------

// rank of each heavy vertex in (deg, id) order, by counting smaller keys
__global__ void __launch_bounds__(256) k_heavy_rank(const int32_t* __restrict__ hlist, int32_t h,
                                                     const int32_t* __restrict__ degp, int32_t* __restrict__ hidx,
                                                     int32_t* __restrict__ horder) {
    __shared__ int32_t kd[256], kx[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    int32_t x = -1, dx = 0;
    if (i < h) { x = hlist[i]; dx = degp[x]; }
    int32_t r = 0;
    for (int j0 = 0; j0 < h; j0 += 256) {
        const int j = j0 + threadIdx.x;
        if (j < h) { kx[threadIdx.x] = hlist[j]; kd[threadIdx.x] = degp[kx[threadIdx.x]]; }
        __syncthreads();
        const int lim = min(256, h - j0);
        if (i < h)
            for (int q = 0; q < lim; ++q) r += rank_below(kd[q], kx[q], dx, x) ? 1 : 0;
        __syncthreads();
    }
    if (i < h) {
        hidx[x] = r;
        horder[r] = x;
    }
}

// U[i][j] = 1 and UT[j][i] = 1 for every oriented edge between heavy ranks i < j
__global__ void __launch_bounds__(256) k_heavy_pack(const int32_t* __restrict__ horder, int32_t h,
                                                     const int32_t* __restrict__ rpO, const int32_t* __restrict__ colO,
                                                     const int32_t* __restrict__ hidx, int32_t hp,
                                                     uint8_t* __restrict__ U, uint8_t* __restrict__ UT) {
    const int i = blockIdx.x;
    if (i >= h) return;
    const int32_t x = horder[i];
    for (int32_t e = rpO[x] + threadIdx.x; e < rpO[x + 1]; e += 256) {
        const int32_t j = hidx[colO[e]];
        U[(int64_t)i * hp + j] = 1;
        UT[(int64_t)j * hp + i] = 1;
    }
}

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef int32_t v16i __attribute__((ext_vector_type(16)));

// One wave per 32x32 output tile (I, J), I <= J, of C = U U restricted to the
// k-blocks I..J where both factors can be non-zero; the epilogue masks with
// U[I,J] and adds into T_H.  Operand fragments: lane l supplies row (l mod 32)
// of the A tile and column (l mod 32) of the B tile, 16 consecutive k-bytes
// starting at 16 * (l / 32); the same k-permutation is used for A and B.
__global__ void __launch_bounds__(256) k_heavy_mfma(const uint8_t* __restrict__ U, const uint8_t* __restrict__ UT,
                                                     int32_t hp, int64_t ntiles, int64_t* __restrict__ acc) {
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= ntiles) return;
    // invert t = J (J + 1) / 2 + I
    int64_t J = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (J * (J + 1) / 2 > t) --J;
    while ((J + 1) * (J + 2) / 2 <= t) ++J;
    const int64_t I = t - J * (J + 1) / 2;
    const int lane = __lane_id();
    const int r = lane & 31;
    const int kh = lane >> 5;
    const uint8_t* arow = U + (I * 32 + r) * (int64_t)hp + kh * 16;
    const uint8_t* brow = UT + (J * 32 + r) * (int64_t)hp + kh * 16;
    v16i c = {0};
    for (int64_t kb = I; kb <= J; ++kb) {
        const v4i a = *(const v4i*)(arow + kb * 32);
        const v4i b = *(const v4i*)(brow + kb * 32);
        c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
    }
    // accumulator element q of lane l: row 8*(q/4) + 4*(l/32) + q%4, column l%32
    int64_t s = 0;
    const int colj = (int)(J * 32) + r;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int row = (int)(I * 32) + 8 * (q >> 2) + 4 * kh + (q & 3);
        s += (int64_t)c[q] * (int64_t)U[(int64_t)row * hp + colj];
    }
    s = wave_sum(s);
    if (lane == 0 && s) atomicAdd((unsigned long long*)&acc[kTH], (unsigned long long)s);
}

}  // namespace

void count_core(const tc_graph_s* g, int sampled, uint64_t thr, uint64_t salt, const CountConfig& cfg,
                hipStream_t s, tc_counts* out) {
    const int64_t n = g->n;
    const int64_t E2 = 2 * g->m;
    tc_counts res{};
    if (n == 0 || E2 == 0) {
        *out = res;
        return;
    }
    const int64_t NW = (E2 + 63) / 64;

    DevBuf<int64_t> acc(kAccN, s);
    fill_i64(acc.get(), 0, kAccN, s);

    // 1. degrees of the counted graph
    DevBuf<uint64_t> keep;
    DevBuf<int32_t> kpre;
    DevBuf<int32_t> degp_buf;
    const int32_t* degp = g->deg;
    if (sampled) {
        keep.reset(NW, s);
        kpre.reset(NW + 1, s);
        degp_buf.reset(n, s);
        sample_keep_bits(g, salt, thr, keep.get(), kpre.get(), s);
        scan_exclusive_i32(kpre.get(), kpre.get(), NW, s);
        positions_at_rows(g->row_ptr, n, E2, keep.get(), kpre.get(), nullptr, degp_buf.get(), s);
        degp = degp_buf.get();
    }

    // 2. orientation by (deg, id): compacted out-lists N+(u)
    DevBuf<uint64_t> obits(NW, s);
    DevBuf<int32_t> opre(NW + 1, s);
    TC_LAUNCH("orient_bits", k_orient_bits, dim3(grid_for(E2, 256)), dim3(256), 0, s, g->src, g->col, E2,
              (const uint64_t*)keep.get(), degp, obits.get(), opre.get());
    scan_exclusive_i32(opre.get(), opre.get(), NW, s);
    const int32_t* mp_dev = opre.get() + NW;  // number of oriented edges = m'
    DevBuf<int32_t> rpO(n + 1, s), dplus(n, s);
    positions_at_rows(g->row_ptr, n, E2, obits.get(), opre.get(), rpO.get(), dplus.get(), s);
    // m' <= m: size the oriented lists by m
    DevBuf<int32_t> colO(g->m, s), srcO(g->m, s);
    compact_kept(g->col, g->src, E2, obits.get(), opre.get(), colO.get(), srcO.get(), s);

    // 3. classification, light work per source, item lists
    DevBuf<int64_t> W(n, s);
    fill_i64(W.get(), 0, n, s);
    TC_LAUNCH("work", k_work, dim3(grid_for(g->m, 256)), dim3(256), 0, s, (const int32_t*)srcO.get(),
              (const int32_t*)colO.get(), degp, (const int32_t*)dplus.get(), mp_dev, cfg.heavy_num, cfg.heavy_den,
              W.get());
    DevBuf<int32_t> heavy(n + 1, s), nsm(n + 1, s), nlg(n + 1, s);
    TC_LAUNCH("classify", k_classify, dim3(grid_for(n, 256)), dim3(256), 0, s, n, degp, (const int32_t*)dplus.get(),
              (const int64_t*)W.get(), mp_dev, cfg.heavy_num, cfg.heavy_den, cfg.small_dmax, cfg.chunk_small,
              cfg.chunk_large, heavy.get(), nsm.get(), nlg.get(), acc.get());
    DevBuf<int32_t> sbase(n + 1, s), lbase(n + 1, s), hpos(n + 1, s);
    scan_exclusive_i32(nsm.get(), sbase.get(), n, s);
    scan_exclusive_i32(nlg.get(), lbase.get(), n, s);
    scan_exclusive_i32(heavy.get(), hpos.get(), n, s);
    DevBuf<int64_t> info(8, s);
    TC_LAUNCH("info", k_info, dim3(1), dim3(64), 0, s, mp_dev, (const int32_t*)sbase.get() + n,
              (const int32_t*)lbase.get() + n, (const int32_t*)hpos.get() + n, (const int64_t*)acc.get(), info.get());
    int64_t hinfo[8] = {0};
    check_hip(hipMemcpyAsync(hinfo, info.get(), sizeof(int64_t) * 5, hipMemcpyDeviceToHost, s), "info");
    check_hip(hipStreamSynchronize(s), "sync");
    const int64_t mp = hinfo[0], n_small = hinfo[1], n_large = hinfo[2], h = hinfo[3], dmax_large = hinfo[4];

    // 4. light phase
    if (n_small > 0) {
        DevBuf<int2> items(n_small, s);
        TC_LAUNCH("items", k_items, dim3(grid_for(n, 256)), dim3(256), 0, s, n, (const int32_t*)nsm.get(),
                  (const int32_t*)sbase.get(), items.get());
        int64_t blocks = (int64_t)num_cus() * cfg.light_blocks_per_cu;
        const int64_t need = (n_small + 3) / 4;
        if (blocks > need) blocks = need;
        TC_LAUNCH("light_small", k_light_small<256>, dim3((unsigned)blocks), dim3(256), 0, s,
                  (const int2*)items.get(), n_small, (const int32_t*)rpO.get(), (const int32_t*)colO.get(),
                  cfg.chunk_small, acc.get());
    }
    if (n_large > 0) {
        DevBuf<int2> items(n_large, s);
        TC_LAUNCH("items", k_items, dim3(grid_for(n, 256)), dim3(256), 0, s, n, (const int32_t*)nlg.get(),
                  (const int32_t*)lbase.get(), items.get());
        int64_t blocks = (int64_t)num_cus() * 2;
        if (blocks > n_large) blocks = n_large;
        int32_t dcap = 64;
        while (dcap < dmax_large) dcap <<= 1;
        // tab: 2*next_pow2(d) <= 4*dcap slots, P: dcap+1, S: dcap
        const size_t lds_bytes = sizeof(int32_t) * (size_t)(4 * dcap + 2 * dcap + 2);
        DevBuf<int32_t> gscr;
        size_t dyn = lds_bytes;
        if (lds_bytes > 64 * 1024) {
            gscr.reset((size_t)blocks * (size_t)(4 * dcap + 2 * dcap + 2), s);
            dyn = 0;
        }
        TC_LAUNCH("light_large", k_light_large, dim3((unsigned)blocks), dim3(256), dyn, s, (const int2*)items.get(),
                  n_large, (const int32_t*)rpO.get(), (const int32_t*)colO.get(), cfg.chunk_large, dcap, gscr.get(),
                  acc.get());
    }

    // 5. heavy phase
    if (h >= 3) {
        DevBuf<int32_t> hlist(h, s), hidx(n, s), horder(h, s);
        TC_LAUNCH("heavy_list", k_heavy_list, dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                  (const int32_t*)heavy.get(), (const int32_t*)hpos.get(), hlist.get());
        TC_LAUNCH("heavy_rank", k_heavy_rank, dim3(ceil_div(h, 256)), dim3(256), 0, s, (const int32_t*)hlist.get(),
                  (int32_t)h, degp, hidx.get(), horder.get());
        const int32_t hp = (int32_t)((h + 31) / 32 * 32);
        DevBuf<uint8_t> U((size_t)hp * hp, s), UT((size_t)hp * hp, s);
        fill_u8(U.get(), 0, (int64_t)hp * hp, s);
        fill_u8(UT.get(), 0, (int64_t)hp * hp, s);
        TC_LAUNCH("heavy_pack", k_heavy_pack, dim3((unsigned)h), dim3(256), 0, s, (const int32_t*)horder.get(),
                  (int32_t)h, (const int32_t*)rpO.get(), (const int32_t*)colO.get(), (const int32_t*)hidx.get(), hp,
                  U.get(), UT.get());
        const int64_t nb = hp / 32;
        const int64_t ntiles = nb * (nb + 1) / 2;
        TC_LAUNCH("heavy_mfma", k_heavy_mfma, dim3(ceil_div(ntiles, 4)), dim3(256), 0, s, (const uint8_t*)U.get(),
                  (const uint8_t*)UT.get(), hp, ntiles, acc.get());
    }

    int64_t hacc[kAccN];
    check_hip(hipMemcpyAsync(hacc, acc.get(), sizeof(hacc), hipMemcpyDeviceToHost, s), "acc");
    check_hip(hipStreamSynchronize(s), "sync");
    res.light = hacc[kTL];
    res.heavy = hacc[kTH];
    res.triangles = res.light + res.heavy;
    res.m = mp;
    res.n_heavy = h;
    res.light_sources = hacc[kLightSources];
    res.light_out_edges = hacc[kLightOut];
    res.wedges = hacc[kWedges];
    res.gather = hacc[kGather];
    res.light_sources_large = hacc[kSrcLarge];
    res.light_out_edges_large = hacc[kOutLarge];
    res.gather_large = hacc[kGatherLarge];
    *out = res;
}

}  // namespace tc
